// Host orchestration of the HSS update (Algorithm 2 and Algorithm 3), the
// rank estimate of eq. (bounds) with the neighbouring-segment rules of
// Section 4.1, the adaptive accuracy check, and the adc_hss_* entry points.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "hss.hpp"

namespace {

constexpr int SP_PROBE = 32;  // padded probe count of the accuracy check
constexpr int S_MAX = 256;

int ceil_log2_ratio(int K, int m) {
  int L = 0;
  while (((int64_t)m << L) < K) ++L;
  return L;
}

std::vector<int> balanced_bounds(int K, int L) {
  std::vector<std::pair<int, int>> r{{0, K}};
  for (int l = 0; l < L; ++l) {
    std::vector<std::pair<int, int>> nx;
    for (auto& p : r) {
      const int h = (p.second - p.first) / 2;
      nx.push_back({p.first, p.first + h});
      nx.push_back({p.first + h, p.second});
    }
    r.swap(nx);
  }
  std::vector<int> b;
  for (auto& p : r) b.push_back(p.first);
  b.push_back(K);
  return b;
}

}  // namespace

std::vector<int> hss_leaf_bounds(int K, int leaf) {
  return balanced_bounds(K, std::max(1, ceil_log2_ratio(K, leaf)));
}

// Rank estimate of eq. (bounds) with the boundary moves of Section 4.1 for
// one merge whose generators d, gam, mu are device arrays: the solver's
// kernel (k_leaf_bounds) on a one-merge descriptor.  `bounds` comes in
// balanced and goes out moved.
adc_status device_rank_estimate(adc_ctx c, const double* d, const double* gam, const double* mu, int K,
                                std::vector<int>& bounds, const adc_opts& o, int* r) {
  hipStream_t st = c->stream;
  const int nleaf = (int)bounds.size() - 1;
  void* dp;
  const size_t need = 256 + sizeof(MergeDev) + 4 * (size_t)(nleaf + 1) + 256;
  ADC_TRY(c->buffer(SLOT_RANK, need, &dp));
  MergeDev md{};
  md.s0 = 0;
  md.n = K;
  md.K = K;
  md.nleaf = nleaf;
  MergeDev* dm = (MergeDev*)dp;
  int32_t* dw = (int32_t*)((char*)dp + sizeof(MergeDev));  // which[0] = 0
  int32_t* db = dw + 64;
  md.lbounds = db;
  LevelBufs B{};
  B.dS = const_cast<double*>(d);
  B.gam = const_cast<double*>(gam);
  B.mu = const_cast<double*>(mu);
  const int32_t zero = 0;
  HIP_OK(hipMemcpyAsync(dm, &md, sizeof(md), hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(dw, &zero, 4, hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(db, bounds.data(), 4 * (size_t)(nleaf + 1), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_leaf_bounds, dim3(1), dim3(64), 0, st, dm, dw, B, o.shift_thresh, o.shift_max, o.rank_eps,
                     o.r_cap);
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(bounds.data(), db, 4 * (size_t)(nleaf + 1), hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(&md, dm, sizeof(md), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  *r = md.rest;
  return ADC_OK;
}

// ---------------------------------------------------------------------------
// A set of HSS merges built together (one DC level, or one adc_hss_build).
struct HssBatch {
  struct One {
    int K = 0, L = 0, s = 0, sp = 0, r = 0;
    uint32_t stream = 0;
    std::vector<int> bounds;
    std::vector<HssNode> nodes;  // host copy
    HssMerge dev{};
    int64_t node_off = 0, map_off = 0, arena_off = 0, iarena_off = 0, vec_off = 0;
    int64_t arena_n = 0, iarena_n = 0;
    bool pass = false;
    double err = 0.0;
    int sat = 0;  // nodes whose row or column ID used every sample with more candidates
    int retries = 0;
    int max_rank = 0;
    std::vector<double> hd, hg, hmu;  // host copies of d, gam, mu (fast sampling lists)
    std::vector<int32_t> grp;         // per leaf: top-only, both, bottom-only columns (solver)
  };
  std::vector<One> ms;
  char* mem = nullptr;
  HssMerge* d_ms = nullptr;
  int64_t nodes_end = 0, host_end = 0;  // ends of the node tables and of the host-written range in mem
  int fmm_p = 0;                   // Chebyshev points per node; 0: direct sampling
  std::function<void()> after_sampling;  // called once, after the first sampling pass is queued
  std::vector<char> sample_host;   // launch lists of the last sampling pass
};

namespace {

// Lay out the nodes and storage of one merge for s samples; fills o.nodes and
// sizes (in doubles / ints).  Offsets are relative to the merge's arenas.
void layout_merge(HssBatch::One& m) {
  const int L = m.L;
  const int nn = (1 << (L + 1)) - 1;
  m.nodes.assign(nn, HssNode{});
  const int sp = m.sp, s = m.s;
  int64_t a = 0, ia = 0;
  for (int l = 0; l <= L; ++l) {
    const int first = (1 << l) - 1;
    const int cnt = 1 << l;
    const int span = 1 << (L - l);
    for (int q = 0; q < cnt; ++q) {
      HssNode& nd = m.nodes[first + q];
      nd.lo = m.bounds[q * span];
      nd.hi = m.bounds[(q + 1) * span];
      nd.leaf = (l == L);
      const int kmax = std::min(s, nd.hi - nd.lo);
      const int cand = nd.leaf ? (nd.hi - nd.lo) : std::min(2 * s, nd.hi - nd.lo);
      nd.offU = a;
      a += (int64_t)cand * kmax;
      nd.offV = a;
      a += (int64_t)cand * kmax;
      nd.offB = a;
      a += (int64_t)kmax * s;
      nd.offPs = a;
      a += (int64_t)kmax * sp;
      nd.offTs = a;
      a += (int64_t)kmax * sp;
      nd.offYh = a;
      a += (int64_t)kmax * sp;
      nd.offZh = a;
      a += (int64_t)kmax * sp;
      nd.offWork = a;  // per side (rows, columns): the block and a working copy
      a += (l == 0) ? 0 : 4 * (int64_t)cand * sp;
      nd.offSr = ia;
      ia += kmax;
      nd.offSc = ia;
      ia += kmax;
      a = (a + 31) & ~(int64_t)31;
    }
  }
  m.arena_n = a;
  m.iarena_n = ia;
}

}  // namespace

// Allocate and upload a batch (all merges' sizes and bounds already set).
static adc_status batch_alloc(adc_ctx c, HssBatch& hb, int slot) {
  int64_t bytes = 0;
  auto take = [&](int64_t n) {
    bytes = (bytes + 255) & ~(int64_t)255;
    const int64_t o = bytes;
    bytes += n;
    return o;
  };
  const int nm = (int)hb.ms.size();
  // what the host writes (merge table, node tables, leaf maps and bounds)
  // first, in one range: one upload; the node tables in one range: one
  // read-back of the ranks
  for (auto& m : hb.ms) layout_merge(m);
  const int64_t off_ms = take(nm * sizeof(HssMerge));
  for (auto& m : hb.ms) m.node_off = take((int64_t)m.nodes.size() * sizeof(HssNode));
  hb.nodes_end = bytes;
  for (auto& m : hb.ms) m.map_off = take((int64_t)m.K * 4 + ((int64_t)m.bounds.size()) * 4);
  hb.host_end = bytes;
  for (auto& m : hb.ms) {
    m.vec_off = take((int64_t)3 * m.K * m.sp * 8);
    m.arena_off = take(m.arena_n * 8);
    m.iarena_off = take(m.iarena_n * 4);
  }
  void* p;
  ADC_TRY(c->buffer(slot, (size_t)bytes + 256, &p));
  hb.mem = (char*)p;
  hb.d_ms = (HssMerge*)(hb.mem + off_ms);
  for (auto& m : hb.ms) {
    char* v = hb.mem + m.vec_off;
    m.dev.omega = (double*)v;
    m.dev.phi = m.dev.omega + (int64_t)m.K * m.sp;
    m.dev.theta = m.dev.phi + (int64_t)m.K * m.sp;
    int32_t* lo = (int32_t*)(hb.mem + m.map_off);
    m.dev.leafof = lo;
    m.dev.bounds = lo + m.K;
    m.dev.nodes = (HssNode*)(hb.mem + m.node_off);
    m.dev.arena = (double*)(hb.mem + m.arena_off);
    m.dev.iarena = (int32_t*)(hb.mem + m.iarena_off);
    m.dev.K = m.K;
    m.dev.s = m.s;
    m.dev.sp = m.sp;
    m.dev.L = m.L;
  }
  return ADC_OK;
}

static adc_status batch_upload(adc_ctx c, HssBatch& hb) {
  // the host-written range of the batch memory, imaged and uploaded at once
  std::vector<char> img((size_t)hb.host_end, 0);
  char* h = img.data();
  const int64_t off_ms = (char*)hb.d_ms - hb.mem;
  for (size_t g = 0; g < hb.ms.size(); ++g) {
    const auto& m = hb.ms[g];
    std::memcpy(h + off_ms + g * sizeof(HssMerge), &m.dev, sizeof(HssMerge));
    std::memcpy(h + m.node_off, m.nodes.data(), m.nodes.size() * sizeof(HssNode));
    int32_t* lo = (int32_t*)(h + m.map_off);
    for (size_t t = 0; t + 1 < m.bounds.size(); ++t)
      for (int i = m.bounds[t]; i < m.bounds[t + 1]; ++i) lo[i] = (int32_t)t;
    std::memcpy(lo + m.K, m.bounds.data(), m.bounds.size() * 4);
  }
  return c->upload(hb.mem, h, img.size());
}

// Sampling and compression of every merge in the batch (omega already drawn).
// Direct sampling: every entry of the off-diagonal blocks generated and
// summed; Y and Z in one launch, the inner dimension split into segments
// until about six waves per SIMD are resident (each 64-row job is four
// waves), the segment partial sums added afterwards.
static adc_status sample_direct(adc_ctx c, HssBatch& hb) {
  hipStream_t st = c->stream;
  const int nm = (int)hb.ms.size();
  int64_t Ksum = 0;
  for (auto& m : hb.ms) Ksum += m.K;
  const int64_t waves = 2 * ((Ksum + 15) / 16);
  const int nseg = (int)std::max<int64_t>(1, std::min<int64_t>(8, (6144 + waves - 1) / waves));
  std::vector<SampleJob> sj;
  std::vector<int64_t> pb(nm, 0);
  int64_t ptot = 0;
  for (int g = 0; g < nm; ++g) {
    const auto& m = hb.ms[g];
    pb[g] = ptot;
    if (nseg > 1) ptot += (int64_t)2 * nseg * m.K * m.sp;
    for (int tr = 0; tr < 2; ++tr)
      for (int sg = 0; sg < nseg; ++sg)
        for (int r0 = 0; r0 < m.K; r0 += 64)
          for (int c0 = 0; c0 < m.sp; c0 += 128)
            sj.push_back(SampleJob{g, r0, c0, tr, sg, nseg, pb[g] + (int64_t)(tr * nseg + sg) * m.K * m.sp});
  }
  double* part = nullptr;
  if (nseg > 1) ADC_TRY(c->buffer(SLOT_HSS2, (size_t)ptot * 8 + 256, (void**)&part));
  void* dj;
  ADC_TRY(c->buffer(SLOT_SAMPLE_JOBS, sj.size() * sizeof(SampleJob) + 256, &dj));
  hb.sample_host.assign((const char*)sj.data(), (const char*)(sj.data() + sj.size()));
  ADC_TRY(c->upload(dj, hb.sample_host.data(), hb.sample_host.size()));
  // algorithmic flops of one sampling pass: the off-diagonal-block part of
  // Q' times s columns; bytes: Omega read, the samples written
  double sfl = 0.0, sby = 0.0;
  for (auto& m : hb.ms) {
    double dsq = 0.0;
    for (size_t i = 0; i + 1 < m.bounds.size(); ++i) dsq += (double)(m.bounds[i + 1] - m.bounds[i]) * (m.bounds[i + 1] - m.bounds[i]);
    sfl += 2.0 * m.s * ((double)m.K * m.K - dsq);
    sby += 16.0 * m.K * m.s;
  }
  c->ktimer.pre(st);
  hipLaunchKernelGGL(k_hss_sample, dim3((unsigned)sj.size()), dim3(256), 0, st, hb.d_ms, (const SampleJob*)dj, 1,
                     part);
  c->ktimer.post(st, KT_SAMPLE, 2.0 * sfl, 2.0 * sby);
  if (nseg > 1) {
    for (int g = 0; g < nm; ++g) {
      const auto& m = hb.ms[g];
      const int64_t n = (int64_t)m.K * m.sp;
      for (int tr = 0; tr < 2; ++tr)
        hipLaunchKernelGGL(k_sample_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                           (const double*)(part + pb[g] + (int64_t)tr * nseg * n), nseg, n,
                           tr ? m.dev.theta : m.dev.phi);
    }
  }
  HIP_OK(hipGetLastError());
  return ADC_OK;
}

// Fast Cauchy products (one-dimensional Chebyshev FMM over each merge's HSS
// tree): P2M at the leaves, M2M by height, M2L over the far lists, L2L by
// depth, then the leaves' local expansions and near fields.  Sides
// side_lo..side_hi (0: Phi-type, targets d; 1: Theta-type, targets lam).
// io[g] gives merge g's Omega, outputs and leading dimension sp (a multiple
// of 32); every job covers one (node, side, 32-column chunk).  `host` keeps
// the launch lists alive until the stream has consumed them.
static adc_status fmm_run(adc_ctx c, HssBatch& hb, std::vector<FmmIo>& io, int side_lo, int side_hi,
                          std::vector<char>& host, int kt_leaf) {
  hipStream_t st = c->stream;
  const int P = hb.fmm_p;
  const int nm = (int)hb.ms.size();
  int64_t tot = 0;
  int Lmax = 0;
  for (int g = 0; g < nm; ++g) {
    io[g].off = tot;
    tot += (int64_t)hb.ms[g].nodes.size() * 2 * P * io[g].sp;
    Lmax = std::max(Lmax, hb.ms[g].L);
  }
  double* W;
  ADC_TRY(c->buffer(SLOT_FMM, (size_t)(2 * tot) * 8 + 256, (void**)&W));
  double* F = W + tot;
  std::vector<int32_t> lists;
  std::vector<FmmJob> p2m, m2l, leaf;
  std::vector<std::vector<FmmJob>> m2m(Lmax + 1), l2l(Lmax + 1);
  double near_fl = 0.0, m2l_fl = 0.0;
  std::vector<std::vector<int32_t>> far, near;
  for (int g = 0; g < nm; ++g) {
    const auto& m = hb.ms[g];
    if ((int64_t)m.hd.size() != m.K || (int64_t)m.hg.size() != m.K || (int64_t)m.hmu.size() != m.K)
      return ADC_ERR_ARG;
    fmm_lists(m.hd.data(), m.hg.data(), m.hmu.data(), m.nodes, far, near);
    const int ncol = io[g].sp == m.sp ? m.s : io[g].sp;  // columns that carry data
    for (int q = 0; q < (int)m.nodes.size(); ++q) {
      const HssNode& nd = m.nodes[q];
      int l = 0;
      while ((2 << l) - 1 <= q) ++l;  // level of heap node q
      const int foff = (int)lists.size();
      lists.insert(lists.end(), far[q].begin(), far[q].end());
      const int noff = (int)lists.size();
      lists.insert(lists.end(), near[q].begin(), near[q].end());
      for (int side = side_lo; side <= side_hi; ++side)
        for (int c0 = 0; c0 < io[g].sp; c0 += 32) {
          if (nd.leaf) {
            p2m.push_back(FmmJob{g, q, side, c0, 0, 0});
            leaf.push_back(FmmJob{g, q, side, c0, noff, (int)near[q].size()});
          } else if (l >= 1) {
            m2m[m.L - l].push_back(FmmJob{g, q, side, c0, 0, 0});
          }
          if (l >= 1) m2l.push_back(FmmJob{g, q, side, c0, foff, (int)far[q].size()});
          if (l >= 2) l2l[l].push_back(FmmJob{g, q, side, c0, 0, 0});
        }
      const double sides = side_hi - side_lo + 1;
      for (int32_t sn : near[q]) near_fl += sides * 2.0 * ncol * (double)(nd.hi - nd.lo) * (m.nodes[sn].hi - m.nodes[sn].lo);
      m2l_fl += sides * 2.0 * ncol * (double)P * P * far[q].size();
    }
  }
  // one upload: operand descriptors, lists and every job array
  host.clear();
  auto put = [&](const void* src, size_t n) {
    const size_t o = host.size();
    host.resize((o + n + 255) & ~(size_t)255);
    if (n) std::memcpy(host.data() + o, src, n);
    return o;
  };
  const size_t o_io = put(io.data(), io.size() * sizeof(FmmIo));
  const size_t o_lists = put(lists.data(), lists.size() * sizeof(int32_t));
  const size_t o_p2m = put(p2m.data(), p2m.size() * sizeof(FmmJob));
  const size_t o_m2l = put(m2l.data(), m2l.size() * sizeof(FmmJob));
  const size_t o_leaf = put(leaf.data(), leaf.size() * sizeof(FmmJob));
  std::vector<size_t> o_m2m(Lmax + 1), o_l2l(Lmax + 1);
  for (int h = 0; h <= Lmax; ++h) o_m2m[h] = put(m2m[h].data(), m2m[h].size() * sizeof(FmmJob));
  for (int l = 0; l <= Lmax; ++l) o_l2l[l] = put(l2l[l].data(), l2l[l].size() * sizeof(FmmJob));
  void* dp;
  ADC_TRY(c->buffer(SLOT_SAMPLE_JOBS, host.size() + 256, &dp));
  char* dj = (char*)dp;
  ADC_TRY(c->upload(dj, host.data(), host.size()));
  const FmmIo* d_io = (const FmmIo*)(dj + o_io);
  const int32_t* d_lists = (const int32_t*)(dj + o_lists);
  if (!p2m.empty())
    hipLaunchKernelGGL(k_fmm_p2m, dim3((unsigned)p2m.size()), dim3(256), 0, st, hb.d_ms,
                       (const FmmJob*)(dj + o_p2m), d_io, P, W);
  for (int h = 1; h <= Lmax; ++h)
    if (!m2m[h].empty())
      hipLaunchKernelGGL(k_fmm_m2m, dim3((unsigned)m2m[h].size()), dim3(256), 0, st, hb.d_ms,
                         (const FmmJob*)(dj + o_m2m[h]), d_io, P, W);
  if (!m2l.empty()) {
    c->ktimer.pre(st);
    hipLaunchKernelGGL(k_fmm_m2l, dim3((unsigned)m2l.size()), dim3(256), 0, st, hb.d_ms,
                       (const FmmJob*)(dj + o_m2l), d_lists, d_io, P, (const double*)W, F);
    c->ktimer.post(st, KT_FMMM2L, m2l_fl, 0.0);
  }
  for (int l = 2; l <= Lmax; ++l)
    if (!l2l[l].empty())
      hipLaunchKernelGGL(k_fmm_l2l, dim3((unsigned)l2l[l].size()), dim3(256), 0, st, hb.d_ms,
                         (const FmmJob*)(dj + o_l2l[l]), d_io, P, F);
  if (kt_leaf >= 0) c->ktimer.pre(st);
  hipLaunchKernelGGL(k_fmm_leaf, dim3((unsigned)leaf.size()), dim3(128), 0, st, hb.d_ms,
                     (const FmmJob*)(dj + o_leaf), d_lists, d_io, P, (const double*)F);
  if (kt_leaf >= 0) c->ktimer.post(st, kt_leaf, near_fl, 0.0);
  HIP_OK(hipGetLastError());
  return ADC_OK;
}

static adc_status sample_fmm(adc_ctx c, HssBatch& hb) {
  std::vector<FmmIo> io(hb.ms.size());
  for (size_t g = 0; g < hb.ms.size(); ++g) {
    const auto& m = hb.ms[g];
    io[g] = FmmIo{m.dev.omega, {m.dev.phi, m.dev.theta}, 0, m.sp, 0};
  }
  return fmm_run(c, hb, io, 0, 1, hb.sample_host, KT_FMMLEAF);
}

static adc_status batch_sample(adc_ctx c, HssBatch& hb) {
  return hb.fmm_p > 0 ? sample_fmm(c, hb) : sample_direct(c, hb);
}

// Sampling and compression of every merge in the batch (omega already drawn).
static adc_status batch_construct(adc_ctx c, HssBatch& hb, adc_report* rep) {
  hipStream_t st = c->stream;
  const int nm = (int)hb.ms.size();
  ADC_TRY(batch_sample(c, hb));
  c->timer.mark(st, 5);
  if (hb.after_sampling) {
    hb.after_sampling();
    hb.after_sampling = nullptr;
  }
  // compression jobs per level
  int Lmax = 0;
  for (auto& m : hb.ms) Lmax = std::max(Lmax, m.L);
  // per level: the parents whose children's B blocks are generated first,
  // then one job per (non-root node, side)
  std::vector<std::vector<NodeJob>> lj(Lmax + 1), bj(Lmax + 1);
  int ncand_max = 0, sp_max = 0;
  for (int g = 0; g < nm; ++g) {
    const auto& m = hb.ms[g];
    sp_max = std::max(sp_max, m.sp);
    for (int l = 0; l <= m.L; ++l) {
      const int first = (1 << l) - 1;
      for (int q = 0; q < (1 << l); ++q) {
        const HssNode& nd = m.nodes[first + q];
        if (!nd.leaf) bj[l].push_back(NodeJob{g, first + q, 0, 0});
        if (l > 0) {
          lj[l].push_back(NodeJob{g, first + q, 0, 0});
          lj[l].push_back(NodeJob{g, first + q, 1, 0});
        }
        const int cand = nd.leaf ? nd.hi - nd.lo : std::min(2 * m.s, nd.hi - nd.lo);
        if (l > 0) ncand_max = std::max(ncand_max, cand);
      }
    }
  }
  size_t jbytes = 256 * (2 * Lmax + 3);
  for (auto& v : lj) jbytes += v.size() * sizeof(NodeJob);
  for (auto& v : bj) jbytes += v.size() * sizeof(NodeJob);
  void* dp;
  ADC_TRY(c->buffer(SLOT_HSS_JOBS, jbytes, &dp));
  char* dj = (char*)dp;
  std::vector<char> hj(jbytes);
  size_t off = 0;
  auto put = [&](const void* src, size_t n) {
    const size_t o = off;
    std::memcpy(hj.data() + off, src, n);
    off = (off + n + 255) & ~(size_t)255;
    return o;
  };
  std::vector<size_t> o_lj(Lmax + 1), o_bj(Lmax + 1);
  for (int l = 0; l <= Lmax; ++l) o_lj[l] = put(lj[l].data(), lj[l].size() * sizeof(NodeJob));
  for (int l = 0; l <= Lmax; ++l) o_bj[l] = put(bj[l].data(), bj[l].size() * sizeof(NodeJob));
  ADC_TRY(c->upload(dj, hj.data(), off));
  // dynamic LDS of every node job: its ID matrix when it fits (odd leading
  // dimension sp + 1), else the staging of its small products
  (void)ncand_max;
  (void)sp_max;
  const int lds = 18432;  // dynamic LDS doubles of a node job (144 KiB)
  static bool attr_set = false;
  if (!attr_set) {
    hipFuncSetAttribute((const void*)k_hss_compress, hipFuncAttributeMaxDynamicSharedMemorySize, lds * 8);
    attr_set = true;
  }
  for (int l = Lmax; l >= 0; --l) {
    if (!bj[l].empty())
      hipLaunchKernelGGL(k_hss_bblocks, dim3((unsigned)bj[l].size()), dim3(256), 0, st, hb.d_ms,
                         (const NodeJob*)(dj + o_bj[l]));
    if (lj[l].empty()) continue;
    c->ktimer.pre(st);
    hipLaunchKernelGGL(k_hss_compress, dim3((unsigned)lj[l].size()), dim3(1024), (size_t)lds * 8, st, hb.d_ms,
                       (const NodeJob*)(dj + o_lj[l]), lds);
    c->ktimer.post(st, KT_COMPRESS, 0.0, 0.0);
    HIP_OK(hipGetLastError());
  }
  c->timer.mark(st, 6);
  // ranks back to the host: the node tables of every merge in one copy
  // through a pinned buffer
  const int64_t n0 = hb.ms.empty() ? 0 : hb.ms[0].node_off;
  char* hp;
  ADC_TRY(c->stage2((size_t)(hb.nodes_end - n0) + 256, (void**)&hp));
  if (hb.nodes_end > n0)
    HIP_OK(hipMemcpyAsync(hp, hb.mem + n0, (size_t)(hb.nodes_end - n0), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  for (auto& m : hb.ms) std::memcpy(m.nodes.data(), hp + (m.node_off - n0), m.nodes.size() * sizeof(HssNode));
  (void)rep;
  for (auto& m : hb.ms) {
    m.max_rank = 0;
    m.sat = 0;
    for (size_t i = 1; i < m.nodes.size(); ++i) {
      const HssNode& nd = m.nodes[i];
      m.max_rank = std::max({m.max_rank, nd.kr, nd.kc});
      m.sat += (nd.kr >= m.s && nd.nr > m.s) || (nd.kc >= m.s && nd.nc > m.s);
    }
  }
  return ADC_OK;
}

// ---------------------------------------------------------------------------
// Algorithm 3 for a list of (merge, X, P, output) products.
struct ApplyJob {
  int g;              // merge in the batch
  const double* X;    // P x K, column-major, ld ldx
  int64_t ldx;
  int P;
  double* C;          // output columns: C + colmap[j] * ldc (colmap may be null)
  int64_t ldc;
  const int32_t* colmap;
  // -1: X's columns in index order; 0 / 1: X holds the top / bottom rows of a
  // solver merge's packed operand, columns leaf-grouped (HssMerge::perm)
  int half = -1;
};

static void push_prob(std::vector<GemmProb>& v, const GemmProb& p) { v.push_back(p); }

// Problem lists of one Algorithm 3 run: pinned host and device arrays filled
// front to back, so that no launch waits for the previous one's descriptors.
struct ProbArena {
  GemmProb* h = nullptr;
  GemmProb* d = nullptr;
  size_t cap = 0, used = 0;
  struct Launch {
    int cls;      // 0: 64-wide tiles, 1: 96, 2: 128
    size_t off;   // first problem in the arena
    int count, tiles;
    double flops, bytes;
  };
  std::vector<Launch> launches;  // in order of issue
  size_t uploaded = 0, issued = 0;  // problems uploaded, launches issued
};

// Upload the problems staged since the last issue (one copy) and launch the
// staged groups in order.
static adc_status issue_probs(adc_ctx c, ProbArena& ar) {
  hipStream_t st = c->stream;
  if (ar.used > ar.uploaded)
    ADC_TRY(c->upload(ar.d + ar.uploaded, ar.h + ar.uploaded, (ar.used - ar.uploaded) * sizeof(GemmProb)));
  ar.uploaded = ar.used;
  for (; ar.issued < ar.launches.size(); ++ar.issued) {
    const auto& l = ar.launches[ar.issued];
    const GemmProb* dp = ar.d + l.off;
    c->ktimer.pre(st);
    if (l.cls == 0)
      hipLaunchKernelGGL(k_gemm_f64_n64, dim3(l.tiles), dim3(512), 0, st, dp, l.count);
    else if (l.cls == 1)
      hipLaunchKernelGGL(k_gemm_f64_n96, dim3(l.tiles), dim3(512), 0, st, dp, l.count);
    else
      hipLaunchKernelGGL(k_gemm_f64, dim3(l.tiles), dim3(512), 0, st, dp, l.count);
    c->ktimer.post(st, l.cls == 0 ? KT_GEMM64 : l.cls == 1 ? KT_GEMM96 : KT_GEMM, l.flops, l.bytes);
  }
  HIP_OK(hipGetLastError());
  return ADC_OK;
}

// Stage one group of independent products (split by tile width), issued at
// once with now, else at the next issue_probs.
static adc_status launch_probs(adc_ctx c, std::vector<GemmProb>& probs, double* flops, ProbArena& ar,
                               bool now) {
  if (probs.empty()) return now ? issue_probs(c, ar) : ADC_OK;
  // tile width by the product width: 64, 96 or 128 columns
  std::vector<GemmProb> cls[3];
  double pf[3] = {0.0, 0.0, 0.0}, pb[3] = {0.0, 0.0, 0.0};
  for (auto& p : probs) {
    if (p.M <= 0 || p.N <= 0) continue;
    const double f = 2.0 * p.M * (double)p.N * (p.K + p.K2);
    const double by = 8.0 * ((double)p.M * (p.K + p.K2) + (double)(p.K + p.K2) * p.N +
                             (double)p.M * p.N * (p.beta != 0.0 ? 2 : 1));
    if (flops) *flops += f;
    const int w = (p.N <= 64) ? 0 : (p.N <= 96) ? 1 : 2;
    pf[w] += f;
    pb[w] += by;
    cls[w].push_back(p);
  }
  static const int BN[3] = {64, 96, 128};
  for (int w = 0; w < 3; ++w) {
    auto& L = cls[w];
    if (L.empty()) continue;
    const int bn = BN[w];
    int tiles = 0;
    for (auto& p : L) {
      p.tiles_m = (p.M + 127) / 128;
      p.tile0 = tiles;
      tiles += p.tiles_m * ((p.N + bn - 1) / bn);
    }
    if (ar.used + L.size() > ar.cap) return ADC_ERR_UNSUPPORTED;  // sized by the caller
    std::memcpy(ar.h + ar.used, L.data(), L.size() * sizeof(GemmProb));
    ar.launches.push_back(ProbArena::Launch{w, ar.used, (int)L.size(), tiles, pf[w], pb[w]});
    ar.used += L.size();
  }
  return now ? issue_probs(c, ar) : ADC_OK;
}

static adc_status batch_apply(adc_ctx c, HssBatch& hb, const std::vector<ApplyJob>& jobs, double* flops) {
  hipStream_t st = c->stream;
  // storage: per job and level, G (P x sum kr) and F (P x sum kc); leaf D blocks
  struct Lay {
    std::vector<int64_t> goff, foff;  // per node: column offset inside its level block
    std::vector<int64_t> lev_g, lev_f;  // per level: element offset of the level block
  };
  std::vector<Lay> lays(jobs.size());
  int64_t total = 0;
  // leaf data once per (merge, flavour): D_i for jobs in index order (0), and
  // D_i and U_i with rows in the leaf-grouped order for grouped jobs (1)
  std::vector<int2> lj[2];
  std::vector<int64_t> doff[2], uoff;
  std::vector<int64_t> leaf_base(2 * hb.ms.size(), -1);
  int64_t dtotal = 0, utotal = 0;
  for (size_t t = 0; t < jobs.size(); ++t) {
    const int flav = jobs[t].half >= 0 ? 1 : 0;
    const auto& m = hb.ms[jobs[t].g];
    Lay& ly = lays[t];
    const int nn = (int)m.nodes.size();
    ly.goff.assign(nn, 0);
    ly.foff.assign(nn, 0);
    ly.lev_g.assign(m.L + 1, 0);
    ly.lev_f.assign(m.L + 1, 0);
    for (int l = 1; l <= m.L; ++l) {
      int64_t sg = 0, sf = 0;
      for (int q = (1 << l) - 1; q < (1 << (l + 1)) - 1; ++q) {
        ly.goff[q] = sg;
        ly.foff[q] = sf;
        sg += m.nodes[q].kr;
        sf += m.nodes[q].kc;
      }
      ly.lev_g[l] = total;
      total += sg * jobs[t].P;
      ly.lev_f[l] = total;
      total += sf * jobs[t].P;
    }
    int64_t& lb = leaf_base[2 * jobs[t].g + flav];
    if (lb >= 0) continue;
    lb = (int64_t)lj[flav].size();
    if (flav && ((int)m.grp.size() != 3 * (1 << m.L) || !m.dev.perm)) return ADC_ERR_ARG;
    for (int q = (1 << m.L) - 1; q < (1 << (m.L + 1)) - 1; ++q) {
      const int mm = m.nodes[q].hi - m.nodes[q].lo;
      lj[flav].push_back(int2{jobs[t].g, q});
      doff[flav].push_back(dtotal);
      dtotal += (int64_t)mm * mm;
      if (flav) {
        uoff.push_back(utotal);
        utotal += (int64_t)mm * m.nodes[q].kr;
      }
    }
  }
  // W_q = B_sib(q) V_q^T (kr(sib) x nc_q, column-major) for every node q
  // strictly between the root and the leaves, once per merge: the downsweep
  // then forms the blocks its children receive from above in one product,
  // E_c = [G_sib(q) E_q] [W_q; V_q^T] (columns of c), where E_q is what q
  // received (zero below the root)
  std::vector<std::vector<int64_t>> woff(hb.ms.size());
  int64_t wtotal = 0;
  for (size_t t = 0; t < jobs.size(); ++t) {
    const auto& m = hb.ms[jobs[t].g];
    auto& wo = woff[jobs[t].g];
    if (!wo.empty()) continue;
    wo.assign(m.nodes.size(), -1);
    for (int q = 1; q < (1 << m.L) - 1; ++q) {
      const int sib = (q & 1) ? q + 1 : q - 1;
      wo[q] = wtotal;
      wtotal += (int64_t)m.nodes[sib].kr * m.nodes[q].nc;
    }
  }
  void* wp;
  auto rup = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t lj_bytes = rup(lj[0].size() * sizeof(int2)) + rup(lj[1].size() * sizeof(int2));
  const size_t of_bytes = rup(doff[0].size() * 8) + rup(doff[1].size() * 8) + rup(uoff.size() * 8);
  ADC_TRY(c->buffer(SLOT_HSS2, (size_t)(total + dtotal + utotal + wtotal) * 8 + lj_bytes + of_bytes + 1024, &wp));
  double* work = (double*)wp;
  double* dmat = work + total;
  double* uperm = dmat + dtotal;
  double* wmat = uperm + utotal;
  char* tail = (char*)(wmat + wtotal);
  int2* d_lj[2];
  int64_t* d_doff[2];
  d_lj[0] = (int2*)tail;
  d_lj[1] = (int2*)(tail + rup(lj[0].size() * sizeof(int2)));
  char* t2 = tail + lj_bytes;
  d_doff[0] = (int64_t*)t2;
  d_doff[1] = (int64_t*)(t2 + rup(doff[0].size() * 8));
  int64_t* d_uoff = (int64_t*)(t2 + rup(doff[0].size() * 8) + rup(doff[1].size() * 8));
  // D_i of both flavours and the grouped U_i
  for (int f = 0; f < 2; ++f) {
    if (lj[f].empty()) continue;
    ADC_TRY(c->upload(d_lj[f], lj[f].data(), lj[f].size() * sizeof(int2)));
    ADC_TRY(c->upload(d_doff[f], doff[f].data(), doff[f].size() * 8));
    hipLaunchKernelGGL(k_hss_dmat, dim3((unsigned)lj[f].size()), dim3(256), 0, st, hb.d_ms, d_lj[f], dmat,
                       d_doff[f], f);
  }
  if (!lj[1].empty()) {
    ADC_TRY(c->upload(d_uoff, uoff.data(), uoff.size() * 8));
    hipLaunchKernelGGL(k_hss_urows, dim3((unsigned)lj[1].size()), dim3(256), 0, st, hb.d_ms, d_lj[1], uperm,
                       d_uoff);
  }
  HIP_OK(hipGetLastError());
  auto dmat_of = [&](const ApplyJob& J, int li) {
    const int f = J.half >= 0 ? 1 : 0;
    return dmat + doff[f][leaf_base[2 * J.g + f] + li];
  };
  // the leaf column range of a grouped job: top rows meet top-only and both,
  // bottom rows both and bottom-only
  auto leaf_range = [&](const ApplyJob& J, int li, int& kb, int& kl) {
    const int32_t* gc = hb.ms[J.g].grp.data() + 3 * li;
    kb = J.half == 0 ? 0 : gc[0];
    kl = J.half == 0 ? gc[0] + gc[1] : gc[1] + gc[2];
  };

  int Lmax = 0;
  size_t nodes_all = 0;
  for (auto& j : jobs) {
    Lmax = std::max(Lmax, hb.ms[j.g].L);
    nodes_all += hb.ms[j.g].nodes.size();
  }
  // every node appears in at most one W product, one problem of the
  // upsweep, one of the downsweep and one of the leaf step
  ProbArena ar;
  std::vector<GemmProb> hprobs;
  ar.cap = 4 * nodes_all + 64;
  {
    void* dbuf;
    ADC_TRY(c->buffer(SLOT_GEMM_A, ar.cap * sizeof(GemmProb) + 256, &dbuf));
    hprobs.resize(ar.cap);
    ar.h = hprobs.data();
    ar.d = (GemmProb*)dbuf;
  }
  std::vector<GemmProb> probs;
  auto G = [&](size_t t, int node) {
    const auto& m = hb.ms[jobs[t].g];
    int l = 0;
    while ((1 << (l + 1)) - 1 <= node) ++l;
    (void)m;
    return work + lays[t].lev_g[l] + lays[t].goff[node] * jobs[t].P;
  };
  auto F = [&](size_t t, int node) {
    int l = 0;
    while ((1 << (l + 1)) - 1 <= node) ++l;
    return work + lays[t].lev_f[l] + lays[t].foff[node] * jobs[t].P;
  };
  // the W_q products, in the first launch group
  probs.clear();
  for (size_t g = 0; g < hb.ms.size(); ++g) {
    if (woff[g].empty()) continue;
    const auto& m = hb.ms[g];
    for (int q = 1; q < (1 << m.L) - 1; ++q) {
      const int sib = (q & 1) ? q + 1 : q - 1;
      const HssNode& nd = m.nodes[q];
      const HssNode& sj = m.nodes[sib];
      GemmProb p{};
      p.M = sj.kr;
      p.N = nd.nc;
      p.K = nd.kc;
      p.A = m.dev.arena + sj.offB;  // kr(sib) x kc(q)
      p.lda = std::max(sj.kr, 1);
      p.B = m.dev.arena + nd.offV;  // nc x kc, read transposed
      p.ldb = std::max(nd.nc, 1);
      p.transB = 1;
      p.C = wmat + woff[g][q];
      p.ldc = std::max(sj.kr, 1);
      push_prob(probs, p);
    }
  }
  std::vector<GemmProb> wprobs;
  wprobs.swap(probs);
  // upsweep
  for (int l = Lmax; l >= 1; --l) {
    probs.clear();
    if (l == Lmax) probs.swap(wprobs);
    for (size_t t = 0; t < jobs.size(); ++t) {
      const auto& m = hb.ms[jobs[t].g];
      if (l > m.L) continue;
      const ApplyJob& J = jobs[t];
      for (int q = (1 << l) - 1; q < (1 << (l + 1)) - 1; ++q) {
        const HssNode& nd = m.nodes[q];
        GemmProb p{};
        p.M = J.P;
        p.N = nd.kr;
        p.C = G(t, q);
        p.ldc = J.P;
        p.B = m.dev.arena + nd.offU;
        p.ldb = nd.nr;
        if (nd.leaf && J.half >= 0) {
          const int li = q - ((1 << m.L) - 1);
          int kb, kl;
          leaf_range(J, li, kb, kl);
          p.A = J.X + (int64_t)(nd.lo + kb) * J.ldx;
          p.lda = J.ldx;
          p.K = kl;
          p.B = uperm + uoff[leaf_base[2 * J.g + 1] + li] + kb;
          p.ldb = nd.hi - nd.lo;
        } else if (nd.leaf) {
          p.A = J.X + (int64_t)nd.lo * J.ldx;
          p.lda = J.ldx;
          p.K = nd.hi - nd.lo;
        } else {
          p.A = G(t, 2 * q + 1);  // [G_i1 G_i2] are adjacent
          p.lda = J.P;
          p.K = m.nodes[2 * q + 1].kr + m.nodes[2 * q + 2].kr;
        }
        push_prob(probs, p);
      }
    }
    // the first group at once (the GPU starts on it while the host builds
    // the others), the rest staged and issued together after the leaf step's
    // group: one upload, and the launches queued back to back
    ADC_TRY(launch_probs(c, probs, flops, ar, l == Lmax));
  }
  // downsweep, one launch per level l: for every node q at level l above
  // the leaves, its children's incoming blocks [E_c1 E_c2] = [G_sib(q) E_q]
  // [W_q; V_q^T] (E_q = 0 at level 1); at the leaf level, F_i = G_sib(i)
  // B_sib(i) + E_i, which the leaf step multiplies by V_i^T
  for (int l = 1; l <= Lmax; ++l) {
    probs.clear();
    for (size_t t = 0; t < jobs.size(); ++t) {
      const auto& m = hb.ms[jobs[t].g];
      if (l > m.L) continue;
      const ApplyJob& J = jobs[t];
      for (int q = (1 << l) - 1; q < (1 << (l + 1)) - 1; ++q) {
        const HssNode& nd = m.nodes[q];
        const int sib = (q & 1) ? q + 1 : q - 1;
        const HssNode& sj = m.nodes[sib];
        GemmProb p{};
        p.M = J.P;
        p.A = G(t, sib);
        p.lda = J.P;
        p.K = sj.kr;
        if (l < m.L) {
          p.N = nd.nc;  // kc(c1) + kc(c2)
          p.B = wmat + woff[J.g][q];
          p.ldb = std::max(sj.kr, 1);
          if (l > 1) {
            p.A2 = F(t, q);
            p.lda2 = J.P;
            p.K2 = nd.kc;
            p.B2 = m.dev.arena + nd.offV;  // nc x kc, read transposed
            p.ldb2 = std::max(nd.nc, 1);
            p.transB2 = 1;
          }
          p.C = F(t, 2 * q + 1);  // [E_c1 E_c2] are adjacent
        } else {
          p.N = nd.kc;
          p.B = m.dev.arena + sj.offB;  // kr(sib) x kc(i)
          p.ldb = std::max(sj.kr, 1);
          p.C = F(t, q);
          p.beta = (l > 1) ? 1.0 : 0.0;
        }
        p.ldc = J.P;
        push_prob(probs, p);
      }
    }
    ADC_TRY(launch_probs(c, probs, flops, ar, false));
  }
  // leaves: out(:, t_i) = X(:, t_i) D_i + H_i V_i^T
  probs.clear();
  for (size_t t = 0; t < jobs.size(); ++t) {
    const auto& m = hb.ms[jobs[t].g];
    const ApplyJob& J = jobs[t];
    int li = 0;
    for (int q = (1 << m.L) - 1; q < (1 << (m.L + 1)) - 1; ++q, ++li) {
      const HssNode& nd = m.nodes[q];
      const int mm = nd.hi - nd.lo;
      GemmProb p{};
      p.M = J.P;
      p.N = mm;
      p.K = mm;
      p.A = J.X + (int64_t)nd.lo * J.ldx;
      p.lda = J.ldx;
      p.B = dmat_of(J, li);
      p.ldb = mm;
      if (J.half >= 0) {
        int kb, kl;
        leaf_range(J, li, kb, kl);
        p.A = J.X + (int64_t)(nd.lo + kb) * J.ldx;
        p.K = kl;
        p.B += kb;
      }
      if (m.L > 0) {
        p.K2 = nd.kc;
        p.A2 = F(t, q);
        p.lda2 = J.P;
        p.B2 = m.dev.arena + nd.offV;  // mm x kc, read transposed
        p.ldb2 = mm;
        p.transB2 = 1;
      }
      if (J.colmap) {
        p.C = J.C;
        p.colmap = J.colmap + nd.lo;
      } else {
        p.C = J.C + (int64_t)nd.lo * J.ldc;
      }
      p.ldc = J.ldc;
      push_prob(probs, p);
    }
  }
  ADC_TRY(launch_probs(c, probs, flops, ar, true));
  return ADC_OK;
}

// Draw Omega for merge g of the batch (stream id of the merge, 2*id).
static void draw_omega(adc_ctx c, const HssBatch::One& m, uint64_t seed) {
  const int64_t n = (int64_t)m.K * m.sp;
  hipLaunchKernelGGL(k_philox_normal, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, m.dev.omega,
                     (int64_t)m.K, m.s, m.sp, seed, 2u * m.stream);
}

// Accuracy check of every merge: err = ||W^T (Q' - H)||_F / ||W^T Q'||_F for
// nprobe Gaussian probes (stream 2*id + 1).  In three parts so that the
// probe products W^T H can share the launches of another HSS product:
// check_prepare draws W, forms W^T Q' and appends one ApplyJob per merge
// (W H into the check buffer); after those jobs have run, check_finish
// reduces the norms and sets err and pass.
struct CheckBufs {
  double* buf = nullptr;
  double* npart = nullptr;
  double* norms = nullptr;
  std::vector<int64_t> base;
};
constexpr int CHECK_NBLK = 128;  // blocks of the norm partial sums

static adc_status check_prepare(adc_ctx c, HssBatch& hb, const adc_opts& o, CheckBufs& cb,
                                std::vector<ApplyJob>& aj, hipStream_t st) {
  const int nm = (int)hb.ms.size();
  int64_t tot = 0, part_max = 0;
  cb.base.assign(nm, 0);
  std::vector<int> nseg(nm);
  for (int g = 0; g < nm; ++g) {
    cb.base[g] = tot;
    const int K = hb.ms[g].K;
    tot += 3 * (int64_t)K * SP_PROBE;
    // row segments so that a launch has about 2048 single-wave workgroups
    nseg[g] = std::max(1, std::min(64, (2048 + (K + 63) / 64 - 1) / ((K + 63) / 64)));
    part_max = std::max(part_max, (int64_t)nseg[g] * K * 8);
  }
  void* p;
  ADC_TRY(c->buffer(SLOT_HSS_CHECK, (size_t)(tot + part_max + 2 * CHECK_NBLK * nm) * 8 + nm * 16 + 1024, &p));
  cb.buf = (double*)p;
  double* part = cb.buf + tot;
  cb.npart = part + part_max;
  cb.norms = cb.npart + 2 * CHECK_NBLK * nm;
  for (int g = 0; g < nm; ++g) {
    auto& m = hb.ms[g];
    double* W = cb.buf + cb.base[g];
    double* WQ = W + (int64_t)m.K * SP_PROBE;
    double* WH = WQ + (int64_t)m.K * SP_PROBE;
    const int64_t n = (int64_t)m.K * SP_PROBE;
    hipLaunchKernelGGL(k_philox_normal, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, W, (int64_t)m.K,
                       o.nprobe, SP_PROBE, o.seed, 2u * m.stream + 1u);
    aj.push_back(ApplyJob{g, W, SP_PROBE, SP_PROBE, WH, SP_PROBE, nullptr});
  }
  // W^T Q' per merge: FP64 vector kernel over the generated entries (four
  // probes do not fill a matrix-core tile), then the padding columns zeroed.
  // (The FMM of the sampling, with diagonal blocks, was measured slower here:
  // its per-level launch chain outweighs the 4-column direct product.)
  for (int g = 0; g < nm; ++g) {
    auto& m = hb.ms[g];
    double* W = cb.buf + cb.base[g];
    double* WQ = W + (int64_t)m.K * SP_PROBE;
    const int ntj = (m.K + 63) / 64;
    for (int c0 = 0; c0 < o.nprobe; c0 += 8) {
      const int nc = std::min(8, o.nprobe - c0);
      if (nc <= 4)
        hipLaunchKernelGGL(k_probe_qt<4>, dim3((unsigned)(ntj * nseg[g])), dim3(64), 0, st, hb.d_ms, g,
                           (const double*)W, SP_PROBE, c0, nc, nseg[g], part);
      else
        hipLaunchKernelGGL(k_probe_qt<8>, dim3((unsigned)(ntj * nseg[g])), dim3(64), 0, st, hb.d_ms, g,
                           (const double*)W, SP_PROBE, c0, nc, nseg[g], part);
      hipLaunchKernelGGL(k_probe_sum, dim3((unsigned)(((int64_t)m.K * SP_PROBE + 255) / 256)), dim3(256), 0, st,
                         (const double*)part, m.K, nseg[g], c0, nc, o.nprobe, WQ, SP_PROBE);
    }
    HIP_OK(hipGetLastError());
  }
  return ADC_OK;
}

static adc_status check_finish(adc_ctx c, HssBatch& hb, const adc_opts& o, const CheckBufs& cb) {
  hipStream_t st = c->stream;
  const int nm = (int)hb.ms.size();
  for (int g = 0; g < nm; ++g) {
    double* W = cb.buf + cb.base[g];
    double* WQ = W + (int64_t)hb.ms[g].K * SP_PROBE;
    double* WH = WQ + (int64_t)hb.ms[g].K * SP_PROBE;
    hipLaunchKernelGGL(k_diff_norms, dim3(CHECK_NBLK), dim3(256), 0, st, WH, WQ, (int64_t)hb.ms[g].K, SP_PROBE,
                       o.nprobe, cb.npart + 2 * CHECK_NBLK * g);
    hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(64), 0, st, (const double*)(cb.npart + 2 * CHECK_NBLK * g),
                       CHECK_NBLK, cb.norms + 2 * g);
  }
  HIP_OK(hipGetLastError());
  std::vector<double> hn(2 * nm);
  HIP_OK(hipMemcpyAsync(hn.data(), cb.norms, 2 * nm * 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  for (int g = 0; g < nm; ++g) {
    auto& m = hb.ms[g];
    m.err = (hn[2 * g + 1] > 0.0) ? std::sqrt(hn[2 * g] / hn[2 * g + 1]) : 0.0;
    m.pass = std::isfinite(m.err) && m.err <= o.check_tol && !(o.sat_guard && m.sat > 0);
  }
  return ADC_OK;
}

static adc_status batch_check(adc_ctx c, HssBatch& hb, const adc_opts& o, double* flops) {
  CheckBufs cb;
  std::vector<ApplyJob> aj;
  ADC_TRY(check_prepare(c, hb, o, cb, aj, c->stream));
  ADC_TRY(batch_apply(c, hb, aj, flops));
  return check_finish(c, hb, o, cb);
}

// One attempt for every merge of the batch with its current s: storage,
// Omega, sampling, compression and (if asked) the accuracy check.
static adc_status batch_attempt(adc_ctx c, HssBatch& hb, const adc_opts& o, int slot, bool check, adc_report* rep,
                                double* flops, const std::vector<const double*>* omega_given) {
  ADC_TRY(batch_alloc(c, hb, slot));
  ADC_TRY(batch_upload(c, hb));
  for (size_t g = 0; g < hb.ms.size(); ++g) {
    auto& m = hb.ms[g];
    if (omega_given && (*omega_given)[g]) {
      // caller's K x s row-major Omega into the padded layout
      HIP_OK(hipMemset2DAsync(m.dev.omega, m.sp * 8, 0, m.sp * 8, m.K, c->stream));
      HIP_OK(hipMemcpy2DAsync(m.dev.omega, m.sp * 8, (*omega_given)[g], m.s * 8, m.s * 8, m.K,
                              hipMemcpyDeviceToDevice, c->stream));
    } else {
      draw_omega(c, m, o.seed);
    }
  }
  HIP_OK(hipGetLastError());
  ADC_TRY(batch_construct(c, hb, rep));
  if (!check) {
    for (auto& m : hb.ms) m.pass = true;
    return ADC_OK;
  }
  ADC_TRY(batch_check(c, hb, o, flops));
  c->timer.mark(c->stream, 7);
  return ADC_OK;
}

// Double the samples of the failing merges; false when none can grow.
static bool grow_failing(HssBatch& hb) {
  bool any = false;
  for (auto& m : hb.ms) {
    if (!m.pass && m.s < std::min(m.K, S_MAX)) {
      m.s = std::min({2 * m.s, m.K, S_MAX});
      m.sp = (m.s + 31) / 32 * 32;
      m.retries++;
      any = true;
    }
  }
  return any;
}

// The first sample count of every merge: estimated rank plus oversampling.
static void batch_init_s(HssBatch& hb, const adc_opts& o) {
  for (auto& m : hb.ms) {
    m.s = std::min({m.K, m.r + o.oversample, S_MAX});
    m.s = std::max(m.s, 1);
    m.sp = (m.s + 31) / 32 * 32;
    m.retries = 0;
  }
}

// Retries after the first check of `hb`.  Without `rb` a retry rebuilds the
// whole batch in place.  With `rb`, the merges that passed keep their HSS
// forms in `hb`; the ones that failed move to `rb` (own storage) and only they
// are rebuilt with doubled samples; rb_of[g] is the merge's index in `rb`,
// -1 for the merges that stay in `hb`.
static adc_status batch_retry(adc_ctx c, HssBatch& hb, const adc_opts& o, adc_report* rep, double* flops,
                              const std::vector<const double*>* omega_given, HssBatch* rb = nullptr,
                              std::vector<int>* rb_of = nullptr) {
  if (rb_of) rb_of->assign(hb.ms.size(), -1);
  if (rb) {
    rb->ms.clear();
    rb->fmm_p = hb.fmm_p;
  }
  for (int attempt = 1; attempt <= o.max_retries; ++attempt) {
    if (!rb || attempt == 1) {
      // first retry (or every retry in place): the failing merges of hb
      if (!grow_failing(hb)) return ADC_OK;
      if (!rb) {
        ADC_TRY(batch_attempt(c, hb, o, SLOT_HSS, true, rep, flops, omega_given));
        continue;
      }
      for (size_t g = 0; g < hb.ms.size(); ++g) {
        if (hb.ms[g].pass) continue;
        (*rb_of)[g] = (int)rb->ms.size();
        rb->ms.push_back(hb.ms[g]);
      }
    } else if (!grow_failing(*rb)) {
      return ADC_OK;
    }
    ADC_TRY(batch_attempt(c, *rb, o, SLOT_HSS_RETRY, true, rep, flops, nullptr));
    bool all = true;
    for (auto& m : rb->ms) all = all && m.pass;
    if (all) return ADC_OK;
  }
  return ADC_OK;
}

// Build (construct + check + retries in place) for a batch whose merges have
// K, L, bounds, r and stream set.
static adc_status batch_build(adc_ctx c, HssBatch& hb, const adc_opts& o, bool check, adc_report* rep,
                              double* flops, const std::vector<const double*>* omega_given) {
  batch_init_s(hb, o);
  ADC_TRY(batch_attempt(c, hb, o, SLOT_HSS, check, rep, flops, omega_given));
  if (!check) return ADC_OK;
  return batch_retry(c, hb, o, rep, flops, omega_given);
}

// The update product of one solver merge: the top and bottom rows of the
// packed operand, each against its leaf column ranges (columns grouped by row
// support inside leaves).
static void push_update_jobs(std::vector<ApplyJob>& aj, int g, const MergeDev& M, const LevelBufs& B) {
  aj.push_back(ApplyJob{g, B.pk + M.zoff, (int64_t)M.n, M.n1, M.zn, M.ldn, B.posR + M.s0, 0});
  aj.push_back(ApplyJob{g, B.pk + M.zoff + M.n1, (int64_t)M.n, M.n - M.n1, M.zn + M.n1, M.ldn, B.posR + M.s0, 1});
}

// ---------------------------------------------------------------------------
adc_status hss_level_update(adc_ctx c, const adc_opts& o, MergeDev* h_m, MergeDev* d_m, int nm,
                            const LevelBufs& B, int depth, adc_report* rep, double* flops, double* bytes,
                            const std::function<void()>& after_sampling, hipEvent_t operand_ready) {
  (void)bytes;
  hipStream_t st = c->stream;
  HssBatch hb;
  std::vector<int> which;
  for (int g = 0; g < nm; ++g)
    if (h_m[g].mode == 1) which.push_back(g);
  if (which.empty()) return ADC_OK;
  // the host inputs of every merge (leaf bounds moved on the device, d, gam,
  // mu, the column groups of every leaf of the packed operand, the rank
  // estimate) read back through one pinned buffer: each kind of array is
  // copied once over the range that holds every merge's part, so that the
  // number of copies does not grow with the number of merges
  int64_t lo = INT64_MAX, hi = 0, lhi = 0;
  const char *blo = nullptr, *bhi = nullptr;
  for (int g : which) {
    const MergeDev& M = h_m[g];
    const int L = std::max(1, ceil_log2_ratio(M.K, o.hss_leaf));
    if (M.nleaf != (1 << L) || !M.lbounds) return ADC_ERR_ARG;
    lo = std::min(lo, M.s0);
    hi = std::max(hi, M.s0 + M.K);
    lhi = std::max(lhi, M.s0 + 3 * (int64_t)M.nleaf);
    const char* b0 = (const char*)M.lbounds;
    const char* b1 = b0 + (size_t)(M.nleaf + 1) * 4;
    blo = blo ? std::min(blo, b0) : b0;
    bhi = bhi ? std::max(bhi, b1) : b1;
  }
  const size_t nv = (size_t)(hi - lo), nl = (size_t)(lhi - lo), nbd = (size_t)(bhi - blo);
  const size_t o_gam = ((nv * 8 + 255) & ~(size_t)255), o_mu = 2 * o_gam, o_l = 3 * o_gam;
  const size_t o_b = o_l + ((nl * 4 + 255) & ~(size_t)255);
  const size_t o_m = o_b + ((nbd + 255) & ~(size_t)255);
  char* hp;
  ADC_TRY(c->stage2(o_m + nm * sizeof(MergeDev), (void**)&hp));
  HIP_OK(hipMemcpyAsync(hp, B.dS + lo, nv * 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(hp + o_gam, B.gam + lo, nv * 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(hp + o_mu, B.mu + lo, nv * 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(hp + o_l, B.lcnt + lo, nl * 4, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(hp + o_b, blo, nbd, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(hp + o_m, d_m, nm * sizeof(MergeDev), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  c->up_reset();  // every earlier upload on the stream has completed
  const MergeDev* hm_dev = (const MergeDev*)(hp + o_m);
  for (size_t t = 0; t < which.size(); ++t) {
    const MergeDev& M = h_m[which[t]];
    HssBatch::One m;
    m.K = M.K;
    m.L = std::max(1, ceil_log2_ratio(M.K, o.hss_leaf));
    const size_t e0 = (size_t)(M.s0 - lo);
    const double* qd = (const double*)hp + e0;
    const double* qg = (const double*)(hp + o_gam) + e0;
    const double* qm = (const double*)(hp + o_mu) + e0;
    const int32_t* ql = (const int32_t*)(hp + o_l) + e0;
    const int32_t* qb = (const int32_t*)(hp + o_b + ((const char*)M.lbounds - blo));
    m.bounds.assign(qb, qb + M.nleaf + 1);
    m.grp.assign(ql, ql + 3 * (size_t)M.nleaf);
    m.stream = (uint32_t)((depth << 20) + which[t]);
    std::vector<double> d(qd, qd + M.K), g2(qg, qg + M.K), mu(qm, qm + M.K);
    m.r = hm_dev[which[t]].rest;  // k_leaf_bounds: eq. (bounds) over the moved boundaries
    if (o.rank_mode == ADC_RANK_FIXED) m.r = std::max(1, o.fixed_rank);
    if (o.rank_mode == ADC_RANK_MLP && !mlp_collecting(c))
      m.r = mlp_rank(c, B.dS + M.s0, B.gam + M.s0, B.mu + M.s0, M.K, m.bounds, o, m.r);
    m.dev.d = B.dS + M.s0;
    m.dev.gam = B.gam + M.s0;
    m.dev.mu = B.mu + M.s0;
    m.dev.uh = B.uh + M.s0;
    m.dev.v = B.v + M.s0;
    m.dev.perm = B.gorder + M.s0;
    m.dev.id_tol = o.id_tol;
    m.hd = std::move(d);
    m.hg = std::move(g2);
    m.hmu = std::move(mu);
    hb.ms.push_back(std::move(m));
  }
  hb.fmm_p = o.sample_mode == ADC_SAMPLE_FMM ? o.fmm_order : 0;
  // Once the first sampling pass is queued: on the side stream, the first
  // check's probes (W and W^T Q', which read only the generators), then the
  // caller's work (packing, dense merges), all overlapping the compression;
  // the main stream waits for the probes (ev_probe) before the products that
  // read W, and for the packing before those that read the packed operand.
  // The probes go first: they are short, and the main stream's wait for
  // them then ends before the packing does.
  CheckBufs cb;
  std::vector<ApplyJob> aj0;
  bool probes_queued = false;
  adc_status probe_st = ADC_OK;
  hb.after_sampling = [&]() {
    if (c->side && c->ev_probe && c->ev_fork && hipEventRecord(c->ev_fork, st) == hipSuccess &&
        hipStreamWaitEvent(c->side, c->ev_fork, 0) == hipSuccess) {
      probe_st = check_prepare(c, hb, o, cb, aj0, c->side);
      if (probe_st == ADC_OK && hipEventRecord(c->ev_probe, c->side) == hipSuccess) probes_queued = true;
    }
    if (after_sampling) after_sampling();
  };
  // First attempt.  Its accuracy check shares the launches of the update
  // product: the probe products W H and the products of the packed operand
  // by every merge's HSS form run together once the operand is ready.  The
  // columns of a merge that fails the check are written again afterwards
  // (by its retry or by the dense fallback), so writing them now is harmless.
  batch_init_s(hb, o);
  const adc_status ast = batch_attempt(c, hb, o, SLOT_HSS, false, rep, flops, nullptr);
  if (probes_queued) HIP_OK(hipStreamWaitEvent(st, c->ev_probe, 0));  // also before an error return
  ADC_TRY(ast);
  ADC_TRY(probe_st);
  if (!probes_queued) {
    aj0.clear();
    ADC_TRY(check_prepare(c, hb, o, cb, aj0, st));
  }
  for (size_t t = 0; t < which.size(); ++t) push_update_jobs(aj0, (int)t, h_m[which[t]], B);
  if (operand_ready) HIP_OK(hipStreamWaitEvent(st, operand_ready, 0));  // the packed operand
  double fm = 0.0;
  ADC_TRY(batch_apply(c, hb, aj0, &fm));
  ADC_TRY(check_finish(c, hb, o, cb));
  c->timer.mark(st, 8);
  HssBatch rb;
  std::vector<int> rb_of;
  ADC_TRY(batch_retry(c, hb, o, rep, flops, nullptr, &rb, &rb_of));
  std::vector<ApplyJob> ajr;
  std::vector<int> dense_fb;
  for (size_t t = 0; t < which.size(); ++t) {
    const MergeDev& M = h_m[which[t]];
    const bool moved = rb_of[t] >= 0;
    auto& m = moved ? rb.ms[rb_of[t]] : hb.ms[t];
    if (rep) {
      rep->retries += m.retries;
      rep->max_rank = std::max(rep->max_rank, m.max_rank);
      rep->samples = std::max(rep->samples, m.s);
      if (m.pass) rep->check_err_max = std::max(rep->check_err_max, m.err);
      if (m.pass && m.sat) {
        rep->hss_saturated++;
        rep->hss_sat_nodes += m.sat;
      }
      if (m.pass && m.nodes.size() > 1) {
        // the least traffic of Algorithm 3 for the update product: X read
        // by the upsweep and the leaf step and Y written (24 P K bytes),
        // the leaves' G and F blocks written and read (16 P K rbar / mbar)
        double rsum = 0.0;
        for (size_t i = 1; i < m.nodes.size(); ++i) rsum += 0.5 * (m.nodes[i].kr + m.nodes[i].kc);
        const double rbar = rsum / (double)(m.nodes.size() - 1);
        const double mbar = (double)M.K / (double)(1 << m.L);
        const double PK = (double)M.n * (double)M.K;
        rep->phase_bytes[8] += 24.0 * PK + 16.0 * PK * rbar / mbar;
      }
    }
    if (m.pass && mlp_collecting(c)) {
      std::vector<int> lo, hi, kr, kc;
      for (auto& nd : m.nodes) {
        lo.push_back(nd.lo);
        hi.push_back(nd.hi);
        kr.push_back(nd.kr);
        kc.push_back(nd.kc);
      }
      ADC_TRY(mlp_collect_merge(c, B.dS + M.s0, B.gam + M.s0, B.mu + M.s0, M.K, m.bounds, lo, hi, kr, kc));
    }
    if (m.pass && moved) {
      push_update_jobs(ajr, rb_of[t], M, B);
    } else if (!m.pass) {
      dense_fb.push_back(which[t]);
      if (rep) rep->hss_fallbacks++;
    }
  }
  if (!dense_fb.empty() && o.strict) return ADC_ERR_ACCURACY;
  if (!ajr.empty()) {
    ADC_TRY(batch_apply(c, rb, ajr, &fm));
    c->timer.mark(st, 8);
  }
  if (flops) *flops += fm;
  if (rep) {
    rep->phase_flops[8] += fm;
    rep->phase_launches[8] += 1;
  }
  // dense fallback: the packed columns are in pole order, so one product
  // pk (n x K) * Cauchy (K x K) per merge
  for (int g : dense_fb) ADC_TRY(dense_sorted_update(c, d_m, g, h_m[g], B, flops));
  return ADC_OK;
}

// ---------------------------------------------------------------------------
// C ABI: build / apply / info / free
extern "C" adc_status adc_hss_build(adc_ctx c, int64_t K, const double* d, const double* gam, const double* mu,
                                    const double* uh, const double* v, const double* omega, int32_t s,
                                    const adc_opts* opts_in, adc_hss* out) {
  if (!c || !out || K < 2 || K > (1 << 24) || !d || !gam || !mu || !uh || !v) return ADC_ERR_ARG;
  c->ktimer.begin(false);
  *out = nullptr;
  adc_opts o;
  if (opts_in) o = *opts_in;
  else adc_opts_default(&o);
  ADC_TRY(validate_opts_ext(o));
  if (omega && (s < 1 || s > S_MAX)) return ADC_ERR_ARG;
  DeviceGuard gd(c->device);
  hipStream_t st = c->stream;
  adc_hss h = new (std::nothrow) adc_hss_s();
  if (!h) return ADC_ERR_NOMEM;
  h->ctx = c;
  h->K = (int)K;
  // own copies of the generators
  if (hipMalloc(&h->gen, 5 * K * 8) != hipSuccess) {
    delete h;
    return ADC_ERR_NOMEM;
  }
  const double* src[5] = {d, gam, mu, uh, v};
  for (int i = 0; i < 5; ++i)
    HIP_OK(hipMemcpyAsync(h->gen + i * K, src[i], K * 8, hipMemcpyDeviceToDevice, st));
  HssBatch hb;
  HssBatch::One m;
  m.K = (int)K;
  m.L = std::max(1, ceil_log2_ratio((int)K, o.hss_leaf));
  m.bounds = balanced_bounds((int)K, m.L);
  std::vector<double> hd(K), hg(K), hm(K);
  HIP_OK(hipMemcpyAsync(hd.data(), d, K * 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(hg.data(), gam, K * 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(hm.data(), mu, K * 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  ADC_TRY(device_rank_estimate(c, d, gam, mu, (int)K, m.bounds, o, &m.r));
  if (omega) m.r = std::max(0, s - o.oversample);
  else if (o.rank_mode == ADC_RANK_FIXED) m.r = std::max(1, o.fixed_rank);
  m.stream = 0;
  m.dev.d = h->gen;
  m.dev.gam = h->gen + K;
  m.dev.mu = h->gen + 2 * K;
  m.dev.uh = h->gen + 3 * K;
  m.dev.v = h->gen + 4 * K;
  m.dev.id_tol = o.id_tol;
  m.hd = std::move(hd);
  m.hg = std::move(hg);
  m.hmu = std::move(hm);
  hb.ms.push_back(std::move(m));
  hb.fmm_p = o.sample_mode == ADC_SAMPLE_FMM ? o.fmm_order : 0;
  std::vector<const double*> om{omega};
  adc_status sres = batch_build(c, hb, o, omega == nullptr, nullptr, nullptr, omega ? &om : nullptr);
  if (sres != ADC_OK) {
    hipFree(h->gen);
    delete h;
    return sres;
  }
  if (omega) {
    // the caller chose s: use exactly that many samples
  }
  // move the batch memory into the handle (the context slot is reused later)
  HssBatch::One& mm = hb.ms[0];
  const size_t bytes = (size_t)((char*)(mm.dev.iarena + mm.iarena_n) - hb.mem) + 256;
  if (hipMalloc(&h->mem, bytes) != hipSuccess) {
    hipFree(h->gen);
    delete h;
    return ADC_ERR_NOMEM;
  }
  HIP_OK(hipMemcpyAsync(h->mem, hb.mem, bytes, hipMemcpyDeviceToDevice, st));
  const ptrdiff_t shift = (char*)h->mem - hb.mem;
  auto mv = [&](auto* p) { return (decltype(p))((char*)p + shift); };
  h->dev = mm.dev;
  h->dev.omega = mv(mm.dev.omega);
  h->dev.phi = mv(mm.dev.phi);
  h->dev.theta = mv(mm.dev.theta);
  h->dev.leafof = mv(mm.dev.leafof);
  h->dev.bounds = mv(mm.dev.bounds);
  h->dev.nodes = mv(mm.dev.nodes);
  h->dev.arena = mv(mm.dev.arena);
  h->dev.iarena = mv(mm.dev.iarena);
  h->d_merge = mv(hb.d_ms);
  HIP_OK(hipMemcpyAsync(h->d_merge, &h->dev, sizeof(HssMerge), hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  h->nodes = mm.nodes;
  h->L = mm.L;
  h->s = mm.s;
  h->retries = mm.retries;
  h->max_rank = mm.max_rank;
  h->check_err = mm.err;
  h->dense_fallback = !mm.pass;
  h->bounds = mm.bounds;
  *out = h;
  return ADC_OK;
}

extern "C" adc_status adc_rank_estimate(adc_ctx c, int64_t K, const double* d, const double* gam,
                                        const double* mu, const adc_opts* opts_in, int32_t* r, int32_t* bounds,
                                        int32_t bounds_cap, int32_t* nbounds) {
  if (!c || K < 2 || K > (1 << 24) || !d || !gam || !mu || !r || !bounds) return ADC_ERR_ARG;
  adc_opts o;
  if (opts_in) o = *opts_in;
  else adc_opts_default(&o);
  ADC_TRY(validate_opts_ext(o));
  const int L = std::max(1, ceil_log2_ratio((int)K, o.hss_leaf));
  const int nbd = (1 << L) + 1;
  if (nbounds) *nbounds = nbd;
  if (bounds_cap < nbd) return ADC_ERR_ARG;
  DeviceGuard gd(c->device);
  std::vector<int> b = balanced_bounds((int)K, L);
  int rr = 0;
  ADC_TRY(device_rank_estimate(c, d, gam, mu, (int)K, b, o, &rr));
  std::copy(b.begin(), b.end(), bounds);
  *r = rr;
  return ADC_OK;
}

extern "C" adc_status adc_hss_sample(adc_ctx c, int64_t K, const double* d, const double* gam, const double* mu,
                                     const double* uh, const double* v, const double* omega, int32_t s,
                                     const adc_opts* opts_in, double* phi, double* theta) {
  if (!c || K < 2 || K > (1 << 24) || !d || !gam || !mu || !uh || !v || !omega || !phi || !theta || s < 1 ||
      s > S_MAX)
    return ADC_ERR_ARG;
  c->ktimer.begin(false);
  adc_opts o;
  if (opts_in) o = *opts_in;
  else adc_opts_default(&o);
  ADC_TRY(validate_opts_ext(o));
  DeviceGuard gd(c->device);
  hipStream_t st = c->stream;
  HssBatch hb;
  HssBatch::One m;
  m.K = (int)K;
  m.L = std::max(1, ceil_log2_ratio((int)K, o.hss_leaf));
  m.bounds = balanced_bounds((int)K, m.L);
  m.s = s;
  m.sp = (s + 31) / 32 * 32;
  m.hd.resize(K);
  m.hg.resize(K);
  m.hmu.resize(K);
  HIP_OK(hipMemcpyAsync(m.hd.data(), d, K * 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(m.hg.data(), gam, K * 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(m.hmu.data(), mu, K * 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  m.dev.d = d;
  m.dev.gam = gam;
  m.dev.mu = mu;
  m.dev.uh = uh;
  m.dev.v = v;
  m.dev.id_tol = o.id_tol;
  hb.ms.push_back(std::move(m));
  hb.fmm_p = o.sample_mode == ADC_SAMPLE_FMM ? o.fmm_order : 0;
  ADC_TRY(batch_alloc(c, hb, SLOT_HSS));
  ADC_TRY(batch_upload(c, hb));
  HssBatch::One& mm = hb.ms[0];
  HIP_OK(hipMemset2DAsync(mm.dev.omega, mm.sp * 8, 0, mm.sp * 8, mm.K, st));
  HIP_OK(hipMemcpy2DAsync(mm.dev.omega, mm.sp * 8, omega, (size_t)s * 8, (size_t)s * 8, mm.K,
                          hipMemcpyDeviceToDevice, st));
  ADC_TRY(batch_sample(c, hb));
  HIP_OK(hipMemcpy2DAsync(phi, (size_t)s * 8, mm.dev.phi, mm.sp * 8, (size_t)s * 8, mm.K, hipMemcpyDeviceToDevice,
                          st));
  HIP_OK(hipMemcpy2DAsync(theta, (size_t)s * 8, mm.dev.theta, mm.sp * 8, (size_t)s * 8, mm.K,
                          hipMemcpyDeviceToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  return ADC_OK;
}

extern "C" adc_status adc_hss_apply(adc_ctx c, adc_hss h, int64_t P, const double* X, int64_t ldx, double* Y,
                                    int64_t ldy) {
  if (!c || !h || P < 0 || P > INT32_MAX || !X || !Y || ldx < P || ldy < P) return ADC_ERR_ARG;
  c->ktimer.begin(false);
  if (P == 0) return ADC_OK;
  DeviceGuard gd(c->device);
  HssBatch hb;
  HssBatch::One m;
  m.K = h->K;
  m.L = h->L;
  m.s = h->s;
  m.nodes = h->nodes;
  m.dev = h->dev;
  m.bounds = h->bounds;
  hb.ms.push_back(m);
  hb.d_ms = h->d_merge;
  std::vector<ApplyJob> aj{ApplyJob{0, X, ldx, (int)P, Y, ldy, nullptr}};
  ADC_TRY(batch_apply(c, hb, aj, nullptr));
  return ADC_OK;
}

extern "C" adc_status adc_hss_info(adc_hss h, int32_t* levels, int32_t* leaves, int32_t* max_rank, int32_t* samples,
                                   int32_t* retries, double* check_err) {
  if (!h) return ADC_ERR_ARG;
  if (levels) *levels = h->L;
  if (leaves) *leaves = 1 << h->L;
  if (max_rank) *max_rank = h->max_rank;
  if (samples) *samples = h->s;
  if (retries) *retries = h->retries;
  if (check_err) *check_err = h->check_err;
  return ADC_OK;
}

extern "C" adc_status adc_hss_nodes(adc_hss h, int32_t nmax, int32_t* lo, int32_t* hi, int32_t* kr, int32_t* kc,
                                    int32_t* count) {
  if (!h || nmax < 0) return ADC_ERR_ARG;
  const int n = (int)h->nodes.size();
  for (int i = 0; i < std::min(n, (int)nmax); ++i) {
    if (lo) lo[i] = h->nodes[i].lo;
    if (hi) hi[i] = h->nodes[i].hi;
    if (kr) kr[i] = h->nodes[i].kr;
    if (kc) kc[i] = h->nodes[i].kc;
  }
  if (count) *count = n;
  return ADC_OK;
}

extern "C" adc_status adc_hss_free(adc_hss h) {
  if (!h) return ADC_ERR_ARG;
  DeviceGuard gd(h->ctx->device);
  hipStreamSynchronize(h->ctx->stream);
  if (h->mem) hipFree(h->mem);
  if (h->gen) hipFree(h->gen);
  delete h;
  return ADC_OK;
}
