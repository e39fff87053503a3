// The divide-and-conquer tree of Algorithm 1 on one GPU.
//
// Tree: balanced binary splits k = floor(n/2) down to leaves of size <=
// dc_leaf.  All tears are applied to the diagonal at once (eq. T2: every
// split at k removes |b_k| from a_k and a_{k+1}); the leaves are solved in
// one launch; the merges of one tree depth form a "level" whose phases each
// run as one launch over all merges of the level.  Results of depth t live in
// buffer t mod 2 (depth 0 = the caller's Z), so that the children of a merge
// are read from one buffer while the merged block is written to the other.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "adc_internal.hpp"
#include "hss.hpp"

__global__ void k_check_finite(const double* __restrict__ x, int64_t n, int* __restrict__ flag) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

__global__ void k_set_int(int* p, int v) { *p = v; }

// a_i = diag_i - |b_i| [i is a split] - |b_{i-1}| [i-1 is a split]
__global__ void k_tear(const double* __restrict__ diag, const double* __restrict__ off,
                       const int64_t* __restrict__ splits, int nsplit, double* __restrict__ a, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  auto has = [&](int64_t k) {
    int lo = 0, hi = nsplit;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (splits[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo < nsplit && splits[lo] == k;
  };
  double x = diag[i];
  if (has(i)) x -= fabs(off[i]);
  if (i > 0 && has(i - 1)) x -= fabs(off[i - 1]);
  a[i] = x;
}

// Counts of one level sequenced on the device, for the report: [0]
// survivors, [1] dense-update flops, [2] its operand bytes, [3] packing
// bytes, [4] merges with survivors.  One workgroup, fixed summation order.
__global__ void __launch_bounds__(256) k_level_stats(const MergeDev* __restrict__ ms, int nm,
                                                     double* __restrict__ out) {
  __shared__ double sh[5][256];
  double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int g = threadIdx.x; g < nm; g += 256) {
    const MergeDev& M = ms[g];
    const double n1 = M.n1, n2 = M.n - M.n1, K = M.K;
    a[0] += K;
    if (M.K > 0) {
      for (int half = 0; half < 2; ++half) {
        const double rows = half ? n2 : n1;
        const double kk = half ? (double)(M.k2 + M.k3) : (double)(M.k1 + M.k2);
        a[1] += 2.0 * rows * K * kk;
        a[2] += 8.0 * (rows * kk + kk * K + rows * K);
      }
      a[4] += 1.0;
    }
    a[3] += 8.0 * (2.0 * ((double)M.k1 * n1 + (double)M.k2 * M.n + (double)M.k3 * n2) +
                   (double)(M.n - M.K) * (0.5 * M.n + M.n));
  }
  for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] = a[q];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 5) out[threadIdx.x] = sh[threadIdx.x][0];
}

namespace {

constexpr int LSTAT = 8;  // doubles of per-level counts

struct Node {
  int64_t s0;
  int32_t n;
  int32_t mat;  // matrix of the solve
};

struct Plan {
  int64_t N = 0;
  int leaf = 32;
  std::vector<std::vector<Node>> merge_levels;  // depth t -> merges (n > leaf)
  std::vector<int64_t> leaf_s0;
  std::vector<int32_t> leaf_m;
  std::vector<int32_t> leaf_depth;
  std::vector<int32_t> leaf_mat;
  std::vector<int64_t> splits;
};

// The trees of every matrix of a solve (matrix i owns the global rows
// [g0_i, g0_i + n_i)); depth counts from each matrix's root, so the merges
// of one depth of every matrix form one level.
Plan make_plan(const std::vector<int64_t>& g0, const std::vector<int64_t>& nn, int leaf) {
  Plan p;
  p.leaf = leaf;
  std::vector<Node> cur;
  for (size_t i = 0; i < nn.size(); ++i) {
    if (nn[i] > 0) cur.push_back(Node{g0[i], (int32_t)nn[i], (int32_t)i});
    p.N += nn[i];
  }
  int depth = 0;
  while (!cur.empty()) {
    std::vector<Node> nxt, merges;
    for (const Node& nd : cur) {
      if (nd.n > leaf) {
        merges.push_back(nd);
        const int32_t h = nd.n / 2;
        p.splits.push_back(nd.s0 + h - 1);
        nxt.push_back({nd.s0, h, nd.mat});
        nxt.push_back({nd.s0 + h, nd.n - h, nd.mat});
      } else {
        p.leaf_s0.push_back(nd.s0);
        p.leaf_m.push_back(nd.n);
        p.leaf_depth.push_back(depth);
        p.leaf_mat.push_back(nd.mat);
      }
    }
    if (!merges.empty()) p.merge_levels.push_back(merges);
    cur.swap(nxt);
    ++depth;
  }
  std::sort(p.splits.begin(), p.splits.end());
  return p;
}

struct WsLayout {
  double *a, *Zb;
  double *dsort, *zsort, *dS, *zS, *lam, *gam, *mu, *uh, *v, *rot_c, *rot_s;
  int32_t *src, *supp, *surv, *defl, *gorder, *rot_i, *rot_j, *rot_f, *posR, *posD, *colmerge;
  int32_t *pidx, *ginv, *rot_i_of, *rot_j_of, *lcnt;
  double *pk, *qc;
  int* noconv;
  double* lstat;  // per-level counts of the levels sequenced on the device
  double *din, *offg, *wg;  // several matrices: gathered inputs, eigenvalues
  size_t bytes;
};

// N rows in all; zb_elems doubles of second eigenvector buffers (n_i^2 per
// matrix with merges); pk_elems doubles per packed operand and Cauchy matrix
// (N x the largest n); gather: the inputs and eigenvalues of several
// matrices in one index space.  One matrix: zb_elems = pk_elems = n^2.
WsLayout layout_ws(char* base, int64_t N, size_t zb_elems, size_t pk_elems, bool gather) {
  Arena ar{base, 0, 0};
  WsLayout L{};
  L.a = ar.take<double>(N);
  L.dsort = ar.take<double>(N);
  L.zsort = ar.take<double>(N);
  L.dS = ar.take<double>(N);
  L.zS = ar.take<double>(N);
  L.lam = ar.take<double>(N);
  L.gam = ar.take<double>(N);
  L.mu = ar.take<double>(N);
  L.uh = ar.take<double>(N);
  L.v = ar.take<double>(N);
  L.rot_c = ar.take<double>(N);
  L.rot_s = ar.take<double>(N);
  L.src = ar.take<int32_t>(N);
  L.supp = ar.take<int32_t>(N);
  L.surv = ar.take<int32_t>(N);
  L.defl = ar.take<int32_t>(N);
  L.gorder = ar.take<int32_t>(N);
  L.rot_i = ar.take<int32_t>(N);
  L.rot_j = ar.take<int32_t>(N);
  L.rot_f = ar.take<int32_t>(N);
  L.posR = ar.take<int32_t>(N);
  L.posD = ar.take<int32_t>(N);
  L.colmerge = ar.take<int32_t>(N);
  L.pidx = ar.take<int32_t>(N);
  L.ginv = ar.take<int32_t>(N);
  L.rot_i_of = ar.take<int32_t>(N);
  L.rot_j_of = ar.take<int32_t>(N);
  L.lcnt = ar.take<int32_t>(N);
  L.noconv = ar.take<int>(64);
  L.lstat = ar.take<double>(64 * LSTAT);
  L.din = gather ? ar.take<double>(N) : nullptr;
  L.offg = gather ? ar.take<double>(N) : nullptr;
  L.wg = gather ? ar.take<double>(N) : nullptr;
  L.Zb = zb_elems ? ar.take<double>(zb_elems) : nullptr;
  L.pk = ar.take<double>(pk_elems);
  L.qc = ar.take<double>(pk_elems);
  L.bytes = ar.off + 256;
  return L;
}

}  // namespace

adc_status dense_sorted_update(adc_ctx c, const MergeDev* d_m, int g, const MergeDev& M, const LevelBufs& B,
                               double* flops) {
  if (M.K == 0) return ADC_OK;
  hipStream_t st = c->stream;
  const int ncols = 8;
  std::vector<int32_t> tm, tc;
  for (int j0 = 0; j0 < M.K; j0 += ncols) {
    tm.push_back(g);
    tc.push_back(j0);
  }
  GemmProb P{};
  P.M = M.n;
  P.N = M.K;
  P.K = M.K;
  P.A = B.pk + M.zoff;
  P.lda = M.n;
  P.B = B.qc + M.zoff;
  P.ldb = M.K;
  P.C = M.zn;
  P.ldc = M.ldn;
  P.colmap = B.posR + M.s0;
  P.vscale = B.v + M.s0;
  P.tiles_m = (P.M + 255) / 256;
  P.tile0 = 0;
  const int tiles = P.tiles_m * ((P.N + 127) / 128);
  const size_t nt = tm.size();
  void* dp;
  ADC_TRY(c->buffer(SLOT_FB, sizeof(GemmProb) + 2 * nt * 4 + 1024, &dp));
  GemmProb* dg = (GemmProb*)dp;
  int32_t* dtm = (int32_t*)((char*)dp + 256);
  int32_t* dtc = dtm + nt;
  ADC_TRY(c->upload(dg, &P, sizeof(P)));
  ADC_TRY(c->upload(dtm, tm.data(), nt * 4));
  ADC_TRY(c->upload(dtc, tc.data(), nt * 4));
  // rows of qc in the packed order of the merge's columns; the packed
  // columns' unsupported halves zeroed, since this product reads all n rows
  hipLaunchKernelGGL(k_zero_unsupported, dim3((unsigned)M.K), dim3(256), 0, st, d_m, g, B);
  hipLaunchKernelGGL(k_cauchy, dim3((unsigned)nt), dim3(256), 0, st, d_m, dtm, dtc, B, ncols, 1);
  hipLaunchKernelGGL(k_gemm_f64_big, dim3(tiles), dim3(1024), 0, st, dg, 1, (const int*)nullptr);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(st));
  if (flops) *flops += 2.0 * P.M * (double)P.N * P.K;
  return ADC_OK;
}

extern "C" adc_status adc_workspace_query(adc_ctx c, int64_t n, const adc_opts* opts, size_t* bytes) {
  if (!c || n < 0 || !bytes) return ADC_ERR_ARG;
  (void)opts;
  const size_t n2 = (size_t)std::max<int64_t>(n, 1) * (size_t)std::max<int64_t>(n, 1);
  *bytes = layout_ws(nullptr, std::max<int64_t>(n, 1), n2, n2, false).bytes;
  return ADC_OK;
}

// ---------------------------------------------------------------------------
// The matrices of one solve.  One matrix: the caller's arrays are used in
// place.  Several: they are laid side by side in one index space (matrix i
// owns the global rows [g0_i, g0_i + n_i)), their inputs gathered into the
// workspace and their eigenvalues scattered back at the end; every tree
// level then runs over the merges of all matrices at once.
struct Forest {
  std::vector<int64_t> n, g0;
  std::vector<const double*> diag, off;
  std::vector<double*> w, Z;
  std::vector<int64_t> ldz;
};

static adc_status solve_forest(adc_ctx c, const Forest& F, void* ws, size_t ws_bytes, const adc_opts& o,
                               adc_report* rep) {
  const int count = (int)F.n.size();
  const auto t_start = std::chrono::steady_clock::now();
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->info_index = -1;
  }
  for (int i = 0; i < count; ++i) {
    bool ok = true;
    ADC_TRY(check_finite(c, F.diag[i], F.n[i], &ok));
    if (ok && F.n[i] > 1) ADC_TRY(check_finite(c, F.off[i], F.n[i] - 1, &ok));
    if (!ok) {
      // several matrices: a row of the offending one
      if (rep && count > 1) rep->info_index = (int32_t)F.g0[i];
      return ADC_ERR_ARG;
    }
  }

  const Plan plan = make_plan(F.g0, F.n, o.dc_leaf);
  const int64_t n = plan.N;  // rows of the whole solve
  const int nlev = (int)plan.merge_levels.size();
  const bool gather = count > 1;
  // second eigenvector buffers (matrices with merges) and the packed operand
  std::vector<size_t> zb_off(count, 0);
  size_t zb_elems = 0;
  int64_t nbig = 1;
  for (int i = 0; i < count; ++i)
    if (F.n[i] > o.dc_leaf) {
      zb_off[i] = zb_elems;
      zb_elems += (size_t)F.n[i] * (size_t)F.n[i];
      nbig = std::max(nbig, F.n[i]);
    }
  const size_t pk_elems = (size_t)n * (size_t)nbig;
  const size_t need = layout_ws(nullptr, n, zb_elems, pk_elems, gather).bytes;
  char* base;
  if (ws) {
    if (ws_bytes < need) return ADC_ERR_ARG;
    base = (char*)ws;
  } else {
    ADC_TRY(c->buffer(SLOT_WS, need, (void**)&base));
  }
  WsLayout L = layout_ws(base, n, zb_elems, pk_elems, gather);
  hipStream_t st = c->stream;
  const double* diag = F.diag[0];
  const double* offdiag = F.off[0];
  double* w = F.w[0];
  if (gather) {
    // the entry after each matrix's last row stays zero (never read)
    HIP_OK(hipMemsetAsync(L.offg, 0, (size_t)n * 8, st));
    for (int i = 0; i < count; ++i) {
      if (F.n[i] == 0) continue;
      HIP_OK(hipMemcpyAsync(L.din + F.g0[i], F.diag[i], F.n[i] * 8, hipMemcpyDeviceToDevice, st));
      if (F.n[i] > 1)
        HIP_OK(hipMemcpyAsync(L.offg + F.g0[i], F.off[i], (F.n[i] - 1) * 8, hipMemcpyDeviceToDevice, st));
    }
    diag = L.din;
    offdiag = L.offg;
    w = L.wg;
  }
  // per merge: the matrix's output and second buffer at the merge's corner
  auto zbuf = [&](int mat, int parity, int64_t s0, int64_t* ld) -> double* {
    const int64_t r = s0 - F.g0[mat];
    if (parity == 0) {
      *ld = F.ldz[mat];
      return F.Z[mat] + r + r * F.ldz[mat];
    }
    *ld = F.n[mat];
    return L.Zb + zb_off[mat] + r + r * F.n[mat];
  };

  // --- host staging for descriptors
  const int64_t nleaf = (int64_t)plan.leaf_s0.size();
  size_t max_merges = 1;
  for (auto& lv : plan.merge_levels) max_merges = std::max(max_merges, lv.size());
  const size_t blocks64 = (size_t)(n / 64 + 2 * max_merges + 8);
  const size_t desc_bytes = 4096 + nleaf * 32 + plan.splits.size() * 8 + max_merges * sizeof(MergeDev) +
                            3 * blocks64 * sizeof(RootBlock) + 2 * max_merges * sizeof(GemmProb) +
                            (size_t)n * 8 + 2 * ((size_t)n / 8 + max_merges + 8) * 4 + 32 * 256 +
                            12 * ((size_t)n / 8 + 2 * max_merges) + 256 * (max_merges + 4);
  // pinned staging of the host-sequenced levels: one half per level parity
  // (no synchronisation ends a level, so the copies queued from one level's
  // half may still be pending while the next level fills the other half),
  // then the per-level counts of the levels sequenced on the device
  char* hs;
  const size_t desc_half = (desc_bytes + 255) & ~(size_t)255;
  const size_t lstat_off = 2 * desc_half;
  ADC_TRY(c->stage(lstat_off + 64 * LSTAT * 8, (void**)&hs));
  double* h_lstat = (double*)(hs + lstat_off);
  char* dd;
  ADC_TRY(c->buffer(SLOT_DESC, desc_bytes, (void**)&dd));

  // --- tear all splits and solve the leaves
  std::vector<char> img;
  {
    img.assign(desc_bytes, 0);
    Arena ha{img.data(), 0, 0}, da{dd, 0, 0};
    int64_t* h_sp = ha.take<int64_t>(plan.splits.size() + 1);
    int64_t* d_sp = da.take<int64_t>(plan.splits.size() + 1);
    int64_t* h_ls = ha.take<int64_t>(nleaf);
    int64_t* d_ls = da.take<int64_t>(nleaf);
    int32_t* h_lm = ha.take<int32_t>(nleaf);
    int32_t* d_lm = da.take<int32_t>(nleaf);
    LeafOut* h_lo = ha.take<LeafOut>(nleaf);
    LeafOut* d_lo = da.take<LeafOut>(nleaf);
    if (!plan.splits.empty()) std::memcpy(h_sp, plan.splits.data(), plan.splits.size() * 8);
    // each leaf writes to its matrix's buffer of its depth's parity
    for (int64_t i = 0; i < nleaf; ++i) {
      h_ls[i] = plan.leaf_s0[i];
      h_lm[i] = plan.leaf_m[i];
      int64_t ld;
      double* zp = zbuf(plan.leaf_mat[i], plan.leaf_depth[i] & 1, plan.leaf_s0[i], &ld);
      h_lo[i] = LeafOut{zp, ld};
    }
    if (ha.off > desc_bytes) return ADC_ERR_UNSUPPORTED;
    ADC_TRY(c->upload(dd, img.data(), ha.off));
    c->ktimer.begin(rep != nullptr);
    c->timer.reset();
    c->timer.start(st, rep != nullptr);
    hipLaunchKernelGGL(k_tear, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, diag, offdiag, d_sp,
                       (int)plan.splits.size(), L.a, n);
    launch_leaf_jacobi(st, nleaf, plan.leaf, L.a, offdiag, d_ls, d_lm, w, (const LeafOut*)d_lo, 40);
    HIP_OK(hipGetLastError());
    c->timer.mark(st, 0);
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, L.noconv, INT32_MAX);
  }

  if (rep) rep->levels = nlev;
  double flops = 0.0, bytes = 0.0;

  // A level on which no merge can take the HSS route (every merge below
  // hss_min_k, or its dense update below hss_min_flops even with no
  // deflation, or HSS not allowed at that depth) is sequenced on the device
  // alone, as the batched solver does: every launch is sized for the worst
  // case K = n (the kernels read K from the merge descriptors and skip the
  // blocks beyond it), the dense products are filled in on the device, and
  // the level's counts stay in device memory until the next synchronisation.
  auto hss_possible = [&](int t) {
    if (o.force_dense || (o.hss_levels >= 0 && t >= o.hss_levels)) return false;
    const int min_k = std::max(o.hss_min_k, 8);
    for (const Node& nd : plan.merge_levels[t]) {
      const double nn = nd.n;
      // the dense update costs at most 2 K^2 n <= 2 n^3 flops
      if (nd.n >= min_k && 2.0 * nn * nn * nn >= o.hss_min_flops) return true;
    }
    return false;
  };
  struct Pending {
    int t, nm;
    int64_t nsum;
    size_t k_pack, k_gemm;
  };
  std::vector<Pending> pend;
  // before a synchronisation: queue the copy of the pending levels' counts
  auto fetch_pending = [&]() -> adc_status {
    if (!pend.empty())
      HIP_OK(hipMemcpyAsync(h_lstat, L.lstat, 64 * LSTAT * 8, hipMemcpyDeviceToHost, st));
    return ADC_OK;
  };
  // after it: the counts into the report and the kernel timings
  auto resolve_pending = [&]() {
    for (const Pending& p : pend) {
      const double* v = h_lstat + (size_t)(p.t % 64) * LSTAT;
      flops += v[1];
      bytes += v[2];
      c->ktimer.set_work(p.k_pack, 0.0, v[3]);
      c->ktimer.set_work(p.k_gemm, v[1], v[2]);
      if (rep) {
        rep->phase_flops[4] += v[1];
        rep->phase_bytes[4] += v[2];
        if (v[4] > 0.0) rep->phase_launches[4] += 1;
        if (p.t < 64) {
          rep->n_per_level[p.t] = p.nsum;
          rep->K_per_level[p.t] = (int64_t)v[0];
          rep->hss_per_level[p.t] = 0;
        }
        rep->merges += p.nm;
      }
    }
    pend.clear();
  };

  // --- merge levels, deepest first
  for (int t = nlev - 1; t >= 0; --t) {
    const std::vector<Node>& lev = plan.merge_levels[t];
    const int nm = (int)lev.size();
    LevelBufs B{};
    B.w_in = w;
    B.w_out = w;
    B.off = offdiag;
    // results of depth t in buffer t mod 2 of their matrix, the children's in the other
    const int par_new = t & 1;
    auto set_z = [&](MergeDev& M, int mat) {
      M.zn = zbuf(mat, par_new, M.s0, &M.ldn);
      M.zo = zbuf(mat, par_new ^ 1, M.s0, &M.ldo);
    };
    B.dsort = L.dsort;
    B.zsort = L.zsort;
    B.src = L.src;
    B.supp = L.supp;
    B.surv = L.surv;
    B.defl = L.defl;
    B.gorder = L.gorder;
    B.rot_i = L.rot_i;
    B.rot_j = L.rot_j;
    B.rot_f = L.rot_f;
    B.rot_c = L.rot_c;
    B.rot_s = L.rot_s;
    B.dS = L.dS;
    B.zS = L.zS;
    B.lam = L.lam;
    B.gam = L.gam;
    B.mu = L.mu;
    B.uh = L.uh;
    B.v = L.v;
    B.posR = L.posR;
    B.posD = L.posD;
    B.pk = L.pk;
    B.qc = L.qc;
    B.pidx = L.pidx;
    B.ginv = L.ginv;
    B.rot_i_of = L.rot_i_of;
    B.rot_j_of = L.rot_j_of;
    B.lcnt = L.lcnt;

    if (!hss_possible(t) && t < 64) {
      // descriptors fixed by the tree alone, in one upload
      int nob = 0, nrb = 0, njob = 0, ntile = 0, gtiles = 0;
      int32_t nmax = 0;
      int64_t nsum = 0;
      for (const Node& nd : lev) {
        nob += (nd.n + 255) / 256;
        nrb += (nd.n + 63) / 64;
        njob += nd.n;
        ntile += (nd.n + 7) / 8;
        nmax = std::max(nmax, nd.n);
        nsum += nd.n;
      }
      size_t off = 0;
      auto take = [&](size_t b) {
        const size_t r = off;
        off += (b + 255) & ~(size_t)255;
        return r;
      };
      const size_t om = take(nm * sizeof(MergeDev)), oob = take(nob * sizeof(RootBlock)),
                   orb = take(nrb * sizeof(RootBlock)), ocm = take((size_t)njob * 4), occ = take((size_t)njob * 4),
                   otm = take((size_t)ntile * 4), otc = take((size_t)ntile * 4),
                   ogp = take(2 * (size_t)nm * sizeof(GemmProb)), ogt = take(sizeof(int));
      if (off > desc_bytes) return ADC_ERR_UNSUPPORTED;  // descriptor space sized too small
      img.assign(off, 0);
      char* h = img.data();
      MergeDev* hm = (MergeDev*)(h + om);
      RootBlock* hob = (RootBlock*)(h + oob);
      RootBlock* hrb = (RootBlock*)(h + orb);
      int32_t* hcm = (int32_t*)(h + ocm);
      int32_t* hcc = (int32_t*)(h + occ);
      int32_t* htm = (int32_t*)(h + otm);
      int32_t* htc = (int32_t*)(h + otc);
      GemmProb* hgp = (GemmProb*)(h + ogp);
      int iob = 0, irb = 0, ij = 0, it = 0;
      for (int g2 = 0; g2 < nm; ++g2) {
        MergeDev& M = hm[g2];
        M.s0 = lev[g2].s0;
        M.gbase = lev[g2].s0;
        M.n = lev[g2].n;
        M.n1 = lev[g2].n / 2;
        set_z(M, lev[g2].mat);
        M.zoff = M.s0 * (int64_t)nmax;
        M.mode = 0;
        for (int i0 = 0; i0 < M.n; i0 += 256) hob[iob++] = RootBlock{g2, i0};
        for (int i0 = 0; i0 < M.n; i0 += 64) hrb[irb++] = RootBlock{g2, i0};
        for (int c2 = 0; c2 < M.n; ++c2) {
          hcm[ij] = g2;
          hcc[ij] = c2;
          ++ij;
        }
        for (int j0 = 0; j0 < M.n; j0 += 8) {
          htm[it] = g2;
          htc[it] = j0;
          ++it;
        }
        const int rows[2] = {M.n1, M.n - M.n1};
        for (int half = 0; half < 2; ++half) {
          GemmProb& P = hgp[2 * g2 + half];
          P.M = rows[half];
          P.tiles_m = (rows[half] + 255) / 256;
          P.tile0 = gtiles;
          gtiles += P.tiles_m * ((M.n + 127) / 128);
        }
      }
      ADC_TRY(c->upload(dd, h, off));
      MergeDev* d_m = (MergeDev*)(dd + om);
      const RootBlock* d_ob = (const RootBlock*)(dd + oob);
      const RootBlock* d_rb = (const RootBlock*)(dd + orb);
      const int32_t* d_cm = (const int32_t*)(dd + ocm);
      const int32_t* d_cc = (const int32_t*)(dd + occ);
      const int32_t* d_tm = (const int32_t*)(dd + otm);
      const int32_t* d_tc = (const int32_t*)(dd + otc);
      GemmProb* d_gp = (GemmProb*)(dd + ogp);
      int* d_gt = (int*)(dd + ogt);
      const int W = pick_waves(nmax);
      c->timer.start(st, rep != nullptr);
      hipLaunchKernelGGL(k_merge_sort, dim3(nob), dim3(256), 0, st, d_m, d_ob, B);
      hipLaunchKernelGGL(k_merge_prep, dim3(nm), dim3(prep_threads(nmax)), 0, st, d_m, B);
      hipLaunchKernelGGL(k_level_stats, dim3(1), dim3(256), 0, st, d_m, nm, L.lstat + (size_t)t * LSTAT);
      c->timer.mark(st, 1);
      c->ktimer.pre(st);
      hipLaunchKernelGGL(k_secular, dim3(nrb), dim3(64 * W), 0, st, d_m, d_rb, L.dS, L.zS, L.lam, L.gam, L.mu,
                         o.max_iter, L.noconv);
      c->ktimer.post(st, KT_SECULAR, 0.0, 0.0);
      c->timer.mark(st, 2);
      hipLaunchKernelGGL(k_lowner, dim3(nrb), dim3(64 * W), 0, st, d_m, d_rb, L.dS, L.zS, L.gam, L.mu, L.uh);
      hipLaunchKernelGGL(k_vnorm, dim3(nrb), dim3(64 * W), 0, st, d_m, d_rb, L.dS, L.gam, L.mu, L.uh, L.v);
      c->timer.mark(st, 3);
      hipLaunchKernelGGL(k_final_order, dim3(nob), dim3(256), 0, st, d_m, B, d_ob);
      Pending p{t, nm, nsum, 0, 0};
      c->ktimer.pre(st);
      hipLaunchKernelGGL(k_pack_rot, dim3((unsigned)((njob + 3) / 4)), dim3(256), 0, st, d_m, d_cm, d_cc, B, njob);
      c->ktimer.post(st, KT_PACK, 0.0, 0.0);
      p.k_pack = c->ktimer.last();
      hipLaunchKernelGGL(k_cauchy, dim3(ntile), dim3(256), 0, st, d_m, d_tm, d_tc, B, 8, 1);
      hipLaunchKernelGGL(k_build_probs, dim3((nm + 63) / 64), dim3(64), 0, st, d_m, nm, d_gp, (GemmProb*)nullptr,
                         (GemmProb*)nullptr, L.pk, L.qc, L.v, L.posR);
      hipLaunchKernelGGL(k_gemm_compact, dim3(1), dim3(1024), 0, st, d_gp, 2 * nm, 128, d_gt);
      c->timer.mark(st, 9);
      c->ktimer.pre(st);
      hipLaunchKernelGGL(k_gemm_f64_big, dim3(gtiles), dim3(1024), 0, st, d_gp, 2 * nm, (const int*)d_gt);
      c->ktimer.post(st, KT_GEMMBIG, 0.0, 0.0);
      p.k_gemm = c->ktimer.last();
      c->timer.mark(st, 4);
      HIP_OK(hipGetLastError());
      pend.push_back(p);
      continue;
    }

    Arena ha{hs + (size_t)(t & 1) * desc_half, 0, 0}, da{dd, 0, 0};
    MergeDev* h_m = ha.take<MergeDev>(nm);
    MergeDev* d_m = da.take<MergeDev>(nm);
    // blocks of 256 elements over every merge (the merged order, later the
    // final order) and of 64 roots for the secular solver, Loewner and v,
    // for the worst case K = n: those launches are queued before the host
    // reads the deflation results (their blocks past K exit)
    RootBlock* h_ob = ha.take<RootBlock>(blocks64);
    RootBlock* d_ob = da.take<RootBlock>(blocks64);
    RootBlock* h_rb = ha.take<RootBlock>(blocks64);
    RootBlock* d_rb = da.take<RootBlock>(blocks64);
    int nob = 0, nrb = 0;
    int32_t nmax = 0;
    for (int g2 = 0; g2 < nm; ++g2) nmax = std::max(nmax, lev[g2].n);
    for (int g2 = 0; g2 < nm; ++g2) {
      MergeDev& M = h_m[g2];
      std::memset(&M, 0, sizeof(M));
      M.s0 = lev[g2].s0;
      M.gbase = lev[g2].s0;
      M.n = lev[g2].n;
      M.n1 = lev[g2].n / 2;
      set_z(M, lev[g2].mat);
      M.zoff = M.s0 * (int64_t)nmax;
    }
    for (int g2 = 0; g2 < nm; ++g2) {
      for (int i0 = 0; i0 < h_m[g2].n; i0 += 256) h_ob[nob++] = RootBlock{g2, i0};
      for (int i0 = 0; i0 < h_m[g2].n; i0 += 64) h_rb[nrb++] = RootBlock{g2, i0};
    }
    const size_t first_bytes = ha.off;
    HIP_OK(hipMemcpyAsync(dd, ha.base, first_bytes, hipMemcpyHostToDevice, st));
    c->timer.start(st, rep != nullptr);
    hipLaunchKernelGGL(k_merge_sort, dim3(nob), dim3(256), 0, st, d_m, d_ob, B);
    hipLaunchKernelGGL(k_merge_prep, dim3(nm), dim3(prep_threads(nmax)), 0, st, d_m, B);
    HIP_OK(hipGetLastError());
    c->timer.mark(st, 1);
    HIP_OK(hipMemcpyAsync(h_m, d_m, nm * sizeof(MergeDev), hipMemcpyDeviceToHost, st));
    ADC_TRY(fetch_pending());
    hipEvent_t ev_meta;
    ADC_TRY(c->meta_event(&ev_meta));
    HIP_OK(hipEventRecord(ev_meta, st));

    // --- secular, Loewner, v, final order: queued before the host waits
    const int W = pick_waves(nmax);
    c->ktimer.pre(st);
    hipLaunchKernelGGL(k_secular, dim3(nrb), dim3(64 * W), 0, st, d_m, d_rb, L.dS, L.zS, L.lam, L.gam, L.mu,
                       o.max_iter, L.noconv);
    c->ktimer.post(st, KT_SECULAR, 0.0, 0.0);
    c->timer.mark(st, 2);
    hipLaunchKernelGGL(k_lowner, dim3(nrb), dim3(64 * W), 0, st, d_m, d_rb, L.dS, L.zS, L.gam, L.mu, L.uh);
    hipLaunchKernelGGL(k_vnorm, dim3(nrb), dim3(64 * W), 0, st, d_m, d_rb, L.dS, L.gam, L.mu, L.uh, L.v);
    c->timer.mark(st, 3);
    hipLaunchKernelGGL(k_final_order, dim3(nob), dim3(256), 0, st, d_m, B, d_ob);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventSynchronize(ev_meta));
    resolve_pending();

    // --- host decisions and launch lists
    int64_t Ksum = 0, nsum = 0;
    int hss_here = 0;
    // HSS on a merge whose dense update reaches hss_min_flops; once the
    // level takes the HSS route, merges of a quarter of that join it, since
    // their share of the route's fixed costs is already paid
    auto dense_flops = [](const MergeDev& M) {
      return 2.0 * M.K * ((double)M.n1 * (M.k1 + M.k2) + (double)(M.n - M.n1) * (M.k2 + M.k3));
    };
    const bool level_ok = !o.force_dense && ((o.hss_levels < 0) || (t < o.hss_levels));
    const int min_k = std::max(o.hss_min_k, 8);  // at least two leaves of four
    bool level_hss = false;
    for (int g2 = 0; g2 < nm; ++g2)
      level_hss |= level_ok && h_m[g2].K >= min_k && dense_flops(h_m[g2]) >= o.hss_min_flops;
    for (int g2 = 0; g2 < nm; ++g2) {
      MergeDev& M = h_m[g2];
      M.mode = (level_hss && M.K >= min_k && dense_flops(M) >= 0.25 * o.hss_min_flops) ? 1 : 0;
      hss_here += M.mode == 1;
      Ksum += M.K;
      nsum += M.n;
    }
    // HSS merges: the leaf boundaries of their HSS trees (leaves of at most
    // hss_leaf <= 256 survivors) and one column-grouping job per leaf
    std::vector<int2> lg_jobs;
    std::vector<int32_t> lg_merges;
    for (int g2 = 0; g2 < nm; ++g2) {
      MergeDev& M = h_m[g2];
      M.lbounds = nullptr;
      M.nleaf = 0;
      if (M.mode != 1) continue;
      const std::vector<int> bd = hss_leaf_bounds(M.K, o.hss_leaf);
      int32_t* hbd = ha.take<int32_t>(bd.size());
      int32_t* dbd = da.take<int32_t>(bd.size());
      std::copy(bd.begin(), bd.end(), hbd);
      M.lbounds = dbd;
      M.nleaf = (int)bd.size() - 1;
      lg_merges.push_back(g2);
      for (int i = 0; i < M.nleaf; ++i) lg_jobs.push_back(int2{g2, i});
    }
    int2* h_lg = ha.take<int2>(lg_jobs.size() + 1);
    int2* d_lg = da.take<int2>(lg_jobs.size() + 1);
    std::copy(lg_jobs.begin(), lg_jobs.end(), h_lg);
    int32_t* h_lgm = ha.take<int32_t>(lg_merges.size() + 1);
    int32_t* d_lgm = da.take<int32_t>(lg_merges.size() + 1);
    std::copy(lg_merges.begin(), lg_merges.end(), h_lgm);
    int32_t* h_cm = ha.take<int32_t>(n);
    int32_t* d_cm = da.take<int32_t>(n);
    int32_t* h_cc = ha.take<int32_t>(n);
    int32_t* d_cc = da.take<int32_t>(n);
    int njob = 0;
    for (int g2 = 0; g2 < nm; ++g2)
      for (int c2 = 0; c2 < h_m[g2].n; ++c2) {
        h_cm[njob] = g2;
        h_cc[njob] = c2;
        ++njob;
      }
    const int ncols = 8;
    const size_t maxtiles = (size_t)n / 8 + max_merges + 8;
    int32_t* h_tm = ha.take<int32_t>(maxtiles);
    int32_t* d_tm = da.take<int32_t>(maxtiles);
    int32_t* h_tc = ha.take<int32_t>(maxtiles);
    int32_t* d_tc = da.take<int32_t>(maxtiles);
    int ntile = 0;
    GemmProb* h_gp = ha.take<GemmProb>(2 * nm);
    GemmProb* d_gp = da.take<GemmProb>(2 * nm);
    int ngp = 0, gtiles = 0;
    double lvl_gf = 0.0, lvl_gb = 0.0;
    for (int g2 = 0; g2 < nm; ++g2) {
      const MergeDev& M = h_m[g2];
      if (M.K == 0 || M.mode != 0) continue;
      for (int j0 = 0; j0 < M.K; j0 += ncols) {
        h_tm[ntile] = g2;
        h_tc[ntile] = j0;
        ++ntile;
      }
      const int n2 = M.n - M.n1;
      for (int half = 0; half < 2; ++half) {
        GemmProb& P = h_gp[ngp];
        std::memset(&P, 0, sizeof(P));
        P.M = half ? n2 : M.n1;
        P.N = M.K;
        P.K = half ? (M.k2 + M.k3) : (M.k1 + M.k2);
        P.A = L.pk + M.zoff + (half ? (M.n1 + (int64_t)M.k1 * M.n) : 0);
        P.lda = M.n;
        P.B = L.qc + M.zoff + (half ? M.k1 : 0);
        P.ldb = M.K;
        P.C = M.zn + (half ? M.n1 : 0);
        P.ldc = M.ldn;
        P.colmap = L.posR + M.s0;
        P.vscale = L.v + M.s0;
        P.tiles_m = (P.M + 255) / 256;
        P.tile0 = gtiles;
        gtiles += P.tiles_m * ((P.N + 127) / 128);
        ++ngp;
        const double f = 2.0 * P.M * (double)P.N * P.K;
        const double by = 8.0 * ((double)P.M * P.K + (double)P.K * P.N + (double)P.M * P.N);
        flops += f;
        bytes += by;
        lvl_gf += f;
        lvl_gb += by;
        if (rep) {
          rep->phase_flops[4] += f;
          rep->phase_bytes[4] += by;
        }
      }
    }
    if (rep && gtiles) rep->phase_launches[4] += 1;
    if (ha.off > desc_bytes) return ADC_ERR_UNSUPPORTED;  // descriptor space sized too small
    // the merge descriptors with the host's decisions, and the launch lists
    HIP_OK(hipMemcpyAsync(dd, ha.base, ha.off, hipMemcpyHostToDevice, st));
    // packing: a survivor column reads and writes its support rows (top
    // half, bottom half or both), a deflated column reads its child's half
    // and writes all n rows of its final place
    double pack_by = 0.0;
    for (int g2 = 0; g2 < nm; ++g2) {
      const MergeDev& M = h_m[g2];
      const double n1 = M.n1, n2 = M.n - M.n1;
      pack_by += 8.0 * (2.0 * ((double)M.k1 * n1 + (double)M.k2 * M.n + (double)M.k3 * n2) +
                        (double)(M.n - M.K) * (0.5 * M.n + M.n));
    }
    if (!lg_jobs.empty()) {
      hipLaunchKernelGGL(k_leaf_bounds, dim3((unsigned)lg_merges.size()), dim3(64), 0, st, d_m, d_lgm, B,
                         o.shift_thresh, o.shift_max, o.rank_eps, o.r_cap);
      hipLaunchKernelGGL(k_leaf_group, dim3((unsigned)lg_jobs.size()), dim3(512), 0, st, d_m, d_lg, B);
    }
    // The packing and the dense merges' update.  With HSS merges in the
    // level they read nothing the HSS construction writes and vice versa:
    // the HSS update starts them on the side stream once its sampling is
    // queued (so that they overlap the latency-bound compression rather
    // than the sampling) and waits for them only before its products read
    // the packed operand.
    auto pack = [&](hipStream_t sp) {
      c->ktimer.pre(sp);
      hipLaunchKernelGGL(k_pack_rot, dim3((unsigned)std::min((njob + 3) / 4, 2 * c->num_cu)), dim3(256), 0, sp,
                         d_m, d_cm, d_cc, B, njob);
      c->ktimer.post(sp, KT_PACK, 0.0, pack_by);
      if (ntile) hipLaunchKernelGGL(k_cauchy, dim3(ntile), dim3(256), 0, sp, d_m, d_tm, d_tc, B, ncols, 1);
    };
    auto dense = [&](hipStream_t sp) {
      if (!gtiles) return;
      c->ktimer.pre(sp);
      hipLaunchKernelGGL(k_gemm_f64_big, dim3(gtiles), dim3(1024), 0, sp, d_gp, ngp, (const int*)nullptr);
      c->ktimer.post(sp, KT_GEMMBIG, lvl_gf, lvl_gb);
    };
    if (!hss_here) {
      pack(st);
      c->timer.mark(st, 9);
      dense(st);
      c->timer.mark(st, 4);
      HIP_OK(hipGetLastError());
    } else {
      ADC_TRY(c->side_stream());
      c->timer.mark(st, 9);
      c->timer.mark(st, 4);
      bool forked = false;
      auto fork = [&]() {
        if (forked) return;
        forked = true;
        hipEventRecord(c->ev_fork, st);
        hipStreamWaitEvent(c->side, c->ev_fork, 0);
        pack(c->side);
        dense(c->side);
        hipEventRecord(c->ev_join, c->side);
      };
      const adc_status hst = hss_level_update(c, o, h_m, d_m, nm, B, t, rep, &flops, &bytes, fork, c->ev_join);
      fork();                                         // when the update returned before sampling
      HIP_OK(hipStreamWaitEvent(st, c->ev_join, 0));  // joined even when the update failed
      HIP_OK(hipGetLastError());
      ADC_TRY(hst);
    }

    if (rep && t < 64) {
      rep->n_per_level[t] = nsum;
      rep->K_per_level[t] = Ksum;
      rep->hss_per_level[t] = hss_here;
      rep->merges += nm;
      rep->hss_merges += hss_here;
    }
  }

  if (gather)
    for (int i = 0; i < count; ++i)
      if (F.n[i] > 0)
        HIP_OK(hipMemcpyAsync(F.w[i], L.wg + F.g0[i], F.n[i] * 8, hipMemcpyDeviceToDevice, st));
  int nc = INT32_MAX;
  HIP_OK(hipMemcpyAsync(&nc, L.noconv, sizeof(int), hipMemcpyDeviceToHost, st));
  ADC_TRY(fetch_pending());
  HIP_OK(hipStreamSynchronize(st));
  resolve_pending();
  c->up_reset();
  c->timer.collect(rep);
  c->ktimer.collect(rep);
  c->ktimer.begin(false);
  if (rep) {
    rep->flops_model += flops;
    rep->bytes_model += bytes;
    rep->t_phase[10] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    double covered = 0.0;
    for (int p = 0; p < 10; ++p) covered += rep->t_phase[p];
    rep->t_phase[11] = rep->t_phase[10] - covered;
  }
  if (nc != INT32_MAX) {
    if (rep) rep->info_index = nc;
    return ADC_ERR_NOCONV;
  }
  return ADC_OK;
}

extern "C" adc_status adc_stedc(adc_ctx c, int64_t n, const double* diag, const double* offdiag, double* w,
                                double* Z, int64_t ldz, void* ws, size_t ws_bytes, const adc_opts* opts_in,
                                adc_report* rep) {
  if (!c || n < 0) return ADC_ERR_ARG;
  if (n == 0) return ADC_OK;
  if (!diag || !w || !Z || ldz < n || (n > 1 && !offdiag)) return ADC_ERR_ARG;
  if (n > 1000000) return ADC_ERR_UNSUPPORTED;
  adc_opts o;
  if (opts_in) o = *opts_in;
  else adc_opts_default(&o);
  ADC_TRY(validate_opts_ext(o));
  DeviceGuard g(c->device);
  Forest F;
  F.n = {n};
  F.g0 = {0};
  F.diag = {diag};
  F.off = {offdiag};
  F.w = {w};
  F.Z = {Z};
  F.ldz = {ldz};
  return solve_forest(c, F, ws, ws_bytes, o, rep);
}

namespace {

// Adds the figures of one forest solve to a running report.
void report_add(adc_report* a, const adc_report& b) {
  a->levels = std::max(a->levels, b.levels);
  a->merges += b.merges;
  a->hss_merges += b.hss_merges;
  a->retries += b.retries;
  a->hss_fallbacks += b.hss_fallbacks;
  a->max_rank = std::max(a->max_rank, b.max_rank);
  a->samples = std::max(a->samples, b.samples);
  a->hss_saturated += b.hss_saturated;
  a->hss_sat_nodes += b.hss_sat_nodes;
  a->check_err_max = std::max(a->check_err_max, b.check_err_max);
  a->flops_model += b.flops_model;
  a->bytes_model += b.bytes_model;
  for (int t = 0; t < 64; ++t) {
    a->n_per_level[t] += b.n_per_level[t];
    a->K_per_level[t] += b.K_per_level[t];
    a->hss_per_level[t] += b.hss_per_level[t];
  }
  for (int p = 0; p < 12; ++p) {
    a->t_phase[p] += b.t_phase[p];
    a->phase_flops[p] += b.phase_flops[p];
    a->phase_bytes[p] += b.phase_bytes[p];
    a->phase_launches[p] += b.phase_launches[p];
    a->kern_time[p] += b.kern_time[p];
    a->kern_flops[p] += b.kern_flops[p];
    a->kern_bytes[p] += b.kern_bytes[p];
    a->kern_launches[p] += b.kern_launches[p];
  }
}

}  // namespace

// Several matrices in level-batched solves with the single-matrix sequencing
// (HSS levels by the host); arguments checked by the caller.  The matrices
// are taken in order into forests of at most 10^6 rows whose workspace
// (second eigenvector buffers, n^2 per matrix, and two packed operands of
// rows x largest n) stays within opts.batch_bytes; a matrix that alone
// exceeds it forms a forest of its own.  On failure rep->info_index is a row of the failing matrix
// in the concatenation of the nonempty matrices.
adc_status stedc_forest(adc_ctx c, int count, const int64_t* n, const double* const* diag,
                        const double* const* offdiag, double* const* w, double* const* Z, const int64_t* ldz,
                        const adc_opts& o, adc_report* rep) {
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->info_index = -1;
  }
  const double budget = o.batch_bytes > 0.0 ? o.batch_bytes : 32.0 * 1073741824.0;
  int64_t row0 = 0;  // first row of the current forest in the concatenation
  int i = 0;
  while (i < count) {
    Forest F;
    int64_t g0 = 0, nbig = 0;
    double sumsq = 0.0;
    for (; i < count; ++i) {
      if (n[i] == 0) continue;
      const int64_t nb = std::max(nbig, n[i]);
      const double sq = sumsq + (double)n[i] * (double)n[i];
      const double bytes = 8.0 * (sq + 2.0 * (double)(g0 + n[i]) * (double)nb) + 256.0 * (double)(g0 + n[i]);
      if (!F.n.empty() && (g0 + n[i] > 1000000 || bytes > budget)) break;
      F.n.push_back(n[i]);
      F.g0.push_back(g0);
      F.diag.push_back(diag[i]);
      F.off.push_back(n[i] > 1 ? offdiag[i] : diag[i]);  // n = 1: never read
      F.w.push_back(w[i]);
      F.Z.push_back(Z[i]);
      F.ldz.push_back(ldz[i]);
      g0 += n[i];
      nbig = nb;
      sumsq = sq;
    }
    if (F.n.empty()) break;
    adc_report r1;
    const adc_status st = solve_forest(c, F, nullptr, 0, o, rep ? &r1 : nullptr);
    if (rep) {
      const int32_t info = r1.info_index;
      report_add(rep, r1);
      if (st != ADC_OK) rep->info_index = (int32_t)(row0 + std::max<int32_t>(info, 0));
    }
    if (st != ADC_OK) return st;
    row0 += g0;
  }
  return ADC_OK;
}
