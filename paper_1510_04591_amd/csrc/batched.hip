// Many independent eigendecompositions on one GPU, level-batched.
//
// Every matrix of the batch gets its own divide-and-conquer tree (Algorithm 1,
// splits at floor(n/2)); the trees are laid side by side in one global index
// space (matrix i owns [g0_i, g0_i + N_i)), and the merges of one tree depth
// of every matrix form one level.  Unlike the single-matrix solver, the host
// never reads the deflation results: every launch of a level is sized for the
// worst case (K = n) and each workgroup reads its merge's K from device
// memory and exits when it has no work; the GEMM problem descriptors of the
// dense update are filled in on the device.  Every call first gathers the
// inputs and checks them (non-finite input is rejected before any solver
// kernel runs); the sequence after that (tears, leaves, all levels, output
// scatter) is fixed by the sizes alone: the first call for a size set runs it
// eagerly, tuning the GEMM tile shape and the secular kernel's wave count per
// level with HIP events, and captures it in a HIP graph that later calls
// with the same sizes replay.  Caller pointers live in device descriptor arrays refreshed before
// each replay, so they may change between calls.
//
// The update here is the dense one (merges up to a few thousand, where HSS
// does not pay); matrices large enough for an HSS merge (unless
// opts.force_dense is set) are solved together by the single-matrix level
// loop over all of them (stedc_forest), which takes the HSS route at the
// levels where it applies.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "adc_internal.hpp"
#include "hss.hpp"

// The two block products of each merge's dense update (rows of the first
// child against survivors of rows top-only and both, rows of the second
// child against both and bottom-only), from the deflation results.  tile0
// and tiles_m were set by the host for the worst case N = n.  One to three
// arrays (one per tile class); a null array is skipped.
__global__ void k_build_probs(const MergeDev* __restrict__ ms, int nm, GemmProb* __restrict__ pa,
                              GemmProb* __restrict__ pb, GemmProb* __restrict__ pc, const double* __restrict__ pk,
                              const double* __restrict__ qc, const double* __restrict__ v,
                              const int32_t* __restrict__ posR) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nm) return;
  const MergeDev& M = ms[g];
  for (int which = 0; which < 3; ++which) {
    GemmProb* arr = (which == 0) ? pa : (which == 1) ? pb : pc;
    if (!arr) continue;
    for (int half = 0; half < 2; ++half) {
      GemmProb& P = arr[2 * g + half];
      P.N = M.K;
      P.K = half ? (M.k2 + M.k3) : (M.k1 + M.k2);
      P.K2 = 0;
      P.A = pk + M.zoff + (half ? (M.n1 + (int64_t)M.k1 * M.n) : 0);
      P.lda = M.n;
      P.B = qc + M.zoff + (half ? M.k1 : 0);
      P.ldb = (M.K > 0) ? M.K : 1;
      P.C = M.zn + (half ? M.n1 : 0);
      P.ldc = M.ldn;
      P.colmap = posR + M.s0;
      P.vscale = v + M.s0;
      P.beta = 0.0;
      P.transB = 0;
    }
  }
}

namespace {

// concatenate the inputs: din = [diag_0, diag_1, ...], offg likewise with a
// zero after each matrix's last row
__global__ void k_gather(int count, const double* const* __restrict__ diag, const double* const* __restrict__ off,
                         const int64_t* __restrict__ g0, const int64_t* __restrict__ nn, double* __restrict__ din,
                         double* __restrict__ offg) {
  const int i = blockIdx.x;
  if (i >= count) return;
  const int64_t base = g0[i], n = nn[i];
  const double* __restrict__ d = diag[i];
  const double* __restrict__ o = off[i];
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    din[base + r] = d[r];
    offg[base + r] = (r + 1 < n) ? o[r] : 0.0;
  }
}

__global__ void k_scatter_w(int count, const double* __restrict__ wg, double* const* __restrict__ w,
                            const int64_t* __restrict__ g0, const int64_t* __restrict__ nn) {
  const int i = blockIdx.x;
  if (i >= count) return;
  const int64_t base = g0[i], n = nn[i];
  double* __restrict__ o = w[i];
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) o[r] = wg[base + r];
}

struct Node {
  int64_t s0;
  int32_t n;
  int32_t mat;
};

struct BLevel {
  int nm = 0, nmax = 0;
  size_t o_m = 0, o_rb = 0, o_ob = 0, o_cm = 0, o_cc = 0, o_tm = 0, o_tc = 0, o_ga = 0, o_gb = 0, o_gc = 0, o_gt = 0;
  int nrb = 0, nob = 0, njob = 0, ntile = 0, tiles[3] = {0, 0, 0};
  int W = 1;      // waves per secular / Loewner block
  int gv = 0;     // GEMM tile shape: 0 128x128, 1 128x64, 2 256x128
  bool tuned = false;
};

struct BEntry {
  std::vector<int64_t> N, g0;
  int64_t Ntot = 0;
  int leaf = 32;
  int max_iter = 60;
  char* dev = nullptr;
  size_t dev_bytes = 0;
  // global vectors
  double *din, *offg, *a, *w, *dsort, *zsort, *dS, *zS, *lam, *gam, *mu, *uh, *v, *rot_c, *rot_s;
  int32_t *src, *supp, *surv, *defl, *gorder, *rot_i, *rot_j, *rot_f, *posR, *posD, *pidx, *ginv, *rot_i_of,
      *rot_j_of;
  int* flags;  // [0] noconv, [1] non-finite input
  double *pk, *qc;
  std::vector<double*> Zb;  // per matrix scratch eigenvector buffer (nullptr if no merges)
  // descriptors
  char* desc = nullptr;  // device region of every descriptor array
  std::vector<char> hdesc;  // host image
  size_t o_sp = 0, o_ls = 0, o_lm = 0, o_lo = 0, o_pd = 0, o_po = 0, o_pw = 0, o_g0 = 0, o_n = 0;
  int nsplit = 0, nleaf = 0;
  std::vector<std::vector<Node>> lev_nodes;
  std::vector<BLevel> levels;
  std::vector<Node> leaves;
  std::vector<int> leaf_depth;
  std::vector<const void*> last_ptrs;
  bool captured = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct BCache {
  std::map<std::tuple<std::vector<int64_t>, int, int>, BEntry*> entries;
  // level signature (merges, largest n, sum of n) -> (waves, GEMM tile shape)
  std::map<std::tuple<int, int, int64_t>, std::pair<int, int>> tune;
  hipStream_t cap = nullptr;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

void free_entry(BEntry* e) {
  if (e->exec) hipGraphExecDestroy(e->exec);
  if (e->graph) hipGraphDestroy(e->graph);
  if (e->dev) hipFree(e->dev);
  delete e;
}

// tree of one matrix: merges per depth (top = 0), leaves with their depth
void plan_matrix(int64_t N, int64_t g0, int mat, int leaf, std::vector<std::vector<Node>>& levs,
                 std::vector<Node>& leaves, std::vector<int>& ldepth, std::vector<int64_t>& splits) {
  std::vector<Node> cur{{g0, (int32_t)N, mat}};
  int depth = 0;
  while (!cur.empty()) {
    std::vector<Node> nxt;
    for (const Node& nd : cur) {
      if (nd.n > leaf) {
        if ((int)levs.size() <= depth) levs.resize(depth + 1);
        levs[depth].push_back(nd);
        const int32_t h = nd.n / 2;
        splits.push_back(nd.s0 + h - 1);
        nxt.push_back({nd.s0, h, mat});
        nxt.push_back({nd.s0 + h, nd.n - h, mat});
      } else {
        leaves.push_back(nd);
        ldepth.push_back(depth);
      }
    }
    cur.swap(nxt);
    ++depth;
  }
}

adc_status build_entry(const std::vector<int64_t>& N, int leaf, int max_iter, BEntry** out) {
  BEntry* e = new BEntry();
  e->N = N;
  e->leaf = leaf;
  e->max_iter = max_iter;
  const int count = (int)N.size();
  e->g0.resize(count);
  int64_t tot = 0;
  for (int i = 0; i < count; ++i) {
    e->g0[i] = tot;
    tot += N[i];
  }
  e->Ntot = tot;
  std::vector<int64_t> splits;
  for (int i = 0; i < count; ++i) plan_matrix(N[i], e->g0[i], i, leaf, e->lev_nodes, e->leaves, e->leaf_depth, splits);
  std::sort(splits.begin(), splits.end());
  e->nsplit = (int)splits.size();
  e->nleaf = (int)e->leaves.size();
  const int nlev = (int)e->lev_nodes.size();
  e->levels.resize(nlev);

  // --- device memory plan
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t V8 = (size_t)tot * 8, V4 = (size_t)tot * 4;
  std::vector<size_t> ov8(15), ov4(14);
  for (auto& x : ov8) x = take(V8);
  for (auto& x : ov4) x = take(V4);
  const size_t o_flags = take(64);
  int64_t pksz = 1;
  for (int t = 0; t < nlev; ++t) {
    int64_t s = 0;
    for (auto& nd : e->lev_nodes[t]) s += (int64_t)nd.n * nd.n;
    pksz = std::max(pksz, s);
  }
  const size_t o_pk = take((size_t)pksz * 8), o_qc = take((size_t)pksz * 8);
  std::vector<size_t> o_zb(count, 0);
  std::vector<char> has_merge(count, 0);
  for (auto& lv : e->lev_nodes)
    for (auto& nd : lv) has_merge[nd.mat] = 1;
  for (int i = 0; i < count; ++i)
    if (has_merge[i]) o_zb[i] = take((size_t)N[i] * N[i] * 8);
  // descriptors (host image mirrors the device region)
  size_t doff = 0;
  auto dtake = [&](size_t bytes) {
    const size_t o = doff;
    doff = align256(doff + bytes);
    return o;
  };
  e->o_sp = dtake(std::max<size_t>(1, splits.size()) * 8);
  e->o_ls = dtake(std::max(1, e->nleaf) * 8);
  e->o_lm = dtake(std::max(1, e->nleaf) * 4);
  e->o_lo = dtake(std::max(1, e->nleaf) * sizeof(LeafOut));
  e->o_pd = dtake(count * 8);
  e->o_po = dtake(count * 8);
  e->o_pw = dtake(count * 8);
  e->o_g0 = dtake(count * 8);
  e->o_n = dtake(count * 8);
  for (int t = 0; t < nlev; ++t) {
    BLevel& L = e->levels[t];
    const auto& nodes = e->lev_nodes[t];
    L.nm = (int)nodes.size();
    int64_t nsum = 0;
    for (auto& nd : nodes) {
      L.nmax = std::max<int>(L.nmax, nd.n);
      L.nrb += (nd.n + 63) / 64;
      L.nob += (nd.n + 255) / 256;
      L.njob += nd.n;
      L.ntile += (nd.n + 7) / 8;
      const int n1 = nd.n / 2, n2 = nd.n - n1;
      const int tn128 = (nd.n + 127) / 128, tn64 = (nd.n + 63) / 64;
      L.tiles[0] += ((n1 + 127) / 128 + (n2 + 127) / 128) * tn128;
      L.tiles[1] += ((n1 + 127) / 128 + (n2 + 127) / 128) * tn64;
      L.tiles[2] += ((n1 + 255) / 256 + (n2 + 255) / 256) * tn128;
      nsum += nd.n;
    }
    (void)nsum;
    L.W = pick_waves(L.nmax);
    L.o_m = dtake(L.nm * sizeof(MergeDev));
    L.o_rb = dtake(L.nrb * sizeof(RootBlock));
    L.o_ob = dtake(L.nob * sizeof(RootBlock));
    L.o_cm = dtake((size_t)L.njob * 4);
    L.o_cc = dtake((size_t)L.njob * 4);
    L.o_tm = dtake((size_t)L.ntile * 4);
    L.o_tc = dtake((size_t)L.ntile * 4);
    L.o_ga = dtake(2 * (size_t)L.nm * sizeof(GemmProb));
    L.o_gb = dtake(2 * (size_t)L.nm * sizeof(GemmProb));
    L.o_gc = dtake(2 * (size_t)L.nm * sizeof(GemmProb));
    L.o_gt = dtake(sizeof(int));  // working tiles of the wide-tile problems (k_gemm_compact)
  }
  const size_t o_desc = take(doff);
  e->dev_bytes = off;
  if (hipMalloc((void**)&e->dev, off) != hipSuccess) {
    delete e;
    return ADC_ERR_NOMEM;
  }
  char* b = e->dev;
  double** v8[15] = {&e->din, &e->offg, &e->a, &e->w, &e->dsort, &e->zsort, &e->dS,
                     &e->zS, &e->lam, &e->gam, &e->mu, &e->uh, &e->v, &e->rot_c, &e->rot_s};
  for (int q = 0; q < 15; ++q) *v8[q] = (double*)(b + ov8[q]);
  int32_t** v4[14] = {&e->src, &e->supp, &e->surv, &e->defl, &e->gorder, &e->rot_i, &e->rot_j,
                      &e->rot_f, &e->posR, &e->posD, &e->pidx, &e->ginv, &e->rot_i_of, &e->rot_j_of};
  for (int q = 0; q < 14; ++q) *v4[q] = (int32_t*)(b + ov4[q]);
  e->flags = (int*)(b + o_flags);
  e->pk = (double*)(b + o_pk);
  e->qc = (double*)(b + o_qc);
  e->Zb.assign(count, nullptr);
  for (int i = 0; i < count; ++i)
    if (has_merge[i]) e->Zb[i] = (double*)(b + o_zb[i]);
  e->desc = b + o_desc;

  // --- pointer-independent descriptors
  e->hdesc.assign(doff, 0);
  char* h = e->hdesc.data();
  if (!splits.empty()) std::memcpy(h + e->o_sp, splits.data(), splits.size() * 8);
  for (int l = 0; l < e->nleaf; ++l) {
    ((int64_t*)(h + e->o_ls))[l] = e->leaves[l].s0;
    ((int32_t*)(h + e->o_lm))[l] = e->leaves[l].n;
  }
  std::memcpy(h + e->o_g0, e->g0.data(), count * 8);
  std::memcpy(h + e->o_n, N.data(), count * 8);
  for (int t = 0; t < nlev; ++t) {
    BLevel& L = e->levels[t];
    const auto& nodes = e->lev_nodes[t];
    MergeDev* hm = (MergeDev*)(h + L.o_m);
    RootBlock* rb = (RootBlock*)(h + L.o_rb);
    RootBlock* ob = (RootBlock*)(h + L.o_ob);
    int32_t* cm = (int32_t*)(h + L.o_cm);
    int32_t* cc = (int32_t*)(h + L.o_cc);
    int32_t* tm = (int32_t*)(h + L.o_tm);
    int32_t* tc = (int32_t*)(h + L.o_tc);
    GemmProb* ga = (GemmProb*)(h + L.o_ga);
    GemmProb* gb = (GemmProb*)(h + L.o_gb);
    GemmProb* gc = (GemmProb*)(h + L.o_gc);
    int irb = 0, iob = 0, ij = 0, it = 0, t128 = 0, t64 = 0, tbig = 0;
    int64_t zoff = 0;
    for (int g = 0; g < L.nm; ++g) {
      const Node& nd = nodes[g];
      MergeDev& M = hm[g];
      std::memset(&M, 0, sizeof(M));
      M.s0 = nd.s0;
      M.gbase = nd.s0;
      M.n = nd.n;
      M.n1 = nd.n / 2;
      M.zoff = zoff;
      M.mode = 0;
      zoff += (int64_t)nd.n * nd.n;
      for (int i0 = 0; i0 < nd.n; i0 += 64) rb[irb++] = RootBlock{g, i0};
      for (int i0 = 0; i0 < nd.n; i0 += 256) ob[iob++] = RootBlock{g, i0};
      for (int c2 = 0; c2 < nd.n; ++c2) {
        cm[ij] = g;
        cc[ij] = c2;
        ++ij;
      }
      for (int j0 = 0; j0 < nd.n; j0 += 8) {
        tm[it] = g;
        tc[it] = j0;
        ++it;
      }
      const int rows[2] = {nd.n / 2, nd.n - nd.n / 2};
      for (int half = 0; half < 2; ++half) {
        GemmProb& A = ga[2 * g + half];
        GemmProb& B = gb[2 * g + half];
        GemmProb& C = gc[2 * g + half];
        A.M = B.M = C.M = rows[half];
        A.tiles_m = B.tiles_m = (rows[half] + 127) / 128;
        C.tiles_m = (rows[half] + 255) / 256;
        A.tile0 = t128;
        B.tile0 = t64;
        C.tile0 = tbig;
        t128 += A.tiles_m * ((nd.n + 127) / 128);
        t64 += B.tiles_m * ((nd.n + 63) / 64);
        tbig += C.tiles_m * ((nd.n + 127) / 128);
      }
    }
  }
  *out = e;
  return ADC_OK;
}

// caller pointers into the descriptors: leaf outputs, merge blocks, input and
// output pointer arrays
void fill_pointers(BEntry* e, const double* const* diag, const double* const* offdiag, double* const* w,
                   double* const* Z, const int64_t* ldz) {
  char* h = e->hdesc.data();
  const int count = (int)e->N.size();
  for (int l = 0; l < e->nleaf; ++l) {
    const Node& nd = e->leaves[l];
    const int i = nd.mat;
    const int64_t r = nd.s0 - e->g0[i];
    const bool user = (e->leaf_depth[l] & 1) == 0;
    double* base = user ? Z[i] : e->Zb[i];
    const int64_t ld = user ? ldz[i] : e->N[i];
    ((LeafOut*)(h + e->o_lo))[l] = LeafOut{base + r + r * ld, ld};
  }
  for (int i = 0; i < count; ++i) {
    ((const double**)(h + e->o_pd))[i] = diag[i];
    ((const double**)(h + e->o_po))[i] = offdiag[i];
    ((double**)(h + e->o_pw))[i] = w[i];
  }
  for (size_t t = 0; t < e->levels.size(); ++t) {
    BLevel& L = e->levels[t];
    MergeDev* hm = (MergeDev*)(h + L.o_m);
    const bool user = (t % 2) == 0;
    for (int g = 0; g < L.nm; ++g) {
      const Node& nd = e->lev_nodes[t][g];
      const int i = nd.mat;
      const int64_t r = nd.s0 - e->g0[i];
      double* zn = user ? Z[i] : e->Zb[i];
      const int64_t ldn = user ? ldz[i] : e->N[i];
      const double* zo = user ? e->Zb[i] : Z[i];
      const int64_t ldo = user ? e->N[i] : ldz[i];
      MergeDev& M = hm[g];
      M.zn = zn + r + r * ldn;
      M.ldn = ldn;
      M.zo = zo + r + r * ldo;
      M.ldo = ldo;
    }
  }
}

LevelBufs level_bufs(BEntry* e) {
  LevelBufs B{};
  B.w_in = e->w;
  B.w_out = e->w;
  B.off = e->offg;
  B.dsort = e->dsort;
  B.zsort = e->zsort;
  B.src = e->src;
  B.supp = e->supp;
  B.surv = e->surv;
  B.defl = e->defl;
  B.gorder = e->gorder;
  B.rot_i = e->rot_i;
  B.rot_j = e->rot_j;
  B.rot_f = e->rot_f;
  B.rot_c = e->rot_c;
  B.rot_s = e->rot_s;
  B.dS = e->dS;
  B.zS = e->zS;
  B.lam = e->lam;
  B.gam = e->gam;
  B.mu = e->mu;
  B.uh = e->uh;
  B.v = e->v;
  B.posR = e->posR;
  B.posD = e->posD;
  B.pk = e->pk;
  B.qc = e->qc;
  B.pidx = e->pidx;
  B.ginv = e->ginv;
  B.rot_i_of = e->rot_i_of;
  B.rot_j_of = e->rot_j_of;
  return B;
}

// Launch the secular / Loewner / v kernels of a level with W waves.
void launch_roots(BEntry* e, const BLevel& L, int W, hipStream_t st) {
  const MergeDev* dm = (const MergeDev*)(e->desc + L.o_m);
  const RootBlock* rb = (const RootBlock*)(e->desc + L.o_rb);
  hipLaunchKernelGGL(k_secular, dim3(L.nrb), dim3(64 * W), 0, st, dm, rb, e->dS, e->zS, e->lam, e->gam, e->mu,
                     e->max_iter, e->flags);
}

void launch_gemm(BEntry* e, const BLevel& L, int gv, hipStream_t st) {
  if (gv == 0)
    hipLaunchKernelGGL(k_gemm_f64, dim3(L.tiles[0]), dim3(512), 0, st, (const GemmProb*)(e->desc + L.o_ga),
                       2 * L.nm);
  else if (gv == 1)
    hipLaunchKernelGGL(k_gemm_f64_n64, dim3(L.tiles[1]), dim3(512), 0, st, (const GemmProb*)(e->desc + L.o_gb),
                       2 * L.nm);
  else
    hipLaunchKernelGGL(k_gemm_f64_big, dim3(L.tiles[2]), dim3(1024), 0, st, (const GemmProb*)(e->desc + L.o_gc),
                       2 * L.nm, (const int*)(e->desc + L.o_gt));
}

// The whole device sequence.  With tune, every level times its candidate
// wave counts and tile widths (HIP events, synchronising after each
// candidate set) and re-runs the winner last, so that the results are those
// of the configuration the graph will hold.
// Before every call (eager or graph replay): the flags reset, the batch's
// inputs gathered into the entry's buffers and checked, so that non-finite
// input returns ADC_ERR_ARG before any solver kernel reads it.
adc_status gather_and_check(BEntry* e, hipStream_t st) {
  const int count = (int)e->N.size();
  const int64_t tot = e->Ntot;
  char* d = e->desc;
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, e->flags, INT32_MAX);
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, e->flags + 1, 0);
  hipLaunchKernelGGL(k_gather, dim3(count), dim3(256), 0, st, count, (const double* const*)(d + e->o_pd),
                     (const double* const*)(d + e->o_po), (const int64_t*)(d + e->o_g0),
                     (const int64_t*)(d + e->o_n), e->din, e->offg);
  hipLaunchKernelGGL(k_check_finite, dim3(256), dim3(256), 0, st, e->din, tot, e->flags + 1);
  hipLaunchKernelGGL(k_check_finite, dim3(256), dim3(256), 0, st, e->offg, tot, e->flags + 1);
  HIP_OK(hipGetLastError());
  int bad = 0;
  HIP_OK(hipMemcpyAsync(&bad, e->flags + 1, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  return bad ? ADC_ERR_ARG : ADC_OK;
}

// The solver sequence from the tear on (the gathered inputs are in place).
adc_status run_sequence(adc_ctx c, BCache* bc, BEntry* e, hipStream_t st, bool tune) {
  const int count = (int)e->N.size();
  const int64_t tot = e->Ntot;
  char* d = e->desc;
  hipLaunchKernelGGL(k_tear, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, e->din, e->offg,
                     (const int64_t*)(d + e->o_sp), e->nsplit, e->a, tot);
  launch_leaf_jacobi(st, e->nleaf, e->leaf, e->a, e->offg, (const int64_t*)(d + e->o_ls),
                     (const int32_t*)(d + e->o_lm), e->w, (const LeafOut*)(d + e->o_lo), 40);
  HIP_OK(hipGetLastError());
  const LevelBufs B = level_bufs(e);
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (tune) {
    HIP_OK(hipEventCreate(&ev[0]));
    HIP_OK(hipEventCreate(&ev[1]));
  }
  adc_status status = ADC_OK;
  for (int t = (int)e->levels.size() - 1; t >= 0 && status == ADC_OK; --t) {
    BLevel& L = e->levels[t];
    MergeDev* dm = (MergeDev*)(d + L.o_m);
    hipLaunchKernelGGL(k_merge_sort, dim3(L.nob), dim3(256), 0, st, dm, (const RootBlock*)(d + L.o_ob), B);
    hipLaunchKernelGGL(k_merge_prep, dim3(L.nm), dim3(prep_threads(L.nmax)), 0, st, dm, B);
    const auto key = std::make_tuple(L.nm, L.nmax, (int64_t)L.njob);
    if (tune && !L.tuned) {
      auto it = bc->tune.find(key);
      if (it != bc->tune.end()) {
        L.W = it->second.first;
        L.gv = it->second.second;
        L.tuned = true;
      }
    }
    const bool tune_here = tune && !L.tuned;
    auto timed = [&](auto&& fn) -> float {
      hipEventRecord(ev[0], st);
      fn();
      hipEventRecord(ev[1], st);
      hipEventSynchronize(ev[1]);
      float ms = 0.f;
      hipEventElapsedTime(&ms, ev[0], ev[1]);
      return ms;
    };
    // roots
    if (tune_here) {
      const int cand[3] = {1, 4, 8};
      int best = L.W, last = -1;
      float tb = 1e30f;
      for (int w : cand) {
        if (w > 1 && L.nmax < 32 * w) continue;
        const float ms = timed([&] { launch_roots(e, L, w, st); });
        last = w;
        if (ms < tb) {
          tb = ms;
          best = w;
        }
      }
      L.W = best;
      if (last != best) launch_roots(e, L, best, st);
    } else {
      launch_roots(e, L, L.W, st);
    }
    const RootBlock* rb = (const RootBlock*)(d + L.o_rb);
    hipLaunchKernelGGL(k_lowner, dim3(L.nrb), dim3(64 * L.W), 0, st, dm, rb, e->dS, e->zS, e->gam, e->mu, e->uh);
    hipLaunchKernelGGL(k_vnorm, dim3(L.nrb), dim3(64 * L.W), 0, st, dm, rb, e->dS, e->gam, e->mu, e->uh, e->v);
    hipLaunchKernelGGL(k_final_order, dim3(L.nob), dim3(256), 0, st, dm, B, (const RootBlock*)(d + L.o_ob));
    hipLaunchKernelGGL(k_pack_rot, dim3((unsigned)((L.njob + 3) / 4)), dim3(256), 0, st, dm,
                       (const int32_t*)(d + L.o_cm), (const int32_t*)(d + L.o_cc), B, (int)L.njob);
    hipLaunchKernelGGL(k_cauchy, dim3(L.ntile), dim3(256), 0, st, dm, (const int32_t*)(d + L.o_tm),
                       (const int32_t*)(d + L.o_tc), B, 8, 1);
    hipLaunchKernelGGL(k_build_probs, dim3((L.nm + 63) / 64), dim3(64), 0, st, dm, L.nm,
                       (GemmProb*)(d + L.o_ga), (GemmProb*)(d + L.o_gb), (GemmProb*)(d + L.o_gc), e->pk, e->qc,
                       e->v, e->posR);
    hipLaunchKernelGGL(k_gemm_compact, dim3(1), dim3(1024), 0, st, (GemmProb*)(d + L.o_gc), 2 * L.nm, 128,
                       (int*)(d + L.o_gt));
    if (tune_here) {
      // every tile shape writes the same values (same summation order)
      float best = 1e30f;
      for (int gv = 0; gv < 3; ++gv) {
        const float ms = timed([&] { launch_gemm(e, L, gv, st); });
        if (ms < best) {
          best = ms;
          L.gv = gv;
        }
      }
      L.tuned = true;
      bc->tune[key] = std::make_pair(L.W, L.gv);
    } else {
      launch_gemm(e, L, L.gv, st);
    }
    if (hipGetLastError() != hipSuccess) status = ADC_ERR_HIP;
  }
  if (ev[0]) hipEventDestroy(ev[0]);
  if (ev[1]) hipEventDestroy(ev[1]);
  if (status != ADC_OK) return status;
  hipLaunchKernelGGL(k_scatter_w, dim3(count), dim3(256), 0, st, count, e->w, (double* const*)(d + e->o_pw),
                     (const int64_t*)(d + e->o_g0), (const int64_t*)(d + e->o_n));
  HIP_OK(hipGetLastError());
  (void)c;
  return ADC_OK;
}

}  // namespace

void batch_release(adc_ctx c) {
  BCache* bc = (BCache*)c->batch_cache;
  if (!bc) return;
  for (auto& kv : bc->entries) free_entry(kv.second);
  if (bc->cap) hipStreamDestroy(bc->cap);
  delete bc;
  c->batch_cache = nullptr;
}

extern "C" adc_status adc_stedc_batched(adc_ctx c, int32_t count, const int64_t* n, const double* const* diag,
                                        const double* const* offdiag, double* const* w, double* const* Z,
                                        const int64_t* ldz, const adc_opts* opts_in, adc_report* rep) {
  if (!c || count < 0 || (count > 0 && (!n || !diag || !offdiag || !w || !Z || !ldz))) return ADC_ERR_ARG;
  adc_opts o;
  if (opts_in) o = *opts_in;
  else adc_opts_default(&o);
  ADC_TRY(validate_opts_ext(o));
  for (int i = 0; i < count; ++i) {
    if (n[i] < 0 || n[i] > 1000000) return ADC_ERR_ARG;
    if (n[i] > 0 && (!diag[i] || !w[i] || !Z[i] || ldz[i] < n[i] || (n[i] > 1 && !offdiag[i]))) return ADC_ERR_ARG;
  }
  DeviceGuard g(c->device);
  const auto t_start = std::chrono::steady_clock::now();
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->info_index = -1;
  }
  // matrices whose merges may take the HSS update run one by one
  const bool hss_possible = !o.force_dense && o.hss_levels != 0;
  std::vector<int> solo, batch;
  for (int i = 0; i < count; ++i) {
    if (n[i] == 0) continue;
    // the top merge's dense update is at most 2 n (n1^2 + n2^2) flops
    const double n1 = (double)(n[i] / 2), n2 = (double)(n[i] - n[i] / 2);
    const double top_f = 2.0 * n[i] * (n1 * n1 + n2 * n2);
    if (hss_possible && n[i] >= o.hss_min_k && top_f >= o.hss_min_flops) solo.push_back(i);
    else batch.push_back(i);
  }
  if (!solo.empty()) {
    // together, level-batched, with the single-matrix sequencing
    std::vector<int64_t> sn, sl;
    std::vector<const double*> sd, so;
    std::vector<double*> sw, sz;
    for (int i : solo) {
      sn.push_back(n[i]);
      sd.push_back(diag[i]);
      so.push_back(offdiag[i]);
      sw.push_back(w[i]);
      sz.push_back(Z[i]);
      sl.push_back(ldz[i]);
    }
    adc_report r1;
    const adc_status st = stedc_forest(c, (int)solo.size(), sn.data(), sd.data(), so.data(), sw.data(), sz.data(),
                                       sl.data(), o, &r1);
    if (st != ADC_OK) {
      if (rep) {
        // the matrix that holds the reported global row
        rep->info_index = solo[0];
        int64_t g0 = 0;
        for (size_t u = 0; u < solo.size(); ++u) {
          if (r1.info_index >= g0 && r1.info_index < g0 + sn[u]) rep->info_index = solo[u];
          g0 += sn[u];
        }
      }
      return st;
    }
    if (rep) {
      rep->levels = std::max(rep->levels, r1.levels);
      rep->merges += r1.merges;
      rep->hss_merges += r1.hss_merges;
      rep->retries += r1.retries;
      rep->hss_fallbacks += r1.hss_fallbacks;
      rep->max_rank = std::max(rep->max_rank, r1.max_rank);
      rep->samples = std::max(rep->samples, r1.samples);
      for (int t = 0; t < 64; ++t) {
        rep->n_per_level[t] += r1.n_per_level[t];
        rep->K_per_level[t] += r1.K_per_level[t];
        rep->hss_per_level[t] += r1.hss_per_level[t];
      }
    }
  }
  if (batch.empty()) {
    if (rep)
      rep->t_phase[10] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return ADC_OK;
  }

  if (!c->batch_cache) c->batch_cache = new BCache();
  BCache* bc = (BCache*)c->batch_cache;
  std::vector<int64_t> Nb;
  std::vector<const double*> pd, po;
  std::vector<double*> pw, pz;
  std::vector<int64_t> pl;
  for (int i : batch) {
    Nb.push_back(n[i]);
    pd.push_back(diag[i]);
    po.push_back(offdiag[i] ? offdiag[i] : diag[i]);  // n = 1: never read
    pw.push_back(w[i]);
    pz.push_back(Z[i]);
    pl.push_back(ldz[i]);
  }
  const auto key = std::make_tuple(Nb, o.dc_leaf, o.max_iter);
  BEntry* e;
  auto it = bc->entries.find(key);
  if (it == bc->entries.end()) {
    ADC_TRY(build_entry(Nb, o.dc_leaf, o.max_iter, &e));
    bc->entries[key] = e;
  } else {
    e = it->second;
  }
  std::vector<const void*> ptrs;
  for (size_t q = 0; q < Nb.size(); ++q) {
    ptrs.push_back(pd[q]);
    ptrs.push_back(po[q]);
    ptrs.push_back(pw[q]);
    ptrs.push_back(pz[q]);
    ptrs.push_back((const void*)(intptr_t)pl[q]);
  }
  hipStream_t st = c->stream;
  if (ptrs != e->last_ptrs) {
    fill_pointers(e, pd.data(), po.data(), pw.data(), pz.data(), pl.data());
    HIP_OK(hipMemcpyAsync(e->desc, e->hdesc.data(), e->hdesc.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
    e->last_ptrs = ptrs;
  }
  ADC_TRY(gather_and_check(e, st));
  if (!e->captured) {
    // first call: eager run with tuning, then capture for later calls
    ADC_TRY(run_sequence(c, bc, e, st, true));
    HIP_OK(hipStreamSynchronize(st));
    if (!bc->cap) HIP_OK(hipStreamCreateWithFlags(&bc->cap, hipStreamNonBlocking));
    HIP_OK(hipStreamBeginCapture(bc->cap, hipStreamCaptureModeThreadLocal));
    const adc_status cs = run_sequence(c, bc, e, bc->cap, false);
    hipGraph_t gph = nullptr;
    const hipError_t ce = hipStreamEndCapture(bc->cap, &gph);
    if (cs != ADC_OK) {
      if (gph) hipGraphDestroy(gph);
      return cs;
    }
    if (ce != hipSuccess || !gph) return ADC_ERR_HIP;
    e->graph = gph;
    if (hipGraphInstantiate(&e->exec, gph, nullptr, nullptr, 0) != hipSuccess) {
      e->exec = nullptr;
      return ADC_ERR_HIP;
    }
    e->captured = true;
  } else {
    HIP_OK(hipGraphLaunch(e->exec, st));
  }
  int flags[2] = {0, 0};
  HIP_OK(hipMemcpyAsync(flags, e->flags, 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  if (rep) {
    const int nlev = (int)e->levels.size();
    rep->levels = std::max(rep->levels, nlev);
    for (int t = 0; t < nlev; ++t) {
      const BLevel& L = e->levels[t];
      std::vector<MergeDev> ms(L.nm);
      HIP_OK(hipMemcpy(ms.data(), e->desc + L.o_m, L.nm * sizeof(MergeDev), hipMemcpyDeviceToHost));
      for (auto& M : ms) {
        rep->n_per_level[t] += M.n;
        rep->K_per_level[t] += M.K;
      }
      rep->merges += L.nm;
    }
    rep->t_phase[10] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  }
  if (flags[1]) return ADC_ERR_ARG;
  if (flags[0] != INT32_MAX) {
    if (rep) rep->info_index = flags[0];
    return ADC_ERR_NOCONV;
  }
  return ADC_OK;
}
