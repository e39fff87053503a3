// Merge-step kernels around the secular solve (Algorithm 1: the rank-one
// problem of the two children's spectra, deflation, and the assembly of the
// merged eigenpairs).
//
// k_merge_sort   the stable merge of the two sorted child spectra, one thread
//                per element (binary search in the other child), with the
//                entries of z = [last row of Q1; first row of Q2] (second
//                half negated when b_k < 0, eq. T3), not yet normalised.
// k_merge_prep   rho = |b_k| ||z||^2, z normalised; deflation with
//                tol = 8 eps max(max|d|, rho max|z|): type 1 when |rho z_j| <=
//                tol, type 2 (a Givens rotation of two columns) when the
//                coupling |(d_j - d_i) c s| <= tol.  The scan is sequential
//                in the pole order and runs on one lane per merge.
// k_final_order  merged eigenvalues in ascending order (roots before
//                deflated values on ties, deflated values in scan order).
// k_rotate       applies the type-2 rotations to the eigenvector columns in
//                place; the rows outside a column's support are implicit
//                zeros of the block-diagonal diag(Q1, Q2).
// k_pack         survivor columns into a dense n x K operand; deflated
//                columns straight to their final place.
// k_cauchy       the Cauchy-like matrix uh_i/(d_i - lam_j) (eq. Ev-Q without
//                the column scale v, which the GEMM applies), differences by
//                eq. (d-lambda).
#include "common.hpp"
#include "kernels.hpp"

namespace {

__device__ __forceinline__ int lower_bound_d(const double* __restrict__ x, int n, double v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (x[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int upper_bound_d(const double* __restrict__ x, int n, double v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (x[mid] <= v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <typename T, typename Op>
__device__ T block_reduce(T x, T* sh, Op op) {
  const int tid = threadIdx.x;
  sh[tid] = x;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (tid < st) sh[tid] = op(sh[tid], sh[tid + st]);
    __syncthreads();
  }
  T r = sh[0];
  __syncthreads();
  return r;
}

struct OpAdd {
  __device__ double operator()(double a, double b) const { return a + b; }
};
struct OpMax {
  __device__ double operator()(double a, double b) const { return fmax(a, b); }
};

// Exclusive prefix sum of one int per thread over the block; sh needs
// blockDim.x + 1 ints and holds the total at sh[blockDim.x] on return.
__device__ int block_exclusive_scan(int x, int* sh) {
  const int tid = threadIdx.x;
  __syncthreads();
  sh[tid] = x;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const int y = (tid >= off) ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += y;
    __syncthreads();
  }
  const int incl = sh[tid];
  if (tid == blockDim.x - 1) sh[blockDim.x] = incl;
  __syncthreads();
  return incl - x;
}

}  // namespace

// ---------------------------------------------------------------------------
// Blocks of 256 elements (merge, first element), one thread per element j of
// the merge: its place in the merged order is j plus the number of the other
// child's values below it (ties: the first child's value first), where it
// writes d_j, u_j = z_j before normalisation, its origin j and its support.
__global__ void __launch_bounds__(256) k_merge_sort(const MergeDev* __restrict__ merges,
                                                    const RootBlock* __restrict__ blocks, LevelBufs B) {
  const RootBlock rb = blocks[blockIdx.x];
  const MergeDev& M = merges[rb.merge];
  const int n = M.n, n1 = M.n1, n2 = n - n1;
  const int j = rb.i0 + (int)threadIdx.x;
  if (j >= n) return;
  const int64_t s0 = M.s0;
  const double beta = B.off[s0 + n1 - 1];
  const double sg = (beta >= 0.0) ? 1.0 : -1.0;
  const double* __restrict__ win = B.w_in + s0;
  const double u = (j < n1) ? M.zo[(n1 - 1) + j * M.ldo] : sg * M.zo[n1 + j * M.ldo];
  const double dj = win[j];
  const int pos = (j < n1) ? j + lower_bound_d(win + n1, n2, dj) : (j - n1) + upper_bound_d(win, n1, dj);
  B.dsort[s0 + pos] = dj;
  B.zsort[s0 + pos] = u;
  B.src[s0 + pos] = j;
  B.supp[s0 + pos] = (j < n1) ? 1 : 2;
}

__global__ void __launch_bounds__(1024) k_merge_prep(MergeDev* __restrict__ merges, LevelBufs B) {
  __shared__ double sh[PREP_VL + 1];
  MergeDev& M = merges[blockIdx.x];
  const int64_t s0 = M.s0;
  const int n = M.n, n1 = M.n1;
  const double beta = B.off[s0 + n1 - 1];
  const int tid = threadIdx.x;

  // ||u||^2 over the merged order (k_merge_sort placed u unnormalised), in
  // one fixed order whatever the block size: 1024 partial sums, partial v
  // over the entries v, v + 1024, ..., then added pairwise (v, v + 512),
  // (v, v + 256), ...; so every launch shape gives the same bits.
  for (int v = tid; v < PREP_VL; v += blockDim.x) {
    double ss = 0.0;
    for (int p = v; p < n; p += PREP_VL) {
      const double u = B.zsort[s0 + p];
      ss += u * u;
    }
    sh[v] = ss;
  }
  __syncthreads();
  for (int st = PREP_VL / 2; st > 0; st >>= 1) {
    for (int v = tid; v < st; v += blockDim.x) sh[v] += sh[v + st];
    __syncthreads();
  }
  const double nu2 = sh[0];
  __syncthreads();
  const double rho = fabs(beta) * nu2;
  const double inv = (nu2 > 0.0) ? 1.0 / sqrt(nu2) : 0.0;

  double md = 0.0, mz = 0.0;
  for (int p = tid; p < n; p += blockDim.x) {
    const double zj = B.zsort[s0 + p] * inv;
    B.zsort[s0 + p] = zj;
    md = fmax(md, fabs(B.dsort[s0 + p]));
    mz = fmax(mz, fabs(zj));
  }
  md = block_reduce(md, sh, OpMax());
  mz = block_reduce(mz, sh, OpMax());
  const double tol = 8.0 * ADC_EPS * fmax(md, rho * mz);
  __syncthreads();

  // --- type-1 flags and the candidate list (positions that are not type 1),
  // each candidate's rotation test against its predecessor candidate taken
  // with the original values; scratch: posD = candidate list, posR = flags,
  // gam / lam / mu = r, c, s of that test.
  int32_t* __restrict__ cand = B.posD + s0;
  int32_t* __restrict__ flg = B.posR + s0;
  double* __restrict__ tr_r = B.gam + s0;
  double* __restrict__ tr_c = B.lam + s0;
  double* __restrict__ tr_s = B.mu + s0;
  const double* __restrict__ ds0 = B.dsort + s0;
  const double* __restrict__ zs0 = B.zsort + s0;
  int* shi = reinterpret_cast<int*>(sh);
  const int per = (n + blockDim.x - 1) / blockDim.x;
  const int j0 = tid * per, j1 = min(n, j0 + per);
  int cnt = 0;
  for (int j = j0; j < j1; ++j) cnt += !(rho * fabs(zs0[j]) <= tol);
  const int base = block_exclusive_scan(cnt, shi);
  for (int j = j0, q = base; j < j1; ++j)
    if (!(rho * fabs(zs0[j]) <= tol)) cand[q++] = j;
  __syncthreads();
  const int ncand = shi[blockDim.x];  // total written by the scan
  __syncthreads();
  for (int q = tid; q < n; q += blockDim.x) flg[q] = 1;  // type 1 unless listed below
  __syncthreads();
  for (int q = tid; q < ncand; q += blockDim.x) {
    const int j = cand[q];
    int f = 0;
    if (q > 0) {
      const int i = cand[q - 1];
      const double zi = zs0[i], zj = zs0[j];
      const double r = hypot(zi, zj);
      const double c = zj / r, s = -zi / r;
      tr_r[j] = r;
      tr_c[j] = c;
      tr_s[j] = s;
      f = (fabs((ds0[j] - ds0[i]) * c * s) <= tol) ? 2 : 0;
    }
    flg[j] = f;
  }
  __syncthreads();

  // --- parallel resolution of the scan.  With R[q] "candidate q is rotated
  // with its predecessor", T[q] the test with original values (bit 2) and
  // F[q] the test after q-1 was itself rotated with q-2 (bit 4), the scan
  // obeys R[0] = 0, R[q] = R[q-1] ? F[q] : T[q]: a composition of maps on
  // {0, 1}, resolved by a block-wide scan.  F[q] assumes that rotation of q-1
  // started from original values, which holds unless two rotations are
  // adjacent; then the lane-by-lane scan below takes over.
  for (int q = 2 + tid; q < ncand; q += blockDim.x) {
    const int i2 = cand[q - 2], i1 = cand[q - 1], j = cand[q];
    const double c1 = tr_c[i1], s1 = tr_s[i1];
    const double pd = s1 * s1 * ds0[i2] + c1 * c1 * ds0[i1];
    const double pz = tr_r[i1];
    const double zj = zs0[j];
    const double r = hypot(pz, zj);
    const double c = zj / r, s = -pz / r;
    if (fabs((ds0[j] - pd) * c * s) <= tol) flg[j] |= 4;
  }
  __syncthreads();
  // maps encoded as out(0) | out(1) << 1; identity = 2; a-then-b composition
  auto mbit = [](int m, int b) { return (m >> b) & 1; };
  auto mcomp = [&](int a, int b) { return mbit(b, mbit(a, 0)) | (mbit(b, mbit(a, 1)) << 1); };
  const int perQ = (ncand + blockDim.x - 1) / blockDim.x;
  const int qa = min(ncand, tid * perQ), qb = min(ncand, qa + perQ);
  int mp = 2;
  for (int q = qa; q < qb; ++q) {
    const int f = flg[cand[q]];
    const int mq = (q == 0) ? 0 : (((f >> 1) & 1) | (((f >> 2) & 1) << 1));
    mp = mcomp(mp, mq);
  }
  __syncthreads();
  shi[tid] = mp;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const int y = (tid >= off) ? shi[tid - off] : 2;
    __syncthreads();
    shi[tid] = mcomp(y, shi[tid]);
    __syncthreads();
  }
  int bcur = (tid == 0) ? 0 : mbit(shi[tid - 1], 0);
  __syncthreads();
  for (int q = qa; q < qb; ++q) {
    const int f = flg[cand[q]];
    const int mq = (q == 0) ? 0 : (((f >> 1) & 1) | (((f >> 2) & 1) << 1));
    bcur = mbit(mq, bcur);
    if (bcur) flg[cand[q]] = f | 8;
  }
  __syncthreads();
  __shared__ int s_adj;
  if (tid == 0) s_adj = 0;
  __syncthreads();
  for (int q = 1 + tid; q < ncand; q += blockDim.x)
    if ((flg[cand[q]] & 8) && (flg[cand[q - 1]] & 8)) s_adj = 1;
  __syncthreads();
  const bool parallel_ok = (s_adj == 0);

  __shared__ int st_K, st_nd, st_nrot, st_prev, st_psupp, st_pmod;
  __shared__ double st_pd, st_pz;
  int32_t* __restrict__ sp = B.supp + s0;
  double* __restrict__ ds = B.dsort + s0;
  double* __restrict__ zs = B.zsort + s0;
  if (parallel_ok) {
    // every position of this thread's range [j0, j1): type 1, rotated into
    // (the predecessor deflates, event here), deflated by its successor, or
    // survivor; lists in position order of their events
    int q = base;  // candidate index of the first candidate in the range
    int nev = 0, nsv = 0, nrt = 0;
    for (int j = j0; j < j1; ++j) {
      const int f = flg[j];
      if (f == 1) {
        ++nev;
        continue;
      }
      const bool rin = f & 8;
      const bool rnext = (q + 1 < ncand) && (flg[cand[q + 1]] & 8);
      nev += rin;
      nrt += rin;
      nsv += !rnext;
      ++q;
    }
    const int bev = block_exclusive_scan(nev, shi);
    const int tot_ev = shi[blockDim.x];
    __syncthreads();
    const int bsv = block_exclusive_scan(nsv, shi);
    const int tot_sv = shi[blockDim.x];
    __syncthreads();
    const int brt = block_exclusive_scan(nrt, shi);
    const int tot_rt = shi[blockDim.x];
    __syncthreads();
    q = base;
    int iev = bev, isv = bsv, irt = brt;
    for (int j = j0; j < j1; ++j) {
      const int f = flg[j];
      if (f == 1) {
        B.defl[s0 + iev++] = j;
        continue;
      }
      const bool rin = f & 8;
      const bool rnext = (q + 1 < ncand) && (flg[cand[q + 1]] & 8);
      double pd = ds0[j], pz = zs0[j];
      if (rin) {
        const int i = cand[q - 1];
        const double c = tr_c[j], s = tr_s[j];
        const double di = ds0[i];
        B.defl[s0 + iev++] = i;
        B.rot_i[s0 + irt] = i;
        B.rot_j[s0 + irt] = j;
        B.rot_c[s0 + irt] = c;
        B.rot_s[s0 + irt] = s;
        B.rot_f[s0 + irt] = sp[i] | (sp[j] << 2);
        ++irt;
        ds[i] = c * c * di + s * s * pd;
        pd = s * s * di + c * c * pd;
        pz = tr_r[j];
      }
      if (!rnext) {
        B.surv[s0 + isv] = j;
        B.dS[s0 + isv] = pd;
        B.zS[s0 + isv] = pz;
        ++isv;
      }
      ++q;
    }
    __syncthreads();
    // supports of rotated pairs become the union (after every flag was read)
    for (int t = tid; t < tot_rt; t += blockDim.x) {
      const int i = B.rot_i[s0 + t], j = B.rot_j[s0 + t];
      const int u = sp[i] | sp[j];
      sp[i] = u;
      sp[j] = u;
      zs[i] = 0.0;
    }
    if (tid == 0) {
      st_K = tot_sv;
      st_nd = tot_ev;
      st_nrot = tot_rt;
    }
    __syncthreads();
  }

  // --- the scan in pole order, one lane, over LDS-staged chunks; the test of
  // a candidate is recomputed only when its predecessor was just rotated.
  constexpr int CH = 2048;
  __shared__ double c_d[CH], c_z[CH], c_r[CH], c_c[CH], c_s[CH];
  __shared__ int c_f[CH], c_p[CH];
  if (tid == 0 && !parallel_ok) {
    st_K = st_nd = st_nrot = 0;
    st_prev = -1;
    st_psupp = 0;
    st_pmod = 0;
    st_pd = st_pz = 0.0;
  }
  for (int c0 = 0; !parallel_ok && c0 < n; c0 += CH) {
    const int cl = min(CH, n - c0);
    __syncthreads();
    for (int t = tid; t < cl; t += blockDim.x) {
      const int j = c0 + t;
      c_d[t] = ds0[j];
      c_z[t] = zs0[j];
      c_f[t] = flg[j];
      c_p[t] = sp[j];
      c_r[t] = tr_r[j];
      c_c[t] = tr_c[j];
      c_s[t] = tr_s[j];
    }
    __syncthreads();
    if (tid == 0) {
      int K = st_K, nd = st_nd, nrot = st_nrot, prev = st_prev, psupp = st_psupp, pmod = st_pmod;
      double pd = st_pd, pz = st_pz;
      int32_t* __restrict__ surv = B.surv + s0;
      int32_t* __restrict__ defl = B.defl + s0;
      double* __restrict__ dS = B.dS + s0;
      double* __restrict__ zS = B.zS + s0;
      for (int t = 0; t < cl; ++t) {
        const int j = c0 + t;
        const int f = c_f[t];
        if (f == 1) {
          defl[nd++] = j;
          continue;
        }
        const double dj = c_d[t], zj = c_z[t];
        if (prev < 0) {
          prev = j;
          pd = dj;
          pz = zj;
          psupp = c_p[t];
          pmod = 0;
          continue;
        }
        double r, c, s;
        bool rot;
        if (!pmod) {
          r = c_r[t];
          c = c_c[t];
          s = c_s[t];
          rot = (f & 2) != 0;
        } else {
          r = hypot(pz, zj);
          c = zj / r;
          s = -pz / r;
          rot = fabs((dj - pd) * c * s) <= tol;
        }
        if (rot) {
          const int fj = c_p[t];
          B.rot_i[s0 + nrot] = prev;
          B.rot_j[s0 + nrot] = j;
          B.rot_c[s0 + nrot] = c;
          B.rot_s[s0 + nrot] = s;
          B.rot_f[s0 + nrot] = psupp | (fj << 2);
          ++nrot;
          psupp |= fj;
          sp[prev] = psupp;
          sp[j] = psupp;
          ds[prev] = c * c * pd + s * s * dj;
          zs[prev] = 0.0;
          defl[nd++] = prev;
          pd = s * s * pd + c * c * dj;
          pz = r;
          prev = j;
          pmod = 1;
        } else {
          surv[K] = prev;
          dS[K] = pd;
          zS[K] = pz;
          ++K;
          prev = j;
          pd = dj;
          pz = zj;
          psupp = c_p[t];
          pmod = 0;
        }
      }
      st_K = K;
      st_nd = nd;
      st_nrot = nrot;
      st_prev = prev;
      st_psupp = psupp;
      st_pmod = pmod;
      st_pd = pd;
      st_pz = pz;
    }
  }
  __syncthreads();
  if (tid == 0 && !parallel_ok && st_prev >= 0) {
    B.surv[s0 + st_K] = st_prev;
    B.dS[s0 + st_K] = st_pd;
    B.zS[s0 + st_K] = st_pz;
    ++st_K;
  }
  __syncthreads();
  const int K = st_K;

  // --- survivor groups by row support: top only (1), both (3), bottom only
  // (2), and the grouped order (stable inside every group)
  const int perK = (K + blockDim.x - 1) / blockDim.x;
  const int r0 = tid * perK, r1 = min(K, r0 + perK);
  int c1 = 0, c2 = 0, c3 = 0;
  for (int r = r0; r < r1; ++r) {
    const int f = sp[B.surv[s0 + r]];
    c1 += (f == 1);
    c2 += (f == 3);
    c3 += (f == 2);
  }
  const int b1 = block_exclusive_scan(c1, shi);
  const int k1 = shi[blockDim.x];
  __syncthreads();
  const int b2 = block_exclusive_scan(c2, shi);
  const int k2 = shi[blockDim.x];
  __syncthreads();
  const int b3 = block_exclusive_scan(c3, shi);
  const int k3 = shi[blockDim.x];
  __syncthreads();
  int32_t* __restrict__ go = B.gorder + s0;
  for (int r = r0, p1 = b1, p2 = k1 + b2, p3 = k1 + k2 + b3; r < r1; ++r) {
    const int f = sp[B.surv[s0 + r]];
    if (f == 1) go[p1++] = r;
    else if (f == 3) go[p2++] = r;
    else go[p3++] = r;
  }
  // --- maps used by the packing: role of every position, grouped position of
  // every survivor, rotation of every position
  const int nrot = st_nrot;
  for (int p = tid; p < n; p += blockDim.x) {
    B.rot_i_of[s0 + p] = -1;
    B.rot_j_of[s0 + p] = -1;
  }
  __syncthreads();
  for (int r = tid; r < K; r += blockDim.x) {
    B.pidx[s0 + B.surv[s0 + r]] = r;
    B.ginv[s0 + go[r]] = r;
  }
  for (int q = tid; q < n - K; q += blockDim.x) B.pidx[s0 + B.defl[s0 + q]] = -1 - q;
  for (int t = tid; t < nrot; t += blockDim.x) {
    B.rot_i_of[s0 + B.rot_i[s0 + t]] = t;
    B.rot_j_of[s0 + B.rot_j[s0 + t]] = t;
  }
  // deflated values in scan order: non-decreasing unless a rotated value
  // passed a pole deflated between the pair (then the ordering counts)
  double uns = 0.0;
  for (int q = tid + 1; q < n - K; q += blockDim.x)
    if (B.dsort[s0 + B.defl[s0 + q - 1]] > B.dsort[s0 + B.defl[s0 + q]]) uns = 1.0;
  uns = block_reduce(uns, sh, OpMax());
  if (tid == 0) {
    M.dsorted = (uns == 0.0) ? 1 : 0;
    M.K = K;
    M.nrot = nrot;
    M.k1 = k1;
    M.k2 = k2;
    M.k3 = k3;
    M.rho = rho;
    M.tol = tol;
  }
}

// ---------------------------------------------------------------------------
// HSS merges: the leaf boundaries and the rank estimate (Section 4.1).  From
// the balanced boundaries, every interior boundary b whose segments are
// closer than `thresh` moves by up to shift_max indices to the largest
// distance, boundaries taken in order (a window starts after the previous,
// already moved, boundary).  The distance of the segments split before b is
// min(|lam_b - d_{b-1}|, |d_b - lam_{b-1}|) by eq. (d-lambda); with
// interlacing roots it is mu_{b-1}, the first term never being smaller.
// Then every boundary gives the bound of eq. (bounds) with
// R = (lam_{K-1} - d_0) / dist and the merge's estimate is the largest,
// capped at r_cap (also for a zero distance).  One 64-lane workgroup per
// merge: lane 0 moves the boundaries, the lanes share the bounds.
__global__ void __launch_bounds__(64) k_leaf_bounds(MergeDev* __restrict__ merges,
                                                    const int32_t* __restrict__ which, LevelBufs B,
                                                    double thresh, int shift_max, double rank_eps, int r_cap) {
  __shared__ int rmax;
  MergeDev& M = merges[which[blockIdx.x]];
  const int64_t s0 = M.s0;
  const int K = M.K;
  const double* d = B.dS + s0;
  const double* gam = B.gam + s0;
  const double* mu = B.mu + s0;
  int32_t* bd = M.lbounds;
  auto dist = [&](int b) {
    const double x = (b < K) ? (d[b] - d[b - 1]) + gam[b] : INFINITY;
    return fmin(fabs(x), fabs(mu[b - 1]));
  };
  if (threadIdx.x == 0) {
    rmax = 0;
    for (int t = 1; t < M.nleaf; ++t) {
      const int b = bd[t];
      double best_d = dist(b);
      if (!(best_d < thresh)) continue;
      int best = b;
      const int lo = max(bd[t - 1] + 1, b - shift_max);
      const int hi = min(bd[t + 1] - 1, b + shift_max);
      for (int bb = lo; bb <= hi; ++bb) {
        const double dd = dist(bb);
        if (dd > best_d) {
          best = bb;
          best_d = dd;
        }
      }
      bd[t] = best;
    }
  }
  __syncthreads();
  const double span = (d[K - 1] + gam[K - 1]) - d[0];
  int r = 0;
  for (int t = 1 + (int)threadIdx.x; t < M.nleaf; t += 64) {
    const double ds = dist(bd[t]);
    const double R = (ds > 0.0) ? span / ds : INFINITY;
    int rb = r_cap;
    if (isfinite(R)) rb = min(r_cap, (int)ceil(log(16.0 / rank_eps) * log(8.0 * fmax(R, 1.0)) / (M_PI * M_PI)));
    r = max(r, rb);
  }
  atomicMax(&rmax, r);
  __syncthreads();
  if (threadIdx.x == 0) M.rest = min(rmax, r_cap);
}

// HSS merges: inside every leaf of the HSS tree (survivors in pole order)
// the packed columns are grouped by row support, top only, both, then bottom
// only (stable), so that each half of the rows meets one contiguous column
// range of the leaf in Algorithm 3.  Writes ginv (survivor -> packed column),
// gorder (packed column -> survivor) and lcnt[3 leaf + g], the three group
// sizes.  One workgroup per (merge, leaf); leaves hold at most 512 survivors
// (hss_leaf <= 256, boundaries moved by at most shift_max each).
__global__ void __launch_bounds__(512) k_leaf_group(const MergeDev* __restrict__ merges,
                                                    const int2* __restrict__ jobs, LevelBufs B) {
  __shared__ int grp[512];
  const int2 jb = jobs[blockIdx.x];
  const MergeDev& M = merges[jb.x];
  const int64_t s0 = M.s0;
  const int lo = M.lbounds[jb.y], hi = M.lbounds[jb.y + 1];
  const int m = hi - lo;
  const int t = threadIdx.x;
  int g = 3;
  if (t < m) {
    const int f = B.supp[s0 + B.surv[s0 + lo + t]];
    g = (f == 1) ? 0 : (f == 3) ? 1 : 2;
  }
  grp[t] = g;
  __syncthreads();
  if (t < m) {
    int pos = 0;
    for (int u = 0; u < m; ++u) {
      const int gu = grp[u];
      pos += (gu < g) || (gu == g && u < t);
    }
    B.ginv[s0 + lo + t] = lo + pos;
    B.gorder[s0 + lo + pos] = lo + t;
  }
  if (t < 3) {
    int cnt = 0;
    for (int u = 0; u < m; ++u) cnt += grp[u] == t;
    B.lcnt[s0 + 3 * jb.y + t] = cnt;
  }
}

// The zero rows of the packed operand of merge `g` (rows outside each
// column's support, which the packing leaves unwritten), for a product that
// reads whole columns.  One workgroup per packed column.
__global__ void __launch_bounds__(256) k_zero_unsupported(const MergeDev* __restrict__ merges, int g, LevelBufs B) {
  const MergeDev& M = merges[g];
  const int c = blockIdx.x;
  if (c >= M.K) return;
  const int64_t s0 = M.s0;
  const int f = B.supp[s0 + B.surv[s0 + B.gorder[s0 + c]]];
  const int n = M.n, n1 = M.n1;
  double* col = B.pk + M.zoff + (int64_t)c * n;
  const int lo = (f & 1) ? n1 : 0, hi = (f & 2) ? n1 : n;  // the unsupported half
  if (f == 3) return;
  for (int r = lo + threadIdx.x; r < hi; r += blockDim.x) col[r] = 0.0;
}

// Packing with the type-2 rotations applied on the fly.  One block per sorted
// position of the level (job -> merge col_merge[job], position col_idx[job]).
// A position untouched by rotations copies its column; the first position of
// a rotation chain (rot_i[t+1] == rot_j[t]) carries the chain's columns
// through its rotations, writing every deflated column to its final place in
// the merged block and the last (surviving) column into the packed operand;
// the other chain members do nothing.  Rows outside a column's original
// support are the zeros of diag(Q1, Q2).
// With heads = false a plain position is copied and a chain head only
// reported (true); with heads = true the chain of a head is carried.
__device__ __forceinline__ bool pack_rot_job(const MergeDev* __restrict__ merges,
                                             const int32_t* __restrict__ col_merge,
                                             const int32_t* __restrict__ col_idx, const LevelBufs& B, int job,
                                             int tid, int bs, bool heads) {
  constexpr int CHMAX = 8;  // rotation steps held in registers
  constexpr int RU = 4;     // rows per lane and iteration of a chain (loads in flight)
  constexpr int RC = 8;     // the same for a plain copy
  const MergeDev& M = merges[col_merge[job]];
  const int64_t s0 = M.s0;
  const int n = M.n, n1 = M.n1;
  const int p = col_idx[job];
  if (B.rot_j_of[s0 + p] >= 0) return false;  // inside a chain: done by its head
  auto dst_of = [&](int pos) -> double* {
    const int role = B.pidx[s0 + pos];
    if (role >= 0) {
      const int pk = B.ginv[s0 + role];
      return B.pk + M.zoff + (int64_t)pk * n;
    }
    const int q = -1 - role;
    return M.zn + B.posD[s0 + q] * M.ldn;
  };
  auto src_of = [&](int pos) -> const double* { return M.zo + B.src[s0 + pos] * M.ldo; };
  auto supp_of = [&](int pos) { return (B.src[s0 + pos] < n1) ? 1 : 2; };
  const int t0 = B.rot_i_of[s0 + p];
  if (t0 >= 0 && !heads) return true;
  if (t0 < 0) {
    const double* __restrict__ sc = src_of(p);
    double* __restrict__ dc = dst_of(p);
    const int f = supp_of(p);
    // rows outside the support are zero; no product reads them in a packed
    // column (the grouped GEMMs of the dense update and the row-half
    // products of Algorithm 3 skip them; the dense fallback of a failed HSS
    // merge fills them first), a deflated column's final place needs them
    const bool zero = B.pidx[s0 + p] < 0;
    const int lo = (f & 1) ? 0 : n1, hi = (f & 2) ? n : n1;
    if (zero) {
      for (int r = tid; r < lo; r += bs) dc[r] = 0.0;
      for (int r = hi + tid; r < n; r += bs) dc[r] = 0.0;
    }
    int r = lo + tid;
    for (; r + (RC - 1) * bs < hi; r += RC * bs) {
      double x[RC];
#pragma unroll
      for (int v = 0; v < RC; ++v) x[v] = sc[r + v * bs];
#pragma unroll
      for (int v = 0; v < RC; ++v) dc[r + v * bs] = x[v];
    }
    for (; r < hi; r += bs) dc[r] = sc[r];
    return false;
  }
  // chain t0, t0+1, ... while rot_i[t+1] == rot_j[t]
  const int nrot = M.nrot;
  int t1 = t0;
  while (t1 + 1 < nrot && B.rot_i[s0 + t1 + 1] == B.rot_j[s0 + t1]) ++t1;
  const int fa = supp_of(p);
  const double* __restrict__ sa = src_of(p);
  if (t1 - t0 < CHMAX) {
    // every step's operands in registers, so that the row loop reloads
    // nothing but the column entries
    const int L = t1 - t0 + 1;
    const double* sj[CHMAX];
    double* di[CHMAX];
    double cs[CHMAX], sn[CHMAX];
    int fj[CHMAX];
#pragma unroll
    for (int u = 0; u < CHMAX; ++u) {
      if (u < L) {
        const int t = t0 + u;
        const int pj = B.rot_j[s0 + t];
        sj[u] = src_of(pj);
        fj[u] = supp_of(pj);
        di[u] = dst_of(B.rot_i[s0 + t]);
        cs[u] = B.rot_c[s0 + t];
        sn[u] = B.rot_s[s0 + t];
      }
    }
    double* __restrict__ dlast = dst_of(B.rot_j[s0 + t1]);
    // rows of the first child, then of the second: which source columns
    // have support there is fixed per half, so the loads are unconditional
    // inside the loop and four rows of them are in flight
    for (int half = 0; half < 2; ++half) {
      const int bit = half ? 2 : 1;
      const int r0 = half ? n1 : 0, r1 = half ? n : n1;
      const bool ha = (fa & bit) != 0;
      bool hj[CHMAX];
#pragma unroll
      for (int u = 0; u < CHMAX; ++u) hj[u] = (u < L) && (fj[u] & bit) != 0;
      int r = r0 + tid;
      for (; r + (RU - 1) * bs < r1; r += RU * bs) {
        double a[RU];
#pragma unroll
        for (int v = 0; v < RU; ++v) a[v] = ha ? sa[r + v * bs] : 0.0;
#pragma unroll
        for (int u = 0; u < CHMAX; ++u) {
          if (u < L) {
            const double* __restrict__ su = sj[u];
            double* __restrict__ du = di[u];
            double b[RU];
#pragma unroll
            for (int v = 0; v < RU; ++v) b[v] = hj[u] ? su[r + v * bs] : 0.0;
#pragma unroll
            for (int v = 0; v < RU; ++v) {
              du[r + v * bs] = cs[u] * a[v] + sn[u] * b[v];
              a[v] = -sn[u] * a[v] + cs[u] * b[v];
            }
          }
        }
#pragma unroll
        for (int v = 0; v < RU; ++v) dlast[r + v * bs] = a[v];
      }
      for (; r < r1; r += bs) {
        double a = ha ? sa[r] : 0.0;
#pragma unroll
        for (int u = 0; u < CHMAX; ++u) {
          if (u < L) {
            const double b = hj[u] ? sj[u][r] : 0.0;
            di[u][r] = cs[u] * a + sn[u] * b;
            a = -sn[u] * a + cs[u] * b;
          }
        }
        dlast[r] = a;
      }
    }
    return false;
  }
  for (int r = tid; r < n; r += bs) {
    const int bit = (r < n1) ? 1 : 2;
    double a = (fa & bit) ? sa[r] : 0.0;
    for (int t = t0; t <= t1; ++t) {
      const int pj = B.rot_j[s0 + t];
      const double c = B.rot_c[s0 + t], s = B.rot_s[s0 + t];
      const double b = (supp_of(pj) & bit) ? src_of(pj)[r] : 0.0;
      dst_of(B.rot_i[s0 + t])[r] = c * a + s * b;
      a = -s * a + c * b;
    }
    dst_of(B.rot_j[s0 + t1])[r] = a;
  }
  return false;
}

// Four consecutive jobs per workgroup, one wavefront each for a plain copy
// (a short column is a few rows per lane, a long one keeps eight loads per
// lane in flight); the heads of rotation chains among them are then carried
// by the whole workgroup, one after the other (a chain's steps are
// sequential per row, so its rows need every lane).  Jobs are strided over
// the grid: with fewer workgroups than jobs the packing leaves room on the
// CUs for a kernel that needs a whole CU's LDS (the node compression, which
// runs beside the packing at HSS levels; the solver launches two workgroups
// per CU there).
__global__ void __launch_bounds__(256) k_pack_rot(const MergeDev* __restrict__ merges,
                                                  const int32_t* __restrict__ col_merge,
                                                  const int32_t* __restrict__ col_idx, LevelBufs B, int njob) {
  __shared__ int s_head[4];
  const int wv = wave_index(), lane = threadIdx.x & 63;
  for (int base = blockIdx.x * 4; base < njob; base += gridDim.x * 4) {
    const int job = base + wv;
    const bool head = job < njob && pack_rot_job(merges, col_merge, col_idx, B, job, lane, 64, false);
    if (lane == 0) s_head[wv] = head ? job : -1;
    __syncthreads();
    for (int u = 0; u < 4; ++u) {
      const int hj = s_head[u];
      if (hj >= 0) pack_rot_job(merges, col_merge, col_idx, B, hj, (int)threadIdx.x, 256, true);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// blocks: RootBlock(merge, i0) with 256 items each, items [0, K) are roots,
// [K, n) deflated values.
__global__ void __launch_bounds__(256) k_final_order(const MergeDev* __restrict__ merges, LevelBufs B,
                                                     const RootBlock* __restrict__ blocks) {
  __shared__ double tile[256];
  const RootBlock rb = blocks[blockIdx.x];
  const MergeDev& M = merges[rb.merge];
  const int64_t s0 = M.s0;
  const int n = M.n, K = M.K, D = n - K;
  const int item = rb.i0 + threadIdx.x;
  if (rb.i0 >= n) return;
  const bool valid = item < n;
  const bool isroot = item < K;
  const int q = item - K;
  double x = 0.0;
  if (valid) x = isroot ? B.lam[s0 + item] : B.dsort[s0 + B.defl[s0 + q]];
  int cnt = 0;
  if (M.dsorted) {
    // sorted deflated values: a root counts those strictly below it (binary
    // search), a deflated value counts exactly its predecessors
    if (valid) {
      if (isroot) {
        const int32_t* __restrict__ df = B.defl + s0;
        const double* __restrict__ ds = B.dsort + s0;
        int lo = 0, hi = D;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (ds[df[mid]] < x) lo = mid + 1;
          else hi = mid;
        }
        cnt = lo;
      } else {
        cnt = q;
      }
    }
  } else
  for (int t0 = 0; t0 < D; t0 += 256) {
    const int tq = t0 + threadIdx.x;
    tile[threadIdx.x] = (tq < D) ? B.dsort[s0 + B.defl[s0 + tq]] : 0.0;
    __syncthreads();
    const int lim = min(256, D - t0);
    if (valid) {
      if (isroot) {
        for (int u = 0; u < lim; ++u) cnt += tile[u] < x;
      } else {
        for (int u = 0; u < lim; ++u) {
          const double y = tile[u];
          cnt += (y < x) || (y == x && (t0 + u) < q);
        }
      }
    }
    __syncthreads();
  }
  if (!valid) return;
  int pos;
  if (isroot) {
    pos = item + cnt;
    B.posR[s0 + item] = pos;
  } else {
    pos = upper_bound_d(B.lam + s0, K, x) + cnt;
    B.posD[s0 + q] = pos;
  }
  B.w_out[s0 + pos] = x;
}

// ---------------------------------------------------------------------------
// Cauchy matrix qc(r', j) = uh_i / (d_i - lam_j), i = gorder[r'] (grouped) or
// r'; column-major with leading dimension K.  One block per (merge, column
// tile of ncols columns); tile lists built by the host.
__global__ void __launch_bounds__(256) k_cauchy(const MergeDev* __restrict__ merges,
                                                const int32_t* __restrict__ tile_merge,
                                                const int32_t* __restrict__ tile_col0, LevelBufs B, int ncols,
                                                int grouped) {
  const MergeDev& M = merges[tile_merge[blockIdx.x]];
  const int K = M.K;
  const int j0 = tile_col0[blockIdx.x];
  if (j0 >= K) return;
  const int64_t s0 = M.s0;
  const double* __restrict__ d = B.dS + s0;
  const double* __restrict__ gam = B.gam + s0;
  const double* __restrict__ mu = B.mu + s0;
  const double* __restrict__ uh = B.uh + s0;
  const int32_t* __restrict__ go = B.gorder + s0;
  double* __restrict__ qc = B.qc + M.zoff;
  const int j1 = min(K, j0 + ncols);
  for (int rr = threadIdx.x; rr < K; rr += blockDim.x) {
    const int i = grouped ? go[rr] : rr;
    const double di = d[i];
    const double ui = uh[i];
    for (int j = j0; j < j1; ++j) {
      const double dj = d[j];
      const double dj1 = (j + 1 < K) ? d[j + 1] : 0.0;
      const double dl = d_minus_lam(i, j, di, dj, dj1, gam[j], mu[j]);
      qc[rr + (int64_t)j * K] = ui / dl;
    }
  }
}
