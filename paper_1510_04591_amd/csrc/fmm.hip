// Fast sampling for Algorithm 2: the off-diagonal Cauchy sums
//   Phi_ic   = uh_i sum_{j not in t(i)} v_j  Omega_jc / (d_i - lam_j)
//   Theta_jc = v_j  sum_{i not in t(j)} uh_i Omega_ic / (d_i - lam_j)
// by a one-dimensional fast multipole method with Chebyshev interpolation on
// both sides of 1/(x - y), over the HSS tree (the FMM-accelerated sampling the
// paper names for lowering the O(K^2 s) sampling cost, Sections 1, 3 and 5).
//
// Geometry: a node [lo, hi) lives in coordinates local to its anchor pole
// d_lo; its interval is [0, w], w = (d_{hi-1} - d_lo) + gam_{hi-1}, with P
// Chebyshev points (w/2)(1 + cos((2k+1) pi / (2P))).  A pole maps to
// d_i - d_lo, a root to (d_j - d_lo) + gam_j.  Two nodes are well separated
// when their gap, (d_{lo_S} - d_{hi_T}) + mu_{hi_T - 1} for S right of T
// (eq. d-lambda), is at least the larger width; a dual traversal of the tree
// gives every node its far list (well-separated nodes of its level) and every
// leaf its near list (the other leaves not covered by a far pair).
//
// Side 0 computes Phi (targets d, sources lam, weights v Omega), side 1
// Theta (targets lam, sources d, weights uh Omega, kernel of opposite sign).
// Near-field entries use the rule of eq. (d-lambda) entry by entry, so a
// leaf's near list may also hold the leaf itself (its diagonal block).  Every
// kernel works on 32-column chunks; the operands of a merge are io[merge]
// (Omega in, out[side], row-major with leading dimension sp), and the W
// (multipole) and F (local) coefficients live at io[merge].off as
// [(node * 2 + side) * P + k] * sp + column.
#include <algorithm>
#include <cmath>
#include <vector>

#include "hss.hpp"

namespace {

// 1/x: hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r), each of which squares the relative error.
__device__ __forceinline__ double rcp_refined(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

constexpr int PMAX = 32;   // Chebyshev points per node at most
constexpr int CW = 32;     // sample columns per job
constexpr int PCH = 64;    // source points staged at a time (P2M)
constexpr int NCH = 128;   // source points staged at a time (near field)

__device__ inline void cheb_init(int P, double* t, double* beta) {
  for (int k = threadIdx.x; k < P; k += blockDim.x) {
    const double th = (2 * k + 1) * M_PI / (2.0 * P);
    t[k] = cos(th);
    beta[k] = (k & 1) ? -sin(th) : sin(th);
  }
}

// half of the node's width = the centre of its interval [0, w]
__device__ inline double half_width(const HssMerge& M, const HssNode& nd) {
  return 0.5 * ((M.d[nd.hi - 1] - M.d[nd.lo]) + M.gam[nd.hi - 1]);
}

// Lagrange basis of the P Chebyshev points h(1 + t_k) at x (barycentric
// formula of the second kind), written to out[k * ld]
__device__ inline void lagrange_col(double x, double h, int P, const double* t, const double* beta, double* out,
                                    int ld) {
  double sum = 0.0;
  int hit = -1;
  for (int k = 0; k < P; ++k) {
    const double df = x - h * (1.0 + t[k]);
    if (df == 0.0) hit = k;
    const double q = beta[k] / df;
    out[k * ld] = q;
    sum += q;
  }
  if (hit >= 0) {
    for (int k = 0; k < P; ++k) out[k * ld] = (k == hit) ? 1.0 : 0.0;
  } else {
    const double r = 1.0 / sum;
    for (int k = 0; k < P; ++k) out[k * ld] *= r;
  }
}

__device__ inline int64_t coef_base(const FmmIo& io, const FmmJob& jb, int node, int P) {
  return io.off + ((int64_t)node * 2 + jb.side) * P * io.sp;
}

}  // namespace

// P2M at the leaves: W_S = sum_{j in S} ell^S(y_j) q_j for one 32-column chunk.
// 256 threads; thread (k0, c) = (tid / 32, tid % 32) owns rows k0 + 8 r.
__global__ __launch_bounds__(256) void k_fmm_p2m(const HssMerge* __restrict__ ms, const FmmJob* __restrict__ jobs,
                                                 const FmmIo* __restrict__ io, int P, double* __restrict__ W) {
  __shared__ double t[PMAX], beta[PMAX];
  __shared__ double ell[PMAX * PCH];
  __shared__ double q[PCH * CW];
  const FmmJob jb = jobs[blockIdx.x];
  const HssMerge& M = ms[jb.merge];
  const HssNode nd = M.nodes[jb.node];
  const FmmIo IO = io[jb.merge];
  cheb_init(P, t, beta);
  const double h = half_width(M, nd);
  const double a = M.d[nd.lo];
  const int tid = threadIdx.x, c = tid % CW, k0 = tid / CW;
  const double* wgt = jb.side == 0 ? M.v : M.uh;
  double acc[PMAX / 8];
#pragma unroll
  for (int r = 0; r < PMAX / 8; ++r) acc[r] = 0.0;
  __syncthreads();
  for (int j0 = nd.lo; j0 < nd.hi; j0 += PCH) {
    const int nj = min(PCH, nd.hi - j0);
    for (int j = tid; j < nj; j += blockDim.x) {
      const int gj = j0 + j;
      const double y = jb.side == 0 ? (M.d[gj] - a) + M.gam[gj] : M.d[gj] - a;
      lagrange_col(y, h, P, t, beta, ell + j, PCH);
    }
    for (int e = tid; e < nj * CW; e += blockDim.x) {
      const int j = e / CW, cc = e % CW;
      q[e] = wgt[j0 + j] * IO.omega[(int64_t)(j0 + j) * IO.sp + jb.c0 + cc];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PMAX / 8; ++r) {
      const int k = k0 + 8 * r;
      if (k < P) {
        double s = acc[r];
        for (int j = 0; j < nj; ++j) s = fma(ell[k * PCH + j], q[j * CW + c], s);
        acc[r] = s;
      }
    }
    __syncthreads();
  }
  double* Wn = W + coef_base(IO, jb, jb.node, P);
#pragma unroll
  for (int r = 0; r < PMAX / 8; ++r) {
    const int k = k0 + 8 * r;
    if (k < P) Wn[(int64_t)k * IO.sp + jb.c0 + c] = acc[r];
  }
}

// M2M: W_P = sum over the two children C of E_PC W_C,
// E_PC[k][l] = ell_k^P(tau_l^C + d_lo(C) - d_lo(P)).
__global__ __launch_bounds__(256) void k_fmm_m2m(const HssMerge* __restrict__ ms, const FmmJob* __restrict__ jobs,
                                                 const FmmIo* __restrict__ io, int P, double* __restrict__ W) {
  __shared__ double t[PMAX], beta[PMAX];
  __shared__ double E[2 * PMAX * PMAX];
  const FmmJob jb = jobs[blockIdx.x];
  const HssMerge& M = ms[jb.merge];
  const FmmIo IO = io[jb.merge];
  const int sp = IO.sp;
  const HssNode nd = M.nodes[jb.node];
  cheb_init(P, t, beta);
  __syncthreads();
  const double h = half_width(M, nd);
  const double a = M.d[nd.lo];
  const int tid = threadIdx.x;
  if (tid < 2 * P) {
    const int ci = tid / P, l = tid % P;
    const HssNode ch = M.nodes[2 * jb.node + 1 + ci];
    const double hc = half_width(M, ch);
    lagrange_col(hc * (1.0 + t[l]) + (M.d[ch.lo] - a), h, P, t, beta, E + ci * PMAX * PMAX + l, PMAX);
  }
  __syncthreads();
  const int c = tid % CW, k0 = tid / CW;
  const double* W1 = W + coef_base(IO, jb, 2 * jb.node + 1, P) + jb.c0 + c;
  const double* W2 = W + coef_base(IO, jb, 2 * jb.node + 2, P) + jb.c0 + c;
  double* Wn = W + coef_base(IO, jb, jb.node, P) + jb.c0 + c;
#pragma unroll
  for (int r = 0; r < PMAX / 8; ++r) {
    const int k = k0 + 8 * r;
    if (k < P) {
      double s = 0.0;
      for (int l = 0; l < P; ++l) {
        s = fma(E[k * PMAX + l], W1[(int64_t)l * sp], s);
        s = fma(E[PMAX * PMAX + k * PMAX + l], W2[(int64_t)l * sp], s);
      }
      Wn[(int64_t)k * sp] = s;
    }
  }
}

// M2L: F_T = sum over the far list of G_TS W_S,
// G_TS[l][k] = sigma / ((d_lo(T) - d_lo(S)) + (tau_l^T - tau_k^S)); sigma = +1
// for side 0, -1 for side 1.  Writes F_T (zero for an empty list).
__global__ __launch_bounds__(256) void k_fmm_m2l(const HssMerge* __restrict__ ms, const FmmJob* __restrict__ jobs,
                                                 const int32_t* __restrict__ lists, const FmmIo* __restrict__ io,
                                                 int P, const double* __restrict__ W, double* __restrict__ F) {
  __shared__ double t[PMAX], beta[PMAX];
  __shared__ double G[PMAX * PMAX];
  const FmmJob jb = jobs[blockIdx.x];
  const HssMerge& M = ms[jb.merge];
  const FmmIo IO = io[jb.merge];
  const int sp = IO.sp;
  const HssNode nd = M.nodes[jb.node];
  cheb_init(P, t, beta);
  const double hT = half_width(M, nd);
  const double aT = M.d[nd.lo];
  const double sigma = jb.side == 0 ? 1.0 : -1.0;
  const int tid = threadIdx.x, c = tid % CW, k0 = tid / CW;
  double acc[PMAX / 8];
#pragma unroll
  for (int r = 0; r < PMAX / 8; ++r) acc[r] = 0.0;
  __syncthreads();
  for (int e = 0; e < jb.lcnt; ++e) {
    const int sn = lists[jb.loff + e];
    const HssNode S = M.nodes[sn];
    const double hS = half_width(M, S);
    const double shift = aT - M.d[S.lo];
    for (int x = tid; x < P * P; x += blockDim.x) {
      const int l = x / P, k = x % P;
      G[l * PMAX + k] = sigma / (shift + (hT * (1.0 + t[l]) - hS * (1.0 + t[k])));
    }
    __syncthreads();
    const double* Ws = W + coef_base(IO, jb, sn, P) + jb.c0 + c;
#pragma unroll
    for (int r = 0; r < PMAX / 8; ++r) {
      const int l = k0 + 8 * r;
      if (l < P) {
        double s = acc[r];
        for (int k = 0; k < P; ++k) s = fma(G[l * PMAX + k], Ws[(int64_t)k * sp], s);
        acc[r] = s;
      }
    }
    __syncthreads();
  }
  double* Fn = F + coef_base(IO, jb, jb.node, P) + jb.c0 + c;
#pragma unroll
  for (int r = 0; r < PMAX / 8; ++r) {
    const int l = k0 + 8 * r;
    if (l < P) Fn[(int64_t)l * sp] = acc[r];
  }
}

// L2L: F_C += E_PC^T F_P for the child C of the job (its parent's F is final).
__global__ __launch_bounds__(256) void k_fmm_l2l(const HssMerge* __restrict__ ms, const FmmJob* __restrict__ jobs,
                                                 const FmmIo* __restrict__ io, int P, double* __restrict__ F) {
  __shared__ double t[PMAX], beta[PMAX];
  __shared__ double E[PMAX * PMAX];
  const FmmJob jb = jobs[blockIdx.x];
  const HssMerge& M = ms[jb.merge];
  const FmmIo IO = io[jb.merge];
  const int sp = IO.sp;
  const int pn = (jb.node - 1) / 2;
  const HssNode ch = M.nodes[jb.node];
  const HssNode par = M.nodes[pn];
  cheb_init(P, t, beta);
  __syncthreads();
  const double hp = half_width(M, par);
  const int tid = threadIdx.x;
  if (tid < P) {
    const double hc = half_width(M, ch);
    lagrange_col(hc * (1.0 + t[tid]) + (M.d[ch.lo] - M.d[par.lo]), hp, P, t, beta, E + tid, PMAX);
  }
  __syncthreads();
  const int c = tid % CW, k0 = tid / CW;
  const double* Fp = F + coef_base(IO, jb, pn, P) + jb.c0 + c;
  double* Fc = F + coef_base(IO, jb, jb.node, P) + jb.c0 + c;
#pragma unroll
  for (int r = 0; r < PMAX / 8; ++r) {
    const int l = k0 + 8 * r;
    if (l < P) {
      double s = Fc[(int64_t)l * sp];
      for (int k = 0; k < P; ++k) s = fma(E[k * PMAX + l], Fp[(int64_t)k * sp], s);
      Fc[(int64_t)l * sp] = s;
    }
  }
}

// Leaf evaluation: L2P of F_T plus the near field, entry by entry with the
// differences of eq. (d-lambda), scaled by uh_i (side 0) or v_j (side 1);
// writes the leaf's rows of Phi or Theta for one 32-column chunk.  128
// threads, one target row each (leaves longer than 128 rows take passes).
__global__ __launch_bounds__(128) void k_fmm_leaf(const HssMerge* __restrict__ ms, const FmmJob* __restrict__ jobs,
                                                  const int32_t* __restrict__ lists, const FmmIo* __restrict__ io,
                                                  int P, const double* __restrict__ F) {
  __shared__ double t[PMAX], beta[PMAX];
  __shared__ double Fl[PMAX * CW];
  __shared__ double qs[NCH * CW];
  __shared__ double s0[NCH], s1[NCH], s2[NCH], s3[NCH];
  const FmmJob jb = jobs[blockIdx.x];
  const HssMerge& M = ms[jb.merge];
  const HssNode T = M.nodes[jb.node];
  const FmmIo IO = io[jb.merge];
  const int K = M.K, sp = IO.sp;
  cheb_init(P, t, beta);
  const double* Fn = F + coef_base(IO, jb, jb.node, P) + jb.c0;
  for (int e = threadIdx.x; e < P * CW; e += blockDim.x) Fl[e] = Fn[(int64_t)(e / CW) * sp + e % CW];
  const double hT = half_width(M, T);
  const double aT = M.d[T.lo];
  const double* wgt = jb.side == 0 ? M.v : M.uh;
  double* out = IO.out[jb.side];
  __syncthreads();
  for (int row0 = T.lo; row0 < T.hi; row0 += blockDim.x) {
    const int i = row0 + threadIdx.x;
    const bool active = i < T.hi;
    double acc[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) acc[c] = 0.0;
    // target data: side 0 a pole d_i; side 1 a root lam_i with d_i, gam_i,
    // d_{i+1}, mu_i for the differences
    double td = 0.0, tg = 0.0, tdn = 0.0, tm = 0.0, x = 0.0;
    if (active) {
      td = M.d[i];
      tg = M.gam[i];
      tdn = M.d[min(i + 1, K - 1)];
      tm = M.mu[i];
      x = jb.side == 0 ? td - aT : (td - aT) + tg;
      // L2P
      double sum = 0.0;
      int hit = -1;
      for (int k = 0; k < P; ++k) {
        const double df = x - hT * (1.0 + t[k]);
        if (df == 0.0) hit = k;
        sum += beta[k] / df;
      }
      const double rs = 1.0 / sum;
      for (int k = 0; k < P; ++k) {
        const double wk = hit >= 0 ? (k == hit ? 1.0 : 0.0) : (beta[k] / (x - hT * (1.0 + t[k]))) * rs;
#pragma unroll
        for (int c = 0; c < CW; ++c) acc[c] = fma(wk, Fl[k * CW + c], acc[c]);
      }
    }
    for (int e = 0; e < jb.lcnt; ++e) {
      const HssNode S = M.nodes[lists[jb.loff + e]];
      for (int j0 = S.lo; j0 < S.hi; j0 += NCH) {
        const int nj = min(NCH, S.hi - j0);
        __syncthreads();
        for (int j = threadIdx.x; j < nj; j += blockDim.x) {
          const int gj = j0 + j;
          s0[j] = M.d[gj];
          s1[j] = M.gam[gj];
          s2[j] = M.d[min(gj + 1, K - 1)];
          s3[j] = M.mu[gj];
        }
        for (int x2 = threadIdx.x; x2 < nj * CW; x2 += blockDim.x) {
          const int j = x2 / CW, cc = x2 % CW;
          qs[x2] = wgt[j0 + j] * IO.omega[(int64_t)(j0 + j) * sp + jb.c0 + cc];
        }
        __syncthreads();
        if (active) {
          // both forms of each difference are formed and one is selected (no
          // branch per source); two sources per step, so that two reciprocal
          // chains are in flight
          auto diff = [&](int j) {
            const int gj = j0 + j;
            if (jb.side == 0) {  // target pole i, source root gj: d_i - lam_gj
              const double a = (td - s0[j]) - s1[j];
              const double b = (td - s2[j]) + s3[j];
              return (i <= gj) ? a : b;
            }
            // target root i, source pole gj: d_gj - lam_i
            const double a = (s0[j] - td) - tg;
            const double b = (s0[j] - tdn) + tm;
            return (gj <= i) ? a : b;
          };
          int j = 0;
          for (; j + 1 < nj; j += 2) {
            const double inv0 = rcp_refined(diff(j));
            const double inv1 = rcp_refined(diff(j + 1));
#pragma unroll
            for (int c = 0; c < CW; ++c) acc[c] = fma(inv1, qs[(j + 1) * CW + c], fma(inv0, qs[j * CW + c], acc[c]));
          }
          if (j < nj) {
            const double inv = rcp_refined(diff(j));
#pragma unroll
            for (int c = 0; c < CW; ++c) acc[c] = fma(inv, qs[j * CW + c], acc[c]);
          }
        }
      }
    }
    if (active) {
      const double sc = jb.side == 0 ? M.uh[i] : M.v[i];
      double* o = out + (int64_t)i * sp + jb.c0;
#pragma unroll
      for (int c = 0; c < CW; ++c) o[c] = sc * acc[c];
    }
    __syncthreads();
  }
}

// Far and near lists by the dual traversal from (root, root); far[T] holds
// the nodes S of T's level well separated from T and not covered by an
// ancestor pair, near[T] (leaves only) the other leaves not covered at all.
void fmm_lists(const double* d, const double* gam, const double* mu, const std::vector<HssNode>& nodes,
               std::vector<std::vector<int32_t>>& far, std::vector<std::vector<int32_t>>& near) {
  const int nn = (int)nodes.size();
  far.assign(nn, {});
  near.assign(nn, {});
  auto width = [&](const HssNode& n) { return (d[n.hi - 1] - d[n.lo]) + gam[n.hi - 1]; };
  std::vector<std::pair<int, int>> stack{{0, 0}};
  while (!stack.empty()) {
    const auto [ti, si] = stack.back();
    stack.pop_back();
    const HssNode& T = nodes[ti];
    const HssNode& S = nodes[si];
    if (ti != si) {
      const double gap = (S.lo >= T.hi) ? (d[S.lo] - d[T.hi]) + mu[T.hi - 1] : (d[T.lo] - d[S.hi]) + mu[S.hi - 1];
      if (gap >= std::max(width(T), width(S))) {
        far[ti].push_back(si);
        continue;
      }
    }
    if (T.leaf && S.leaf) {
      if (ti != si) near[ti].push_back(si);
      continue;
    }
    for (int a = 1; a <= 2; ++a)
      for (int b = 1; b <= 2; ++b) stack.push_back({2 * ti + a, 2 * si + b});
  }
}
