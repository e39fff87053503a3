// Device kernels of the randomized HSS construction (Algorithm 2), of the
// Gaussian sampling matrices and of the accuracy check.
//
// k_philox_normal  Omega, standard normal by Philox4x32-10 (Salmon et al.
//                  2011) and the Box-Muller transform; element (i, c) is normal
//                  number i*s + c of the stream.
// k_hss_sample     Y = A Omega and Z = A^T Omega restricted to the HSS block
//                  rows / columns of the leaves, i.e. Phi_i = Y_i - D_i Omega_i
//                  and Theta_i = Z_i - D_i^T Omega_i of Algorithm 2 computed
//                  without forming D_i Omega_i: the entries of the leaf's own
//                  diagonal block are skipped.  A = Q' is never stored: every
//                  16 x 4 operand fragment of v_mfma_f64_16x16x4f64 is generated
//                  in registers from the generators (eq. Ev-Q, differences by
//                  eq. d-lambda), Omega tiles are staged in LDS.
// k_hss_bblocks    the B blocks of a parent's children from the generators
//                  (one workgroup per parent, before the parent's level).
// k_hss_compress   one workgroup per tree node, level and side (row ID and
//                  column ID run side by side): the compressed block row
//                  Phi_i or column Theta_i (leaves from the samples, parents
//                  from the children as in Algorithm 2), its interpolative
//                  decomposition by column-pivoted Householder QR truncated
//                  at |R_kk| <= tol |R_11|, the generator U_i or V_i, and
//                  Zhat_i or Yhat_i.
// k_hss_dmat       the leaf diagonal blocks D_i = A(t_i, t_i) for Algorithm 3.
#include "hss.hpp"

namespace {

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Q'(i, j) = uh_i v_j / (d_i - lam_j)
__device__ __forceinline__ double cauchy_entry(int i, int j, double di, double ui, double dj, double dj1, double gj,
                                               double mj, double vj) {
  return ui * vj / d_minus_lam(i, j, di, dj, dj1, gj, mj);
}

__device__ __forceinline__ double gen_entry(const HssMerge& M, int i, int j) {
  const double dj1 = (j + 1 < M.K) ? M.d[j + 1] : 0.0;
  return cauchy_entry(i, j, M.d[i], M.uh[i], M.d[j], dj1, M.gam[j], M.mu[j], M.v[j]);
}

}  // namespace

__global__ void k_philox_normal(double* __restrict__ out, int64_t K, int s, int sp, uint64_t seed,
                                uint32_t stream) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= K * sp) return;
  const int64_t i = idx / sp;
  const int c = (int)(idx % sp);
  if (c >= s) {
    out[idx] = 0.0;
    return;
  }
  const uint64_t e = (uint64_t)i * (uint64_t)s + (uint64_t)c;
  const uint64_t ctr = e >> 1;
  uint32_t x[4] = {(uint32_t)ctr, (uint32_t)(ctr >> 32), stream, 0u};
  philox10(x, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double u1 = ((double)(x[0] >> 5) * 67108864.0 + (double)(x[1] >> 6)) * 0x1.0p-53;
  const double u2 = ((double)(x[2] >> 5) * 67108864.0 + (double)(x[3] >> 6)) * 0x1.0p-53;
  const double r = sqrt(-2.0 * log(1.0 - u1));
  const double th = 6.283185307179586 * u2;
  out[idx] = (e & 1ull) ? r * sin(th) : r * cos(th);
}

// ---------------------------------------------------------------------------
// sampling: rows r0..r0+63 (16 per wave) x columns c0..c0+127 of the output
// (those below sp).  Each lane generates one 16 x 4 fragment entry of Q' per
// step and feeds it to every 16-column tile of the job, so that an entry is
// generated once for all samples; Omega is staged through LDS 32 rows at a
// time (row stride = 16 (mod 32) doubles: the four k-rows of a fragment read
// fall on the two bank halves).
namespace {
__device__ __forceinline__ double rcp2(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
}  // namespace

__global__ void __launch_bounds__(256) k_hss_sample(const HssMerge* __restrict__ ms,
                                                    const SampleJob* __restrict__ jobs, int exclude_diag,
                                                    double* __restrict__ part) {
  constexpr int JT = 32;   // rows of Omega per staging round
  constexpr int NT = 8;    // 16-column tiles per job
  constexpr int LDO = 16 * NT + 16;
  __shared__ double s_om[JT][LDO];
  __shared__ double s_g0[JT + 1], s_g1[JT], s_g2[JT], s_g3[JT];
  const SampleJob jb = jobs[blockIdx.x];
  const HssMerge& M = ms[jb.merge];
  const int K = M.K;
  const int sp = M.sp;
  const int trans = jb.trans;
  const double* __restrict__ om = M.omega;
  double* __restrict__ out = (jb.nseg > 1) ? part + jb.pbase : (trans ? M.theta : M.phi);
  // inner-dimension segment, whole staging rounds
  const int len = ((K + jb.nseg - 1) / jb.nseg + JT - 1) / JT * JT;
  const int qa = jb.seg * len, qb = min(K, qa + len);
  const int tid = threadIdx.x, lane = tid & 63, wv = wave_index();
  const int li = lane & 15, lk = lane >> 4;
  const int ncols = min(16 * NT, sp - jb.c0);
  const int ntl = (ncols + 15) / 16;
  const int rr = jb.r0 + wv * 16 + li;  // this lane's output row
  const bool rvalid = rr < K;
  int lo_r = 0, hi_r = 0;
  double rd = 0.0, rd1 = 0.0, rg = 0.0, rm = 0.0, ru = 0.0, rv = 0.0;
  if (rvalid) {
    if (exclude_diag) {
      const int lf = M.leafof[rr];
      lo_r = M.bounds[lf];
      hi_r = M.bounds[lf + 1];
    }
    rd = M.d[rr];
    if (trans) {  // the row of the output is a column j of Q'
      rd1 = (rr + 1 < K) ? M.d[rr + 1] : 0.0;
      rg = M.gam[rr];
      rm = M.mu[rr];
      rv = M.v[rr];
    } else {
      ru = M.uh[rr];
    }
  }
  dbl4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int q0 = qa; q0 < qb; q0 += JT) {
    __syncthreads();
    for (int e = tid; e < JT * 16 * NT; e += 256) {
      const int qr = e / (16 * NT), cc = e % (16 * NT);
      const int q = q0 + qr;
      s_om[qr][cc] = (q < qb && cc < ncols) ? om[(int64_t)q * sp + jb.c0 + cc] : 0.0;
    }
    if (tid < JT) {
      const int q = q0 + tid;
      if (q < K) {
        s_g0[tid] = M.d[q];
        if (trans) {
          s_g1[tid] = M.uh[q];
        } else {
          s_g1[tid] = M.gam[q];
          s_g2[tid] = M.mu[q];
          s_g3[tid] = M.v[q];
        }
      } else {
        s_g0[tid] = 0.0;
        s_g1[tid] = s_g2[tid] = s_g3[tid] = 0.0;
      }
    }
    if (tid == 0) s_g0[JT] = (q0 + JT < K) ? M.d[q0 + JT] : 0.0;
    __syncthreads();
#pragma unroll 2
    for (int kk = 0; kk < JT / 4; ++kk) {
      const int ql = kk * 4 + lk;
      const int q = q0 + ql;
      double a = 0.0;
      if (rvalid && q < qb && !(q >= lo_r && q < hi_r)) {
        if (trans) {
          // Q'(q, rr): i = q (inner), j = rr
          a = s_g1[ql] * rv * rcp2(d_minus_lam(q, rr, s_g0[ql], rd, rd1, rg, rm));
        } else {
          // Q'(rr, q): i = rr, j = q
          const double dq1 = (q + 1 < K) ? s_g0[ql + 1] : 0.0;
          a = ru * s_g3[ql] * rcp2(d_minus_lam(rr, q, rd, s_g0[ql], dq1, s_g1[ql], s_g2[ql]));
        }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t)
        if (t < ntl) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, s_om[ql][16 * t + li], acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t >= ntl) continue;
    const int col = jb.c0 + 16 * t + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = jb.r0 + wv * 16 + lk + 4 * r;
      if (row < K && col < sp) out[(int64_t)row * sp + col] = acc[t][r];
    }
  }
}

// out[e] = sum over the nseg partial blocks of n elements each
__global__ void k_sample_sum(const double* __restrict__ part, int nseg, int64_t n, double* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  double x = 0.0;
  for (int sg = 0; sg < nseg; ++sg) x += part[(int64_t)sg * n + e];
  out[e] = x;
}

// ---------------------------------------------------------------------------
// Column interpolative decomposition of A (m x n, column-major, ld lda) by
// column-pivoted Householder QR (pivot: largest remaining norm, recomputed
// every step; ties to the smaller index), stopped when that norm is <= tol
// times the first one.  Columns are not moved: perm lists the chosen columns
// first, and on return column perm[c] of A holds, in rows 0:k, R11^-1 R12's
// column c for c >= k.  All threads of the block take part.
namespace {
constexpr int CMAX = 512;  // candidates

// (value, index) maximum with ties to the smaller index
__device__ __forceinline__ void argmax_merge(double& v, int& i, double ov, int oi) {
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}

// Lane exchanges inside a wave by DPP (no LDS round trip): CTRL 0xB1 swaps
// neighbours (quad_perm 1,0,3,2), 0x4E swaps pairs (quad_perm 2,3,0,1),
// 0x141 mirrors each half row of 8 lanes, 0x140 each row of 16.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
// sum over an aligned group of 8 lanes, the same value in every lane of it
__device__ __forceinline__ double sum8(double x) {
  x += dpp_d<0xB1>(x);
  x += dpp_d<0x4E>(x);
  x += dpp_d<0x141>(x);
  return x;
}
template <int CTRL>
__device__ __forceinline__ void argmax_step(double& v, int& i) {
  const double ov = dpp_d<CTRL>(v);
  const int oi = dpp_i<CTRL>(i);
  argmax_merge(v, i, ov, oi);
}

// The work on columns is spread over groups of 8 lanes (rows split between
// the lanes, sums by DPP inside the group); wave 0 takes the pivot and builds
// the reflector.  IN_GLOBAL: A lives in global memory, where stores of one
// lane are fenced before other lanes of the group read them.  (One
// instantiation per address space, inlined into the kernel, so that the LDS
// one is compiled to LDS instructions rather than generic ones.)
template <bool IN_GLOBAL>
__device__ __forceinline__ int cpqr_id(double* A, int lda, int m, int n, double tol, int* perm, double* nrm,
                                       double* redv, int* redi) {
  constexpr bool in_global = IN_GLOBAL;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = wave_index();
  const int grp = tid >> 3, q = tid & 7, ngrp = (int)(blockDim.x >> 3);
  __shared__ int s_stop, s_pc;
  __shared__ double s_f2, s_vk;
  for (int c = tid; c < n; c += blockDim.x) perm[c] = c;
  // squared column norms
  for (int c0 = 0; c0 < n; c0 += ngrp) {
    const int c = c0 + grp;
    double s2 = 0.0;
    if (c < n) {
      const double* col = A + (int64_t)c * lda;
      for (int r = q; r < m; r += 8) s2 = fma(col[r], col[r], s2);
    }
    s2 = sum8(s2);
    if (c < n && q == 0) nrm[c] = s2;
  }
  __syncthreads();
  const int kmax = min(m, n);
  int k = 0;
  double r11 = 0.0;  // |R_11|, kept by wave 0
  for (; k < kmax; ++k) {
    if (wv == 0) {
      // pivot: largest remaining norm, ties to the smaller index; rows of 16
      // lanes by DPP, the four rows through LDS
      double best = -1.0;
      int bi = n;
      for (int c = k + lane; c < n; c += 64) argmax_merge(best, bi, nrm[c], c);
      argmax_step<0xB1>(best, bi);
      argmax_step<0x4E>(best, bi);
      argmax_step<0x141>(best, bi);
      argmax_step<0x140>(best, bi);
      if ((lane & 15) == 0) {
        redv[lane >> 4] = best;
        redi[lane >> 4] = bi;
      }
      __builtin_amdgcn_wave_barrier();
      best = redv[0];
      bi = redi[0];
      for (int w = 1; w < 4; ++w) argmax_merge(best, bi, redv[w], redi[w]);
      const double pn = sqrt(fmax(best, 0.0));
      if (k == 0) r11 = pn;
      const int stop = (bi >= n) || (pn == 0.0) || (pn <= tol * r11);
      if (!stop) {
        // Columns stay in place: perm maps the pivot order to them, so the
        // swap is one of indices.  The Householder vector v = x - alpha e_1
        // (alpha = -sign(x_0)||x||, v^T v = 2 ||x|| (||x|| + |x_0|)) is read
        // from the pivot column below row k and from s_vk at row k, where
        // the column takes R(k, k) = alpha; its rows below k are not part
        // of R and are left as they are.
        const int pb = perm[bi];
        double* pc = A + (int64_t)pb * lda;
        const double x0 = pc[k];
        const double alpha = (x0 != 0.0) ? -copysign(pn, x0) : -pn;
        if (lane == 0) {
          if (bi != k) {
            perm[bi] = perm[k];
            perm[k] = pb;
            nrm[bi] = nrm[k];
          }
          pc[k] = alpha;
          const double vn2 = 2.0 * pn * (pn + fabs(x0));
          s_f2 = (vn2 > 0.0) ? 2.0 / vn2 : 0.0;  // the reflection factor 2 / v^T v
          s_vk = x0 - alpha;
          s_pc = pb;
        }
      }
      if (lane == 0) s_stop = stop;
    }
    __syncthreads();
    if (s_stop) break;
    const double f2 = s_f2, vk = s_vk;
    const double* __restrict__ v = A + (int64_t)s_pc * lda;  // rows > k of the reflector
    // a group per remaining column: reflect it and take its norm below row k
    for (int c0 = k + 1; c0 < n; c0 += ngrp) {
      const int c = c0 + grp;
      const bool act = c < n;
      double d0 = 0.0, d1 = 0.0;
      double* __restrict__ col = A;
      if (act) {
        col = A + (int64_t)perm[c] * lda;
        int r = k + q;
        if (q == 0) {
          d0 = vk * col[k];
          r += 8;
        }
        for (; r + 8 < m; r += 16) {
          d0 = fma(v[r], col[r], d0);
          d1 = fma(v[r + 8], col[r + 8], d1);
        }
        if (r < m) d0 = fma(v[r], col[r], d0);
      }
      const double dt = sum8(d0 + d1);
      const double f = dt * f2;
      double s2 = 0.0;
      if (act) {
        int r = k + q;
        if (q == 0) {
          col[k] -= f * vk;
          r += 8;
        }
        for (; r < m; r += 8) {
          const double x = col[r] - f * v[r];
          col[r] = x;
          s2 = fma(x, x, s2);
        }
      }
      s2 = sum8(s2);
      if (act && q == 0) nrm[c] = s2;
    }
    __syncthreads();
  }
  // T = R11^-1 R12 in place: back substitution, a group per column (rows of
  // the update split between its lanes); column c of the pivot order is
  // stored in column perm[c].  The reciprocals of R11's diagonal go first
  // into nrm (no longer needed).
  for (int j = tid; j < k; j += blockDim.x) nrm[j] = 1.0 / A[j + (int64_t)perm[j] * lda];
  __syncthreads();
  for (int c0 = k; c0 < n; c0 += ngrp) {
    const int c = c0 + grp;
    if (c < n) {
      double* col = A + (int64_t)perm[c] * lda;
      for (int j = k - 1; j >= 0; --j) {
        const double* aj = A + (int64_t)perm[j] * lda;
        const double xj = col[j] * nrm[j];
        for (int r = q; r < j; r += 8) col[r] = fma(-xj, aj[r], col[r]);
        if (q == 0) col[j] = xj;
        if (in_global) __threadfence_block();
      }
    }
  }
  __syncthreads();
  return k;
}

// C[r ldc + col] = (Cinit ? Cinit[r ldi + col] : 0) + sgn sum_q A(r, q) Y[q ldy + col]
// for r < R, col < ncol, with A(r, q) = A[r ars + q acs]; both operands are
// staged through `lds` (cap doubles) in chunks of q, A transposed with its
// rows padded to groups of four.  A thread owns four rows of one column and
// keeps them in registers, so that each staged Y entry feeds four FMAs (one
// LDS read of Y and one of four consecutive A entries per four FMAs).
// Every output element is owned by one thread, so Cinit may alias C.
__device__ __forceinline__ void block_small_gemm(double* C, int ldc, const double* Cinit, int ldi, double sgn,
                                                 const double* A, int ars, int acs, const double* Y, int ldy, int R,
                                                 int Q, int ncol, double* lds, int cap) {
  const int tid = threadIdx.x;
  if (R <= 0 || ncol <= 0) return;
  const int Rp = (R + 3) & ~3;
  int qc = (cap > 0) ? cap / (Rp + ncol) : 0;
  if (qc <= 0) {
    for (int e = tid; e < R * ncol; e += blockDim.x) {
      const int r = e / ncol, col = e % ncol;
      double x = 0.0;
      for (int q = 0; q < Q; ++q) x += A[(int64_t)r * ars + (int64_t)q * acs] * Y[(int64_t)q * ldy + col];
      C[(int64_t)r * ldc + col] = (Cinit ? Cinit[(int64_t)r * ldi + col] : 0.0) + sgn * x;
    }
    __syncthreads();
    return;
  }
  qc = min(qc, max(Q, 1));
  double* As = lds;                     // qc x Rp: As[qq Rp + r] = A(r, q0 + qq), padding rows zero
  double* Ys = lds + (int64_t)qc * Rp;  // qc x ncol
  const int ngrp = Rp / 4;
  const int items = ngrp * ncol;        // (row group, column) pairs
  for (int q0 = 0; q0 == 0 || q0 < Q; q0 += qc) {
    const int qn = max(0, min(qc, Q - q0));
    __syncthreads();
    // staging, consecutive threads on A's contiguous index
    if (acs == 1) {
      for (int e = tid; e < Rp * qn; e += blockDim.x) {
        const int r = e / qn, qq = e % qn;
        As[qq * Rp + r] = (r < R) ? A[(int64_t)r * ars + q0 + qq] : 0.0;
      }
    } else {
      for (int e = tid; e < Rp * qn; e += blockDim.x) {
        const int qq = e / Rp, r = e % Rp;
        As[qq * Rp + r] = (r < R) ? A[(int64_t)r * ars + (int64_t)(q0 + qq) * acs] : 0.0;
      }
    }
    for (int e = tid; e < qn * ncol; e += blockDim.x) {
      const int qq = e / ncol, col = e % ncol;
      Ys[qq * ncol + col] = Y[(int64_t)(q0 + qq) * ldy + col];
    }
    __syncthreads();
    for (int e = tid; e < items; e += blockDim.x) {
      const int g = e / ncol, col = e % ncol;
      const int r0 = 4 * g;
      const double* ap = As + r0;
      const double* yp = Ys + col;
      double x0 = 0.0, x1 = 0.0, x2 = 0.0, x3 = 0.0;
      for (int qq = 0; qq < qn; ++qq) {
        const double y = yp[qq * ncol];
        const double* a4 = ap + qq * Rp;
        x0 = fma(a4[0], y, x0);
        x1 = fma(a4[1], y, x1);
        x2 = fma(a4[2], y, x2);
        x3 = fma(a4[3], y, x3);
      }
      const double xs[4] = {x0, x1, x2, x3};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = r0 + u;
        if (r < R) {
          double* cp = C + (int64_t)r * ldc + col;
          const double base = (q0 == 0) ? (Cinit ? Cinit[(int64_t)r * ldi + col] : 0.0) : *cp;
          *cp = base + sgn * xs[u];
        }
      }
    }
    if (Q <= 0) break;
  }
  __syncthreads();
}

// Write U (n x k, column-major, ld n): rows perm[j] (j < k) are e_j, rows
// perm[c] (c >= k) are T(:, c)^T, which the back substitution left in
// column perm[c] of A.
__device__ __forceinline__ void write_interp(const double* A, int lda, int n, int k, const int* perm, int* inv,
                                             double* U) {
  const int tid = threadIdx.x;
  for (int c = tid; c < n; c += blockDim.x) inv[perm[c]] = c;
  __syncthreads();
  const int lane = tid & 63, wv = wave_index(), nw = blockDim.x >> 6;
  for (int j = wv; j < k; j += nw)
    for (int row = lane; row < n; row += 64) {
      const int pos = inv[row];
      double x;
      if (pos < k) x = (pos == j) ? 1.0 : 0.0;
      else x = A[j + (int64_t)row * lda];
      U[row + (int64_t)j * n] = x;
    }
  __syncthreads();
}
}  // namespace

__global__ void __launch_bounds__(1024) k_hss_compress(const HssMerge* __restrict__ ms,
                                                      const NodeJob* __restrict__ jobs, int lds_doubles) {
  extern __shared__ double dyn[];
  __shared__ double s_nrm[CMAX];
  __shared__ int s_perm[CMAX];
  __shared__ int s_inv[CMAX];
  __shared__ int s_cand[CMAX];
  __shared__ double s_redv[16];
  __shared__ int s_redi[16];

  const NodeJob jb = jobs[blockIdx.x];
  const HssMerge& M = ms[jb.merge];
  HssNode* nodes = M.nodes;
  HssNode& nd = nodes[jb.node];
  const int tid = threadIdx.x;
  const int s = M.s, sp = M.sp;
  double* ar = M.arena;
  int* ia = M.iarena;

  {
    const int side = jb.side;  // 0: rows (Phi, U), 1: columns (Theta, V)
    // candidates and the compressed block (cand x sp, row-major) in this
    // side's half of the work area
    const int cand_alloc = nd.leaf ? (nd.hi - nd.lo) : min(2 * s, nd.hi - nd.lo);
    double* W0 = ar + nd.offWork + (int64_t)side * 2 * cand_alloc * sp;
    int nc;
    if (nd.leaf) {
      nc = nd.hi - nd.lo;
      const double* src = side ? M.theta : M.phi;
      for (int e = tid; e < nc * sp; e += blockDim.x) W0[e] = src[(int64_t)nd.lo * sp + e];
      for (int c = tid; c < nc; c += blockDim.x) s_cand[c] = nd.lo + c;
    } else {
      const HssNode& a = nodes[2 * jb.node + 1];
      const HssNode& b = nodes[2 * jb.node + 2];
      const int ka = side ? a.kc : a.kr, kb = side ? b.kc : b.kr;
      nc = ka + kb;
      const int* la = ia + (side ? a.offSc : a.offSr);
      const int* lb = ia + (side ? b.offSc : b.offSr);
      for (int c = tid; c < nc; c += blockDim.x) s_cand[c] = (c < ka) ? la[c] : lb[c - ka];
      const double* Ba = ar + a.offB;  // a.kr x b.kc
      const double* Bb = ar + b.offB;  // b.kr x a.kc
      if (side == 0) {
        // [Phi_a|sk - B_a Yhat_b ; Phi_b|sk - B_b Yhat_a]
        block_small_gemm(W0, sp, ar + a.offPs, sp, -1.0, Ba, 1, ka, ar + b.offYh, sp, ka, b.kc, s, dyn,
                         lds_doubles);
        block_small_gemm(W0 + (int64_t)ka * sp, sp, ar + b.offPs, sp, -1.0, Bb, 1, kb, ar + a.offYh, sp, kb, a.kc,
                         s, dyn, lds_doubles);
      } else {
        // [Theta_a|sk - B_b^T Zhat_b ; Theta_b|sk - B_a^T Zhat_a]
        block_small_gemm(W0, sp, ar + a.offTs, sp, -1.0, Bb, b.kr, 1, ar + b.offZh, sp, ka, b.kr, s, dyn,
                         lds_doubles);
        block_small_gemm(W0 + (int64_t)ka * sp, sp, ar + b.offTs, sp, -1.0, Ba, a.kr, 1, ar + a.offZh, sp, kb,
                         a.kr, s, dyn, lds_doubles);
      }
    }
    __syncthreads();
    // working copy: columns = candidates, rows = samples (ld sp)
    // working copy with an odd leading dimension in LDS (no bank aliasing of
    // columns), or the second half of the work area
    // in LDS the column stride is = 8 (mod 32) doubles, so that the eight
    // 8-lane column groups of a wave fall on different banks
    const int lw_lds = s + (((8 - s) % 32) + 32) % 32;
    const bool in_lds = lds_doubles >= nc * lw_lds;
    double* U = ar + (side ? nd.offV : nd.offU);
    int k;
    // the two address spaces in separate branches, with the LDS one reading
    // the shared array itself
    if (in_lds) {
      const int lw = lw_lds;
      for (int c = wave_index(); c < nc; c += blockDim.x >> 6)
        for (int r = tid & 63; r < s; r += 64) dyn[r + c * lw] = W0[r + (int64_t)c * sp];
      __syncthreads();
      k = cpqr_id<false>(dyn, lw, s, nc, M.id_tol, s_perm, s_nrm, s_redv, s_redi);
      write_interp(dyn, lw, nc, k, s_perm, s_inv, U);
    } else {
      const int lw = sp;
      double* Aw = W0 + (int64_t)nc * sp;
      for (int c = wave_index(); c < nc; c += blockDim.x >> 6)
        for (int r = tid & 63; r < s; r += 64) Aw[r + (int64_t)c * lw] = W0[r + (int64_t)c * sp];
      __syncthreads();
      k = cpqr_id<true>(Aw, lw, s, nc, M.id_tol, s_perm, s_nrm, s_redv, s_redi);
      write_interp(Aw, lw, nc, k, s_perm, s_inv, U);
    }
    int* skel = ia + (side ? nd.offSc : nd.offSr);
    double* sk = ar + (side ? nd.offTs : nd.offPs);
    for (int j = tid; j < k; j += blockDim.x) skel[j] = s_cand[s_perm[j]];
    for (int j = wave_index(); j < k; j += blockDim.x >> 6)
      for (int col = tid & 63; col < sp; col += 64) sk[(int64_t)j * sp + col] = W0[(int64_t)s_perm[j] * sp + col];
    if (tid == 0) {
      if (side) {
        nd.kc = k;
        nd.nc = nc;
      } else {
        nd.kr = k;
        nd.nr = nc;
      }
    }
    __syncthreads();
  }

  // Yhat_i = V_i^T Om_c (the column side) and Zhat_i = U_i^T Om_r (the row
  // side) with Om = Omega(t_i) for a leaf, the children's stacked Yhat / Zhat
  // for a parent.  Each side reads only its own ID's results.
  // U^T(j, c) = U[c + j nr]: row stride nr, column stride 1
  if (jb.side == 1) {
    const int kc = nd.kc, ncc = nd.nc;
    const double* V = ar + nd.offV;  // ncc x kc
    double* Yh = ar + nd.offYh;
    if (nd.leaf) {
      const double* Om = M.omega + (int64_t)nd.lo * sp;
      block_small_gemm(Yh, sp, nullptr, 0, 1.0, V, ncc, 1, Om, sp, kc, ncc, s, dyn, lds_doubles);
    } else {
      const HssNode& a = nodes[2 * jb.node + 1];
      const HssNode& b = nodes[2 * jb.node + 2];
      block_small_gemm(Yh, sp, nullptr, 0, 1.0, V, ncc, 1, ar + a.offYh, sp, kc, a.kc, s, dyn, lds_doubles);
      block_small_gemm(Yh, sp, Yh, sp, 1.0, V + a.kc, ncc, 1, ar + b.offYh, sp, kc, b.kc, s, dyn, lds_doubles);
    }
  } else {
    const int kr = nd.kr, nr = nd.nr;
    const double* U = ar + nd.offU;  // nr x kr
    double* Zh = ar + nd.offZh;
    if (nd.leaf) {
      const double* Om = M.omega + (int64_t)nd.lo * sp;
      block_small_gemm(Zh, sp, nullptr, 0, 1.0, U, nr, 1, Om, sp, kr, nr, s, dyn, lds_doubles);
    } else {
      const HssNode& a = nodes[2 * jb.node + 1];
      const HssNode& b = nodes[2 * jb.node + 2];
      block_small_gemm(Zh, sp, nullptr, 0, 1.0, U, nr, 1, ar + a.offZh, sp, kr, a.kr, s, dyn, lds_doubles);
      block_small_gemm(Zh, sp, Zh, sp, 1.0, U + a.kr, nr, 1, ar + b.offZh, sp, kr, b.kr, s, dyn, lds_doubles);
    }
  }
}

// B blocks of a parent's children from the generators: B_{i1} =
// A(skel_r(i1), skel_c(i2)) and B_{i2} = A(skel_r(i2), skel_c(i1)) (one
// workgroup per parent, run before the parent's level is compressed).
__global__ void __launch_bounds__(256) k_hss_bblocks(const HssMerge* __restrict__ ms,
                                                     const NodeJob* __restrict__ jobs) {
  const NodeJob jb = jobs[blockIdx.x];
  const HssMerge& M = ms[jb.merge];
  const HssNode* nodes = M.nodes;
  const HssNode& a = nodes[2 * jb.node + 1];
  const HssNode& b = nodes[2 * jb.node + 2];
  const int* ia = M.iarena;
  double* ar = M.arena;
  const int* sra = ia + a.offSr;
  const int* sca = ia + a.offSc;
  const int* srb = ia + b.offSr;
  const int* scb = ia + b.offSc;
  double* Ba = ar + a.offB;
  double* Bb = ar + b.offB;
  for (int e = threadIdx.x; e < a.kr * b.kc; e += blockDim.x) {
    const int r = e % a.kr, q = e / a.kr;
    Ba[e] = gen_entry(M, sra[r], scb[q]);
  }
  for (int e = threadIdx.x; e < b.kr * a.kc; e += blockDim.x) {
    const int r = e % b.kr, q = e / b.kr;
    Bb[e] = gen_entry(M, srb[r], sca[q]);
  }
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_hss_dmat(const HssMerge* __restrict__ ms, const int2* __restrict__ leafjobs,
                                                  double* __restrict__ dmat, const int64_t* __restrict__ doff,
                                                  int grouped) {
  const int2 jb = leafjobs[blockIdx.x];
  const HssMerge& M = ms[jb.x];
  const HssNode& nd = M.nodes[jb.y];
  const int m = nd.hi - nd.lo;
  double* D = dmat + doff[blockIdx.x];
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int r = e % m, c = e / m;
    const int i = grouped ? M.perm[nd.lo + r] : nd.lo + r;
    D[e] = gen_entry(M, i, nd.lo + c);
  }
}

// U_i of every leaf with its rows in the packed (leaf-grouped) order of the
// solver's operand: out[a + k m] = U_i[perm(lo + a) - lo, k], m x kr.
__global__ void __launch_bounds__(256) k_hss_urows(const HssMerge* __restrict__ ms, const int2* __restrict__ leafjobs,
                                                   double* __restrict__ out, const int64_t* __restrict__ uoff) {
  const int2 jb = leafjobs[blockIdx.x];
  const HssMerge& M = ms[jb.x];
  const HssNode& nd = M.nodes[jb.y];
  const int m = nd.hi - nd.lo;
  const double* U = M.arena + nd.offU;
  double* O = out + uoff[blockIdx.x];
  for (int e = threadIdx.x; e < m * nd.kr; e += blockDim.x) {
    const int a = e % m, k = e / m;
    O[e] = U[(M.perm[nd.lo + a] - nd.lo) + (int64_t)k * nd.nr];
  }
}

// Probe products of the accuracy check, (W^T Q')^T = Q'^T W, with W K x ldw
// row-major and 8 probe columns c0..c0+7 per pass: one column j of Q' per
// lane, the row range split into nseg segments (one per workgroup row) whose
// partial sums part[seg][j][8] k_probe_sum adds.  Q'(i, j) = uh_i v_j /
// (d_i - lam_j) (eq. Ev-Q, differences by eq. d-lambda) is generated in FP64
// registers; the reciprocal is the hardware estimate refined by two Newton
// steps.
__device__ __forceinline__ double rcp_refined(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

template <int NCP>
__global__ void __launch_bounds__(64) k_probe_qt(const HssMerge* __restrict__ ms, int g, const double* __restrict__ W,
                                                 int ldw, int c0, int nc, int nseg, double* __restrict__ part) {
  __shared__ double s_d[65], s_u[64], s_w[64][NCP];
  const HssMerge& M = ms[g];
  const int K = M.K;
  const int ntj = (K + 63) / 64;
  const int jt = blockIdx.x % ntj, seg = blockIdx.x / ntj;
  const int lane = threadIdx.x;
  const int j = jt * 64 + lane;
  const bool valid = j < K;
  const int len = (K + nseg - 1) / nseg;
  const int ia = seg * len, ib = min(K, ia + len);
  double dj = 0.0, dj1 = 0.0, gj = 0.0, mj = 0.0, vj = 0.0;
  if (valid) {
    dj = M.d[j];
    dj1 = (j + 1 < K) ? M.d[j + 1] : 0.0;
    gj = M.gam[j];
    mj = M.mu[j];
    vj = M.v[j];
  }
  double acc[NCP];
#pragma unroll
  for (int c = 0; c < NCP; ++c) acc[c] = 0.0;
  for (int i0 = ia; i0 < ib; i0 += 64) {
    __syncthreads();
    const int i = i0 + lane;
    s_d[lane] = (i < ib) ? M.d[i] : 0.0;
    s_u[lane] = (i < ib) ? M.uh[i] : 0.0;
#pragma unroll
    for (int c = 0; c < NCP; ++c) s_w[lane][c] = (i < ib && c < nc) ? W[(int64_t)i * ldw + c0 + c] : 0.0;
    __syncthreads();
    const int cnt = min(64, ib - i0);
    if (valid) {
      for (int t = 0; t < cnt; ++t) {
        const double dl = d_minus_lam(i0 + t, j, s_d[t], dj, dj1, gj, mj);
        const double q = s_u[t] * vj * rcp_refined(dl);
#pragma unroll
        for (int c = 0; c < NCP; ++c) acc[c] = fma(q, s_w[t][c], acc[c]);
      }
    }
  }
  if (valid) {
#pragma unroll
    for (int c = 0; c < NCP; ++c) part[((int64_t)seg * K + j) * 8 + c] = acc[c];
  }
}
template __global__ void k_probe_qt<4>(const HssMerge*, int, const double*, int, int, int, int, double*);
template __global__ void k_probe_qt<8>(const HssMerge*, int, const double*, int, int, int, int, double*);

// out[j ldo + col] = sum over segments of part[seg][j][col - c0] for col in
// [c0, c0 + nc); columns at or beyond ntot (the probe count) are zeroed.
__global__ void k_probe_sum(const double* __restrict__ part, int K, int nseg, int c0, int nc, int ntot,
                            double* __restrict__ out, int ldo) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)K * ldo) return;
  const int j = (int)(e / ldo), col = (int)(e % ldo);
  if (col >= c0 && col < c0 + nc) {
    double x = 0.0;
    for (int sg = 0; sg < nseg; ++sg) x += part[((int64_t)sg * K + j) * 8 + (col - c0)];
    out[e] = x;
  } else if (col >= ntot) {
    out[e] = 0.0;
  }
}

// Partial sums of the check norms over rows of a K x ld row-major pair,
// columns < nc: part[2 blk] = sum (a - b)^2, part[2 blk + 1] = sum b^2 over
// the block's rows (fixed order); k_sum_pairs adds the blocks' pairs.
__global__ void __launch_bounds__(256) k_diff_norms(const double* __restrict__ a, const double* __restrict__ b,
                                                    int64_t K, int ld, int nc, double* __restrict__ part) {
  __shared__ double s0[256], s1[256];
  double x0 = 0.0, x1 = 0.0;
  const int64_t n = K * nc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = (e / nc) * ld + (e % nc);
    const double dd = a[i] - b[i];
    x0 += dd * dd;
    x1 += b[i] * b[i];
  }
  s0[threadIdx.x] = x0;
  s1[threadIdx.x] = x1;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      s0[threadIdx.x] += s0[threadIdx.x + st];
      s1[threadIdx.x] += s1[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s0[0];
    part[2 * blockIdx.x + 1] = s1[0];
  }
}

__global__ void k_sum_pairs(const double* __restrict__ part, int nblk, double* __restrict__ out2) {
  if (threadIdx.x != 0) return;
  double x0 = 0.0, x1 = 0.0;
  for (int i = 0; i < nblk; ++i) {
    x0 += part[2 * i];
    x1 += part[2 * i + 1];
  }
  out2[0] = x0;
  out2[1] = x1;
}
