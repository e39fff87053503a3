// FP64 MFMA GEMM of the dense eigenvector update (Algorithm 1, "compute
// Q = diag(Q1, Q2) Q'"), grouped over independent problems.
//
// C(:, colmap[j]) = vscale[j] * (A * B)(:, j), A M x K, B K x N, column-major.
// Workgroup tile 128 x 128, K step 16, four waves in a 2 x 2 grid, each wave
// owning 64 x 64 outputs as 4 x 4 tiles of v_mfma_f64_16x16x4f64.  Operand
// tiles are staged through LDS (double-buffered; the next tile is fetched into
// registers while the current one feeds the matrix cores).  Lane layout of the
// 16x16x4 f64 instruction: A[i][k] from lane i + 16k, B[k][j] from lane
// j + 16k, D[lane/16 + 4r][lane % 16] in accumulator r.
#include "common.hpp"
#include "kernels.hpp"

namespace {
constexpr int BM = 128, BN = 128, BK = 16;
constexpr int PADA = 4, PADB = 4;
}  // namespace

__global__ void __launch_bounds__(256) k_gemm_f64(const GemmProb* __restrict__ probs, int nprobs) {
  __shared__ double As[2][BK][BM + PADA];
  __shared__ double Bs[2][BK][BN + PADB];

  // locate the problem of this tile
  const int bid = blockIdx.x;
  int p = 0;
  {
    int lo = 0, hi = nprobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (probs[mid].tile0 <= bid) lo = mid; else hi = mid - 1;
    }
    p = lo;
  }
  const GemmProb P = probs[p];
  const int local = bid - P.tile0;
  const int tm = local % P.tiles_m;
  const int tn = local / P.tiles_m;
  const int m0 = tm * BM, n0 = tn * BN;
  if (m0 >= P.M || n0 >= P.N) return;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wm = wv & 1, wn = wv >> 1;
  const int li = lane & 15, lk = lane >> 4;

  const double* __restrict__ A = P.A;
  const double* __restrict__ Bm = P.B;
  const int64_t lda = P.lda, ldb = P.ldb;
  const int M = P.M, N = P.N, Kd = P.K;

  dbl4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

  double ra[8], rb[8];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q;
      const int r = e & (BM - 1), c = e >> 7;  // A: 128 rows x 16 cols
      const int gr = m0 + r, gc = k0 + c;
      ra[q] = (gr < M && gc < Kd) ? A[gr + (int64_t)gc * lda] : 0.0;
      const int kr = e & (BK - 1), cc = e >> 4;  // B: 16 rows x 128 cols
      const int gk = k0 + kr, gn = n0 + cc;
      rb[q] = (gk < Kd && gn < N) ? Bm[gk + (int64_t)gn * ldb] : 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q;
      As[buf][e >> 7][e & (BM - 1)] = ra[q];
      Bs[buf][e & (BK - 1)][e >> 4] = rb[q];
    }
  };

  const int nk = (Kd + BK - 1) / BK;
  if (nk > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int k = kk * 4 + lk;
      double av[4], bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        av[t] = As[buf][k][wm * 64 + t * 16 + li];
        bv[t] = Bs[buf][k][wn * 64 + t * 16 + li];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  // epilogue
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int col = n0 + wn * 64 + b * 16 + li;
    if (col >= N) continue;
    const double vs = P.vscale ? P.vscale[col] : 1.0;
    const int64_t cc = (int64_t)(P.colmap ? P.colmap[col] : col) * P.ldc;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int row0 = m0 + wm * 64 + a * 16 + lk;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + 4 * r;
        if (row < M) P.C[row + cc] = acc[a][b][r] * vs;
      }
    }
  }
}
