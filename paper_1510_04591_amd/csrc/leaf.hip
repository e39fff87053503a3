// Leaf eigenproblems of the DC tree (Algorithm 1, first branch).
//
// The paper solves the leaves (size below the leaf size m) with the QR
// algorithm; here every leaf is one workgroup running parallel-order cyclic
// Jacobi (Brent-Luk round-robin pairing) on the dense leaf matrix held in
// LDS: all m/2 disjoint rotations of a round are computed together, then
// applied to the columns of A and V and to the rows of A, until the
// off-diagonal mass falls below 16 eps^2 ||A||_F^2.  Eigenvalues are sorted
// ascending and the eigenvectors written into the leaf's output block.
//
// The LDS holds exactly the leaf (A and V, m x (m + 1) each, dynamic), so a
// compute unit keeps eight 32 x 32 leaves of four wavefronts in flight.
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int NT = 256;  // threads per leaf

__global__ void __launch_bounds__(NT) k_leaf_jacobi(const double* __restrict__ a, const double* __restrict__ b,
                                                    const int64_t* __restrict__ leaf_s0,
                                                    const int32_t* __restrict__ leaf_m, double* __restrict__ w,
                                                    const LeafOut* __restrict__ outs, int max_sweeps) {
  extern __shared__ double lds[];  // A then V, m x (m + 1) each, row-major
  __shared__ double s_c[32], s_s[32], s_w[64], s_red[NT / 64];
  __shared__ int s_p[32], s_q[32], s_rk[64];
  const int tid = threadIdx.x;
  const int64_t s0 = leaf_s0[blockIdx.x];
  const int m = leaf_m[blockIdx.x];
  const int ld = m + 1;
  double* __restrict__ A = lds;
  double* __restrict__ V = lds + m * ld;
  const int me = m + (m & 1);  // even number of players for the round robin
  const int np = me / 2;

  // sum over the workgroup, the same value in every lane
  auto block_sum = [&](double x) {
    x = wave_sum(x);
    if ((tid & 63) == 0) s_red[tid >> 6] = x;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < NT / 64; ++i) t += s_red[i];
    __syncthreads();
    return t;
  };

  double part = 0.0;
  for (int e = tid; e < m * m; e += NT) {
    const int r = e % m, c = e / m;
    double x = 0.0;
    if (r == c) x = a[s0 + r];
    else if (r == c + 1) x = b[s0 + c];
    else if (c == r + 1) x = b[s0 + r];
    A[r * ld + c] = x;
    V[r * ld + c] = (r == c) ? 1.0 : 0.0;
    part += x * x;
  }
  const double fro2 = block_sum(part);
  __syncthreads();

  for (int sweep = 0; sweep < max_sweeps && m > 1; ++sweep) {
    part = 0.0;
    for (int e = tid; e < m * m; e += NT) {
      const int r = e % m, c = e / m;
      if (r != c) part += A[r * ld + c] * A[r * ld + c];
    }
    if (block_sum(part) <= 16.0 * ADC_EPS * ADC_EPS * fro2) break;

    for (int round = 0; round < me - 1; ++round) {
      if (tid < np) {
        // circle method: position 0 fixed, the others rotate
        const int pa = tid, pb = me - 1 - tid;
        const int p = (pa == 0) ? 0 : ((pa - 1 + round) % (me - 1)) + 1;
        const int q = (pb == 0) ? 0 : ((pb - 1 + round) % (me - 1)) + 1;
        double c = 1.0, s = 0.0;
        if (p < m && q < m) {
          const double apq = A[p * ld + q];
          if (apq != 0.0) {
            const double theta = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        s_p[tid] = p;
        s_q[tid] = q;
        s_c[tid] = c;
        s_s[tid] = s;
      }
      __syncthreads();
      // A <- A J and V <- V J (columns p, q of every pair)
      for (int e = tid; e < np * m; e += NT) {
        const int k = e / m, r = e % m;
        const int p = s_p[k], q = s_q[k];
        if (p < m && q < m) {
          const double c = s_c[k], s = s_s[k];
          const double ap = A[r * ld + p], aq = A[r * ld + q];
          A[r * ld + p] = c * ap - s * aq;
          A[r * ld + q] = s * ap + c * aq;
          const double vp = V[r * ld + p], vq = V[r * ld + q];
          V[r * ld + p] = c * vp - s * vq;
          V[r * ld + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
      // A <- J^T A (rows p, q)
      for (int e = tid; e < np * m; e += NT) {
        const int k = e / m, col = e % m;
        const int p = s_p[k], q = s_q[k];
        if (p < m && q < m) {
          const double c = s_c[k], s = s_s[k];
          const double ap = A[p * ld + col], aq = A[q * ld + col];
          A[p * ld + col] = c * ap - s * aq;
          A[q * ld + col] = s * ap + c * aq;
        }
      }
      __syncthreads();
    }
  }

  if (tid < m) s_w[tid] = A[tid * ld + tid];
  __syncthreads();
  // stable rank of each eigenvalue
  if (tid < m) {
    const double wi = s_w[tid];
    int rk = 0;
    for (int j = 0; j < m; ++j) {
      const double wj = s_w[j];
      rk += (wj < wi) || (wj == wi && j < tid);
    }
    w[s0 + rk] = wi;
    s_rk[tid] = rk;
  }
  __syncthreads();
  double* __restrict__ Z = outs[blockIdx.x].z;
  const int64_t ldz = outs[blockIdx.x].ld;
  for (int e = tid; e < m * m; e += NT) {
    const int r = e % m, i = e / m;
    Z[r + s_rk[i] * ldz] = V[r * ld + i];
  }
}

}  // namespace

// Leaves above 63 rows take more than the default 64 KiB of dynamic LDS:
// raised once for the largest leaf (64 rows) with the device current, at
// context creation, outside any stream capture.
void leaf_init() {
  hipFuncSetAttribute((const void*)k_leaf_jacobi, hipFuncAttributeMaxDynamicSharedMemorySize,
                      2 * 64 * 65 * (int)sizeof(double));
}

void launch_leaf_jacobi(hipStream_t st, int64_t nleaf, int leaf_max, const double* a, const double* b,
                        const int64_t* leaf_s0, const int32_t* leaf_m, double* w, const LeafOut* outs,
                        int max_sweeps) {
  if (nleaf <= 0) return;
  const size_t lds = (size_t)2 * leaf_max * (leaf_max + 1) * sizeof(double);
  hipLaunchKernelGGL(k_leaf_jacobi, dim3((unsigned)nleaf), dim3(NT), lds, st, a, b, leaf_s0, leaf_m, w, outs,
                     max_sweeps);
}
