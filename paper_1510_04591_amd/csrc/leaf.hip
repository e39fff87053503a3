// Leaf eigenproblems of the DC tree (Algorithm 1, first branch).
//
// The paper solves the leaves (size < m) with the QR algorithm; here every
// leaf is one workgroup running parallel-order cyclic Jacobi (Brent-Luk
// round-robin pairing) on the dense leaf matrix held in LDS: all m/2 disjoint
// rotations of a round are computed together, then applied to the columns of
// A and V and to the rows of A.  Eigenvalues are sorted ascending and the
// eigenvectors written into the leaf's output block.
#include "common.hpp"
#include "kernels.hpp"

#define LEAF_MAX 64

__global__ void __launch_bounds__(256) k_leaf_jacobi(const double* __restrict__ a, const double* __restrict__ b,
                                                     const int64_t* __restrict__ leaf_s0,
                                                     const int32_t* __restrict__ leaf_m, double* __restrict__ w,
                                                     const LeafOut* __restrict__ outs, int max_sweeps) {
  __shared__ double A[LEAF_MAX][LEAF_MAX + 1];
  __shared__ double V[LEAF_MAX][LEAF_MAX + 1];
  __shared__ double s_c[LEAF_MAX / 2], s_s[LEAF_MAX / 2];
  __shared__ int s_p[LEAF_MAX / 2], s_q[LEAF_MAX / 2];
  __shared__ double s_red[256];
  __shared__ double s_w[LEAF_MAX];

  const int tid = threadIdx.x;
  const int64_t s0 = leaf_s0[blockIdx.x];
  const int m = leaf_m[blockIdx.x];
  const int me = m + (m & 1);  // even number of players for the round robin
  const int np = me / 2;

  for (int e = tid; e < m * m; e += blockDim.x) {
    const int r = e % m, c = e / m;
    double x = 0.0;
    if (r == c) x = a[s0 + r];
    else if (r == c + 1) x = b[s0 + c];
    else if (c == r + 1) x = b[s0 + r];
    A[r][c] = x;
    V[r][c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();

  // ||A||_F
  double part = 0.0;
  for (int e = tid; e < m * m; e += blockDim.x) {
    const double x = A[e % m][e / m];
    part += x * x;
  }
  s_red[tid] = part;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (tid < st) s_red[tid] += s_red[tid + st];
    __syncthreads();
  }
  const double fro2 = s_red[0];
  __syncthreads();

  for (int sweep = 0; sweep < max_sweeps && m > 1; ++sweep) {
    // off-diagonal mass
    part = 0.0;
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int r = e % m, c = e / m;
      if (r != c) part += A[r][c] * A[r][c];
    }
    s_red[tid] = part;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
      if (tid < st) s_red[tid] += s_red[tid + st];
      __syncthreads();
    }
    const double off2 = s_red[0];
    __syncthreads();
    if (off2 <= 16.0 * ADC_EPS * ADC_EPS * fro2) break;

    for (int round = 0; round < me - 1; ++round) {
      if (tid < np) {
        // circle method: position 0 fixed, the others rotate
        const int pa = tid, pb = me - 1 - tid;
        const int p = (pa == 0) ? 0 : ((pa - 1 + round) % (me - 1)) + 1;
        const int q = (pb == 0) ? 0 : ((pb - 1 + round) % (me - 1)) + 1;
        double c = 1.0, s = 0.0;
        if (p < m && q < m) {
          const double apq = A[p][q];
          if (apq != 0.0) {
            const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
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
      for (int e = tid; e < np * m; e += blockDim.x) {
        const int k = e / m, r = e % m;
        const int p = s_p[k], q = s_q[k];
        if (p < m && q < m) {
          const double c = s_c[k], s = s_s[k];
          const double ap = A[r][p], aq = A[r][q];
          A[r][p] = c * ap - s * aq;
          A[r][q] = s * ap + c * aq;
          const double vp = V[r][p], vq = V[r][q];
          V[r][p] = c * vp - s * vq;
          V[r][q] = s * vp + c * vq;
        }
      }
      __syncthreads();
      // A <- J^T A (rows p, q)
      for (int e = tid; e < np * m; e += blockDim.x) {
        const int k = e / m, col = e % m;
        const int p = s_p[k], q = s_q[k];
        if (p < m && q < m) {
          const double c = s_c[k], s = s_s[k];
          const double ap = A[p][col], aq = A[q][col];
          A[p][col] = c * ap - s * aq;
          A[q][col] = s * ap + c * aq;
        }
      }
      __syncthreads();
    }
  }

  if (tid < m) s_w[tid] = A[tid][tid];
  __syncthreads();
  // stable rank of each eigenvalue
  for (int i = tid; i < m; i += blockDim.x) {
    const double wi = s_w[i];
    int rk = 0;
    for (int j = 0; j < m; ++j) {
      const double wj = s_w[j];
      rk += (wj < wi) || (wj == wi && j < i);
    }
    w[s0 + rk] = wi;
    s_red[i] = (double)rk;
  }
  __syncthreads();
  double* __restrict__ Z = outs[blockIdx.x].z;
  const int64_t ldz = outs[blockIdx.x].ld;
  for (int e = tid; e < m * m; e += blockDim.x) {
    const int r = e % m, i = e / m;
    const int rk = (int)s_red[i];
    Z[r + rk * ldz] = V[r][i];
  }
}
