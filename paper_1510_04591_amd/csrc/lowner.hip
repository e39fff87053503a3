// Loewner recompute of z (eq. ev_z) and the column scales v of eq. (EVec).
//
// k_lowner: one lane per index i, the product over j split across the waves
// of the workgroup:
//     uh_i^2 = prod_j (lam_j - d_i) / (rho prod_{j != i} (d_j - d_i)),
// with lam_j - d_i taken from the accurate differences of Remark 1.  The
// numerator and denominator are accumulated as separate running products
// whose binary exponents are split off every four factors (no division per
// term); sign(uh_i) = sign(z_i).
// k_vnorm: one lane per column j, v_j = 1/sqrt(sum_i (uh_i/(d_i - lam_j))^2),
// the reciprocals refined from the hardware estimate by two Newton steps.
#include "common.hpp"
#include "kernels.hpp"

namespace {
constexpr int MAXW = 16;

__device__ __forceinline__ double rcp_nr2(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ void renorm(double& m, int& e) {
  int ex;
  m = frexp(m, &ex);
  e += ex;
}
}  // namespace

__global__ void __launch_bounds__(1024) k_lowner(const MergeDev* __restrict__ merges,
                                                 const RootBlock* __restrict__ blocks,
                                                 const double* __restrict__ dS, const double* __restrict__ zS,
                                                 const double* __restrict__ gamS, const double* __restrict__ muS,
                                                 double* __restrict__ uhS) {
  __shared__ double s_nm[MAXW][64], s_dm[MAXW][64];
  __shared__ int s_ne[MAXW][64], s_de[MAXW][64];
  const RootBlock rb = blocks[blockIdx.x];
  const MergeDev& M = merges[rb.merge];
  const int K = M.K;
  if (rb.i0 >= K) return;
  const int lane = threadIdx.x & 63, wv = wave_index(), W = blockDim.x >> 6;
  const int64_t base = M.s0;
  const double* __restrict__ d = dS + base;
  const double* __restrict__ gam = gamS + base;
  const double* __restrict__ mu = muS + base;
  const int i = rb.i0 + lane;
  const bool valid = i < K;
  const double di = valid ? d[i] : 0.0;
  const int chunk = (K + W - 1) / W;
  const int j0 = wv * chunk, j1 = min(K, j0 + chunk);
  double nm = 1.0, dm = 1.0;
  int ne = 0, de = 0;
  if (valid) {
    // four factors per step, the (wave-uniform) loads of a step issued
    // together; exponents split off after every step
    int j = j0;
    for (; j + 3 < j1; j += 4) {
      const double e0 = d[j], e1 = d[j + 1], e2 = d[j + 2], e3 = d[j + 3];
      const double e4 = (j + 4 < K) ? d[j + 4] : 0.0;
      const double g0 = gam[j], g1 = gam[j + 1], g2 = gam[j + 2], g3 = gam[j + 3];
      const double m0 = mu[j], m1 = mu[j + 1], m2 = mu[j + 2], m3 = mu[j + 3];
      // lam_j - d_i = -(d_i - lam_j), Remark 1
      nm *= -d_minus_lam(i, j, di, e0, e1, g0, m0);
      nm *= -d_minus_lam(i, j + 1, di, e1, e2, g1, m1);
      nm *= -d_minus_lam(i, j + 2, di, e2, e3, g2, m2);
      nm *= -d_minus_lam(i, j + 3, di, e3, e4, g3, m3);
      dm *= (j == i) ? 1.0 : (e0 - di);
      dm *= (j + 1 == i) ? 1.0 : (e1 - di);
      dm *= (j + 2 == i) ? 1.0 : (e2 - di);
      dm *= (j + 3 == i) ? 1.0 : (e3 - di);
      renorm(nm, ne);
      renorm(dm, de);
    }
    for (; j < j1; ++j) {
      const double dj = d[j];
      const double dj1 = (j + 1 < K) ? d[j + 1] : 0.0;
      nm *= -d_minus_lam(i, j, di, dj, dj1, gam[j], mu[j]);
      if (j != i) dm *= (dj - di);
    }
    renorm(nm, ne);
    renorm(dm, de);
  }
  s_nm[wv][lane] = nm;
  s_dm[wv][lane] = dm;
  s_ne[wv][lane] = ne;
  s_de[wv][lane] = de;
  __syncthreads();
  if (wv == 0 && valid) {
    double N = 1.0, D = 1.0;
    int en = 0, ed = 0;
    for (int w2 = 0; w2 < W; ++w2) {
      N *= s_nm[w2][lane];
      D *= s_dm[w2][lane];
      en += s_ne[w2][lane];
      ed += s_de[w2][lane];
      renorm(N, en);
      renorm(D, ed);
    }
    const double u2 = ldexp(N / (D * M.rho), en - ed);
    const double zi = zS[base + i];
    const double u = sqrt(u2);
    uhS[base + i] = (zi < 0.0) ? -u : u;
  }
}

__global__ void __launch_bounds__(1024) k_vnorm(const MergeDev* __restrict__ merges,
                                                const RootBlock* __restrict__ blocks,
                                                const double* __restrict__ dS, const double* __restrict__ gamS,
                                                const double* __restrict__ muS, const double* __restrict__ uhS,
                                                double* __restrict__ vS) {
  __shared__ double s_p[MAXW][64];
  const RootBlock rb = blocks[blockIdx.x];
  const MergeDev& M = merges[rb.merge];
  const int K = M.K;
  if (rb.i0 >= K) return;
  const int lane = threadIdx.x & 63, wv = wave_index(), W = blockDim.x >> 6;
  const int64_t base = M.s0;
  const double* __restrict__ d = dS + base;
  const double* __restrict__ uh = uhS + base;
  const int j = rb.i0 + lane;
  const bool valid = j < K;
  double dj = 0.0, dj1 = 0.0, gj = 0.0, mj = 0.0;
  if (valid) {
    dj = d[j];
    dj1 = (j + 1 < K) ? d[j + 1] : 0.0;
    gj = gamS[base + j];
    mj = muS[base + j];
  }
  const int chunk = (K + W - 1) / W;
  const int i0 = wv * chunk, i1 = min(K, i0 + chunk);
  double acc = 0.0, acc1 = 0.0;
  if (valid) {
    // reciprocals from the hardware estimate and two Newton steps; four
    // terms per step with their loads issued together
    int i = i0;
    for (; i + 3 < i1; i += 4) {
      const double u0 = uh[i], u1 = uh[i + 1], u2 = uh[i + 2], u3 = uh[i + 3];
      const double x0 = d[i], x1 = d[i + 1], x2 = d[i + 2], x3 = d[i + 3];
      const double q0 = u0 * rcp_nr2(d_minus_lam(i, j, x0, dj, dj1, gj, mj));
      const double q1 = u1 * rcp_nr2(d_minus_lam(i + 1, j, x1, dj, dj1, gj, mj));
      const double q2 = u2 * rcp_nr2(d_minus_lam(i + 2, j, x2, dj, dj1, gj, mj));
      const double q3 = u3 * rcp_nr2(d_minus_lam(i + 3, j, x3, dj, dj1, gj, mj));
      acc = fma(q0, q0, fma(q2, q2, acc));
      acc1 = fma(q1, q1, fma(q3, q3, acc1));
    }
    for (; i < i1; ++i) {
      const double q = uh[i] * rcp_nr2(d_minus_lam(i, j, d[i], dj, dj1, gj, mj));
      acc = fma(q, q, acc);
    }
    acc += acc1;
  }
  s_p[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && valid) {
    double s = 0.0;
    for (int w2 = 0; w2 < W; ++w2) s += s_p[w2][lane];
    vS[base + j] = 1.0 / sqrt(s);
  }
}
