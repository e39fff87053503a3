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
// In both, each wave stages its share of the pole data through LDS in chunks
// of 64 (coalesced vector loads, one chunk prefetched) and reads it back as
// broadcasts.
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
  __shared__ double s_stage[MAXW][200];
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
  // the wave's poles staged through its LDS buffer in chunks of 64 (d with
  // one more entry for d_{j+1}, gam, mu), the next chunk loaded while this
  // one is used; every lane takes part, lanes beyond K discard their result
  double* bd = s_stage[wv];
  double* bg = bd + 72;
  double* bm = bg + 64;
  auto ld = [&](int c, double& xd, double& xg, double& xm) {
    const int jj = c + lane;
    xd = (jj < j1) ? d[jj] : 0.0;
    xg = (jj < j1) ? gam[jj] : 0.0;
    xm = (jj < j1) ? mu[jj] : 0.0;
  };
  double nd = 0.0, ng = 0.0, nmu = 0.0;
  if (j0 < j1) ld(j0, nd, ng, nmu);
  for (int c0 = j0; c0 < j1; c0 += 64) {
    const int cnt = min(64, j1 - c0);
    bd[lane] = nd;
    bg[lane] = ng;
    bm[lane] = nmu;
    if (lane == 0) bd[cnt] = (c0 + cnt < K) ? d[c0 + cnt] : 0.0;  // d_{j+1} of the chunk's last pole
    ld(c0 + 64, nd, ng, nmu);
    int u = 0;
    // four factors per step; exponents split off after every step
    for (; u + 3 < cnt; u += 4) {
      const int j = c0 + u;
      const double e0 = bd[u], e1 = bd[u + 1], e2 = bd[u + 2], e3 = bd[u + 3], e4 = bd[u + 4];
      // lam_j - d_i = -(d_i - lam_j), Remark 1
      nm *= -d_minus_lam(i, j, di, e0, e1, bg[u], bm[u]);
      nm *= -d_minus_lam(i, j + 1, di, e1, e2, bg[u + 1], bm[u + 1]);
      nm *= -d_minus_lam(i, j + 2, di, e2, e3, bg[u + 2], bm[u + 2]);
      nm *= -d_minus_lam(i, j + 3, di, e3, e4, bg[u + 3], bm[u + 3]);
      dm *= (j == i) ? 1.0 : (e0 - di);
      dm *= (j + 1 == i) ? 1.0 : (e1 - di);
      dm *= (j + 2 == i) ? 1.0 : (e2 - di);
      dm *= (j + 3 == i) ? 1.0 : (e3 - di);
      renorm(nm, ne);
      renorm(dm, de);
    }
    for (; u < cnt; ++u) {
      const int j = c0 + u;
      nm *= -d_minus_lam(i, j, di, bd[u], bd[u + 1], bg[u], bm[u]);
      if (j != i) dm *= (bd[u] - di);
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
  __shared__ double s_stage[MAXW][128];
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
  // the wave's rows staged through its LDS buffer in chunks of 64 (uh, d),
  // the next chunk loaded while this one is used; every lane takes part,
  // lanes beyond K discard their result
  double* bu = s_stage[wv];
  double* bx = bu + 64;
  double nu = (i0 + lane < i1) ? uh[i0 + lane] : 0.0;
  double nx = (i0 + lane < i1) ? d[i0 + lane] : 0.0;
  for (int c0 = i0; c0 < i1; c0 += 64) {
    const int cnt = min(64, i1 - c0);
    bu[lane] = nu;
    bx[lane] = nx;
    nu = (c0 + 64 + lane < i1) ? uh[c0 + 64 + lane] : 0.0;
    nx = (c0 + 64 + lane < i1) ? d[c0 + 64 + lane] : 0.0;
    // reciprocals from the hardware estimate and two Newton steps; four
    // terms per step
    int u = 0;
    for (; u + 3 < cnt; u += 4) {
      const int i = c0 + u;
      const double q0 = bu[u] * rcp_nr2(d_minus_lam(i, j, bx[u], dj, dj1, gj, mj));
      const double q1 = bu[u + 1] * rcp_nr2(d_minus_lam(i + 1, j, bx[u + 1], dj, dj1, gj, mj));
      const double q2 = bu[u + 2] * rcp_nr2(d_minus_lam(i + 2, j, bx[u + 2], dj, dj1, gj, mj));
      const double q3 = bu[u + 3] * rcp_nr2(d_minus_lam(i + 3, j, bx[u + 3], dj, dj1, gj, mj));
      acc = fma(q0, q0, fma(q2, q2, acc));
      acc1 = fma(q1, q1, fma(q3, q3, acc1));
    }
    for (; u < cnt; ++u) {
      const double q = bu[u] * rcp_nr2(d_minus_lam(c0 + u, j, bx[u], dj, dj1, gj, mj));
      acc = fma(q, q, acc);
    }
  }
  acc += acc1;
  s_p[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && valid) {
    double s = 0.0;
    for (int w2 = 0; w2 < W; ++w2) s += s_p[w2][lane];
    vS[base + j] = 1.0 / sqrt(s);
  }
}
