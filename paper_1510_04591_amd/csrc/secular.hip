// Secular equation of D + rho z z^T (Theorem 1) on gfx950.
//
// One root per lane; a workgroup owns 64 consecutive roots of one merge and
// splits the pole sum over its W waves (W = blockDim/64), so that large
// secular sizes still put many waves on every SIMD.  Each wave stages its
// share of the poles d_j and weights z_j through LDS in chunks of 64 (one
// coalesced vector load per chunk, prefetched one chunk ahead) and reads
// them back as broadcasts; only the few poles whose side of the split differs
// between the block's roots are read directly.
//
// Iteration (written from the rational-interpolation literature: Bunch,
// Nielsen & Sorensen 1978; Li 1993): with origin d_o the nearer pole and
// tau = lam - d_o, the function
//     g(tau) = 1/rho + psi(tau) + phi(tau),
//     psi = sum_{j<=sp} z_j^2/(delta_j - tau),  phi = sum_{j>sp} z_j^2/(delta_j - tau)
// (delta_j = d_j - d_o, sp = i for interior roots, K-2 for the last) is
// modelled near tau by  C + q/(D1 - eta) + Q/(D2 - eta)  with the poles
// D1 = delta_sp - tau, D2 = delta_{sp+1} - tau, q = D1^2 psi', Q = D2^2 phi'
// and C fixed by g(tau); the model root of the quadratic is the next step.
// A bracket from the signs of g guards every step; a step leaving it is
// replaced by a bisection over the representable doubles.  Convergence: |g|
// below its rounding-error bound, or an exhausted bracket.
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int MAXW = 16;

// 1/x: hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r), each of which squares the relative error.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// s += sum z_j^2/(delta_j - t), ds += sum z_j^2/(delta_j - t)^2 over j in
// [ja, jb), delta_j = d_j - dorg; two independent accumulator pairs.  The
// wave's poles are staged through its own LDS buffer (buf: 128 doubles, d
// then z) in chunks of 64, one pole per lane by a coalesced vector load, the
// next chunk loaded while this one is summed; every lane of the wave takes
// part (its own t and dorg).  (The sum of the terms' magnitudes that the
// error bound needs is not summed here: all terms of poles left of the root
// have one sign and all others the other, so it follows from psi and phi.)
__device__ __forceinline__ void pole_sums_staged(const double* __restrict__ d, const double* __restrict__ z, int ja,
                                                 int jb, double dorg, double t, double& s, double& ds, double* buf,
                                                 int lane) {
  double s0 = 0.0, s1 = 0.0, q0 = 0.0, q1 = 0.0;
  if (ja >= jb) return;
  double dn = (ja + lane < jb) ? d[ja + lane] : 0.0;
  double zn = (ja + lane < jb) ? z[ja + lane] : 0.0;
  for (int c0 = ja; c0 < jb; c0 += 64) {
    const int cnt = min(64, jb - c0);
    buf[lane] = dn;
    buf[64 + lane] = zn;
    const int c1 = c0 + 64;
    dn = (c1 + lane < jb) ? d[c1 + lane] : 0.0;
    zn = (c1 + lane < jb) ? z[c1 + lane] : 0.0;
    int u = 0;
    for (; u + 3 < cnt; u += 4) {
      const double z0 = buf[64 + u], z1 = buf[65 + u], z2 = buf[66 + u], z3 = buf[67 + u];
      const double t0 = z0 * rcp_nr((buf[u] - dorg) - t);
      const double t1 = z1 * rcp_nr((buf[u + 1] - dorg) - t);
      const double t2 = z2 * rcp_nr((buf[u + 2] - dorg) - t);
      const double t3 = z3 * rcp_nr((buf[u + 3] - dorg) - t);
      s0 = fma(z0, t0, fma(z2, t2, s0));
      s1 = fma(z1, t1, fma(z3, t3, s1));
      q0 = fma(t0, t0, fma(t2, t2, q0));
      q1 = fma(t1, t1, fma(t3, t3, q1));
    }
    for (; u < cnt; ++u) {
      const double za = buf[64 + u];
      const double ta = za * rcp_nr((buf[u] - dorg) - t);
      s0 = fma(za, ta, s0);
      q0 = fma(ta, ta, q0);
    }
  }
  s += s0 + s1;
  ds += q0 + q1;
}

__device__ __forceinline__ double bits_mid(double lo, double hi) {
  // midpoint over the ordered set of doubles of one sign (|lo| < |hi| or the
  // reverse); both have the sign of hi or are zero.
  unsigned long long a = (unsigned long long)__double_as_longlong(fabs(lo));
  unsigned long long b = (unsigned long long)__double_as_longlong(fabs(hi));
  unsigned long long m = a + (b - a) / 2ull;
  if (b < a) m = b + (a - b) / 2ull;
  double r = __longlong_as_double((long long)m);
  return (hi < 0.0 || lo < 0.0) ? -r : r;
}

}  // namespace

__global__ void __launch_bounds__(1024) k_secular(const MergeDev* __restrict__ merges,
                                                  const RootBlock* __restrict__ blocks,
                                                  const double* __restrict__ dS,
                                                  const double* __restrict__ zS, double* __restrict__ lamS,
                                                  double* __restrict__ gamS, double* __restrict__ muS,
                                                  int max_iter, int* __restrict__ noconv) {
  __shared__ double s_part[4][MAXW][64];
  __shared__ double s_stage[MAXW][128];
  __shared__ double s_tau[64];
  __shared__ int s_org[64];
  __shared__ int s_done[64];
  __shared__ int s_any;

  const RootBlock rb = blocks[blockIdx.x];
  const MergeDev& M = merges[rb.merge];
  const int K = M.K;
  const int lane = threadIdx.x & 63;
  const int wv = wave_index();
  const int W = blockDim.x >> 6;
  if (rb.i0 >= K) return;  // block-uniform
  const int64_t base = M.s0;
  const double* __restrict__ d = dS + base;
  const double* __restrict__ z = zS + base;
  const double rho = M.rho;
  const double rhoinv = 1.0 / rho;
  const int i = rb.i0 + lane;
  const bool valid = i < K;
  const bool last = (i == K - 1);

  // j range of this wave
  const int chunk = (K + W - 1) / W;
  const int j0 = wv * chunk;
  const int j1 = min(K, j0 + chunk);
  // split index sp_i = i (K-2 for the last root): its range over the block
  const int spmin = min(rb.i0, K - 2);
  const int spmax = min(rb.i0 + 63, K - 2);

  // wave-0 lane state
  double lo = 0.0, hi = 0.0, gap = 0.0, tau = 0.0;
  int org = 0, it = 0;
  bool done = !valid;

  if (K == 1) {
    if (threadIdx.x == 0) {
      const double g = rho * z[0] * z[0];
      gamS[base] = g;
      muS[base] = INFINITY;
      if (lamS) lamS[base] = d[0] + g;
    }
    return;
  }

  if (wv == 0) {
    if (valid) {
      gap = last ? INFINITY : (d[i + 1] - d[i]);
      // phase 0 point, frame d_i: the midpoint for interior roots; for the
      // last root rho z_K^2, a lower bound of its distance to d_K
      tau = last ? fmax(rho * z[i] * z[i], 1e-300) : 0.5 * gap;
      org = i;
    }
    s_tau[lane] = tau;
    s_org[lane] = valid ? i : 0;
    s_done[lane] = done ? 1 : 0;
  }
  __syncthreads();

  for (int iter = 0;; ++iter) {
    // ---- partial sums over this wave's poles
    const double t_l = s_tau[lane];
    const int o_l = s_org[lane];
    const bool act = !s_done[lane];
    const int sp = last ? K - 2 : i;
    const double dorg = valid ? d[o_l] : 0.0;
    double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
    // poles j <= spmin belong to psi for every lane, j > spmax to phi
    const int ja = min(j1, max(j0, spmin + 1));
    const int jb = min(j1, max(ja, spmax + 1));
    if (__any(act)) {
      // the whole wave stages the poles; lanes already done discard theirs
      pole_sums_staged(d, z, j0, ja, dorg, t_l, psi, dpsi, s_stage[wv], lane);
      pole_sums_staged(d, z, jb, j1, dorg, t_l, phi, dphi, s_stage[wv], lane);
    }
    if (act) {
      for (int j = ja; j < jb; ++j) {
        const double zj = z[j];
        const double t = zj * rcp_nr((d[j] - dorg) - t_l);
        if (j <= sp) {
          psi = fma(zj, t, psi);
          dpsi = fma(t, t, dpsi);
        } else {
          phi = fma(zj, t, phi);
          dphi = fma(t, t, dphi);
        }
      }
    }
    s_part[0][wv][lane] = psi;
    s_part[1][wv][lane] = dpsi;
    s_part[2][wv][lane] = phi;
    s_part[3][wv][lane] = dphi;
    __syncthreads();

    if (wv == 0) {
      if (!done) {
        psi = dpsi = phi = dphi = 0.0;
        for (int w2 = 0; w2 < W; ++w2) {
          psi += s_part[0][w2][lane];
          dpsi += s_part[1][w2][lane];
          phi += s_part[2][w2][lane];
          dphi += s_part[3][w2][lane];
        }
        const double g = rhoinv + psi + phi;
        // sum of the terms' magnitudes: the poles d_j, j <= sp, lie left of
        // the root (negative terms), the others right of it (positive), but
        // for the last root, where every pole lies to its left
        const double eabs = last ? -(psi + phi) : (phi - psi);
        if (iter == 0) {
          // origin choice (frame d_i): root left of the midpoint iff g >= 0
          if (last) {
            lo = 0.0;
            hi = rho;
          } else if (g >= 0.0) {
            org = i;
            lo = 0.0;
            hi = 0.5 * gap;
          } else {
            org = i + 1;
            tau = -0.5 * gap;  // same point seen from d_{i+1}
            lo = 0.0;
            hi = -0.5 * gap;
          }
        }
        // error bound of the computed g (rounding of every term, of 1/rho
        // and of tau itself)
        const double ebound = ADC_EPS * (8.0 * eabs + 2.0 * rhoinv + 3.0 * fabs(tau) * (dpsi + dphi));
        bool conv = (iter > 0) && (fabs(g) <= ebound);
        if (g == 0.0) conv = true;
        if (!conv) {
          // bracket update from the sign of g (g increases with tau)
          if (iter > 0 || last) {
            if (org == i) {  // tau > 0
              if (g < 0.0) lo = tau; else hi = tau;
            } else {         // tau < 0, |tau| small means near d_{i+1}: g > 0 there
              if (g < 0.0) hi = tau; else lo = tau;
            }
          }
          // model step
          const double dsp = d[sp] - d[org];
          const double dsp1 = d[sp + 1] - d[org];
          const double D1 = dsp - tau;
          const double D2 = dsp1 - tau;
          const double q = D1 * D1 * dpsi;
          const double Q = D2 * D2 * dphi;
          const double C = g - D1 * dpsi - D2 * dphi;
          const double a = C * (D1 + D2) + q + Q;
          const double b = D1 * D2 * g;
          const double disc = sqrt(fabs(a * a - 4.0 * b * C));
          double eta;
          if (!last) {
            eta = (a <= 0.0) ? (a - disc) / (2.0 * C) : (2.0 * b) / (a + disc);
          } else {
            eta = (a >= 0.0) ? (a + disc) / (2.0 * C) : (2.0 * b) / (a - disc);
          }
          double tn = tau + eta;
          // the bracket is (lo, hi) for org == i (0 <= lo < hi) and
          // (hi, lo) for org == i+1 (hi < lo <= 0)
          const double bl = fmin(lo, hi), bh = fmax(lo, hi);
          if (!(tn > bl && tn < bh) || !isfinite(tn)) tn = bits_mid(lo, hi);
          if (tn == tau || tn == lo || tn == hi) conv = true;
          else tau = tn;
          ++it;
          if (it >= max_iter && !conv) {
            conv = true;
            atomicMin(noconv, (int)(M.gbase + i));
          }
        }
        done = conv;
      }
      s_tau[lane] = tau;
      s_org[lane] = org;
      s_done[lane] = done ? 1 : 0;
    }
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    if (wv == 0) {
      const int nd = __any(!done) ? 1 : 0;
      if (lane == 0) s_any = nd;
    }
    __syncthreads();
    if (!s_any) break;
  }

  if (wv == 0 && valid) {
    double gm, mu;
    if (last) {
      gm = tau;
      mu = INFINITY;
    } else if (org == i) {
      gm = tau;
      mu = gap - tau;
    } else {
      mu = -tau;
      gm = gap + tau;
    }
    gamS[base + i] = gm;
    muS[base + i] = mu;
    if (lamS) lamS[base + i] = d[org] + tau;
  }
}
