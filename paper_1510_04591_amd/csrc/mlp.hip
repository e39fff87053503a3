// Learned HSS rank predictor on gfx950.
//
// The sample count of Algorithm 2 comes from a rank per boundary between
// neighbouring leaf segments, maximised over the boundaries (eq. (bounds),
// Section 4.1).  This file replaces the a-priori bound by a learned estimate
// of log2 of the rank the IDs find at each boundary:
//
//   k_mlp_features  16 features per interior leaf boundary of a merge, from
//                   the generators d, gam, mu (differences by eq. (d-lambda));
//                   one workgroup per boundary, FP64, stored as FP32.
//   k_mlp_infer     y = W3 relu(W2 relu(W1 x + b1) + b2) + b3, 16-64-64-1,
//                   FP32, one sample per lane, weights in LDS.
//   k_mlp_train     minibatch forward, backward and Adam (Kingma and Ba
//                   2015) for a whole training run in one workgroup: chunks
//                   of 64 samples through LDS, every parameter's gradient
//                   and Adam moments held by the lane that owns it.  The
//                   same kernel returns the full-batch gradient for checks.
//
// Feature list (cl(x) = log2 x clamped to [-64, 64], -64 for x <= 0; span =
// lam_{K-1} - d_0; dist(q) = min(|lam_q - d_{q-1}|, |d_q - lam_{q-1}|);
// segments [lo, p) and [p, hi); gaps g_j = d_{j+1} - d_j, j in [lo, hi-1)):
//   0 log2 K/16, 1 log2(p-lo)/8, 2 log2(hi-p)/8, 3 cl(span/dist(p))/32,
//   4 cl(span/min_{lo<q<hi} dist(q))/32, 5-7 min/mean/max cl(g_j/span)/32,
//   8 std cl(g_j/span)/8, 9-10 mean/min over [lo, hi) of
//   cl(min(gam_j, mu_j)/span)/32, 11 fraction of g_j < 1e-10 span, 12 p/K,
//   13 log2(leaves)/8, 14 cl((d_{hi-1}-d_lo)/span)/32,
//   15 cl(dist(p)/(d_p - d_{p-1}))/32.
#include <cmath>
#include <cstring>
#include <random>

#include "adc_internal.hpp"

namespace {

constexpr int NF = 16, NH = 64;
constexpr int OW1 = 0, OB1 = NH * NF, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH, OB3 = OW3 + NH;
constexpr int NP = OB3 + 1;  // 5313
constexpr int TPB = 256;
constexpr int PPT = (NP + TPB - 1) / TPB;  // parameters owned per lane
constexpr int CH = 64;                      // samples per chunk
constexpr int LDH = NH + 1;
// dynamic LDS of k_mlp_train, in floats
constexpr int LDS_TRAIN = NP + CH * NF + CH + CH + 4 * CH * LDH;
constexpr int RANK_MARGIN = 4;
constexpr double RANK_SCALE = 1.25;  // the prediction's rank is scaled up before the margin
constexpr int RANK_FLOOR = 8;

__device__ __forceinline__ double clg(double x) {
  if (!(x > 0.0)) return -64.0;
  return fmin(64.0, fmax(-64.0, log2(x)));
}

__device__ __forceinline__ double dist_at(const double* d, const double* gam, const double* mu, int q) {
  const double x = (d[q] - d[q - 1]) + gam[q];
  const double y = mu[q - 1];
  return fmin(fabs(x), fabs(y));
}

}  // namespace

struct MlpState {
  float* theta = nullptr;  // NP parameters, then m (NP), v (NP), loss (4)
  float* m = nullptr;
  float* v = nullptr;
  float* loss = nullptr;
  int64_t t = 0;  // Adam steps taken
  bool ready = false;
  // collection sink (adc_mlp_collect)
  bool collect = false;
  float* cX = nullptr;
  float* cy = nullptr;
  int64_t cap = 0, rows = 0;
};

__global__ void __launch_bounds__(256) k_mlp_features(int K, const double* __restrict__ d,
                                                      const double* __restrict__ gam, const double* __restrict__ mu,
                                                      const int64_t* __restrict__ bounds, int nb,
                                                      float* __restrict__ feat) {
  __shared__ double s_sum[256], s_sq[256], s_min[256], s_max[256], s_tsum[256], s_tmin[256], s_dmin[256];
  __shared__ int s_cnt[256];
  const int b = blockIdx.x;
  if (b >= nb) return;
  const int tid = threadIdx.x;
  const int lo = (int)bounds[b], p = (int)bounds[b + 1], hi = (int)bounds[b + 2];
  const double span = (d[K - 1] + gam[K - 1]) - d[0];
  double sum = 0.0, sq = 0.0, mn = INFINITY, mx = -INFINITY, tsum = 0.0, tmn = INFINITY, dmn = INFINITY;
  int cnt = 0;
  for (int j = lo + tid; j < hi; j += blockDim.x) {
    if (j + 1 < hi) {
      const double g = d[j + 1] - d[j];
      const double lg = clg(g / span);
      sum += lg;
      sq += lg * lg;
      mn = fmin(mn, lg);
      mx = fmax(mx, lg);
      cnt += (g < 1e-10 * span) ? 1 : 0;
    }
    tsum += clg(fmin(gam[j], mu[j]) / span);
    tmn = fmin(tmn, clg(fmin(gam[j], mu[j]) / span));
    if (j > lo) dmn = fmin(dmn, dist_at(d, gam, mu, j));
  }
  s_sum[tid] = sum;
  s_sq[tid] = sq;
  s_min[tid] = mn;
  s_max[tid] = mx;
  s_tsum[tid] = tsum;
  s_tmin[tid] = tmn;
  s_dmin[tid] = dmn;
  s_cnt[tid] = cnt;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (tid < h) {
      s_sum[tid] += s_sum[tid + h];
      s_sq[tid] += s_sq[tid + h];
      s_min[tid] = fmin(s_min[tid], s_min[tid + h]);
      s_max[tid] = fmax(s_max[tid], s_max[tid + h]);
      s_tsum[tid] += s_tsum[tid + h];
      s_tmin[tid] = fmin(s_tmin[tid], s_tmin[tid + h]);
      s_dmin[tid] = fmin(s_dmin[tid], s_dmin[tid + h]);
      s_cnt[tid] += s_cnt[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double dp = dist_at(d, gam, mu, p);
    const int ng = hi - lo - 1;
    double f[NF];
    f[0] = log2((double)K) / 16.0;
    f[1] = log2((double)(p - lo)) / 8.0;
    f[2] = log2((double)(hi - p)) / 8.0;
    f[3] = clg(span / dp) / 32.0;
    f[4] = clg(span / s_dmin[0]) / 32.0;
    if (ng > 0) {
      const double mean = s_sum[0] / ng;
      f[5] = s_min[0] / 32.0;
      f[6] = mean / 32.0;
      f[7] = s_max[0] / 32.0;
      f[8] = sqrt(fmax(s_sq[0] / ng - mean * mean, 0.0)) / 8.0;
      f[11] = (double)s_cnt[0] / ng;
    } else {
      f[5] = f[6] = f[7] = f[8] = f[11] = 0.0;
    }
    f[9] = s_tsum[0] / (hi - lo) / 32.0;
    f[10] = s_tmin[0] / 32.0;
    f[12] = (double)p / K;
    f[13] = log2((double)(nb + 1)) / 8.0;
    f[14] = clg((d[hi - 1] - d[lo]) / span) / 32.0;
    f[15] = clg(dp / (d[p] - d[p - 1])) / 32.0;
    for (int k = 0; k < NF; ++k) feat[(int64_t)b * NF + k] = (float)f[k];
  }
}

__global__ void __launch_bounds__(256) k_mlp_infer(const float* __restrict__ theta, int B, const float* __restrict__ X,
                                                   float* __restrict__ y) {
  __shared__ float P[NP];
  for (int i = threadIdx.x; i < NP; i += blockDim.x) P[i] = theta[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  float x[NF], h1[NH];
#pragma unroll
  for (int k = 0; k < NF; ++k) x[k] = X[(int64_t)s * NF + k];
#pragma unroll
  for (int o = 0; o < NH; ++o) {
    float z = P[OB1 + o];
#pragma unroll
    for (int k = 0; k < NF; ++k) z = fmaf(P[OW1 + o * NF + k], x[k], z);
    h1[o] = fmaxf(z, 0.0f);
  }
  float out = P[OB3];
  for (int o = 0; o < NH; ++o) {
    float z = P[OB2 + o];
#pragma unroll
    for (int i = 0; i < NH; ++i) z = fmaf(P[OW2 + o * NH + i], h1[i], z);
    out = fmaf(P[OW3 + o], fmaxf(z, 0.0f), out);
  }
  y[s] = out;
}

// One workgroup of 256 lanes.  mode 0: `epochs` passes of Adam over
// minibatches of `bs` rows in order, parameters/moments read from and written
// back to theta/m/v, loss[0] = mean squared error of the last pass (each
// minibatch before its update).  mode 1: one minibatch of all B rows, its
// gradient written to g_out and its loss to loss[0]; no update.
__global__ void __launch_bounds__(TPB) k_mlp_train(float* __restrict__ theta, float* __restrict__ mom1,
                                                   float* __restrict__ mom2, const float* __restrict__ X,
                                                   const float* __restrict__ Y, int B, int bs, int epochs, float lr,
                                                   float beta1, float beta2, float eps, int64_t t0, int mode,
                                                   float* __restrict__ g_out, float* __restrict__ loss) {
  extern __shared__ float lds[];
  float* P = lds;                  // NP
  float* Xc = P + NP;              // CH x NF
  float* Yc = Xc + CH * NF;        // CH
  float* Dy = Yc + CH;             // CH
  float* H1 = Dy + CH;             // CH x LDH
  float* H2 = H1 + CH * LDH;
  float* D2 = H2 + CH * LDH;
  float* D1 = D2 + CH * LDH;
  __shared__ float s_sse[TPB / 64];
  const int tid = threadIdx.x;
  for (int i = tid; i < NP; i += TPB) P[i] = theta[i];
  float m1[PPT], m2[PPT], g[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int pi = tid + q * TPB;
    m1[q] = (mode == 0 && pi < NP) ? mom1[pi] : 0.0f;
    m2[q] = (mode == 0 && pi < NP) ? mom2[pi] : 0.0f;
  }
  if (mode == 1) {
    bs = B;
    epochs = 1;
  }
  int64_t t = t0;
  double sse_epoch = 0.0;
  for (int e = 0; e < epochs; ++e) {
    sse_epoch = 0.0;
    for (int i0 = 0; i0 < B; i0 += bs) {
      const int nrow = min(bs, B - i0);
#pragma unroll
      for (int q = 0; q < PPT; ++q) g[q] = 0.0f;
      float sse_lane = 0.0f;
      for (int c0 = 0; c0 < nrow; c0 += CH) {
        const int nc = min(CH, nrow - c0);
        __syncthreads();  // previous chunk's LDS reads are done
        for (int e2 = tid; e2 < CH * NF; e2 += TPB) {
          const int s = e2 / NF;
          Xc[e2] = (s < nc) ? X[(int64_t)(i0 + c0 + s) * NF + (e2 % NF)] : 0.0f;
        }
        if (tid < CH) Yc[tid] = (tid < nc) ? Y[i0 + c0 + tid] : 0.0f;
        __syncthreads();
        // layer 1
        for (int e2 = tid; e2 < CH * NH; e2 += TPB) {
          const int s = e2 / NH, o = e2 % NH;
          float z = P[OB1 + o];
#pragma unroll
          for (int k = 0; k < NF; ++k) z = fmaf(P[OW1 + o * NF + k], Xc[s * NF + k], z);
          H1[s * LDH + o] = (s < nc) ? fmaxf(z, 0.0f) : 0.0f;
        }
        __syncthreads();
        // layer 2
        for (int e2 = tid; e2 < CH * NH; e2 += TPB) {
          const int s = e2 / NH, o = e2 % NH;
          float z = P[OB2 + o];
          for (int i = 0; i < NH; ++i) z = fmaf(P[OW2 + o * NH + i], H1[s * LDH + i], z);
          H2[s * LDH + o] = (s < nc) ? fmaxf(z, 0.0f) : 0.0f;
        }
        __syncthreads();
        // output and d loss / d out = 2 (out - y) / nrow
        if (tid < CH) {
          float out = P[OB3];
          for (int i = 0; i < NH; ++i) out = fmaf(P[OW3 + i], H2[tid * LDH + i], out);
          const float r = (tid < nc) ? out - Yc[tid] : 0.0f;
          sse_lane += r * r;
          Dy[tid] = 2.0f * r / (float)nrow;
        }
        __syncthreads();
        for (int e2 = tid; e2 < CH * NH; e2 += TPB) {
          const int s = e2 / NH, o = e2 % NH;
          D2[s * LDH + o] = (H2[s * LDH + o] > 0.0f) ? Dy[s] * P[OW3 + o] : 0.0f;
        }
        __syncthreads();
        for (int e2 = tid; e2 < CH * NH; e2 += TPB) {
          const int s = e2 / NH, i = e2 % NH;
          float a = 0.0f;
          if (H1[s * LDH + i] > 0.0f)
            for (int o = 0; o < NH; ++o) a = fmaf(D2[s * LDH + o], P[OW2 + o * NH + i], a);
          D1[s * LDH + i] = a;
        }
        __syncthreads();
        // gradients of the parameters this lane owns
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          const int pi = tid + q * TPB;
          if (pi >= NP) continue;
          float a = 0.0f;
          if (pi < OB1) {
            const int o = pi / NF, k = pi % NF;
            for (int s = 0; s < nc; ++s) a = fmaf(D1[s * LDH + o], Xc[s * NF + k], a);
          } else if (pi < OW2) {
            const int o = pi - OB1;
            for (int s = 0; s < nc; ++s) a += D1[s * LDH + o];
          } else if (pi < OB2) {
            const int o = (pi - OW2) / NH, i = (pi - OW2) % NH;
            for (int s = 0; s < nc; ++s) a = fmaf(D2[s * LDH + o], H1[s * LDH + i], a);
          } else if (pi < OW3) {
            const int o = pi - OB2;
            for (int s = 0; s < nc; ++s) a += D2[s * LDH + o];
          } else if (pi < OB3) {
            const int i = pi - OW3;
            for (int s = 0; s < nc; ++s) a = fmaf(Dy[s], H2[s * LDH + i], a);
          } else {
            for (int s = 0; s < nc; ++s) a += Dy[s];
          }
          g[q] += a;
        }
      }
      // squared errors of this minibatch (lanes 0..63 of wave 0 hold them)
      float v = sse_lane;
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if ((tid & 63) == 0) s_sse[tid >> 6] = v;
      __syncthreads();
      if (tid == 0) {
        float tot = 0.0f;
        for (int w = 0; w < TPB / 64; ++w) tot += s_sse[w];
        s_sse[0] = tot;
      }
      __syncthreads();
      sse_epoch += (double)s_sse[0];
      if (mode == 1) break;
      // Adam
      ++t;
      const float c1 = (float)(1.0 - pow((double)beta1, (double)t));
      const float c2 = (float)(1.0 - pow((double)beta2, (double)t));
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        const int pi = tid + q * TPB;
        if (pi >= NP) continue;
        m1[q] = beta1 * m1[q] + (1.0f - beta1) * g[q];
        m2[q] = beta2 * m2[q] + (1.0f - beta2) * g[q] * g[q];
        const float mh = m1[q] / c1, vh = m2[q] / c2;
        P[pi] -= lr * mh / (sqrtf(vh) + eps);
      }
      __syncthreads();
    }
  }
  if (mode == 0) {
    for (int i = tid; i < NP; i += TPB) theta[i] = P[i];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int pi = tid + q * TPB;
      if (pi < NP) {
        mom1[pi] = m1[q];
        mom2[pi] = m2[q];
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int pi = tid + q * TPB;
      if (pi < NP) g_out[pi] = g[q];
    }
  }
  if (tid == 0) loss[0] = (float)(sse_epoch / B);
}

// ---------------------------------------------------------------------------
static adc_status mlp_state(adc_ctx c, MlpState** out) {
  if (!c->mlp) {
    MlpState* s = new MlpState();
    if (hipMalloc((void**)&s->theta, (3 * (size_t)NP + 64) * sizeof(float)) != hipSuccess) {
      delete s;
      return ADC_ERR_NOMEM;
    }
    s->m = s->theta + NP;
    s->v = s->m + NP;
    s->loss = s->v + NP;
    c->mlp = s;
  }
  *out = c->mlp;
  return ADC_OK;
}

void mlp_release(adc_ctx c) {
  if (c->mlp) {
    hipFree(c->mlp->theta);
    delete c->mlp;
    c->mlp = nullptr;
  }
}

static adc_status launch_features(adc_ctx c, int K, const double* d, const double* gam, const double* mu,
                                  const std::vector<int64_t>& bounds, float* feat) {
  const int nb = (int)bounds.size() - 2;
  if (nb <= 0) return ADC_OK;
  void* p;
  ADC_TRY(c->buffer(SLOT_MLP, bounds.size() * 8 + 256, &p));
  HIP_OK(hipMemcpyAsync(p, bounds.data(), bounds.size() * 8, hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_mlp_features, dim3(nb), dim3(256), 0, c->stream, K, d, gam, mu, (const int64_t*)p, nb, feat);
  HIP_OK(hipGetLastError());
  // the bounds staging buffer is reused by the next call
  HIP_OK(hipStreamSynchronize(c->stream));
  return ADC_OK;
}

static adc_status launch_train(adc_ctx c, MlpState* s, int B, const float* X, const float* y, int epochs, int bs,
                               float lr, int mode, float* g_out) {
  static bool attr_set = false;
  if (!attr_set) {
    HIP_OK(hipFuncSetAttribute((const void*)k_mlp_train, hipFuncAttributeMaxDynamicSharedMemorySize,
                               LDS_TRAIN * (int)sizeof(float)));
    attr_set = true;
  }
  hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(TPB), (size_t)LDS_TRAIN * sizeof(float), c->stream, s->theta, s->m,
                     s->v, X, y, B, bs, epochs, lr, 0.9f, 0.999f, 1e-8f, s->t, mode, g_out, s->loss);
  HIP_OK(hipGetLastError());
  return ADC_OK;
}

// Rank of one HSS merge from the predictor: ceil(1.25 2^max_b yhat_b) + margin,
// clamped to [8, r_cap]; r_bound when no model has been initialised.
int mlp_rank(adc_ctx c, const double* d, const double* gam, const double* mu, int K, const std::vector<int>& bounds,
             const adc_opts& o, int r_bound) {
  if (!c->mlp || !c->mlp->ready) return r_bound;
  const int nb = (int)bounds.size() - 2;
  if (nb <= 0) return std::max(RANK_FLOOR, std::min(o.r_cap, r_bound));
  std::vector<int64_t> b64(bounds.begin(), bounds.end());
  void* p;
  const size_t off = ((b64.size() * 8 + 255) / 256) * 256;
  if (c->buffer(SLOT_MLP, off + (size_t)nb * (NF + 1) * 4 + 256, &p) != ADC_OK) return r_bound;
  float* feat = (float*)((char*)p + off);
  float* yh = feat + (size_t)nb * NF;
  hipMemcpyAsync(p, b64.data(), b64.size() * 8, hipMemcpyHostToDevice, c->stream);
  hipLaunchKernelGGL(k_mlp_features, dim3(nb), dim3(256), 0, c->stream, K, d, gam, mu, (const int64_t*)p, nb, feat);
  hipLaunchKernelGGL(k_mlp_infer, dim3((nb + 255) / 256), dim3(256), 0, c->stream, c->mlp->theta, nb, feat, yh);
  std::vector<float> h(nb);
  hipMemcpyAsync(h.data(), yh, nb * 4, hipMemcpyDeviceToHost, c->stream);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return r_bound;
  float mx = -INFINITY;
  for (float v : h) mx = std::max(mx, v);
  if (!std::isfinite(mx)) return r_bound;
  const double r = std::ceil(RANK_SCALE * std::exp2(std::min(mx, 7.0f))) + RANK_MARGIN;
  return std::max(RANK_FLOOR, std::min(o.r_cap, (int)r));
}

// Collection: features and observed boundary ranks of one HSS merge.
adc_status mlp_collect_merge(adc_ctx c, const double* d, const double* gam, const double* mu, int K,
                             const std::vector<int>& bounds, const std::vector<int>& lo, const std::vector<int>& hi,
                             const std::vector<int>& kr, const std::vector<int>& kc) {
  MlpState* s = c->mlp;
  if (!s || !s->collect) return ADC_OK;
  const int nb = (int)bounds.size() - 2;
  if (nb <= 0 || s->rows + nb > s->cap) return ADC_OK;
  std::vector<int64_t> b64(bounds.begin(), bounds.end());
  ADC_TRY(launch_features(c, K, d, gam, mu, b64, s->cX + s->rows * NF));
  std::vector<float> t(nb);
  for (int b = 0; b < nb; ++b) {
    const int p = bounds[b + 1];
    int r = 1;
    for (size_t i = 1; i < lo.size(); ++i)
      if (lo[i] == p || hi[i] == p) r = std::max({r, kr[i], kc[i]});
    t[b] = (float)std::log2((double)r);
  }
  HIP_OK(hipMemcpyAsync(s->cy + s->rows, t.data(), nb * 4, hipMemcpyHostToDevice, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  s->rows += nb;
  return ADC_OK;
}

bool mlp_collecting(adc_ctx c) { return c->mlp && c->mlp->collect; }

extern "C" {

adc_status adc_mlp_features(adc_ctx c, int64_t K, const double* d, const double* gam, const double* mu,
                            const int64_t* bounds, int32_t nb, float* feat) {
  if (!c || K < 2 || K > INT32_MAX || !d || !gam || !mu || !bounds || nb < 0 || (nb > 0 && !feat))
    return ADC_ERR_ARG;
  if (bounds[0] != 0 || bounds[nb + 1] != K) return ADC_ERR_ARG;
  for (int b = 0; b <= nb; ++b)
    if (bounds[b + 1] <= bounds[b]) return ADC_ERR_ARG;
  DeviceGuard g(c->device);
  std::vector<int64_t> b64(bounds, bounds + nb + 2);
  return launch_features(c, (int)K, d, gam, mu, b64, feat);
}

adc_status adc_mlp_init(adc_ctx c, uint64_t seed) {
  if (!c) return ADC_ERR_ARG;
  DeviceGuard g(c->device);
  MlpState* s;
  ADC_TRY(mlp_state(c, &s));
  // uniform fan-in initialisation, biases zero; Adam moments cleared
  std::vector<float> h(3 * (size_t)NP, 0.0f);
  std::mt19937_64 gen(seed);
  auto fill = [&](int off, int n, int fan_in) {
    const float a = std::sqrt(6.0f / (float)fan_in);
    std::uniform_real_distribution<float> U(-a, a);
    for (int i = 0; i < n; ++i) h[off + i] = U(gen);
  };
  fill(OW1, NH * NF, NF);
  fill(OW2, NH * NH, NH);
  fill(OW3, NH, NH);
  HIP_OK(hipMemcpyAsync(s->theta, h.data(), h.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  s->t = 0;
  s->ready = true;
  return ADC_OK;
}

adc_status adc_mlp_train(adc_ctx c, int32_t B, const float* X, const float* y, int32_t epochs, int32_t batch,
                         float lr, float* loss_out) {
  if (!c || B <= 0 || !X || !y || epochs < 0 || batch <= 0 || !(lr > 0.0f)) return ADC_ERR_ARG;
  if (!c->mlp || !c->mlp->ready) return ADC_ERR_ARG;
  DeviceGuard g(c->device);
  MlpState* s = c->mlp;
  if (epochs == 0) return ADC_OK;
  ADC_TRY(launch_train(c, s, B, X, y, epochs, batch, lr, 0, nullptr));
  float l = 0.0f;
  HIP_OK(hipMemcpyAsync(&l, s->loss, 4, hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  s->t += (int64_t)epochs * ((B + batch - 1) / batch);
  if (loss_out) *loss_out = l;
  return ADC_OK;
}

adc_status adc_mlp_infer(adc_ctx c, int32_t B, const float* X, float* y) {
  if (!c || B < 0 || (B > 0 && (!X || !y))) return ADC_ERR_ARG;
  if (!c->mlp || !c->mlp->ready) return ADC_ERR_ARG;
  if (B == 0) return ADC_OK;
  DeviceGuard g(c->device);
  hipLaunchKernelGGL(k_mlp_infer, dim3((B + 255) / 256), dim3(256), 0, c->stream, c->mlp->theta, B, X, y);
  HIP_OK(hipGetLastError());
  return ADC_OK;
}

adc_status adc_mlp_grad(adc_ctx c, int32_t B, const float* X, const float* y, float* g_out, float* loss_out) {
  if (!c || B <= 0 || !X || !y || !g_out) return ADC_ERR_ARG;
  if (!c->mlp || !c->mlp->ready) return ADC_ERR_ARG;
  DeviceGuard g(c->device);
  MlpState* s = c->mlp;
  ADC_TRY(launch_train(c, s, B, X, y, 1, B, 1.0f, 1, g_out));
  float l = 0.0f;
  HIP_OK(hipMemcpyAsync(&l, s->loss, 4, hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  if (loss_out) *loss_out = l;
  return ADC_OK;
}

adc_status adc_mlp_get(adc_ctx c, float* params) {
  if (!c || !params || !c->mlp || !c->mlp->ready) return ADC_ERR_ARG;
  DeviceGuard g(c->device);
  HIP_OK(hipMemcpyAsync(params, c->mlp->theta, NP * 4, hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  return ADC_OK;
}

adc_status adc_mlp_set(adc_ctx c, const float* params) {
  if (!c || !params) return ADC_ERR_ARG;
  DeviceGuard g(c->device);
  MlpState* s;
  ADC_TRY(mlp_state(c, &s));
  HIP_OK(hipMemcpyAsync(s->theta, params, NP * 4, hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(hipMemsetAsync(s->m, 0, 2 * (size_t)NP * 4, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  s->t = 0;
  s->ready = true;
  return ADC_OK;
}

adc_status adc_mlp_collect(adc_ctx c, int64_t n, const double* diag, const double* offdiag, double* w, double* Z,
                           int64_t ldz, const adc_opts* opts, int64_t max_rows, float* X, float* y,
                           int64_t* rows_out) {
  if (!c || max_rows < 0 || (max_rows > 0 && (!X || !y)) || !rows_out) return ADC_ERR_ARG;
  DeviceGuard g(c->device);
  MlpState* s;
  ADC_TRY(mlp_state(c, &s));
  adc_opts o;
  if (opts) o = *opts; else adc_opts_default(&o);
  o.rank_mode = ADC_RANK_BOUND;
  s->collect = true;
  s->cX = X;
  s->cy = y;
  s->cap = max_rows;
  s->rows = 0;
  const adc_status st = adc_stedc(c, n, diag, offdiag, w, Z, ldz, nullptr, 0, &o, nullptr);
  s->collect = false;
  *rows_out = s->rows;
  return st;
}

}  // extern "C"
