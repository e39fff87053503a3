// Host driver of the ADC library: context, memory pool, the DC tree
// (Algorithm 1) and the kernel-level entry points of the C ABI.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "adc_internal.hpp"

// ---------------------------------------------------------------- static scratch
// Scratch of adc_cauchy_gemm_noalloc: the explicit Cauchy-like matrix
// (K x K, K <= NOALLOC_KMAX) followed by its launch descriptors.  One copy
// per GPU, held while the library is loaded.  Host code never passes the
// array's name to a kernel or a copy: it uses the device address taken once
// per device by hipGetSymbolAddress (noalloc_scratch_init).
namespace {
constexpr int64_t NOALLOC_KMAX = 2048;
constexpr size_t NOALLOC_QBYTES = (size_t)NOALLOC_KMAX * NOALLOC_KMAX * sizeof(double);
constexpr size_t NOALLOC_DBYTES = 64 * 1024;
constexpr size_t NOALLOC_BYTES = NOALLOC_QBYTES + NOALLOC_DBYTES;
constexpr int NOALLOC_MAXDEV = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAXDEV] = {};
bool g_noalloc_tried[NOALLOC_MAXDEV] = {};
}  // namespace

__device__ __align__(256) char scratch[NOALLOC_BYTES];

// Device address of `scratch` on the current device `device` (taken once).
static void* noalloc_scratch_init(int device) {
  if (device < 0 || device >= NOALLOC_MAXDEV) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_tried[device]) {
    g_noalloc_tried[device] = true;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_noalloc_ptr[device] = ptr;
    else (void)hipGetLastError();
  }
  return g_noalloc_ptr[device];
}

// ---------------------------------------------------------------- status
extern "C" const char* adc_status_string(adc_status s) {
  switch (s) {
    case ADC_OK: return "ADC_OK";
    case ADC_ERR_ARG: return "ADC_ERR_ARG: invalid argument or non-finite input";
    case ADC_ERR_NOMEM: return "ADC_ERR_NOMEM: device allocation failed";
    case ADC_ERR_HIP: return "ADC_ERR_HIP: HIP runtime error";
    case ADC_ERR_NOCONV: return "ADC_ERR_NOCONV: secular root did not converge";
    case ADC_ERR_ACCURACY: return "ADC_ERR_ACCURACY: HSS accuracy check failed";
    case ADC_ERR_UNSUPPORTED: return "ADC_ERR_UNSUPPORTED: size or option not supported";
  }
  return "ADC_UNKNOWN";
}

extern "C" adc_status adc_opts_default(adc_opts* o) {
  if (!o) return ADC_ERR_ARG;
  std::memset(o, 0, sizeof(*o));
  o->dc_leaf = 32;
  o->hss_min_k = 2048;
  o->hss_levels = -1;
  o->hss_leaf = 128;
  o->id_tol = 1e-14;
  o->oversample = 16;
  o->rank_mode = ADC_RANK_BOUND;
  o->fixed_rank = 0;
  o->max_retries = 2;
  o->max_iter = 60;
  o->seed = 20151015ull;
  o->force_dense = 0;
  o->strict = 0;
  o->check_tol = 1e-13;
  o->nprobe = 4;
  o->shift_max = 5;
  o->shift_thresh = 1e-10;
  o->r_cap = 100;
  o->rank_eps = 1e-16;
  o->hss_min_flops = 2.5e10;
  o->sample_mode = ADC_SAMPLE_FMM;
  o->fmm_order = 20;
  o->sat_guard = 0;
  o->batch_bytes = 0.0;
  return ADC_OK;
}

adc_status validate_opts_ext(const adc_opts& o) {
  if (o.dc_leaf < 2 || o.dc_leaf > 64) return ADC_ERR_ARG;
  if (o.hss_leaf < 16 || o.hss_leaf > 256) return ADC_ERR_ARG;
  if (!(o.id_tol >= 0.0) || o.oversample < 0 || o.max_retries < 0 || o.max_iter < 1) return ADC_ERR_ARG;
  if (o.nprobe < 1 || o.nprobe > 32 || o.r_cap < 1 || !(o.rank_eps > 0.0) ||
      !(o.hss_min_flops >= 0.0))
    return ADC_ERR_ARG;
  if (o.sample_mode < 0 || o.sample_mode > 1 || o.fmm_order < 4 || o.fmm_order > 32) return ADC_ERR_ARG;
  if (o.shift_max < 0 || o.shift_max > 64) return ADC_ERR_ARG;
  if (o.rank_mode < 0 || o.rank_mode > 2) return ADC_ERR_ARG;
  if (o.sat_guard < 0 || o.sat_guard > 1) return ADC_ERR_ARG;
  if (!(o.batch_bytes >= 0.0) || !std::isfinite(o.batch_bytes)) return ADC_ERR_ARG;
  return ADC_OK;
}

// ---------------------------------------------------------------- context
extern "C" adc_status adc_create(adc_ctx* out, int device, void* stream) {
  if (!out) return ADC_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  HIP_OK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return ADC_ERR_ARG;
  adc_ctx c = new (std::nothrow) adc_ctx_s();
  if (!c) return ADC_ERR_NOMEM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
      c->num_cu = ncu;
  }
  {
    DeviceGuard g(device);
    c->noalloc_scratch = noalloc_scratch_init(device);  // null: the no-alloc entry reports ADC_ERR_HIP
    leaf_init();
  }
  *out = c;
  return ADC_OK;
}

extern "C" adc_status adc_destroy(adc_ctx c) {
  if (!c) return ADC_ERR_ARG;
  DeviceGuard g(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  else hipDeviceSynchronize();
  c->release();
  delete c;
  return ADC_OK;
}

adc_status adc_ctx_s::side_stream() {
  if (side) return ADC_OK;
  if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess) {
    side = nullptr;
    return ADC_ERR_HIP;
  }
  if (hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ev_probe, hipEventDisableTiming) != hipSuccess)
    return ADC_ERR_HIP;
  return ADC_OK;
}

adc_status adc_ctx_s::meta_event(hipEvent_t* e) {
  if (!ev_meta && hipEventCreateWithFlags(&ev_meta, hipEventDisableTiming) != hipSuccess) {
    ev_meta = nullptr;
    return ADC_ERR_HIP;
  }
  *e = ev_meta;
  return ADC_OK;
}

void adc_ctx_s::release() {
  if (side) {
    hipStreamSynchronize(side);
    hipStreamDestroy(side);
    side = nullptr;
  }
  if (ev_fork) hipEventDestroy(ev_fork);
  if (ev_join) hipEventDestroy(ev_join);
  if (ev_probe) hipEventDestroy(ev_probe);
  if (ev_meta) hipEventDestroy(ev_meta);
  ev_fork = ev_join = ev_probe = ev_meta = nullptr;
  for (auto& b : bufs) {
    if (b.ptr) hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
  }
  if (host_stage) hipHostFree(host_stage);
  host_stage = nullptr;
  host_stage_bytes = 0;
  if (host_stage2) hipHostFree(host_stage2);
  host_stage2 = nullptr;
  if (host_up) hipHostFree(host_up);
  host_up = nullptr;
  host_up_bytes = host_up_used = 0;
  host_stage2_bytes = 0;
  timer.destroy();
  ktimer.destroy();
  mlp_release(this);
  batch_release(this);
}

adc_status adc_ctx_s::buffer(int slot, size_t bytes, void** p) {
  if (slot < 0 || slot >= NSLOT) return ADC_ERR_ARG;
  Buf& b = bufs[slot];
  if (b.bytes < bytes) {
    if (b.ptr) {
      hipStreamSynchronize(stream);
      hipFree(b.ptr);
    }
    b.ptr = nullptr;
    b.bytes = 0;
    size_t want = std::max(bytes, (size_t)256);
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
      b.ptr = nullptr;
      return ADC_ERR_NOMEM;
    }
    b.bytes = want;
  }
  *p = b.ptr;
  return ADC_OK;
}

adc_status adc_ctx_s::stage(size_t bytes, void** p) {
  if (host_stage_bytes < bytes) {
    if (host_stage) {
      hipStreamSynchronize(stream);
      hipHostFree(host_stage);
    }
    host_stage = nullptr;
    host_stage_bytes = 0;
    size_t want = std::max(bytes, (size_t)(1 << 20));
    if (hipHostMalloc(&host_stage, want, hipHostMallocDefault) != hipSuccess) return ADC_ERR_NOMEM;
    host_stage_bytes = want;
  }
  *p = host_stage;
  return ADC_OK;
}

adc_status adc_ctx_s::upload(void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return ADC_OK;
  const size_t need = (bytes + 255) & ~(size_t)255;
  if (host_up_used + need > host_up_bytes) {
    // the regions handed out so far may still be read by queued copies:
    // wait for them, then grow
    HIP_OK(hipStreamSynchronize(stream));
    host_up_used = 0;
    if (need > host_up_bytes) {
      if (host_up) hipHostFree(host_up);
      host_up = nullptr;
      host_up_bytes = 0;
      const size_t want = std::max(need, (size_t)(16 << 20));
      if (hipHostMalloc((void**)&host_up, want, hipHostMallocDefault) != hipSuccess) return ADC_ERR_NOMEM;
      host_up_bytes = want;
    }
  }
  char* h = host_up + host_up_used;
  std::memcpy(h, src, bytes);
  host_up_used += need;
  HIP_OK(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, stream));
  return ADC_OK;
}

adc_status adc_ctx_s::stage2(size_t bytes, void** p) {
  if (host_stage2_bytes < bytes) {
    if (host_stage2) {
      hipStreamSynchronize(stream);
      hipHostFree(host_stage2);
    }
    host_stage2 = nullptr;
    host_stage2_bytes = 0;
    size_t want = std::max(bytes, (size_t)(1 << 20));
    if (hipHostMalloc(&host_stage2, want, hipHostMallocDefault) != hipSuccess) return ADC_ERR_NOMEM;
    host_stage2_bytes = want;
  }
  *p = host_stage2;
  return ADC_OK;
}

// ---------------------------------------------------------------- helpers
adc_status check_finite(adc_ctx c, const double* x, int64_t n, bool* ok) {
  int* flag;
  ADC_TRY(c->buffer(SLOT_FLAG, 64, (void**)&flag));
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, c->stream, flag, 0);
  if (n > 0) {
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_check_finite, dim3(blocks), dim3(256), 0, c->stream, x, n, flag);
    HIP_OK(hipGetLastError());
  }
  int h = 0;
  HIP_OK(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  *ok = (h == 0);
  return ADC_OK;
}

int pick_waves(int64_t K) {
  if (K <= 128) return 1;
  if (K <= 1024) return 4;
  if (K <= 4096) return 8;
  return 16;
}

// ---------------------------------------------------------------- kernel-level entries
extern "C" adc_status adc_secular(adc_ctx c, int64_t K, const double* d, const double* z, double rho,
                                  double* lam, double* gam, double* mu) {
  if (!c || K < 0 || K > (int64_t)INT32_MAX / 2) return ADC_ERR_ARG;
  if (K == 0) return ADC_OK;
  if (!d || !z || !gam || !mu || !(rho > 0.0) || !std::isfinite(rho)) return ADC_ERR_ARG;
  DeviceGuard g(c->device);
  MergeDev md{};
  md.s0 = 0;
  md.gbase = 0;
  md.n = (int32_t)K;
  md.K = (int32_t)K;
  md.rho = rho;
  std::vector<RootBlock> rbs;
  for (int64_t i0 = 0; i0 < K; i0 += 64) rbs.push_back(RootBlock{0, (int32_t)i0});
  void* dev;
  const size_t need = sizeof(MergeDev) + rbs.size() * sizeof(RootBlock) + 64;
  ADC_TRY(c->buffer(SLOT_DESC, need, &dev));
  MergeDev* dm = (MergeDev*)dev;
  RootBlock* drb = (RootBlock*)((char*)dev + sizeof(MergeDev));
  HIP_OK(hipMemcpyAsync(dm, &md, sizeof(md), hipMemcpyHostToDevice, c->stream));
  HIP_OK(hipMemcpyAsync(drb, rbs.data(), rbs.size() * sizeof(RootBlock), hipMemcpyHostToDevice, c->stream));
  int* noconv;
  ADC_TRY(c->buffer(SLOT_FLAG, 64, (void**)&noconv));
  const int W = pick_waves(K);
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, c->stream, noconv, INT32_MAX);
  hipLaunchKernelGGL(k_secular, dim3((unsigned)rbs.size()), dim3(64 * W), 0, c->stream, dm, drb, d, z, lam, gam, mu,
                     60, noconv);
  HIP_OK(hipGetLastError());
  // the host-side structures above were copied from stack memory: wait
  HIP_OK(hipStreamSynchronize(c->stream));
  return ADC_OK;
}

extern "C" adc_status adc_lowner(adc_ctx c, int64_t K, const double* d, const double* z, double rho,
                                 const double* gam, const double* mu, double* uh, double* v) {
  if (!c || K < 0 || K > (int64_t)INT32_MAX / 2) return ADC_ERR_ARG;
  if (K == 0) return ADC_OK;
  if (!d || !z || !gam || !mu || !uh || !(rho > 0.0)) return ADC_ERR_ARG;
  DeviceGuard g(c->device);
  MergeDev md{};
  md.n = (int32_t)K;
  md.K = (int32_t)K;
  md.rho = rho;
  std::vector<RootBlock> rbs;
  for (int64_t i0 = 0; i0 < K; i0 += 64) rbs.push_back(RootBlock{0, (int32_t)i0});
  void* dev;
  ADC_TRY(c->buffer(SLOT_DESC, sizeof(MergeDev) + rbs.size() * sizeof(RootBlock) + 64, &dev));
  MergeDev* dm = (MergeDev*)dev;
  RootBlock* drb = (RootBlock*)((char*)dev + sizeof(MergeDev));
  HIP_OK(hipMemcpyAsync(dm, &md, sizeof(md), hipMemcpyHostToDevice, c->stream));
  HIP_OK(hipMemcpyAsync(drb, rbs.data(), rbs.size() * sizeof(RootBlock), hipMemcpyHostToDevice, c->stream));
  const int W = pick_waves(K);
  hipLaunchKernelGGL(k_lowner, dim3((unsigned)rbs.size()), dim3(64 * W), 0, c->stream, dm, drb, d, z, gam, mu, uh);
  if (v)
    hipLaunchKernelGGL(k_vnorm, dim3((unsigned)rbs.size()), dim3(64 * W), 0, c->stream, dm, drb, d, gam, mu, uh, v);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(c->stream));
  return ADC_OK;
}

extern "C" adc_status adc_cauchy_gemm(adc_ctx c, int64_t P, int64_t K, const double* d, const double* gam,
                                      const double* mu, const double* uh, const double* v, const double* X,
                                      int64_t ldx, double* Y, int64_t ldy) {
  if (!c || P < 0 || K < 0 || K > 65536 || P > (int64_t)INT32_MAX) return ADC_ERR_ARG;
  if (P == 0 || K == 0) return ADC_OK;
  if (!d || !gam || !mu || !uh || !v || !X || !Y || ldx < P || ldy < P) return ADC_ERR_ARG;
  DeviceGuard g(c->device);
  double* qc;
  ADC_TRY(c->buffer(SLOT_QC, (size_t)K * K * sizeof(double), (void**)&qc));
  MergeDev md{};
  md.n = (int32_t)K;
  md.K = (int32_t)K;
  md.zoff = 0;
  LevelBufs B{};
  B.dS = const_cast<double*>(d);
  B.gam = const_cast<double*>(gam);
  B.mu = const_cast<double*>(mu);
  B.uh = const_cast<double*>(uh);
  B.qc = qc;
  const int ncols = 8;
  std::vector<int32_t> tm, tc;
  for (int64_t j0 = 0; j0 < K; j0 += ncols) {
    tm.push_back(0);
    tc.push_back((int32_t)j0);
  }
  GemmProb gp{};
  gp.A = X;
  gp.B = qc;
  gp.C = Y;
  gp.colmap = nullptr;
  gp.vscale = v;
  gp.lda = ldx;
  gp.ldb = K;
  gp.ldc = ldy;
  gp.M = (int32_t)P;
  gp.N = (int32_t)K;
  gp.K = (int32_t)K;
  gp.tile0 = 0;
  gp.tiles_m = (int32_t)((P + 255) / 256);
  const int tiles = gp.tiles_m * (int)((K + 127) / 128);
  void* dev;
  const size_t need = sizeof(MergeDev) + sizeof(GemmProb) + 2 * tm.size() * sizeof(int32_t) + 256;
  ADC_TRY(c->buffer(SLOT_DESC, need, &dev));
  char* p = (char*)dev;
  MergeDev* dm = (MergeDev*)p;
  p += sizeof(MergeDev);
  GemmProb* dg = (GemmProb*)p;
  p += sizeof(GemmProb);
  int32_t* dtm = (int32_t*)p;
  int32_t* dtc = dtm + tm.size();
  HIP_OK(hipMemcpyAsync(dm, &md, sizeof(md), hipMemcpyHostToDevice, c->stream));
  HIP_OK(hipMemcpyAsync(dg, &gp, sizeof(gp), hipMemcpyHostToDevice, c->stream));
  HIP_OK(hipMemcpyAsync(dtm, tm.data(), tm.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_OK(hipMemcpyAsync(dtc, tc.data(), tc.size() * 4, hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_cauchy, dim3((unsigned)tm.size()), dim3(256), 0, c->stream, dm, dtm, dtc, B, ncols, 0);
  hipLaunchKernelGGL(k_gemm_f64_big, dim3(tiles), dim3(1024), 0, c->stream, dg, 1, (const int*)nullptr);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(c->stream));
  return ADC_OK;
}

// Descriptors of the allocation-free Cauchy update, written on the device
// into the static scratch: the one-merge descriptor of k_cauchy, its column
// tiles of 8 and the GEMM problem.
__global__ void k_noalloc_desc(MergeDev* md, int32_t* tm, int32_t* tc, int ntile, GemmProb* gp, int64_t P,
                               int64_t K, double* qc, const double* X, int64_t ldx, double* Y, int64_t ldy,
                               const double* v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ntile) {
    tm[t] = 0;
    tc[t] = 8 * t;
  }
  if (t == 0) {
    MergeDev m{};
    m.n = (int32_t)K;
    m.K = (int32_t)K;
    m.zoff = 0;
    *md = m;
    GemmProb g{};
    g.A = X;
    g.B = qc;
    g.C = Y;
    g.colmap = nullptr;
    g.vscale = v;
    g.lda = ldx;
    g.ldb = K;
    g.ldc = ldy;
    g.M = (int32_t)P;
    g.N = (int32_t)K;
    g.K = (int32_t)K;
    g.tile0 = 0;
    g.tiles_m = (int32_t)((P + 255) / 256);
    *gp = g;
  }
}

extern "C" adc_status adc_cauchy_gemm_noalloc(adc_ctx c, int64_t P, int64_t K, const double* d,
                                              const double* gam, const double* mu, const double* uh,
                                              const double* v, const double* X, int64_t ldx, double* Y,
                                              int64_t ldy) {
  if (!c || P < 0 || K < 0 || P > (int64_t)INT32_MAX) return ADC_ERR_ARG;
  if (K > NOALLOC_KMAX) return ADC_ERR_UNSUPPORTED;
  if (P == 0 || K == 0) return ADC_OK;
  if (!d || !gam || !mu || !uh || !v || !X || !Y || ldx < P || ldy < P) return ADC_ERR_ARG;
  if (!c->noalloc_scratch) return ADC_ERR_HIP;
  DeviceGuard g(c->device);
  char* base = (char*)c->noalloc_scratch;
  double* qc = (double*)base;
  char* desc = base + NOALLOC_QBYTES;
  MergeDev* dm = (MergeDev*)desc;
  GemmProb* dg = (GemmProb*)(desc + 256);
  int32_t* dtm = (int32_t*)(desc + 1024);
  const int ntile = (int)((K + 7) / 8);
  int32_t* dtc = dtm + ntile;
  // 1024 + 2 * 4 * 256 bytes of descriptors at most, inside NOALLOC_DBYTES
  static_assert(1024 + 8 * ((NOALLOC_KMAX + 7) / 8) <= NOALLOC_DBYTES, "descriptor space");
  LevelBufs B{};
  B.dS = const_cast<double*>(d);
  B.gam = const_cast<double*>(gam);
  B.mu = const_cast<double*>(mu);
  B.uh = const_cast<double*>(uh);
  B.qc = qc;
  hipLaunchKernelGGL(k_noalloc_desc, dim3((unsigned)((ntile + 255) / 256)), dim3(256), 0, c->stream, dm, dtm, dtc,
                     ntile, dg, P, K, qc, X, ldx, Y, ldy, v);
  hipLaunchKernelGGL(k_cauchy, dim3((unsigned)ntile), dim3(256), 0, c->stream, (const MergeDev*)dm, dtm, dtc, B, 8,
                     0);
  const int tiles = (int)((P + 255) / 256) * (int)((K + 127) / 128);
  hipLaunchKernelGGL(k_gemm_f64_big, dim3(tiles), dim3(1024), 0, c->stream, (const GemmProb*)dg, 1,
                     (const int*)nullptr);
  HIP_OK(hipGetLastError());
  return ADC_OK;
}
