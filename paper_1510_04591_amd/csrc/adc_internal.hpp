// Host-side internals of the ADC library.
#pragma once
#include <vector>

#include "kernels.hpp"

enum Slot {
  SLOT_WS = 0,     // solver workspace (vectors, second eigenvector buffer, operands)
  SLOT_DESC,       // per-level descriptors
  SLOT_FLAG,       // small flags
  SLOT_QC,         // standalone Cauchy matrix
  SLOT_HSS,        // HSS workspace of the solver
  SLOT_HSS2,       // HSS work arrays of the solver (second arena)
  SLOT_HSS_RETRY,  // HSS workspace of the merges rebuilt with more samples
  SLOT_FMM,        // fast-sampling coefficients (multipole and local)
  SLOT_SAMPLE_JOBS, // sampling launch lists (direct or fast)
  SLOT_BATCH,      // batched solver workspace
  SLOT_BATCH_DESC, // batched solver descriptors
  SLOT_MLP,        // MLP scratch
  SLOT_HSS_JOBS,   // HSS launch lists
  SLOT_HSS_CHECK,  // HSS accuracy-check probes
  SLOT_GEMM_A,     // grouped GEMM descriptors (narrow tiles)
  SLOT_GEMM_B,     // grouped GEMM descriptors (wide tiles)
  SLOT_FB,         // dense-fallback descriptors
  SLOT_RANK,       // one-merge rank-estimate descriptor
  NSLOT
};

struct MlpState;

// Phase timing with HIP events on the context stream: start() opens an
// interval, mark(p) closes it as phase p and opens the next; collect() (after
// a stream synchronisation) adds the closed intervals to the report.  A
// start() before the previous intervals were collected keeps them: the time
// from their last mark to the new start is not attributed to any phase.
struct PhaseTimer {
  std::vector<hipEvent_t> ev;
  std::vector<int> phase;
  size_t n = 0;
  bool on = false;
  void record(hipStream_t s, int p) {
    if (n == ev.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        on = false;
        return;
      }
      ev.push_back(e);
      phase.push_back(-1);
    }
    hipEventRecord(ev[n], s);
    phase[n] = p;
    ++n;
  }
  void reset() { n = 0; }
  void start(hipStream_t s, bool enable) {
    on = enable;
    if (!on) {
      n = 0;
      return;
    }
    record(s, -1);
  }
  void mark(hipStream_t s, int p) {
    if (on) record(s, p);
  }
  void collect(adc_report* rep) {
    if (on && rep)
      for (size_t i = 1; i < n; ++i) {
        float ms = 0.f;
        if (phase[i] >= 0 && hipEventElapsedTime(&ms, ev[i - 1], ev[i]) == hipSuccess)
          rep->t_phase[phase[i]] += 1e-3 * ms;
      }
    n = 0;
  }
  void destroy() {
    for (auto e : ev) hipEventDestroy(e);
    ev.clear();
    phase.clear();
    n = 0;
  }
};

// Per-launch timing of selected kernels: an event pair around each launch,
// resolved after the stream has been synchronised.
enum KernId {
  KT_GEMM = 0,
  KT_GEMM64 = 1,
  KT_SAMPLE = 2,
  KT_PACK = 3,
  KT_SECULAR = 4,
  KT_COMPRESS = 5,
  KT_GEMMBIG = 6,
  KT_GEMM96 = 7,
  KT_FMMLEAF = 8,
  KT_FMMM2L = 9
};
struct KernTimer {
  std::vector<hipEvent_t> ev;
  std::vector<int> kid;
  std::vector<double> fl, by;
  bool on = false;
  void begin(bool enable) {
    on = enable;
    kid.clear();
    fl.clear();
    by.clear();
  }
  void pre(hipStream_t s) {
    if (!on) return;
    const size_t i = kid.size();
    while (ev.size() < 2 * i + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        on = false;
        return;
      }
      ev.push_back(e);
    }
    hipEventRecord(ev[2 * i], s);
  }
  void post(hipStream_t s, int k, double flops, double bytes) {
    if (!on) return;
    const size_t i = kid.size();
    hipEventRecord(ev[2 * i + 1], s);
    kid.push_back(k);
    fl.push_back(flops);
    by.push_back(bytes);
  }
  // index of the last recorded launch, and its work figures set afterwards
  // (launches sized on the device, whose work is known once read back)
  size_t last() const { return kid.empty() ? 0 : kid.size() - 1; }
  void set_work(size_t i, double flops, double bytes) {
    if (!on || i >= kid.size()) return;
    fl[i] = flops;
    by[i] = bytes;
  }
  // the stream must have been synchronised
  void collect(adc_report* rep) {
    if (!on) return;
    for (size_t i = 0; i < kid.size(); ++i) {
      float ms = 0.f;
      if (rep && hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess) {
        rep->kern_time[kid[i]] += 1e-3 * ms;
        rep->kern_flops[kid[i]] += fl[i];
        rep->kern_bytes[kid[i]] += by[i];
        rep->kern_launches[kid[i]] += 1;
      }
    }
    kid.clear();
    fl.clear();
    by.clear();
  }
  void destroy() {
    for (auto e : ev) hipEventDestroy(e);
    ev.clear();
  }
};

struct adc_ctx_s {
  struct Buf {
    void* ptr = nullptr;
    size_t bytes = 0;
  };
  int device = 0;
  int num_cu = 256;  // compute units of the device
  hipStream_t stream = nullptr;
  Buf bufs[NSLOT];
  void* host_stage = nullptr;
  size_t host_stage_bytes = 0;
  void* host_stage2 = nullptr;  // pinned staging of GEMM problem lists
  size_t host_stage2_bytes = 0;
  // pinned bump arena for small host-to-device uploads on `stream` (launch
  // lists, node tables): a copy from pageable memory blocks the host, one
  // from pinned memory is queued.  Regions are not reused until up_reset,
  // which callers invoke only right after synchronising `stream`.
  char* host_up = nullptr;
  size_t host_up_bytes = 0, host_up_used = 0;
  MlpState* mlp = nullptr;
  void* batch_cache = nullptr;  // graph cache of the batched solver
  void* noalloc_scratch = nullptr;  // device address of the static scratch on `device`
  PhaseTimer timer;
  KernTimer ktimer;
  // second stream (default priority) for work that overlaps the HSS
  // construction inside one level; joined back before the level ends
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_probe = nullptr;
  adc_status side_stream();
  // event after a level's merge descriptors are copied back (the host waits
  // on it while the roots of the level are computed)
  hipEvent_t ev_meta = nullptr;
  adc_status meta_event(hipEvent_t* e);
  adc_status buffer(int slot, size_t bytes, void** p);
  adc_status stage(size_t bytes, void** p);
  adc_status stage2(size_t bytes, void** p);
  adc_status upload(void* dst, const void* src, size_t bytes);  // queued on `stream`
  void up_reset() { host_up_used = 0; }
  void release();
};

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
  }
};

// bump allocator over one device region
struct Arena {
  char* base = nullptr;
  size_t off = 0;
  size_t cap = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
};

adc_status check_finite(adc_ctx c, const double* x, int64_t n, bool* ok);
int pick_waves(int64_t K);
// Several matrices (count, arrays indexed by matrix) in one level-batched
// solve with the HSS route where it applies; dc.hip.
adc_status stedc_forest(adc_ctx c, int count, const int64_t* n, const double* const* diag,
                        const double* const* offdiag, double* const* w, double* const* Z, const int64_t* ldz,
                        const adc_opts& o, adc_report* rep);
void mlp_release(adc_ctx c);
void batch_release(adc_ctx c);

__global__ void k_check_finite(const double* __restrict__ x, int64_t n, int* __restrict__ flag);
__global__ void k_set_int(int* p, int v);
__global__ void k_tear(const double* __restrict__ diag, const double* __restrict__ off,
                       const int64_t* __restrict__ splits, int nsplit, double* __restrict__ a, int64_t n);
adc_status validate_opts_ext(const adc_opts& o);

// Dense Cauchy update of merge g whose survivor columns were packed in pole
// order (the fallback of a failed HSS check).
adc_status dense_sorted_update(adc_ctx c, const MergeDev* d_m, int g, const MergeDev& M, const LevelBufs& B,
                               double* flops);
// HSS sample rank from the learned predictor (r_bound when no model is
// loaded); d, gam, mu are device arrays of the merge.
int mlp_rank(adc_ctx c, const double* d, const double* gam, const double* mu, int K, const std::vector<int>& bounds,
             const adc_opts& o, int r_bound);
// Collection mode of adc_mlp_collect: features and observed boundary ranks
// of one HSS merge (device generators, host node table).
bool mlp_collecting(adc_ctx c);
adc_status mlp_collect_merge(adc_ctx c, const double* d, const double* gam, const double* mu, int K,
                             const std::vector<int>& bounds, const std::vector<int>& lo, const std::vector<int>& hi,
                             const std::vector<int>& kr, const std::vector<int>& kc);
// Rank estimate of eq. (bounds) over the leaf boundaries of one merge
// (device generators), moving boundaries closer than shift_thresh: `bounds`
// in balanced, out moved.
adc_status device_rank_estimate(adc_ctx c, const double* d, const double* gam, const double* mu, int K,
                                std::vector<int>& bounds, const adc_opts& o, int* r);
