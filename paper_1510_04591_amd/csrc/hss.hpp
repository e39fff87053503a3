// Randomized HSS approximation of the Cauchy-like eigenvector matrix
// (Algorithm 2) and its product from the right (Algorithm 3) on gfx950.
#pragma once
#include <functional>

#include "adc_internal.hpp"

// One HSS tree node (heap numbering inside its merge: root 0, children of p
// at 2p+1 and 2p+2; level l holds nodes 2^l - 1 .. 2^(l+1) - 2).
struct HssNode {
  int32_t lo, hi;      // index range t_i in [0, K)
  int32_t leaf;        // 1 for a leaf
  int32_t kr, kc;      // row / column ranks (written by the compression)
  int32_t nr, nc;      // candidate rows / columns of the IDs (written)
  int64_t offU, offV;  // U_i (nr x kr) and V_i (nc x kc), column-major, in the arena
  int64_t offB;        // B_i = A(skel_r(i), skel_c(sibling)), kr x kc(sib), column-major
  int64_t offSr, offSc;  // skeleton index lists (int32) in the index arena
  int64_t offPs, offTs;  // Phi_i|skel (kr x s) and Theta_i|skel (kc x s), row-major
  int64_t offYh, offZh;  // Yhat_i (kc x s) and Zhat_i (kr x s), row-major
  int64_t offWork;     // scratch: the node's Phi_i / Theta_i before the ID (cand x s)
};

// One HSS merge on the device.
struct HssMerge {
  int32_t K, s, sp;    // size, samples, padded sample count (multiple of 32)
  int32_t L;           // levels below the root
  const double* d;     // generators (length K)
  const double* gam;
  const double* mu;
  const double* uh;
  const double* v;
  const int32_t* leafof;  // leaf number of every index
  const int32_t* bounds;  // leaf boundaries (2^L + 1)
  double* omega;       // K x sp Gaussian, row-major
  double* phi;         // K x sp leaf row samples, row-major
  double* theta;       // K x sp leaf column samples, row-major
  HssNode* nodes;      // 2^(L+1) - 1 nodes
  const int32_t* perm; // packed column -> index (leaf-grouped operand of the
                       // solver's Algorithm 3), or null
  double* arena;       // generator and work storage
  int32_t* iarena;     // skeleton index storage
  double id_tol;
};

// Host-side view of a built HSS matrix (adc_hss handle).
struct adc_hss_s {
  adc_ctx ctx = nullptr;
  int K = 0, L = 0, s = 0, retries = 0, max_rank = 0;
  double check_err = 0.0;
  bool dense_fallback = false;
  std::vector<HssNode> nodes;       // host copy (ranks, offsets)
  void* mem = nullptr;              // device allocation owning everything below
  HssMerge dev{};                   // device pointers
  HssMerge* d_merge = nullptr;      // device copy of dev
  double* gen = nullptr;            // generator copies (d, gam, mu, uh, v)
  std::vector<int> bounds;          // leaf boundaries
};

// kernels
__global__ void k_philox_normal(double* __restrict__ out, int64_t K, int s, int sp, uint64_t seed,
                                uint32_t stream);
struct SampleJob {
  int32_t merge;
  int32_t r0;     // first output row
  int32_t c0;     // first sample column (multiple of 128)
  int32_t trans;  // 0: rows of Q' (Y = Q' Omega), 1: columns (Z = Q'^T Omega)
  int32_t seg;    // segment of the inner dimension
  int32_t nseg;   // segments; > 1: partial sums go to part + pbase
  int64_t pbase;  // element offset of this (merge, trans, seg) partial block
};
__global__ void k_hss_sample(const HssMerge* __restrict__ ms, const SampleJob* __restrict__ jobs, int exclude_diag,
                             double* __restrict__ part);
__global__ void k_sample_sum(const double* __restrict__ part, int nseg, int64_t n, double* __restrict__ out);
struct NodeJob {
  int32_t merge;
  int32_t node;  // heap index
  int32_t side;  // compression: 0 row ID (U, Zhat), 1 column ID (V, Yhat)
  int32_t pad;
};
__global__ void k_hss_bblocks(const HssMerge* __restrict__ ms, const NodeJob* __restrict__ jobs);
__global__ void k_hss_compress(const HssMerge* __restrict__ ms, const NodeJob* __restrict__ jobs, int lds_doubles);
// NCP: probe columns per launch held in registers (4 or 8, nc <= NCP)
template <int NCP>
__global__ void k_probe_qt(const HssMerge* __restrict__ ms, int g, const double* __restrict__ W, int ldw, int c0,
                           int nc, int nseg, double* __restrict__ part);
__global__ void k_probe_sum(const double* __restrict__ part, int K, int nseg, int c0, int nc, int ntot,
                            double* __restrict__ out, int ldo);
__global__ void k_hss_dmat(const HssMerge* __restrict__ ms, const int2* __restrict__ leafjobs,
                           double* __restrict__ dmat, const int64_t* __restrict__ doff, int grouped);
__global__ void k_hss_urows(const HssMerge* __restrict__ ms, const int2* __restrict__ leafjobs,
                            double* __restrict__ out, const int64_t* __restrict__ uoff);
__global__ void k_diff_norms(const double* __restrict__ a, const double* __restrict__ b, int64_t K, int ld, int nc,
                             double* __restrict__ part);
__global__ void k_sum_pairs(const double* __restrict__ part, int nblk, double* __restrict__ out2);

// Fast sampling (one-dimensional Chebyshev FMM over the HSS tree)
struct FmmJob {
  int32_t merge;
  int32_t node;  // heap index
  int32_t side;  // 0: Phi (targets d, sources lam), 1: Theta (targets lam, sources d)
  int32_t c0;    // first sample column of the job's 32-column chunk
  int32_t loff;  // offset of the node's far (M2L) or near (leaf) list
  int32_t lcnt;  // its length
};
// Operands of one merge's fast product: omega (K x sp row-major) in, out[side]
// (K x sp row-major) written; coefficient storage at off.
struct FmmIo {
  const double* omega;
  double* out[2];
  int64_t off;
  int32_t sp;
  int32_t pad;
};
__global__ void k_fmm_p2m(const HssMerge* __restrict__ ms, const FmmJob* __restrict__ jobs,
                          const FmmIo* __restrict__ io, int P, double* __restrict__ W);
__global__ void k_fmm_m2m(const HssMerge* __restrict__ ms, const FmmJob* __restrict__ jobs,
                          const FmmIo* __restrict__ io, int P, double* __restrict__ W);
__global__ void k_fmm_m2l(const HssMerge* __restrict__ ms, const FmmJob* __restrict__ jobs,
                          const int32_t* __restrict__ lists, const FmmIo* __restrict__ io, int P,
                          const double* __restrict__ W, double* __restrict__ F);
__global__ void k_fmm_l2l(const HssMerge* __restrict__ ms, const FmmJob* __restrict__ jobs,
                          const FmmIo* __restrict__ io, int P, double* __restrict__ F);
__global__ void k_fmm_leaf(const HssMerge* __restrict__ ms, const FmmJob* __restrict__ jobs,
                           const int32_t* __restrict__ lists, const FmmIo* __restrict__ io, int P,
                           const double* __restrict__ F);
void fmm_lists(const double* d, const double* gam, const double* mu, const std::vector<HssNode>& nodes,
               std::vector<std::vector<int32_t>>& far, std::vector<std::vector<int32_t>>& near);

// Leaf boundaries of the HSS tree over K indices with leaves of at most
// `leaf` rows: L = ceil(log2(K / leaf)) levels (at least one), balanced.
std::vector<int> hss_leaf_bounds(int K, int leaf);

// HSS update of the level's HSS merges.  `after_sampling` (may be empty) is
// called once the first sampling pass is queued; the packed operand is ready
// once `operand_ready` (may be null) has completed.
adc_status hss_level_update(adc_ctx c, const adc_opts& o, MergeDev* h_m, MergeDev* d_m, int nm,
                            const LevelBufs& B, int depth, adc_report* rep, double* flops, double* bytes,
                            const std::function<void()>& after_sampling, hipEvent_t operand_ready);
