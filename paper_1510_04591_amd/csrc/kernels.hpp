// Device-side descriptors and kernel declarations of the ADC library.
#pragma once
#include "common.hpp"

// One merge of the DC tree (Algorithm 1).  Every per-merge vector lives at
// offset s0 of an N-long array, because the merges of one level partition
// [0, N).  Fields below "prep" are written by k_merge_prep.
struct MergeDev {
  int64_t s0;      // first row/column of the merge block (global)
  int64_t gbase;   // global index base used in error reports
  int64_t zoff;    // element offset of this merge's packed / Cauchy buffers
  int32_t n, n1;   // merge size and size of the first child
  double beta;     // off-diagonal entry b_k at the tear (eq. T2)
  // prep
  int32_t K;       // survivors of deflation (secular size)
  int32_t nrot;    // Givens rotations of type-2 deflation
  int32_t k1, k2, k3;  // survivors whose column lives in rows: top only, both, bottom only
  int32_t mode;    // 0 dense update, 1 HSS update (host decision)
  int32_t dsorted; // 1 when the deflated values are non-decreasing in scan order
  double rho;      // rho after normalising z
  double tol;      // deflation tolerance
  // eigenvector blocks: zo = the children's (block diagonal), zn = the merged
  // block; both point at the merge's (first row, first column) corner
  const double* zo;
  double* zn;
  int64_t ldo, ldn;
  // HSS merges: leaf boundaries of the HSS tree over the survivors (pole
  // order), nleaf + 1 entries, balanced then moved by k_leaf_bounds; the
  // packing groups each leaf's columns by row support (top only, both,
  // bottom only)
  int32_t* lbounds;
  int32_t nleaf;
  int32_t rest;    // rank estimate of eq. (bounds) over the moved boundaries (k_leaf_bounds)
};

// Output block of one leaf: z points at its (first row, first column) corner.
struct LeafOut {
  double* z;
  int64_t ld;
};

// 64 consecutive roots (columns) of one merge.
struct RootBlock {
  int32_t merge;
  int32_t i0;
};

// One product C(:, colmap[j]) = beta C(:, colmap[j]) + vscale[j] ([A A2] [B; B2])(:, j).
// Column-major; the inner dimension is K (first segment) + K2 (second, may be 0);
// a transposed B segment is read as B(k, n) = B[n + k ldb].
struct GemmProb {
  const double* A;
  const double* B;
  double* C;
  const double* A2;
  const double* B2;
  const int32_t* colmap;  // may be null (identity)
  const double* vscale;   // may be null (1)
  int64_t lda, ldb, ldc, lda2, ldb2;
  int32_t M, N, K, K2;
  int32_t transB, transB2;
  double beta;
  int32_t tile0;          // first flat tile index of this problem
  int32_t tiles_m;        // tiles along M
};

// Per-level scratch pointers shared by the merge kernels.
struct LevelBufs {
  const double* w_in;   // children's eigenvalues: w itself (only k_merge_sort reads it,
                        // before the level's k_final_order writes w_out = w)
  double* w_out;        // merged eigenvalues
  const double* off;    // off-diagonal of T (b_k of every tear)
  double* dsort;        // d after merging the two runs (and rotation updates)
  double* zsort;        // z likewise
  int32_t* src;         // sorted position -> block-local source column
  int32_t* supp;        // sorted position -> row support (1 top, 2 bottom, 3 both)
  int32_t* surv;        // survivor r -> sorted position
  int32_t* defl;        // deflated q -> sorted position
  int32_t* gorder;      // grouped order (dense GEMM) -> survivor r
  int32_t* rot_i;       // rotation t -> sorted positions (i, j)
  int32_t* rot_j;
  int32_t* rot_f;       // supports of i and j before the rotation: fi | fj << 2
  double* rot_c;
  double* rot_s;
  double* dS;           // survivor poles d'
  double* zS;           // survivor weights z'
  double* lam;          // roots
  double* gam;          // lam_i - d_i
  double* mu;           // d_{i+1} - lam_i
  double* uh;           // Loewner vector
  double* v;            // column scales
  int32_t* posR;        // survivor r -> final position in the block
  int32_t* posD;        // deflated q -> final position in the block
  double* pk;           // packed survivor columns of U
  double* qc;           // materialised Cauchy matrix (dense update)
  int32_t* pidx;        // sorted position -> survivor r (>= 0) or -1 - deflated q
  int32_t* ginv;        // survivor r -> packed column: the grouped order (dense
                        // update) or the leaf-grouped order (HSS update)
  int32_t* lcnt;        // HSS merges: per leaf the counts of top-only, both and
                        // bottom-only survivors (3 per leaf, at the merge's s0)
  int32_t* rot_i_of;    // sorted position -> rotation t with rot_i[t] = position, else -1
  int32_t* rot_j_of;    // sorted position -> rotation t with rot_j[t] = position, else -1
};

// ---- kernels
// leaf eigensolves (sizes <= leaf_max <= 64) into w and each leaf's block;
// leaf_init once per device (the LDS limit for 64-row leaves)
void leaf_init();
void launch_leaf_jacobi(hipStream_t st, int64_t nleaf, int leaf_max, const double* a, const double* b,
                        const int64_t* leaf_s0, const int32_t* leaf_m, double* w, const LeafOut* outs,
                        int max_sweeps);

// k_merge_prep: one workgroup per merge, any power of two from 64 to
// PREP_VL threads (the results do not depend on it); prep_threads picks the
// smallest that gives every element of the level's largest merge a lane.
constexpr int PREP_VL = 1024;
inline int prep_threads(int nmax) {
  int t = 64;
  while (t < nmax && t < PREP_VL) t <<= 1;
  return t;
}
__global__ void k_merge_sort(const MergeDev* __restrict__ merges, const RootBlock* __restrict__ blocks,
                             LevelBufs B);
__global__ void k_merge_prep(MergeDev* __restrict__ merges, LevelBufs B);

__global__ void k_secular(const MergeDev* __restrict__ merges, const RootBlock* __restrict__ blocks,
                          const double* __restrict__ dS, const double* __restrict__ zS,
                          double* __restrict__ lamS, double* __restrict__ gamS, double* __restrict__ muS,
                          int max_iter, int* __restrict__ noconv);

__global__ void k_lowner(const MergeDev* __restrict__ merges, const RootBlock* __restrict__ blocks,
                         const double* __restrict__ dS, const double* __restrict__ zS,
                         const double* __restrict__ gamS, const double* __restrict__ muS,
                         double* __restrict__ uhS);

__global__ void k_vnorm(const MergeDev* __restrict__ merges, const RootBlock* __restrict__ blocks,
                        const double* __restrict__ dS, const double* __restrict__ gamS,
                        const double* __restrict__ muS, const double* __restrict__ uhS,
                        double* __restrict__ vS);

__global__ void k_final_order(const MergeDev* __restrict__ merges, LevelBufs B,
                              const RootBlock* __restrict__ blocks);

__global__ void k_leaf_bounds(MergeDev* __restrict__ merges, const int32_t* __restrict__ which, LevelBufs B,
                              double thresh, int shift_max, double rank_eps, int r_cap);
__global__ void k_leaf_group(const MergeDev* __restrict__ merges, const int2* __restrict__ jobs, LevelBufs B);

__global__ void k_zero_unsupported(const MergeDev* __restrict__ merges, int g, LevelBufs B);

__global__ void k_pack_rot(const MergeDev* __restrict__ merges, const int32_t* __restrict__ col_merge,
                           const int32_t* __restrict__ col_idx, LevelBufs B, int njob);

__global__ void k_cauchy(const MergeDev* __restrict__ merges, const int32_t* __restrict__ tile_merge,
                         const int32_t* __restrict__ tile_col0, LevelBufs B, int ncols, int grouped);

// The dense update's two block products per merge from its deflation results
// (sizes, operand offsets); row counts and tile offsets are the host's, for
// the worst case N = n.  pb and pc may be null.
__global__ void k_build_probs(const MergeDev* __restrict__ ms, int nm, GemmProb* __restrict__ pa,
                              GemmProb* __restrict__ pb, GemmProb* __restrict__ pc, const double* __restrict__ pk,
                              const double* __restrict__ qc, const double* __restrict__ v,
                              const int32_t* __restrict__ posR);

__global__ void k_gemm_f64(const GemmProb* __restrict__ probs, int nprobs);
__global__ void k_gemm_f64_n64(const GemmProb* __restrict__ probs, int nprobs);
__global__ void k_gemm_f64_n96(const GemmProb* __restrict__ probs, int nprobs);
__global__ void k_gemm_f64_big(const GemmProb* __restrict__ probs, int nprobs, const int* __restrict__ ntiles);
__global__ void k_gemm_compact(GemmProb* __restrict__ probs, int nprobs, int bn, int* __restrict__ ntiles);
