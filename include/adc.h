/*
 * adc.h -- C ABI of the MI355X (gfx950) accelerated divide-and-conquer
 * tridiagonal eigensolver.
 *
 * The problem (Section 2, eq. T): a real symmetric tridiagonal matrix T with
 * diagonal a[0..n) and off-diagonal b[0..n-1); all eigenvalues Lambda and an
 * orthonormal eigenvector matrix Q with T Q = Q Lambda (Algorithm 1, ADC(T,Q,
 * Lambda)).  The merge step of Algorithm 1 solves the secular equation of
 * D + rho z z^T (Theorem 1), recomputes z by Loewner's formula (eq. ev_z),
 * forms the Cauchy-like eigenvector matrix Q' from its generators (eq. Ev-Q,
 * eq. cauchylike, Remark 1) and updates the eigenvectors either by a dense
 * product diag(Q1,Q2) Q' or through an HSS approximation of Q' built by
 * Algorithm 2 and applied by Algorithm 3.
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers (HIP global memory of the
 *    context's device) unless the comment says "host".  Matrices are FP64,
 *    column-major, with the stated leading dimension.
 *  - The caller owns every array it passes.  The library never keeps a
 *    pointer to caller memory after the call returns.
 *  - Calls are ordered on the context's HIP stream.  Entry points marked
 *    "blocking" synchronise that stream before returning; the others only
 *    enqueue work.
 *  - The library never aborts and never prints.  Errors are reported by the
 *    return value; adc_status_string() names them.  Invalid arguments give
 *    ADC_ERR_ARG before any work is enqueued.
 *  - A context is not thread-safe: use one context per host thread.
 */
#ifndef ADC_H
#define ADC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum adc_status {
  ADC_OK = 0,
  ADC_ERR_ARG = 1,          /* invalid argument or non-finite input          */
  ADC_ERR_NOMEM = 2,        /* device allocation failed                      */
  ADC_ERR_HIP = 3,          /* a HIP runtime call failed                     */
  ADC_ERR_NOCONV = 4,       /* a secular root did not converge (info_index)  */
  ADC_ERR_ACCURACY = 5,     /* HSS check failed and opts.strict was set      */
  ADC_ERR_UNSUPPORTED = 6   /* size or option outside what is implemented    */
} adc_status;

typedef struct adc_ctx_s* adc_ctx;
typedef struct adc_hss_s* adc_hss;

/* How the HSS sample count s = r + p is chosen for one merge.
 * BOUND: r from eq. (bounds) over neighbouring leaf segments (Section 4.1).
 * MLP:   r from the learned rank predictor (adc_mlp_*): per leaf boundary a
 *        prediction y_b of log2 of the ID rank, r = ceil(1.25 2^max_b y_b) + 4,
 *        clamped to [8, r_cap]; the BOUND estimate while no model is set.
 *        The adaptive check (opts.check_tol) judges either choice.
 * FIXED: r = opts.fixed_rank. */
typedef enum adc_rank_mode { ADC_RANK_BOUND = 0, ADC_RANK_MLP = 1, ADC_RANK_FIXED = 2 } adc_rank_mode;

/* Sampling of Algorithm 2, i.e. Phi = the block rows of the Cauchy-like matrix
 * without their diagonal blocks times Omega, and Theta likewise for the
 * block columns.
 * DIRECT: every entry generated from (d, gam, mu, uh, v) and summed, O(K^2 s).
 * FMM:    the off-diagonal Cauchy sums by a one-dimensional fast multipole
 *         method (the acceleration the paper names for this step, Sections 1,
 *         3 and 5): Chebyshev interpolation with fmm_order points per node of
 *         the HSS tree, nodes in coordinates local to their first pole, two
 *         nodes well separated when their gap (eq. d-lambda) is at least the
 *         larger width; pairs of leaves that are not are summed entry by
 *         entry with the differences of eq. (d-lambda).  O(K s (P + m)) for
 *         well-spread spectra; agrees with DIRECT to about 1e-15 relative at
 *         fmm_order 20. */
typedef enum adc_sample_mode { ADC_SAMPLE_DIRECT = 0, ADC_SAMPLE_FMM = 1 } adc_sample_mode;

/* Options.  adc_opts_default() fills the values in brackets. */
typedef struct adc_opts {
  int32_t dc_leaf;       /* [32] DC leaf size m (Algorithm 1); 2..64            */
  int32_t hss_min_k;     /* [2048] HSS update only if the deflated size K >= this
                            (and K >= 8 in any case); Section 4.3 sets the
                            threshold near 2000 for its CPUs                   */
  int32_t hss_levels;    /* [-1] only the top hss_levels merge levels may use
                            HSS; <0 means every level                         */
  int32_t hss_leaf;      /* [128] HSS leaf size (rows per leaf node)          */
  double  id_tol;        /* [1e-14] ID truncation |R_kk| <= id_tol |R_11|       */
  int32_t oversample;    /* [16] p, samples beyond the rank estimate (Section 3
                            takes 10; 16 keeps the check at 1e-13 from
                            failing at the top merges, whose retries cost
                            more than the extra columns)                  */
  int32_t rank_mode;     /* [ADC_RANK_BOUND] adc_rank_mode                      */
  int32_t fixed_rank;    /* [0] r for ADC_RANK_FIXED                            */
  int32_t max_retries;   /* [2] sample doublings before the dense fallback     */
  int32_t max_iter;      /* [60] secular iterations per root                   */
  uint64_t seed;         /* [20151015] seed of the Gaussian sampling matrices  */
  int32_t force_dense;   /* [0] 1: plain DC, never HSS                          */
  int32_t strict;        /* [0] 1: a failed HSS check is ADC_ERR_ACCURACY       */
  double  check_tol;     /* [1e-13] relative error allowed by the HSS check     */
  int32_t nprobe;        /* [4] Gaussian probe vectors of the HSS check, 1..32  */
  int32_t shift_max;     /* [5] max boundary move of the rank estimate, 0..64   */
  double  shift_thresh;  /* [1e-10] move a boundary when its distance is below  */
  int32_t r_cap;         /* [100] cap of the estimated rank                     */
  double  rank_eps;      /* [1e-16] epsilon of eq. (bounds)                     */
  double  hss_min_flops; /* [2.5e10] HSS update only if the merge's dense
                            update, 2 n1 K (k1+k2) + 2 n2 K (k2+k3) flops
                            with the column classes of the deflated Q
                            (Section 2.1), reaches this (about 0.5 ms of FP64
                            MFMA GEMM; the HSS route's fixed costs outweigh
                            smaller updates); once one merge of a level qualifies,
                            merges of the level reaching a quarter of it
                            (and hss_min_k) join; 0 disables the test     */
  int32_t sample_mode;   /* [ADC_SAMPLE_FMM] adc_sample_mode: how Algorithm 2
                            takes its samples                                */
  int32_t fmm_order;     /* [20] Chebyshev points per tree node of the fast
                            sampling, 4..32                                  */
  int32_t sat_guard;     /* [0] 1: an HSS merge whose interpolative
                            decompositions saturate (a node rank equal to s
                            with more than s candidates, so the samples may
                            not span the block) fails its check like a large
                            probe error: its samples double and it is rebuilt;
                            0: saturated merges are only counted            */
  double  batch_bytes;   /* [0] adc_stedc_batched: device bytes one group of
                            HSS-eligible matrices solved together may take
                            (second eigenvector buffers n^2 per matrix plus
                            two packed operands of rows x largest n, 8 bytes
                            each); a larger set is split into consecutive
                            groups; 0 means 32 GiB                         */
} adc_opts;

/* Report of one solve (host struct, optional). */
typedef struct adc_report {
  int32_t levels;            /* merge levels of the DC tree                    */
  int32_t merges;            /* merges performed                               */
  int32_t hss_merges;        /* merges updated through HSS                     */
  int32_t retries;           /* HSS sample doublings                           */
  int32_t hss_fallbacks;     /* HSS merges that fell back to the dense update  */
  int32_t info_index;        /* failing argument / root index, else -1         */
  int64_t n_per_level[64];   /* sum of merge sizes n per level (top = 0)       */
  int64_t K_per_level[64];   /* sum of deflated sizes K per level               */
  int32_t hss_per_level[64]; /* HSS merges per level                            */
  int32_t max_rank;          /* largest HSS node rank seen                      */
  int32_t samples;           /* largest sample count s used                     */
  double  t_phase[12];       /* seconds, from HIP events on the context stream:
                                0 tear+leaves, 1 merge prep and deflation,
                                2 secular, 3 Loewner+v, 4 dense update GEMM,
                                5 HSS rank estimate+sampling, 6 HSS compression,
                                7 HSS check, 8 HSS multiply, 9 ordering,
                                rotations, packing and the Cauchy matrix,
                                10 total wall time (host clock), 11 wall time
                                not covered by phases 0-9                      */
  double  phase_flops[12];   /* algorithmic flops per phase (same indices)     */
  double  phase_bytes[12];   /* algorithmic HBM bytes per phase; for 8 (HSS
                                multiply) the least traffic of Algorithm 3 over
                                the accepted HSS merges' update products:
                                24 P K + 16 P K r/m bytes per merge (P rows,
                                K columns, r the mean node rank, m the mean
                                leaf size)                                     */
  int32_t phase_launches[12];/* kernel launches of the phase's main kernel     */
  double  flops_model;       /* algorithmic flops of the eigenvector updates   */
  double  bytes_model;       /* algorithmic HBM bytes of the updates           */
  double  check_err_max;     /* largest HSS check error accepted               */
  /* Per-kernel figures, each launch bracketed by HIP events on the context
   * stream: 0 k_gemm_f64 (128 x 128 FP64 MFMA GEMM tiles), 1 k_gemm_f64_n64
   * (128 x 64), 2 k_hss_sample, 3 k_pack_rot, 4 k_secular, 5 k_hss_compress,
   * 6 k_gemm_f64_big (256 x 128, the dense update), 7 k_gemm_f64_n96
   * (128 x 96), 8 k_fmm_leaf (fast sampling: near field and local
   * expansions), 9 k_fmm_m2l (fast sampling: far-field translations),
   * 10-11 unused.
   * Times in seconds; flops and bytes are the algorithmic counts of the
   * launches (operands read once, results written once). */
  double  kern_time[12];
  double  kern_flops[12];
  double  kern_bytes[12];
  int32_t kern_launches[12];
  int32_t hss_saturated;     /* accepted HSS merges with a saturated node
                                (see adc_opts.sat_guard)                      */
  int32_t hss_sat_nodes;     /* saturated nodes in those merges              */
} adc_report;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`, ordered on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the context. */
adc_status adc_create(adc_ctx* out, int device, void* hip_stream);
/* Release the context and its device memory pool. */
adc_status adc_destroy(adc_ctx ctx);
/* Fill *opts with the defaults listed above. */
adc_status adc_opts_default(adc_opts* opts);
/* Static string naming a status. */
const char* adc_status_string(adc_status s);
/* Device bytes adc_stedc needs for size n with the given options.  Passing a
 * caller workspace of that size avoids the context's own pool. */
adc_status adc_workspace_query(adc_ctx ctx, int64_t n, const adc_opts* opts, size_t* bytes);

/* ----------------------------------------------------------------- solve */

/* Eigendecomposition of T (Algorithm 1).  Blocking.
 *   diag[n], offdiag[n-1] : input (read-only); offdiag may be NULL iff n == 1
 *   w[n]                  : eigenvalues, ascending
 *   Z[ldz*n]              : eigenvectors, column j belongs to w[j]; ldz >= n
 *   ws, ws_bytes          : optional workspace (NULL: the context pool)
 *   opts                  : host struct, NULL = defaults
 *   rep                   : host struct, may be NULL
 * Non-finite input returns ADC_ERR_ARG.  A root that fails to converge
 * returns ADC_ERR_NOCONV with rep->info_index = its global index. */
adc_status adc_stedc(adc_ctx ctx, int64_t n, const double* diag, const double* offdiag,
                     double* w, double* Z, int64_t ldz, void* ws, size_t ws_bytes,
                     const adc_opts* opts, adc_report* rep);

/* Many independent eigendecompositions (level-batched).  Blocking.
 *   count                 : number of matrices
 *   n[count]              : host array of sizes
 *   diag, offdiag, w, Z   : host arrays of `count` device pointers
 *   ldz[count]            : host array of leading dimensions
 * Every DC level of every matrix runs as one launch per merge phase over a
 * device work queue.  The matrices whose merges cannot take the HSS update
 * (all of them with opts->force_dense = 1) form one level sequence that is
 * captured once in a HIP graph keyed by their size set and replayed by later
 * calls with the same sizes.  The matrices that may reach an HSS merge
 * (n >= hss_min_k and a top-merge dense update of at least hss_min_flops)
 * are solved together in a second level-batched pass that takes the HSS
 * route where it applies (Section 4.3), with host decisions at its HSS
 * levels; they are taken in order in groups of at most 10^6 rows whose
 * workspace fits opts->batch_bytes, one pass per group.  rep may be NULL
 * (one report for the whole batch otherwise; rep->info_index is the index
 * of the matrix that failed). */
adc_status adc_stedc_batched(adc_ctx ctx, int32_t count, const int64_t* n,
                             const double* const* diag, const double* const* offdiag,
                             double* const* w, double* const* Z, const int64_t* ldz,
                             const adc_opts* opts, adc_report* rep);

/* ------------------------------------------- merge-step kernels (parity) */

/* Secular roots of D + rho z z^T (Theorem 1), d strictly increasing,
 * ||z|| = 1, rho > 0.  Outputs gam[i] = lam_i - d_i and mu[i] = d_{i+1} -
 * lam_i (mu[K-1] = +inf), each taken from the iterate relative to the nearer
 * pole (Remark 1; Section 4.3).  lam may be NULL.  Asynchronous. */
adc_status adc_secular(adc_ctx ctx, int64_t K, const double* d, const double* z, double rho,
                       double* lam, double* gam, double* mu);

/* Loewner recompute (eq. ev_z): uh[i] = sign(z_i) sqrt(prod_j (lam_j - d_i) /
 * (rho prod_{j!=i} (d_j - d_i))), every difference by eq. (d-lambda); and the
 * column scales v[j] = 1/||(uh_i/(d_i - lam_j))_i|| of eq. (EVec).
 * Asynchronous. */
adc_status adc_lowner(adc_ctx ctx, int64_t K, const double* d, const double* z, double rho,
                      const double* gam, const double* mu, double* uh, double* v);

/* Dense Cauchy update (the plain DC update): Y[P x K] = X[P x K] * Q', with
 * Q'_{ij} = uh_i v_j / (d_i - lam_j) (eq. Ev-Q, differences by eq. d-lambda),
 * on the FP64 MFMA GEMM.  Y must not overlap X.  Asynchronous. */
adc_status adc_cauchy_gemm(adc_ctx ctx, int64_t P, int64_t K, const double* d, const double* gam,
                           const double* mu, const double* uh, const double* v,
                           const double* X, int64_t ldx, double* Y, int64_t ldy);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as adc_cauchy_gemm, same kernels, with no allocation of any kind.
 * The explicit Cauchy-like matrix and the launch descriptors live in one
 * static device array of 32 MiB + 64 KiB per GPU, held while the library is
 * loaded; hence K <= 2048 (larger K: ADC_ERR_UNSUPPORTED; nothing launched).
 * Every call on a GPU shares that array: calls ordered on one stream are
 * safe, calls that overlap on one GPU (other streams or contexts) race.
 * ADC_ERR_HIP when the array's device address could not be taken at
 * adc_create.  Asynchronous on the context stream (X, Y and the generators
 * must stay valid until the stream reaches the call). */
adc_status adc_cauchy_gemm_noalloc(adc_ctx ctx, int64_t P, int64_t K, const double* d,
                                   const double* gam, const double* mu, const double* uh,
                                   const double* v, const double* X, int64_t ldx, double* Y,
                                   int64_t ldy);

/* Rank estimate of Section 4.1 for one merge, the solver's own kernel: the
 * balanced leaf boundaries for opts->hss_leaf (L = ceil(log2(K / hss_leaf))
 * levels, at least one) are moved where two neighbouring segments are closer
 * than opts->shift_thresh (by at most opts->shift_max rows, to the largest
 * distance, boundaries in order), then *r = min(opts->r_cap, max over the
 * interior boundaries of ceil(log(16/eps) log(8R) / pi^2)) (eq. bounds, eps =
 * opts->rank_eps) with R = (lam_K - d_1) / dist and dist the distance of the
 * two segments by eq. (dist_xy), every difference by eq. (d-lambda).
 * d, gam, mu: device FP64 generators (d increasing, K >= 2).  bounds: host
 * array of bounds_cap entries receiving the 2^L + 1 moved boundaries (first
 * 0, last K); *nbounds (host, may be NULL) gets 2^L + 1; ADC_ERR_ARG when
 * bounds_cap is smaller.  Blocking. */
adc_status adc_rank_estimate(adc_ctx ctx, int64_t K, const double* d, const double* gam,
                             const double* mu, const adc_opts* opts, int32_t* r, int32_t* bounds,
                             int32_t bounds_cap, int32_t* nbounds);

/* Randomized HSS approximation H ~ Q' (Algorithm 2) of the Cauchy-like matrix
 * with generators (d, gam, mu, uh, v).  omega: K x s row-major Gaussian
 * sampling matrix, or NULL to draw it (Philox4x32-10, opts->seed) with s from
 * the rank estimate (s argument ignored).  The adaptive check (Gaussian
 * probes; sample doubling up to max_retries) runs unless omega is given.
 * Blocking.  *out is released by adc_hss_free. */
adc_status adc_hss_build(adc_ctx ctx, int64_t K, const double* d, const double* gam,
                         const double* mu, const double* uh, const double* v,
                         const double* omega, int32_t s, const adc_opts* opts, adc_hss* out);

/* The samples of Algorithm 2 alone: phi = Phi and theta = Theta (K x s,
 * row-major, device), row i of Phi being block row t(i) of the Cauchy-like
 * matrix with generators (d, gam, mu, uh, v) without its diagonal block,
 * times omega (K x s row-major, device), and Theta the same for block
 * columns.  The leaves are those of adc_hss_build for opts->hss_leaf
 * (balanced, L = ceil(log2(K / hss_leaf)) levels, at least one); the method
 * is opts->sample_mode with opts->fmm_order points per node.  1 <= s <= 256.
 * Blocking. */
adc_status adc_hss_sample(adc_ctx ctx, int64_t K, const double* d, const double* gam, const double* mu,
                          const double* uh, const double* v, const double* omega, int32_t s,
                          const adc_opts* opts, double* phi, double* theta);

/* Y[P x K] = X[P x K] * H (Algorithm 3, HSS times a general matrix from the
 * right).  Y must not overlap X.  Asynchronous. */
adc_status adc_hss_apply(adc_ctx ctx, adc_hss h, int64_t P, const double* X, int64_t ldx,
                         double* Y, int64_t ldy);

/* Host summary of an HSS matrix: levels below the root, leaves, max rank,
 * samples used, retries, check error (any pointer may be NULL). */
adc_status adc_hss_info(adc_hss h, int32_t* levels, int32_t* leaves, int32_t* max_rank,
                        int32_t* samples, int32_t* retries, double* check_err);
/* Per-node ranks in heap order (root 0, children of p at 2p+1, 2p+2): kr =
 * row-ID rank (columns of U_i), kc = column-ID rank (columns of V_i), lo/hi =
 * index range t_i.  Host arrays of nmax entries; writes min(nmax, nodes) and
 * returns the node count in *count. */
adc_status adc_hss_nodes(adc_hss h, int32_t nmax, int32_t* lo, int32_t* hi, int32_t* kr, int32_t* kc,
                         int32_t* count);
adc_status adc_hss_free(adc_hss h);

/* -------------------------------------------- learned rank predictor (MLP) */

/* The predictor replaces the a-priori rank of eq. (bounds) (Section 4.1):
 * per interior leaf boundary of an HSS merge it predicts log2 of the rank
 * the interpolative decompositions find there (the largest row or column
 * ID rank of the HSS nodes whose index range starts or ends at it).  It is a
 * 16-64-64-1 FP32 MLP with ReLU whose weights the context owns: 5313
 * parameters packed as W1 (64x16), b1, W2 (64x64), b2, W3 (1x64), b3, each W
 * row-major [out][in].
 *
 * adc_mlp_features: for the generators (d, gam, mu; device FP64, eq.
 *   (d-lambda)) of a merge of size K and the leaf boundaries bounds[nb+2]
 *   (host, strictly increasing, first 0, last K), writes feat[nb x 16]
 *   (device FP32, row-major), row b for the boundary bounds[b+1].  The 16
 *   features are scale-free ratios of pole gaps and root distances (the
 *   list is in mlp.hip).  Asynchronous.
 * adc_mlp_init:  uniform fan-in initialisation from `seed`, biases zero, Adam
 *   state cleared.  Blocking.
 * adc_mlp_train: `epochs` passes of Adam (beta1 0.9, beta2 0.999, eps 1e-8,
 *   step lr) over the B rows of X[B x 16], y[B] (device FP32) in minibatches
 *   of `batch` rows taken in order (shuffle beforehand if wanted); loss: mean
 *   squared error; *loss_out (host) gets the last pass's mean of the
 *   minibatch losses before their updates.  Blocking.  ADC_ERR_ARG before
 *   adc_mlp_init / adc_mlp_set.
 * adc_mlp_infer: y[B] = MLP(X[B x 16]), device FP32.  Asynchronous.
 * adc_mlp_grad:  loss and gradient of the mean squared error over all B rows
 *   (g_out: device FP32, 5313 values packed like the parameters).  Blocking.
 * adc_mlp_get/set: copy the 5313 parameters to / from a device FP32 array
 *   (set clears the Adam state).  Blocking.
 * adc_mlp_collect: runs adc_stedc on (diag, offdiag) with `opts` (rank
 *   estimate forced to BOUND) and, for every HSS merge that passes the check,
 *   appends one row per leaf boundary to X[max_rows x 16] (features) and
 *   y[max_rows] (log2 of the observed boundary rank), device FP32, as long
 *   as the merge's rows fit; *rows_out (host) receives the count.  Use opts
 *   with small hss_min_k and hss_leaf and hss_levels = -1 to collect from
 *   matrices whose merges would not use HSS otherwise.  Blocking. */
adc_status adc_mlp_features(adc_ctx ctx, int64_t K, const double* d, const double* gam,
                            const double* mu, const int64_t* bounds, int32_t nb, float* feat);
adc_status adc_mlp_init(adc_ctx ctx, uint64_t seed);
adc_status adc_mlp_train(adc_ctx ctx, int32_t B, const float* X, const float* y, int32_t epochs,
                         int32_t batch, float lr, float* loss_out);
adc_status adc_mlp_infer(adc_ctx ctx, int32_t B, const float* X, float* y);
adc_status adc_mlp_grad(adc_ctx ctx, int32_t B, const float* X, const float* y, float* g_out,
                        float* loss_out);
adc_status adc_mlp_get(adc_ctx ctx, float* params);
adc_status adc_mlp_set(adc_ctx ctx, const float* params);
adc_status adc_mlp_collect(adc_ctx ctx, int64_t n, const double* diag, const double* offdiag,
                           double* w, double* Z, int64_t ldz, const adc_opts* opts,
                           int64_t max_rows, float* X, float* y, int64_t* rows_out);

#ifdef __cplusplus
}
#endif
#endif /* ADC_H */
