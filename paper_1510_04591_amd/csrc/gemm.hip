// Grouped FP64 MFMA GEMM used by the dense update (Algorithm 1: the block
// diagonal of the children's eigenvectors times the Cauchy-like Q') and by
// every generator product of the HSS multiply (Algorithm 3).
//
// For each problem: C(:, colmap[j]) = beta C(:, colmap[j]) + vscale[j] *
// ([A A2] [B; B2])(:, j), all column-major, the inner dimension split into a
// first segment of K columns of A (rows of B) and an optional second segment
// of K2; either B segment may be stored transposed.  Workgroup tile BM x BN,
// K step 16, WM x WN waves each owning a (BM/WM) x (BN/WN) block as tiles of
// v_mfma_f64_16x16x4f64.  Operand tiles are staged through LDS
// (double-buffered; the next tile is fetched into registers while the current
// one feeds the matrix cores).  Eight or sixteen waves per workgroup keep
// enough loads in flight to cover the memory latency (measured: 8 waves
// reach about 1.5x the throughput of 4 on the same tile).  Lane layout of
// the 16x16x4 f64 instruction: A[i][k] from lane i + 16k, B[k][j] from lane
// j + 16k, D[lane/16 + 4r][lane % 16] in accumulator r.
//
//   k_gemm_f64       128 x 128, 4 x 2 waves (512 lanes)
//   k_gemm_f64_n64   128 x 64,  4 x 2 waves (512 lanes), narrow products
//   k_gemm_f64_n96   128 x 96,  4 x 2 waves (512 lanes), products 65..96 wide
//   k_gemm_f64_big   256 x 128, 4 x 4 waves (1024 lanes), large updates
#include "common.hpp"
#include "kernels.hpp"

namespace {
typedef double dbl2 __attribute__((ext_vector_type(2)));
constexpr int BK = 16;
constexpr int PAD = 4;

// PF2: the operand tiles of two K steps ahead in flight (two register sets);
// otherwise one step ahead.  The deeper prefetch costs registers and pays
// only where occupancy is not the limit (the 256 x 128 tiles).
// Operand loads of one K step.  Lane mapping (fixed for the tile):
//   A (column-major, BM x BK): row tid % BM, columns tid / BM + (NT / BM) q;
//   B (BK x BN): k index kb, columns cb0 + (NT / BK) q, with kb = tid % BK,
//     cb0 = tid / BK when B is read as stored (k fastest in memory), and
//     kb = (tid / 32) % BK, cb0 = tid % 32 + 32 (tid / (32 BK)) when it is
//     read transposed (n fastest in memory), so that a wave reads whole
//     128- or 256-byte runs in both cases.
// The pointers advance by one K step per call; rows, columns and the K
// range of the segment are checked only where a step can leave them.
template <int BM, int BN, int NT>
struct TileLoader {
  static constexpr int ALOADS = BM * BK / NT, BLOADS = BK * BN / NT;
  static constexpr int AST = NT / BM, BST = NT / BK;
  static_assert(NT % BM == 0 && NT % BK == 0 && NT % (32 * BK) == 0 && BN % 32 == 0, "loader layout");
  int ar, ac0, kb, cb0;
  bool row_ok, interior;
  bool col_ok[BLOADS];
  // current segment
  gcdouble* pa;
  gcdouble* pb;
  int64_t a_q, a_step, b_q, b_step;
  int kpos, kend;  // step start and end of the segment's K range
  bool trans;
  int seg;         // 0: first segment, 1: second, 2: done

  __device__ __forceinline__ void start_segment(const GemmProb& P, int m0, int n0, int s) {
    seg = s;
    const int K = s == 0 ? P.K : P.K2;
    if (K <= 0) {
      if (s == 0) start_segment(P, m0, n0, 1);
      else seg = 2;
      return;
    }
    const double* A = s == 0 ? P.A : P.A2;
    const double* B = s == 0 ? P.B : P.B2;
    const int64_t lda = s == 0 ? P.lda : P.lda2, ldb = s == 0 ? P.ldb : P.ldb2;
    trans = (s == 0 ? P.transB : P.transB2) != 0;
    const int tid = threadIdx.x;
    kb = trans ? (tid / 32) % BK : tid % BK;
    cb0 = trans ? tid % 32 + 32 * (tid / (32 * BK)) : tid / BK;
    kpos = 0;
    kend = K;
    pa = gmem(A) + (m0 + ar) + (int64_t)ac0 * lda;
    a_q = (int64_t)AST * lda;
    a_step = (int64_t)BK * lda;
    if (trans) {
      pb = gmem(B) + (n0 + cb0) + (int64_t)kb * ldb;
      b_q = BST;
      b_step = (int64_t)BK * ldb;
    } else {
      pb = gmem(B) + kb + (int64_t)(n0 + cb0) * ldb;
      b_q = (int64_t)BST * ldb;
      b_step = BK;
    }
    interior = row_ok;
#pragma unroll
    for (int q = 0; q < BLOADS; ++q) {
      col_ok[q] = n0 + cb0 + BST * q < P.N;
      interior = interior && col_ok[q];
    }
  }

  __device__ __forceinline__ void init(const GemmProb& P, int m0, int n0) {
    const int tid = threadIdx.x;
    ar = tid % BM;
    ac0 = tid / BM;
    row_ok = m0 + ar < P.M;
    start_segment(P, m0, n0, 0);
  }

  // One step's operands in registers, with the B lane mapping they were
  // loaded with (the two segments may read B differently).
  struct Regs {
    double a[ALOADS], b[BLOADS];
    int kb, cb0;
  };

  // loads of the step at kpos into r; then one step on (next segment when
  // this one is used up)
  __device__ __forceinline__ void load(const GemmProb& P, int m0, int n0, Regs& r) {
    double* ra = r.a;
    double* rb = r.b;
    r.kb = kb;
    r.cb0 = cb0;
    const bool full = kpos + BK <= kend;
    // the wave-uniform fast case: every row, column and k index inside
    if (__builtin_amdgcn_readfirstlane((int)(full && interior)) && full && interior) {
#pragma unroll
      for (int q = 0; q < ALOADS; ++q) ra[q] = pa[q * a_q];
#pragma unroll
      for (int q = 0; q < BLOADS; ++q) rb[q] = pb[q * b_q];
    } else {
#pragma unroll
      for (int q = 0; q < ALOADS; ++q) ra[q] = (row_ok && kpos + ac0 + AST * q < kend) ? pa[q * a_q] : 0.0;
#pragma unroll
      for (int q = 0; q < BLOADS; ++q) rb[q] = (col_ok[q] && kpos + kb < kend) ? pb[q * b_q] : 0.0;
    }
    kpos += BK;
    pa += a_step;
    pb += b_step;
    if (kpos >= kend && seg == 0) start_segment(P, m0, n0, 1);
  }
};

// PF2: the operand tiles of two K steps ahead in flight (two register sets);
// otherwise one step ahead.  The deeper prefetch costs registers and pays
// only where occupancy is not the limit (the 256 x 128 tiles).
template <int BM, int BN, int WM, int WN, bool PF2>
__device__ __forceinline__ void gemm_tile(const GemmProb& P, int m0, int n0) {
  constexpr int NT = 64 * WM * WN;
  constexpr int WTM = BM / WM, WTN = BN / WN;  // rows / columns per wave
  constexpr int TM = WTM / 16, TN = WTN / 16;  // 16 x 16 tiles per wave
  using LD = TileLoader<BM, BN, NT>;
  constexpr int ALOADS = LD::ALOADS, BLOADS = LD::BLOADS;
  (void)ALOADS;
  (void)BLOADS;
  __shared__ double As[2][BK][BM + PAD];
  __shared__ double Bs[2][BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = wave_index();
  const int wm = wv % WM, wn = wv / WM;
  const int li = lane & 15, lk = lane >> 4;
  const int M = P.M, N = P.N;

  dbl4 acc[TM][TN];
  #pragma unroll
  for (int a = 0; a < TM; ++a)
    #pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

  LD ld;
  ld.init(P, m0, n0);
  const int nk = (P.K + BK - 1) / BK + (P.K2 + BK - 1) / BK;
  using Regs = typename LD::Regs;
  // LDS places of a register set's loads
  auto sstore = [&](int buf, const Regs& r) {
    #pragma unroll
    for (int q = 0; q < ALOADS; ++q) As[buf][ld.ac0 + LD::AST * q][ld.ar] = r.a[q];
    #pragma unroll
    for (int q = 0; q < BLOADS; ++q) Bs[buf][r.kb][r.cb0 + LD::BST * q] = r.b[q];
  };
  auto mfma_step = [&](int buf) {
    #pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int k = kk * 4 + lk;
      double av[TM], bv[TN];
      #pragma unroll
      for (int t = 0; t < TM; ++t) av[t] = As[buf][k][wm * WTM + t * 16 + li];
      #pragma unroll
      for (int t = 0; t < TN; ++t) bv[t] = Bs[buf][k][wn * WTN + t * 16 + li];
      #pragma unroll
      for (int a = 0; a < TM; ++a)
        #pragma unroll
        for (int b = 0; b < TN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  };
  if constexpr (PF2) {
    // Two register sets of operand loads: the tile two K steps ahead is in
    // flight while the next one is stored to LDS and the current one feeds
    // the matrix cores (set indices are compile-time: the loop is unrolled
    // by two).  The per-step segment bookkeeping is in the loader; the B
    // layout of a step does not depend on the segment (LDS is [k][n]).
    Regs r0, r1;
    // step kt: LDS buffer kt & 1 holds tile kt; the set `nx` holds tile kt + 1
    // (stored at the end of the step), the set `fr` is free and receives tile
    // kt + 2
    auto step = [&](int kt, const Regs& nx, Regs& fr) {
      if (kt + 2 < nk) ld.load(P, m0, n0, fr);
      mfma_step(kt & 1);
      if (kt + 1 < nk) sstore((kt + 1) & 1, nx);
      __syncthreads();
    };
    if (nk > 0) {
      ld.load(P, m0, n0, r0);
      sstore(0, r0);
    }
    if (nk > 1) ld.load(P, m0, n0, r1);
    __syncthreads();
    for (int kt = 0; kt < nk; kt += 2) {
      step(kt, r1, r0);
      if (kt + 1 < nk) step(kt + 1, r0, r1);
    }
  } else {
    Regs r;
    if (nk > 0) {
      ld.load(P, m0, n0, r);
      sstore(0, r);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) ld.load(P, m0, n0, r);
      mfma_step(buf);
      if (kt + 1 < nk) sstore(buf ^ 1, r);
      __syncthreads();
    }
  }
  if constexpr (BM == 128) {
    // Epilogue through LDS: the tile goes out 32 columns at a time, each
    // column as 128 contiguous rows, one wave per column (two rows of 16
    // bytes per lane) instead of the MFMA result layout's 16 columns of 4
    // rows per store instruction.  The operand buffer As is free by now.
    constexpr int CW = 32;                 // columns per pass
    constexpr int LDC = BM + PAD;          // 132 doubles per staged column
    static_assert(CW * LDC <= 2 * BK * (BM + PAD), "staging fits in As");
    double* Cs = &As[0][0][0];
    gdouble* const gC = gmem(P.C);
    const bool vec = ((reinterpret_cast<uintptr_t>(P.C) | (uintptr_t)(P.ldc * 8)) & 15) == 0;
    #pragma unroll
    for (int pass = 0; pass < BN / CW; ++pass) {
      __syncthreads();
      #pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int cl = wn * WTN + b * 16;  // first tile column of the block
        if (cl / CW != pass) continue;
        #pragma unroll
        for (int a = 0; a < TM; ++a)
          #pragma unroll
          for (int r = 0; r < 4; ++r) Cs[(cl - pass * CW + li) * LDC + wm * WTM + a * 16 + lk + 4 * r] = acc[a][b][r];
      }
      __syncthreads();
      #pragma unroll
      for (int q = 0; q < CW * (BM / 2) / NT; ++q) {
        const int e = tid + NT * q;
        const int rp = e % (BM / 2), cl = e / (BM / 2);
        const int col = n0 + pass * CW + cl;
        const int row = m0 + 2 * rp;
        if (col >= N || row >= M) continue;
        const double vs = P.vscale ? gmem(P.vscale)[col] : 1.0;
        const int64_t cc = (int64_t)(P.colmap ? gmem(P.colmap)[col] : col) * P.ldc;
        double x0 = Cs[cl * LDC + 2 * rp] * vs, x1 = Cs[cl * LDC + 2 * rp + 1] * vs;
        gdouble* cp = gC + row + cc;
        if (vec && row + 1 < M) {
          if (P.beta != 0.0) {
            const dbl2 o = *(const __attribute__((address_space(1))) dbl2*)cp;
            x0 += P.beta * o.x;
            x1 += P.beta * o.y;
          }
          *(__attribute__((address_space(1))) dbl2*)cp = dbl2{x0, x1};
        } else {
          cp[0] = (P.beta != 0.0) ? (P.beta * cp[0] + x0) : x0;
          if (row + 1 < M) cp[1] = (P.beta != 0.0) ? (P.beta * cp[1] + x1) : x1;
        }
      }
    }
  } else {
  #pragma unroll
  for (int b = 0; b < TN; ++b) {
    const int col = n0 + wn * WTN + b * 16 + li;
    if (col >= N) continue;
    const double vs = P.vscale ? gmem(P.vscale)[col] : 1.0;
    const int64_t cc = (int64_t)(P.colmap ? gmem(P.colmap)[col] : col) * P.ldc;
    #pragma unroll
    for (int a = 0; a < TM; ++a) {
      const int row0 = m0 + wm * WTM + a * 16 + lk;
      #pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + 4 * r;
        if (row < M) {
          gdouble* cp = gmem(P.C) + row + cc;
          const double x = acc[a][b][r] * vs;
          *cp = (P.beta != 0.0) ? (P.beta * *cp + x) : x;
        }
      }
    }
  }
  }
}

__device__ __forceinline__ int find_prob(const GemmProb* __restrict__ probs, int nprobs, int bid) {
  int lo = 0, hi = nprobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile0 <= bid) lo = mid; else hi = mid - 1;
  }
  return lo;
}
}  // namespace

// Workgroups are handed to the eight XCDs round-robin by index.  With
// XCD_GROUPED the flat tile index is first renumbered so that every XCD
// works on one contiguous range of tiles, and inside a problem the tiles are
// walked in groups of GROUP_M row tiles (all column tiles of a group before
// the next group): the workgroups resident on one XCD at a time then share a
// few A row panels and B column panels, which stay in that XCD's L2.
constexpr int NXCD = 8;
constexpr int GROUP_M = 8;

__device__ __forceinline__ int xcd_contiguous(int bid, int nblk) {
  const int per = nblk / NXCD, rem = nblk % NXCD;
  const int x = bid % NXCD, i = bid / NXCD;
  return (x < rem) ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// ntiles (optional): the number of tiles that carry work, for a launch sized
// for the worst case whose problems were compacted by k_gemm_compact; the
// workgroups past it leave at once, and the XCD ranges cover only the
// working tiles.
template <int BM, int BN, int WM, int WN, bool PF2 = false, bool XCD_GROUPED = false>
__device__ __forceinline__ void gemm_dispatch(const GemmProb* __restrict__ probs, int nprobs,
                                              const int* __restrict__ ntiles = nullptr) {
  int nblk = (int)gridDim.x;
  if (ntiles) {
    nblk = min(*ntiles, nblk);
    if ((int)blockIdx.x >= nblk) return;
  }
  const int bid = XCD_GROUPED ? xcd_contiguous((int)blockIdx.x, nblk) : (int)blockIdx.x;
  const GemmProb P = probs[find_prob(probs, nprobs, bid)];
  const int local = bid - P.tile0;
  int mt, nt;
  if constexpr (XCD_GROUPED) {
    const int tiles_n = (P.N + BN - 1) / BN;
    if (local >= P.tiles_m * tiles_n) return;  // problems sized for a larger N (batched solver)
    const int gsize = GROUP_M * tiles_n;
    const int g = local / gsize, first = g * GROUP_M;
    const int gm = min(P.tiles_m - first, GROUP_M);
    const int in = local - g * gsize;
    mt = first + in % gm;
    nt = in / gm;
  } else {
    mt = local % P.tiles_m;
    nt = local / P.tiles_m;
  }
  const int m0 = mt * BM, n0 = nt * BN;
  if (m0 >= P.M || n0 >= P.N) return;
  gemm_tile<BM, BN, WM, WN, PF2>(P, m0, n0);
}

__global__ void __launch_bounds__(512) k_gemm_f64(const GemmProb* __restrict__ probs, int nprobs) {
  gemm_dispatch<128, 128, 4, 2>(probs, nprobs);
}

__global__ void __launch_bounds__(512) k_gemm_f64_n64(const GemmProb* __restrict__ probs, int nprobs) {
  gemm_dispatch<128, 64, 4, 2>(probs, nprobs);
}

__global__ void __launch_bounds__(512) k_gemm_f64_n96(const GemmProb* __restrict__ probs, int nprobs) {
  gemm_dispatch<128, 96, 4, 2>(probs, nprobs);
}

__global__ void __launch_bounds__(1024) k_gemm_f64_big(const GemmProb* __restrict__ probs, int nprobs,
                                                      const int* __restrict__ ntiles) {
  gemm_dispatch<256, 128, 4, 4, true, true>(probs, nprobs, ntiles);
}

// Tile offsets of a grouped product built on the device, made compact: each
// problem's tile0 becomes the number of tiles (tiles_m x ceil(N / bn)) of
// the problems before it at their actual sizes, and the total goes to
// *ntiles.  One workgroup: a chunk of problems per lane, a scan of the chunk
// sums in LDS.
__global__ void __launch_bounds__(1024) k_gemm_compact(GemmProb* __restrict__ probs, int nprobs, int bn,
                                                       int* __restrict__ ntiles) {
  __shared__ int part[1024];
  const int T = (int)blockDim.x, tid = (int)threadIdx.x;
  const int per = (nprobs + T - 1) / T;
  const int b = min(nprobs, tid * per), e = min(nprobs, b + per);
  auto tiles = [&](const GemmProb& P) { return P.N > 0 ? P.tiles_m * ((P.N + bn - 1) / bn) : 0; };
  int s = 0;
  for (int i = b; i < e; ++i) s += tiles(probs[i]);
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {
    const int v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - s;
  for (int i = b; i < e; ++i) {
    probs[i].tile0 = run;
    run += tiles(probs[i]);
  }
  if (tid == T - 1) *ntiles = part[T - 1];
}
