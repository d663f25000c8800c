// Batched complex GEMM on the gfx950 matrix cores: FP64 (v_mfma_f64_16x16x4_f64)
// and FP32 (v_mfma_f32_16x16x4_f32) schemes.
//
// The complex block products dominate the selected solve (Section IV of the
// paper); this is the FP64 reference scheme.  A complex product is four real
// MFMA chains: C_re += A_re B_re - A_im B_im, C_im += A_re B_im + A_im B_re.
//
// Tiling: a 256-thread workgroup computes a 64 x 64 complex tile of C.  Each of
// its four waves owns four 16 x 16 MFMA blocks, interleaved (wave (wm, wn) takes
// row blocks wm, wm+2 and column blocks wn, wn+2), with separate real and
// imaginary accumulators: 8 independent MFMA chains per wave.  A launch whose
// 64 x 64 tiling pads C by more than 8% or gives few workgroups per CU uses
// 32 x 32 tiles instead, one 16 x 16 block per wave (four times the workgroups,
// less padding at b = 416).  Every output element is
// accumulated in the same K order by either tile size, so the results are
// bitwise the same.  Blocks that lie
// entirely outside C are skipped (wave-uniform), and the interleaving spreads
// such blocks of an edge tile evenly over the waves (b = 416 is 6.5 tiles).
// K advances 32 complex elements per step.  Operand tiles are copied to LDS in
// their natural global layout (row-major, coalesced loads, padded rows, the
// conjugate applied on the way in); the MFMA fragment reads do any transpose
// through the padded stride, so no LDS write is transposed.  The next K tile is
// prefetched into registers while the current one is consumed.  Tiles are
// assigned XCD-aware: consecutive workgroup ids land on different XCDs, so tile
// ids are remapped so that all tiles of one batch entry run on one XCD and
// share its L2.
#include "qtx_internal.h"

namespace qtx {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Arithmetic of the block products: FP64 MFMA (reference) or FP32 MFMA with the
// operands rounded to FP32 (round to nearest even) on their way into LDS.
// Accumulator layouts of the 16x16x4 instructions on gfx950 (lane l, element v):
//   f64: row l/16 + 4v, column l%16;   f32: row 4(l/16) + v, column l%16.
struct MathF64 {
  typedef double2 lds_t;
  typedef d4 acc_t;
  static __device__ inline lds_t cvt(double2 x) { return x; }
  static __device__ inline acc_t zero() { return d4{0.0, 0.0, 0.0, 0.0}; }
  static __device__ inline acc_t mfma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int v) { return lk + 4 * v; }
};
struct MathF32 {
  typedef float2 lds_t;
  typedef f4 acc_t;
  static __device__ inline lds_t cvt(double2 x) { float2 r; r.x = (float)x.x; r.y = (float)x.y; return r; }
  static __device__ inline acc_t zero() { return f4{0.0f, 0.0f, 0.0f, 0.0f}; }
  static __device__ inline acc_t mfma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int v) { return 4 * lk + v; }
};

namespace {

constexpr int BM = 64, BN = 64, BK = 32, NT = 256;
// LDS row strides (complex elements) of the two natural layouts of a tile:
// 64 rows x 32 (+1 pad) or 32 rows x 64 (+1 pad).
constexpr int RS_WIDE = BK + 1;    // rows are M (or N), columns K
constexpr int RS_LONG = BM + 1;    // rows are K, columns M (or N)
constexpr int TILE_ELEMS = (BM * RS_WIDE > BK * RS_LONG) ? BM * RS_WIDE : BK * RS_LONG;

__device__ inline int xcd_remap(int pid, int total) {
  // Workgroup `pid` is dispatched to XCD pid % 8.  Give XCD x a contiguous
  // range of logical tiles (bijective for any total).
  const int nx = 8;
  int per = total / nx, rem = total % nx;
  int x = pid % nx, local = pid / nx;
  return (x < rem) ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

// One operand tile in its natural layout: ROWS x COLS elements of a row-major
// source (leading dimension ld), rows [r0, r0+ROWS) bounded by nrows, columns
// [c0, c0+COLS) bounded by ncols; zero outside.  EPT elements per thread
// (8 for a 64 x 32 tile, 4 for 32 x 32): element e = tid + 256 j, so each wave
// loads and stores contiguous 1 KB runs (coalesced global reads, conflict-free
// LDS writes).
template <int ROWS, int COLS>
struct TileLoader {
  static constexpr int EPT = ROWS * COLS / NT;
  double2 v[EPT];
  __device__ inline void load(const double2* __restrict__ src, int64_t ld, int r0, int c0, int nrows, int ncols,
                              int tid) {
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = tid + NT * j;
      const int r = r0 + e / COLS, c = c0 + e % COLS;
      v[j] = (r < nrows && c < ncols) ? src[(int64_t)r * ld + c] : cmk(0.0, 0.0);
    }
  }
  template <bool CONJ, class MATH, class L>
  __device__ inline void store(L* lds, int rs, int tid) const {
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = tid + NT * j;
      lds[(e / COLS) * rs + e % COLS] = MATH::cvt(CONJ ? cconj(v[j]) : v[j]);
    }
  }
};

// KIND only separates kernel symbols by use (block products of the solve, the
// inversion's trailing update, elementwise assembly with K = 0) so profilers
// report them apart; the code is the same.
template <int OPA, int OPB, int KIND, class MATH, int TM>
__global__ __launch_bounds__(NT) void zgemm_mfma_kernel(GemmDesc d) {
  typedef typename MATH::lds_t lds_t;
  typedef typename MATH::acc_t acc_t;
  // TM x TM output tile; each wave owns NW x NW blocks of 16 x 16
  constexpr int BM = TM, BN = TM, NW = TM / 32;
  constexpr int RS_LONG = TM + 1;
  constexpr int TILE_ELEMS = (BM * RS_WIDE > BK * RS_LONG) ? BM * RS_WIDE : BK * RS_LONG;
  __shared__ lds_t As[TILE_ELEMS];
  __shared__ lds_t Bs[TILE_ELEMS];

  const int tiles_m = (d.M + BM - 1) / BM;
  const int tiles_n = (d.N + BN - 1) / BN;
  const int per = tiles_m * tiles_n;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int z = tile / per;
  const int t = tile - z * per;
  const int m0 = (t % tiles_m) * BM;
  const int n0 = (t / tiles_m) * BN;
  const bool skew = d.skew != 0;
  if (skew && m0 >= n0 + BN) return;   // strictly below the diagonal: written as mirror images

  const double2* __restrict__ A = d.tA ? d.tA[z] : d.A + (int64_t)z * d.sA;
  const double2* __restrict__ B = d.tB ? d.tB[z] : d.B + (int64_t)z * d.sB;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int M = d.M, N = d.N, K = d.K;

  // this wave's blocks: rows m0 + 16*(wm + 2i), columns n0 + 16*(wn + 2j); a block
  // is live if it lies in C (and, for a skew-Hermitian C, touches r <= c)
  bool live[NW][NW];
#pragma unroll
  for (int i = 0; i < NW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int rb = m0 + 16 * (wm + 2 * i), cb = n0 + 16 * (wn + 2 * j);
      live[i][j] = rb < M && cb < N && !(skew && rb >= cb + 16);
    }

  acc_t acc_re[NW][NW], acc_im[NW][NW];
#pragma unroll
  for (int i = 0; i < NW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      acc_re[i][j] = MATH::zero();
      acc_im[i][j] = MATH::zero();
    }

  // natural tiles: op(A) = N -> A rows are M (64 x 32); op(A) = C -> source rows are K (32 x 64)
  TileLoader<OPA == OP_N ? BM : BK, OPA == OP_N ? BK : BM> la;
  TileLoader<OPB == OP_N ? BK : BN, OPB == OP_N ? BN : BK> lb;
  auto gload = [&](int k0) {
    if (OPA == OP_N) la.load(A, d.lda, m0, k0, M, K, tid);
    else la.load(A, d.lda, k0, m0, K, M, tid);
    if (OPB == OP_N) lb.load(B, d.ldb, k0, n0, K, N, tid);
    else lb.load(B, d.ldb, n0, k0, N, K, tid);
  };

  const int nk = (K + BK - 1) / BK;
  if (nk > 0) gload(0);
  const int li = lane & 15;
  const int lk = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
    la.template store<OPA == OP_C, MATH>(As, OPA == OP_N ? RS_WIDE : RS_LONG, tid);
    lb.template store<OPB == OP_C, MATH>(Bs, OPB == OP_N ? RS_LONG : RS_WIDE, tid);
    __syncthreads();
    if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + lk;
      lds_t a[NW], b[NW];
      decltype(a[0].y) na[NW];
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const int m = 16 * (wm + 2 * i) + li;
        a[i] = (OPA == OP_N) ? As[m * RS_WIDE + kr] : As[kr * RS_LONG + m];
        const int n = 16 * (wn + 2 * i) + li;
        b[i] = (OPB == OP_N) ? Bs[kr * RS_LONG + n] : Bs[n * RS_WIDE + kr];
        na[i] = -a[i].y;
      }
      // Four product kinds over the (up to) 4 blocks: a chain is revisited only
      // after 8 MFMAs.  Skipped blocks are wave-uniform.
#pragma unroll
      for (int i = 0; i < NW; ++i)
#pragma unroll
        for (int j = 0; j < NW; ++j)
          if (live[i][j]) acc_re[i][j] = MATH::mfma(a[i].x, b[j].x, acc_re[i][j]);
#pragma unroll
      for (int i = 0; i < NW; ++i)
#pragma unroll
        for (int j = 0; j < NW; ++j)
          if (live[i][j]) acc_im[i][j] = MATH::mfma(a[i].x, b[j].y, acc_im[i][j]);
#pragma unroll
      for (int i = 0; i < NW; ++i)
#pragma unroll
        for (int j = 0; j < NW; ++j)
          if (live[i][j]) acc_re[i][j] = MATH::mfma(na[i], b[j].y, acc_re[i][j]);
#pragma unroll
      for (int i = 0; i < NW; ++i)
#pragma unroll
        for (int j = 0; j < NW; ++j)
          if (live[i][j]) acc_im[i][j] = MATH::mfma(a[i].y, b[j].x, acc_im[i][j]);
    }
  }

  // Epilogue (FP64): accumulator element v of lane l sits at MATH::row(l/16, v), column l%16.
  double2* __restrict__ C = d.tC ? d.tC[z] : d.C + (int64_t)z * d.sC;
  const double bs = d.bscal ? d.bscal[z] : 1.0;
  double2 coef[kMaxAddends];
  const double2* X[kMaxAddends];
#pragma unroll
  for (int q = 0; q < kMaxAddends; ++q) {
    coef[q] = d.add[q].coef;
    if (d.add[q].scale_by_batch) coef[q] = cmk(coef[q].x * bs, coef[q].y * bs);
    X[q] = d.add[q].tX ? d.add[q].tX[z] : (d.add[q].X ? d.add[q].X + (int64_t)z * d.add[q].stride : nullptr);
  }
  const double2 dg = d.diag_by_batch ? cmk(d.diag.x * bs, d.diag.y * bs) : d.diag;
#pragma unroll
  for (int i = 0; i < NW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      if (!live[i][j]) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + 16 * (wm + 2 * i) + MATH::row(lk, v);
        const int c = n0 + 16 * (wn + 2 * j) + li;
        if (r < M && c < N && !(skew && r > c)) {
          double2 out = cmul(d.alpha, cmk((double)acc_re[i][j][v], (double)acc_im[i][j][v]));
#pragma unroll
          for (int q = 0; q < kMaxAddends; ++q) {
            if (X[q] && (!d.add[q].diag || r == c)) {
              const double2 x = addend_value(X[q], d.add[q].diag, d.add[q].op, d.add[q].ld, r, c);
              out = cadd(out, cmul(coef[q], x));
            }
          }
          if (r == c) out = cadd(out, dg);
          // a skew-Hermitian diagonal is imaginary: its rounding-level real part is
          // dropped (left in, the lesser recurrences amplify it coherently)
          if (skew && r == c) out.x = 0.0;
          C[(int64_t)r * d.ldc + c] = out;
          if (skew && r < c) C[(int64_t)c * d.ldc + r] = cmk(-out.x, out.y);
        }
      }
    }
}

// The inversion's trailing update C = X + A B with K <= BK (one operand tile,
// A = Wp row-major M x K, B = Tp row-major K x N, the only addend X in C's own
// layout), in TM x TM tiles chosen as for the products (the sums and the final
// addition are the same for both, so are the results).  It is bound by reading and rewriting X, so it is a single-tile
// kernel without a K loop: the operand tiles are staged through LDS, then this
// thread's X values are requested (in the registers the staging used) and arrive
// while the MFMAs run.
template <int TM>
__global__ __launch_bounds__(NT) void zgemm_update_kernel(GemmDesc d) {
  // TM x TM output tile; each wave owns NW x NW blocks of 16 x 16
  constexpr int BM = TM, BN = TM, NW = TM / 32;
  constexpr int RS_LONG = TM + 1;
  constexpr int TILE_ELEMS = (BM * RS_WIDE > BK * RS_LONG) ? BM * RS_WIDE : BK * RS_LONG;
  __shared__ double2 As[TILE_ELEMS];
  __shared__ double2 Bs[TILE_ELEMS];
  const int tiles_m = (d.M + BM - 1) / BM;
  const int tiles_n = (d.N + BN - 1) / BN;
  const int per = tiles_m * tiles_n;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int z = tile / per;
  const int t = tile - z * per;
  const int m0 = (t % tiles_m) * BM;
  const int n0 = (t / tiles_m) * BN;
  // a tile whose columns all lie where B is zero keeps X (workgroup-uniform)
  if (n0 >= d.skip_c0 && min(n0 + BN, d.N) <= d.skip_c1) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1, li = lane & 15, lk = lane >> 4;
  const int M = d.M, N = d.N, K = d.K;
  const double2* __restrict__ A = d.tA ? d.tA[z] : d.A + (int64_t)z * d.sA;
  const double2* __restrict__ B = d.tB ? d.tB[z] : d.B + (int64_t)z * d.sB;
  const double2* __restrict__ X = d.add[0].tX ? d.add[0].tX[z] : d.add[0].X + (int64_t)z * d.add[0].stride;
  double2* __restrict__ C = d.tC ? d.tC[z] : d.C + (int64_t)z * d.sC;
  bool rv[NW], cv[NW];
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    rv[i] = m0 + 16 * (wm + 2 * i) < M;
    cv[i] = n0 + 16 * (wn + 2 * i) < N;
  }
  {
    TileLoader<BM, BK> la;
    TileLoader<BK, BN> lb;
    la.load(A, d.lda, m0, 0, M, K, tid);
    lb.load(B, d.ldb, 0, n0, K, N, tid);
    la.template store<false, MathF64>(As, RS_WIDE, tid);
    lb.template store<false, MathF64>(Bs, RS_LONG, tid);
  }
  double2 x[NW][NW][4];
#pragma unroll
  for (int i = 0; i < NW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + 16 * (wm + 2 * i) + MathF64::row(lk, v);
        const int c = n0 + 16 * (wn + 2 * j) + li;
        x[i][j][v] = (rv[i] && cv[j] && r < M && c < N) ? X[(int64_t)r * d.add[0].ld + c] : cmk(0.0, 0.0);
      }
  __syncthreads();
  d4 acc_re[NW][NW], acc_im[NW][NW];
#pragma unroll
  for (int i = 0; i < NW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      acc_re[i][j] = MathF64::zero();
      acc_im[i][j] = MathF64::zero();
    }
#pragma unroll
  for (int kk = 0; kk < BK; kk += 4) {
    const int kr = kk + lk;
    double2 a[NW], b[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      a[i] = As[(16 * (wm + 2 * i) + li) * RS_WIDE + kr];
      b[i] = Bs[kr * RS_LONG + 16 * (wn + 2 * i) + li];
    }
#pragma unroll
    for (int i = 0; i < NW; ++i)
#pragma unroll
      for (int j = 0; j < NW; ++j)
        if (rv[i] && cv[j]) {
          acc_re[i][j] = MathF64::mfma(a[i].x, b[j].x, acc_re[i][j]);
          acc_im[i][j] = MathF64::mfma(a[i].x, b[j].y, acc_im[i][j]);
          acc_re[i][j] = MathF64::mfma(-a[i].y, b[j].y, acc_re[i][j]);
          acc_im[i][j] = MathF64::mfma(a[i].y, b[j].x, acc_im[i][j]);
        }
  }
#pragma unroll
  for (int i = 0; i < NW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      if (!(rv[i] && cv[j])) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + 16 * (wm + 2 * i) + MathF64::row(lk, v);
        const int c = n0 + 16 * (wn + 2 * j) + li;
        if (r < M && c < N) C[(int64_t)r * d.ldc + c] = cmk(x[i][j][v].x + acc_re[i][j][v], x[i][j][v].y + acc_im[i][j][v]);
      }
    }
}

}  // namespace

template <int KIND, class MATH, int TM>
static void launch_kind_tm(const GemmDesc& d, hipStream_t s) {
  const int64_t total = (int64_t)((d.M + TM - 1) / TM) * ((d.N + TM - 1) / TM) * d.batch;
  dim3 grid((unsigned)total), block(NT);
  if (d.opA == OP_N && d.opB == OP_N) hipLaunchKernelGGL((zgemm_mfma_kernel<OP_N, OP_N, KIND, MATH, TM>), grid, block, 0, s, d);
  else if (d.opA == OP_N) hipLaunchKernelGGL((zgemm_mfma_kernel<OP_N, OP_C, KIND, MATH, TM>), grid, block, 0, s, d);
  else if (d.opB == OP_N) hipLaunchKernelGGL((zgemm_mfma_kernel<OP_C, OP_N, KIND, MATH, TM>), grid, block, 0, s, d);
  else hipLaunchKernelGGL((zgemm_mfma_kernel<OP_C, OP_C, KIND, MATH, TM>), grid, block, 0, s, d);
}

// 64 x 64 tiles, or 32 x 32 (the descriptor's tile when it names one, else the rule:
// 32 x 32 when the 64 x 64 tiling pads C by more than 8% (its edge
// tiles leave matrix cores idle: b = 416 is 6.5 tiles of 64 but 13 of 32; measured at
// 256 products of 416^3, 2.385 ms with 32 x 32 tiles against 2.621 ms) or when the
// launch has fewer than 4096 of them (16 per CU of the MI355X: at 8 to 64 energies of
// b = 416 the smaller tiles were 10% faster, at one energy 25%)).
constexpr int64_t kSmallTileBelow = 4096;
static bool small_tiles(const GemmDesc& d) {
  if (d.tile == 32) return true;
  if (d.tile == 64) return false;
  const int64_t tm64 = (d.M + 63) / 64, tn64 = (d.N + 63) / 64, tm32 = (d.M + 31) / 32, tn32 = (d.N + 31) / 32;
  const int64_t area64 = tm64 * tn64 * 4096, area32 = tm32 * tn32 * 1024;
  return tm64 * tn64 * d.batch < kSmallTileBelow || 100 * area64 > 108 * area32;
}
template <int KIND, class MATH>
static void launch_kind(const GemmDesc& d, hipStream_t s) {
  if (small_tiles(d)) launch_kind_tm<KIND, MATH, 32>(d, s);
  else launch_kind_tm<KIND, MATH, 64>(d, s);
}

static hipError_t launch_zgemm_mfma(const GemmDesc& d, hipStream_t s, int kind, bool fp32) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  if (d.skew && d.M != d.N) return hipErrorInvalidValue;
  // the 32 x 32 tiling has 4x the tiles of the 64 x 64 one
  const int64_t total = (int64_t)((d.M + 31) / 32) * ((d.N + 31) / 32) * d.batch;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  const int tiles = ((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN);
  dim3 grid((unsigned)((int64_t)tiles * d.batch)), block(NT);
  if (d.K == 0) {
    GemmDesc e = d;
    e.opA = OP_N; e.opB = OP_N;
    launch_kind<GEMM_ELEMENTWISE, MathF64>(e, s);
  } else if (kind == GEMM_INV_UPDATE) {
    if (d.skew) return hipErrorInvalidValue;
    // contract of the update form: C = X + A B, op N, K <= BK, X the only addend (op N)
    if (d.K > BK || d.opA != OP_N || d.opB != OP_N || d.alpha.x != 1.0 || d.alpha.y != 0.0 ||
        (!d.add[0].X && !d.add[0].tX) || d.add[0].op != OP_N || d.add[0].coef.x != 1.0 || d.add[0].coef.y != 0.0 ||
        d.add[0].scale_by_batch || d.add[0].diag || d.add[1].X || d.add[1].tX || d.add[2].X || d.add[2].tX || d.diag.x != 0.0 ||
        d.diag.y != 0.0)
      return hipErrorInvalidValue;
    if (small_tiles(d)) {
      const int64_t t32 = (int64_t)((d.M + 31) / 32) * ((d.N + 31) / 32) * d.batch;
      hipLaunchKernelGGL(zgemm_update_kernel<32>, dim3((unsigned)t32), block, 0, s, d);
    } else {
      hipLaunchKernelGGL(zgemm_update_kernel<64>, grid, block, 0, s, d);
    }
  } else if (fp32) {
    launch_kind<GEMM_PRODUCT, MathF32>(d, s);
  } else {
    launch_kind<GEMM_PRODUCT, MathF64>(d, s);
  }
  return hipGetLastError();
}

hipError_t launch_zgemm_f64(const GemmDesc& d, hipStream_t s, int kind) {
  return launch_zgemm_mfma(d, s, kind, false);
}

hipError_t launch_zgemm_f32(const GemmDesc& d, hipStream_t s) {
  return launch_zgemm_mfma(d, s, GEMM_PRODUCT, true);
}

}  // namespace qtx
