// Batched complex GEMM on the gfx950 FP64 matrix cores (v_mfma_f64_16x16x4_f64).
//
// The complex block products dominate the selected solve (Section IV of the
// paper); this is the FP64 reference scheme.  A complex product is four real
// MFMA chains: C_re += A_re B_re - A_im B_im, C_im += A_re B_im + A_im B_re.
//
// Tiling: a 256-thread workgroup computes a 64 x 64 complex tile of C; its four
// waves each own a 32 x 32 sub-tile (2 x 2 MFMA blocks of 16 x 16, with separate
// real and imaginary accumulators: 8 independent MFMA chains per wave, so
// consecutive MFMAs never wait on each other).  K advances in steps of 16
// complex elements staged through LDS as interleaved (re, im) pairs laid out
// k-major, so that the MFMA operand of lane l (row l%16, k l/16) is one 16-byte
// LDS read.  Global loads are coalesced along the contiguous dimension of each
// operand and transposed into LDS when needed (op = N for A, op = C for B); the
// next K tile is prefetched into registers while the current one is consumed.
// Tiles are assigned XCD-aware: consecutive workgroup ids land on different
// XCDs, so tile ids are remapped so that all tiles of one batch entry execute on
// one XCD and share its L2.
#include "qtx_internal.h"

namespace qtx {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 64, BN = 64, BK = 16, PAD = 1, NT = 256;

__device__ inline int xcd_remap(int pid, int total) {
  // Workgroup `pid` is dispatched to XCD pid % 8.  Give XCD x a contiguous
  // range of logical tiles (bijective for any total).
  const int nx = 8;
  int per = total / nx, rem = total % nx;
  int x = pid % nx, local = pid / nx;
  return (x < rem) ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

__device__ inline double2 ldg_or_zero(const double2* p, bool ok) {
  return ok ? *p : cmk(0.0, 0.0);
}

// KIND only separates kernel symbols by use (block products of the solve, the
// inversion's trailing update, elementwise assembly with K = 0) so profilers
// report them apart; the code is the same.
template <int OPA, int OPB, int KIND>
__global__ __launch_bounds__(NT) void zgemm_f64_kernel(GemmDesc d) {
  __shared__ double2 As[BK][BM + PAD];
  __shared__ double2 Bs[BK][BN + PAD];

  const int tiles_m = (d.M + BM - 1) / BM;
  const int tiles_n = (d.N + BN - 1) / BN;
  const int per = tiles_m * tiles_n;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int z = tile / per;
  const int t = tile - z * per;
  const int m0 = (t % tiles_m) * BM;
  const int n0 = (t / tiles_m) * BN;

  const double2* __restrict__ A = d.A + (int64_t)z * d.sA;
  const double2* __restrict__ B = d.B + (int64_t)z * d.sB;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  d4 acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc_re[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      acc_im[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }

  double2 ra[4], rb[4];
  const int M = d.M, N = d.N, K = d.K;

  // Global -> registers for the K tile starting at k0.
  auto gload = [&](int k0) {
    if (OPA == OP_N) {          // A is M x K: thread -> row tid/4, 4 consecutive k
      int m = m0 + (tid >> 2), kb = k0 + (tid & 3) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) ra[j] = ldg_or_zero(A + (int64_t)m * d.lda + kb + j, m < M && kb + j < K);
    } else {                    // source is K x M: thread -> k tid/16, 4 consecutive m
      int k = k0 + (tid >> 4), mb = m0 + (tid & 15) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) ra[j] = ldg_or_zero(A + (int64_t)k * d.lda + mb + j, k < K && mb + j < M);
    }
    if (OPB == OP_N) {          // B is K x N: thread -> k tid/16, 4 consecutive n
      int k = k0 + (tid >> 4), nb = n0 + (tid & 15) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) rb[j] = ldg_or_zero(B + (int64_t)k * d.ldb + nb + j, k < K && nb + j < N);
    } else {                    // source is N x K: thread -> n tid/4, 4 consecutive k
      int n = n0 + (tid >> 2), kb = k0 + (tid & 3) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) rb[j] = ldg_or_zero(B + (int64_t)n * d.ldb + kb + j, n < N && kb + j < K);
    }
  };
  // Registers -> LDS (k-major, conjugated for op = C).
  auto lstore = [&]() {
    if (OPA == OP_N) {
      int m = tid >> 2, kb = (tid & 3) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) As[kb + j][m] = ra[j];
    } else {
      int k = tid >> 4, mb = (tid & 15) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) As[k][mb + j] = cconj(ra[j]);
    }
    if (OPB == OP_N) {
      int k = tid >> 4, nb = (tid & 15) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) Bs[k][nb + j] = rb[j];
    } else {
      int n = tid >> 2, kb = (tid & 3) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) Bs[kb + j][n] = cconj(rb[j]);
    }
  };

  const int nk = (K + BK - 1) / BK;
  if (nk > 0) gload(0);
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
    lstore();
    __syncthreads();
    if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const int li = lane & 15;
      double2 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kr][wm * 32 + i * 16 + li];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kr][wn * 32 + j * 16 + li];
      double na[2] = {-a[0].y, -a[1].y};
      // Four product kinds, each over the 4 blocks: a chain is revisited only
      // after 8 MFMAs.
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc_re[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].y, acc_im[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(na[i], b[j].y, acc_re[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].x, acc_im[i][j], 0, 0, 0);
    }
  }

  // Epilogue.  f64 16x16x4 result layout: lane l, element v -> row l/16 + 4v, col l%16.
  double2* __restrict__ C = d.C + (int64_t)z * d.sC;
  const double bs = d.bscal ? d.bscal[z] : 1.0;
  double2 coef[kMaxAddends];
  const double2* X[kMaxAddends];
#pragma unroll
  for (int q = 0; q < kMaxAddends; ++q) {
    coef[q] = d.add[q].coef;
    if (d.add[q].scale_by_batch) coef[q] = cmk(coef[q].x * bs, coef[q].y * bs);
    X[q] = d.add[q].X ? d.add[q].X + (int64_t)z * d.add[q].stride : nullptr;
  }
  const double2 dg = d.diag_by_batch ? cmk(d.diag.x * bs, d.diag.y * bs) : d.diag;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + wm * 32 + i * 16 + (lane >> 4) + 4 * v;
        const int c = n0 + wn * 32 + j * 16 + (lane & 15);
        if (r < M && c < N) {
          double2 out = cmul(d.alpha, cmk(acc_re[i][j][v], acc_im[i][j][v]));
#pragma unroll
          for (int q = 0; q < kMaxAddends; ++q) {
            if (X[q]) {
              double2 x = (d.add[q].op == OP_N) ? X[q][(int64_t)r * d.add[q].ld + c]
                                                 : cconj(X[q][(int64_t)c * d.add[q].ld + r]);
              out = cadd(out, cmul(coef[q], x));
            }
          }
          if (r == c) out = cadd(out, dg);
          C[(int64_t)r * d.ldc + c] = out;
        }
      }
}

}  // namespace

template <int KIND>
static void launch_kind(const GemmDesc& d, dim3 grid, dim3 block, hipStream_t s) {
  if (d.opA == OP_N && d.opB == OP_N) hipLaunchKernelGGL((zgemm_f64_kernel<OP_N, OP_N, KIND>), grid, block, 0, s, d);
  else if (d.opA == OP_N) hipLaunchKernelGGL((zgemm_f64_kernel<OP_N, OP_C, KIND>), grid, block, 0, s, d);
  else if (d.opB == OP_N) hipLaunchKernelGGL((zgemm_f64_kernel<OP_C, OP_N, KIND>), grid, block, 0, s, d);
  else hipLaunchKernelGGL((zgemm_f64_kernel<OP_C, OP_C, KIND>), grid, block, 0, s, d);
}

hipError_t launch_zgemm_f64(const GemmDesc& d, hipStream_t s, int kind) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  const int tiles = ((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN);
  const int64_t total = (int64_t)tiles * d.batch;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)total), block(NT);
  if (d.K == 0) {
    GemmDesc e = d;
    e.opA = OP_N; e.opB = OP_N;
    launch_kind<GEMM_ELEMENTWISE>(e, grid, block, s);
  } else if (kind == GEMM_INV_UPDATE) {
    launch_kind<GEMM_INV_UPDATE>(d, grid, block, s);
  } else {
    launch_kind<GEMM_PRODUCT>(d, grid, block, s);
  }
  return hipGetLastError();
}

}  // namespace qtx
