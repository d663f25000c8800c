// Complex GEMM from exact 16-bit slice products (Ozaki scheme I, Section II-D
// of the paper) on the gfx950 FP16/BF16 matrix cores, recombined in FP64.
//
// Split (two passes per operand): an operand is viewed as R rows of K values,
// k contiguous (rows of op(A), or columns of op(B)).  Every row gets a
// power-of-two scale 2^e with max|x| 2^-e in [1/4, 1/2) over the row (real and
// imaginary parts share it).  The scaled value r = x 2^-e is written as NS
// signed digits of W bits,
//     r = sum_s sigma_s 2^{-W s},  sigma_s = rint(...) in [-2^{W-1}, 2^{W-1}],
// digit s stored as sigma_s 2^{-W(s-1)} in the 16-bit format (exact: FP16 holds
// W = 10 bit digits, BF16 W = 8 bit digits; FP16 is limited to NS <= 3 so the
// weighted digits stay representable).  Rounding is to nearest even throughout.
//
// Product: sum_k A B = 2^{eA + eB - 2W} * sum_{s,t} sum_k sigma^A_s sigma^B_t
// 2^{-W(s+t-2)}, keeping the pairs with s + t <= NS + 1.  Three FP32
// accumulators per output: the s + t = 2 pairs and the s + t = 3 pairs hold
// integers (times 2^-W) whose sums stay below 2^24 for up to FLUSH_K terms, so
// the matrix cores add them exactly; all pairs with s + t >= 4 share a third
// accumulator whose rounding is 2^-24 of a term already 2^-2W smaller.  Every
// FLUSH_K values of k (512 for BF16, 64 for FP16) the accumulators are scaled by
// 2^{eA + eB - 2W} and added into FP64 sums; when K <= FLUSH_K there is a
// single conversion at the end.  Complex arithmetic uses four real products (4M).
//
// Layout of a split operand, per batch entry: digits [KT][R][NS*2][32] as 16-bit
// words (q = 2 s + part, part 0 = real, 1 = imaginary), KT = ceil(K / 32), and
// one exponent per row [R] (int32).  A GEMM tile (64 rows x one 32-wide strip)
// is one contiguous block.
#include <type_traits>

#include "qtx_internal.h"

namespace qtx {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));   // 16 bytes: 8 digits

namespace {

constexpr int KS = 32;     // K strip = MFMA K of the 16-bit instructions
constexpr int NT = 256;

__device__ inline int xcd_remap(int pid, int total) {
  const int nx = 8;
  int per = total / nx, rem = total % nx;
  int x = pid % nx, local = pid / nx;
  return (x < rem) ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

template <int FMT>
struct DigitFmt;
template <>
struct DigitFmt<0> {   // FP16, 10-bit digits
  static constexpr int W = 10;
  static __device__ inline uint16_t bits(double v) {
    _Float16 h = (_Float16)(float)v;
    return __builtin_bit_cast(uint16_t, h);
  }
};
template <>
struct DigitFmt<1> {   // BF16, 8-bit digits
  static constexpr int W = 8;
  static __device__ inline uint16_t bits(double v) {
    // v has at most 8 significant bits, so the upper half of its FP32 pattern is exact
    return (uint16_t)(__builtin_bit_cast(uint32_t, (float)v) >> 16);
  }
};

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, class F>
__device__ inline void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

__device__ inline double pow2(int e) {
  e = e < -1020 ? -1020 : (e > 1020 ? 1020 : e);
  return __builtin_bit_cast(double, (uint64_t)(e + 1023) << 52);
}

// ---------------------------------------------------------------- split pass
// Two kernels over 64-row blocks of S = op(X): S[r][k] = X[r][k] (trans = 0) or
// X[k][r] (trans = 1), conjugated when conj = 1.  The first finds the row
// exponents (looping over the 32-wide strips), the second writes the digits of
// one strip per workgroup.  Both load a strip with coalesced reads into LDS.
__device__ inline void load_strip(const SplitDesc& sd, const double2* X, int r0, int k0, int tid,
                                  double2 (*tile)[KS + 1]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int e = tid + NT * j;
    double2 v = cmk(0.0, 0.0);
    int r, k;
    if (!sd.trans) { r = e / KS; k = e % KS; }
    else { k = e / 64; r = e % 64; }
    if (r0 + r < sd.rows && k0 + k < sd.cols)
      v = sd.trans ? X[(int64_t)(k0 + k) * sd.ld + r0 + r] : X[(int64_t)(r0 + r) * sd.ld + k0 + k];
    tile[r][k] = sd.conj ? cconj(v) : v;
  }
}

__global__ __launch_bounds__(NT) void split_exp_kernel(SplitDesc sd) {
  __shared__ double2 tile[64][KS + 1];
  const int z = blockIdx.y;
  const int r0 = blockIdx.x * 64;
  const int tid = threadIdx.x;
  const double2* X = sd.tX ? sd.tX[z] : sd.X + (int64_t)z * sd.stride;
  const int r = tid >> 2, kq = (tid & 3) * 8;
  double mx = 0.0;
  int bad = 0;   // NaN or Inf in the row (fmax alone would skip a NaN)
  for (int k0 = 0; k0 < sd.cols; k0 += KS) {
    __syncthreads();
    load_strip(sd, X, r0, k0, tid, tile);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double2 v = tile[r][kq + j];
      bad |= !(isfinite(v.x) && isfinite(v.y));
      mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
    }
  }
  mx = fmax(mx, __shfl_xor(mx, 1));
  mx = fmax(mx, __shfl_xor(mx, 2));
  bad |= __shfl_xor(bad, 1);
  bad |= __shfl_xor(bad, 2);
  int e = 0;
  if (bad) e = kExpNonFinite;
  else if (mx > 0.0 && mx <= 1.7e308) e = ilogb(mx) + 2;   // max * 2^-e in [1/4, 1/2)
  if ((tid & 3) == 0 && r0 + r < sd.rows) sd.E[(int64_t)z * sd.e_stride + r0 + r] = e;
}

template <int FMT, int NS>
__global__ __launch_bounds__(NT) void split_kernel(SplitDesc sd) {
  constexpr int W = DigitFmt<FMT>::W;
  constexpr int NQ = 2 * NS;
  __shared__ double2 tile[64][KS + 1];
  const int z = blockIdx.z;
  const int kt = blockIdx.y;
  const int r0 = blockIdx.x * 64;
  const int tid = threadIdx.x;
  const double2* X = sd.tX ? sd.tX[z] : sd.X + (int64_t)z * sd.stride;
  load_strip(sd, X, r0, kt * KS, tid, tile);
  __syncthreads();
  // thread -> row tid/4, k = 8 (tid%4) .. +7
  const int r = tid >> 2, kq = (tid & 3) * 8;
  if (r0 + r >= sd.rows) return;
  const int er = sd.E[(int64_t)z * sd.e_stride + r0 + r];
  const bool fin = er != kExpNonFinite;   // a non-finite row gets zero digits
  const double sc = fin ? pow2(-er) : 0.0;
  uint16_t dig[NQ][8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double2 v = tile[r][kq + j];
    double part[2] = {fin ? v.x * sc : 0.0, fin ? v.y * sc : 0.0};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double rem = part[c];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const double t = rem * (double)(1 << W);
        const double sg = rint(t);
        rem = t - sg;                                   // exact
        dig[2 * s + c][j] = DigitFmt<FMT>::bits(sg * pow2(-W * s));
      }
    }
  }
  uint16_t* out = (uint16_t*)sd.S + (int64_t)z * sd.s_stride + ((int64_t)kt * sd.rows + r0 + r) * NQ * KS + kq;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    uint4 pk;
    pk.x = (uint32_t)dig[q][0] | ((uint32_t)dig[q][1] << 16);
    pk.y = (uint32_t)dig[q][2] | ((uint32_t)dig[q][3] << 16);
    pk.z = (uint32_t)dig[q][4] | ((uint32_t)dig[q][5] << 16);
    pk.w = (uint32_t)dig[q][6] | ((uint32_t)dig[q][7] << 16);
    *(uint4*)(out + q * KS) = pk;
  }
}

// ---------------------------------------------------------------- product kernel
template <int FMT>
__device__ inline f4 mfma16(u4 a, u4 b, f4 c) {
  if constexpr (FMT == 0)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a), __builtin_bit_cast(b8, b), c, 0, 0, 0);
}

// Strips (of 32 k) between FP64 flushes: the exact groups stay below 2^24.
// BF16: |sigma sigma| <= 2^14, two pairs in group 3 -> 512 k.  FP16: 2^18 -> 32 k.
template <int FMT>
constexpr int flush_strips() { return FMT == 1 ? 16 : 1; }

// TM x TM output tile (TM = 64: each wave owns 2 x 2 blocks of 16 x 16; TM = 32: one
// block per wave); both tilings sum every element in the same order, so they give the
// same bits.
template <int FMT, int NS, bool ONEFLUSH, int TM>
__global__ __launch_bounds__(NT) void zgemm_split_kernel(SplitGemmDesc g) {
  constexpr int W = DigitFmt<FMT>::W;
  constexpr int FLUSH = flush_strips<FMT>();
  constexpr int NQ = 2 * NS;
  constexpr int BM = TM, BN = TM, NW = TM / 32;
  constexpr int ROW_U4 = NQ * KS / 8 + 1;         // u4 per LDS row (+1 pad: conflict-free reads)
  constexpr int TILE_U4 = TM * NQ * KS / 8;       // u4 per operand tile in global memory
  constexpr int PER_T = TILE_U4 / NT;             // u4 per thread
  static_assert(TILE_U4 % NT == 0, "tile copy split");
  __shared__ u4 As[TM * ROW_U4];
  __shared__ u4 Bs[TM * ROW_U4];
  __shared__ int Ea[TM], Eb[TM];

  const GemmDesc& d = g.d;
  const int tiles_m = (d.M + BM - 1) / BM;
  const int tiles_n = (d.N + BN - 1) / BN;
  const int per = tiles_m * tiles_n;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int z = tile / per;
  const int t = tile - z * per;
  const int m0 = (t % tiles_m) * BM;
  const int n0 = (t / tiles_m) * BN;
  const int M = d.M, N = d.N;
  const int KT = (d.K + KS - 1) / KS;

  const u4* SA = (const u4*)((const uint16_t*)g.SA + (int64_t)z * g.sa_stride);
  const u4* SB = (const u4*)((const uint16_t*)g.SB + (int64_t)z * g.sb_stride);
  const int32_t* EA = g.EA + (int64_t)z * g.ea_stride;
  const int32_t* EB = g.EB + (int64_t)z * g.eb_stride;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;
  bool rv[NW], cv[NW];
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    rv[i] = m0 + 16 * (wm + 2 * i) < M;
    cv[i] = n0 + 16 * (wn + 2 * i) < N;
  }

  f4 acc[NW][NW][2][3];   // [i][j][re/im][group]
  double sum[NW][NW][2][4];
#pragma unroll
  for (int i = 0; i < NW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[i][j][c][q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int v = 0; v < 4; ++v) sum[i][j][c][v] = 0.0;
      }
  // row / column exponents of this tile (one per row of op(A), column of op(B))
  if (tid < TM) Ea[tid] = (m0 + tid < M) ? EA[m0 + tid] : 0;
  else if (tid < 2 * TM) Eb[tid - TM] = (n0 + tid - TM < N) ? EB[n0 + tid - TM] : 0;
  // FP64 sums += 2^{eA + eB - 2W} (g2 + g3 + g4), then the groups restart.  16-bit
  // MFMA result layout: lane l, element v -> row 4(l/16) + v, column l%16.
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < NW; ++i)
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const int eb = Eb[16 * (wn + 2 * j) + li];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ea = Ea[16 * (wm + 2 * i) + 4 * lk + v];
          // non-finite rows / columns have zero digits; their outputs are set to NaN below
          const double sc = (ea == kExpNonFinite || eb == kExpNonFinite) ? 0.0 : pow2(ea + eb - 2 * W);
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const double part = ((double)acc[i][j][c][0][v] + (double)acc[i][j][c][1][v]) + (double)acc[i][j][c][2][v];
            sum[i][j][c][v] = fma(sc, part, sum[i][j][c][v]);
          }
        }
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int q = 0; q < 3; ++q) acc[i][j][c][q] = f4{0.f, 0.f, 0.f, 0.f};
      }
  };

  // next strip prefetched into registers (a plain struct keeps the arrays in VGPRs)
  struct Prefetch {
    u4 a[PER_T], b[PER_T];
  } pf;
  const u4 zero4 = {0u, 0u, 0u, 0u};
#define QTX_GLOAD(KTV)                                                                         \
  do {                                                                                         \
    const int kt_ = (KTV);                                                                     \
    _Pragma("unroll") for (int p = 0; p < PER_T; ++p) {                                        \
      const int u = tid + NT * p;                                                              \
      const int row = u / (NQ * KS / 8);                                                       \
      pf.a[p] = (m0 + row < M) ? SA[((int64_t)kt_ * M + m0) * (NQ * KS / 8) + u] : zero4;     \
      pf.b[p] = (n0 + row < N) ? SB[((int64_t)kt_ * N + n0) * (NQ * KS / 8) + u] : zero4;     \
    }                                                                                          \
  } while (0)

  if (KT > 0) QTX_GLOAD(0);
  for (int kt = 0; kt < KT; ++kt) {
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER_T; ++p) {
      const int u = tid + NT * p;
      const int row = u / (NQ * KS / 8), col = u % (NQ * KS / 8);
      As[row * ROW_U4 + col] = pf.a[p];
      Bs[row * ROW_U4 + col] = pf.b[p];
    }
    __syncthreads();
    if (kt + 1 < KT) QTX_GLOAD(kt + 1);

    // Slice pairs (s, t) with s + t <= NS + 1, grouped 2 / 3 / >= 4 (all indices
    // compile-time).  Every A digit fragment is read from LDS once per strip and
    // every B digit fragment once per strip; blocks outside C run on the zero
    // padding, so the MFMA stream has no branches.
    u4 a[NS][NW][2], an[NS][NW];
    static_for<0, NS>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const int row = 16 * (wm + 2 * i) + li;
        a[s][i][0] = As[row * ROW_U4 + (2 * s + 0) * (KS / 8) + lk];
        a[s][i][1] = As[row * ROW_U4 + (2 * s + 1) * (KS / 8) + lk];
        an[s][i] = a[s][i][1] ^ (u4){0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
      }
    });
    static_for<0, NS>([&](auto tc) {
      constexpr int tt = decltype(tc)::value;
      u4 b[NW][2];
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const int col = 16 * (wn + 2 * j) + li;
        b[j][0] = Bs[col * ROW_U4 + (2 * tt + 0) * (KS / 8) + lk];
        b[j][1] = Bs[col * ROW_U4 + (2 * tt + 1) * (KS / 8) + lk];
      }
      static_for<0, NS>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        if constexpr (s + tt + 2 <= NS + 1) {
          constexpr int grp = (s + tt == 0) ? 0 : (s + tt == 1 ? 1 : 2);
#pragma unroll
          for (int i = 0; i < NW; ++i)
#pragma unroll
            for (int j = 0; j < NW; ++j) acc[i][j][0][grp] = mfma16<FMT>(a[s][i][0], b[j][0], acc[i][j][0][grp]);
#pragma unroll
          for (int i = 0; i < NW; ++i)
#pragma unroll
            for (int j = 0; j < NW; ++j) acc[i][j][1][grp] = mfma16<FMT>(a[s][i][0], b[j][1], acc[i][j][1][grp]);
#pragma unroll
          for (int i = 0; i < NW; ++i)
#pragma unroll
            for (int j = 0; j < NW; ++j) acc[i][j][0][grp] = mfma16<FMT>(an[s][i], b[j][1], acc[i][j][0][grp]);
#pragma unroll
          for (int i = 0; i < NW; ++i)
#pragma unroll
            for (int j = 0; j < NW; ++j) acc[i][j][1][grp] = mfma16<FMT>(a[s][i][1], b[j][0], acc[i][j][1][grp]);
        }
      });
    });
    if (!ONEFLUSH && (kt + 1) % FLUSH == 0 && kt + 1 < KT) flush();
  }
  flush();

  // epilogue in FP64 (same addend semantics as the FP64 kernels)
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
      if (!(rv[i] && cv[j])) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + 16 * (wm + 2 * i) + 4 * lk + v;
        const int c = n0 + 16 * (wn + 2 * j) + li;
        if (r < M && c < N) {
          const bool nf = Ea[16 * (wm + 2 * i) + 4 * lk + v] == kExpNonFinite || Eb[16 * (wn + 2 * j) + li] == kExpNonFinite;
          const double nan = __builtin_nan("");
          double2 out = nf ? cmk(nan, nan) : cmul(d.alpha, cmk(sum[i][j][0][v], sum[i][j][1][v]));
#pragma unroll
          for (int q = 0; q < kMaxAddends; ++q) {
            if (X[q] && (!d.add[q].diag || r == c)) {
              const double2 x = addend_value(X[q], d.add[q].diag, d.add[q].op, d.add[q].ld, r, c);
              out = cadd(out, cmul(coef[q], x));
            }
          }
          if (r == c) out = cadd(out, dg);
          C[(int64_t)r * d.ldc + c] = out;
        }
      }
    }
}

template <int FMT, int NS>
hipError_t launch_split_t(const SplitDesc& sd, hipStream_t s) {
  hipLaunchKernelGGL(split_exp_kernel, dim3((sd.rows + 63) / 64, sd.batch), dim3(NT), 0, s, sd);
  dim3 grid((sd.rows + 63) / 64, (sd.cols + KS - 1) / KS, sd.batch);
  hipLaunchKernelGGL((split_kernel<FMT, NS>), grid, dim3(NT), 0, s, sd);
  return hipGetLastError();
}

template <int FMT, int NS, int TM>
hipError_t launch_gemm_tm(const SplitGemmDesc& g, hipStream_t s) {
  const GemmDesc& d = g.d;
  const int64_t total = (int64_t)((d.M + TM - 1) / TM) * ((d.N + TM - 1) / TM) * d.batch;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  const int KT = (d.K + KS - 1) / KS;
  if (KT <= flush_strips<FMT>())
    hipLaunchKernelGGL((zgemm_split_kernel<FMT, NS, true, TM>), dim3((unsigned)total), dim3(NT), 0, s, g);
  else
    hipLaunchKernelGGL((zgemm_split_kernel<FMT, NS, false, TM>), dim3((unsigned)total), dim3(NT), 0, s, g);
  return hipGetLastError();
}

// 64 x 64 tiles unless the descriptor asks for 32 x 32 (the autotuner's choice).
template <int FMT, int NS>
hipError_t launch_gemm_t(const SplitGemmDesc& g, hipStream_t s) {
  if (g.d.tile == 32) return launch_gemm_tm<FMT, NS, 32>(g, s);
  return launch_gemm_tm<FMT, NS, 64>(g, s);
}

}  // namespace

bool split_supported(int fmt, int ns) {
  if (fmt == 0) return ns >= 2 && ns <= 3;
  if (fmt == 1) return ns >= 2 && ns <= 5;
  return false;
}

size_t split_bytes(int rows, int cols, int ns, int batch) {
  const size_t kt = (size_t)(cols + KS - 1) / KS;
  const size_t dig = kt * rows * 2 * ns * KS * sizeof(uint16_t);
  const size_t ex = (size_t)rows * sizeof(int32_t);
  return ((dig + 255) / 256 * 256 + (ex + 255) / 256 * 256) * batch;
}

int64_t split_digit_stride(int rows, int cols, int ns) {
  return (int64_t)((cols + KS - 1) / KS) * rows * 2 * ns * KS;
}

int64_t split_exp_stride(int rows, int cols) { (void)cols; return (int64_t)rows; }

hipError_t launch_split(const SplitDesc& sd, int fmt, int ns, hipStream_t s) {
  if (sd.rows <= 0 || sd.cols <= 0 || sd.batch <= 0) return hipSuccess;
#define QTX_SPLIT_CASE(F, N) \
  if (fmt == F && ns == N) return launch_split_t<F, N>(sd, s);
  QTX_SPLIT_CASE(0, 2) QTX_SPLIT_CASE(0, 3)
  QTX_SPLIT_CASE(1, 2) QTX_SPLIT_CASE(1, 3) QTX_SPLIT_CASE(1, 4) QTX_SPLIT_CASE(1, 5)
#undef QTX_SPLIT_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_split_exp(const SplitDesc& sd, hipStream_t s) {
  if (sd.rows <= 0 || sd.cols <= 0 || sd.batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_exp_kernel, dim3((sd.rows + 63) / 64, sd.batch), dim3(NT), 0, s, sd);
  return hipGetLastError();
}

hipError_t launch_zgemm_split(const SplitGemmDesc& g, int fmt, int ns, hipStream_t s) {
  if (g.d.M <= 0 || g.d.N <= 0 || g.d.batch <= 0) return hipSuccess;
#define QTX_GEMM_CASE(F, N) \
  if (fmt == F && ns == N) return launch_gemm_t<F, N>(g, s);
  QTX_GEMM_CASE(0, 2) QTX_GEMM_CASE(0, 3)
  QTX_GEMM_CASE(1, 2) QTX_GEMM_CASE(1, 3) QTX_GEMM_CASE(1, 4) QTX_GEMM_CASE(1, 5)
#undef QTX_GEMM_CASE
  return hipErrorInvalidValue;
}

}  // namespace qtx
