// FPX storage codec (Section V-A of the paper): FP64 <-> X-bit byte-aligned floats,
// X in {16, 24, 32, 40, 48, 56}, with FP32's 8-bit exponent and bias and X - 9
// significand bits, rounded to nearest even (IEEE-754); X = 32 is IEEE FP32.
//
// HBM-bound elementwise passes.  A group of 8 consecutive values is exactly X bytes
// (X / 8 whole 64-bit words, since X is a multiple of 8) of codes, so the packed side
// is read and written in aligned 8-byte words; a partial last tile is written byte by
// byte.  Element i's code sits in bits [X i, X (i + 1)) of the little-endian byte
// stream.
#include "qtx_internal.h"

namespace qtx {
namespace {

// The X-bit code of an FP64 value.  |x| = Mi 2^(E - 52) with Mi the 53-bit integer
// significand; the target keeps m = X - 9 fraction bits in the normal range
// (E >= -126) and counts units of 2^(-126 - m) below it.  Shifting Mi right to that
// unit and rounding to nearest even gives q; the code of a normal value is
// ((E + 126) << m) + q (a carry out of q moves into the exponent field), of a
// subnormal one q itself, and anything at or above the infinity code is infinite.
template <int X>
__device__ inline uint64_t fpx_code(double x) {
  constexpr int m = X - 9;
  constexpr uint64_t kInf = 255ull << m;
  const uint64_t u = __double_as_longlong(x);
  const uint64_t sign = u >> 63;
  const int e64 = (int)((u >> 52) & 0x7FF);
  const uint64_t f = u & ((1ull << 52) - 1);
  uint64_t code;
  if (e64 == 0x7FF) {
    code = f ? (kInf | (1ull << (m - 1))) : kInf;           // NaN (quiet) or infinity
  } else if (e64 == 0 && f == 0) {
    code = 0;
  } else {
    const uint64_t Mi = e64 ? (f | (1ull << 52)) : f;
    const int E = e64 ? e64 - 1023 : -1022;
    const int sh = (E >= -126) ? 52 - m : 52 - m + (-126 - E);   // >= 5
    uint64_t q = 0;
    if (sh < 64) {                                          // else |x| < half a unit: 0
      q = Mi >> sh;
      const uint64_t rem = Mi & ((1ull << sh) - 1), half = 1ull << (sh - 1);
      if (rem > half || (rem == half && (q & 1))) ++q;
    }
    code = ((E >= -126) ? ((uint64_t)(E + 126) << m) : 0) + q;
    if (code > kInf) code = kInf;
  }
  return code | (sign << (X - 1));
}

template <int X>
__device__ inline double fpx_value(uint64_t c) {
  constexpr int m = X - 9;
  const uint64_t sign = (c >> (X - 1)) & 1;
  const int be = (int)((c >> m) & 0xFF);
  const uint64_t f = c & ((1ull << m) - 1);
  uint64_t bits;
  if (be == 255) {
    bits = f ? 0x7FF8000000000000ull : 0x7FF0000000000000ull;
  } else if (be == 0) {
    // f 2^(-126 - m): a normal FP64 number (or zero); the scaling is exact
    const double v = (double)f * __longlong_as_double((uint64_t)(1023 - 126 - m) << 52);
    bits = __double_as_longlong(v);
  } else {
    bits = ((uint64_t)(be - 127 + 1023) << 52) | (f << (52 - m));
  }
  return __longlong_as_double(bits | (sign << 63));
}

// One workgroup of 256 threads converts a tile of 2048 consecutive values: 16 KB of
// FP64 and 256 X bytes of codes.  Both sides go through LDS so that every global load
// and store is contiguous across the wave (16-byte FP64 loads / stores, 8-byte code
// words); thread t packs or unpacks group t (values 8t .. 8t + 7) in LDS, reading its
// FP64 values in a rotated order to spread the LDS banks.
constexpr int kTile = 2048;

// Tile `tile` of the encode of n values x -> out (the body of the encode kernels).
template <int X>
__device__ inline void fpx_encode_tile(int64_t n, const double* __restrict__ x, uint8_t* __restrict__ out,
                                       int64_t tile) {
  constexpr int W = X / 8;   // 64-bit words per group of 8 values
  __shared__ __align__(16) double vin[kTile];
  __shared__ uint64_t wout[256 * W];
  const int t = threadIdx.x;
  const int64_t base = tile * kTile;
  if (base >= n) return;
  const int cnt = (n - base >= kTile) ? kTile : (int)(n - base);   // values in this tile
  if (cnt == kTile && ((uintptr_t)x & 15) == 0) {   // 16-byte loads need 16-byte alignment
    const double2* src = (const double2*)(x + base);
#pragma unroll
    for (int q = 0; q < kTile / 512; ++q) ((double2*)vin)[t + 256 * q] = src[t + 256 * q];
  } else {
    for (int e = t; e < kTile; e += 256) vin[e] = (e < cnt) ? x[base + e] : 0.0;
  }
  __syncthreads();
  uint64_t w[W];
#pragma unroll
  for (int k = 0; k < W; ++k) w[k] = 0;
#pragma unroll
  for (int jj = 0; jj < 8; ++jj) {
    const int j = (jj + t) & 7;
    const uint64_t c = fpx_code<X>(vin[8 * t + j]);
    // place value j's code at bits [j X, (j + 1) X) of the group
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int lo = 64 * k - j * X;                    // bit of the code at the word's bit 0
      if (lo >= X || lo <= -64) continue;
      w[k] |= (lo >= 0) ? (c >> lo) : (c << (-lo));
    }
  }
#pragma unroll
  for (int k = 0; k < W; ++k) wout[t * W + k] = w[k];
  __syncthreads();
  const int64_t obase = base / 8 * X;                   // byte offset of the tile's codes
  const int nbytes = cnt * (X / 8);
  uint8_t* dst = out + obase;
  if (nbytes % 8 == 0 && ((uintptr_t)dst & 7) == 0) {
    for (int q = t; q < nbytes / 8; q += 256) ((uint64_t*)dst)[q] = wout[q];
  } else {
    for (int q = t; q < nbytes; q += 256) dst[q] = (uint8_t)(wout[q / 8] >> (8 * (q % 8)));
  }
}

template <int X>
__global__ __launch_bounds__(256) void fpx_encode_kernel(int64_t n, const double* __restrict__ x,
                                                          uint8_t* __restrict__ out) {
  fpx_encode_tile<X>(n, x, out, blockIdx.x);
}

// Batch entry z = blockIdx.y: n values at x + z * sx into the byte buffer dst[z].
template <int X>
__global__ __launch_bounds__(256) void fpx_encode_entries_kernel(int64_t n, const double* __restrict__ x, int64_t sx,
                                                                  uint8_t* const* __restrict__ dst) {
  fpx_encode_tile<X>(n, x + (int64_t)blockIdx.y * sx, dst[blockIdx.y], blockIdx.x);
}

// The quiet-NaN code of every one of n values of the byte buffers dst[z] of failed
// entries (status[z] != 0).
template <int X>
__global__ __launch_bounds__(256) void fpx_nan_fill_entries_kernel(const int64_t* __restrict__ counts,
                                                                    uint8_t* const* __restrict__ dst,
                                                                    const int32_t* __restrict__ status) {
  const int z = blockIdx.y;
  if (status[z] == 0) return;
  const uint64_t code = fpx_code<X>(__builtin_nan(""));
  uint8_t* out = dst[z];
  const int64_t nbytes = 2 * counts[z] * (X / 8);   // counts: complex elements
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nbytes; q += (int64_t)gridDim.x * blockDim.x)
    out[q] = (uint8_t)(code >> (8 * (q % (X / 8))));
}

template <int X>
__global__ __launch_bounds__(256) void fpx_decode_kernel(int64_t n, const uint8_t* __restrict__ in,
                                                          double* __restrict__ y) {
  constexpr int W = X / 8;
  constexpr uint64_t kMask = (1ull << X) - 1;
  __shared__ uint64_t win[256 * W + 1];
  __shared__ __align__(16) double vout[kTile];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const int cnt = (n - base >= kTile) ? kTile : (int)(n - base);
  const int nbytes = cnt * (X / 8);
  const uint8_t* src = in + base / 8 * X;
  if (nbytes % 8 == 0) {
    for (int q = t; q < nbytes / 8; q += 256) win[q] = ((const uint64_t*)src)[q];
  } else {
    for (int q = t; q < 256 * W; q += 256) win[q] = 0;
    __syncthreads();
    for (int q = t; q < nbytes; q += 256) atomicOr((unsigned long long*)&win[q / 8], (unsigned long long)src[q] << (8 * (q % 8)));
  }
  __syncthreads();
  uint64_t w[W + 1];
#pragma unroll
  for (int k = 0; k < W; ++k) w[k] = win[t * W + k];
  w[W] = 0;
#pragma unroll
  for (int jj = 0; jj < 8; ++jj) {
    const int j = (jj + t) & 7;
    const int bit = j * X, word = bit / 64, sh = bit % 64;
    uint64_t c = 0;
#pragma unroll
    for (int k = 0; k < W; ++k)
      if (k == word) c = (w[k] >> sh) | (sh ? (w[k + 1] << (64 - sh)) : 0);
    vout[8 * t + j] = fpx_value<X>(c & kMask);
  }
  __syncthreads();
  if (cnt == kTile && ((uintptr_t)y & 15) == 0) {
    double2* dst = (double2*)(y + base);
#pragma unroll
    for (int q = 0; q < kTile / 512; ++q) dst[t + 256 * q] = ((const double2*)vout)[t + 256 * q];
  } else {
    for (int e = t; e < cnt; e += 256) y[base + e] = vout[e];
  }
}

template <int X>
hipError_t launch_x(bool enc, int64_t n, const void* a, void* b, hipStream_t s) {
  const int64_t blocks = (n + kTile - 1) / kTile;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (enc) hipLaunchKernelGGL(fpx_encode_kernel<X>, dim3((unsigned)blocks), dim3(256), 0, s, n, (const double*)a, (uint8_t*)b);
  else hipLaunchKernelGGL(fpx_decode_kernel<X>, dim3((unsigned)blocks), dim3(256), 0, s, n, (const uint8_t*)a, (double*)b);
  return hipGetLastError();
}

template <int X>
hipError_t launch_entries_x(int64_t n, const double* x, int64_t sx, uint8_t* const* dst, int count,
                            const int64_t* counts, const int32_t* status, hipStream_t s) {
  if (status) {
    hipLaunchKernelGGL(fpx_nan_fill_entries_kernel<X>, dim3(256, count), dim3(256), 0, s, counts, dst, status);
  } else {
    const int64_t blocks = (n + kTile - 1) / kTile;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fpx_encode_entries_kernel<X>, dim3((unsigned)blocks, count), dim3(256), 0, s, n, x, sx, dst);
  }
  return hipGetLastError();
}

hipError_t launch_entries(int bits, int64_t n, const double* x, int64_t sx, uint8_t* const* dst, int count,
                          const int64_t* counts, const int32_t* status, hipStream_t s) {
  if ((!status && n <= 0) || count <= 0) return hipSuccess;
  if (!dst || (!status && !x)) return hipErrorInvalidValue;
  switch (bits) {
    case 16: return launch_entries_x<16>(n, x, sx, dst, count, counts, status, s);
    case 24: return launch_entries_x<24>(n, x, sx, dst, count, counts, status, s);
    case 32: return launch_entries_x<32>(n, x, sx, dst, count, counts, status, s);
    case 40: return launch_entries_x<40>(n, x, sx, dst, count, counts, status, s);
    case 48: return launch_entries_x<48>(n, x, sx, dst, count, counts, status, s);
    case 56: return launch_entries_x<56>(n, x, sx, dst, count, counts, status, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_fpx_encode_entries(int bits, int64_t n, const double* x, int64_t sx, uint8_t* const* dst, int count,
                                     hipStream_t s) {
  return launch_entries(bits, n, x, sx, dst, count, nullptr, nullptr, s);
}

hipError_t launch_fpx_nan_fill_entries(int bits, const int64_t* counts, uint8_t* const* dst, int count,
                                       const int32_t* status, hipStream_t s) {
  return launch_entries(bits, 0, nullptr, 0, dst, count, counts, status, s);
}

bool fpx_supported(int bits) {
  return bits == 16 || bits == 24 || bits == 32 || bits == 40 || bits == 48 || bits == 56;
}

hipError_t launch_fpx(bool encode, int bits, int64_t n, const void* src, void* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (bits) {
    case 16: return launch_x<16>(encode, n, src, dst, s);
    case 24: return launch_x<24>(encode, n, src, dst, s);
    case 32: return launch_x<32>(encode, n, src, dst, s);
    case 40: return launch_x<40>(encode, n, src, dst, s);
    case 48: return launch_x<48>(encode, n, src, dst, s);
    case 56: return launch_x<56>(encode, n, src, dst, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace qtx
