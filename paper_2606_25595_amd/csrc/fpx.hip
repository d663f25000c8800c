// FPX storage codec (Section V-A of the paper): FP64 <-> X-bit byte-aligned floats,
// X in {16, 24, 32, 40, 48, 56}, with FP32's 8-bit exponent and bias and X - 9
// significand bits, rounded to nearest even (IEEE-754); X = 32 is IEEE FP32.
//
// HBM-bound elementwise passes.  One thread takes a group of 8 consecutive
// elements: 64 bytes of FP64 on one side and exactly X bytes (X / 8 whole 64-bit
// words, since X is a multiple of 8) of codes on the other, so the packed side is
// written and read with aligned 8-byte accesses; a partial last group is written
// byte by byte.  Element i's code sits in bits [X i, X (i + 1)) of the little-endian
// byte stream.
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

template <int X>
__global__ __launch_bounds__(256) void fpx_encode_kernel(int64_t n, const double* __restrict__ x,
                                                          uint8_t* __restrict__ out) {
  constexpr int W = X / 8;   // 64-bit words per group of 8 elements
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i0 = g * 8;
  if (i0 >= n) return;
  const int cnt = (n - i0 >= 8) ? 8 : (int)(n - i0);
  uint64_t w[W];
#pragma unroll
  for (int k = 0; k < W; ++k) w[k] = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint64_t c = (j < cnt) ? fpx_code<X>(x[i0 + j]) : 0;
    const int bit = j * X, word = bit / 64, s = bit % 64;
    w[word] |= c << s;
    if (s + X > 64) w[word + 1] |= c >> (64 - s);
  }
  uint8_t* dst = out + g * X;
  if (cnt == 8) {
    uint64_t* d = (uint64_t*)dst;
#pragma unroll
    for (int k = 0; k < W; ++k) d[k] = w[k];
  } else {
    const int nbytes = cnt * (X / 8);
    for (int k = 0; k < nbytes; ++k) dst[k] = (uint8_t)(w[k / 8] >> (8 * (k % 8)));
  }
}

template <int X>
__global__ __launch_bounds__(256) void fpx_decode_kernel(int64_t n, const uint8_t* __restrict__ in,
                                                          double* __restrict__ y) {
  constexpr int W = X / 8;
  constexpr uint64_t kMask = (1ull << X) - 1;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i0 = g * 8;
  if (i0 >= n) return;
  const int cnt = (n - i0 >= 8) ? 8 : (int)(n - i0);
  const uint8_t* src = in + g * X;
  uint64_t w[W + 1];
  w[W] = 0;
  if (cnt == 8) {
    const uint64_t* s = (const uint64_t*)src;
#pragma unroll
    for (int k = 0; k < W; ++k) w[k] = s[k];
  } else {
#pragma unroll
    for (int k = 0; k < W; ++k) w[k] = 0;
    const int nbytes = cnt * (X / 8);
    for (int k = 0; k < nbytes; ++k) w[k / 8] |= (uint64_t)src[k] << (8 * (k % 8));
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int bit = j * X, word = bit / 64, s = bit % 64;
    uint64_t c = w[word] >> s;
    if (s + X > 64) c |= w[word + 1] << (64 - s);
    if (j < cnt) y[i0 + j] = fpx_value<X>(c & kMask);
  }
}

template <int X>
hipError_t launch_x(bool enc, int64_t n, const void* a, void* b, hipStream_t s) {
  const int64_t groups = (n + 7) / 8;
  const int64_t blocks = (groups + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (enc) hipLaunchKernelGGL(fpx_encode_kernel<X>, dim3((unsigned)blocks), dim3(256), 0, s, n, (const double*)a, (uint8_t*)b);
  else hipLaunchKernelGGL(fpx_decode_kernel<X>, dim3((unsigned)blocks), dim3(256), 0, s, n, (const uint8_t*)a, (double*)b);
  return hipGetLastError();
}

}  // namespace

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
