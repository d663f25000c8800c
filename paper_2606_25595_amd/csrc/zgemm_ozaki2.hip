// Complex GEMM emulated with INT8 modular products (Ozaki scheme II, the
// emulation of Section V-A), on the gfx950 v_mfma_i32_32x32x32_i8 matrix cores.
//
// Scaling.  Every row r of op(A) (every column of op(B)) gets the power-of-two
// exponent E[r] of the split pass (max |x| 2^-E in [1/4, 1/2), real and imaginary
// parts together) and becomes the integer vector X' = rint(x 2^{kbits + 1 - E}),
// |X'| <= 2^kbits.  The only approximation of the scheme is this rounding.
//
// Residues.  For odd, pairwise coprime moduli m_0..m_{p-1} <= 255 each integer is
// stored as its symmetric residue in [-(m-1)/2, (m-1)/2] (fits int8).  Layout per
// batch entry: [p][KT][4][R][32] bytes (KT = ceil(K / 64) strips of 64 k; part
// P = 2 c + t of a strip holds plane c (0 = real, 1 = imaginary) and k = 32 t .. +31 of
// the strip, one 32-byte run per row, i.e. the k of one 32-k matrix-core step; k beyond
// K is zero).  32 rows of a part are one contiguous 1 KB run: one wave's global-to-LDS
// copy.
//
// Product (4M).  For each modulus the INT32 matrix cores accumulate, exactly,
//   rr = sum Ar' Br',  ii = sum Ai' Bi',  ri = sum Ar' Bi' + Ai' Br'
// over all of K (|sum| <= 2 K 127^2 < 2^31).  Then Cr = rr - ii and Ci = ri are
// folded into a CRT sum per output, in FP64:
//   S += ((c u_i) mod m_i) / m_i,   u_i = (M / m_i)^-1 mod m_i,  M = prod m_i,
// which is C' / M modulo 1.  Since |C'| <= 2 K 4^kbits < M / 4, C' = M (S - rint(S))
// up to the FP64 rounding of S (p terms below 2^-50, against C' / M >= 1/16 of
// the largest possible |C'| / M), and C = C' 2^{E_A + E_B - 2 kbits - 2}.
#include "qtx_internal.h"

namespace qtx {

typedef int i4 __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int KS = 64;                 // k per strip (two MFMA k-steps of 32)
constexpr int BM = 64, BN = 64, NT = 256;

// Odd, pairwise coprime moduli (largest first).
constexpr int kModuli[kO2MaxModuli] = {255, 253, 251, 247, 241, 239, 233, 229,
                                       227, 223, 217, 211, 199, 197, 193, 191};

__device__ inline int xcd_remap(int pid, int total) {
  const int nx = 8;
  int per = total / nx, rem = total % nx;
  int x = pid % nx, local = pid / nx;
  return (x < rem) ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

__device__ inline double pow2(int e) {
  e = e < -1020 ? -1020 : (e > 1020 ? 1020 : e);
  return __builtin_bit_cast(double, (uint64_t)(e + 1023) << 52);
}

// 64 rows x 32 k of S = op(X) into LDS (coalesced along the contiguous index),
// zero outside rows x cols.
__device__ inline void load_half_strip(const SplitDesc& sd, const double2* X, int r0, int k0, int tid,
                                       double2 (*tile)[33]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int e = tid + NT * j;
    int r, k;
    if (!sd.trans) { r = e / 32; k = e % 32; }
    else { k = e / 64; r = e % 64; }
    double2 v = cmk(0.0, 0.0);
    if (r0 + r < sd.rows && k0 + k < sd.cols)
      v = sd.trans ? X[(int64_t)(k0 + k) * sd.ld + r0 + r] : X[(int64_t)(r0 + r) * sd.ld + k0 + k];
    tile[r][k] = sd.conj ? cconj(v) : v;
  }
}

// One workgroup per (64 rows, one 64-k strip, batch entry).  Thread t handles row
// t/4 and k = 8 (t%4) .. +7 of each 32-k half.
__global__ __launch_bounds__(NT) void o2_residue_kernel(SplitDesc sd, O2Params P) {
  __shared__ double2 tile[64][33];
  const int z = blockIdx.z, kt = blockIdx.y, r0 = blockIdx.x * 64, tid = threadIdx.x;
  const double2* X = sd.tX ? sd.tX[z] : sd.X + (int64_t)z * sd.stride;
  const int r = tid >> 2, kq = (tid & 3) * 8;
  const bool live = r0 + r < sd.rows;
  const int KT = (sd.cols + KS - 1) / KS;
  const int er = live ? sd.E[(int64_t)z * sd.e_stride + r0 + r] : 0;
  const bool fin = er != kExpNonFinite;   // a non-finite row gets zero residues
  const double sc = (live && fin) ? pow2(P.kbits + 1 - er) : 0.0;
  int8_t* out = (int8_t*)sd.S + (int64_t)z * sd.s_stride;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();
    load_half_strip(sd, X, r0, kt * KS + 32 * h, tid, tile);
    __syncthreads();
    if (!live) continue;
    double a[2][8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double2 v = tile[r][kq + j];
      a[0][j] = fin ? rint(v.x * sc) : 0.0;   // exact scaling, then the one rounding of the scheme
      a[1][j] = fin ? rint(v.y * sc) : 0.0;
    }
    for (int i = 0; i < P.p; ++i) {
      const double m = P.m[i], im = P.inv_m[i];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        uint32_t w[2] = {0u, 0u};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          // |a| <= 2^47: a/m is off an integer + 1/2 by >= 1/(2m), far above the
          // rounding of a * (1/m), so q = rint(a / m) exactly and r is exact.
          const double q = rint(a[c][j] * im);
          const int rr = (int)fma(-q, m, a[c][j]);
          w[j >> 2] |= ((uint32_t)rr & 0xffu) << (8 * (j & 3));
        }
        uint2 pk;
        pk.x = w[0];
        pk.y = w[1];
        *(uint2*)(out + ((((int64_t)i * KT + kt) * 4 + 2 * c + h) * sd.rows + r0 + r) * 32 + kq) = pk;
      }
    }
  }
}

// Single-pass conversion for K <= kO2FusedMaxK: one workgroup of RB waves holds RB
// rows of S = op(X) over all of K in LDS (coalesced loads; element (r, k) at
// r KP + (k ^ r), so the rows of one k fall in distinct banks), finds the row
// exponents (wave w reduces row w), and writes every (modulus, strip) block of its
// rows, 16 bytes per lane (lane -> strip of its wave's pass, row, plane, 16
// consecutive k); wave w converts strips 8w / RB .. 8(w + 1) / RB - 1, then the next
// RB such groups.
constexpr int kO2FusedMaxK = 512;   // RB rows x 512 x 16 B of LDS (64 KB at RB = 8)
constexpr int kO2ConvRows = 4;      // rows per conversion workgroup (4: five workgroups per CU at K = 512;
                                    // faster than 8 or 2 on MI355X for both load orders)

template <int RB>
__global__ __launch_bounds__(64 * RB) void o2_convert_kernel(SplitDesc sd, O2Params P) {
  static_assert(RB == 2 || RB == 4 || RB == 8, "rows per workgroup");
  constexpr int CT = 64 * RB;          // threads
  extern __shared__ double2 rows_lds[];   // [RB][KP], KP = KT * 64 (zero-padded), swizzled
  // 1-D grid over (entry, row group), remapped so that each XCD takes a contiguous run of
  // row groups of one entry: with trans = 1 a group is RB adjacent columns (RB * 16 bytes
  // of each source row), and its neighbours then read the rest of the same cache lines
  // through the same L2 instead of fetching them again into another XCD's.
  const int gx = (sd.rows + RB - 1) / RB;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int z = lb / gx, r0 = (lb - z * gx) * RB, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int K = sd.cols, KT = (K + KS - 1) / KS, KP = KT * KS, pitch = KP;
  const double2* X = sd.tX ? sd.tX[z] : sd.X + (int64_t)z * sd.stride;
  // load (zero outside rows x K, conjugate on the way in): thread t takes row t / 64
  // (trans 0: rows contiguous) or t % RB (trans 1: RB adjacent columns of X), and
  // k = its base + 64 j; all loads are issued before the LDS stores.
  {
    const int r = sd.trans ? (tid % RB) : (tid >> 6);
    const int kb = sd.trans ? (tid / RB) : (tid & 63);
    const bool rok = r0 + r < sd.rows;
    const int nj = KP / 64;   // <= 8
    double2 v[kO2FusedMaxK / 64];
#pragma unroll
    for (int j = 0; j < kO2FusedMaxK / 64; ++j) {
      const int k = kb + 64 * j;
      v[j] = cmk(0.0, 0.0);
      if (j < nj && rok && k < K)
        v[j] = sd.trans ? X[(int64_t)k * sd.ld + r0 + r] : X[(int64_t)(r0 + r) * sd.ld + k];
    }
#pragma unroll
    for (int j = 0; j < kO2FusedMaxK / 64; ++j) {
      const int k = kb + 64 * j;
      if (j < nj) rows_lds[r * pitch + (k ^ r)] = sd.conj ? cconj(v[j]) : v[j];
    }
  }
  __syncthreads();
  // row exponents: wave w reduces row w
  {
    const int r = wave;
    double mx = 0.0;
    bool bad = false;   // NaN or Inf in the row (fmax alone would skip a NaN)
    for (int k = lane; k < KP; k += 64) {
      const double2 v = rows_lds[r * pitch + k];   // any order: all k of the row
      bad |= !(isfinite(v.x) && isfinite(v.y));
      mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    bad = __any(bad);
    int e = 0;
    if (bad) e = kExpNonFinite;
    else if (mx > 0.0 && mx <= 1.7e308) e = ilogb(mx) + 2;   // max * 2^-e in [1/4, 1/2)
    if (lane == 0 && r0 + r < sd.rows) sd.E[(int64_t)z * sd.e_stride + r0 + r] = e;
  }
  __syncthreads();   // the exponents are read back below (same workgroup)
  // Residues: a lane takes 16 consecutive k of one (row, plane) of a strip, so a wave
  // covers SPW = 8 / RB strips per pass and stores 16 bytes per lane and modulus.  The
  // symmetric residue a - m rint(a / m) is formed exactly with the rounding constant
  // R = 1.5 2^52 (|a| <= 2^47, |a / m| < 2^40): fma(a, 1/m, R) - R is the nearest integer
  // q to a / m (the fraction of a / m is a multiple of 1/m, m odd, so the rounded 1/m
  // cannot move it across a half), and fma(-q, m, a + R) = R + (a - q m) exactly, whose
  // low byte is the residue's two's-complement byte.
  constexpr int SPW = 8 / RB;
  const int ks = lane & 3, c = (lane >> 2) & 1, r = (lane >> 3) % RB, sub = lane / (8 * RB);
  const bool live = r0 + r < sd.rows;
  const int er = live ? sd.E[(int64_t)z * sd.e_stride + r0 + r] : 0;
  const bool fin = er != kExpNonFinite;   // a non-finite row gets zero residues
  const double sc = (live && fin) ? pow2(P.kbits + 1 - er) : 0.0;
  constexpr double R = 6755399441055744.0;   // 1.5 * 2^52
  int8_t* out = (int8_t*)sd.S + (int64_t)z * sd.s_stride;
  for (int kt0 = wave * SPW; kt0 < KT; kt0 += RB * SPW) {
    const int kt = kt0 + sub;
    const bool ok = live && kt < KT;
    double a[16], ar[16];
    const double2* src = rows_lds + r * pitch;
    const int k0 = (kt < KT ? kt : KT - 1) * KS + 16 * ks;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double2 v = src[(k0 + j) ^ r];
      a[j] = fin ? rint((c ? v.y : v.x) * sc) : 0.0;
      ar[j] = a[j] + R;
    }
    int8_t* dst = out + (((int64_t)kt * 4 + 2 * c + (ks >> 1)) * sd.rows + r0 + r) * 32 + 16 * (ks & 1);
    const int64_t mstride = (int64_t)KT * 4 * sd.rows * 32;   // bytes per modulus
#pragma unroll
    for (int i = 0; i < kO2MaxModuli; ++i) {
      if (i < P.p) {
        const double m = P.m[i], im = P.inv_m[i];
        uint32_t lo[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const double q = fma(a[j], im, R) - R;
          lo[j] = (uint32_t)__builtin_bit_cast(uint64_t, fma(-q, m, ar[j]));
        }
        u4 pk;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const uint32_t p01 = __builtin_amdgcn_perm(lo[4 * w + 1], lo[4 * w], 0x0c0c0400u);
          const uint32_t p23 = __builtin_amdgcn_perm(lo[4 * w + 3], lo[4 * w + 2], 0x0c0c0400u);
          pk[w] = __builtin_amdgcn_perm(p23, p01, 0x05040100u);
        }
        if (ok) *(u4*)(dst + i * mstride) = pk;
      }
    }
  }
}

__device__ inline i16v mfma_i8(i4 a, i4 b, i16v c) {
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// Negate 16 packed int8 values (residues in [-127, 127], so -x fits): per byte,
// (0x80 - (x & 0x7f)) ^ (~x & 0x80); the subtraction never borrows across bytes.
__device__ inline i4 neg_i8x16(i4 x) {
  i4 r;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t u = (uint32_t)x[q];
    r[q] = (int)((0x80808080u - (u & 0x7f7f7f7fu)) ^ (~u & 0x80808080u));
  }
  return r;
}

// S += ((c u) mod m) / m.  |c| < 2^31 and u < 2^8, so c u is exact in FP64; its
// quotient by m is never within 1/(2m) of a half-integer (m odd), so q is exact and
// so is the remainder.
__device__ inline void crt_fold(int c, double m, double im, double u, double& S) {
  const double cu = (double)c * u;
  const double q = rint(cu * im);
  const double r = fma(-q, m, cu);
  S = fma(r, im, S);
}

// BM x BN complex output tile per workgroup; each wave owns WM x WN blocks of 32 x 32
// (rows 32 (WM wm + i), columns 32 (WN wn + j) of the tile, wave w = wm + WAVES_M wn), so
// one A fragment feeds WN products and one B fragment WM.  MFMA 32x32x32 i8 layouts:
// operand lane l holds row (column) l % 32 and k = 16 (l / 32) .. +15 of a 32-k step;
// result lane l, element v -> row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32.
//
// The (modulus, strip) tiles, modulus-major, stream through an NSTAGE-deep LDS
// ring filled by direct global->LDS loads (no registers held for them), so
// NSTAGE - 1 steps of SPI strips are in flight while one feeds the matrix
// cores.  A stage holds SPI strips, each A's 4 parts of BM rows then B's 4 parts of
// BN rows (32 bytes per row and part, the global layout's order, with the halves of
// rows 8..15 of every 16 swapped).  The LDS of gfx950 has 64 banks and serves a
// 16-byte-per-lane read 16 lanes per cycle: the 16 consecutive rows one cycle of a
// fragment read touches (one 16-byte half each) fall into 16 distinct groups of four
// banks, and every fragment address is the lane's slot plus a compile-time offset.
// Each thread
// issues exactly LPT loads per strip, so "strip j has landed" is a fixed count
// of outstanding vector-memory operations.  Rows beyond M (N) load row M - 1
// (N - 1): they only feed outputs that are never stored.
//
// Tile variants (the launch takes one by index; all give bitwise the same result,
// since every output's INT32 sums and CRT fold run in the same order):
//   0: 128 x 64, one block per wave, 512 threads, 2 strips per step, 3 stages
//      (144 KB of LDS, one workgroup per CU)
//   1: 64 x 64, one block per wave, 256 threads, 2 strips per step, 2 stages (64 KB,
//      two per CU)
//   2: 64 x 64, 256 threads, 1 strip per step, 3 stages (48 KB, two per CU)
//   3: as 2, three per CU (registers capped at 168 per lane; no spills in the strip loop)
//   4: 64 x 64, 256 threads, 1 strip per step, 2 stages (32 KB, three per CU)
//   5, 6: variants 4 and 1 with one tile per workgroup instead of persistent
//      workgroups (the hardware then keeps a window of consecutive tiles -- the
//      same energies on one XCD -- in flight, in place of rounds that drift apart)
//   7: 32 x 64, 128 threads (two waves), 1 strip per step, 2 stages (24 KB, six per
//      CU): covers b = 416 (13 x 32) without padding rows and gives twice the
//      workgroups of a 64 x 64 tiling, for about 1.4x the operand strips per output
//   8: 64 x 64, two blocks (64 x 32) per wave, 128 threads, 2 stages (32 KB, four per
//      CU): a quarter fewer fragment reads per product than one block per wave
//   9: 64 x 128, two blocks (32 x 64) per wave, 256 threads, 3 stages (72 KB, two per CU):
//      a quarter fewer operand bytes per product than 64 x 64
//  10: 128 x 128, two blocks (64 x 32) per wave, 512 threads, 2 stages (64 KB, one per
//      CU, two waves per SIMD): half the operand bytes per product of 64 x 64
//  11: variant 8 with one tile per workgroup
//  12: 64 x 64, one block per wave, 256 threads, 4 stages (64 KB, two per CU); 13: the
//      same, one tile per workgroup
constexpr int kBufWord3 = 0x00020000;           // buffer descriptor word 3: raw 32-bit data, no swizzle

template <int BM_, int BN_, int WM_, int WN_, int SPI_, int NSTAGE_, int WPC_>
struct O2Cfg {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, SPI = SPI_, NSTAGE = NSTAGE_;
  static constexpr int WAVES_M = BM / (32 * WM), WAVES_N = BN / (32 * WN);
  static constexpr int NT = 64 * WAVES_M * WAVES_N;
  static constexpr int STRIP_U4 = (BM + BN) * 8;      // 16-byte slots per strip
  static constexpr int STAGE_U4 = SPI * STRIP_U4;     // per stage
  static constexpr int LPS = STRIP_U4 / NT;           // copies per thread per strip
  static constexpr int LPS_A = BM * 8 / NT;           // of which the first LPS_A copy A rows
  static constexpr int LPT = SPI * LPS;               // copies per thread per step
  static constexpr int WPC = WPC_;                    // workgroups per CU (LDS / registers)
  static constexpr int WAVES_PER_SIMD = (WPC * NT / 256) > 0 ? WPC * NT / 256 : 1;
  static constexpr bool TWO_ACC = WM * WN > 1;   // O2Acc layout (two blocks per wave: two accumulators)
  static_assert(BM % (32 * WM) == 0 && BN % (32 * WN) == 0, "wave blocks");
  static_assert(STRIP_U4 % NT == 0 && (BM * 8) % NT == 0, "copy split");
  static_assert(NSTAGE >= 2 && NSTAGE <= 4, "ring depth");
  static_assert(LPT < 64, "vmcnt range");
  static_assert(NT >= BM + BN && NT >= 16, "exponent and constant fills");
};
typedef O2Cfg<128, 64, 1, 1, 2, 3, 1> O2V0;
typedef O2Cfg<64, 64, 1, 1, 2, 2, 2> O2V1;
typedef O2Cfg<64, 64, 1, 1, 1, 3, 2> O2V2;
typedef O2Cfg<64, 64, 1, 1, 1, 3, 3> O2V3;
typedef O2Cfg<64, 64, 1, 1, 1, 2, 3> O2V4;
typedef O2Cfg<32, 64, 1, 1, 1, 2, 6> O2V7;
typedef O2Cfg<64, 64, 2, 1, 1, 2, 4> O2V8;
typedef O2Cfg<64, 128, 1, 2, 1, 3, 2> O2V9;
typedef O2Cfg<128, 128, 2, 1, 1, 2, 1> O2V10;
typedef O2Cfg<64, 64, 1, 1, 1, 4, 2> O2V12;

typedef __attribute__((address_space(3))) u4 lds_u4;
typedef __attribute__((address_space(3))) double lds_f64;

// Accumulators of one 32 x 32 output block.  INT32 sums of the current modulus:
// with TWO, re = rr - ii in one accumulator (the imaginary B fragment negated in
// registers: 16 fewer VGPRs per block, which the variants with two blocks per wave
// need) and im = ri + ir; else rr, ii and ri + ir apart (no negation work in the
// strip loop; the subtraction rr - ii happens once per modulus, in the fold).  The INT32 sums, and
// so the results, are the same either way.
template <bool TWO>
struct O2Acc;
template <>
struct O2Acc<true> {
  i16v are, aim;
  double sre[16], sim[16];   // CRT sums (real, imaginary)
  __device__ inline void clear(int v) { are[v] = 0; aim[v] = 0; }
  __device__ inline int re(int v) const { return are[v]; }
  __device__ inline int im(int v) const { return aim[v]; }
  // bn = the imaginary B fragment negated.  FIRST: the first k-step of a modulus, whose
  // products start from zero (the matrix cores take the zero addend, so the sums of the
  // previous modulus need no clearing).
  template <bool FIRST>
  __device__ inline void step(i4 ar, i4 ai, i4 br, i4 bi, i4 bn) {
    const i16v z = {};
    are = mfma_i8(ar, br, FIRST ? z : are);
    aim = mfma_i8(ar, bi, FIRST ? z : aim);
    are = mfma_i8(ai, bn, are);
    aim = mfma_i8(ai, br, aim);
  }
  // the same with B conjugated (bi -> -bi): the negation moves to the other product
  template <bool FIRST>
  __device__ inline void step_conj(i4 ar, i4 ai, i4 br, i4 bi, i4 bn) {
    const i16v z = {};
    are = mfma_i8(ar, br, FIRST ? z : are);
    aim = mfma_i8(ar, bn, FIRST ? z : aim);
    are = mfma_i8(ai, bi, are);
    aim = mfma_i8(ai, br, aim);
  }
};
template <>
struct O2Acc<false> {
  i16v arr, aii, ari;
  double sre[16], sim[16];
  __device__ inline void clear(int v) { arr[v] = 0; aii[v] = 0; ari[v] = 0; }
  __device__ inline int re(int v) const { return arr[v] - aii[v]; }
  __device__ inline int im(int v) const { return ari[v]; }
  template <bool FIRST>
  __device__ inline void step(i4 ar, i4 ai, i4 br, i4 bi, i4) {
    const i16v z = {};
    arr = mfma_i8(ar, br, FIRST ? z : arr);
    aii = mfma_i8(ai, bi, FIRST ? z : aii);
    ari = mfma_i8(ar, bi, FIRST ? z : ari);
    ari = mfma_i8(ai, br, ari);
  }
  template <bool FIRST>
  __device__ inline void step_conj(i4 ar, i4 ai, i4 br, i4 bi, i4 bn) { step<FIRST>(ar, ai, br, bn, bi); }
};

// Per-thread constants of the strip loop.
template <int LPS, int WM, int WN>
struct O2Ctx {
  int off[LPS];              // byte offset (in A's or B's residues) of each of the thread's slots of a strip
  int sstride_a, sstride_b;  // bytes from one strip to the next (residue offsets are < 2^31)
  const lds_f64* cst;        // moduli, their reciprocals, the CRT factors u (LDS)
  int tid, wbase, lb[WN], lk, KT, K, NSTRIP;   // wbase: the wave's first thread (scalar)
  int pa[WM], pb[WN];        // ring slot of the lane's 16 bytes (k half lk) in part 0 of A / of B
  bool live[WM][WN];         // the wave's 32 x 32 blocks that hold outputs (wave-uniform)
  bool wlive;                // any of them
};

// Ring position of 16-byte half h of a row's 32 bytes (an involution: the same map
// takes a ring position back to the half stored there).
__device__ inline int ring_half(int row, int h) { return h ^ ((row >> 3) & 1); }

__device__ inline void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// s_waitcnt vmcnt(N) (expcnt and lgkmcnt left unconstrained)
template <int N>
__device__ inline void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// One step s of the strip loop (s = -(NSTAGE-1) .. NSTEP-1; a step is SPI strips):
// wait until step s's strips have landed (this thread's copies, then everyone's
// via the barrier), start the copy of step s + NSTAGE - 1 into stage `dma` (the
// stage step s - 1 used), then read step s's fragments from stage `rd` and feed
// them to the matrix cores.  After the last strip of a modulus the INT32 sums
// are folded into the CRT sums.  `rd` and `dma` are distinct restrict pointers
// (as are the residue arrays), which gives the copies and the reads their own
// alias scopes: the compiler's wait-count insertion then leaves the copies of
// later steps in flight during the reads; their completion is awaited
// explicitly.  Every thread issues exactly LPT copies per step (a step past the
// last strip re-copies that strip into its unused part), so "step s landed" is a
// fixed count of outstanding vector-memory operations: with NSTAGE stages steps
// s + 1 .. s + NSTAGE - 2 may still be in flight.
// (fi, fkt): modulus and strip of the next strip this step consumes (advanced here).
template <class CF, bool CONJB>
__device__ __attribute__((always_inline)) inline void o2_step(int s, const lds_u4* __restrict__ rd,
                                                            lds_u4* __restrict__ dma, const int8_t* __restrict__ gA,
                                                            const int8_t* __restrict__ gB,
                                                            const O2Ctx<CF::LPS, CF::WM, CF::WN>& c,
                                                            O2Acc<CF::TWO_ACC> (&a)[CF::WM][CF::WN], int& fi,
                                                            int& fkt) {
  constexpr int SPI = CF::SPI, NSTAGE = CF::NSTAGE, LPS = CF::LPS, LPT = CF::LPT, WM = CF::WM, WN = CF::WN;
  const int nstep = (c.NSTRIP + SPI - 1) / SPI;
  if (s >= 0) {
    // steps s + 1 .. s + NSTAGE - 2 (those that exist) may still be pending
    const int pend = min(NSTAGE - 2, nstep - 1 - s);
    if (NSTAGE >= 4 && pend >= 2) wait_vm<(NSTAGE >= 4 ? 2 : 0) * LPT>();
    else if (NSTAGE >= 3 && pend >= 1) wait_vm<LPT>();
    else wait_vm<0>();
  }
  lds_barrier();
  const int sd = s + NSTAGE - 1;   // >= 0
  if (sd < nstep) {
    // (the resources are made here from the restrict pointers: built once per tile
    // instead, the copies lose their alias scope and the compiler drains them before
    // every fragment read)
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc((void*)gA, 0, 0x7fffffff, kBufWord3);
    const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc((void*)gB, 0, 0x7fffffff, kBufWord3);
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int f = min(SPI * sd + q / LPS, c.NSTRIP - 1);
      // the strip's offset is wave-uniform: it travels as the scalar offset, so the
      // per-lane offset is the tile's fixed c.off and no vector add is needed per copy
      __builtin_amdgcn_raw_ptr_buffer_load_lds(q % LPS < CF::LPS_A ? ra : rb,
                                               (__attribute__((address_space(3))) void*)(dma + q * CF::NT + c.wbase),
                                               16, c.off[q % LPS], f * (q % LPS < CF::LPS_A ? c.sstride_a : c.sstride_b),
                                               0, 0);
    }
  }
  if (s < 0) return;
#pragma unroll
  for (int h = 0; h < SPI; ++h) {
    const int f = SPI * s + h;
    if (f >= c.NSTRIP) break;
    const int i = fi;
    const int kt = fkt;
    if (++fkt == c.KT) { fkt = 0; ++fi; }
    const lds_u4* st = rd + h * CF::STRIP_U4;
    const bool two = !(kt == c.KT - 1 && c.K - kt * KS <= 32);   // a half strip at the end has one step
    // A wave with no output in the tile skips the strip.  The blocks of a wave with
    // several run unconditionally (a block past the matrix edge computes on the
    // clamped rows and is never stored): branches per block cost more registers than
    // the idle products at the edges.
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      if (t == 1 && !two) break;
      if (!c.wlive) break;
      // parts t (real) and 2 + t (imaginary): the lane's slot plus a compile-time offset
      i4 far_[WM], fai[WM], fbr[WN], fbi[WN], fbn[WN];
#pragma unroll
      for (int x = 0; x < WM; ++x) {
        far_[x] = __builtin_bit_cast(i4, st[c.pa[x] + t * 2 * CF::BM]);
        fai[x] = __builtin_bit_cast(i4, st[c.pa[x] + (2 + t) * 2 * CF::BM]);
      }
#pragma unroll
      for (int y = 0; y < WN; ++y) {
        fbr[y] = __builtin_bit_cast(i4, st[c.pb[y] + t * 2 * CF::BN]);
        fbi[y] = __builtin_bit_cast(i4, st[c.pb[y] + (2 + t) * 2 * CF::BN]);
        fbn[y] = (CF::TWO_ACC || CONJB) ? neg_i8x16(fbi[y]) : fbi[y];
      }
      const bool first = t == 0 && kt == 0;   // wave-uniform
#pragma unroll
      for (int x = 0; x < WM; ++x)
#pragma unroll
        for (int y = 0; y < WN; ++y) {
          if (first) {
            if (CONJB) a[x][y].template step_conj<true>(far_[x], fai[x], fbr[y], fbi[y], fbn[y]);
            else a[x][y].template step<true>(far_[x], fai[x], fbr[y], fbi[y], fbn[y]);
          } else {
            if (CONJB) a[x][y].template step_conj<false>(far_[x], fai[x], fbr[y], fbi[y], fbn[y]);
            else a[x][y].template step<false>(far_[x], fai[x], fbr[y], fbi[y], fbn[y]);
          }
        }
    }
    if (kt == c.KT - 1) {
      const double m = c.cst[i], im = c.cst[kO2MaxModuli + i], u = c.cst[2 * kO2MaxModuli + i];
#pragma unroll
      for (int x = 0; x < WM; ++x)
#pragma unroll
        for (int y = 0; y < WN; ++y)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            crt_fold(a[x][y].re(v), m, im, u, a[x][y].sre[v]);
            crt_fold(a[x][y].im(v), m, im, u, a[x][y].sim[v]);
          }
    }
  }
}

// The product descriptor as the kernel's first argument in the kernel-argument segment,
// through a pointer laundered by an empty asm: loads through it cannot be hoisted above
// the call site (the strip loop's barriers order it), so the epilogue's parameters are
// read where they are used.
typedef const __attribute__((address_space(4))) SplitGemmDesc KSplitGemmDesc;
typedef const __attribute__((address_space(4))) GemmDesc KGemmDesc;
__device__ inline KGemmDesc& kernarg_desc() {
  uint64_t v = (uint64_t)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(v));
  return ((KSplitGemmDesc*)v)->d;
}

// Persistent grid (persist = 1): WPC workgroups per CU; workgroup w runs on XCD
// w % 8 and takes that XCD's tiles (a contiguous range) in rounds of the XCD's
// workgroup count, so the workgroups sharing an L2 work on adjacent tiles of the
// same energies in step and read each residue strip from HBM about once.
// Otherwise one tile per workgroup.  A skew-Hermitian product's tile index runs over
// the tiles that reach the upper triangle only.
template <class CF, bool CONJB>
__global__ __launch_bounds__(CF::NT) __attribute__((amdgpu_waves_per_eu(CF::WAVES_PER_SIMD)))
void zgemm_o2_kernel(SplitGemmDesc g, O2Params P, int total_tiles, int persist) {
  constexpr int BM = CF::BM, BN = CF::BN, NT = CF::NT, NSTAGE = CF::NSTAGE, SPI = CF::SPI, LPS = CF::LPS;
  constexpr int WM = CF::WM, WN = CF::WN;
  __shared__ u4 ring[NSTAGE][CF::STAGE_U4];
  __shared__ int Ea[BM], Eb[BN];
  __shared__ double cst[3 * kO2MaxModuli];

  if (threadIdx.x < kO2MaxModuli) {
    cst[threadIdx.x] = P.m[threadIdx.x];
    cst[kO2MaxModuli + threadIdx.x] = P.inv_m[threadIdx.x];
    cst[2 * kO2MaxModuli + threadIdx.x] = P.u[threadIdx.x];
  }
  const int tiles_m = (g.d.M + BM - 1) / BM;
  const int tiles_n = (g.d.N + BN - 1) / BN;
  const bool skew = g.d.skew != 0;
  // a skew-Hermitian result enumerates only the tiles that reach the upper triangle:
  // column tn keeps the first ceil((tn + 1) BN / BM) row tiles
  int per = tiles_m * tiles_n;
  if (skew) {
    per = 0;
    for (int tn = 0; tn < tiles_n; ++tn) per += min(tiles_m, ((tn + 1) * BN + BM - 1) / BM);
  }
  int first, last, step;
  if (persist) {
    const int nx = 8, x = blockIdx.x % nx, wpx = gridDim.x / nx;
    const int tpx = (total_tiles + nx - 1) / nx;
    first = x * tpx + (int)blockIdx.x / nx;
    last = min((x + 1) * tpx, total_tiles);
    step = wpx;
  } else {
    first = xcd_remap(blockIdx.x, gridDim.x);
    last = first + 1;
    step = 1;
  }
  for (int tile = first; tile < last; tile += step) {
  const int z = tile / per;
  int t = tile - z * per;
  int m0, n0;
  if (skew) {
    int tn = 0;
    for (;;) {
      const int cn = min(tiles_m, ((tn + 1) * BN + BM - 1) / BM);
      if (t < cn) break;
      t -= cn;
      ++tn;
    }
    m0 = t * BM;
    n0 = tn * BN;
  } else {
    m0 = (t % tiles_m) * BM;
    n0 = (t / tiles_m) * BN;
  }
  const int M = g.d.M, N = g.d.N, K = g.d.K;
  const int KT = (K + KS - 1) / KS;
  const int NSTRIP = P.p * KT;                  // (modulus, strip) pairs, modulus-major

  const int8_t* SA = (const int8_t*)g.SA + (int64_t)z * g.sa_stride;
  const int8_t* SB = (const int8_t*)g.SB + (int64_t)z * g.sb_stride;
  const int32_t* EA = g.EA + (int64_t)z * g.ea_stride;
  const int32_t* EB = g.EB + (int64_t)z * g.eb_stride;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % CF::WAVES_M, wn = wave / CF::WAVES_M;

  if (tid < BM) Ea[tid] = (m0 + tid < M) ? EA[m0 + tid] : 0;
  else if (tid < BM + BN) Eb[tid - BM] = (n0 + tid - BM < N) ? EB[n0 + tid - BM] : 0;
  __syncthreads();   // also drains these loads before the counted ring loads start

  // Per-thread source of each of its LPS slots of a strip (the strip offset added
  // per strip): slot cs = q * NT + tid; the ring holds a strip as A's 4 parts of BM
  // rows, then B's 4 parts of BN rows, 32 bytes per row (slot = 2 (part * rows + row) +
  // half), the two 16-byte halves of a row swapped when bit 3 of the row is set
  // (ring_half): a matrix-core fragment read then takes 16 rows of one half in 16
  // distinct groups of four of gfx950's 64 LDS banks.
  O2Ctx<LPS, WM, WN> c;
#pragma unroll
  for (int q = 0; q < LPS; ++q) {
    const int cs = q * NT + tid;
    const bool isa = cs < 8 * BM;            // q < LPS_A: A
    const int rows = isa ? BM : BN, ce = isa ? cs : cs - 8 * BM;
    const int part = ce / (2 * rows), row = (ce % (2 * rows)) >> 1, half = ring_half(row, ce & 1);
    const int rg = isa ? min(m0 + row, M - 1) : min(n0 + row, N - 1);
    c.off[q] = ((part * (isa ? M : N) + rg) * 2 + half) * 16;
  }
  c.sstride_a = M * 128;
  c.sstride_b = N * 128;
  c.cst = (const lds_f64*)&cst[0];
  c.tid = tid;
  c.wbase = __builtin_amdgcn_readfirstlane(tid & ~63);
  c.lk = lane >> 5;
#pragma unroll
  for (int x = 0; x < WM; ++x) {
    const int row = 32 * (WM * wm + x) + (lane & 31);
    c.pa[x] = 2 * row + ring_half(row, c.lk);
  }
#pragma unroll
  for (int y = 0; y < WN; ++y) {
    const int row = 32 * (WN * wn + y) + (lane & 31);
    c.lb[y] = BM + row;
    c.pb[y] = 8 * BM + 2 * row + ring_half(row, c.lk);
  }
  c.KT = KT;
  c.K = K;
  c.NSTRIP = NSTRIP;
#pragma unroll
  for (int x = 0; x < WM; ++x)
#pragma unroll
    for (int y = 0; y < WN; ++y) {
      const int rb = m0 + 32 * (WM * wm + x), cb = n0 + 32 * (WN * wn + y);
      c.live[x][y] = rb < M && cb < N && !(skew && rb >= cb + 32);   // wave-uniform
    }
  c.wlive = false;
#pragma unroll
  for (int x = 0; x < WM; ++x)
#pragma unroll
    for (int y = 0; y < WN; ++y) c.wlive |= c.live[x][y];

  O2Acc<CF::TWO_ACC> acc[WM][WN];
#pragma unroll
  for (int x = 0; x < WM; ++x)
#pragma unroll
    for (int y = 0; y < WN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc[x][y].clear(v);
        acc[x][y].sre[v] = 0.0; acc[x][y].sim[v] = 0.0;
      }
  // Step s reads stage (s + NSTAGE) % NSTAGE and copies into stage (s - 1 + NSTAGE) % NSTAGE;
  // unrolled NSTAGE steps at a time (s = st0 + u with st0 = 1 mod NSTAGE), so that both
  // stages are compile-time constants and every LDS address is a register plus an
  // immediate offset.
  const int nstep = (NSTRIP + SPI - 1) / SPI;
  int fi = 0, fkt = 0;
  for (int st0 = -(NSTAGE - 1); st0 < nstep; st0 += NSTAGE) {
#pragma unroll
    for (int u = 0; u < NSTAGE; ++u) {
      if (st0 + u >= nstep) break;
      o2_step<CF, CONJB>(st0 + u, (const lds_u4*)&ring[(u + 1) % NSTAGE][0], (lds_u4*)&ring[u][0], SA, SB, c, acc,
                         fi, fkt);
    }
  }

  // epilogue in FP64 (same addend semantics as the FP64 kernels).  Its parameters are
  // read here from the kernel-argument segment through a pointer the compiler cannot
  // see through, so that they are loaded after the strip loop instead of being held in
  // scalar registers across it (about 40 of them: they used to spill, and the spill
  // slots cost vector registers the strip loop needs).
  KGemmDesc& d = kernarg_desc();
  double2* __restrict__ C = d.tC ? d.tC[z] : d.C + (int64_t)z * d.sC;
  const double bs = d.bscal ? d.bscal[z] : 1.0;
  const double2 alpha = cmk(d.alpha.x, d.alpha.y);
  double2 coef[kMaxAddends];
  const double2* X[kMaxAddends];
#pragma unroll
  for (int q = 0; q < kMaxAddends; ++q) {
    coef[q] = cmk(d.add[q].coef.x, d.add[q].coef.y);
    if (d.add[q].scale_by_batch) coef[q] = cmk(coef[q].x * bs, coef[q].y * bs);
    X[q] = d.add[q].tX ? d.add[q].tX[z] : (d.add[q].X ? d.add[q].X + (int64_t)z * d.add[q].stride : nullptr);
  }
  const double2 dg = d.diag_by_batch ? cmk(d.diag.x * bs, d.diag.y * bs) : cmk(d.diag.x, d.diag.y);
  const int lk = c.lk;
#pragma unroll
  for (int x = 0; x < WM; ++x)
#pragma unroll
    for (int y = 0; y < WN; ++y) {
      if (!c.live[x][y]) continue;
      const int colt = c.lb[y] - BM;
      const int col = n0 + colt;
      const int eb = Eb[colt];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rl = 32 * (WM * wm + x) + 8 * (v >> 2) + 4 * lk + (v & 3);
        const int r = m0 + rl;
        if (r < M && col < N && !(skew && r > col)) {
          // a row of op(A) or column of op(B) with NaN / Inf gives NaN, as in FP64
          const bool nf = Ea[rl] == kExpNonFinite || eb == kExpNonFinite;
          const double sc = nf ? __builtin_nan("") : pow2(Ea[rl] + eb - 2 * P.kbits - 2) * P.M;
          const double cr = (acc[x][y].sre[v] - rint(acc[x][y].sre[v])) * sc;
          const double ci = (acc[x][y].sim[v] - rint(acc[x][y].sim[v])) * sc;
          double2 out = cmul(alpha, cmk(cr, ci));
#pragma unroll
          for (int q = 0; q < kMaxAddends; ++q) {
            if (X[q] && (!d.add[q].diag || r == col)) {
              const double2 xv = addend_value(X[q], d.add[q].diag, d.add[q].op, d.add[q].ld, r, col);
              out = cadd(out, cmul(coef[q], xv));
            }
          }
          if (r == col) out = cadd(out, dg);
          if (skew && r == col) out.x = 0.0;   // a skew-Hermitian diagonal is imaginary
          C[(int64_t)r * d.ldc + col] = out;
          if (skew && r < col) C[(int64_t)col * d.ldc + r] = cmk(-out.x, out.y);
        }
      }
    }
  __syncthreads();   // Ea / Eb and the ring are reused by the next tile
  }
}

// Modular inverse of a mod m (gcd 1), by the extended Euclidean algorithm.
int64_t inv_mod(int64_t a, int64_t m) {
  int64_t t = 0, nt = 1, r = m, nr = ((a % m) + m) % m;
  while (nr != 0) {
    const int64_t q = r / nr;
    int64_t tmp = t - q * nt; t = nt; nt = tmp;
    tmp = r - q * nr; r = nr; nr = tmp;
  }
  return t < 0 ? t + m : t;
}

}  // namespace

bool o2_params(int p, int K, O2Params* out) {
  if (p < 2 || p > kO2MaxModuli || K < 1 || K > 65536) return false;
  // kbits(q) = largest k with 8 K 4^k < M_q = m_0 ... m_{q-1}: then |C'| <= 2 K 4^k < M / 4,
  // so C' / M is within 1/4 of the integer the CRT sum S lands near and rint(S) is
  // exact.  Moduli beyond those that 47-bit operands can use only widen M against
  // C' (the FP64 sum S = C' / M mod 1 then loses log2(M / C') bits), so p is
  // clipped to the largest count whose kbits stays <= 47.
  auto kbits_of = [&](int q) {
    unsigned __int128 Mx = 1;
    for (int i = 0; i < q; ++i) Mx *= (unsigned)kModuli[i];
    int kb = -1;
    while (kb < 60) {
      const unsigned __int128 lhs = ((unsigned __int128)(8 * (int64_t)K)) << (2 * (kb + 1));
      if (!(lhs < Mx)) break;
      ++kb;
    }
    return kb;
  };
  int q = p, kb = kbits_of(q);
  while (kb > 47 && q > 2) kb = kbits_of(--q);
  if (kb < 1 || kb > 47) return false;
  O2Params P;
  P.p = q;
  P.kbits = kb;
  double Md = 1.0;
  for (int i = 0; i < q; ++i) Md *= kModuli[i];
  for (int i = 0; i < q; ++i) {
    const int64_t m = kModuli[i];
    int64_t rest = 1;   // (M / m_i) mod m_i
    for (int j = 0; j < q; ++j)
      if (j != i) rest = rest * (kModuli[j] % m) % m;
    P.m[i] = (double)m;
    P.inv_m[i] = 1.0 / (double)m;
    P.u[i] = (double)inv_mod(rest, m);
  }
  for (int i = q; i < kO2MaxModuli; ++i) { P.m[i] = 1.0; P.inv_m[i] = 1.0; P.u[i] = 0.0; }
  P.M = Md;
  *out = P;
  return true;
}

int o2_modulus(int i) { return (i >= 0 && i < kO2MaxModuli) ? kModuli[i] : 0; }

int64_t o2_res_stride(int rows, int cols, int p) {
  return (int64_t)p * ((cols + KS - 1) / KS) * rows * 2 * KS;
}

hipError_t launch_o2_convert(const SplitDesc& sd, const O2Params& P, hipStream_t s) {
  if (sd.rows <= 0 || sd.cols <= 0 || sd.batch <= 0) return hipSuccess;
  if (sd.cols <= kO2FusedMaxK) {
    constexpr int RB = kO2ConvRows;
    const int KP = (sd.cols + KS - 1) / KS * KS;
    const size_t lds = (size_t)RB * KP * sizeof(double2);
    const int64_t blocks = (int64_t)((sd.rows + RB - 1) / RB) * sd.batch;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(o2_convert_kernel<RB>, dim3((unsigned)blocks), dim3(64 * RB), lds, s, sd, P);
    return hipGetLastError();
  }
  hipError_t e = launch_split_exp(sd, s);
  if (e != hipSuccess) return e;
  dim3 grid((sd.rows + 63) / 64, (sd.cols + KS - 1) / KS, sd.batch);
  hipLaunchKernelGGL(o2_residue_kernel, grid, dim3(NT), 0, s, sd, P);
  return hipGetLastError();
}

namespace {

template <class CF>
hipError_t launch_o2_variant(const SplitGemmDesc& g, const O2Params& P, hipStream_t s, bool allow_persist) {
  const GemmDesc& d = g.d;
  const int tm = (d.M + CF::BM - 1) / CF::BM, tn = (d.N + CF::BN - 1) / CF::BN;
  int64_t per = (int64_t)tm * tn;
  if (d.skew) {   // the tiles that reach the upper triangle (as the kernel enumerates them)
    per = 0;
    for (int j = 0; j < tn; ++j) per += std::min(tm, ((j + 1) * CF::BN + CF::BM - 1) / CF::BM);
  }
  const int64_t total = per * d.batch;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  // WPC workgroups per CU (what the kernel's LDS and registers admit) when there are more tiles
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 8;
    cus[dev] = n;
  }
  const int grid_p = cus[dev] / 8 * 8 * CF::WPC;
  const bool persist = allow_persist && grid_p >= 8 && total > grid_p;
  const unsigned grid = persist ? (unsigned)grid_p : (unsigned)total;
  // CONJB: the imaginary B fragments are negated in registers (SplitGemmDesc::conj_b)
  if (g.conj_b) hipLaunchKernelGGL((zgemm_o2_kernel<CF, true>), dim3(grid), dim3(CF::NT), 0, s, g, P, (int)total, persist ? 1 : 0);
  else hipLaunchKernelGGL((zgemm_o2_kernel<CF, false>), dim3(grid), dim3(CF::NT), 0, s, g, P, (int)total, persist ? 1 : 0);
  return hipGetLastError();
}

}  // namespace

int o2_variant_count() { return kO2Variants; }

hipError_t launch_zgemm_o2(const SplitGemmDesc& g, const O2Params& P, hipStream_t s, int variant) {
  const GemmDesc& d = g.d;
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  if (d.skew && d.M != d.N) return hipErrorInvalidValue;
  if (o2_res_stride(d.M, d.K, P.p) > 0x7fffffff || o2_res_stride(d.N, d.K, P.p) > 0x7fffffff)
    return hipErrorInvalidValue;   // per-entry residue offsets are 32-bit in the kernel
  const bool persist = true;
  switch (variant) {
    case 0: return launch_o2_variant<O2V0>(g, P, s, persist);
    case 1: return launch_o2_variant<O2V1>(g, P, s, persist);
    case 2: return launch_o2_variant<O2V2>(g, P, s, persist);
    case 3: return launch_o2_variant<O2V3>(g, P, s, persist);
    case 4: return launch_o2_variant<O2V4>(g, P, s, persist);
    case 5: return launch_o2_variant<O2V4>(g, P, s, false);
    case 6: return launch_o2_variant<O2V1>(g, P, s, false);
    case 7: return launch_o2_variant<O2V7>(g, P, s, persist);
    case 8: return launch_o2_variant<O2V8>(g, P, s, persist);
    case 9: return launch_o2_variant<O2V9>(g, P, s, persist);
    case 10: return launch_o2_variant<O2V10>(g, P, s, persist);
    case 11: return launch_o2_variant<O2V8>(g, P, s, false);
    case 12: return launch_o2_variant<O2V12>(g, P, s, persist);
    case 13: return launch_o2_variant<O2V12>(g, P, s, false);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace qtx
