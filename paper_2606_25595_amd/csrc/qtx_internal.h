// Internal declarations shared by the gfx950 kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace qtx {

// ---------------------------------------------------------------- complex helpers
__host__ __device__ inline double2 cmk(double re, double im) { double2 r; r.x = re; r.y = im; return r; }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return cmk(a.x - b.x, a.y - b.y); }
// Explicit FMAs: with contraction left to the compiler, two instantiations of
// one kernel may fuse different products and round differently.
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return cmk(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
__host__ __device__ inline double2 cconj(double2 a) { return cmk(a.x, -a.y); }
__host__ __device__ inline double2 cinv(double2 a) {
  // 1/a with Smith's scaling to avoid overflow of |a|^2
  if (fabs(a.x) >= fabs(a.y)) {
    double r = a.y / a.x, den = a.x + a.y * r;
    return cmk(1.0 / den, -r / den);
  } else {
    double r = a.x / a.y, den = a.x * r + a.y;
    return cmk(r / den, -1.0 / den);
  }
}

enum Op { OP_N = 0, OP_C = 1 };

// An epilogue addend: out += coef * (scale_by_batch ? bscal[z] : 1) * op(X_z), or with
// diag = 1 the diagonal matrix of the vector X_z (element r at X_z[r], added where r == c).
struct Addend {
  const double2* const* tX = nullptr;   // per-batch-entry pointers (overrides X + z*stride)
  const double2* X = nullptr;
  int64_t ld = 0, stride = 0;
  double2 coef = {0.0, 0.0};
  int op = OP_N;
  int scale_by_batch = 0;
  int diag = 0;
};

// op(X)[r][c] of an addend (the caller checks diag addends for r == c).
__device__ inline double2 addend_value(const double2* X, int diag, int op, int64_t ld, int r, int c) {
  if (diag) return op == OP_N ? X[r] : cconj(X[r]);
  return op == OP_N ? X[(int64_t)r * ld + c] : cconj(X[(int64_t)c * ld + r]);
}

constexpr int kMaxAddends = 3;

// Batched complex GEMM with a fused epilogue:
//   C_z = alpha * op(A_z) op(B_z) + sum_t addend_t + diag * (diag_by_batch ? bscal[z] : 1) * I
// op(A) is M x K, op(B) is K x N, C is M x N, row-major; batch strides in elements.
struct GemmDesc {
  // Optional per-batch-entry operand pointers (device arrays indexed by z); when
  // set they replace base + z * stride.
  const double2* const* tA = nullptr;
  const double2* const* tB = nullptr;
  double2* const* tC = nullptr;
  int M = 0, N = 0, K = 0;
  int opA = OP_N, opB = OP_N;
  const double2* A = nullptr; int64_t lda = 0, sA = 0;
  const double2* B = nullptr; int64_t ldb = 0, sB = 0;
  double2* C = nullptr; int64_t ldc = 0, sC = 0;
  double2 alpha = {1.0, 0.0};
  Addend add[kMaxAddends];
  double2 diag = {0.0, 0.0};
  int diag_by_batch = 0;
  const double* bscal = nullptr;   // per-batch real scalars (the energies), device
  int batch = 1;
  // skew = 1: the caller guarantees that C_z is skew-Hermitian (M == N, every addend
  // skew-Hermitian, diag purely imaginary).  The FP64, FP32 and INT8 kernels then
  // compute only the elements r <= c, write each r < c element also at (c, r) as
  // -conj, and store the diagonal with its real part set to zero; the other schemes
  // compute every element.
  int skew = 0;
  // Output tile edge of the FP64 / FP32 and split-digit products: 32 or 64, or 0 for the
  // rule from the shape (the autotuner's choice when it has one).  Results do not depend
  // on it.
  int tile = 0;
  // Inversion update only (C = X + A B with X = C): columns [skip_c0, skip_c1) of B are
  // zero, so C keeps its values there and output tiles inside that range are skipped.
  int skip_c0 = 0, skip_c1 = 0;
};

// Precision schemes of the complex block products.
enum Prec { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16_SPLIT = 2, PREC_FP16_SPLIT = 3, PREC_INT8_OZAKI2 = 4 };

// Kernel symbol families of the complex GEMM (same code, separate names).
enum GemmKind { GEMM_PRODUCT = 0, GEMM_INV_UPDATE = 1, GEMM_ELEMENTWISE = 2 };
hipError_t launch_zgemm_f64(const GemmDesc& d, hipStream_t s, int kind = GEMM_PRODUCT);
// Same product with operands rounded to FP32 and FP32 accumulation (epilogue in FP64).
hipError_t launch_zgemm_f32(const GemmDesc& d, hipStream_t s);

// Split operands for the slice-product GEMM (FP16 / BF16 digits, FP64 recombination).
// S = op(X) viewed as rows x cols (cols = the contraction dimension K):
// S[r][k] = X[r][k] (trans = 0) or X[k][r] (trans = 1), conjugated if conj = 1.
struct SplitDesc {
  const double2* const* tX = nullptr;   // per-batch-entry source pointers (optional)
  const double2* X = nullptr; int64_t ld = 0, stride = 0;
  int rows = 0, cols = 0;
  int trans = 0, conj = 0;
  void* S = nullptr; int64_t s_stride = 0;       // digits / residues per batch entry (elements)
  int32_t* E = nullptr; int64_t e_stride = 0;    // row exponents per batch entry
  int batch = 1;
};
struct SplitGemmDesc {
  GemmDesc d;                                     // M, N, K, C, alpha, epilogue (A/B unused)
  const void* SA = nullptr; int64_t sa_stride = 0;   // rows = M
  const void* SB = nullptr; int64_t sb_stride = 0;   // rows = N
  const int32_t* EA = nullptr; int64_t ea_stride = 0;
  const int32_t* EB = nullptr; int64_t eb_stride = 0;
  // INT8 scheme: SB / EB hold the conversion of the matrix X whose conjugate transpose
  // op(B) is, made for X as a left operand (same rows, exponents and layout); the
  // product negates its imaginary residues (exactly the right-operand conversion of X^H).
  int conj_b = 0;
};
bool split_supported(int fmt, int ns);                    // fmt 0 = FP16, 1 = BF16
size_t split_bytes(int rows, int cols, int ns, int batch);
int64_t split_digit_stride(int rows, int cols, int ns);
int64_t split_exp_stride(int rows, int cols);
hipError_t launch_split(const SplitDesc& sd, int fmt, int ns, hipStream_t s);
hipError_t launch_zgemm_split(const SplitGemmDesc& g, int fmt, int ns, hipStream_t s);
// Row exponents only: E[r] with max_k |S[r][k]| 2^-E[r] in [1/4, 1/2) (0 for a zero row,
// kExpNonFinite for a row holding NaN or Inf).
hipError_t launch_split_exp(const SplitDesc& sd, hipStream_t s);
// Exponent of an operand row (column of op(B)) that holds a NaN or an Inf.  Its digits
// or residues are written as zeros and every product output in that row (column) is
// NaN, so a non-finite operand element spoils the same outputs it would in FP64
// arithmetic and the solver's finiteness check sees it.
constexpr int kExpNonFinite = 0x40000000;

// Modular (Ozaki II) INT8 products.  Moduli m_0 > m_1 > ... are odd and pairwise
// coprime (kO2Moduli); an operand row r becomes the integer vector
// X'[r][k] = rint(S[r][k] 2^{k_bits + 1 - E[r]}), |X'| <= 2^k_bits, stored as its
// symmetric residues mod every m_i (int8).  The product of the residues is exact
// in INT32 and the CRT gives sum_k A' B' exactly modulo M = prod m_i, which holds
// the true value because 2 K 4^k_bits < M / 2.
constexpr int kO2MaxModuli = 16;
struct O2Params {
  int p = 0;                     // number of moduli
  int kbits = 0;                 // operand integer bits
  double m[kO2MaxModuli];        // moduli
  double inv_m[kO2MaxModuli];    // 1 / m_i (rounded)
  double u[kO2MaxModuli];        // (M / m_i)^-1 mod m_i
  double M = 0.0;                // prod m_i (rounded)
};
bool o2_params(int p, int K, O2Params* out);               // false if p or K is out of range
int o2_modulus(int i);                                      // i-th modulus (0 outside 0..15)
int64_t o2_res_stride(int rows, int cols, int p);           // bytes of residues per batch entry
// Row exponents (as launch_split_exp) and residues of one operand.
hipError_t launch_o2_convert(const SplitDesc& sd, const O2Params& P, hipStream_t s);
// Tile variants of the INT8 product kernel (bitwise the same results; they differ
// in tile height, threads, LDS ring shape and workgroups per CU).
constexpr int kO2Variants = 14;
int o2_variant_count();
hipError_t launch_zgemm_o2(const SplitGemmDesc& g, const O2Params& P, hipStream_t s, int variant);

// Gauss-Jordan inversion with implicit partial pivoting, batched.
// X_z (n x n, ld n, stride sX) is overwritten; the inverse is written to Out_z.
struct GjeWork {
  double2* Wp = nullptr;      // [batch][n][nb]   panel transform minus pivot unit columns
  double2* Tp = nullptr;      // [batch][nb][n]   pivot rows (panel columns zeroed)
  int32_t* prow = nullptr;    // [batch][n]       physical pivot row of each step
  int32_t* used = nullptr;    // [batch][n]       row already used as pivot
};
int gje_panel_width(int n);
size_t gje_work_bytes(int n, int batch);
GjeWork gje_carve(void* base, int n, int batch);
hipError_t launch_gje_invert(int n, double2* X, int64_t sX, double2* Out, int64_t sOut, int batch,
                             const GjeWork& w, int32_t* status, hipStream_t s,
                             double2* const* tOut = nullptr);

// FPX storage codec: FP64 <-> X-bit floats (X in 16..56, multiples of 8), encode
// reads n doubles and writes n X / 8 bytes, decode the reverse.
bool fpx_supported(int bits);
hipError_t launch_fpx(bool encode, int bits, int64_t n, const void* src, void* dst, hipStream_t s);
// Batched: entry z encodes n doubles at x + z * sx into the byte buffer dst[z] (a device
// table of count pointers); the NaN fill writes the NaN code over the 2 counts[z] values
// (counts in complex elements) of dst[z] of every entry with status[z] != 0.
hipError_t launch_fpx_encode_entries(int bits, int64_t n, const double* x, int64_t sx, uint8_t* const* dst, int count,
                                     hipStream_t s);
hipError_t launch_fpx_nan_fill_entries(int bits, const int64_t* counts, uint8_t* const* dst, int count,
                                       const int32_t* status, hipStream_t s);

// Status / NaN fill / observables helpers.
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_hash(double2* p, int64_t n, uint32_t seed, hipStream_t s);
hipError_t launch_nan_fill_failed(double2* X, int64_t per_batch, int64_t stride, int batch,
                                  const int32_t* status, hipStream_t s);
hipError_t launch_check_finite(const double2* X, int64_t per_batch, int64_t stride, int batch,
                               int32_t* status, hipStream_t s);
// Per-entry variants (pointer tables): entry z covers counts[z] elements at t[z].
hipError_t launch_check_finite_entries(const double2* const* t, int64_t count, int batch, int32_t* status,
                                       hipStream_t s);
hipError_t launch_nan_fill_entries(double2* const* t, const int64_t* counts, int batch, const int32_t* status,
                                   hipStream_t s);
// Split energies: st[z] takes st[part[z]] where part[z] >= 0 and st[z] is OK.
hipError_t launch_status_merge(int32_t* st, const int32_t* part, int batch, hipStream_t s);
// X <- -X^H in place for `count` b x b blocks t[0 .. count-1].
hipError_t launch_neg_ctrans_entries(double2* const* t, int b, int count, hipStream_t s);
// dst[m] = -src[m]^H for `count` b x b blocks (distinct buffers).
hipError_t launch_neg_ctrans_copy(const double2* const* src, double2* const* dst, int b, int count, hipStream_t s);
hipError_t launch_scatter_status(const int32_t* st, int32_t* const* dst, int batch, hipStream_t s);
// J[e][i] = 2 Re Tr[(Hu_i - E_e Su_i) G^<_{i+1,i}] for the n_b - 1 bonds of n_e energies
// (G^<_{i+1,i} = -(GLu_i)^H; Su may be null for S = I; GLu of energy e at e * sGu).
hipError_t launch_bond_currents(int b, int n_b, int n_e, const double2* Hu, const double2* Su, const double* E,
                                const double2* GLu, int64_t sGu, double* J, hipStream_t s);
hipError_t launch_observables(int b, int n_e, const double2* G, const double2* GL, int64_t sG,
                              const double2* M1, const double2* M2, const double2* gam,
                              const double* fL, double* T, double* j, hipStream_t s);

}  // namespace qtx
