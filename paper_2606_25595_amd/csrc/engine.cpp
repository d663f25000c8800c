// Host engine and C ABI of the selected Green's-function solver.
//
// Per energy the solve is block Gaussian elimination of the BT system
// M(E) = E S - H - Sigma^R(E) (Section IV-A) in recursive Green's function form,
// applied to the quadratic system M G^< M^H = Sigma^< of Eq. 2 (G row of
// Table I, Section II-A).  All energies of a chunk advance together: every
// step below is one batched launch over the chunk (energies are independent,
// Section II-A), so each launch carries chunk x (tiles per block) workgroups.
//
// Forward (i = 0 .. n_b-1), x_i = left-connected G^R, xl_i = left-connected G^<:
//   x_0 = A_0^-1,  x_i = (A_i - L_{i-1} x_{i-1} U_{i-1})^-1
//   xl_i = x_i Q_i x_i^H,  Q_0 = B_0,  Q_i = B_i + L_{i-1} xl_{i-1} L_{i-1}^H
// Backward (i = n_b-2 .. 0), from G_{n-1} = x_{n-1}, G^<_{n-1} = xl_{n-1}:
//   P = x_i U_i, R = L_i x_i
//   G^R_{i,i+1} = -P G_{i+1},  G^R_{i+1,i} = -G_{i+1} R,  G^R_ii = x_i - G^R_{i,i+1} R
//   V = P G^<_{i+1},  W = G^R_{i,i+1} L_i,  Y = W xl_i,  Z = xl_i L_i^H
//   G^<_{i,i+1} = -V - Z G_{i+1}^H
//   G^<_ii = xl_i + V P^H - Y + Y^H       (Y^H = -xl_i L_i^H (G^R_{i,i+1})^H because
//                                           xl_i is skew-Hermitian, Section II-A)
// x_i is stored in the G^R_ii output slot and xl_i in the G^<_ii slot, and both
// are overwritten in place by the backward pass.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qtx_internal.h"
#include "../../include/qtx_rgf.h"

using namespace qtx;

struct ProfFamily {
  struct Rec { hipEvent_t a, b; double flops; };
  std::vector<Rec> pending;
  double ms = 0.0, flops = 0.0;
  int64_t launches = 0;
};

struct qtx_rgf_ctx_s {
  int device = 0;
  size_t ws_cap = 0;       // 0 = automatic
  void* ws = nullptr;
  size_t ws_size = 0;
  qtx_status sticky = QTX_OK;
  std::string tune_path;
  bool profiling = false;
  ProfFamily prof[2];
  std::vector<hipEvent_t> event_pool;
};

namespace {

hipEvent_t pool_event(qtx_rgf_ctx ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Bracket a launch with events when profiling is on.
struct ProfScope {
  qtx_rgf_ctx ctx;
  int fam;
  hipStream_t s;
  double flops;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(qtx_rgf_ctx c, int f, hipStream_t st, double fl) : ctx(c), fam(f), s(st), flops(fl) {
    if (!ctx || !ctx->profiling) return;
    a = pool_event(ctx);
    b = pool_event(ctx);
    if (a) (void)hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (!a || !b) return;
    (void)hipEventRecord(b, s);
    ctx->prof[fam].pending.push_back({a, b, flops});
  }
};

}  // namespace

namespace {

const size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

qtx_status hip_fail(qtx_rgf_ctx ctx, hipError_t e) {
  if (e == hipSuccess) return QTX_OK;
  if (ctx) ctx->sticky = QTX_ERR_HIP;
  return QTX_ERR_HIP;
}

#define QTX_TRY(expr)                                  \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return hip_fail(ctx, _e);    \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Make sure the context holds at least `bytes` of workspace.  Growing waits for
// all work on the device first (the old buffer may still be in use).
qtx_status ensure_ws(qtx_rgf_ctx ctx, size_t bytes) {
  if (bytes <= ctx->ws_size) return QTX_OK;
  QTX_TRY(hipDeviceSynchronize());
  if (ctx->ws) {
    QTX_TRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_size = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return QTX_ERR_NOMEM;
  }
  ctx->ws = p;
  ctx->ws_size = bytes;
  return QTX_OK;
}

size_t ws_budget(qtx_rgf_ctx ctx) {
  if (ctx->ws_cap) return ctx->ws_cap;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return (size_t)1 << 30;
  return (fr + ctx->ws_size) / 4;
}

// ---------------------------------------------------------------- operands

// A per-batch matrix operand: element (z, r, c) at p + z*stride + r*ld + c.
struct Mat {
  const double2* p = nullptr;
  int64_t stride = 0;
  int64_t ld = 0;
};

// Precision scheme of the block products: qtx_prec -> (kind, 16-bit format, slices).
struct Scheme {
  int prec = QTX_FP64;
  int fmt = 0;      // split: 0 = FP16 digits, 1 = BF16 digits
  int ns = 0;       // split: slices per operand
  bool split() const { return prec == QTX_BF16_SPLIT || prec == QTX_FP16_SPLIT; }
};

bool make_scheme(int prec, int n_slices, Scheme* out) {
  Scheme sc;
  sc.prec = prec;
  if (prec == QTX_FP64 || prec == QTX_FP32) { *out = sc; return true; }
  if (prec != QTX_BF16_SPLIT && prec != QTX_FP16_SPLIT) return false;
  sc.fmt = (prec == QTX_BF16_SPLIT) ? 1 : 0;
  sc.ns = n_slices > 0 ? n_slices : 2;
  if (!split_supported(sc.fmt, sc.ns)) return false;
  *out = sc;
  return true;
}

// Workspace of one split operand (rows = cols = b), per batch entry.
size_t split_operand_bytes(int b, const Scheme& sc) {
  return sc.split() ? split_bytes(b, b, sc.ns, 1) + 512 : 0;
}

struct SplitBufs {
  uint16_t* S[2] = {nullptr, nullptr};
  int32_t* E[2] = {nullptr, nullptr};
};

// Carve two split operands for `batch` entries from w (advances w).
SplitBufs carve_split(char*& w, int b, const Scheme& sc, int batch) {
  SplitBufs sb;
  if (!sc.split()) return sb;
  for (int q = 0; q < 2; ++q) {
    const size_t dig = (size_t)split_digit_stride(b, b, sc.ns) * sizeof(uint16_t) * batch;
    const size_t ex = (size_t)split_exp_stride(b, b) * sizeof(int32_t) * batch;
    sb.S[q] = (uint16_t*)w; w += align_up(dig);
    sb.E[q] = (int32_t*)w; w += align_up(ex);
  }
  return sb;
}

// One batched complex block product with the context's precision scheme.
// Elementwise (K = 0) launches and anything but b x b x b products stay FP64.
hipError_t run_product(const GemmDesc& d, const Scheme& sc, const SplitBufs& sb, hipStream_t s) {
  if (d.K == 0 || sc.prec == QTX_FP64) return launch_zgemm_f64(d, s);
  if (sc.prec == QTX_FP32) return launch_zgemm_f32(d, s);
  // split: operand A as rows of op(A) (M x K), operand B as columns of op(B) (N x K)
  SplitDesc sa;
  sa.X = d.A; sa.ld = d.lda; sa.stride = d.sA;
  sa.rows = d.M; sa.cols = d.K;
  sa.trans = (d.opA == OP_C); sa.conj = (d.opA == OP_C);
  sa.S = sb.S[0]; sa.E = sb.E[0];
  sa.s_stride = split_digit_stride(d.M, d.K, sc.ns);
  sa.e_stride = split_exp_stride(d.M, d.K);
  sa.batch = d.sA == 0 ? 1 : d.batch;
  SplitDesc sbd;
  sbd.X = d.B; sbd.ld = d.ldb; sbd.stride = d.sB;
  sbd.rows = d.N; sbd.cols = d.K;
  sbd.trans = (d.opB == OP_N); sbd.conj = (d.opB == OP_C);
  sbd.S = sb.S[1]; sbd.E = sb.E[1];
  sbd.s_stride = split_digit_stride(d.N, d.K, sc.ns);
  sbd.e_stride = split_exp_stride(d.N, d.K);
  sbd.batch = d.sB == 0 ? 1 : d.batch;
  hipError_t e = launch_split(sa, sc.fmt, sc.ns, s);
  if (e != hipSuccess) return e;
  e = launch_split(sbd, sc.fmt, sc.ns, s);
  if (e != hipSuccess) return e;
  SplitGemmDesc g;
  g.d = d;
  g.SA = sa.S; g.sa_stride = (d.sA == 0) ? 0 : sa.s_stride;
  g.SB = sbd.S; g.sb_stride = (d.sB == 0) ? 0 : sbd.s_stride;
  g.EA = sa.E; g.ea_stride = (d.sA == 0) ? 0 : sa.e_stride;
  g.EB = sbd.E; g.eb_stride = (d.sB == 0) ? 0 : sbd.e_stride;
  return launch_zgemm_split(g, sc.fmt, sc.ns, s);
}

struct Gemm {
  qtx_rgf_ctx ctx;
  hipStream_t s;
  int b;
  int batch;
  const double* energies;   // device, per batch entry
  Scheme sc;
  SplitBufs sb;

  // C = alpha * op(A) op(B) + addends (+ diag * E_z I)
  hipError_t run(int opA, Mat A, int opB, Mat B, double2* C, int64_t sC, double2 alpha,
                 std::initializer_list<Addend> adds, double2 diag = cmk(0, 0), int K = -1) const {
    GemmDesc d;
    d.M = b; d.N = b; d.K = (K < 0) ? b : K;
    d.opA = opA; d.opB = opB;
    d.A = A.p; d.lda = A.ld ? A.ld : b; d.sA = A.stride;
    d.B = B.p; d.ldb = B.ld ? B.ld : b; d.sB = B.stride;
    d.C = C; d.ldc = b; d.sC = sC;
    d.alpha = alpha;
    int q = 0;
    for (const Addend& a : adds) {
      if (q < kMaxAddends) {
        d.add[q] = a;
        if (d.add[q].ld == 0) d.add[q].ld = b;   // blocks are b x b unless stated
        ++q;
      }
    }
    d.diag = diag;
    d.diag_by_batch = 1;
    d.bscal = energies;
    d.batch = batch;
    if (d.K == b) {
      ProfScope ps(ctx, QTX_KERNEL_GEMM, s, 8.0 * (double)b * b * b * batch);
      return run_product(d, sc, sb, s);
    }
    return run_product(d, sc, sb, s);
  }
};

inline Addend addend(const double2* X, int64_t stride, double2 coef, int op = OP_N, int64_t ld = 0,
                     int by_batch = 0) {
  Addend a;
  a.X = X; a.stride = stride; a.coef = coef; a.op = op; a.ld = ld; a.scale_by_batch = by_batch;
  return a;
}

// Per-energy workspace of the RGF path, in b*b blocks.
constexpr int kTemps = 6;

size_t per_energy_bytes(int b, const Scheme& sc) {
  const size_t bb = (size_t)b * b * sizeof(double2);
  return align_up(bb) * (1 + kTemps + 2) + align_up(gje_work_bytes(b, 1)) + 2 * split_operand_bytes(b, sc) + 64;
}

bool valid_problem(const qtx_rgf_problem* p) {
  if (!p) return false;
  if (p->n_b < 1 || p->b < 1 || p->n_e < 1 || p->b > 1024) return false;
  if (!p->energies || !p->H_d || !p->SR_d || !p->SL_d) return false;
  if (p->n_b > 1 && (!p->H_u || !p->H_l)) return false;
  if (!(p->flags & QTX_S_IDENTITY)) {
    if (!p->S_d) return false;
    if (p->n_b > 1 && (!p->S_u || !p->S_l)) return false;
  }
  if (!p->GR_d || !p->GL_d) return false;
  if (p->n_b > 1 && (!p->GR_u || !p->GR_l || !p->GL_u)) return false;
  if (p->flags & QTX_WANT_GREATER) {
    if (!p->SG_d || !p->GG_d) return false;
    if (p->n_b > 1 && !p->GG_u) return false;
  }
  for (int i = 0; i < p->n_e; ++i)
    if (!std::isfinite(p->energies[i])) return false;
  return true;
}

qtx_status check_supported(const qtx_rgf_problem* p) {
  if (p->SL_u || p->SL_l || p->SG_u || p->SG_l) return QTX_ERR_UNSUPPORTED;   // BT Sigma^<, Sigma^>
  Scheme sc;
  if (!make_scheme(p->prec, p->n_slices, &sc)) return QTX_ERR_UNSUPPORTED;
  if (p->prec_lesser >= 0 && !make_scheme(p->prec_lesser, p->n_slices_lesser, &sc)) return QTX_ERR_UNSUPPORTED;
  if (p->flags & ~(uint32_t)(QTX_S_IDENTITY | QTX_WANT_GREATER)) return QTX_ERR_ARG;
  return QTX_OK;
}

// One energy chunk [e0, e0+ne) of problem p.
qtx_status solve_chunk(qtx_rgf_ctx ctx, const qtx_rgf_problem& p, int e0, int ne, hipStream_t s,
                       const double* d_en) {
  const int b = p.b, nb = p.n_b;
  const int64_t bb = (int64_t)b * b;
  const int64_t sE = (int64_t)nb * bb;           // per-energy stride of [n_e][n_b] arrays
  const int64_t sEu = (int64_t)(nb - 1) * bb;    // per-energy stride of [n_e][n_b-1] arrays
  const bool S_id = (p.flags & QTX_S_IDENTITY) != 0;
  const bool greater = (p.flags & QTX_WANT_GREATER) != 0;

  // carve the workspace
  char* w = (char*)ctx->ws;
  const size_t blk = align_up((size_t)ne * bb * sizeof(double2));
  double2* X = (double2*)w; w += blk;
  double2* Tm[kTemps];
  for (int t = 0; t < kTemps; ++t) { Tm[t] = (double2*)w; w += blk; }
  double2* Uw = (double2*)w; w += blk;           // per-energy U_i when it depends on E
  double2* Lw = (double2*)w; w += blk;           // per-energy L_i when it depends on E
  GjeWork gw = gje_carve(w, b, ne); w += align_up(gje_work_bytes(b, ne));
  int32_t* st = (int32_t*)w; w += align_up((size_t)ne * sizeof(int32_t));
  const double* en = d_en + e0;
  Scheme scheme, scheme_l;
  make_scheme(p.prec, p.n_slices, &scheme);
  if (p.prec_lesser >= 0) make_scheme(p.prec_lesser, p.n_slices_lesser, &scheme_l);
  else scheme_l = scheme;
  // split buffers sized for the larger of the two schemes
  Scheme big = (scheme_l.split() && (!scheme.split() || scheme_l.ns > scheme.ns)) ? scheme_l : scheme;
  SplitBufs sbufs = carve_split(w, b, big, ne);

  const double2* H_d = (const double2*)p.H_d;
  const double2* H_u = (const double2*)p.H_u;
  const double2* H_l = (const double2*)p.H_l;
  const double2* S_d = (const double2*)p.S_d;
  const double2* S_u = (const double2*)p.S_u;
  const double2* S_l = (const double2*)p.S_l;
  const double2* SR_d = (const double2*)p.SR_d + (int64_t)e0 * sE;
  const double2* SR_u = p.SR_u ? (const double2*)p.SR_u + (int64_t)e0 * sEu : nullptr;
  const double2* SR_l = p.SR_l ? (const double2*)p.SR_l + (int64_t)e0 * sEu : nullptr;
  double2* GR_d = (double2*)p.GR_d + (int64_t)e0 * sE;
  double2* GR_u = nb > 1 ? (double2*)p.GR_u + (int64_t)e0 * sEu : nullptr;
  double2* GR_l = nb > 1 ? (double2*)p.GR_l + (int64_t)e0 * sEu : nullptr;

  struct Rhs {
    const double2* B;   // diagonal blocks of Sigma^< or Sigma^>
    double2* Gd;
    double2* Gu;
  };
  std::vector<Rhs> rhs;
  rhs.push_back({(const double2*)p.SL_d + (int64_t)e0 * sE, (double2*)p.GL_d + (int64_t)e0 * sE,
                 nb > 1 ? (double2*)p.GL_u + (int64_t)e0 * sEu : nullptr});
  if (greater)
    rhs.push_back({(const double2*)p.SG_d + (int64_t)e0 * sE, (double2*)p.GG_d + (int64_t)e0 * sE,
                   nb > 1 ? (double2*)p.GG_u + (int64_t)e0 * sEu : nullptr});

  QTX_TRY(launch_fill_i32(st, 0, ne, s));

  Gemm g{ctx, s, b, ne, en, scheme, sbufs};     // retarded chain
  Gemm gl{ctx, s, b, ne, en, scheme_l, sbufs};  // lesser / greater chain
  const double2 one = cmk(1, 0), mone = cmk(-1, 0), zero = cmk(0, 0);

  // The coupling operands: U_i = E S_{i,i+1} - H_{i,i+1} - Sigma^R_{i,i+1}(E) and the
  // same for L_i.  With S = I and no Sigma^R coupling they are -H_u, -H_l, shared
  // by all energies: the operand is H with sign -1.  Otherwise they are assembled
  // per energy into the workspace (sign +1).
  const bool shared_UL = S_id && !SR_u && !SR_l;
  auto coupling = [&](int i, Mat& U, double& sU, Mat& L, double& sL) -> hipError_t {
    if (shared_UL) {
      U = Mat{H_u + (int64_t)i * bb, 0, b}; sU = -1.0;
      L = Mat{H_l + (int64_t)i * bb, 0, b}; sL = -1.0;
      return hipSuccess;
    }
    hipError_t e;
    // U_i
    e = g.run(OP_N, Mat{}, OP_N, Mat{}, Uw, bb, zero,
              {addend(S_id ? nullptr : S_u + (int64_t)i * bb, 0, one, OP_N, 0, 1),
               addend(H_u + (int64_t)i * bb, 0, mone),
               addend(SR_u ? SR_u + (int64_t)i * bb : nullptr, sEu, mone)}, zero, 0);
    if (e != hipSuccess) return e;
    e = g.run(OP_N, Mat{}, OP_N, Mat{}, Lw, bb, zero,
              {addend(S_id ? nullptr : S_l + (int64_t)i * bb, 0, one, OP_N, 0, 1),
               addend(H_l + (int64_t)i * bb, 0, mone),
               addend(SR_l ? SR_l + (int64_t)i * bb : nullptr, sEu, mone)}, zero, 0);
    U = Mat{Uw, bb, b}; sU = 1.0;
    L = Mat{Lw, bb, b}; sL = 1.0;
    return e;
  };
  // The diagonal block A_i = E S_ii - H_ii - Sigma^R_ii(E) as epilogue addends.
  auto A_addends = [&](int i, Addend out[3], double2& dg) {
    out[0] = addend(H_d + (int64_t)i * bb, 0, mone);
    out[1] = addend(SR_d + (int64_t)i * bb, sE, mone);
    if (S_id) { out[2] = Addend{}; dg = one; }
    else { out[2] = addend(S_d + (int64_t)i * bb, 0, one, OP_N, 0, 1); dg = zero; }
  };

  Mat U, L;
  double sU = 0, sL = 0;
  // ------------------------------------------------------------ forward
  for (int i = 0; i < nb; ++i) {
    Addend aa[3];
    double2 dg;
    A_addends(i, aa, dg);
    if (i == 0) {
      QTX_TRY(g.run(OP_N, Mat{}, OP_N, Mat{}, X, bb, zero, {aa[0], aa[1], aa[2]}, dg, 0));
    } else {
      QTX_TRY(coupling(i - 1, U, sU, L, sL));
      // T' = L' x_{i-1};   X = A_i - sL sU T' U'
      QTX_TRY(g.run(OP_N, L, OP_N, Mat{GR_d + (int64_t)(i - 1) * bb, sE, b}, Tm[0], bb, one, {}));
      QTX_TRY(g.run(OP_N, Mat{Tm[0], bb, b}, OP_N, U, X, bb, cmk(-sL * sU, 0), {aa[0], aa[1], aa[2]}, dg));
    }
    {
      ProfScope ps(ctx, QTX_KERNEL_INV, s, 8.0 * (double)b * b * b * ne);
      QTX_TRY(launch_gje_invert(b, X, bb, GR_d + (int64_t)i * bb, sE, ne, gw, st, s));
    }
    const Mat xi{GR_d + (int64_t)i * bb, sE, b};
    for (const Rhs& r : rhs) {
      const double2* Bi = r.B + (int64_t)i * bb;
      if (i == 0) {
        QTX_TRY(gl.run(OP_N, xi, OP_N, Mat{Bi, sE, b}, Tm[2], bb, one, {}));
      } else {
        // Y' = L' xl_{i-1};  Q = B_i + Y' L'^H;  Z = x_i Q
        QTX_TRY(gl.run(OP_N, L, OP_N, Mat{r.Gd + (int64_t)(i - 1) * bb, sE, b}, Tm[1], bb, one, {}));
        QTX_TRY(gl.run(OP_N, Mat{Tm[1], bb, b}, OP_C, L, Tm[3], bb, one, {addend(Bi, sE, one)}));
        QTX_TRY(gl.run(OP_N, xi, OP_N, Mat{Tm[3], bb, b}, Tm[2], bb, one, {}));
      }
      // xl_i = Z x_i^H
      QTX_TRY(gl.run(OP_N, Mat{Tm[2], bb, b}, OP_C, xi, r.Gd + (int64_t)i * bb, sE, one, {}));
    }
  }
  // ------------------------------------------------------------ backward
  double2* Pp = Tm[0];
  double2* Rp = Tm[1];
  double2* Vp = Tm[2];
  double2* Wp = Tm[3];
  double2* Yp = Tm[4];
  double2* Zp = Tm[5];
  for (int i = nb - 2; i >= 0; --i) {
    QTX_TRY(coupling(i, U, sU, L, sL));
    const Mat xi{GR_d + (int64_t)i * bb, sE, b};
    const Mat Gn{GR_d + (int64_t)(i + 1) * bb, sE, b};
    double2* GRu = GR_u + (int64_t)i * bb;
    double2* GRl = GR_l + (int64_t)i * bb;
    QTX_TRY(g.run(OP_N, xi, OP_N, U, Pp, bb, one, {}));                       // P' = x_i U'
    QTX_TRY(g.run(OP_N, L, OP_N, xi, Rp, bb, one, {}));                       // R' = L' x_i
    QTX_TRY(g.run(OP_N, Mat{Pp, bb, b}, OP_N, Gn, GRu, sEu, cmk(-sU, 0), {}));   // G_{i,i+1}
    QTX_TRY(g.run(OP_N, Gn, OP_N, Mat{Rp, bb, b}, GRl, sEu, cmk(-sL, 0), {}));   // G_{i+1,i}
    QTX_TRY(g.run(OP_N, Mat{GRu, sEu, b}, OP_N, Mat{Rp, bb, b}, GR_d + (int64_t)i * bb, sE, cmk(-sL, 0),
                  {addend(GR_d + (int64_t)i * bb, sE, one)}));                 // G_ii (in place)
    QTX_TRY(gl.run(OP_N, Mat{GRu, sEu, b}, OP_N, L, Wp, bb, one, {}));        // W' = G_{i,i+1} L' (lesser chain)
    for (const Rhs& r : rhs) {
      const Mat xl{r.Gd + (int64_t)i * bb, sE, b};
      const Mat Gln{r.Gd + (int64_t)(i + 1) * bb, sE, b};
      QTX_TRY(gl.run(OP_N, Mat{Pp, bb, b}, OP_N, Gln, Vp, bb, one, {}));       // V' = P' G<_{i+1}
      QTX_TRY(gl.run(OP_N, Mat{Wp, bb, b}, OP_N, xl, Yp, bb, one, {}));        // Y' = W' xl_i
      QTX_TRY(gl.run(OP_N, xl, OP_C, L, Zp, bb, one, {}));                     // Z' = xl_i L'^H
      // G<_{i,i+1} = -sU V' - sL Z' G_{i+1}^H
      QTX_TRY(gl.run(OP_N, Mat{Zp, bb, b}, OP_C, Gn, r.Gu + (int64_t)i * bb, sEu, cmk(-sL, 0),
                    {addend(Vp, bb, cmk(-sU, 0))}));
      // G<_ii = xl_i + V' P'^H - sL Y' + sL Y'^H   (in place)
      QTX_TRY(gl.run(OP_N, Mat{Vp, bb, b}, OP_C, Mat{Pp, bb, b}, r.Gd + (int64_t)i * bb, sE, one,
                    {addend(r.Gd + (int64_t)i * bb, sE, one), addend(Yp, bb, cmk(-sL, 0)),
                     addend(Yp, bb, cmk(sL, 0), OP_C)}));
    }
  }
  // ------------------------------------------------------------ status
  // Non-finite values propagate into the first blocks; check them.
  QTX_TRY(launch_check_finite(GR_d, bb, sE, ne, st, s));
  for (const Rhs& r : rhs) QTX_TRY(launch_check_finite(r.Gd, bb, sE, ne, st, s));
  QTX_TRY(launch_nan_fill_failed(GR_d, sE, sE, ne, st, s));
  if (nb > 1) {
    QTX_TRY(launch_nan_fill_failed(GR_u, sEu, sEu, ne, st, s));
    QTX_TRY(launch_nan_fill_failed(GR_l, sEu, sEu, ne, st, s));
  }
  for (const Rhs& r : rhs) {
    QTX_TRY(launch_nan_fill_failed(r.Gd, sE, sE, ne, st, s));
    if (nb > 1) QTX_TRY(launch_nan_fill_failed(r.Gu, sEu, sEu, ne, st, s));
  }
  if (p.status) QTX_TRY(hipMemcpyAsync(p.status + e0, st, ne * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  return QTX_OK;
}

}  // namespace

extern "C" {

const char* qtx_status_str(qtx_status s) {
  switch (s) {
    case QTX_OK: return "QTX_OK";
    case QTX_ERR_ARG: return "QTX_ERR_ARG";
    case QTX_ERR_NOMEM: return "QTX_ERR_NOMEM";
    case QTX_ERR_HIP: return "QTX_ERR_HIP";
    case QTX_ERR_UNSUPPORTED: return "QTX_ERR_UNSUPPORTED";
    case QTX_ERR_SINGULAR: return "QTX_ERR_SINGULAR";
    case QTX_ERR_NONFINITE: return "QTX_ERR_NONFINITE";
  }
  return "QTX_ERR_UNKNOWN";
}

qtx_status qtx_rgf_create(qtx_rgf_ctx* out, int device, size_t workspace_bytes, const char* tune_cache_path) {
  if (!out) return QTX_ERR_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return QTX_ERR_ARG;
  qtx_rgf_ctx ctx = new (std::nothrow) qtx_rgf_ctx_s();
  if (!ctx) return QTX_ERR_NOMEM;
  ctx->device = device;
  ctx->ws_cap = workspace_bytes;
  if (tune_cache_path) ctx->tune_path = tune_cache_path;
  *out = ctx;
  return QTX_OK;
}

qtx_status qtx_rgf_profile(qtx_rgf_ctx ctx, int enable) {
  if (!ctx) return QTX_ERR_ARG;
  ctx->profiling = enable != 0;
  return QTX_OK;
}

qtx_status qtx_rgf_profile_read(qtx_rgf_ctx ctx, int family, double* total_ms, int64_t* launches,
                                double* flops) {
  if (!ctx || family < 0 || family > 1) return QTX_ERR_ARG;
  DeviceGuard guard(ctx->device);
  ProfFamily& f = ctx->prof[family];
  for (auto& r : f.pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      return hip_fail(ctx, hipErrorUnknown);
    f.ms += ms;
    f.flops += r.flops;
    f.launches += 1;
    ctx->event_pool.push_back(r.a);
    ctx->event_pool.push_back(r.b);
  }
  f.pending.clear();
  if (total_ms) *total_ms = f.ms;
  if (launches) *launches = f.launches;
  if (flops) *flops = f.flops;
  f.ms = 0.0; f.flops = 0.0; f.launches = 0;
  return QTX_OK;
}

qtx_status qtx_rgf_destroy(qtx_rgf_ctx ctx) {
  if (!ctx) return QTX_ERR_ARG;
  {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->ws) (void)hipFree(ctx->ws);
    for (auto& f : ctx->prof)
      for (auto& r : f.pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  }
  delete ctx;
  return QTX_OK;
}

size_t qtx_rgf_footprint(const qtx_rgf_problem* p) {
  if (!valid_problem(p)) return 0;
  Scheme sc, scl;
  if (!make_scheme(p->prec, p->n_slices, &sc)) return 0;
  if (p->prec_lesser >= 0 && make_scheme(p->prec_lesser, p->n_slices_lesser, &scl) &&
      scl.split() && (!sc.split() || scl.ns > sc.ns))
    sc = scl;
  return per_energy_bytes(p->b, sc);
}

qtx_status qtx_rgf_solve(qtx_rgf_ctx ctx, const qtx_rgf_problem* probs, int32_t n_probs, void* hip_stream) {
  if (!ctx || !probs || n_probs < 1) return QTX_ERR_ARG;
  if (ctx->sticky != QTX_OK) return ctx->sticky;
  for (int k = 0; k < n_probs; ++k) {
    if (!valid_problem(&probs[k])) return QTX_ERR_ARG;
    qtx_status st = check_supported(&probs[k]);
    if (st != QTX_OK) return st;
  }
  DeviceGuard guard(ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  // plan: energies per chunk from the workspace budget
  const size_t budget = ws_budget(ctx);
  size_t need = 0;
  std::vector<int> chunk(n_probs);
  int max_ne = 0;
  for (int k = 0; k < n_probs; ++k) {
    const qtx_rgf_problem& p = probs[k];
    Scheme sc, scl;
    make_scheme(p.prec, p.n_slices, &sc);
    if (p.prec_lesser >= 0) make_scheme(p.prec_lesser, p.n_slices_lesser, &scl);
    if (scl.split() && (!sc.split() || scl.ns > sc.ns)) sc = scl;
    const size_t per = per_energy_bytes(p.b, sc);
    size_t c = budget > per ? budget / per : 1;
    if (c > (size_t)p.n_e) c = p.n_e;
    if (c < 1) c = 1;
    chunk[k] = (int)c;
    need = std::max(need, per * c + 4096);
    max_ne = std::max(max_ne, p.n_e);
  }
  const size_t en_bytes = align_up((size_t)max_ne * sizeof(double));
  qtx_status st = ensure_ws(ctx, need + en_bytes);
  if (st != QTX_OK) return st;
  double* d_en = (double*)((char*)ctx->ws + ctx->ws_size - en_bytes);
  for (int k = 0; k < n_probs; ++k) {
    const qtx_rgf_problem& p = probs[k];
    QTX_TRY(hipMemcpyAsync(d_en, p.energies, p.n_e * sizeof(double), hipMemcpyHostToDevice, s));
    for (int e0 = 0; e0 < p.n_e; e0 += chunk[k]) {
      const int ne = std::min(chunk[k], p.n_e - e0);
      st = solve_chunk(ctx, p, e0, ne, s, d_en);
      if (st != QTX_OK) return st;
    }
  }
  return QTX_OK;
}

qtx_status qtx_zgemm(qtx_rgf_ctx ctx, char opA, char opB, int32_t M, int32_t N, int32_t K, double alpha_re,
                     double alpha_im, const void* A, int64_t lda, int64_t sA, const void* B, int64_t ldb,
                     int64_t sB, double beta_re, double beta_im, void* C, int64_t ldc, int64_t sC, int32_t batch,
                     int32_t prec, int32_t n_slices, void* hip_stream) {
  if (!ctx) return QTX_ERR_ARG;
  if (ctx->sticky != QTX_OK) return ctx->sticky;
  if ((opA != 'N' && opA != 'C') || (opB != 'N' && opB != 'C')) return QTX_ERR_ARG;
  if (M < 0 || N < 0 || K < 0 || batch < 1 || !C || ldc < N) return QTX_ERR_ARG;
  if (K > 0 && (!A || !B)) return QTX_ERR_ARG;
  if (K > 0 && (lda < (opA == 'N' ? K : M) || ldb < (opB == 'N' ? N : K))) return QTX_ERR_ARG;
  Scheme sc;
  if (!make_scheme(prec, n_slices, &sc)) return QTX_ERR_UNSUPPORTED;
  DeviceGuard guard(ctx->device);
  GemmDesc d;
  d.M = M; d.N = N; d.K = K;
  d.opA = opA == 'N' ? OP_N : OP_C;
  d.opB = opB == 'N' ? OP_N : OP_C;
  d.A = (const double2*)A; d.lda = lda; d.sA = sA;
  d.B = (const double2*)B; d.ldb = ldb; d.sB = sB;
  d.C = (double2*)C; d.ldc = ldc; d.sC = sC;
  d.alpha = cmk(alpha_re, alpha_im);
  if (beta_re != 0.0 || beta_im != 0.0) {
    d.add[0].X = (const double2*)C; d.add[0].ld = ldc; d.add[0].stride = sC; d.add[0].coef = cmk(beta_re, beta_im);
  }
  d.batch = batch;
  SplitBufs sb;
  if (sc.split() && K > 0) {
    const size_t need = split_bytes(M, K, sc.ns, batch) + split_bytes(N, K, sc.ns, batch) + 4096;
    qtx_status st = ensure_ws(ctx, need);
    if (st != QTX_OK) return st;
    char* w = (char*)ctx->ws;
    sb.S[0] = (uint16_t*)w; w += align_up((size_t)split_digit_stride(M, K, sc.ns) * 2 * batch);
    sb.E[0] = (int32_t*)w; w += align_up((size_t)split_exp_stride(M, K) * 4 * batch);
    sb.S[1] = (uint16_t*)w; w += align_up((size_t)split_digit_stride(N, K, sc.ns) * 2 * batch);
    sb.E[1] = (int32_t*)w;
  }
  QTX_TRY(run_product(d, sc, sb, (hipStream_t)hip_stream));
  return QTX_OK;
}

qtx_status qtx_zinv(qtx_rgf_ctx ctx, int32_t n, const void* A, int64_t sA, void* Ainv, int64_t sAinv,
                    int32_t batch, int32_t* status, void* hip_stream) {
  if (!ctx) return QTX_ERR_ARG;
  if (ctx->sticky != QTX_OK) return ctx->sticky;
  if (n < 1 || n > 1024 || batch < 1 || !A || !Ainv) return QTX_ERR_ARG;
  if (sA < (int64_t)n * n || sAinv < (int64_t)n * n) return QTX_ERR_ARG;
  DeviceGuard guard(ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t nn = (int64_t)n * n;
  const size_t need = align_up((size_t)batch * nn * sizeof(double2)) + align_up(gje_work_bytes(n, batch)) +
                      align_up((size_t)batch * sizeof(int32_t));
  qtx_status st = ensure_ws(ctx, need);
  if (st != QTX_OK) return st;
  char* w = (char*)ctx->ws;
  double2* X = (double2*)w; w += align_up((size_t)batch * nn * sizeof(double2));
  GjeWork gw = gje_carve(w, n, batch); w += align_up(gje_work_bytes(n, batch));
  int32_t* stw = (int32_t*)w;
  QTX_TRY(launch_fill_i32(stw, 0, batch, s));
  // copy A into the workspace through the GEMM epilogue (K = 0)
  GemmDesc d;
  d.M = n; d.N = n; d.K = 0;
  d.C = X; d.ldc = n; d.sC = nn;
  d.alpha = cmk(0, 0);
  d.add[0].X = (const double2*)A; d.add[0].ld = n; d.add[0].stride = sA; d.add[0].coef = cmk(1, 0);
  d.batch = batch;
  QTX_TRY(launch_zgemm_f64(d, s));
  QTX_TRY(launch_gje_invert(n, X, nn, (double2*)Ainv, sAinv, batch, gw, stw, s));
  if (status) QTX_TRY(hipMemcpyAsync(status, stw, batch * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  return QTX_OK;
}

qtx_status qtx_rgf_observables(qtx_rgf_ctx ctx, int32_t b, int32_t n_e, const void* GR_11, const void* GL_11,
                               int64_t sG, const void* gamma_L, const double* f_L, double* T_L, double* j_L,
                               void* hip_stream) {
  if (!ctx) return QTX_ERR_ARG;
  if (ctx->sticky != QTX_OK) return ctx->sticky;
  if (b < 1 || n_e < 1 || !GR_11 || !GL_11 || !gamma_L || !f_L || !T_L || !j_L || sG < (int64_t)b * b)
    return QTX_ERR_ARG;
  DeviceGuard guard(ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t bb = (int64_t)b * b;
  qtx_status st = ensure_ws(ctx, 2 * align_up((size_t)n_e * bb * sizeof(double2)));
  if (st != QTX_OK) return st;
  double2* M1 = (double2*)ctx->ws;
  double2* M2 = (double2*)((char*)ctx->ws + align_up((size_t)n_e * bb * sizeof(double2)));
  GemmDesc d;
  d.M = b; d.N = b; d.K = b;
  d.opA = OP_N; d.opB = OP_N;
  d.A = (const double2*)gamma_L; d.lda = b; d.sA = 0;
  d.B = (const double2*)GR_11; d.ldb = b; d.sB = sG;
  d.C = M1; d.ldc = b; d.sC = bb;
  d.batch = n_e;
  QTX_TRY(launch_zgemm_f64(d, s));
  d.opB = OP_C; d.C = M2;
  QTX_TRY(launch_zgemm_f64(d, s));
  QTX_TRY(launch_observables(b, n_e, (const double2*)GR_11, (const double2*)GL_11, sG, M1, M2,
                             (const double2*)gamma_L, f_L, T_L, j_L, s));
  return QTX_OK;
}

}  // extern "C"
