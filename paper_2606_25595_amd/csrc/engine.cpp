// Host engine and C ABI of the selected Green's-function solver.
//
// Per energy the solve is block Gaussian elimination of the BT system
// M(E) = E S - H - Sigma^R(E) (Section IV-A) in recursive Green's function form,
// applied to the quadratic system M G^< M^H = Sigma^< of Eq. 2 (G row of
// Table I, Section II-A).
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
//
// Batching.  Energies are independent (Section II-A).  A batch is a set of
// entries -- one entry per (problem, energy) -- that share the block size b and
// the precision schemes; its entries are sorted by n_b (descending) so that the
// entries still active at a step form a prefix, and every step of the
// recurrences is one launch over that prefix.  Operands are addressed per entry
// through pointer tables built on the host: a dry pass over the step sequence
// collects every table, one copy uploads them, and the second pass launches.
// Tables that are affine in the entry index (all energies of one problem)
// collapse to base + z * stride.  Batches of different block size run on
// parallel streams; with the graph option the solve is captured once into a
// hipGraph (cached by its signature) and replayed with a single launch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
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

struct GraphCacheEntry {
  uint64_t sig = 0;
  hipGraphExec_t exec = nullptr;
};

// Autotuner record: the tile variant of a product kernel chosen for one product shape
// (M, N, K), batch class and scheme code (the modulus count of the INT8 scheme, else
// kTileCodeBase + 10 prec + slices, whose variants are 0 = 32 x 32 and 1 = 64 x 64
// tiles), with the measured ms per variant.
struct TuneRec {
  int variant = 0;
  std::vector<double> ms;
};
typedef std::tuple<int, int, int, int, int> TuneKey;   // M, N, K, batch class, scheme code
constexpr int kTileCodeBase = 100;

struct qtx_rgf_ctx_s {
  int device = 0;
  size_t ws_cap = 0;       // 0 = automatic
  void* ws = nullptr;
  size_t ws_size = 0;
  qtx_status sticky = QTX_OK;
  std::string tune_path;
  std::map<TuneKey, TuneRec> tune;
  int o2_force = -1;       // >= 0: every INT8 product uses this tile variant
  int tile_force = 0;      // 32 / 64: every FP64 / FP32 / split product uses this tile (the tuner's timing runs)
  bool overlap = false;    // run independent products on a side stream during inversions
  int lane_split = 1;      // stream lanes each batch group is split over
  bool profiling = false;
  bool use_graph = false;
  bool capturing = false;
  ProfFamily prof[3];
  std::vector<hipEvent_t> event_pool;
  // pinned staging of the pointer tables, and the event of its last upload
  void* pinned = nullptr;
  size_t pinned_size = 0;
  hipEvent_t upload_done = nullptr;
  // auxiliary streams (default priority) and fork/join events for parallel batches
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> fork_ev, join_ev;
  // per lane: a side stream for products that overlap the inversion, and its fork/join events
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> side_fork, side_join;
  std::vector<GraphCacheEntry> graphs;
  int64_t graph_launches = 0, graph_captures = 0;
  // split solves with a BT Sigma^< / Sigma^>: the bottom halves' upper blocks -(SL_u)^H
  void* rbt = nullptr;
  size_t rbt_size = 0;
  // the stream of the last call that enqueued work, and the event recorded at its end
  hipStream_t last_s = nullptr;
  hipEvent_t last_done = nullptr;
};

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

#define QTX_TRYS(expr)                                 \
  do {                                                 \
    qtx_status _s = (expr);                            \
    if (_s != QTX_OK) return _s;                       \
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

}  // namespace

// ---------------------------------------------------------------- fixed scratch of qtx_zgemm_noalloc
// The converted operands (digits or residues, and exponents) of qtx_zgemm_noalloc live in
// this fixed device array instead of the context's workspace: one copy per GPU, created by
// the runtime when the library's code object is loaded on that GPU and held until the
// process ends.  On the host the name is only a stand-in, never a device address: the
// address of each GPU's copy is looked up once per device (noalloc_scratch, first from
// qtx_rgf_create) and that address is what the kernels receive.  Nothing in it needs to
// start at zero: a conversion writes every byte the product kernel then reads.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up with that device current on the first
// call for the device and kept.
qtx_status noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return QTX_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    DeviceGuard guard(device);
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return QTX_ERR_HIP;
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return QTX_OK;
}

void drop_graphs(qtx_rgf_ctx ctx) {
  for (auto& g : ctx->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  ctx->graphs.clear();
}

// Make sure the context holds at least `bytes` of workspace.  Growing waits for
// all work on the device first (the old buffer may still be in use) and drops
// cached graphs (they hold addresses inside the old buffer).
qtx_status ensure_ws(qtx_rgf_ctx ctx, size_t bytes) {
  if (bytes <= ctx->ws_size) return QTX_OK;
  QTX_TRY(hipDeviceSynchronize());
  drop_graphs(ctx);
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

// Room for the bottom halves' reversed BT right-hand-side blocks (same growth rule as
// the workspace).
qtx_status ensure_rbt(qtx_rgf_ctx ctx, size_t bytes) {
  if (bytes <= ctx->rbt_size) return QTX_OK;
  QTX_TRY(hipDeviceSynchronize());
  drop_graphs(ctx);
  if (ctx->rbt) {
    QTX_TRY(hipFree(ctx->rbt));
    ctx->rbt = nullptr;
    ctx->rbt_size = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return QTX_ERR_NOMEM;
  }
  ctx->rbt = p;
  ctx->rbt_size = bytes;
  return QTX_OK;
}

qtx_status ensure_pinned(qtx_rgf_ctx ctx, size_t bytes) {
  if (ctx->upload_done) QTX_TRY(hipEventSynchronize(ctx->upload_done));   // the last upload has read it
  if (bytes <= ctx->pinned_size) return QTX_OK;
  if (ctx->pinned) QTX_TRY(hipHostFree(ctx->pinned));
  ctx->pinned = nullptr;
  ctx->pinned_size = 0;
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return QTX_ERR_NOMEM;
  }
  ctx->pinned = p;
  ctx->pinned_size = bytes;
  return QTX_OK;
}

qtx_status ensure_aux(qtx_rgf_ctx ctx, size_t n) {
  while (ctx->aux.size() < n) {
    hipStream_t st;
    hipEvent_t a, b;
    QTX_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    QTX_TRY(hipEventCreateWithFlags(&a, hipEventDisableTiming));
    QTX_TRY(hipEventCreateWithFlags(&b, hipEventDisableTiming));
    ctx->aux.push_back(st);
    ctx->fork_ev.push_back(a);
    ctx->join_ev.push_back(b);
  }
  return QTX_OK;
}

qtx_status ensure_side(qtx_rgf_ctx ctx, size_t n) {
  while (ctx->side.size() < n) {
    hipStream_t st;
    hipEvent_t a, b;
    QTX_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    QTX_TRY(hipEventCreateWithFlags(&a, hipEventDisableTiming));
    QTX_TRY(hipEventCreateWithFlags(&b, hipEventDisableTiming));
    ctx->side.push_back(st);
    ctx->side_fork.push_back(a);
    ctx->side_join.push_back(b);
  }
  return QTX_OK;
}

size_t ws_budget(qtx_rgf_ctx ctx) {
  if (ctx->ws_cap) return ctx->ws_cap;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return (size_t)1 << 30;
  return (fr + ctx->ws_size) / 4;
}

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

// Bracket a launch with events when profiling is on (never inside a capture).
struct ProfScope {
  qtx_rgf_ctx ctx;
  int fam;
  hipStream_t s;
  double flops;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(qtx_rgf_ctx c, int f, hipStream_t st, double fl, bool active) : ctx(c), fam(f), s(st), flops(fl) {
    if (!active || !ctx || !ctx->profiling || ctx->capturing) return;
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

// Every call on a context uses the context's one workspace (temporaries, converted
// operands, pointer tables).  A call on a different stream than the previous call
// first makes its stream wait for the event recorded at the end of that call, so
// that two calls never use the workspace at the same time.  Calls on a stream that
// is being captured into a caller's graph are not ordered this way (the header says
// so): the graph's launches are the caller's to order.
struct StreamOrder {
  qtx_rgf_ctx ctx;
  hipStream_t s;
  bool track = false;
  StreamOrder(qtx_rgf_ctx c, hipStream_t st) : ctx(c), s(st) {}
  qtx_status enter() {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s != nullptr) QTX_TRY(hipStreamIsCapturing(s, &cs));
    track = cs == hipStreamCaptureStatusNone;
    if (track && ctx->last_done && ctx->last_s != s) QTX_TRY(hipStreamWaitEvent(s, ctx->last_done, 0));
    return QTX_OK;
  }
  // After the call's work is enqueued (also after a failed call: the event then marks
  // whatever was enqueued).
  qtx_status leave() {
    if (!track) return QTX_OK;
    if (!ctx->last_done) QTX_TRY(hipEventCreateWithFlags(&ctx->last_done, hipEventDisableTiming));
    QTX_TRY(hipEventRecord(ctx->last_done, s));
    ctx->last_s = s;
    return QTX_OK;
  }
};

// The same as a scope: leave() runs when the call returns (its status is dropped).
struct OrderScope {
  StreamOrder o;
  bool entered = false;
  OrderScope(qtx_rgf_ctx c, hipStream_t st) : o(c, st) {}
  qtx_status enter() {
    const qtx_status st = o.enter();
    entered = st == QTX_OK;
    return st;
  }
  ~OrderScope() {
    if (entered) (void)o.leave();
  }
};

// Run f() between enter() and leave() of the stream order of ctx on stream s.
template <class F>
qtx_status ordered(qtx_rgf_ctx ctx, hipStream_t s, F&& f) {
  StreamOrder o(ctx, s);
  QTX_TRYS(o.enter());
  const qtx_status st = f();
  const qtx_status sl = o.leave();
  return st != QTX_OK ? st : sl;
}

// ---------------------------------------------------------------- precision schemes

struct Scheme {
  int prec = QTX_FP64;
  int fmt = 0;      // split: 0 = FP16 digits, 1 = BF16 digits
  int ns = 0;       // split: slices per operand; Ozaki II: moduli
  bool split() const { return prec == QTX_BF16_SPLIT || prec == QTX_FP16_SPLIT; }
  bool o2() const { return prec == QTX_INT8_OZAKI2; }
  bool sliced() const { return split() || o2(); }   // operands converted into a workspace first
  bool operator==(const Scheme& o) const { return prec == o.prec && fmt == o.fmt && ns == o.ns; }
};

constexpr int kO2DefaultModuli = 11;

bool make_scheme(int prec, int n_slices, Scheme* out) {
  Scheme sc;
  sc.prec = prec;
  if (prec == QTX_FP64 || prec == QTX_FP32) { *out = sc; return true; }
  if (prec == QTX_INT8_OZAKI2) {
    sc.ns = n_slices > 0 ? n_slices : kO2DefaultModuli;
    O2Params P;
    if (!o2_params(sc.ns, 1024, &P)) return false;   // every block size up to 1024
    *out = sc;
    return true;
  }
  if (prec != QTX_BF16_SPLIT && prec != QTX_FP16_SPLIT) return false;
  sc.fmt = (prec == QTX_BF16_SPLIT) ? 1 : 0;
  sc.ns = n_slices > 0 ? n_slices : 2;
  if (!split_supported(sc.fmt, sc.ns)) return false;
  *out = sc;
  return true;
}

void problem_schemes(const qtx_rgf_problem& p, Scheme* r, Scheme* l) {
  make_scheme(p.prec, p.n_slices, r);
  if (p.prec_lesser >= 0) make_scheme(p.prec_lesser, p.n_slices_lesser, l);
  else *l = *r;
}

// Converted-operand bytes (digits or residues, then row exponents) of a rows x cols
// operand, per batch entry.
size_t operand_digit_bytes(int rows, int cols, const Scheme& sc) {
  if (sc.split()) return (size_t)split_digit_stride(rows, cols, sc.ns) * sizeof(uint16_t);
  if (sc.o2()) return (size_t)o2_res_stride(rows, cols, sc.ns);
  return 0;
}
size_t operand_bytes(int rows, int cols, const Scheme& sc, int batch) {
  if (!sc.sliced()) return 0;
  return align_up(operand_digit_bytes(rows, cols, sc) * batch) +
         align_up((size_t)split_exp_stride(rows, cols) * sizeof(int32_t) * batch);
}

// The scheme of the two whose converted operands need more room.
Scheme larger_split(const Scheme& a, const Scheme& b) {
  return operand_bytes(64, 64, b, 1) > operand_bytes(64, 64, a, 1) ? b : a;
}

// Converted-operand slots: 0 and 1 take a product's A and B by default; a batch also
// has kKeepSlots more, where an operand converted for one product is kept for a later
// product of the same scheme that uses it on the same side.
constexpr int kKeepSlots = 4;
struct SplitBufs {
  void* S[2 + kKeepSlots] = {};
  int32_t* E[2 + kKeepSlots] = {};
};

// Which slots a product converts its operands into, and whether an operand is already
// there (then it is not converted again).  Ignored by the unsliced schemes.
struct ConvUse {
  int a = 0, b = 1;
  bool have_a = false, have_b = false;
  bool conj_b = false;   // INT8 only: op(B) = X^H and slot b holds X converted as a left operand
};

size_t split_pair_bytes(int b, const Scheme& sc, int batch, int slots = 2) {
  return slots * operand_bytes(b, b, sc, batch);
}

SplitBufs carve_split(char*& w, int b, const Scheme& sc, int batch, int slots = 2) {
  SplitBufs sb;
  if (!sc.sliced()) return sb;
  for (int q = 0; q < slots; ++q) {
    sb.S[q] = w; w += align_up(operand_digit_bytes(b, b, sc) * batch);
    sb.E[q] = (int32_t*)w; w += align_up((size_t)split_exp_stride(b, b) * sizeof(int32_t) * batch);
  }
  return sb;
}

// Batch class of the autotuner: ceil(log2(batch)), 0 .. 9 (512 and more share one).
int batch_class(int batch) {
  int c = 0;
  while (c < 9 && (1 << c) < batch) ++c;
  return c;
}

// Tile variant for an INT8 product with p moduli: the forced one, else the tuned
// record of the shape and p at the nearest batch class, else a default from the shape: 64 x 64 tiles
// three per CU (variant 4) for long contractions with enough tiles to fill the
// chip three times over, else 64 x 64 tiles two per CU (variant 1), which wins
// for short contractions and small batches (measured on MI355X over b = 128 .. 512
// and batch 1 .. 256).
int o2_variant_for(qtx_rgf_ctx ctx, const GemmDesc& d, int p) {
  if (ctx->o2_force >= 0) return ctx->o2_force;
  const int bc = batch_class(d.batch);
  int best = -1, dist = 1 << 30;
  for (int c = 0; c <= 9; ++c) {
    auto it = ctx->tune.find(TuneKey(d.M, d.N, d.K, c, p));
    if (it != ctx->tune.end() && std::abs(c - bc) < dist) { dist = std::abs(c - bc); best = it->second.variant; }
  }
  if (best >= 0) return best;
  const int64_t tiles = (int64_t)((d.M + 63) / 64) * ((d.N + 63) / 64) * d.batch;
  return (d.K >= 256 && tiles >= 512) ? 4 : 1;
}

// Scheme code of the tile records of the FP64 / FP32 / split products.
int tile_code(const Scheme& sc) { return kTileCodeBase + 10 * sc.prec + sc.ns; }

// Output tile of an FP64 / FP32 / split product: the forced one, else the tuned record
// of the shape and scheme at the nearest batch class, else 0 (the kernels' rule from
// the shape).
int tile_for(qtx_rgf_ctx ctx, const GemmDesc& d, const Scheme& sc) {
  if (ctx->tile_force) return ctx->tile_force;
  const int bc = batch_class(d.batch), code = tile_code(sc);
  int best = -1, dist = 1 << 30;
  for (int c = 0; c <= 9; ++c) {
    auto it = ctx->tune.find(TuneKey(d.M, d.N, d.K, c, code));
    if (it != ctx->tune.end() && std::abs(c - bc) < dist) { dist = std::abs(c - bc); best = it->second.variant; }
  }
  return best < 0 ? 0 : (best ? 64 : 32);
}

// One batched complex block product with a precision scheme.  Elementwise (K = 0)
// launches stay FP64.
hipError_t run_product(qtx_rgf_ctx ctx, const GemmDesc& d0, const Scheme& sc, const SplitBufs& sb, hipStream_t s,
                       ConvUse use = ConvUse()) {
  GemmDesc d = d0;
  if (d.K > 0 && !sc.o2() && d.tile == 0) d.tile = tile_for(ctx, d, sc);
  // per-launch timers: the matrix-core kernel (its own operations) and the operand
  // conversion passes (their algorithmic bytes) separately
  // a skew-Hermitian result needs only its elements r <= c (the split scheme
  // computes them all)
  const bool half = d.skew && !sc.split();
  const double mnk = 2.0 * (half ? 0.5 * d.M * (d.M + 1.0) : (double)d.M * d.N) * d.K * d.batch;
  double core_ops = 4.0 * mnk;   // FP64 / FP32: four real products
  if (sc.split()) core_ops = 4.0 * (sc.ns * (sc.ns + 1) / 2) * mnk;
  const bool prof = d.K > 0;
  if (d.K == 0 || sc.prec == QTX_FP64) {
    ProfScope ps(ctx, QTX_KERNEL_GEMM, s, core_ops, prof);
    return launch_zgemm_f64(d, s);
  }
  if (sc.prec == QTX_FP32) {
    ProfScope ps(ctx, QTX_KERNEL_GEMM, s, core_ops, prof);
    return launch_zgemm_f32(d, s);
  }
  O2Params P;
  if (sc.o2() && !o2_params(sc.ns, d.K, &P)) return hipErrorInvalidValue;
  if (sc.o2()) core_ops = 4.0 * P.p * mnk;
  // operand A as rows of op(A) (M x K), operand B as columns of op(B) (N x K)
  const bool shA = (d.sA == 0 && !d.tA), shB = (d.sB == 0 && !d.tB);
  auto stride = [&](int rows) {
    return sc.o2() ? o2_res_stride(rows, d.K, sc.ns) : split_digit_stride(rows, d.K, sc.ns);
  };
  SplitDesc sa;
  sa.tX = d.tA; sa.X = d.A; sa.ld = d.lda; sa.stride = d.sA;
  sa.rows = d.M; sa.cols = d.K;
  sa.trans = (d.opA == OP_C); sa.conj = (d.opA == OP_C);
  sa.S = sb.S[use.a]; sa.E = sb.E[use.a];
  sa.s_stride = stride(d.M);
  sa.e_stride = split_exp_stride(d.M, d.K);
  sa.batch = shA ? 1 : d.batch;
  SplitDesc sbd;
  sbd.tX = d.tB; sbd.X = d.B; sbd.ld = d.ldb; sbd.stride = d.sB;
  sbd.rows = d.N; sbd.cols = d.K;
  sbd.trans = (d.opB == OP_N); sbd.conj = (d.opB == OP_C);
  sbd.S = sb.S[use.b]; sbd.E = sb.E[use.b];
  sbd.s_stride = stride(d.N);
  sbd.e_stride = split_exp_stride(d.N, d.K);
  sbd.batch = shB ? 1 : d.batch;
  if (use.conj_b && (!sc.o2() || !use.have_b || d.opB != OP_C)) return hipErrorInvalidValue;
  SplitGemmDesc g;
  g.d = d;
  g.conj_b = use.conj_b ? 1 : 0;
  g.SA = sa.S; g.sa_stride = shA ? 0 : sa.s_stride;
  g.SB = sbd.S; g.sb_stride = shB ? 0 : sbd.s_stride;
  g.EA = sa.E; g.ea_stride = shA ? 0 : sa.e_stride;
  g.EB = sbd.E; g.eb_stride = shB ? 0 : sbd.e_stride;
  // conversion bytes: read the operand, write digits / residues and exponents
  const double conv_bytes =
      (use.have_a ? 0.0 : (double)sa.batch * ((double)d.M * d.K * 16.0 + (double)operand_digit_bytes(d.M, d.K, sc))) +
      (use.have_b ? 0.0 : (double)sbd.batch * ((double)d.N * d.K * 16.0 + (double)operand_digit_bytes(d.N, d.K, sc)));
  hipError_t e;
  if (!use.have_a || !use.have_b) {
    ProfScope ps(ctx, QTX_KERNEL_CONVERT, s, conv_bytes, prof);
    if (sc.o2()) {
      if (!use.have_a && (e = launch_o2_convert(sa, P, s)) != hipSuccess) return e;
      if (!use.have_b && (e = launch_o2_convert(sbd, P, s)) != hipSuccess) return e;
    } else {
      if (!use.have_a && (e = launch_split(sa, sc.fmt, sc.ns, s)) != hipSuccess) return e;
      if (!use.have_b && (e = launch_split(sbd, sc.fmt, sc.ns, s)) != hipSuccess) return e;
    }
  }
  ProfScope ps(ctx, QTX_KERNEL_GEMM, s, core_ops, prof);
  if (sc.o2()) return launch_zgemm_o2(g, P, s, o2_variant_for(ctx, d, P.p));
  return launch_zgemm_split(g, sc.fmt, sc.ns, s);
}

// ---------------------------------------------------------------- problem validation

// Width of the off-diagonal outputs: 64 (complex128) or an FPX width.
int out_fpx_bits(const qtx_rgf_problem& p) { return (p.out_bits == 0 || p.out_bits == 64) ? 64 : p.out_bits; }

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
  // BT Sigma^< / Sigma^> come as their upper blocks only: the lower blocks of a
  // skew-Hermitian matrix are -(upper)^H and are never read.
  if (p->SL_l || p->SG_l) return QTX_ERR_UNSUPPORTED;
  if (p->SG_u && !(p->flags & QTX_WANT_GREATER)) return QTX_ERR_ARG;
  Scheme sc;
  if (!make_scheme(p->prec, p->n_slices, &sc)) return QTX_ERR_UNSUPPORTED;
  if (p->prec_lesser >= 0 && !make_scheme(p->prec_lesser, p->n_slices_lesser, &sc)) return QTX_ERR_UNSUPPORTED;
  if (p->flags & ~(uint32_t)(QTX_S_IDENTITY | QTX_SIGMA_DIAG | QTX_WANT_GREATER | QTX_SPLIT_CHAIN)) return QTX_ERR_ARG;
  if (p->out_bits != 0 && p->out_bits != 64 && !fpx_supported(p->out_bits)) return QTX_ERR_ARG;
  // FPX off-diagonal outputs are encoded per backward step; the bottom halves of split
  // energies fix up their lower blocks after the whole solve, so the two do not combine
  if (out_fpx_bits(*p) < 64 && (p->flags & QTX_SPLIT_CHAIN) && p->n_b >= 3) return QTX_ERR_UNSUPPORTED;
  if (p->partitions < 0 || p->partitions > 64) return QTX_ERR_ARG;
  if (p->partitions > 1) {
    if ((p->flags & QTX_SPLIT_CHAIN) || p->n_b < 2 * p->partitions - 1) return QTX_ERR_ARG;
    if (out_fpx_bits(*p) < 64) return QTX_ERR_UNSUPPORTED;
  }
  return QTX_OK;
}

// ---------------------------------------------------------------- batches

constexpr int kTemps = 6;

// Arrays an operand can come from.
enum Arr {
  A_HD, A_HU, A_HL, A_SD, A_SU, A_SL,               // per problem, [n_b] / [n_b-1] blocks
  A_SRD, A_SLD, A_SGD, A_GRD, A_GLD, A_GGD,         // per energy, [n_b] blocks
  A_SRU, A_SRL, A_GRU, A_GRL, A_GLU, A_GGU,         // per energy, [n_b-1] blocks
  A_SLU, A_SGU,
  A_RBL, A_RBG                                      // bottom halves: -(SL_u)^H, -(SG_u)^H (context buffer)
};

// One chain of the recurrences.  An energy is one entry, or two with QTX_SPLIT_CHAIN:
// the top half (blocks 0 .. c-1, forward steps 0 .. c-1, backward from block c) and the
// bottom half, which runs the same recurrences on the block-reversed system
// (logical block j = physical n_b - 1 - j) from block n_b - 1 up to the separator c,
// where it adds the top half's coupling terms before inverting (its last x is G_cc).
struct Entry {
  const qtx_rgf_problem* p;
  int e;
  int nf = 0;         // forward steps
  int nbk = 0;        // backward steps + 1 (backward from logical block nbk - 1)
  bool rev = false;   // bottom half: logical block j is physical block n_b - 1 - j
  int c = 0;          // separator block of a split energy
  int part = -1;      // top half: index of its bottom half in the batch
  int64_t rbt_l = -1, rbt_g = -1;   // bottom half with a BT Sigma^< / Sigma^>: element offsets
                                    // of its -(SL_u)^H / -(SG_u)^H copies (blocks c .. n_b - 2)
  int q = -1;         // partitioned solve: partition index (logical block j = physical off + j;
  int off = 0;        // nf interior blocks; upper separator off - 1, lower separator off + nf)
};

// The common properties of a batch's entries.
struct BatchKey {
  int b = 0;
  Scheme r, l;
  bool s_id = true, greater = false, coupled = false;
  bool l_bt = false, g_bt = false;   // Sigma^< / Sigma^> with off-diagonal blocks
  bool sdiag = false;                // the diagonal self-energy blocks come as vectors
  int obits = 64;                    // width of the off-diagonal outputs (64 or FPX)
  int parts = 1;                     // partitioned solve: partitions per energy
  int nb = 0;                        // and the chain length (one partition layout per batch)
  bool operator==(const BatchKey& o) const {
    return b == o.b && r == o.r && l == o.l && s_id == o.s_id && greater == o.greater && coupled == o.coupled &&
           l_bt == o.l_bt && g_bt == o.g_bt && sdiag == o.sdiag && obits == o.obits && parts == o.parts && nb == o.nb;
  }
};

BatchKey key_of(const qtx_rgf_problem& p) {
  BatchKey k;
  k.b = p.b;
  problem_schemes(p, &k.r, &k.l);
  k.s_id = (p.flags & QTX_S_IDENTITY) != 0;
  k.greater = (p.flags & QTX_WANT_GREATER) != 0;
  k.coupled = !k.s_id || p.SR_u || p.SR_l;
  k.l_bt = p.n_b > 1 && p.SL_u != nullptr;
  k.g_bt = k.greater && p.n_b > 1 && p.SG_u != nullptr;
  k.sdiag = (p.flags & QTX_SIGMA_DIAG) != 0;
  k.obits = out_fpx_bits(p);
  if (p.partitions > 1) { k.parts = p.partitions; k.nb = p.n_b; }
  return k;
}

// Off-diagonal output blocks staged in FP64 before their FPX encoding: G^R_{i,i+1},
// G^R_{i+1,i}, G^<_{i,i+1}, G^>_{i,i+1}.
constexpr int kOutTemps = 4;

// Per-entry blocks of a partitioned batch (see PartWs).
constexpr int kPartTemps = 8;
int part_blocks(const BatchKey& k) {
  if (k.parts <= 1) return 0;
  const int nr = k.greater ? 2 : 1;
  return 4 + 3 * nr + 1 + nr + kPartTemps;
}

// Workspace of a batch of Z entries (excluding its pointer tables).
size_t batch_ws_bytes(const BatchKey& k, int Z) {
  const size_t blk = align_up((size_t)Z * k.b * k.b * sizeof(double2));
  return blk * (1 + kTemps + 2 + (k.obits < 64 ? kOutTemps : 0) + part_blocks(k)) + align_up(gje_work_bytes(k.b, Z)) +
         align_up((size_t)Z * sizeof(int32_t)) +
         split_pair_bytes(k.b, larger_split(k.r, k.l), Z, 2 + kKeepSlots) + split_pair_bytes(k.b, k.l, Z) + 1024;
}

size_t per_entry_bytes(const BatchKey& k) { return batch_ws_bytes(k, 1); }

struct Batch {
  BatchKey key;
  std::vector<Entry> ent;     // sorted by (nf, nbk, rev), descending
  int max_nf = 0, max_nbk = 0;
  bool split = false;         // holds split energies
  int lane = 0;               // stream lane (batches of one lane run in order)
  size_t ws_off = 0;          // workspace region (bytes from the workspace start)
  size_t tab_off = 0;         // table area (bytes from the table block start)
};

// A pointer table request: array, indexing mode, step, block offset.
// mode 0: forward step i -> logical block i + delta (active prefix of step i)
// mode 1: backward step k -> logical block nbk - 2 - k + delta (active prefix of step k)
// mode 2: logical block delta of every entry, always a table (status handling)
// mode 3: bottom halves that reach their separator c at forward step `step` ->
//         physical block c - 1 + delta (the top half's last forward block)
// mode 4: every physical upper block c .. n_b - 2 of every bottom half
// mode 8: partitioned solve, logical block nf + delta of every entry (the lower separator)
// mode 9: partitioned solve, logical block -1 + delta of every entry (the upper separator)
struct TabKey {
  int arr, mode, step, delta;
  bool operator<(const TabKey& o) const {
    return std::tie(arr, mode, step, delta) < std::tie(o.arr, o.mode, o.step, o.delta);
  }
};

struct TabVal {
  const double2* base = nullptr;   // affine: base + z * stride
  int64_t stride = 0;
  int64_t off = -1;                // table: byte offset in the batch's table area
};

// Operand handle: affine (p, stride) or a device table.
struct Mat {
  const double2* p = nullptr;
  int64_t stride = 0;
  const double2* const* tab = nullptr;
};

// Per-entry data at the head of a batch's table area.
struct EntryData {
  size_t en, ust, cnt_d, cnt_u, part, end;
};
EntryData entry_data_layout(int Z) {
  EntryData d;
  d.en = 0;
  d.ust = align_up(d.en + (size_t)Z * sizeof(double));
  d.cnt_d = align_up(d.ust + (size_t)Z * sizeof(void*));
  d.cnt_u = align_up(d.cnt_d + (size_t)Z * sizeof(int64_t));
  d.part = align_up(d.cnt_u + (size_t)Z * sizeof(int64_t));
  d.end = align_up(d.part + (size_t)Z * sizeof(int32_t));
  return d;
}

// State of one batch run: the dry pass plans tables, the launch pass uses them.
struct Run {
  qtx_rgf_ctx ctx;
  hipStream_t s = nullptr;
  hipStream_t side = nullptr;          // launch pass: stream for products that overlap the inversion
  hipEvent_t side_fork = nullptr, side_join = nullptr;
  Batch* B = nullptr;
  bool dry = true;
  bool late = false;   // a pointer table was first requested after the dry pass (an internal error)
  std::map<TabKey, TabVal> tabs;
  std::vector<char> host;          // this batch's table area (per-entry data + tables)
  char* dev = nullptr;             // its device copy (launch pass)
  int64_t bb = 0;

  int active_fwd(int i) const {
    int n = 0;
    while (n < (int)B->ent.size() && B->ent[n].nf > i) ++n;
    return n;
  }
  int active_bwd(int k) const {
    int n = 0;
    while (n < (int)B->ent.size() && B->ent[n].nbk - 2 >= k) ++n;
    return n;
  }
  // Bottom halves whose last forward step is i: entries [*lo, *hi) (a contiguous run,
  // by the sort order).
  void merge_range(int i, int* lo, int* hi) const {
    *lo = *hi = 0;
    const int n = (int)B->ent.size();
    int z = 0;
    while (z < n && !(B->ent[z].rev && B->ent[z].nf == i + 1)) ++z;
    *lo = z;
    while (z < n && B->ent[z].rev && B->ent[z].nf == i + 1) ++z;
    *hi = z;
  }

  // Base pointer of array a for entry z at logical block j (nullptr for an absent
  // array).  For a bottom half the logical system is the block-reversed one: its
  // diagonal block j is physical n_b - 1 - j and its upper (lower) coupling j is the
  // physical lower (upper) block n_b - 2 - j.  Its G^</G^> upper blocks are written
  // to the physical upper slot n_b - 2 - j as the logical block and transformed
  // afterwards (mode 4).
  const double2* ptr(int a, int z, int j, bool physical = false) const {
    const qtx_rgf_problem& p = *B->ent[z].p;
    const int64_t e = B->ent[z].e;
    if (B->ent[z].rev && !physical) {
      static const int swap[][2] = {{A_HU, A_HL}, {A_SU, A_SL}, {A_SRU, A_SRL}, {A_GRU, A_GRL}};
      bool diag = true;
      for (const auto& sw : swap) {
        if (a == sw[0]) { a = sw[1]; diag = false; break; }
        if (a == sw[1]) { a = sw[0]; diag = false; break; }
      }
      // the reversed system's upper Sigma^<> blocks are the physical lower ones, -(upper)^H
      if (a == A_SLU) a = A_RBL;
      if (a == A_SGU) a = A_RBG;
      if (a == A_GLU || a == A_GGU || a == A_RBL || a == A_RBG) diag = false;
      j = diag ? p.n_b - 1 - j : p.n_b - 2 - j;
    }
    const int64_t nd = p.n_b, nu = (int64_t)p.n_b - 1;
    if (B->ent[z].q >= 0) {
      // partitioned solve: logical block j of the entry is physical off + j; blocks past
      // either end of the chain do not exist
      j += B->ent[z].off;
      const bool upper = a == A_HU || a == A_HL || a == A_SU || a == A_SL || a == A_SRU || a == A_SRL ||
                         a == A_GRU || a == A_GRL || a == A_GLU || a == A_GGU || a == A_SLU || a == A_SGU;
      if (j < 0 || j >= (upper ? nu : nd)) return nullptr;
    }
    const void* base = nullptr;
    int64_t idx = 0;
    switch (a) {
      case A_HD: base = p.H_d; idx = j; break;
      case A_HU: base = p.H_u; idx = j; break;
      case A_HL: base = p.H_l; idx = j; break;
      case A_SD: base = p.S_d; idx = j; break;
      case A_SU: base = p.S_u; idx = j; break;
      case A_SL: base = p.S_l; idx = j; break;
      case A_SRD: base = p.SR_d; idx = e * nd + j; break;
      case A_SLD: base = p.SL_d; idx = e * nd + j; break;
      case A_SGD: base = p.SG_d; idx = e * nd + j; break;
      case A_GRD: base = p.GR_d; idx = e * nd + j; break;
      case A_GLD: base = p.GL_d; idx = e * nd + j; break;
      case A_GGD: base = p.GG_d; idx = e * nd + j; break;
      case A_SRU: base = p.SR_u; idx = e * nu + j; break;
      case A_SRL: base = p.SR_l; idx = e * nu + j; break;
      case A_GRU: base = p.GR_u; idx = e * nu + j; break;
      case A_GRL: base = p.GR_l; idx = e * nu + j; break;
      case A_GLU: base = p.GL_u; idx = e * nu + j; break;
      case A_GGU: base = p.GG_u; idx = e * nu + j; break;
      case A_SLU: base = p.SL_u; idx = e * nu + j; break;
      case A_SGU: base = p.SG_u; idx = e * nu + j; break;
      case A_RBL:
      case A_RBG: {
        const int64_t o = a == A_RBL ? B->ent[z].rbt_l : B->ent[z].rbt_g;
        if (o < 0 || !ctx->rbt) return nullptr;
        return (const double2*)ctx->rbt + o + (int64_t)(j - B->ent[z].c) * bb;
      }
    }
    if (!base) return nullptr;
    // diagonal self-energy blocks given as vectors: b elements per block
    if (B->key.sdiag && (a == A_SRD || a == A_SLD || a == A_SGD)) return (const double2*)base + idx * B->key.b;
    // FPX off-diagonal outputs: bb * obits / 4 bytes per block (a byte address)
    if (is_fpx(a)) return (const double2*)((const char*)base + idx * bb * (B->key.obits / 4));
    return (const double2*)base + idx * bb;
  }

  // Arrays of this batch stored as FPX bytes (always addressed through tables).
  bool is_fpx(int a) const {
    return B->key.obits < 64 && (a == A_GRU || a == A_GRL || a == A_GLU || a == A_GGU);
  }

  Mat get(int a, int mode, int step, int delta) {
    const TabKey key{a, mode, step, delta};
    auto it = tabs.find(key);
    if (it == tabs.end()) {
      std::vector<const double2*> v;
      if (mode == 3) {
        int lo, hi;
        merge_range(step, &lo, &hi);
        for (int z = lo; z < hi; ++z) v.push_back(ptr(a, z, B->ent[z].c - 1 + delta, true));
      } else if (mode == 4) {
        for (int z = 0; z < (int)B->ent.size(); ++z)
          if (B->ent[z].rev)
            for (int j = B->ent[z].c; j <= B->ent[z].p->n_b - 2; ++j) v.push_back(ptr(a, z, j, true));
      } else if (mode == 8 || mode == 9) {
        for (int z = 0; z < (int)B->ent.size(); ++z)
          v.push_back(ptr(a, z, (mode == 8 ? B->ent[z].nf : -1) + delta));
      } else {
        const int Z = mode == 0 ? active_fwd(step) : (mode == 1 ? active_bwd(step) : (int)B->ent.size());
        for (int z = 0; z < Z; ++z) {
          const int j = mode == 0 ? step + delta : (mode == 1 ? B->ent[z].nbk - 2 - step + delta : delta);
          v.push_back(ptr(a, z, j));
        }
      }
      const int Z = (int)v.size();
      bool any_null = false;
      for (int z = 0; z < Z; ++z) any_null |= (v[z] == nullptr);
      TabVal tv;
      bool affine = mode != 2 && mode != 4 && Z > 0 && !any_null && !is_fpx(a);
      int64_t stride = 0;
      if (affine && Z > 1) {
        stride = v[1] - v[0];
        for (int z = 2; z < Z && affine; ++z) affine = (v[z] - v[z - 1] == stride);
      }
      // an absent array: no pointer (a partitioned batch has entries without some blocks,
      // and its products run over entry ranges)
      bool all_null = true;
      for (int z = 0; z < Z; ++z) all_null &= (v[z] == nullptr);
      const bool absent = B->key.parts > 1 ? all_null : (mode != 2 && v[0] == nullptr);
      if (Z == 0 || absent) {
        tv.base = nullptr;
      } else if (affine) {
        tv.base = v[0];
        tv.stride = stride;
      } else if (!dry) {
        // A pointer table first asked for after the dry pass has no uploaded copy: the
        // launch pass must request exactly the tables of the dry pass.  Refuse (null
        // operand; products and the entry launchers return an error) rather than
        // hand a kernel an address past the uploaded tables.
        late = true;
        return Mat{};
      } else {
        const size_t off = align_up(host.size());
        host.resize(off + (size_t)Z * sizeof(void*));
        std::memcpy(host.data() + off, v.data(), (size_t)Z * sizeof(void*));
        tv.off = (int64_t)off;
      }
      it = tabs.emplace(key, tv).first;
    }
    const TabVal& tv = it->second;
    Mat m;
    if (tv.off >= 0) {
      // a placeholder in the dry pass (non-null so operand presence is preserved)
      m.tab = dry ? (const double2* const*)(uintptr_t)1 : (const double2* const*)(dev + tv.off);
    } else {
      m.p = tv.base;
      m.stride = tv.stride;
    }
    return m;
  }
};

inline Addend addend_of(const Mat& m, double2 coef, int op = OP_N, int by_batch = 0, int diag = 0) {
  Addend a;
  a.X = m.p; a.stride = m.stride; a.tX = m.tab; a.coef = coef; a.op = op; a.scale_by_batch = by_batch;
  a.diag = diag;
  return a;
}

struct Gemm {
  Run* run;
  int b;
  const double* energies;   // device, per entry
  Scheme sc;
  SplitBufs sb;
  bool on_side = false;     // launch on the run's side stream

  // C = alpha * op(A) op(B) + addends (+ diag * E_z I), over the first Z entries;
  // skew: the result is skew-Hermitian (only r <= c computed, mirrored)
  hipError_t go(int Z, int opA, Mat A, int opB, Mat B, Mat C, double2 alpha, std::initializer_list<Addend> adds,
                double2 diag = cmk(0, 0), int K = -1, bool skew = false, ConvUse use = ConvUse()) const {
    if (run->dry || Z <= 0) return hipSuccess;
    if (run->late) return hipErrorInvalidValue;
    GemmDesc d;
    d.M = b; d.N = b; d.K = (K < 0) ? b : K;
    d.opA = opA; d.opB = opB;
    d.A = A.p; d.sA = A.stride; d.tA = A.tab; d.lda = b;
    d.B = B.p; d.sB = B.stride; d.tB = B.tab; d.ldb = b;
    d.C = (double2*)C.p; d.sC = C.stride; d.tC = (double2* const*)C.tab; d.ldc = b;
    d.alpha = alpha;
    int q = 0;
    for (const Addend& a : adds) {
      if (q < kMaxAddends && (a.X || a.tX)) {
        d.add[q] = a;
        if (d.add[q].ld == 0) d.add[q].ld = b;   // blocks are b x b
        ++q;
      }
    }
    d.diag = diag;
    d.diag_by_batch = 1;
    d.bscal = energies;
    d.batch = Z;
    d.skew = skew ? 1 : 0;
    return run_product(run->ctx, d, sc, sb, on_side ? run->side : run->s, use);
  }
};

// Device layout of a batch's workspace.
struct BatchWs {
  double2* X = nullptr;
  double2* Tm[kTemps] = {};
  double2* Uw = nullptr;
  double2* Lw = nullptr;
  double2* Ot[kOutTemps] = {};   // FPX outputs: the FP64 off-diagonal blocks of a backward step
  // Partitioned solve, per entry z (partition q of energy e, z = q n_e + e): the separator
  // system's blocks -- Ahd: M-hat of the lower separator e_q with the terms from above it
  // (M_dd, the eliminated partition q), AhU: the terms of e_(q-1) from below it (the
  // eliminated partition q); Ahu / Ahl: the couplings M-hat_{e_(q-1), e_q} /
  // M-hat_{e_q, e_(q-1)}; Bhd, BhU, Bhu the same for each right-hand side; XL / XLl: the
  // left-connected x, x^< of the upper separator e_(q-1) (everything above it
  // eliminated), from which partition q's one-chain forward recurrence restarts; Pt:
  // temporaries.
  double2 *Ahd = nullptr, *AhU = nullptr, *Ahu = nullptr, *Ahl = nullptr, *XL = nullptr;
  double2* Bhd[2] = {};
  double2* BhU[2] = {};
  double2* Bhu[2] = {};
  double2* XLl[2] = {};
  double2* Pt[kPartTemps] = {};
  GjeWork gw;
  int32_t* st = nullptr;
  SplitBufs sb;
  SplitBufs sb_side;   // converted operands of the products on the side stream
  // per-entry data (inside the table area)
  const double* en = nullptr;
  int32_t* const* ust = nullptr;
  const int64_t* cnt_d = nullptr;
  const int64_t* cnt_u = nullptr;
  const int32_t* part = nullptr;
};

BatchWs carve_batch(char* w, const BatchKey& k, int Z) {
  BatchWs L;
  const size_t blk = align_up((size_t)Z * k.b * k.b * sizeof(double2));
  L.X = (double2*)w; w += blk;
  for (int t = 0; t < kTemps; ++t) { L.Tm[t] = (double2*)w; w += blk; }
  L.Uw = (double2*)w; w += blk;
  L.Lw = (double2*)w; w += blk;
  if (k.obits < 64)
    for (int t = 0; t < kOutTemps; ++t) { L.Ot[t] = (double2*)w; w += blk; }
  if (k.parts > 1) {
    const int nr = k.greater ? 2 : 1;
    auto take = [&]() { double2* p = (double2*)w; w += blk; return p; };
    L.Ahd = take(); L.AhU = take(); L.Ahu = take(); L.Ahl = take(); L.XL = take();
    for (int r = 0; r < nr; ++r) { L.Bhd[r] = take(); L.BhU[r] = take(); L.Bhu[r] = take(); L.XLl[r] = take(); }
    for (int t = 0; t < kPartTemps; ++t) L.Pt[t] = take();
  }
  L.gw = gje_carve(w, k.b, Z); w += align_up(gje_work_bytes(k.b, Z));
  L.st = (int32_t*)w; w += align_up((size_t)Z * sizeof(int32_t));
  L.sb = carve_split(w, k.b, larger_split(k.r, k.l), Z, 2 + kKeepSlots);
  L.sb_side = carve_split(w, k.b, k.l, Z);
  return L;
}

// The step sequence of one batch (the dry pass and the launch pass both run it).
qtx_status run_batch(Run& R, const BatchWs& W) {
  qtx_rgf_ctx ctx = R.ctx;
  Batch& B = *R.B;
  const BatchKey& k = B.key;
  const int b = k.b;
  const int64_t bb = (int64_t)b * b;
  const int Zall = (int)B.ent.size();
  hipStream_t s = R.s;
  const bool dry = R.dry;
  Gemm g{&R, b, W.en, k.r, W.sb};     // retarded chain
  Gemm gl{&R, b, W.en, k.l, W.sb};    // lesser / greater chain
  Gemm gl_side{&R, b, W.en, k.l, W.sb_side, true};   // lesser chain on the side stream
  const double2 one = cmk(1, 0), mone = cmk(-1, 0), zero = cmk(0, 0);
  auto ws = [&](double2* p) { Mat m; m.p = p; m.stride = bb; return m; };

  if (!dry) QTX_TRY(launch_fill_i32(W.st, 0, Zall, s));

  // Right-hand sides: Sigma^< (and Sigma^>), with their upper blocks when BT.
  struct Rhs { int S, SU, Gd, Gu; };
  std::vector<Rhs> rhs{{A_SLD, k.l_bt ? A_SLU : -1, A_GLD, A_GLU}};
  if (k.greater) rhs.push_back({A_SGD, k.g_bt ? A_SGU : -1, A_GGD, A_GGU});

  // Bottom halves with a BT right-hand side read it block-reversed: their upper blocks
  // are the physical lower ones, -(SL_u)^H, copied once per solve (mode 4 lists the
  // physical blocks c .. n_b - 2 of every bottom half).
  if (B.split) {
    int nfix = 0;
    for (const Entry& en : B.ent)
      if (en.rev) nfix += en.p->n_b - 1 - en.c;
    for (const Rhs& r : rhs) {
      if (r.SU < 0) continue;
      const Mat src = R.get(r.SU, 4, 0, 0);
      const Mat dst = R.get(r.SU == A_SLU ? A_RBL : A_RBG, 4, 0, 0);
      if (!dry && nfix > 0) QTX_TRY(launch_neg_ctrans_copy(src.tab, (double2* const*)dst.tab, b, nfix, s));
    }
  }

  // The coupling operands: U_i = E S_{i,i+1} - H_{i,i+1} - Sigma^R_{i,i+1}(E) and the
  // same for L_i.  With S = I and no Sigma^R coupling they are -H_u, -H_l: the
  // operand is H with sign -1.  Otherwise they are assembled per entry (sign +1).
  Mat U, L;
  double sU = -1.0, sL = -1.0;
  auto coupling = [&](int Z, int mode, int step, int delta) -> hipError_t {
    if (!k.coupled) {
      U = R.get(A_HU, mode, step, delta); sU = -1.0;
      L = R.get(A_HL, mode, step, delta); sL = -1.0;
      return hipSuccess;
    }
    const Mat SU = k.s_id ? Mat{} : R.get(A_SU, mode, step, delta);
    const Mat SL = k.s_id ? Mat{} : R.get(A_SL, mode, step, delta);
    hipError_t e = g.go(Z, OP_N, Mat{}, OP_N, Mat{}, ws(W.Uw), zero,
                        {addend_of(SU, one, OP_N, 1), addend_of(R.get(A_HU, mode, step, delta), mone),
                         addend_of(R.get(A_SRU, mode, step, delta), mone)}, zero, 0);
    if (e != hipSuccess) return e;
    e = g.go(Z, OP_N, Mat{}, OP_N, Mat{}, ws(W.Lw), zero,
             {addend_of(SL, one, OP_N, 1), addend_of(R.get(A_HL, mode, step, delta), mone),
              addend_of(R.get(A_SRL, mode, step, delta), mone)}, zero, 0);
    U = ws(W.Uw); sU = 1.0;
    L = ws(W.Lw); sL = 1.0;
    return e;
  };

  // ------------------------------------------------------------ forward
  // Operand at entry z0 of a per-entry workspace array.
  auto ws_at = [&](double2* p, int z0) { Mat m; m.p = p ? p + (int64_t)z0 * bb : nullptr; m.stride = bb; return m; };
  for (int i = 0; i < B.max_nf; ++i) {
    const int Z = R.active_fwd(i);
    // Bottom halves that reach their separator at this step: [mlo, mhi).
    int mlo = 0, mhi = 0;
    if (B.split) R.merge_range(i, &mlo, &mhi);
    const int Zm = mhi - mlo;
    Gemm gm = g, glm = gl;   // products over the merge range (per-entry energies from mlo)
    if (W.en) { gm.energies = W.en + mlo; glm.energies = W.en + mlo; }
    // A_i = E S_ii - H_ii - Sigma^R_ii(E) as epilogue addends
    const Addend aH = addend_of(R.get(A_HD, 0, i, 0), mone);
    const int sd = k.sdiag ? 1 : 0;   // diagonal self-energy blocks come as vectors
    const Addend aS = addend_of(R.get(A_SRD, 0, i, 0), mone, OP_N, 0, sd);
    const Addend aO = k.s_id ? Addend{} : addend_of(R.get(A_SD, 0, i, 0), one, OP_N, 1);
    const double2 dg = k.s_id ? one : zero;
    if (i == 0) {
      QTX_TRY(g.go(Z, OP_N, Mat{}, OP_N, Mat{}, ws(W.X), zero, {aH, aS, aO}, dg, 0));
    } else {
      QTX_TRY(coupling(Z, 0, i, -1));
      // T' = L' x_{i-1};   X = A_i - sL sU T' U'
      QTX_TRY(g.go(Z, OP_N, L, OP_N, R.get(A_GRD, 0, i, -1), ws(W.Tm[0]), one, {}));
      QTX_TRY(g.go(Z, OP_N, ws(W.Tm[0]), OP_N, U, ws(W.X), cmk(-sL * sU, 0), {aH, aS, aO}, dg));
    }
    const Mat xi = R.get(A_GRD, 0, i, 0);
    // The first lesser recurrence's Y' = L' xl_{i-1} and Q = B_i + Y' L'^H do not
    // need x_i: with a side stream they run there while x_i is inverted (the
    // inversion leaves most matrix cores idle), else before the inversion.  The
    // side stream forks after everything they read is enqueued and joins before Q
    // is used; it owns its own converted-operand buffers.
    const bool side = !dry && R.side != nullptr && !ctx->capturing && Z > 0 && i > 0 && Zm == 0;
    // Q_i = B_i + L xl_{i-1} L^H - BL_{i-1} x_{i-1}^H L^H - L x_{i-1} BU_{i-1}.  With
    // L = sL L' and BL = -BU^H (skew-Hermitian right-hand side) the two cross terms are
    // -sL V + sL V^H with V = T' BU_{i-1}, T' = L' x_{i-1} (still in Tm[0]).
    auto lesser_q = [&](const Gemm& G, const Rhs& r) -> hipError_t {
      const Mat Bi = R.get(r.S, 0, i, 0);
      hipError_t e = G.go(Z, OP_N, L, OP_N, R.get(r.Gd, 0, i, -1), ws(W.Tm[1]), one, {});
      if (e != hipSuccess) return e;
      if (r.SU < 0)
        return G.go(Z, OP_N, ws(W.Tm[1]), OP_C, L, ws(W.Tm[3]), one, {addend_of(Bi, one, OP_N, 0, sd)}, zero, -1, true);
      e = G.go(Z, OP_N, ws(W.Tm[0]), OP_N, R.get(r.SU, 0, i, -1), ws(W.Tm[4]), one, {});
      if (e != hipSuccess) return e;
      return G.go(Z, OP_N, ws(W.Tm[1]), OP_C, L, ws(W.Tm[3]), one,
                  {addend_of(Bi, one, OP_N, 0, sd), addend_of(ws(W.Tm[4]), cmk(-sL, 0)),
                   addend_of(ws(W.Tm[4]), cmk(sL, 0), OP_C)},
                  zero, -1, true);
    };
    if (i > 0) {
      if (side) {
        QTX_TRY(hipEventRecord(R.side_fork, s));
        QTX_TRY(hipStreamWaitEvent(R.side, R.side_fork, 0));
      }
      QTX_TRY(lesser_q(side ? gl_side : gl, rhs[0]));
      if (side) QTX_TRY(hipEventRecord(R.side_join, R.side));
    }
    // Separator of split energies: the bottom half's X = A_c - A_{c,c+1} g_{c+1} A_{c+1,c}
    // and Q = B_c + A_{c,c+1} g<_{c+1} A_{c,c+1}^H get the top half's terms
    // - A_{c,c-1} x_{c-1} A_{c-1,c} and + A_{c,c-1} xl_{c-1} A_{c,c-1}^H (physical
    // couplings of block c - 1; x, xl of the top half), so that its x_c is G_cc and its
    // xl_c is G<_cc.  Greater: the top term goes to Tm[5] and is added to its Q below.
    // With a BT right-hand side the top half's term also has the cross terms -V + V^H,
    // V = A_{c,c-1} x_{c-1} Sigma^<_{c-1,c}.  Temporaries of the merge range: Tm[1], Tm[2]
    // (assembled couplings), Tm[4], Tm[5] (Tm[0] keeps the bottom half's own T' for the
    // cross terms of its later right-hand sides, Tm[3] holds its first Q).
    if (Zm > 0) {
      Mat Um, Lm;
      double sUm = -1.0, sLm = -1.0;
      if (!k.coupled) {
        Um = R.get(A_HU, 3, i, 0);
        Lm = R.get(A_HL, 3, i, 0);
      } else {
        const Mat SUm = k.s_id ? Mat{} : R.get(A_SU, 3, i, 0);
        const Mat SLm = k.s_id ? Mat{} : R.get(A_SL, 3, i, 0);
        Um = ws_at(W.Tm[2], mlo);
        Lm = ws_at(W.Tm[1], mlo);
        QTX_TRY(gm.go(Zm, OP_N, Mat{}, OP_N, Mat{}, Um, zero,
                      {addend_of(SUm, one, OP_N, 1), addend_of(R.get(A_HU, 3, i, 0), mone),
                       addend_of(R.get(A_SRU, 3, i, 0), mone)}, zero, 0));
        QTX_TRY(gm.go(Zm, OP_N, Mat{}, OP_N, Mat{}, Lm, zero,
                      {addend_of(SLm, one, OP_N, 1), addend_of(R.get(A_HL, 3, i, 0), mone),
                       addend_of(R.get(A_SRL, 3, i, 0), mone)}, zero, 0));
        sUm = sLm = 1.0;
      }
      const Mat Xm = ws_at(W.X, mlo), T2 = ws_at(W.Tm[2], mlo), T4 = ws_at(W.Tm[4], mlo),
                T5 = ws_at(W.Tm[5], mlo);
      QTX_TRY(gm.go(Zm, OP_N, Lm, OP_N, R.get(A_GRD, 3, i, 0), T4, one, {}));              // T' = Lm' x_{c-1}
      QTX_TRY(gm.go(Zm, OP_N, T4, OP_N, Um, Xm, cmk(-sLm * sUm, 0), {addend_of(Xm, one)}));
      // V_q = T' Sigma_q,{c-1,c}: V_0 in Tm[2] (Um is dead), V_1 in Tm[5]
      Mat Vq[2];
      for (size_t q = 0; q < rhs.size(); ++q) {
        if (rhs[q].SU < 0) continue;
        Vq[q] = q == 0 ? T2 : T5;
        QTX_TRY(glm.go(Zm, OP_N, T4, OP_N, R.get(rhs[q].SU, 3, i, 0), Vq[q], one, {}));
      }
      const double2 msl = cmk(-sLm, 0), psl = cmk(sLm, 0);
      for (size_t q = 0; q < rhs.size(); ++q) {
        QTX_TRY(glm.go(Zm, OP_N, Lm, OP_N, R.get(rhs[q].Gd, 3, i, 0), T4, one, {}));       // Lm' xl_{c-1}
        const bool bt = rhs[q].SU >= 0;
        if (q == 0) {
          const Mat Qm = ws_at(W.Tm[3], mlo);
          QTX_TRY(glm.go(Zm, OP_N, T4, OP_C, Lm, Qm, one,
                         {addend_of(Qm, one), addend_of(bt ? Vq[0] : Mat{}, msl), addend_of(bt ? Vq[0] : Mat{}, psl, OP_C)},
                         zero, -1, true));
        } else if (!bt) {
          QTX_TRY(glm.go(Zm, OP_N, T4, OP_C, Lm, T5, one, {}, zero, -1, true));
        } else {
          // out of place (V_1 is read transposed), then kept in Tm[5] past the inversion
          QTX_TRY(glm.go(Zm, OP_N, T4, OP_C, Lm, T2, one, {addend_of(T5, msl), addend_of(T5, psl, OP_C)}, zero, -1,
                         true));
          QTX_TRY(glm.go(Zm, OP_N, Mat{}, OP_N, Mat{}, T5, zero, {addend_of(T2, one)}, zero, 0));
        }
      }
    }
    if (!dry && Z > 0) {
      ProfScope ps(ctx, QTX_KERNEL_INV, s, 8.0 * (double)b * b * b * Z, true);
      QTX_TRY(launch_gje_invert(b, W.X, bb, (double2*)xi.p, xi.stride, Z, W.gw, W.st, s, (double2* const*)xi.tab));
    }
    if (side) QTX_TRY(hipStreamWaitEvent(s, R.side_join, 0));
    // x_i is converted once (slot 2) as the left operand of Z = x_i Q for every right-hand
    // side; with the INT8 scheme the same residues, imaginary part negated, are the right
    // operand x_i^H of x^<_i = Z x_i^H.
    ConvUse xA, xH;
    xA.a = 2;
    if (k.l.o2()) { xH.b = 2; xH.have_b = true; xH.conj_b = true; }
    for (size_t q = 0; q < rhs.size(); ++q) {
      const Rhs& r = rhs[q];
      const Mat Bi = R.get(r.S, 0, i, 0);
      if (i == 0) {
        if (sd) {
          // a diagonal B_0 is expanded into a dense block first (Tm[3] is free at i = 0)
          QTX_TRY(gl.go(Z, OP_N, Mat{}, OP_N, Mat{}, ws(W.Tm[3]), zero, {addend_of(Bi, one, OP_N, 0, 1)}, zero, 0));
          QTX_TRY(gl.go(Z, OP_N, xi, OP_N, ws(W.Tm[3]), ws(W.Tm[2]), one, {}, zero, -1, false, xA));
        } else {
          QTX_TRY(gl.go(Z, OP_N, xi, OP_N, Bi, ws(W.Tm[2]), one, {}, zero, -1, false, xA));
        }
      } else {
        // Q_i (done above for the first recurrence);  Z = x_i Q
        if (q > 0) {
          QTX_TRY(lesser_q(gl, r));
          if (Zm > 0) {
            const Mat Qm = ws_at(W.Tm[3], mlo);
            QTX_TRY(glm.go(Zm, OP_N, Mat{}, OP_N, Mat{}, Qm, zero,
                           {addend_of(Qm, one), addend_of(ws_at(W.Tm[5], mlo), one)}, zero, 0));
          }
        }
        QTX_TRY(gl.go(Z, OP_N, xi, OP_N, ws(W.Tm[3]), ws(W.Tm[2]), one, {}, zero, -1, false, xA));
      }
      xA.have_a = true;
      // xl_i = Z x_i^H (skew-Hermitian)
      QTX_TRY(gl.go(Z, OP_N, ws(W.Tm[2]), OP_C, xi, R.get(r.Gd, 0, i, 0), one, {}, zero, -1, true, xH));
    }
  }
  // ------------------------------------------------------------ backward (i = n_b - 2 - kk per entry)
  const Mat Pp = ws(W.Tm[0]), Rp = ws(W.Tm[1]), Vp = ws(W.Tm[2]), Wp = ws(W.Tm[3]), Yp = ws(W.Tm[4]),
            Zp = ws(W.Tm[5]);
  for (int kk = 0; kk + 2 <= B.max_nbk; ++kk) {
    const int Z = R.active_bwd(kk);
    if (Z == 0) break;
    QTX_TRY(coupling(Z, 1, kk, 0));
    const Mat xi = R.get(A_GRD, 1, kk, 0);
    const Mat Gn = R.get(A_GRD, 1, kk, 1);
    // With FPX off-diagonal outputs the step's blocks are formed in FP64 temporaries
    // (Ot[0..3]), used from there as operands, and encoded at the end of the step.
    const bool fpx = k.obits < 64;
    const Mat GRu = fpx ? ws(W.Ot[0]) : R.get(A_GRU, 1, kk, 0);
    const Mat GRl = fpx ? ws(W.Ot[1]) : R.get(A_GRL, 1, kk, 0);
    // Converted operands kept for a second use (slots 2..5): P' as A of G_{i,i+1} and V',
    // R' as B of G_{i+1,i} and G_ii, G_{i,i+1} as A of W' and G_ii; across the two chains
    // only when they use the same scheme.  With the INT8 scheme the left-operand residues
    // of G_{i+1,i+1} and P' also serve, imaginary part negated, as the right operands
    // G_{i+1,i+1}^H of G<_{i,i+1} and P'^H of G<_ii.
    const bool same = k.r == k.l;
    ConvUse keepP, keepR, keepG, useP, useRG, gnH, pH;
    keepP.a = 2;
    keepR.a = 5;
    keepR.b = 3;
    if (same) { keepG.a = 4; useP.a = 2; useP.have_a = true; useRG.a = 4; useRG.have_a = true; }
    useRG.b = 3; useRG.have_b = true;
    if (same && k.l.o2()) {
      gnH.b = 5; gnH.have_b = true; gnH.conj_b = true;
      pH.b = 2; pH.have_b = true; pH.conj_b = true;
    }
    QTX_TRY(g.go(Z, OP_N, xi, OP_N, U, Pp, one, {}));                           // P' = x_i U'
    QTX_TRY(g.go(Z, OP_N, L, OP_N, xi, Rp, one, {}));                           // R' = L' x_i
    QTX_TRY(g.go(Z, OP_N, Pp, OP_N, Gn, GRu, cmk(-sU, 0), {}, zero, -1, false, keepP));   // G_{i,i+1}
    QTX_TRY(g.go(Z, OP_N, Gn, OP_N, Rp, GRl, cmk(-sL, 0), {}, zero, -1, false, keepR));   // G_{i+1,i}
    QTX_TRY(gl.go(Z, OP_N, GRu, OP_N, L, Wp, one, {}, zero, -1, false, keepG));          // W' = G_{i,i+1} L'
    // The lesser blocks (x_i is still unchanged here: G_ii overwrites it below).
    //   G<_{i,i+1} = -P G<_{i+1} - xl L^H G_{i+1}^H + x BU G_{i+1}^H
    //   G<_ii = xl + P G<_{i+1} P^H - W xl - xl L^H G_{i,i+1}^H + G_{i,i+1} BL x^H + x BU G_{i,i+1}^H
    // With P = sU P', W = sL W', L = sL L' and the skew-Hermitian xl and BL = -BU^H:
    //   Y = -sL W' xl + x BU G_{i,i+1}^H,  Z = -sL xl L'^H + x BU,
    //   G<_{i,i+1} = Z G_{i+1}^H - sU V',  G<_ii = xl + V' P'^H + Y - Y^H,  V' = P' G<_{i+1}.
    for (size_t q = 0; q < rhs.size(); ++q) {
      const Rhs& r = rhs[q];
      const Mat Gu = fpx ? ws(W.Ot[2 + q]) : R.get(r.Gu, 1, kk, 0);
      const Mat xl = R.get(r.Gd, 1, kk, 0);
      const Mat Gln = R.get(r.Gd, 1, kk, 1);
      const double2 msl = cmk(-sL, 0);
      if (r.SU >= 0) {
        QTX_TRY(gl.go(Z, OP_N, xi, OP_N, R.get(r.SU, 1, kk, 0), Zp, one, {}));   // K' = x_i BU_i
        QTX_TRY(gl.go(Z, OP_N, Zp, OP_C, GRu, Yp, one, {}));                      // K' G_{i,i+1}^H
        QTX_TRY(gl.go(Z, OP_N, Wp, OP_N, xl, Yp, msl, {addend_of(Yp, one)}));     // Y
        QTX_TRY(gl.go(Z, OP_N, xl, OP_C, L, Zp, msl, {addend_of(Zp, one)}));      // Z
      } else {
        QTX_TRY(gl.go(Z, OP_N, Wp, OP_N, xl, Yp, msl, {}));                       // Y = -sL W' xl_i
        QTX_TRY(gl.go(Z, OP_N, xl, OP_C, L, Zp, msl, {}));                        // Z = -sL xl_i L'^H
      }
      QTX_TRY(gl.go(Z, OP_N, Pp, OP_N, Gln, Vp, one, {}, zero, -1, false, useP));   // V' = P' G<_{i+1}
      QTX_TRY(gl.go(Z, OP_N, Zp, OP_C, Gn, Gu, one, {addend_of(Vp, cmk(-sU, 0))}, zero, -1, false, gnH));
      QTX_TRY(gl.go(Z, OP_N, Vp, OP_C, Pp, xl, one,                               // G<_ii (in place)
                    {addend_of(xl, one), addend_of(Yp, one), addend_of(Yp, cmk(-1, 0), OP_C)}, zero, -1, true, pH));
    }
    QTX_TRY(g.go(Z, OP_N, GRu, OP_N, Rp, xi, cmk(-sL, 0), {addend_of(xi, one)}, zero, -1, false, useRG));   // G_ii
    if (fpx) {
      std::vector<std::pair<int, double2*>> enc{{A_GRU, W.Ot[0]}, {A_GRL, W.Ot[1]}};
      for (size_t q = 0; q < rhs.size(); ++q) enc.push_back({rhs[q].Gu, W.Ot[2 + q]});
      for (auto& e : enc) {
        // the table is requested in the dry pass too: tables are laid out and uploaded there
        const Mat dst = R.get(e.first, 1, kk, 0);
        if (!dry)
          QTX_TRY(launch_fpx_encode_entries(k.obits, 2 * bb, (const double*)e.second, 2 * bb, (uint8_t* const*)dst.tab,
                                            Z, s));
      }
    }
  }
  // The bottom halves wrote their logical G^<_{i,i+1} (physical G^<_{j+1,j}) into the
  // physical upper slot j: the upper block is its negated conjugate transpose
  // (G^< is skew-Hermitian).
  if (B.split) {
    int nfix = 0;
    for (const Entry& en : B.ent)
      if (en.rev) nfix += en.p->n_b - 1 - en.c;
    for (const Rhs& r : rhs) {
      const Mat m = R.get(r.Gu, 4, 0, 0);
      if (!dry && nfix > 0) QTX_TRY(launch_neg_ctrans_entries((double2* const*)m.tab, b, nfix, s));
    }
  }
  // ------------------------------------------------------------ status
  // Non-finite values propagate into the first blocks: check those; then every
  // output of a failed entry is NaN-filled and the status is scattered out.  A split
  // energy's status is its top half's, after taking the bottom half's failure (the
  // top half fills and reports the whole energy): a singular pivot in either half
  // first, then non-finite values.
  if (B.split && !dry) QTX_TRY(launch_status_merge(W.st, W.part, Zall, s));
  std::vector<int> first{A_GRD};
  for (const Rhs& r : rhs) first.push_back(r.Gd);
  for (int a : first) {
    const Mat m = R.get(a, 2, 0, 0);
    if (!dry) QTX_TRY(launch_check_finite_entries(m.tab, bb, Zall, W.st, s));
  }
  if (B.split && !dry) QTX_TRY(launch_status_merge(W.st, W.part, Zall, s));
  std::vector<std::pair<int, bool>> outs{{A_GRD, true}, {A_GRU, false}, {A_GRL, false}};
  for (const Rhs& r : rhs) { outs.push_back({r.Gd, true}); outs.push_back({r.Gu, false}); }
  for (auto& o : outs) {
    const Mat m = R.get(o.first, 2, 0, 0);
    if (dry) continue;
    if (R.is_fpx(o.first))
      QTX_TRY(launch_fpx_nan_fill_entries(k.obits, W.cnt_u, (uint8_t* const*)m.tab, Zall, W.st, s));
    else
      QTX_TRY(launch_nan_fill_entries((double2* const*)m.tab, o.second ? W.cnt_d : W.cnt_u, Zall, W.st, s));
  }
  if (!dry) QTX_TRY(launch_scatter_status(W.st, W.ust, Zall, s));
  return R.late ? QTX_ERR_HIP : QTX_OK;
}

// ------------------------------------------------------------------ partitioned solve
// P-way partitioned selected solve of every energy (the spatially parallel selected
// inversion the paper cites): the separators e_0 < .. < e_{P-2} cut the chain into P
// partitions; entry z = q n_e + e is partition q of energy e, with interior blocks
// off .. off + nf - 1 (logical 0 .. nf - 1), upper separator u = off - 1 (q > 0) and
// lower separator d = off + nf (q < P - 1).  Notation: M_jj, U_j = M_{j,j+1} = sU U',
// L_j = M_{j+1,j} = sL L', B a right-hand side (Sigma^<, Sigma^>), BU_j its upper block,
// BL_j = -BU_j^H.
//
// 1. Separator system.  Every interior is eliminated top-down at once (the one-chain
//    forward recurrence x_j, xl_j, started without a previous block), with the fill-ins
//    that couple block j to u, Fr_j = M~_{j,u}, Fc_j = M~_{u,j}, Br_j = B~_{j,u}:
//      Fr_lo = L_u, Fc_lo = U_u, Br_lo = BL_u;
//      Fr_j = -L_{j-1} x_{j-1} Fr_{j-1},  Fc_j = -Fc_{j-1} x_{j-1} U_{j-1},
//      Br_j = -L_{j-1} x_{j-1} Br_{j-1} + L_{j-1} xl_{j-1} Fc_{j-1}^H + (Fc_{j-1} x_{j-1} BU_{j-1})^H.
//    Each eliminated block contributes to its upper separator M^U_uu -= Fc_j x_j Fr_j,
//    B^U_uu += -V + V^H + Fc_j xl_j Fc_j^H (V = Fc_j x_j Br_j); the last one (t) to the
//    lower separator M^_dd = M_dd - L_t x_t U_t, B^_dd = B_dd + L_t xl_t L_t^H - W + W^H
//    (W = L_t x_t BU_t), and to the couplings M^_{d,u} = -L_t x_t Fr_t,
//    M^_{u,d} = -Fc_t x_t U_t, B^_{u,d} = -(B^_{d,u})^H with
//    B^_{d,u} = -L_t x_t Br_t + L_t xl_t Fc_t^H + (Fc_t x_t BU_t)^H.
// 2. The separator chain by the one-chain recurrences on (M^ + M^U, B^ + B^U): G^R,
//    G^<, G^> of the separator blocks (into the outputs); and, per separator c, its
//    left-connected x^L_c, xl^L_c (the same step without the partition below it,
//    M^U and B^U): the functions of the chain's blocks 0 .. e_c alone.
// 3. Every partition q >= 1 runs the one-chain forward recurrence again from x^L, xl^L
//    of its upper separator (which replaces the fill-in chains: those are only used to
//    build the separator system, and carry the cancellation of the isolated interior's
//    1 / eta-sized partial inverses), then every partition runs the one-chain backward
//    recurrence from its lower separator's G (the last partition from its last block);
//    finally the couplings of each upper separator with the first interior block,
//    G_{u,lo} = -x^L U_u G_lo, G_{lo,u} = -G_lo L_u x^L,
//    G^<_{u,lo} = -x^L U_u G^<_lo - xl^L L_u^H G_lo^H + x^L BU_u G_lo^H.
// Products run over entry ranges: the interiors shrink with q, so the active entries of
// a step are a prefix, those with u the entries from n_e on, those with d the entries
// before (P - 1) n_e.
qtx_status run_partition(Run& R, const BatchWs& W) {
  qtx_rgf_ctx ctx = R.ctx;
  const Batch& B = *R.B;
  const BatchKey& k = B.key;
  const int b = k.b;
  const int64_t bb = R.bb;
  const int Zall = (int)B.ent.size();
  const int P = k.parts;
  const int ne = Zall / P;
  const int U0 = ne;               // entries with an upper separator: [ne, Zall)
  const int Zd = Zall - ne;        // entries with a lower separator: [0, Zd)
  hipStream_t s = R.s;
  const bool dry = R.dry;
  // The separator system (phases 1 and 2) is built and solved in FP64 whatever the
  // schemes: its fill-in chains carry the 1 / eta-sized partial inverses of interiors cut
  // off from the contacts, which would scale a sliced scheme's product errors up.  The
  // interiors' one-chain recurrences (phase 3) use the problem's schemes.
  const Gemm g_r{&R, b, W.en, k.r, W.sb}, g_l{&R, b, W.en, k.l, W.sb}, g_64{&R, b, W.en, Scheme{}, W.sb};
  Gemm g = g_64, gl = g_64;
  const double2 one = cmk(1, 0), mone = cmk(-1, 0), zero = cmk(0, 0);
  auto ws_at = [&](double2* p, int z0) { Mat m; m.p = p ? p + (int64_t)z0 * bb : nullptr; m.stride = bb; return m; };
  auto ws = [&](double2* p) { return ws_at(p, 0); };
  auto at = [](Mat m, int z0) {
    if (m.tab) m.tab += z0;
    else if (m.p) m.p += (int64_t)z0 * m.stride;
    return m;
  };
  auto on = [&](const Gemm& G0, int z0) { Gemm G1 = G0; if (W.en) G1.energies = W.en + z0; return G1; };
  const int sd = k.sdiag ? 1 : 0;
  const double2 dg = k.s_id ? one : zero;

  if (!dry) QTX_TRY(launch_fill_i32(W.st, 0, Zall, s));
  struct Rhs { int S, SU, Gd, Gu; };
  std::vector<Rhs> rhs{{A_SLD, k.l_bt ? A_SLU : -1, A_GLD, A_GLU}};
  if (k.greater) rhs.push_back({A_SGD, k.g_bt ? A_SGU : -1, A_GGD, A_GGU});
  const int nr = (int)rhs.size();

  // Couplings of entries [z0, z0 + Z) at (mode, step, delta), as Mats of that range.
  struct Cpl { Mat U, L; double sU = -1.0, sL = -1.0; };
  auto coupling = [&](int z0, int Z, int mode, int step, int delta, Cpl* c) -> hipError_t {
    if (!k.coupled) {
      c->U = at(R.get(A_HU, mode, step, delta), z0); c->sU = -1.0;
      c->L = at(R.get(A_HL, mode, step, delta), z0); c->sL = -1.0;
      return hipSuccess;
    }
    const Mat SU = k.s_id ? Mat{} : at(R.get(A_SU, mode, step, delta), z0);
    const Mat SL = k.s_id ? Mat{} : at(R.get(A_SL, mode, step, delta), z0);
    const Gemm gz = on(g, z0);
    hipError_t e = gz.go(Z, OP_N, Mat{}, OP_N, Mat{}, ws_at(W.Uw, z0), zero,
                         {addend_of(SU, one, OP_N, 1), addend_of(at(R.get(A_HU, mode, step, delta), z0), mone),
                          addend_of(at(R.get(A_SRU, mode, step, delta), z0), mone)}, zero, 0);
    if (e != hipSuccess) return e;
    e = gz.go(Z, OP_N, Mat{}, OP_N, Mat{}, ws_at(W.Lw, z0), zero,
              {addend_of(SL, one, OP_N, 1), addend_of(at(R.get(A_HL, mode, step, delta), z0), mone),
               addend_of(at(R.get(A_SRL, mode, step, delta), z0), mone)}, zero, 0);
    c->U = ws_at(W.Uw, z0); c->sU = 1.0;
    c->L = ws_at(W.Lw, z0); c->sL = 1.0;
    return e;
  };
  // M_jj of the entries' blocks at (mode, step, delta), entries from z0, as epilogue
  // addends (+ E on the diagonal)
  auto diag_terms = [&](int z0, int mode, int step, int delta, Addend* aH, Addend* aS, Addend* aO) {
    *aH = addend_of(at(R.get(A_HD, mode, step, delta), z0), mone);
    *aS = addend_of(at(R.get(A_SRD, mode, step, delta), z0), mone, OP_N, 0, sd);
    *aO = k.s_id ? Addend{} : addend_of(at(R.get(A_SD, mode, step, delta), z0), one, OP_N, 1);
  };

  // One-chain forward step at logical block i of the entries [z0, z0 + Z):
  // X = M_jj - L_{j-1} xp U_{j-1}, x_j = X^-1, xl_j = x_j (B_j + L xlp L^H - V + V^H) x_j^H
  // (V = L xp BU_{j-1}); xp, xlp: the previous block's x, x^<, or for i = 0 with `seed`
  // the upper separator's left-connected ones (XL, XLl), else none.  fwd_x leaves X in
  // W.X and T' = L' xp in Tm[0]; fwd_inv inverts and runs the lesser step.
  struct Step { Cpl c; bool prev = false; };
  auto fwd_x = [&](int z0, int Z, int i, bool seed, Step* st) -> hipError_t {
    Addend aH, aS, aO;
    diag_terms(z0, 0, i, 0, &aH, &aS, &aO);
    const Gemm gz = on(g, z0);
    st->prev = i > 0 || seed;
    if (!st->prev) return gz.go(Z, OP_N, Mat{}, OP_N, Mat{}, ws_at(W.X, z0), zero, {aH, aS, aO}, dg, 0);
    hipError_t e = coupling(z0, Z, 0, i, -1, &st->c);
    if (e != hipSuccess) return e;
    const Mat xp = i > 0 ? at(R.get(A_GRD, 0, i, -1), z0) : ws_at(W.XL, z0);
    e = gz.go(Z, OP_N, st->c.L, OP_N, xp, ws_at(W.Tm[0], z0), one, {});
    if (e != hipSuccess) return e;
    return gz.go(Z, OP_N, ws_at(W.Tm[0], z0), OP_N, st->c.U, ws_at(W.X, z0), cmk(-st->c.sL * st->c.sU, 0),
                 {aH, aS, aO}, dg);
  };
  auto fwd_inv = [&](int z0, int Z, int i, const Step& st) -> hipError_t {
    const Mat xi = at(R.get(A_GRD, 0, i, 0), z0);
    if (!dry && Z > 0) {
      ProfScope ps(ctx, QTX_KERNEL_INV, s, 8.0 * (double)b * b * b * Z, true);
      const hipError_t e = launch_gje_invert(b, W.X + (int64_t)z0 * bb, bb, (double2*)xi.p, xi.stride, Z, W.gw,
                                             W.st + z0, s, (double2* const*)xi.tab);
      if (e != hipSuccess) return e;
    }
    const Gemm glz = on(gl, z0);
    const Mat Q = ws_at(W.Tm[3], z0), T1 = ws_at(W.Tm[1], z0), T4 = ws_at(W.Tm[4], z0), Zq = ws_at(W.Tm[2], z0);
    for (int r = 0; r < nr; ++r) {
      const Addend aB = addend_of(at(R.get(rhs[r].S, 0, i, 0), z0), one, OP_N, 0, sd);
      hipError_t e;
      if (!st.prev) {
        e = glz.go(Z, OP_N, Mat{}, OP_N, Mat{}, Q, zero, {aB}, zero, 0);
      } else {
        const Mat xlp = i > 0 ? at(R.get(rhs[r].Gd, 0, i, -1), z0) : ws_at(W.XLl[r], z0);
        e = glz.go(Z, OP_N, st.c.L, OP_N, xlp, T1, one, {});
        if (e == hipSuccess && rhs[r].SU >= 0) {
          e = glz.go(Z, OP_N, ws_at(W.Tm[0], z0), OP_N, at(R.get(rhs[r].SU, 0, i, -1), z0), T4, one, {});
          if (e == hipSuccess)
            e = glz.go(Z, OP_N, T1, OP_C, st.c.L, Q, one,
                       {aB, addend_of(T4, cmk(-st.c.sL, 0)), addend_of(T4, cmk(st.c.sL, 0), OP_C)});
        } else if (e == hipSuccess) {
          e = glz.go(Z, OP_N, T1, OP_C, st.c.L, Q, one, {aB});
        }
      }
      if (e == hipSuccess) e = glz.go(Z, OP_N, xi, OP_N, Q, Zq, one, {});
      if (e == hipSuccess) e = glz.go(Z, OP_N, Zq, OP_C, xi, at(R.get(rhs[r].Gd, 0, i, 0), z0), one, {});
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };

  // ---------------------------------------------------------- 1. separator system
  // lower-separator blocks start as M_dd, B_dd; the upper-side sums at zero
  {
    Addend aH, aS, aO;
    diag_terms(0, 8, 0, 0, &aH, &aS, &aO);
    QTX_TRY(g.go(Zd, OP_N, Mat{}, OP_N, Mat{}, ws(W.Ahd), zero, {aH, aS, aO}, dg, 0));
    QTX_TRY(g.go(Zd, OP_N, Mat{}, OP_N, Mat{}, ws(W.AhU), zero, {}, zero, 0));
    for (int r = 0; r < nr; ++r) {
      QTX_TRY(gl.go(Zd, OP_N, Mat{}, OP_N, Mat{}, ws(W.Bhd[r]), zero,
                    {addend_of(R.get(rhs[r].S, 8, 0, 0), one, OP_N, 0, sd)}, zero, 0));
      QTX_TRY(gl.go(Zd, OP_N, Mat{}, OP_N, Mat{}, ws(W.BhU[r]), zero, {}, zero, 0));
    }
  }
  // Upper-separator terms of the entries [z0, z0 + Z) (all with u) for their block at
  // logical i: M^U_uu -= C1 Fr, B^U_uu += -V + V^H + Fc xl Fc^H (C1 = Fc x, V = C1 Br).
  // C1 stays in Pt[0].
  auto sep_u_terms = [&](int z0, int Z, int i) -> hipError_t {
    if (Z <= 0) return hipSuccess;
    const Gemm gu = on(g, z0), glu = on(gl, z0);
    const Mat x = at(R.get(A_GRD, 0, i, 0), z0);
    const Mat Fr = at(R.get(A_GRL, 0, i, -1), z0), Fc = at(R.get(A_GRU, 0, i, -1), z0);
    const Mat C1 = ws_at(W.Pt[0], z0), AU = ws_at(W.AhU, z0 - ne);
    hipError_t e = gu.go(Z, OP_N, Fc, OP_N, x, C1, one, {});
    if (e == hipSuccess) e = gu.go(Z, OP_N, C1, OP_N, Fr, AU, mone, {addend_of(AU, one)});
    for (int r = 0; r < nr && e == hipSuccess; ++r) {
      const Mat Br = at(R.get(rhs[r].Gu, 0, i, -1), z0), xl = at(R.get(rhs[r].Gd, 0, i, 0), z0);
      const Mat V = ws_at(W.Pt[1], z0), C2 = ws_at(W.Pt[2], z0), BU = ws_at(W.BhU[r], z0 - ne);
      e = glu.go(Z, OP_N, C1, OP_N, Br, V, one, {});
      if (e == hipSuccess) e = glu.go(Z, OP_N, Fc, OP_N, xl, C2, one, {});
      if (e == hipSuccess)
        e = glu.go(Z, OP_N, C2, OP_C, Fc, BU, one, {addend_of(BU, one), addend_of(V, mone), addend_of(V, one, OP_C)});
    }
    return e;
  };
  for (int i = 0; i < B.max_nf; ++i) {
    const int Z = R.active_fwd(i);
    const int Zu = std::max(0, Z - U0);
    Step st;
    QTX_TRY(fwd_x(0, Z, i, false, &st));
    if (Zu > 0 && i == 0) {
      // fill-in seeds of the entries with u: Fr = L_u, Fc = U_u, Br = BL_u = -(BU_u)^H
      Cpl cs;
      QTX_TRY(coupling(U0, Zu, 0, 0, -1, &cs));
      const Gemm gu = on(g, U0), glu = on(gl, U0);
      QTX_TRY(gu.go(Zu, OP_N, Mat{}, OP_N, Mat{}, at(R.get(A_GRL, 0, 0, -1), U0), zero, {addend_of(cs.L, cmk(cs.sL, 0))},
                    zero, 0));
      QTX_TRY(gu.go(Zu, OP_N, Mat{}, OP_N, Mat{}, at(R.get(A_GRU, 0, 0, -1), U0), zero, {addend_of(cs.U, cmk(cs.sU, 0))},
                    zero, 0));
      for (int r = 0; r < nr; ++r) {
        const Mat BU = rhs[r].SU >= 0 ? at(R.get(rhs[r].SU, 0, 0, -1), U0) : Mat{};
        QTX_TRY(glu.go(Zu, OP_N, Mat{}, OP_N, Mat{}, at(R.get(rhs[r].Gu, 0, 0, -1), U0), zero,
                       {addend_of(BU, mone, OP_C)}, zero, 0));
      }
    } else if (Zu > 0) {
      // block j - 1's upper-separator terms, then the fill-ins of block j
      QTX_TRY(sep_u_terms(U0, Zu, i - 1));
      const Gemm gu = on(g, U0), glu = on(gl, U0);
      const Mat Tp = ws_at(W.Tm[0], U0), C1 = ws_at(W.Pt[0], U0);   // C1 = Fc_{j-1} x_{j-1}
      QTX_TRY(gu.go(Zu, OP_N, Tp, OP_N, at(R.get(A_GRL, 0, i, -2), U0), at(R.get(A_GRL, 0, i, -1), U0),
                    cmk(-st.c.sL, 0), {}));                                                        // Fr_j
      QTX_TRY(gu.go(Zu, OP_N, C1, OP_N, at(st.c.U, U0), at(R.get(A_GRU, 0, i, -1), U0), cmk(-st.c.sU, 0), {}));   // Fc_j
      for (int r = 0; r < nr; ++r) {
        const Mat Yq = ws_at(W.Pt[1], U0), CB = ws_at(W.Pt[2], U0);
        const Mat Brp = at(R.get(rhs[r].Gu, 0, i, -2), U0), Brj = at(R.get(rhs[r].Gu, 0, i, -1), U0);
        const Mat Fcp = at(R.get(A_GRU, 0, i, -2), U0);
        const bool bt = rhs[r].SU >= 0;
        QTX_TRY(glu.go(Zu, OP_N, at(st.c.L, U0), OP_N, at(R.get(rhs[r].Gd, 0, i, -1), U0), Yq, one, {}));   // L' xl_{j-1}
        if (bt) QTX_TRY(glu.go(Zu, OP_N, C1, OP_N, at(R.get(rhs[r].SU, 0, i, -1), U0), CB, one, {}));       // C1 BU_{j-1}
        QTX_TRY(glu.go(Zu, OP_N, Tp, OP_N, Brp, Brj, cmk(-st.c.sL, 0), {}));
        QTX_TRY(glu.go(Zu, OP_N, Yq, OP_C, Fcp, Brj, cmk(st.c.sL, 0),
                       {addend_of(Brj, one), addend_of(bt ? CB : Mat{}, one, OP_C)}));
      }
    }
    QTX_TRY(fwd_inv(0, Z, i, st));
    // entries whose last interior block is i: their separator terms
    int f0 = 0, f1 = 0;
    {
      int z = 0;
      while (z < Zall && B.ent[z].nf > i + 1) ++z;
      f0 = z;
      while (z < Zall && B.ent[z].nf == i + 1) ++z;
      f1 = z;
    }
    if (f1 > f0) {
      const int u0 = std::max(f0, U0);
      QTX_TRY(sep_u_terms(u0, f1 - u0, i));   // leaves C1 = Fc_t x_t in Pt[0]
      const int d1 = std::min(f1, Zd);
      if (d1 > f0) {
        const int Zf = d1 - f0;
        Cpl ct;
        QTX_TRY(coupling(f0, Zf, 0, i, 0, &ct));
        const Gemm gf = on(g, f0), glf = on(gl, f0);
        const Mat x = at(R.get(A_GRD, 0, i, 0), f0), T2 = ws_at(W.Pt[3], f0), Ahd_d = ws_at(W.Ahd, f0);
        QTX_TRY(gf.go(Zf, OP_N, ct.L, OP_N, x, T2, one, {}));                                         // T'' = L'_t x_t
        QTX_TRY(gf.go(Zf, OP_N, T2, OP_N, ct.U, Ahd_d, cmk(-ct.sL * ct.sU, 0), {addend_of(Ahd_d, one)}));
        const int b0 = std::max(f0, U0), Zb = d1 - b0;   // entries with both separators
        if (Zb > 0) {
          const Gemm gb = on(g, b0);
          QTX_TRY(gb.go(Zb, OP_N, ws_at(W.Pt[3], b0), OP_N, at(R.get(A_GRL, 0, i, -1), b0), ws_at(W.Ahl, b0),
                        cmk(-ct.sL, 0), {}));                                                         // M^_{d,u}
          QTX_TRY(gb.go(Zb, OP_N, ws_at(W.Pt[0], b0), OP_N, at(ct.U, b0 - f0), ws_at(W.Ahu, b0), cmk(-ct.sU, 0), {}));
        }
        for (int r = 0; r < nr; ++r) {
          const Mat Yt = ws_at(W.Pt[4], f0), V3 = ws_at(W.Pt[5], f0), Bhd_d = ws_at(W.Bhd[r], f0);
          const bool bt = rhs[r].SU >= 0;
          QTX_TRY(glf.go(Zf, OP_N, ct.L, OP_N, at(R.get(rhs[r].Gd, 0, i, 0), f0), Yt, one, {}));        // L'_t xl_t
          if (bt) QTX_TRY(glf.go(Zf, OP_N, T2, OP_N, at(R.get(rhs[r].SU, 0, i, 0), f0), V3, one, {}));  // T'' BU_t
          QTX_TRY(glf.go(Zf, OP_N, Yt, OP_C, ct.L, Bhd_d, one,
                         {addend_of(Bhd_d, one), addend_of(bt ? V3 : Mat{}, cmk(-ct.sL, 0)),
                          addend_of(bt ? V3 : Mat{}, cmk(ct.sL, 0), OP_C)}));
          if (Zb > 0) {
            // B^_{d,u} = -sL T'' Br_t + sL Y'' Fc_t^H + (C1 BU_t)^H (in Pt[6]);  B^_{u,d} = -(B^_{d,u})^H
            const Gemm glb = on(gl, b0);
            const Mat Bdu = ws_at(W.Pt[6], b0), CB = ws_at(W.Pt[7], b0);
            if (bt) QTX_TRY(glb.go(Zb, OP_N, ws_at(W.Pt[0], b0), OP_N, at(R.get(rhs[r].SU, 0, i, 0), b0), CB, one, {}));
            QTX_TRY(glb.go(Zb, OP_N, ws_at(W.Pt[3], b0), OP_N, at(R.get(rhs[r].Gu, 0, i, -1), b0), Bdu,
                           cmk(-ct.sL, 0), {}));
            QTX_TRY(glb.go(Zb, OP_N, ws_at(W.Pt[4], b0), OP_C, at(R.get(A_GRU, 0, i, -1), b0), Bdu, cmk(ct.sL, 0),
                           {addend_of(Bdu, one), addend_of(bt ? CB : Mat{}, one, OP_C)}));
            QTX_TRY(glb.go(Zb, OP_N, Mat{}, OP_N, Mat{}, ws_at(W.Bhu[r], b0), zero, {addend_of(Bdu, mone, OP_C)}, zero,
                           0));
          }
        }
      }
    }
  }

  // ---------------------------------------------------------- 2. separator chain
  // separator c of energy e lives with entry c n_e + e (partition c, its lower separator);
  // the coupling (c - 1, c) with entry c n_e + e (partition c); x^L_c, xl^L_c go to the
  // slots of entry (c + 1) n_e + e (partition c + 1, whose upper separator c is).
  // Energies: entries 0 .. n_e - 1.
  const int nsep = P - 1;
  auto sep_x = [&](int a, int c) { return at(R.get(a, 8, 0, 0), c * ne); };
  auto invert = [&](const Mat& X, const Mat& out) -> hipError_t {
    if (dry) return hipSuccess;
    ProfScope ps(ctx, QTX_KERNEL_INV, s, 8.0 * (double)b * b * b * ne, true);
    return launch_gje_invert(b, (double2*)X.p, bb, (double2*)out.p, out.stride, ne, W.gw, W.st, s,
                             (double2* const*)out.tab);
  };
  for (int c = 0; c < nsep; ++c) {
    const Mat XLm = ws(W.Pt[0]), xh = sep_x(A_GRD, c), xL = ws_at(W.XL, (c + 1) * ne);
    // M^L = M^_cc - A^_{c,c-1} xh_{c-1} A^_{c-1,c};  x^L = (M^L)^-1,  xh = (M^L + M^U_cc)^-1
    if (c == 0) {
      QTX_TRY(g.go(ne, OP_N, Mat{}, OP_N, Mat{}, XLm, zero, {addend_of(ws_at(W.Ahd, 0), one)}, zero, 0));
    } else {
      QTX_TRY(g.go(ne, OP_N, ws_at(W.Ahl, c * ne), OP_N, sep_x(A_GRD, c - 1), ws(W.Tm[0]), one, {}));
      QTX_TRY(g.go(ne, OP_N, ws(W.Tm[0]), OP_N, ws_at(W.Ahu, c * ne), XLm, mone, {addend_of(ws_at(W.Ahd, c * ne), one)}));
    }
    QTX_TRY(g.go(ne, OP_N, Mat{}, OP_N, Mat{}, ws(W.X), zero, {addend_of(XLm, one)}, zero, 0));
    QTX_TRY(invert(ws(W.X), xL));
    QTX_TRY(g.go(ne, OP_N, Mat{}, OP_N, Mat{}, ws(W.X), zero, {addend_of(XLm, one), addend_of(ws_at(W.AhU, c * ne), one)},
                 zero, 0));
    QTX_TRY(invert(ws(W.X), xh));
    for (int r = 0; r < nr; ++r) {
      // Q^L = B^_cc + A^_{c,c-1} xlh_{c-1} A^_{c,c-1}^H - V + V^H (V = T B^_{c-1,c}, T = A^_{c,c-1} xh_{c-1})
      const Mat QL = ws(W.Pt[1]), Qh = ws(W.Tm[3]);
      if (c == 0) {
        QTX_TRY(gl.go(ne, OP_N, Mat{}, OP_N, Mat{}, QL, zero, {addend_of(ws_at(W.Bhd[r], 0), one)}, zero, 0));
      } else {
        QTX_TRY(gl.go(ne, OP_N, ws_at(W.Ahl, c * ne), OP_N, sep_x(rhs[r].Gd, c - 1), ws(W.Tm[1]), one, {}));
        QTX_TRY(gl.go(ne, OP_N, ws(W.Tm[0]), OP_N, ws_at(W.Bhu[r], c * ne), ws(W.Tm[4]), one, {}));
        QTX_TRY(gl.go(ne, OP_N, ws(W.Tm[1]), OP_C, ws_at(W.Ahl, c * ne), QL, one,
                      {addend_of(ws_at(W.Bhd[r], c * ne), one), addend_of(ws(W.Tm[4]), mone),
                       addend_of(ws(W.Tm[4]), one, OP_C)}));
      }
      QTX_TRY(gl.go(ne, OP_N, xL, OP_N, QL, ws(W.Tm[2]), one, {}));
      QTX_TRY(gl.go(ne, OP_N, ws(W.Tm[2]), OP_C, xL, ws_at(W.XLl[r], (c + 1) * ne), one, {}));
      QTX_TRY(gl.go(ne, OP_N, Mat{}, OP_N, Mat{}, Qh, zero, {addend_of(QL, one), addend_of(ws_at(W.BhU[r], c * ne), one)},
                    zero, 0));
      QTX_TRY(gl.go(ne, OP_N, xh, OP_N, Qh, ws(W.Tm[2]), one, {}));
      QTX_TRY(gl.go(ne, OP_N, ws(W.Tm[2]), OP_C, xh, sep_x(rhs[r].Gd, c), one, {}));
    }
  }
  for (int c = nsep - 2; c >= 0; --c) {
    const Mat x = sep_x(A_GRD, c), Gn = sep_x(A_GRD, c + 1);
    const Mat Au = ws_at(W.Ahu, (c + 1) * ne), Al = ws_at(W.Ahl, (c + 1) * ne);
    const Mat Pp = ws(W.Tm[0]), Rp = ws(W.Tm[1]), Gu = ws(W.Tm[5]);
    QTX_TRY(g.go(ne, OP_N, x, OP_N, Au, Pp, one, {}));                     // x_c A^_{c,c+1}
    QTX_TRY(g.go(ne, OP_N, Al, OP_N, x, Rp, one, {}));                     // A^_{c+1,c} x_c
    QTX_TRY(g.go(ne, OP_N, Pp, OP_N, Gn, Gu, mone, {}));                   // G_{c,c+1}
    for (int r = 0; r < nr; ++r) {
      const Mat xl = sep_x(rhs[r].Gd, c), Gln = sep_x(rhs[r].Gd, c + 1);
      const Mat K1 = ws(W.Tm[2]), Vp = ws(W.Tm[3]), M1 = ws(W.Tm[4]);
      QTX_TRY(gl.go(ne, OP_N, x, OP_N, ws_at(W.Bhu[r], (c + 1) * ne), K1, one, {}));
      QTX_TRY(gl.go(ne, OP_N, xl, OP_C, Al, K1, mone, {addend_of(K1, one)}));      // K1 = x B^u - xl A^l^H
      QTX_TRY(gl.go(ne, OP_N, Pp, OP_N, Gln, Vp, one, {}));
      QTX_TRY(gl.go(ne, OP_N, K1, OP_C, Gu, M1, one, {}));
      QTX_TRY(gl.go(ne, OP_N, Vp, OP_C, Pp, xl, one, {addend_of(xl, one), addend_of(M1, one), addend_of(M1, mone, OP_C)}));
    }
    QTX_TRY(g.go(ne, OP_N, Gu, OP_N, Rp, x, mone, {addend_of(x, one)}));   // G_cc = x - G_{c,c+1} A^l x
  }

  // ---------------------------------------------------------- 3. interiors
  g = g_r;
  gl = g_l;
  // forward again for the partitions with an upper separator, from its x^L, xl^L
  for (int i = 0; i < B.max_nf; ++i) {
    const int Zu = R.active_fwd(i) - U0;
    if (Zu <= 0) break;
    Step st;
    QTX_TRY(fwd_x(U0, Zu, i, i == 0, &st));
    QTX_TRY(fwd_inv(U0, Zu, i, st));
  }
  // one-chain backward recurrence of every partition (the last partition's last block
  // keeps G = x, G^< = xl)
  for (int kk = 0;; ++kk) {
    const int Z = R.active_bwd(kk);
    if (Z == 0) break;
    const int Zn = kk == 0 ? std::min(Z, Zd) : Z;
    if (Zn <= 0) continue;
    Cpl c;
    QTX_TRY(coupling(0, Zn, 1, kk, 0, &c));
    const Mat xi = R.get(A_GRD, 1, kk, 0), Gn = R.get(A_GRD, 1, kk, 1);
    const Mat GRu = R.get(A_GRU, 1, kk, 0), GRl = R.get(A_GRL, 1, kk, 0);
    const Mat Pp = ws(W.Tm[0]), Rp = ws(W.Tm[1]), Vp = ws(W.Tm[2]), Wp = ws(W.Tm[3]), Yp = ws(W.Tm[4]),
              Zp = ws(W.Tm[5]);
    QTX_TRY(g.go(Zn, OP_N, xi, OP_N, c.U, Pp, one, {}));                        // P' = x_j U'
    QTX_TRY(g.go(Zn, OP_N, c.L, OP_N, xi, Rp, one, {}));                        // R' = L' x_j
    QTX_TRY(g.go(Zn, OP_N, Pp, OP_N, Gn, GRu, cmk(-c.sU, 0), {}));              // G_{j,j+1}
    QTX_TRY(g.go(Zn, OP_N, Gn, OP_N, Rp, GRl, cmk(-c.sL, 0), {}));              // G_{j+1,j}
    QTX_TRY(gl.go(Zn, OP_N, GRu, OP_N, c.L, Wp, one, {}));                      // W' = G_{j,j+1} L'
    // Y = -sL W' xl + x BU G_{j,j+1}^H,  Z = -sL xl L'^H + x BU,
    // G^<_{j,j+1} = Z G_{j+1,j+1}^H - sU P' G^<_{j+1,j+1},  G^<_jj = xl + V' P'^H + Y - Y^H
    for (const Rhs& r : rhs) {
      const Mat xl = R.get(r.Gd, 1, kk, 0), Gln = R.get(r.Gd, 1, kk, 1);
      const double2 msl = cmk(-c.sL, 0);
      if (r.SU >= 0) {
        QTX_TRY(gl.go(Zn, OP_N, xi, OP_N, R.get(r.SU, 1, kk, 0), Zp, one, {}));
        QTX_TRY(gl.go(Zn, OP_N, Zp, OP_C, GRu, Yp, one, {}));
        QTX_TRY(gl.go(Zn, OP_N, Wp, OP_N, xl, Yp, msl, {addend_of(Yp, one)}));
        QTX_TRY(gl.go(Zn, OP_N, xl, OP_C, c.L, Zp, msl, {addend_of(Zp, one)}));
      } else {
        QTX_TRY(gl.go(Zn, OP_N, Wp, OP_N, xl, Yp, msl, {}));
        QTX_TRY(gl.go(Zn, OP_N, xl, OP_C, c.L, Zp, msl, {}));
      }
      QTX_TRY(gl.go(Zn, OP_N, Pp, OP_N, Gln, Vp, one, {}));
      QTX_TRY(gl.go(Zn, OP_N, Zp, OP_C, Gn, R.get(r.Gu, 1, kk, 0), one, {addend_of(Vp, cmk(-c.sU, 0))}));
      QTX_TRY(gl.go(Zn, OP_N, Vp, OP_C, Pp, xl, one, {addend_of(xl, one), addend_of(Yp, one), addend_of(Yp, mone, OP_C)}));
    }
    QTX_TRY(g.go(Zn, OP_N, GRu, OP_N, Rp, xi, cmk(-c.sL, 0), {addend_of(xi, one)}));   // G_jj
  }
  // couplings of every upper separator with its partition's first block
  if (Zall > U0) {
    const int Zu = Zall - U0;
    Cpl c;
    QTX_TRY(coupling(U0, Zu, 9, 0, 0, &c));
    const Gemm gu = on(g, U0), glu = on(gl, U0);
    const Mat xL = ws_at(W.XL, U0), Glo = at(R.get(A_GRD, 2, 0, 0), U0);
    const Mat Pp = ws_at(W.Pt[0], U0), Rp = ws_at(W.Pt[1], U0), T = ws_at(W.Pt[2], U0);
    QTX_TRY(gu.go(Zu, OP_N, xL, OP_N, c.U, Pp, one, {}));                        // x^L U'_u
    QTX_TRY(gu.go(Zu, OP_N, c.L, OP_N, xL, Rp, one, {}));                        // L'_u x^L
    QTX_TRY(gu.go(Zu, OP_N, Pp, OP_N, Glo, at(R.get(A_GRU, 9, 0, 0), U0), cmk(-c.sU, 0), {}));
    QTX_TRY(gu.go(Zu, OP_N, Glo, OP_N, Rp, at(R.get(A_GRL, 9, 0, 0), U0), cmk(-c.sL, 0), {}));
    for (const Rhs& r : rhs) {
      const Mat xlL = ws_at(W.XLl[&r - &rhs[0]], U0), Gllo = at(R.get(r.Gd, 2, 0, 0), U0);
      // T = -sL xl^L L'^H (+ x^L BU_u);  G^<_{u,lo} = T G_lo^H - sU P' G^<_lo
      if (r.SU >= 0) {
        QTX_TRY(glu.go(Zu, OP_N, xL, OP_N, at(R.get(r.SU, 9, 0, 0), U0), T, one, {}));
        QTX_TRY(glu.go(Zu, OP_N, xlL, OP_C, c.L, T, cmk(-c.sL, 0), {addend_of(T, one)}));
      } else {
        QTX_TRY(glu.go(Zu, OP_N, xlL, OP_C, c.L, T, cmk(-c.sL, 0), {}));
      }
      QTX_TRY(glu.go(Zu, OP_N, Pp, OP_N, Gllo, ws_at(W.Pt[3], U0), one, {}));
      QTX_TRY(glu.go(Zu, OP_N, T, OP_C, Glo, at(R.get(r.Gu, 9, 0, 0), U0), one,
                     {addend_of(ws_at(W.Pt[3], U0), cmk(-c.sU, 0))}));
    }
  }

  // ---------------------------------------------------------- status
  // Non-finite values reach every partition's first interior block; a failure of any
  // partition (or of the separator chain, recorded on partition 0) is carried to
  // partition 0 (P - 1 passes along the chain of partitions), which fills and reports.
  std::vector<int> first{A_GRD};
  for (const Rhs& r : rhs) first.push_back(r.Gd);
  for (int a : first) {
    const Mat m = R.get(a, 2, 0, 0);
    if (!dry) QTX_TRY(launch_check_finite_entries(m.tab, bb, Zall, W.st, s));
  }
  for (int q = 1; q < P && !dry; ++q) QTX_TRY(launch_status_merge(W.st, W.part, Zall, s));
  std::vector<std::pair<int, bool>> outs{{A_GRD, true}, {A_GRU, false}, {A_GRL, false}};
  for (const Rhs& r : rhs) { outs.push_back({r.Gd, true}); outs.push_back({r.Gu, false}); }
  for (auto& o : outs) {
    const Mat m = R.get(o.first, 2, 0, 0);
    if (!dry) QTX_TRY(launch_nan_fill_entries((double2* const*)m.tab, o.second ? W.cnt_d : W.cnt_u, Zall, W.st, s));
  }
  if (!dry) QTX_TRY(launch_scatter_status(W.st, W.ust, Zall, s));
  return R.late ? QTX_ERR_HIP : QTX_OK;
}

// FNV-1a over bytes.
struct Hasher {
  uint64_t h = 1469598103934665603ull;
  void add(const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  }
  template <class T> void val(const T& v) { add(&v, sizeof(v)); }
};

// Plan, upload and run (or capture / replay) a full solve.
// The separator block of a split chain of n_b >= 3 blocks: the top half runs
// c forward steps and the bottom half n_b - c, so the bottom half reaches the
// separator no earlier than the top half's last step.
int split_point(int n_b) { return (n_b - 1) / 2; }

// The entries of one energy: one chain, or the two halves of a split chain.
// Interior lengths of the P partitions of a chain of n_b blocks: n_b - (P - 1) blocks
// (the separators taken out), as equal as possible, longer ones first.
std::vector<int> partition_lengths(int n_b, int P) {
  const int m = n_b - (P - 1);
  std::vector<int> len(P);
  for (int q = 0; q < P; ++q) len[q] = m / P + (q < m % P ? 1 : 0);
  return len;
}

std::vector<Entry> entries_of(const qtx_rgf_problem& p, int e) {
  Entry a;
  a.p = &p;
  a.e = e;
  if (p.partitions > 1) {
    // partition q: interior blocks off .. off + nf - 1, separators off - 1 (q > 0) and
    // off + nf (q < P - 1); the backward recurrence starts at the last interior block
    std::vector<Entry> out;
    int off = 0;
    for (const int len : partition_lengths(p.n_b, p.partitions)) {
      Entry t = a;
      t.q = (int)out.size();
      t.off = off;
      t.nf = len;
      t.nbk = len + 1;
      out.push_back(t);
      off += len + 1;
    }
    return out;
  }
  if (!(p.flags & QTX_SPLIT_CHAIN) || p.n_b < 3) {
    a.nf = a.nbk = p.n_b;
    return {a};
  }
  const int c = split_point(p.n_b);
  Entry t = a, bt = a;
  t.nf = c; t.nbk = c + 1; t.c = c;
  bt.nf = bt.nbk = p.n_b - c; bt.rev = true; bt.c = c;
  return {t, bt};
}

qtx_status solve_all(qtx_rgf_ctx ctx, const qtx_rgf_problem* probs, int n_probs, hipStream_t s) {
  // 1. group energies by batch key, split each group over lane_split stream lanes
  //    (alternate energies, so that the parts carry the same mix of n_b); each part
  //    becomes one or more batches (chunks) on its own lane.  The two halves of a
  //    split energy stay in one batch.
  using Unit = std::vector<Entry>;
  std::vector<BatchKey> keys;
  std::vector<std::vector<Unit>> groups;
  {
    std::vector<BatchKey> gkeys;
    std::vector<std::vector<Unit>> gents;
    for (int q = 0; q < n_probs; ++q) {
      const BatchKey k = key_of(probs[q]);
      size_t g = 0;
      while (g < gkeys.size() && !(gkeys[g] == k)) ++g;
      if (g == gkeys.size()) { gkeys.push_back(k); gents.emplace_back(); }
      for (int e = 0; e < probs[q].n_e; ++e) gents[g].push_back(entries_of(probs[q], e));
    }
    for (size_t g = 0; g < gkeys.size(); ++g) {
      auto& ent = gents[g];
      std::stable_sort(ent.begin(), ent.end(), [](const Unit& a, const Unit& b) { return a[0].p->n_b > b[0].p->n_b; });
      const size_t parts = std::min<size_t>((size_t)std::max(1, ctx->lane_split), ent.size());
      for (size_t j = 0; j < parts; ++j) {
        keys.push_back(gkeys[g]);
        groups.emplace_back();
        for (size_t z = j; z < ent.size(); z += parts) groups.back().push_back(ent[z]);
      }
    }
  }
  size_t total_need = 0;
  for (size_t g = 0; g < keys.size(); ++g)
    for (const Unit& u : groups[g]) total_need += per_entry_bytes(keys[g]) * u.size();
  int64_t rbt_elems = 0;
  const size_t budget = ws_budget(ctx);
  std::vector<Batch> batches;
  std::vector<size_t> lane_bytes;
  for (size_t g = 0; g < keys.size(); ++g) {
    auto& units = groups[g];
    const size_t per = per_entry_bytes(keys[g]);
    size_t n_ent = 0;
    for (const Unit& u : units) n_ent += u.size();
    const double share = total_need > budget ? (double)(per * n_ent) / (double)total_need : 1.0;
    size_t chunk = n_ent;
    if (total_need > budget) chunk = std::max<size_t>(1, (size_t)(share * (double)budget) / per);
    size_t lane_need = 0;
    for (size_t u0 = 0; u0 < units.size();) {
      Batch B;
      B.key = keys[g];
      size_t u1 = u0;
      while (u1 < units.size() && (B.ent.empty() || B.ent.size() + units[u1].size() <= chunk)) {
        B.ent.insert(B.ent.end(), units[u1].begin(), units[u1].end());
        ++u1;
      }
      u0 = u1;
      // Sort by (nf, nbk, rev) descending: the entries active at a forward step and
      // at a backward step are prefixes (nbk is nf or nf + 1), and the bottom halves
      // that reach their separator at one step are a contiguous run.  A partitioned
      // batch goes partition-major (entry q n_e + e; the interiors shrink with q, so
      // the active entries are still prefixes).
      if (B.key.parts > 1)
        std::stable_sort(B.ent.begin(), B.ent.end(), [](const Entry& a, const Entry& b) { return a.q < b.q; });
      else
        std::stable_sort(B.ent.begin(), B.ent.end(), [](const Entry& a, const Entry& b) {
          return std::make_tuple(a.nf, a.nbk, a.rev) > std::make_tuple(b.nf, b.nbk, b.rev);
        });
      if (B.key.parts > 1) {
        // status chain: partition q takes the failure of partition q + 1 of its energy
        const int ne = (int)B.ent.size() / B.key.parts;
        for (size_t z = 0; z + ne < B.ent.size(); ++z) B.ent[z].part = (int)z + ne;
      }
      for (size_t z = 0; z < B.ent.size(); ++z) {
        B.max_nf = std::max(B.max_nf, B.ent[z].nf);
        B.max_nbk = std::max(B.max_nbk, B.ent[z].nbk);
        if (!B.ent[z].rev) continue;
        B.split = true;
        for (size_t y = 0; y < B.ent.size(); ++y)
          if (!B.ent[y].rev && B.ent[y].p == B.ent[z].p && B.ent[y].e == B.ent[z].e) B.ent[y].part = (int)z;
      }
      B.lane = (int)g;
      lane_need = std::max(lane_need, batch_ws_bytes(B.key, (int)B.ent.size()));
      batches.push_back(std::move(B));
      // bottom halves with a BT right-hand side: room for their reversed upper blocks
      Batch& nb = batches.back();
      const int64_t bbk = (int64_t)nb.key.b * nb.key.b;
      for (Entry& en : nb.ent) {
        if (!en.rev) continue;
        const int64_t blocks = (int64_t)(en.p->n_b - 1 - en.c) * bbk;
        if (nb.key.l_bt) { en.rbt_l = rbt_elems; rbt_elems += blocks; }
        if (nb.key.g_bt) { en.rbt_g = rbt_elems; rbt_elems += blocks; }
      }
    }
    lane_bytes.push_back(align_up(lane_need));
  }
  const int n_lanes = (int)keys.size();
  if (rbt_elems > 0) QTX_TRYS(ensure_rbt(ctx, (size_t)rbt_elems * sizeof(double2)));
  // 2. dry pass: tables and per-entry data of every batch
  std::vector<Run> runs(batches.size());
  size_t tab_total = 0;
  for (size_t bi = 0; bi < batches.size(); ++bi) {
    Run& R = runs[bi];
    R.ctx = ctx;
    R.B = &batches[bi];
    R.dry = true;
    R.bb = (int64_t)R.B->key.b * R.B->key.b;
    const int Z = (int)R.B->ent.size();
    const EntryData ed = entry_data_layout(Z);
    R.host.assign(ed.end, 0);
    for (int z = 0; z < Z; ++z) {
      const Entry& en = R.B->ent[z];
      const double E = en.p->energies[en.e];
      // a bottom half neither reports nor fills: its top half does both for the energy
      // (likewise partitions q > 0: partition 0 reports and fills the whole chain)
      const bool lead = !en.rev && en.q <= 0;
      int32_t* us = en.p->status && lead ? en.p->status + en.e : nullptr;
      const int64_t cd = lead ? (int64_t)en.p->n_b * R.bb : 0, cu = lead ? (int64_t)(en.p->n_b - 1) * R.bb : 0;
      const int32_t part = en.part;
      std::memcpy(R.host.data() + ed.en + z * sizeof(double), &E, sizeof(double));
      std::memcpy(R.host.data() + ed.ust + z * sizeof(void*), &us, sizeof(void*));
      std::memcpy(R.host.data() + ed.cnt_d + z * sizeof(int64_t), &cd, sizeof(int64_t));
      std::memcpy(R.host.data() + ed.cnt_u + z * sizeof(int64_t), &cu, sizeof(int64_t));
      std::memcpy(R.host.data() + ed.part + z * sizeof(int32_t), &part, sizeof(int32_t));
    }
    BatchWs W;
    qtx_status st = R.B->key.parts > 1 ? run_partition(R, W) : run_batch(R, W);
    if (st != QTX_OK) return st;
    batches[bi].tab_off = tab_total;
    tab_total += align_up(R.host.size());
  }
  // 3. workspace: lane regions, then the table block
  size_t ws_total = 0;
  std::vector<size_t> lane_off(n_lanes);
  for (int l = 0; l < n_lanes; ++l) { lane_off[l] = ws_total; ws_total += lane_bytes[l]; }
  const size_t tab_start = ws_total;
  ws_total += tab_total + 4096;
  QTX_TRYS(ensure_ws(ctx, ws_total));
  QTX_TRYS(ensure_pinned(ctx, tab_total + 256));
  char* pin = (char*)ctx->pinned;
  for (size_t bi = 0; bi < batches.size(); ++bi)
    std::memcpy(pin + batches[bi].tab_off, runs[bi].host.data(), runs[bi].host.size());
  char* dev_tab = (char*)ctx->ws + tab_start;
  QTX_TRY(hipMemcpyAsync(dev_tab, pin, tab_total, hipMemcpyHostToDevice, s));
  if (!ctx->upload_done) QTX_TRY(hipEventCreateWithFlags(&ctx->upload_done, hipEventDisableTiming));
  QTX_TRY(hipEventRecord(ctx->upload_done, s));

  // 4. launch (optionally captured into a cached graph)
  uint64_t sig = 0;
  bool replay = false;
  bool capture = ctx->use_graph && s != nullptr;
  if (capture) {
    Hasher h;
    h.val(n_probs);
    for (int q = 0; q < n_probs; ++q) {
      h.val(probs[q]);
      h.add(probs[q].energies, sizeof(double) * probs[q].n_e);
    }
    h.val(ctx->ws);
    h.val(ctx->ws_size);
    sig = h.h;
    for (auto& gce : ctx->graphs)
      if (gce.sig == sig) {
        QTX_TRY(hipGraphLaunch(gce.exec, s));
        ++ctx->graph_launches;
        replay = true;
      }
  }
  if (replay) return QTX_OK;
  if (n_lanes > 1) QTX_TRYS(ensure_aux(ctx, n_lanes));
  // The side stream is used in eager solves only (QTX_OPT_OVERLAP and QTX_OPT_GRAPH
  // exclude each other): a capture that forked the side stream from a lane stream at
  // every forward step ended in a segmentation fault inside the runtime.
  const bool use_side = ctx->overlap && !capture;
  if (use_side) QTX_TRYS(ensure_side(ctx, n_lanes));
  if (capture) {
    QTX_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
  }
  qtx_status result = QTX_OK;
  for (int l = 0; l < n_lanes && result == QTX_OK; ++l) {
    hipStream_t ls = s;
    if (n_lanes > 1) {
      ls = ctx->aux[l];
      if (hipEventRecord(ctx->fork_ev[l], s) != hipSuccess || hipStreamWaitEvent(ls, ctx->fork_ev[l], 0) != hipSuccess) {
        result = hip_fail(ctx, hipErrorUnknown);
        break;
      }
    }
    for (size_t bi = 0; bi < batches.size() && result == QTX_OK; ++bi) {
      if (batches[bi].lane != l) continue;
      Run& R = runs[bi];
      R.dry = false;
      R.s = ls;
      if (use_side) {
        R.side = ctx->side[l];
        R.side_fork = ctx->side_fork[l];
        R.side_join = ctx->side_join[l];
      }
      R.dev = dev_tab + batches[bi].tab_off;
      const int Z = (int)R.B->ent.size();
      BatchWs W = carve_batch((char*)ctx->ws + lane_off[l], R.B->key, Z);
      const EntryData ed = entry_data_layout(Z);
      W.en = (const double*)(R.dev + ed.en);
      W.ust = (int32_t* const*)(R.dev + ed.ust);
      W.cnt_d = (const int64_t*)(R.dev + ed.cnt_d);
      W.cnt_u = (const int64_t*)(R.dev + ed.cnt_u);
      W.part = (const int32_t*)(R.dev + ed.part);
      result = R.B->key.parts > 1 ? run_partition(R, W) : run_batch(R, W);
    }
    if (n_lanes > 1 && result == QTX_OK) {
      if (hipEventRecord(ctx->join_ev[l], ls) != hipSuccess || hipStreamWaitEvent(s, ctx->join_ev[l], 0) != hipSuccess)
        result = hip_fail(ctx, hipErrorUnknown);
    }
  }
  if (capture) {
    ctx->capturing = false;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (result != QTX_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return result;
    }
    if (e != hipSuccess) return hip_fail(ctx, e);
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(ctx, e);
    if (ctx->graphs.size() >= 8) {
      (void)hipGraphExecDestroy(ctx->graphs.front().exec);
      ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back({sig, exec});
    ++ctx->graph_captures;
    QTX_TRY(hipGraphLaunch(exec, s));
    ++ctx->graph_launches;
  }
  return result;
}

// Tuning cache file: a text file, first line "qtx-tune 3 <arch> <CUs>", then one
// line per record "o2 M N K class p variant ms_0 .. ms_{n-1}" (INT8 tile variants) or
// "tm M N K class code variant ms_32 ms_64" (tile edge of the other schemes).  A file
// written on a different device kind or format, or lines that do not parse, are ignored.
std::string device_tag(int device) {
  hipDeviceProp_t pr;
  if (hipGetDeviceProperties(&pr, device) != hipSuccess) return "unknown 0";
  char buf[160];
  std::snprintf(buf, sizeof buf, "%s %d", pr.gcnArchName, pr.multiProcessorCount);
  for (char* c = buf; *c; ++c)
    if (*c == ':' ) { *c = '\0'; break; }   // drop target features
  std::string t(buf);
  if (t.find(' ') == std::string::npos) t += " " + std::to_string(pr.multiProcessorCount);
  return t;
}

void tune_load(qtx_rgf_ctx ctx) {
  if (ctx->tune_path.empty()) return;
  FILE* f = std::fopen(ctx->tune_path.c_str(), "r");
  if (!f) return;
  char line[1024];
  bool ok = false;
  const std::string tag = "qtx-tune 3 " + device_tag(ctx->device);
  if (std::fgets(line, sizeof line, f)) {
    std::string h(line);
    while (!h.empty() && (h.back() == '\n' || h.back() == '\r' || h.back() == ' ')) h.pop_back();
    ok = (h == tag);
  }
  while (ok && std::fgets(line, sizeof line, f)) {
    int M, N, K, c, p, v, used = 0;
    bool tile = false;
    if (std::sscanf(line, "o2 %d %d %d %d %d %d%n", &M, &N, &K, &c, &p, &v, &used) != 6) {
      if (std::sscanf(line, "tm %d %d %d %d %d %d%n", &M, &N, &K, &c, &p, &v, &used) != 6) continue;
      tile = true;
    }
    if (M < 1 || N < 1 || K < 1 || c < 0 || c > 9) continue;
    if (!tile && (p < 1 || p > kO2MaxModuli || v < 0 || v >= o2_variant_count())) continue;
    if (tile && (p < kTileCodeBase || v < 0 || v > 1)) continue;
    TuneRec r;
    r.variant = v;
    const char* q = line + used;
    double ms;
    int n = 0;
    while (std::sscanf(q, "%lf%n", &ms, &n) == 1) { r.ms.push_back(ms); q += n; }
    ctx->tune[TuneKey(M, N, K, c, p)] = r;
  }
  std::fclose(f);
}

bool tune_save(qtx_rgf_ctx ctx) {
  if (ctx->tune_path.empty()) return true;
  const std::string tmp = ctx->tune_path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "qtx-tune 3 %s\n", device_tag(ctx->device).c_str());
  for (const auto& kv : ctx->tune) {
    std::fprintf(f, "%s %d %d %d %d %d %d", std::get<4>(kv.first) >= kTileCodeBase ? "tm" : "o2",
                 std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
                 std::get<4>(kv.first), kv.second.variant);
    for (double ms : kv.second.ms) std::fprintf(f, " %.4f", ms);
    std::fprintf(f, "\n");
  }
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), ctx->tune_path.c_str()) == 0;
}

}  // namespace

extern "C" {

qtx_status qtx_ozaki2_bits(int32_t p, int32_t K, int32_t* moduli, int32_t* p_used, int32_t* kbits) {
  O2Params P;
  if (!o2_params(p, K, &P)) return QTX_ERR_UNSUPPORTED;
  if (moduli)
    for (int i = 0; i < P.p; ++i) moduli[i] = o2_modulus(i);
  if (p_used) *p_used = P.p;
  if (kbits) *kbits = P.kbits;
  return QTX_OK;
}

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
  tune_load(ctx);
  void* scr = nullptr;
  (void)noalloc_scratch(device, &scr);   // set-up of qtx_zgemm_noalloc (it retries and reports a failure)
  *out = ctx;
  return QTX_OK;
}

qtx_status qtx_rgf_set_option(qtx_rgf_ctx ctx, int option, int64_t value) {
  if (!ctx) return QTX_ERR_ARG;
  switch (option) {
    case QTX_OPT_GRAPH:
      // the side-stream overlap is not captured (one capture that forked it at every
      // forward step ended in a host fault inside the runtime): the two are exclusive
      if (value != 0 && ctx->overlap) return QTX_ERR_UNSUPPORTED;
      ctx->use_graph = value != 0;
      return QTX_OK;
    case QTX_OPT_RESERVE_WORKSPACE: {
      if (value < 0) return QTX_ERR_ARG;
      DeviceGuard guard(ctx->device);
      return ensure_ws(ctx, (size_t)value);
    }
    case QTX_OPT_OVERLAP:
      if (value != 0 && ctx->use_graph) return QTX_ERR_UNSUPPORTED;
      if (ctx->overlap != (value != 0)) {
        DeviceGuard guard(ctx->device);
        (void)hipDeviceSynchronize();
        drop_graphs(ctx);   // captured launches carry the old stream structure
      }
      ctx->overlap = value != 0;
      return QTX_OK;
    case QTX_OPT_LANE_SPLIT:
      if (value < 1 || value > 8) return QTX_ERR_ARG;
      if (ctx->lane_split != (int)value) {
        DeviceGuard guard(ctx->device);
        (void)hipDeviceSynchronize();
        drop_graphs(ctx);   // captured launches carry the old stream structure
      }
      ctx->lane_split = (int)value;
      return QTX_OK;
    case QTX_OPT_INT8_TILE_VARIANT:
      if (value < -1 || value >= o2_variant_count()) return QTX_ERR_ARG;
      if (ctx->o2_force != (int)value) {
        DeviceGuard guard(ctx->device);
        (void)hipDeviceSynchronize();
        drop_graphs(ctx);   // captured launches carry the old choice
      }
      ctx->o2_force = (int)value;
      return QTX_OK;
    default:
      return QTX_ERR_ARG;
  }
}

qtx_status qtx_rgf_get_stat(qtx_rgf_ctx ctx, int stat, int64_t* value) {
  if (!ctx || !value) return QTX_ERR_ARG;
  switch (stat) {
    case QTX_STAT_GRAPH_LAUNCHES: *value = ctx->graph_launches; return QTX_OK;
    case QTX_STAT_GRAPH_CAPTURES: *value = ctx->graph_captures; return QTX_OK;
    case QTX_STAT_WORKSPACE_BYTES: *value = (int64_t)ctx->ws_size; return QTX_OK;
    case QTX_STAT_TUNE_RECORDS: *value = (int64_t)ctx->tune.size(); return QTX_OK;
    default: return QTX_ERR_ARG;
  }
}

qtx_status qtx_rgf_profile(qtx_rgf_ctx ctx, int enable) {
  if (!ctx) return QTX_ERR_ARG;
  ctx->profiling = enable != 0;
  return QTX_OK;
}

qtx_status qtx_rgf_profile_read(qtx_rgf_ctx ctx, int family, double* total_ms, int64_t* launches,
                                double* flops) {
  if (!ctx || family < 0 || family > 2) return QTX_ERR_ARG;
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
    drop_graphs(ctx);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->rbt) (void)hipFree(ctx->rbt);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->upload_done) (void)hipEventDestroy(ctx->upload_done);
    if (ctx->last_done) (void)hipEventDestroy(ctx->last_done);
    for (auto& f : ctx->prof)
      for (auto& r : f.pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    for (size_t i = 0; i < ctx->aux.size(); ++i) {
      (void)hipStreamDestroy(ctx->aux[i]);
      (void)hipEventDestroy(ctx->fork_ev[i]);
      (void)hipEventDestroy(ctx->join_ev[i]);
    }
    for (size_t i = 0; i < ctx->side.size(); ++i) {
      (void)hipStreamDestroy(ctx->side[i]);
      (void)hipEventDestroy(ctx->side_fork[i]);
      (void)hipEventDestroy(ctx->side_join[i]);
    }
  }
  delete ctx;
  return QTX_OK;
}

size_t qtx_rgf_footprint(const qtx_rgf_problem* p) {
  if (!valid_problem(p) || check_supported(p) != QTX_OK) return 0;
  const size_t chains = ((p->flags & QTX_SPLIT_CHAIN) && p->n_b >= 3) ? 2 : 1;
  return chains * per_entry_bytes(key_of(*p));
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
  return ordered(ctx, (hipStream_t)hip_stream, [&]() { return solve_all(ctx, probs, n_probs, (hipStream_t)hip_stream); });
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
  if (sc.o2() && K > 0) {
    O2Params P;
    if (!o2_params(sc.ns, K, &P)) return QTX_ERR_UNSUPPORTED;
  }
  if (sc.sliced() && K > 0) {
    const size_t need = operand_bytes(M, K, sc, batch) + operand_bytes(N, K, sc, batch) + 4096;
    qtx_status st = ensure_ws(ctx, need);
    if (st != QTX_OK) return st;
    char* w = (char*)ctx->ws;
    sb.S[0] = w; w += align_up(operand_digit_bytes(M, K, sc) * batch);
    sb.E[0] = (int32_t*)w; w += align_up((size_t)split_exp_stride(M, K) * 4 * batch);
    sb.S[1] = w; w += align_up(operand_digit_bytes(N, K, sc) * batch);
    sb.E[1] = (int32_t*)w;
  }
  return ordered(ctx, (hipStream_t)hip_stream, [&]() -> qtx_status {
    QTX_TRY(run_product(ctx, d, sc, sb, (hipStream_t)hip_stream));
    return QTX_OK;
  });
}

qtx_status qtx_zgemm_noalloc(qtx_rgf_ctx ctx, char opA, char opB, int32_t M, int32_t N, int32_t K,
                             double alpha_re, double alpha_im, const void* A, int64_t lda, int64_t sA, const void* B,
                             int64_t ldb, int64_t sB, double beta_re, double beta_im, void* C, int64_t ldc, int64_t sC,
                             int32_t batch, int32_t prec, int32_t n_slices, void* hip_stream) {
  if (!ctx) return QTX_ERR_ARG;
  if (ctx->sticky != QTX_OK) return ctx->sticky;
  if ((opA != 'N' && opA != 'C') || (opB != 'N' && opB != 'C')) return QTX_ERR_ARG;
  if (M < 0 || N < 0 || K < 0 || batch < 1 || !C || ldc < N) return QTX_ERR_ARG;
  if (K > 0 && (!A || !B)) return QTX_ERR_ARG;
  if (K > 0 && (lda < (opA == 'N' ? K : M) || ldb < (opB == 'N' ? N : K))) return QTX_ERR_ARG;
  Scheme sc;
  if (!make_scheme(prec, n_slices, &sc)) return QTX_ERR_UNSUPPORTED;
  if (sc.o2() && K > 0) {
    O2Params P;
    if (!o2_params(sc.ns, K, &P)) return QTX_ERR_UNSUPPORTED;
  }
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
  if (sc.sliced() && K > 0) {
    // converted operands in the fixed scratch: an operand shared by the batch (stride 0)
    // is converted once, as in qtx_zgemm
    const int ba = sA == 0 ? 1 : batch, bbn = sB == 0 ? 1 : batch;
    const size_t need = operand_bytes(M, K, sc, ba) + operand_bytes(N, K, sc, bbn);
    if (need > kNoAllocScratchBytes) return QTX_ERR_ARG;
    void* base = nullptr;
    QTX_TRYS(noalloc_scratch(ctx->device, &base));
    char* w = (char*)base;
    sb.S[0] = w; w += align_up(operand_digit_bytes(M, K, sc) * ba);
    sb.E[0] = (int32_t*)w; w += align_up((size_t)split_exp_stride(M, K) * 4 * ba);
    sb.S[1] = w; w += align_up(operand_digit_bytes(N, K, sc) * bbn);
    sb.E[1] = (int32_t*)w;
  }
  // no per-launch timer events here (creating one could allocate)
  const bool prof = ctx->profiling;
  ctx->profiling = false;
  const hipError_t e = run_product(ctx, d, sc, sb, (hipStream_t)hip_stream);
  ctx->profiling = prof;
  QTX_TRY(e);
  return QTX_OK;
}

qtx_status qtx_rgf_tune(qtx_rgf_ctx ctx, int32_t b, int32_t prec, int32_t n_slices, int32_t batch,
                        void* hip_stream, int32_t* out_variant, double* out_ms, int32_t max_variants,
                        int32_t* out_count) {
  if (!ctx) return QTX_ERR_ARG;
  if (ctx->sticky != QTX_OK) return ctx->sticky;
  if (b < 1 || b > 1024 || batch < 1 || max_variants < 0 || (max_variants > 0 && !out_ms)) return QTX_ERR_ARG;
  Scheme sc;
  if (!make_scheme(prec, n_slices, &sc)) return QTX_ERR_UNSUPPORTED;
  O2Params P;
  if (sc.o2() && !o2_params(sc.ns, b, &P)) return QTX_ERR_UNSUPPORTED;
  DeviceGuard guard(ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t bb = (int64_t)b * b;
  const size_t bytes = (size_t)bb * batch * sizeof(double2);
  double2* buf[3] = {nullptr, nullptr, nullptr};
  for (auto& p : buf)
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      for (auto& q : buf)
        if (q) (void)hipFree(q);
      return QTX_ERR_NOMEM;
    }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  qtx_status st = QTX_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      launch_fill_hash(buf[0], bb * batch, 1u, s) != hipSuccess ||
      launch_fill_hash(buf[1], bb * batch, 2u, s) != hipSuccess)
    st = hip_fail(ctx, hipErrorUnknown);
  // INT8: the tile variants; the other schemes: 32 x 32 (variant 0) or 64 x 64 tiles
  const int nv = sc.o2() ? o2_variant_count() : 2;
  std::vector<double> ms(nv, 0.0);
  const int saved_force = ctx->o2_force, saved_tile = ctx->tile_force;
  const bool saved_prof = ctx->profiling;
  ctx->profiling = false;
  // A warm-up pass over every variant (the first launches of a cold GPU run at lower
  // clocks: timed first, variant 0 read 20% slow), then two timed rounds in opposite
  // orders; each variant keeps its faster round.
  const int reps = 3;
  auto select = [&](int v) {
    if (sc.o2()) ctx->o2_force = v;
    else ctx->tile_force = v ? 64 : 32;
  };
  auto one = [&]() {
    return qtx_zgemm(ctx, 'N', 'N', b, b, b, 1.0, 0.0, buf[0], b, bb, buf[1], b, bb, 0.0, 0.0, buf[2], b, bb, batch,
                     prec, n_slices, hip_stream);
  };
  for (int v = 0; v < nv && st == QTX_OK; ++v) {
    select(v);
    for (int r = 0; r < 2 && st == QTX_OK; ++r) st = one();
  }
  for (int round = 0; round < 2 && st == QTX_OK; ++round) {
    for (int w = 0; w < nv && st == QTX_OK; ++w) {
      const int v = round == 0 ? w : nv - 1 - w;
      select(v);
      if (hipEventRecord(e0, s) != hipSuccess) { st = hip_fail(ctx, hipErrorUnknown); break; }
      for (int r = 0; r < reps && st == QTX_OK; ++r) st = one();
      if (st != QTX_OK) break;
      float t = 0.0f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
        st = hip_fail(ctx, hipErrorUnknown);
        break;
      }
      ms[v] = round == 0 ? t / reps : std::min(ms[v], (double)t / reps);
    }
  }
  ctx->o2_force = saved_force;
  ctx->tile_force = saved_tile;
  ctx->profiling = saved_prof;
  (void)hipStreamSynchronize(s);
  for (auto& p : buf) (void)hipFree(p);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != QTX_OK) return st;
  int best = 0;
  for (int v = 1; v < nv; ++v)
    if (ms[v] < ms[best]) best = v;
  TuneRec rec;
  rec.variant = best;
  rec.ms = ms;
  ctx->tune[TuneKey(b, b, b, batch_class(batch), sc.o2() ? P.p : tile_code(sc))] = rec;
  drop_graphs(ctx);   // captured launches carry the old choice
  if (out_variant) *out_variant = best;
  if (out_count) *out_count = nv;
  for (int v = 0; v < nv && v < max_variants; ++v) out_ms[v] = ms[v];
  return tune_save(ctx) ? QTX_OK : QTX_ERR_ARG;
}

// ---------------------------------------------------------------- screened Coulomb (W) system
// BT blocks of V P^R and of V P^<> V^H (the W row of Table I), batched over energies.
// V is Hermitian BT (V_{i+1,i} = V_u[i]^H); P^<> is skew-Hermitian BT
// (P_{i+1,i} = -P_u[i]^H).  Row i of Y = V P^< needs Y_{i,i-1}, Y_ii, Y_{i,i+1},
// Y_{i,i+2}; B_ij = sum_k Y_ik (V_jk)^H for j = i, i+1.
qtx_status qtx_w_assemble(qtx_rgf_ctx ctx, int32_t n_b, int32_t b, int32_t n_e, int32_t prec, int32_t n_slices,
                          const void* V_d, const void* V_u, const void* PR_d, const void* PR_u, const void* PR_l,
                          const void* PL_d, const void* PL_u, const void* PG_d, const void* PG_u, void* VPR_d,
                          void* VPR_u, void* VPR_l, void* BL_d, void* BL_u, void* BG_d, void* BG_u,
                          void* hip_stream) {
  if (!ctx) return QTX_ERR_ARG;
  if (ctx->sticky != QTX_OK) return ctx->sticky;
  if (n_b < 1 || b < 1 || b > 1024 || n_e < 1) return QTX_ERR_ARG;
  if (!V_d || !PR_d || !PL_d || !VPR_d || !BL_d) return QTX_ERR_ARG;
  if (n_b > 1 && (!V_u || !PR_u || !PR_l || !PL_u || !VPR_u || !VPR_l || !BL_u)) return QTX_ERR_ARG;
  const bool greater = PG_d != nullptr;
  if (greater != (BG_d != nullptr)) return QTX_ERR_ARG;
  if (greater && n_b > 1 && (!PG_u || !BG_u)) return QTX_ERR_ARG;
  Scheme sc;
  if (!make_scheme(prec, n_slices, &sc)) return QTX_ERR_UNSUPPORTED;
  DeviceGuard guard(ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  OrderScope order(ctx, s);
  QTX_TRYS(order.enter());
  const int64_t bb = (int64_t)b * b;
  const int64_t sd = (int64_t)n_b * bb, su = (int64_t)(n_b - 1) * bb;   // per-energy strides
  // workspace: four Y blocks per energy and the converted operands of one product
  const size_t per_e = 4 * align_up((size_t)bb * sizeof(double2)) + split_pair_bytes(b, sc, 1) + 1024;
  const size_t budget = std::max(ws_budget(ctx), per_e + 4096);
  const int ec = (int)std::max<size_t>(1, std::min<size_t>((size_t)n_e, (budget - 4096) / per_e));
  const size_t blk = align_up((size_t)ec * bb * sizeof(double2));
  QTX_TRYS(ensure_ws(ctx, 4 * blk + split_pair_bytes(b, sc, ec) + 4096));
  char* w = (char*)ctx->ws;
  double2* Y[4];
  for (int q = 0; q < 4; ++q) { Y[q] = (double2*)w; w += blk; }
  const SplitBufs sb = carve_split(w, b, sc, ec);
  const double2 one = cmk(1, 0), mone = cmk(-1, 0);
  auto cpt = [](const void* p) { return (const double2*)p; };
  for (int e0 = 0; e0 < n_e; e0 += ec) {
    const int Z = std::min(ec, n_e - e0);
    // C = alpha op(A) op(B) (+ C); A / B: (pointer, per-energy stride; stride 0 = V, shared)
    auto prod = [&](int opA, const double2* A, int64_t sA, int opB, const double2* B, int64_t sB, double2* C,
                    int64_t sC, double2 alpha, bool acc) -> hipError_t {
      GemmDesc d;
      d.M = b; d.N = b; d.K = b;
      d.opA = opA; d.opB = opB;
      d.A = A; d.lda = b; d.sA = sA;
      d.B = B; d.ldb = b; d.sB = sB;
      d.C = C; d.ldc = b; d.sC = sC;
      d.alpha = alpha;
      if (acc) { d.add[0].X = C; d.add[0].ld = b; d.add[0].stride = sC; d.add[0].coef = one; }
      d.batch = Z;
      return run_product(ctx, d, sc, sb, s);
    };
    // per-energy block k of an array with per-energy stride st, offset to this chunk
    auto at = [&](const void* base, int64_t st, int k) { return cpt(base) + e0 * st + (int64_t)k * bb; };
    auto atw = [&](void* base, int64_t st, int k) { return (double2*)base + e0 * st + (int64_t)k * bb; };
    auto vd = [&](int k) { return cpt(V_d) + (int64_t)k * bb; };
    auto vu = [&](int k) { return cpt(V_u) + (int64_t)k * bb; };
    // ---- BT(V P^R)
    for (int i = 0; i < n_b; ++i) {
      double2* C = atw(VPR_d, sd, i);
      QTX_TRY(prod(OP_N, vd(i), 0, OP_N, at(PR_d, sd, i), sd, C, sd, one, false));
      if (i > 0) QTX_TRY(prod(OP_C, vu(i - 1), 0, OP_N, at(PR_u, su, i - 1), su, C, sd, one, true));
      if (i + 1 < n_b) QTX_TRY(prod(OP_N, vu(i), 0, OP_N, at(PR_l, su, i), su, C, sd, one, true));
    }
    for (int i = 0; i + 1 < n_b; ++i) {
      double2* C = atw(VPR_u, su, i);
      QTX_TRY(prod(OP_N, vd(i), 0, OP_N, at(PR_u, su, i), su, C, su, one, false));
      QTX_TRY(prod(OP_N, vu(i), 0, OP_N, at(PR_d, sd, i + 1), sd, C, su, one, true));
      C = atw(VPR_l, su, i);
      QTX_TRY(prod(OP_C, vu(i), 0, OP_N, at(PR_d, sd, i), sd, C, su, one, false));
      QTX_TRY(prod(OP_N, vd(i + 1), 0, OP_N, at(PR_l, su, i), su, C, su, one, true));
    }
    // ---- BT(V P V^H) for P^< and P^>
    for (int r = 0; r < (greater ? 2 : 1); ++r) {
      const void* Pd = r ? PG_d : PL_d;
      const void* Pu = r ? PG_u : PL_u;
      void* Bd = r ? BG_d : BL_d;
      void* Bu = r ? BG_u : BL_u;
      for (int i = 0; i < n_b; ++i) {
        const bool lo = i > 0, hi = i + 1 < n_b, hi2 = i + 2 < n_b;
        double2 *Ym = Y[0], *Y0 = Y[1], *Yp = Y[2], *Yq = Y[3];
        const int64_t sy = bb;
        if (lo) {   // Y_{i,i-1} = V_u[i-1]^H P_{i-1,i-1} - V_ii P_u[i-1]^H
          QTX_TRY(prod(OP_C, vu(i - 1), 0, OP_N, at(Pd, sd, i - 1), sd, Ym, sy, one, false));
          QTX_TRY(prod(OP_N, vd(i), 0, OP_C, at(Pu, su, i - 1), su, Ym, sy, mone, true));
        }
        // Y_ii = V_u[i-1]^H P_u[i-1] + V_ii P_ii - V_u[i] P_u[i]^H
        QTX_TRY(prod(OP_N, vd(i), 0, OP_N, at(Pd, sd, i), sd, Y0, sy, one, false));
        if (lo) QTX_TRY(prod(OP_C, vu(i - 1), 0, OP_N, at(Pu, su, i - 1), su, Y0, sy, one, true));
        if (hi) QTX_TRY(prod(OP_N, vu(i), 0, OP_C, at(Pu, su, i), su, Y0, sy, mone, true));
        if (hi) {   // Y_{i,i+1} = V_ii P_u[i] + V_u[i] P_{i+1,i+1}
          QTX_TRY(prod(OP_N, vd(i), 0, OP_N, at(Pu, su, i), su, Yp, sy, one, false));
          QTX_TRY(prod(OP_N, vu(i), 0, OP_N, at(Pd, sd, i + 1), sd, Yp, sy, one, true));
        }
        if (hi2) QTX_TRY(prod(OP_N, vu(i), 0, OP_N, at(Pu, su, i + 1), su, Yq, sy, one, false));   // Y_{i,i+2}
        // B_ii = Y_{i,i-1} V_u[i-1] + Y_ii V_ii^H + Y_{i,i+1} V_u[i]^H
        double2* C = atw(Bd, sd, i);
        QTX_TRY(prod(OP_N, Y0, sy, OP_C, vd(i), 0, C, sd, one, false));
        if (lo) QTX_TRY(prod(OP_N, Ym, sy, OP_N, vu(i - 1), 0, C, sd, one, true));
        if (hi) QTX_TRY(prod(OP_N, Yp, sy, OP_C, vu(i), 0, C, sd, one, true));
        if (hi) {   // B_{i,i+1} = Y_ii V_u[i] + Y_{i,i+1} V_{i+1,i+1}^H + Y_{i,i+2} V_u[i+1]^H
          C = atw(Bu, su, i);
          QTX_TRY(prod(OP_N, Y0, sy, OP_N, vu(i), 0, C, su, one, false));
          QTX_TRY(prod(OP_N, Yp, sy, OP_C, vd(i + 1), 0, C, su, one, true));
          if (hi2) QTX_TRY(prod(OP_N, Yq, sy, OP_C, vu(i + 1), 0, C, su, one, true));
        }
      }
    }
  }
  return QTX_OK;
}

// ---------------------------------------------------------------- FPX storage codec
namespace {
qtx_status fpx_call(qtx_rgf_ctx ctx, bool encode, int32_t bits, int64_t n, const void* src, void* dst,
                    void* hip_stream) {
  if (!ctx) return QTX_ERR_ARG;
  if (ctx->sticky != QTX_OK) return ctx->sticky;
  if (!fpx_supported(bits) || n < 0) return QTX_ERR_ARG;
  if (n == 0) return QTX_OK;
  if (!src || !dst || ((uintptr_t)src & 7) || ((uintptr_t)dst & 7)) return QTX_ERR_ARG;
  DeviceGuard guard(ctx->device);
  QTX_TRY(launch_fpx(encode, bits, n, src, dst, (hipStream_t)hip_stream));
  return QTX_OK;
}
}  // namespace

qtx_status qtx_fpx_encode(qtx_rgf_ctx ctx, int32_t bits, int64_t n, const double* x, void* out, void* hip_stream) {
  return fpx_call(ctx, true, bits, n, x, out, hip_stream);
}

qtx_status qtx_fpx_decode(qtx_rgf_ctx ctx, int32_t bits, int64_t n, const void* in, double* y, void* hip_stream) {
  return fpx_call(ctx, false, bits, n, in, y, hip_stream);
}

qtx_status qtx_zinv(qtx_rgf_ctx ctx, int32_t n, const void* A, int64_t sA, void* Ainv, int64_t sAinv,
                    int32_t batch, int32_t* status, void* hip_stream) {
  if (!ctx) return QTX_ERR_ARG;
  if (ctx->sticky != QTX_OK) return ctx->sticky;
  if (n < 1 || n > 1024 || batch < 1 || !A || !Ainv) return QTX_ERR_ARG;
  if (sA < (int64_t)n * n || sAinv < (int64_t)n * n) return QTX_ERR_ARG;
  DeviceGuard guard(ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  OrderScope order(ctx, s);
  QTX_TRYS(order.enter());
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
  OrderScope order(ctx, s);
  QTX_TRYS(order.enter());
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

qtx_status qtx_rgf_bond_currents(qtx_rgf_ctx ctx, int32_t b, int32_t n_b, int32_t n_e, const void* H_u,
                                 const void* S_u, const double* energies, const void* GL_u, int64_t sGu, double* J,
                                 void* hip_stream) {
  if (!ctx) return QTX_ERR_ARG;
  if (ctx->sticky != QTX_OK) return ctx->sticky;
  if (b < 1 || n_b < 2 || n_e < 1 || !H_u || !energies || !GL_u || !J || sGu < (int64_t)(n_b - 1) * b * b)
    return QTX_ERR_ARG;
  DeviceGuard guard(ctx->device);
  QTX_TRY(launch_bond_currents(b, n_b, n_e, (const double2*)H_u, (const double2*)S_u, energies,
                               (const double2*)GL_u, sGu, J, (hipStream_t)hip_stream));
  return QTX_OK;
}

}  // extern "C"
