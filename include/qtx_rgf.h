/* qtx_rgf.h -- C ABI of the MI355X (gfx950) selected Green's-function solver.
 *
 * The library solves, independently for every energy E, the selected
 * quadratic system of the paper (Section II-A, Eq. 2, G row of Table I):
 *
 *     M(E) = E*S - H - Sigma^R(E),   G^R = M^-1,
 *     G^< = G^R Sigma^< G^R^H,       G^> = G^R Sigma^> G^R^H,
 *
 * returning only the blocks on the block-tridiagonal (BT) pattern: the
 * diagonal and first off-diagonal blocks of G^R, and the diagonal and upper
 * blocks of G^< / G^> (their lower blocks are -(upper)^H because lesser and
 * greater functions are skew-Hermitian, Section II-A).  The method is block
 * Gaussian elimination (Section IV-A) in its recursive Green's function
 * form; each Schur complement is inverted by Gauss-Jordan elimination with
 * partial pivoting in FP64.  The complex block products can run in FP64 or
 * in lower precision on the matrix cores (Section IV, Section V-A); the
 * inversions and the final accumulations of G^< / G^> stay FP64.
 *
 * Conventions shared by every entry point:
 *  - Complex numbers are complex128: two doubles (re, im), interleaved.
 *  - A b x b block is row-major and contiguous (b*b complex elements).
 *  - Block arrays are contiguous: a per-device array [k][b][b]; a per-energy
 *    array [n_e][k][b][b] (energy-major).
 *  - Unless stated otherwise, array pointers are DEVICE pointers of the
 *    context's device.  The caller allocates and owns every input and output
 *    buffer; the library never keeps a caller pointer after the enqueued work
 *    has completed.
 *  - Calls validate their arguments synchronously, return a qtx_status, and
 *    enqueue work on the given HIP stream (NULL = the default stream).  On an
 *    argument error nothing is enqueued.  Inputs must not change and outputs
 *    must not be read until the stream has passed the enqueued work.
 *  - No exception crosses the ABI.  A context is not thread-safe: use one
 *    host thread per context (several contexts may coexist).
 *  - Calls on one context share its device workspace.  A call on a different
 *    stream than the context's previous call makes its stream wait (on the
 *    device, without blocking the host) for the previous call's work, so calls
 *    on several streams run one after another.  This ordering does not cover
 *    calls made while the caller captures the stream into a graph of its own:
 *    the caller must not let such a graph's launches overlap other calls on
 *    the same context.
 *  - Outputs must not alias inputs.
 */
#ifndef QTX_RGF_H
#define QTX_RGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qtx_rgf_ctx_s* qtx_rgf_ctx;

typedef enum {
  QTX_OK = 0,
  QTX_ERR_ARG = 1,          /* invalid argument (nothing enqueued)                 */
  QTX_ERR_NOMEM = 2,        /* workspace could not be allocated                    */
  QTX_ERR_HIP = 3,          /* a HIP runtime call failed (sticky for the context)  */
  QTX_ERR_UNSUPPORTED = 4,  /* valid request the library does not implement        */
  QTX_ERR_SINGULAR = 5,     /* per energy: an exactly zero pivot in an inversion   */
  QTX_ERR_NONFINITE = 6     /* per energy: NaN or Inf in the result                */
} qtx_status;

/* Arithmetic of the complex block products (Section IV: the ZGEMMs).
 * QTX_FP64     : FP64 matrix cores (reference path).
 * QTX_FP32     : operands rounded to FP32, FP32 matrix cores, FP32 accumulation.
 * QTX_BF16_SPLIT / QTX_FP16_SPLIT : each operand split into n_slices terms of
 *   the 16-bit format after power-of-two scaling per row (left operand) and per
 *   column (right operand); slice products with i + j <= n_slices + 1 on the
 *   matrix cores with FP32 accumulation, recombined in FP64 (Ozaki scheme I,
 *   Section II-D).  n_slices = 2 is the "3-term" split (hi*hi + hi*lo + lo*hi).
 *   Supported: BF16 n_slices 2..5, FP16 n_slices 2..3.
 * QTX_INT8_OZAKI2 : modular emulation on the INT8 matrix cores (Ozaki scheme II,
 *   the paper's emulation in Section V-A), with n_slices = p moduli (2..16,
 *   default 11).  Each row of the left operand and column of the right operand
 *   is scaled by a power of two and rounded to integers of at most kbits bits
 *   (the only rounding of the scheme); the integer products are computed exactly
 *   modulo each of the p odd, pairwise coprime moduli 255, 253, 251, 247, 241,
 *   239, 233, 229, 227, 223, 217, 211, 199, 197, 193, 191 (first p), with INT32
 *   accumulation over all of K, and recombined by the Chinese remainder theorem
 *   in FP64.  kbits is the largest value with 8 K 4^kbits < prod(moduli), and p
 *   is clipped so that kbits <= 47 (qtx_ozaki2_bits); the error of a product is about
 *   K 2^-kbits max|row of A| max|column of B|.  Complex products use four real
 *   products (4M).  K <= 65536.
 * Non-finite operands: in the split and INT8 schemes a row of op(A) (a column of
 *   op(B)) that holds a NaN or an Inf makes that whole row (column) of the product
 *   NaN, the outputs it would spoil in FP64 arithmetic, so the solver's per-energy
 *   QTX_ERR_NONFINITE status is the same in every scheme.
 * Inversions and the G^< / G^> epilogue sums are FP64 in every mode. */
typedef enum {
  QTX_FP64 = 0,
  QTX_FP32 = 1,
  QTX_BF16_SPLIT = 2,
  QTX_FP16_SPLIT = 3,
  QTX_INT8_OZAKI2 = 4
} qtx_prec;

enum {
  QTX_S_IDENTITY = 1u,      /* S = I: S_d/S_u/S_l are ignored                        */
  QTX_SIGMA_DIAG = 2u,      /* SR_d / SL_d / SG_d hold diagonals [n_e][n_b][b]        */
  QTX_WANT_GREATER = 8u,    /* also compute G^> from Sigma^> (SG_*)                   */
  QTX_SPLIT_CHAIN = 16u     /* solve each energy as two half-chains (see below)        */
};

/* One BT problem: one device (H, S) and n_e energies.
 * Inputs (device pointers unless noted):
 *   energies  HOST pointer, [n_e] doubles (real energies).
 *   H_d [n_b][b][b], H_u [n_b-1][b][b] = H_{i,i+1}, H_l [n_b-1][b][b] = H_{i+1,i}.
 *   S_d/S_u/S_l  same layout as H (ignored with QTX_S_IDENTITY).
 *   SR_d [n_e][n_b][b][b]   retarded self-energy, diagonal blocks (required).
 *   SR_u/SR_l [n_e][n_b-1][b][b]  off-diagonal blocks of Sigma^R, or NULL (= 0).
 *   SL_d [n_e][n_b][b][b]   lesser self-energy, diagonal blocks (required).
 *   SL_u [n_e][n_b-1][b][b] = Sigma^<_{i,i+1} for a BT Sigma^<, or NULL
 *              (block-diagonal Sigma^<).  SL_l must be NULL (else
 *              QTX_ERR_UNSUPPORTED): the lower blocks are -(SL_u)^H.
 *   SG_d, SG_u  greater self-energy, same layout (SG_d required with
 *              QTX_WANT_GREATER; SG_u without that flag is QTX_ERR_ARG); SG_l
 *              must be NULL.
 *   Sigma^< and Sigma^> must be skew-Hermitian (as lesser/greater functions
 *   are): the recurrences use that symmetry to evaluate a term and its
 *   conjugate transpose with one product (the cross terms of a BT Sigma^<
 *   cost one more product per forward step and two per backward step).
 *   QTX_SIGMA_DIAG: the diagonal blocks of the self-energies are diagonal matrices
 *   (as the contact and broadening terms of the paper's synthetic devices are): SR_d,
 *   SL_d and SG_d are then [n_e][n_b][b] complex vectors, block i of energy e at
 *   (e n_b + i) b, instead of b x b blocks (b times less HBM).  SR_u / SR_l / SL_u /
 *   SG_u keep their dense layout.  Results equal those of the dense blocks.
 * Outputs (device, caller-allocated, written entirely):
 *   GR_d [n_e][n_b][b][b], GR_u [n_e][n_b-1][b][b] = G^R_{i,i+1},
 *   GR_l [n_e][n_b-1][b][b] = G^R_{i+1,i},
 *   GL_d [n_e][n_b][b][b], GL_u [n_e][n_b-1][b][b] = G^<_{i,i+1},
 *   GG_d, GG_u  same as GL_* for G^> (with QTX_WANT_GREATER, else ignored).
 *   status  [n_e] int32 per-energy qtx_status (QTX_OK, QTX_ERR_SINGULAR or
 *           QTX_ERR_NONFINITE), or NULL.  An energy that fails has every
 *           output block filled with NaN; other energies are unaffected.
 *   out_bits  64 (or 0): every output is complex128.  16, 24, .., 56: the
 *           off-diagonal outputs GR_u, GR_l, GL_u (and GG_u) are stored in the FPX
 *           format of that width (Section V-A; see qtx_fpx_encode) -- each complex
 *           element as two FPX codes (re, im), block i of energy e at byte
 *           (e (n_b - 1) + i) b^2 out_bits / 4 -- encoded on the GPU from the FP64
 *           result of each backward step (the recurrences themselves stay FP64; the
 *           diagonal outputs GR_d, GL_d, GG_d hold recurrence state and stay
 *           complex128).  A failed energy's FPX blocks hold the FPX NaN code.  With
 *           out_bits = 32 the off-diagonal outputs take half the HBM.  Not available
 *           with QTX_SPLIT_CHAIN (QTX_ERR_UNSUPPORTED).
 *   partitions  P >= 2: the spatially parallel selected solve of each energy (the
 *           partitioned selected inversion the paper cites for long devices).  The
 *           chain is cut by P - 1 separator blocks into P partitions with interiors of
 *           equal length (to within one block).  Every partition eliminates its
 *           interior top-down at the same time (the forward recurrence, plus the fill-in
 *           blocks that couple the interior to the partition's upper separator, for M
 *           and for the right-hand sides), which leaves a block tridiagonal system over
 *           the separators (reduced blocks, couplings and right-hand sides); its solve
 *           gives G^R, G^<, G^> at the separators and each separator's left-connected
 *           functions; then every partition runs the one-chain forward recurrence again
 *           from those of its upper separator, and the backward recurrence from its
 *           lower separator's G.  The sequential step count per energy is about
 *           3 n_b / P + 2 P instead of 2 n_b - 1, with P times the independent products
 *           per step: it lowers the latency of solves with few energies and long
 *           chains.  The separator system comes from fill-in chains over interiors cut
 *           off from the contacts (whose partial inverses reach 1 / broadening), so it
 *           is always built and solved in FP64; the outputs come from the one-chain
 *           recurrences with exact boundary functions (in the problem's schemes) and
 *           keep the one-chain accuracy to within the separator system's rounding.
 *           Requires n_b >= 2 P - 1 (every interior at least one block) and P <= 64;
 *           not with QTX_SPLIT_CHAIN (QTX_ERR_ARG) or FPX outputs
 *           (QTX_ERR_UNSUPPORTED).  Energies of problems with equal (n_b, b, P) and
 *           schemes share launches.
 * Precision per chain: the products that build x_i and G^R (forward Schur
 * complements, backward G^R blocks) use (prec, n_slices); the products of the
 * lesser/greater recurrences use (prec_lesser, n_slices_lesser).  The lesser
 * chain is the more sensitive one, as the paper chooses slice counts per
 * motif (Section V-B, Table IV).
 * QTX_SPLIT_CHAIN (spatially parallel solve of one energy; Section II-A solves
 *   Eq. 2 for the selected blocks only, and the work it cites on parallel quadratic
 *   selected inversion splits the BT chain): each energy with n_b >= 3 runs as two
 *   half-chains in the same launches, a top half over blocks 0 .. c-1 and a bottom
 *   half that eliminates from block n_b-1 upwards, c = (n_b - 1) / 2.  The bottom
 *   half's last step, at the separator block c, also takes the top half's coupling
 *   terms, so its inverse is G^R_cc and its lesser block G^<_cc; both halves then
 *   run the backward recurrence outwards from c.  The sequential step count per
 *   energy drops from 2 n_b - 1 to about n_b + 1 at the same operation count: it
 *   lowers the latency of a solve with few energies and changes nothing for a
 *   large batch, which already fills the GPU.  Results agree with the unsplit
 *   solve to rounding.  With a BT Sigma^< / Sigma^> the bottom half reads the
 *   blocks -(SL_u)^H (copied by the library into a context buffer of its own,
 *   (n_b - 1 - c) blocks per energy and right-hand side).  The workspace per
 *   energy doubles (qtx_rgf_footprint).  n_b <= 2 ignores the flag.
 * Limits: 1 <= b <= 1024, n_b >= 1, n_e >= 1. */
typedef struct {
  int32_t n_b, b, n_e;
  int32_t prec;            /* qtx_prec of the retarded-chain products           */
  int32_t n_slices;        /* split modes: slices per operand, 0 = default (2)  */
  int32_t prec_lesser;     /* qtx_prec of the lesser/greater-chain products,    */
  int32_t n_slices_lesser; /*   -1 = same as prec / n_slices                    */
  uint32_t flags;          /* QTX_S_IDENTITY | QTX_WANT_GREATER | QTX_SPLIT_CHAIN */
  const double* energies;  /* host                                              */
  const void *H_d, *H_u, *H_l;
  const void *S_d, *S_u, *S_l;
  const void *SR_d, *SR_u, *SR_l;
  const void *SL_d, *SL_u, *SL_l;
  const void *SG_d, *SG_u, *SG_l;
  void *GR_d, *GR_u, *GR_l;
  void *GL_d, *GL_u;
  void *GG_d, *GG_u;
  int32_t* status;
  int32_t out_bits;        /* 64 / 0: complex128 outputs; 16..56: FPX off-diagonal outputs */
  int32_t partitions;      /* 0 / 1: one chain per energy; P >= 2: P-way partitioned solve */
} qtx_rgf_problem;

/* Create a context on HIP device `device`.  workspace_bytes caps the device
 * workspace the context may hold (0 = automatic: up to 1/4 of the device's
 * free memory at the first solve); energies are processed in chunks that fit.
 * tune_cache_path: optional text file of autotuner choices (may be NULL): read
 * here when it exists and was written for the same device kind, rewritten by
 * qtx_rgf_tune.
 * Returns QTX_ERR_ARG for a NULL `out` or an invalid device. */
qtx_status qtx_rgf_create(qtx_rgf_ctx* out, int device, size_t workspace_bytes,
                          const char* tune_cache_path);

/* Solve n_probs problems (Section II-A, Eq. 2), enqueued on hip_stream
 * (a hipStream_t, NULL = default stream).  Problems may differ in n_b, b,
 * n_e and precision.  Validation is synchronous (QTX_ERR_ARG /
 * QTX_ERR_UNSUPPORTED / QTX_ERR_NOMEM with nothing enqueued).  The per-energy
 * numerical status lands in each problem's `status` array.
 * All energies of all problems that share b and the precision schemes are
 * solved together: one launch per recurrence step covers every such energy
 * (energies are independent, Section II-A); problems of other block sizes run
 * concurrently on internal streams that join back into hip_stream.  The call
 * may wait for its own previous table upload (host pointers in the problem
 * structs are read during the call only). */
qtx_status qtx_rgf_solve(qtx_rgf_ctx ctx, const qtx_rgf_problem* probs, int32_t n_probs,
                         void* hip_stream);

/* Context options (qtx_rgf_set_option):
 *   QTX_OPT_GRAPH  value != 0: qtx_rgf_solve captures its whole launch sequence
 *                  (all batches, on parallel streams for different block sizes)
 *                  into a hipGraph on the first call with a given set of problems
 *                  and replays it with one graph launch on later identical calls
 *                  (same problem structs, energies and workspace).  Needs a
 *                  non-NULL stream; with the NULL stream the solve runs eagerly.
 * Counters (qtx_rgf_get_stat): graph launches, graph captures, workspace bytes,
 * autotuner records held.
 *   QTX_OPT_RESERVE_WORKSPACE  value = bytes: allocate the device workspace now
 *                  (grows only; for callers that must claim memory before other
 *                  allocators do).  Returns QTX_ERR_NOMEM if it cannot.
 *   QTX_OPT_INT8_TILE_VARIANT  value = -1 (default): INT8 products take the tile
 *                  variant the autotuner recorded for their shape, else a default
 *                  from the shape (64 x 64 tiles three per CU when K >= 256 and
 *                  there are >= 512 such tiles, else 64 x 64 tiles two per CU);
 *                  value = 0 .. count-1: every INT8 product uses that variant.
 *                  All variants give bitwise the same results.
 *   QTX_OPT_OVERLAP  value != 0: during each forward inversion, the two
 *                  lesser-recurrence products that do not need the new inverse run
 *                  on an internal side stream (one per block-size lane, default
 *                  priority) that forks from and joins back into the solve's
 *                  stream; value = 0 (default): everything runs on the solve's
 *                  stream.  The results are bitwise the same either way.  Not
 *                  available together with QTX_OPT_GRAPH: turning either option on
 *                  while the other is on returns QTX_ERR_UNSUPPORTED (the side
 *                  stream is never captured).  Off by default: at 256 energies of b = 416 the
 *                  persistent product kernels occupy every CU, so the overlap only
 *                  adds contention (measured 2% slower).
 *   QTX_OPT_LANE_SPLIT  value = k in 1..8 (default 1): the energies of each group of
 *                  one block size and scheme are split (alternately) into k parts
 *                  that run as independent batches on k internal streams (default
 *                  priority) forking from and joining back into the solve's stream,
 *                  so that one part's inversions and operand conversions overlap the
 *                  other parts' products.  Results are bitwise the same for any k;
 *                  the workspace is the same in total. */
enum { QTX_OPT_GRAPH = 1, QTX_OPT_RESERVE_WORKSPACE = 2, QTX_OPT_INT8_TILE_VARIANT = 3, QTX_OPT_OVERLAP = 4,
       QTX_OPT_LANE_SPLIT = 5 };
enum { QTX_STAT_GRAPH_LAUNCHES = 1, QTX_STAT_GRAPH_CAPTURES = 2, QTX_STAT_WORKSPACE_BYTES = 3,
       QTX_STAT_TUNE_RECORDS = 4 };
qtx_status qtx_rgf_set_option(qtx_rgf_ctx ctx, int option, int64_t value);
qtx_status qtx_rgf_get_stat(qtx_rgf_ctx ctx, int stat, int64_t* value);

/* Autotuner.  Times every tile variant of the product kernel that the scheme
 * (prec, n_slices) uses on synthetic complex b x b x b products over `batch`
 * entries (deterministic pseudo-random operands in [-1, 1)) on hip_stream: two
 * warm-up products of every variant, then two rounds of 3 timed products per
 * variant in opposite orders (a variant's time is its faster round), and records the
 * fastest for the shape (b, b, b),
 * the batch class ceil(log2(batch)) (classes 0..9) and the scheme (modulus count or
 * slice count).  Later products of that shape and scheme (in qtx_rgf_solve and
 * qtx_zgemm) take the recorded variant, from the record of the nearest batch class;
 * cached hipGraphs are dropped.  The table is written to the context's
 * tune_cache_path when one was given (QTX_ERR_ARG if that write fails; the record is
 * kept).  Variants: the INT8 scheme has 14 (tiles of 32 x 64 to 128 x 128 with one or
 * two 32 x 32 blocks per wave, one to six workgroups per CU, LDS rings of two to four
 * stages, each either in persistent workgroups or one tile per workgroup); FP64, FP32
 * and the split schemes have 2 (0: 32 x 32 output tiles, 1: 64 x 64; without a record
 * they take 32 x 32 where a 64 x 64 tiling pads C by more than 8% or gives fewer than
 * 4096 tiles).  All variants of a scheme give bitwise the same products.
 *   out_variant  chosen variant (nullable)
 *   out_ms       ms per product (operand conversion included) of each variant,
 *                up to max_variants entries (nullable when max_variants = 0)
 *   out_count    number of variants (nullable)
 * Allocates and frees three b*b*batch complex128 buffers and synchronizes
 * hip_stream.  b in 1..1024, batch >= 1; QTX_ERR_NOMEM if the buffers do not fit. */
qtx_status qtx_rgf_tune(qtx_rgf_ctx ctx, int32_t b, int32_t prec, int32_t n_slices, int32_t batch,
                        void* hip_stream, int32_t* out_variant, double* out_ms, int32_t max_variants,
                        int32_t* out_count);

/* Free the context and its workspace (synchronizes the device first). */
qtx_status qtx_rgf_destroy(qtx_rgf_ctx ctx);

/* Device workspace bytes one energy of problem p needs; used for admission by
 * HBM footprint.  Returns 0 for an invalid problem. */
size_t qtx_rgf_footprint(const qtx_rgf_problem* p);

/* Human-readable name of a status code (static string). */
const char* qtx_status_str(qtx_status s);

/* Parameters of QTX_INT8_OZAKI2 asked for p moduli at contraction length K
 * (host only, no device work).  The scheme uses the first p_used <= p moduli
 * (p is clipped where more moduli would need operands wider than 47 bits) and
 * operand integers of kbits bits, the largest width with 8 K 4^kbits < M, M the
 * product of the moduli used.  Writes the moduli to moduli[0..p_used-1] (host
 * array of at least p entries), p_used and kbits; each pointer may be NULL.
 * Returns QTX_ERR_UNSUPPORTED if (p, K) is outside the scheme's range
 * (p in 2..16, K in 1..65536, kbits >= 1). */
qtx_status qtx_ozaki2_bits(int32_t p, int32_t K, int32_t* moduli, int32_t* p_used, int32_t* kbits);

/* Screened Coulomb (W) system, the W row of Table I: per energy
 *     M(E) = I - V P^R(E),   B^<>(E) = V P^<>(E) V^H,   W^<> = M^-1 B^<> M^-H,
 * with V the Coulomb matrix (Hermitian, BT, energy independent) and P the
 * polarization (BT).  The products of BT matrices are wider than BT; the system
 * solved is the BT one the paper states (Section II-A: only the BT entries are
 * needed), so this call returns the BT blocks of V P^R and of V P^<> V^H.  The
 * W system is then qtx_rgf_solve on energies 1, S = I, H = 0 (zero blocks),
 * Sigma^R := BT(V P^R) (SR_d/u/l = VPR_d/u/l) and Sigma^< := BT(V P^< V^H)
 * (SL_d/u = BL_d/u), Sigma^> likewise: its G^R outputs are the BT blocks of
 * M^-1 and its G^<> outputs those of W^<>.
 * Inputs (device):
 *   V_d [n_b][b][b], V_u [n_b-1][b][b] = V_{i,i+1}; V_{i+1,i} = V_u^H is implied.
 *   PR_d [n_e][n_b][b][b], PR_u / PR_l [n_e][n_b-1][b][b]  P^R blocks.
 *   PL_d, PL_u  P^< diagonal and upper blocks (P^< skew-Hermitian: the lower
 *               blocks are -(PL_u)^H).  PG_d, PG_u  P^> likewise, or both NULL.
 * Outputs (device, caller-allocated, written entirely):
 *   VPR_d [n_e][n_b][b][b], VPR_u / VPR_l [n_e][n_b-1][b][b]: BT blocks of V P^R.
 *   BL_d, BL_u (and BG_d, BG_u with PG_*): diagonal and upper BT blocks of
 *   V P^<> V^H (skew-Hermitian: lower = -(upper)^H).
 * prec / n_slices: scheme of the block products (qtx_prec), as in qtx_zgemm.
 * Energies are processed in chunks that fit the context's workspace budget
 * (four blocks per energy plus converted operands).  Limits: n_b >= 1,
 * 1 <= b <= 1024, n_e >= 1; u/l pointers may be NULL when n_b = 1. */
qtx_status qtx_w_assemble(qtx_rgf_ctx ctx, int32_t n_b, int32_t b, int32_t n_e, int32_t prec, int32_t n_slices,
                          const void* V_d, const void* V_u, const void* PR_d, const void* PR_u, const void* PR_l,
                          const void* PL_d, const void* PL_u, const void* PG_d, const void* PG_u,
                          void* VPR_d, void* VPR_u, void* VPR_l, void* BL_d, void* BL_u, void* BG_d, void* BG_u,
                          void* hip_stream);

/* FPX storage formats (Section V-A): X-bit byte-aligned floating point, X in
 * {16, 24, 32, 40, 48, 56}, with 1 sign bit, FP32's 8-bit exponent and bias (127)
 * and X - 9 significand bits; FP64 values are rounded to nearest, ties to even
 * (IEEE-754), with FP32's range: subnormals below 2^-126, magnitudes that round to
 * 2^128 or more become infinite, NaN stays NaN (sign kept, payload not).  FPX32 is
 * IEEE FP32 bitwise; FPX16 has the bfloat16 layout.  Element i occupies bytes
 * [i X/8, (i+1) X/8) of the byte stream, little-endian.
 * qtx_fpx_encode: x [n] doubles (device) -> out [n X/8] bytes (device).
 * qtx_fpx_decode: in [n X/8] bytes (device) -> y [n] doubles (device), exact.
 * A complex128 array of k elements is n = 2k doubles.  Both pointers must be
 * 8-byte aligned and must not overlap; n = 0 does nothing.  QTX_ERR_ARG for an
 * unsupported bits value, n < 0, NULL or misaligned pointers (nothing enqueued). */
qtx_status qtx_fpx_encode(qtx_rgf_ctx ctx, int32_t bits, int64_t n, const double* x, void* out, void* hip_stream);
qtx_status qtx_fpx_decode(qtx_rgf_ctx ctx, int32_t bits, int64_t n, const void* in, double* y, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Kernel-level entry points (the building blocks of qtx_rgf_solve), exposed
 * so each can be checked in isolation.
 * ------------------------------------------------------------------------ */

/* Batched complex GEMM  C_z = alpha * op(A_z) op(B_z) + beta * C_z,  z < batch,
 * the complex block product of Section IV.  op: 'N' (as is) or 'C' (conjugate
 * transpose).  op(A) is M x K, op(B) is K x N, C is M x N; all row-major with
 * leading dimensions lda/ldb/ldc (in complex elements) and batch strides
 * sA/sB/sC (in complex elements; 0 = the same matrix for every z).
 * alpha, beta: complex (re, im) given as two doubles each.  prec: qtx_prec,
 * n_slices as in qtx_rgf_problem.  beta = 0 never reads C.
 * Limits: M, N, K >= 0, batch >= 1. */
qtx_status qtx_zgemm(qtx_rgf_ctx ctx, char opA, char opB, int32_t M, int32_t N, int32_t K,
                     double alpha_re, double alpha_im,
                     const void* A, int64_t lda, int64_t sA,
                     const void* B, int64_t ldb, int64_t sB,
                     double beta_re, double beta_im,
                     void* C, int64_t ldc, int64_t sC,
                     int32_t batch, int32_t prec, int32_t n_slices, void* hip_stream);

/* qtx_zgemm for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same product,
 * arguments, kernels and results as qtx_zgemm (bitwise), but the split and INT8 schemes
 * convert their operands into a fixed device buffer of QTX_NOALLOC_SCRATCH_BYTES
 * (64 MiB) per GPU instead of the context's workspace.  That buffer exists once per GPU
 * from the library's load until the process ends; the call itself allocates nothing
 * (no hipMalloc, hipFree or allocating library routine, no timer events).  Limit: the
 * converted operands must fit, about batch * 2 p (M + N) K bytes for p INT8 moduli and
 * batch * 4 n_slices (M + N) K for the split schemes (an operand with batch stride 0
 * counts once); larger calls return QTX_ERR_ARG with nothing enqueued.  FP64 / FP32
 * products use no scratch.  Every call on one GPU uses the same buffer: two calls whose
 * work overlaps on the device (different streams, or different contexts on that GPU)
 * race and give wrong results; calls on one stream are ordered.  Not ordered against
 * the context's other calls (it does not use the context's workspace). */
#define QTX_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
qtx_status qtx_zgemm_noalloc(qtx_rgf_ctx ctx, char opA, char opB, int32_t M, int32_t N, int32_t K,
                             double alpha_re, double alpha_im,
                             const void* A, int64_t lda, int64_t sA,
                             const void* B, int64_t ldb, int64_t sB,
                             double beta_re, double beta_im,
                             void* C, int64_t ldc, int64_t sC,
                             int32_t batch, int32_t prec, int32_t n_slices, void* hip_stream);

/* Batched inverse of n x n complex matrices by Gauss-Jordan elimination with
 * partial pivoting (pivot = largest |re|+|im| among the rows not yet used,
 * lowest row on ties), FP64 throughout.  A: [batch] matrices with stride sA
 * (complex elements), row-major, leading dimension n; Ainv: output, same
 * layout with stride sAinv.  A is not modified.  status: device [batch] int32
 * (QTX_OK or QTX_ERR_SINGULAR; a singular matrix's inverse is NaN-filled), or
 * NULL.  Limits: 1 <= n <= 1024. */
qtx_status qtx_zinv(qtx_rgf_ctx ctx, int32_t n, const void* A, int64_t sA,
                    void* Ainv, int64_t sAinv, int32_t batch, int32_t* status, void* hip_stream);

/* Transport observables per energy from solver outputs (Section II-B uses the
 * current as the accuracy criterion).  With A_11 = i(G^R_11 - G^R_11^H):
 *   T_L[e] = Tr[Gamma_L A_11] - Tr[Gamma_L G^R_11 Gamma_L G^R_11^H]
 *   j_L[e] = Re(i Tr[Gamma_L G^<_11]) + f_L[e] Tr[Gamma_L A_11]
 * GR_11 / GL_11: [n_e] blocks with batch stride sG (complex elements), e.g.
 * the solver's GR_d / GL_d with sG = n_b*b*b.  gamma_L: b x b device matrix
 * (shared by all energies).  f_L: device [n_e] doubles.  T_L, j_L: device
 * [n_e] double outputs.  Uses per-context scratch. */
qtx_status qtx_rgf_observables(qtx_rgf_ctx ctx, int32_t b, int32_t n_e,
                               const void* GR_11, const void* GL_11, int64_t sG,
                               const void* gamma_L, const double* f_L,
                               double* T_L, double* j_L, void* hip_stream);

/* Bond currents from solver outputs (Section II-B: the current, and its conservation
 * along the device, is the accuracy criterion).  For energy e and bond i (blocks i and
 * i + 1, i < n_b - 1):
 *   J[e][i] = 2 Re Tr[(H_{i,i+1} - E_e S_{i,i+1}) G^<_{i+1,i}],  G^<_{i+1,i} = -(G^<_{i,i+1})^H,
 * the particle current from block i to block i + 1 (in units where the contact current
 * j_L of qtx_rgf_observables is the same quantity at the left contact: with no
 * broadening inside the device, J[e][i] = j_L[e] = -j_R[e] for every bond).
 * H_u: [n_b-1][b][b] device couplings H_{i,i+1}; S_u: the same for S, or NULL (S = I,
 * whose off-diagonal blocks are zero).  energies: device [n_e] doubles.  GL_u: the
 * solver's G^<_{i,i+1} blocks, energy e at GL_u + e * sGu (complex elements;
 * sGu >= (n_b-1) b^2).  J: device [n_e][n_b-1] double output.  Limits: b >= 1,
 * n_b >= 2, n_e >= 1.  Uses no workspace. */
qtx_status qtx_rgf_bond_currents(qtx_rgf_ctx ctx, int32_t b, int32_t n_b, int32_t n_e, const void* H_u,
                                 const void* S_u, const double* energies, const void* GL_u, int64_t sGu, double* J,
                                 void* hip_stream);

/* ---------------------------------------------------------------------------
 * Per-launch timing of the library's own kernels (roofline measurement).
 * While enabled, every launch of the families below is bracketed by HIP events
 * recorded on the stream it runs on.  qtx_rgf_profile_read waits for those
 * events, returns the summed duration (ms), the launch count and the
 * algorithmic work of the launches since the previous read of that family, and
 * resets them.  Families (qtx_rgf_solve and qtx_zgemm launches):
 *   QTX_KERNEL_GEMM    : the matrix-core kernel of one complex block product
 *                        (M x N x K, batched); work = the real multiply-adds x 2
 *                        its scheme issues on the matrix cores, in that scheme's
 *                        own arithmetic: 4 real products (FP64, FP32), 4 per
 *                        kept slice pair (BF16/FP16 split), 4 per modulus (INT8);
 *   QTX_KERNEL_INV     : one batched inversion of a Schur complement (all panels,
 *                        trailing updates and the final gather), 8 b^3 flop per
 *                        energy;
 *   QTX_KERNEL_CONVERT : the operand conversion passes of a split / INT8 product
 *                        (both operands); work = bytes read (16 per complex
 *                        element) plus digit / residue bytes written.
 * Any NULL output pointer is skipped. */
enum { QTX_KERNEL_GEMM = 0, QTX_KERNEL_INV = 1, QTX_KERNEL_CONVERT = 2 };
qtx_status qtx_rgf_profile(qtx_rgf_ctx ctx, int enable);
qtx_status qtx_rgf_profile_read(qtx_rgf_ctx ctx, int family, double* total_ms, int64_t* launches,
                                double* flops);

#ifdef __cplusplus
}
#endif

#endif /* QTX_RGF_H */
