/*
 * qsketch: one-pass randomized quaternion low-rank approximation on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: C. Chang and Y. Yang, "Randomized large-scale quaternion matrix
 * approximation: practical rangefinders and one-pass algorithm",
 * arXiv:2404.14783.  For A in Q^{m x n} and sketch sizes r <= k <= l <=
 * min(m, n) (the paper's s is k here; Section 4.1), two independent random
 * test matrices Omega (n x k) and Psi (l x m) give the sketches
 *     Y = A Omega  (m x k)   and   W = Psi A  (l x n)        (Section 4.1)
 * formed by linear updates of column blocks, so that A is read once and never
 * stored (Section 4, opening; Section 5.3).  A rangefinder maps Y to Q (the
 * paper's H, Algs. 1 and 3) and the core solve gives X = (Psi Q)^dagger W
 * (Alg. 4, through Alg. 2), so that A ~ Q X.
 *
 * Conventions for every entry point:
 *  - A quaternion matrix M = M_w + M_x i + M_y j + M_z k is passed as four
 *    real planes {w, x, y, z}, each column-major with a leading dimension:
 *    element (r, c) of plane p is planes[p][r + c * ld].
 *  - Matrix pointers are HIP device pointers on the device that was current
 *    when qsketch_init ran.  Sizes and scalars are host values.
 *  - Calls are stream-ordered on the stream given to qsketch_init and return
 *    before the GPU has finished, except where stated.  The caller keeps every
 *    buffer alive until the stream has passed the call.
 *  - The caller owns its inputs and outputs; the context owns the sketches and
 *    all workspace, allocated in qsketch_init (update and finalize allocate
 *    nothing; qsketch_update_block, qsketch_project and qsketch_truncate grow
 *    work buffers of their own on first use).
 *  - On QSK_E_ARG nothing has happened.  A HIP failure returns QSK_E_HIP and
 *    poisons the context: every later call except qsketch_destroy,
 *    qsketch_last_error and qsketch_strerror returns QSK_E_STATE.
 *  - One context belongs to one stream; calls on one context must not
 *    overlap (the API is not re-entrant per context).
 */
#ifndef QSKETCH_H
#define QSKETCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qsk_ctx qsk_ctx;

typedef enum {
  QSK_OK = 0,
  QSK_E_ARG = 1,          /* invalid argument; no side effects */
  QSK_E_STATE = 2,        /* context poisoned or destroyed */
  QSK_E_NOMEM = 3,        /* device allocation failed: in qsketch_init, or for a work
                             buffer that qsketch_update_block, qsketch_project or
                             qsketch_truncate grows (the context stays usable) */
  QSK_E_HIP = 4,          /* a HIP runtime call failed; context poisoned */
  QSK_E_NUMERIC = 5,      /* no Q/X could be formed (e.g. Y == 0) */
  QSK_E_UNSUPPORTED = 6   /* valid but not implemented combination */
} qsk_status;

/* Element formats.  input_dtype: the planes passed to qsketch_update.
   sketch_dtype: the operands of the sketch products:
     QSK_F64  FP64 data and test matrices, FP64 accumulation, FP64 Y/W;
     QSK_F32  FP32 data, test matrices rounded to FP32, FP32 matrix-core
              products with FP32 accumulation, FP32 Y/W;
     QSK_BF16 data split into split_terms bf16 terms (hi, mid, lo: each term
              rounds what the previous ones left), test matrices rounded to
              bf16 once from their FP64 value, FP32 accumulation, FP32 Y/W;
     QSK_FP8_E4M3 data quantised to OCP fp8 e4m3 (round to nearest even)
              with the smallest power-of-two scale per 32 x 32 tile of each
              plane of the update block that keeps |x / scale| <= 448;
              split_terms = 2 adds the exact FP32 residual x - q * scale as a
              correction term (carried as two bf16 terms, i.e. to 2^-16 of the
              residual); test matrices rounded to e4m3 once from their FP64
              value; FP32 accumulation, FP32 Y/W.  The dequantised fp8 values
              are exact in bf16 and all terms run on the bf16 matrix-core
              product.  Update blocks whose planes need byte offsets of 2^32
              or more return QSK_E_UNSUPPORTED in this format;
     QSK_FP8_MFMA the same tile scales, the data carried as split_terms
              (1..4) e4m3 terms: term t quantises (RNE) what the earlier terms
              left at scale (tile scale) 16^-t, so the operand is
              sum_t q_t scale 16^-t (after term 0 the rest is at most 16 scale
              per value, so no later term saturates; four terms carry about as
              many bits as two bf16 terms near the tile maximum).  Every term
              runs on the fp8 matrix cores (e4m3 x e4m3 with the tile
              exponent as the block scale, FP32 accumulation); the block is
              quantised once per update into bytes (2 split_terms bytes per
              value and plane); test matrices rounded to e4m3.  Update blocks
              whose quantised planes need 2^32 bytes or more return
              QSK_E_UNSUPPORTED.  Not for batches. */
typedef enum { QSK_F64 = 0, QSK_F32 = 1, QSK_BF16 = 2, QSK_FP8_E4M3 = 3, QSK_FP8_MFMA = 4 } qsk_dtype;

/* Test-matrix distributions: quaternion standard Gaussian, all four
   components i.i.d. N(0,1) (Def. 4.1); quaternion Rademacher, components
   i.i.d. +-1 (a centred unit-variance sub-Gaussian matrix, Def. 4.2). */
typedef enum { QSK_GAUSSIAN = 0, QSK_RADEMACHER = 1 } qsk_embedding;

/* Rangefinders (Section 3): pseudo-QR with correction steps (Alg. 1,
   non-orthonormal, well conditioned) and pseudo-SVD (Alg. 3, orthonormal),
   whose bad part is repaired through H_b diag(f) and a second SVD
   (QSK_PSEUDO_SVD) or through Alg. 3's Gram-Schmidt branch
   (QSK_PSEUDO_SVD_GS: the bad columns taken in turn, each orthogonalised
   against those already taken and their J-partners and kept when more than
   1e-8 of its norm remains).  Batches take the first two only. */
typedef enum { QSK_PSEUDO_QR = 0, QSK_PSEUDO_SVD = 1, QSK_PSEUDO_SVD_GS = 2 } qsk_rangefinder;

/* Report flags (numeric events are flags, not errors). */
enum {
  QSK_FLAG_CHOL_FALLBACK = 1,   /* Gram Cholesky broke down: shifted 3-pass CholeskyQR used */
  QSK_FLAG_RANK_DEFICIENT = 2,  /* Q*Q (or (Psi Q)*(Psi Q)) singular: corrections skipped */
  QSK_FLAG_NONFINITE = 4,       /* a non-finite value met in the sketches */
  QSK_FLAG_BAD_PAIRS = 8        /* pseudo-SVD repaired t_bad > 0 singular pairs */
};

typedef struct {
  int64_t m, n;            /* A in Q^{m x n}; 1 <= m, n < 2^31 */
  int32_t k, l;            /* sketch sizes, 1 <= k <= l <= min(m, n), k <= 256, l <= 1024 */
  uint64_t seed;           /* Philox4x32-10 key (seed mod 2^32, seed >> 32) */
  int32_t embedding;       /* qsk_embedding */
  int32_t input_dtype;     /* QSK_F64 | QSK_F32 | QSK_BF16 */
  int32_t sketch_dtype;    /* qsk_dtype, see above */
  int32_t pure;            /* 1: A has no real part; planes[0] is ignored (may be NULL) */
  int32_t split_terms;     /* BF16: 1..3; FP8: 1 or 2 (2 = add FP32 residual term);
                              FP8_MFMA: 1..4 e4m3 terms */
  int32_t n_correction;    /* pseudo-QR correction steps, 0..8 (the paper's experiments use 3) */
  int32_t n_power;         /* power iterates per correction step for eps (paper: 2-3) */
  int64_t max_block_cols;  /* largest ncols of one update; 0 means n */
  int32_t y_only;          /* 1: keep Y only (the two-pass variant): W is neither stored nor
                              updated, qsketch_finalize runs with X == NULL, and
                              qsketch_project forms X in a second pass over A.  Not for batches. */
  int32_t embedding_round; /* QSK_F64 sketches only: the test matrices take the values of this
                              format (QSK_F32, QSK_BF16 or QSK_FP8_E4M3: the FP64 draw rounded
                              once, as a sketch of that format uses them); QSK_F64 (0, the
                              default) keeps them unrounded.  An FP64 sketch with the test
                              matrices of a low-precision one is the reference of the
                              equal-error comparison (a rounded Gaussian matrix is still an
                              entry-independent sub-Gaussian test matrix, Def. 4.2).  Must be 0
                              for other sketch formats. */
  int32_t coalesce_cols;   /* 0 (default): every qsketch_update runs the sketch products on its
                              block.  c > 0: qsketch_update copies a block narrower than c that
                              continues the pending columns (col0 = first pending column +
                              pending count) into a context buffer of c columns and runs the
                              products once the buffer is full, or when another call needs the
                              sketches (finalize, sketches, scale, a general or sub-block
                              update, a non-contiguous or wide block).  The sketches are linear
                              in A, so the result is the same up to rounding order; the buffer
                              (planes x m x c elements of input_dtype) trades memory for
                              fewer read-modify-writes of Y.  In the FP8 format the per-tile
                              scales are those of the gathered block.  Not for batches. */
} qsk_config;

typedef struct {
  double kappa;            /* kappa(Q) = sigma_max / sigma_min of the returned Q */
  double kappa_initial;    /* pseudo-QR: kappa of the raw factor before correction (inf if singular) */
  double eps[8];           /* pseudo-QR: eps of each correction step */
  int32_t n_eps;
  int32_t t_bad;           /* pseudo-SVD: number of repaired pairs */
  int32_t flags;           /* QSK_FLAG_* */
  int32_t passes;          /* CholeskyQR passes used on Y */
  int64_t columns_seen;    /* columns passed to the update calls (or set on restore) */
  double orth_defect;      /* ||Q*Q - I||_max (pseudo-SVD; 0 for pseudo-QR) */
} qsk_report;

/* Fill cfg with defaults: k, l, m, n zero (must be set), seed 0, Gaussian,
   FP64 in and out, split_terms 1, n_correction 3, n_power 3. */
void qsketch_config_default(qsk_config *cfg);

/* Validate cfg, allocate Y, W (zeroed) and all workspace on the current
   device, bind the context to hip_stream (a hipStream_t; NULL = default
   stream).  Synchronous.  Returns QSK_E_ARG for an invalid cfg,
   QSK_E_NOMEM if device memory is short. */
qsk_status qsketch_init(const qsk_config *cfg, void *hip_stream, qsk_ctx **out);

/* Linear update A[:, col0 : col0 + ncols) += H (Section 4, opening), where
   H is the m x ncols quaternion block in planes[0..3] (input_dtype, column-
   major, leading dimension ld >= m):
       Y += H Omega[col0 : col0 + ncols, :],   W[:, col0 : col0 + ncols] += Psi H.
   Overlapping or repeated column ranges are legal (the update is linear).
   Requires 0 <= col0, 1 <= ncols <= max_block_cols, col0 + ncols <= n. */
qsk_status qsketch_update(qsk_ctx *ctx, int64_t col0, int64_t ncols,
                          const void *const planes[4], int64_t ld);

/* A sequence of column-block updates A[:, col0[i] : col0[i] + ncols[i]) += H_i,
   i = 0 .. count - 1, in order, with the same result as count calls of
   qsketch_update (Section 4 opening and Section 5.3: data streamed through
   linear updates).  The first call with a given argument list (the same
   count, offsets, sizes, plane pointers and leading dimensions, starting
   from the same pending-column state when coalescing) captures the whole
   sequence into one HIP graph on a stream of the context; later calls with
   the same list replay it with one launch.  planes holds 4 * count device
   pointers (planes[4 i + p]), the other arrays count host values.  Every
   block is checked before anything runs (QSK_E_ARG: nothing happened).
   Stream-ordered with the context stream; the caller keeps the blocks alive
   until the stream has passed the call, and changes their contents, not
   their addresses, between replays. */
qsk_status qsketch_update_many(qsk_ctx *ctx, int32_t count, const int64_t *col0,
                               const int64_t *ncols, const void *const *planes,
                               const int64_t *ld);

/* General linear update A <- theta A + eta H (Section 5.3 streams the image
   through linear sketch updates of the kind introduced by Tropp et al.; both
   sketches are linear in A), with H zero outside the columns
   [col0, col0 + ncols):
       Y <- theta Y + eta H Omega[col0 : col0 + ncols, :],
       W <- theta W,  W[:, col0 : col0 + ncols] += eta Psi H.
   Same block arguments and limits as qsketch_update; theta and eta must be
   finite (QSK_E_ARG otherwise, with no side effect).  theta = 0 stores exact
   zeros (any earlier content, non-finite values included, is dropped);
   eta = 0 skips the products.  The products are scaled in the precision the
   sketches are stored in (FP32 for the low-precision operand formats, FP64
   otherwise), so eta enters rounded to that precision.  Stream-ordered. */
qsk_status qsketch_update_linear(qsk_ctx *ctx, double theta, double eta, int64_t col0,
                                 int64_t ncols, const void *const planes[4], int64_t ld);

/* Sub-block update A[row0 : row0 + nrows, col0 : col0 + ncols) += H (row
   blocks included), with H the nrows x ncols block in planes (input_dtype,
   ld >= nrows): the column-block update of the full-height block that is H
   on those rows and zero elsewhere (the sketches are linear in A), so it
   costs a whole m-row column block.  The operand formats see that
   full-height block (FP8 tile scales count tile rows from row 0 of A).
   Requires 0 <= row0, 1 <= nrows, row0 + nrows <= m, and the column limits
   of qsketch_update.  The first call allocates a 4 x m x max_block_cols
   staging block (input_dtype) that the context keeps.  Stream-ordered. */
qsk_status qsketch_update_block(qsk_ctx *ctx, int64_t row0, int64_t nrows, int64_t col0,
                                int64_t ncols, const void *const planes[4], int64_t ld);

/* A <- theta A: Y <- theta Y, W <- theta W (theta finite; 0 stores zeros).
   Stream-ordered. */
qsk_status qsketch_scale(qsk_ctx *ctx, double theta);

/* Load sketches (checkpoint restore): Y (m x k) and W (l x n) from FP64
   planes, rounded to the storage precision of ctx (exact for values that
   qsketch_sketches exported from a context of the same configuration), and
   set the column count to columns_seen.  Y or W may be NULL to keep the
   current one.  The caller must have created ctx with the configuration
   (sizes, seed, embedding, operand format) that formed the sketches: the
   test matrices are regenerated from it.  The FP64 planes are device memory
   that must stay valid until the stream passes this call.  Stream-ordered. */
qsk_status qsketch_set_sketches(qsk_ctx *ctx, const double *const Y[4], int64_t ldy,
                                const double *const W[4], int64_t ldw, int64_t columns_seen);

/* QB stage (Alg. 4) on the current sketches, in FP64 on the device:
   Q = F(Y) with F the chosen rangefinder (Alg. 1 or Alg. 3), then
   X = (Psi Q)^dagger W by least squares (Alg. 2), with Psi regenerated to the
   exact values that formed W.  Q: m x k FP64 planes (ldq >= m); X: k x n FP64
   planes (ldx >= k), or X == NULL to run the rangefinder only (required in
   a y_only context, which has no W).  Non-destructive: may be called again (either
   rangefinder) and interleaved with further updates.  Synchronises the stream
   before returning (to read the report); report may be NULL. */
qsk_status qsketch_finalize(qsk_ctx *ctx, qsk_rangefinder rf,
                            double *const Q[4], int64_t ldq,
                            double *const X[4], int64_t ldx,
                            qsk_report *report);

/* Two QB stages (Alg. 4) of the current sketches, e.g. with the pseudo-QR
   (Alg. 1) and the pseudo-SVD (Alg. 3) rangefinder: the same results,
   reports and errors as qsketch_finalize(ctx, rf_a, Qa, ...) followed by
   qsketch_finalize(ctx, rf_b, Qb, ...), bit for bit, but the two stages run
   side by side on the device.  Most of a QB stage is k x k work that keeps
   a few compute units busy, so one stage runs on the context stream (a
   pseudo-QR stage if there is one, else the first) and the other on a
   second stream of the context with a workspace of its own (allocated on
   the first call and kept: two m x k FP64 quaternion buffers and the k x k
   and l x k scratch); results and reports go where the caller's arguments
   say.
   Each pair (Qa, ldqa, Xa, ldxa) and (Qb, ldqb, Xb, ldxb) is checked as in
   qsketch_finalize; no plane of one result may be a plane of the other
   (QSK_E_ARG).  A stage whose factorisation needs the careful path is run
   again on the context stream, as qsketch_finalize does.  Synchronises the
   context stream, which continues after both stages; reports may be NULL. */
qsk_status qsketch_finalize_pair(qsk_ctx *ctx,
                                 qsk_rangefinder rf_a, double *const Qa[4], int64_t ldqa,
                                 double *const Xa[4], int64_t ldxa, qsk_report *report_a,
                                 qsk_rangefinder rf_b, double *const Qb[4], int64_t ldqb,
                                 double *const Xb[4], int64_t ldxb, qsk_report *report_b);

/* Second pass of the two-pass variant (randomized QSVD: the one-pass
   algorithm with Psi = I, Section 4.1, after eq. reconstructionOfTwoSketch):
       X[:, col0 : col0 + ncols) = Q^* A[:, col0 : col0 + ncols),
   which is Q^dagger A when Q has orthonormal columns (the pseudo-SVD
   rangefinder).  Q: m x k FP64 planes (ldq >= m), e.g. from
   qsketch_finalize; planes: the block of A as in qsketch_update (input_dtype,
   ld >= m, 1 <= ncols <= max_block_cols, col0 + ncols <= n); X: k x n FP64
   planes (ldx >= k), only the block's columns are written.  FP64 matrix-core
   products with the m-long contraction split over row chunks.  A call on a
   block wider than any before allocates the chunk partial-sum buffer (up to
   12 k x ncols FP64 quaternion matrices), and the first call on pure input a
   zeroed real plane of the block's shape; the context keeps both.
   Stream-ordered; works in any context (y_only or not) and leaves the
   sketches unchanged. */
qsk_status qsketch_project(qsk_ctx *ctx, double *const Q[4], int64_t ldq, int64_t col0,
                           int64_t ncols, const void *const planes[4], int64_t ld,
                           double *const X[4], int64_t ldx);

/* qsketch_project for callers that cannot allocate device memory (code
   under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc): the same arguments, result and errors as qsketch_project, but
   no call to hipMalloc, hipFree or any allocating routine.  Its work
   memory is a static 32 MiB device array of the library, one per device,
   held until the process ends: the zeroed real plane of a pure-quaternion
   block (cleared on every call) and the partial sums of the split
   contraction (the split shrinks to what the rest of the array holds, down
   to none).  A pure-quaternion block needing more than 32 MiB for its zero
   plane ((ncols - 1) ld + m elements of input_dtype) is rejected with
   QSK_E_ARG.  All calls on one device share the array: calls that overlap
   on one device (different streams or contexts without ordering between
   them) race and give undefined results.  Stream-ordered. */
qsk_status qsketch_project_noalloc(qsk_ctx *ctx, double *const Q[4], int64_t ldq, int64_t col0,
                                   int64_t ncols, const void *const planes[4], int64_t ld,
                                   double *const X[4], int64_t ldx);

/* Truncation stage (Alg. 5): the rank-r QSVD of the approximation Q X,
       Q X ~= (Q U_r) diag(sigma) V_r^*,
   with (U, Sigma, V) the QSVD of X (k x n).  Computed from the eigenpairs of
   the k x k Gram X X^* = U Sigma^2 U^* (the quaternion Hermitian eigensolver
   of the pseudo-SVD rangefinder), V_r = X^* U_r Sigma_r^{-1}; a singular
   value carries a relative error of about 1e-16 (sigma_1 / sigma_i)^2, and a
   zero singular value gets a zero column of V.  Q: m x k, X: k x n FP64
   planes as from qsketch_finalize (ldq >= m, ldx >= k); 1 <= r <= k.
   Outputs: HU = Q U_r (m x r planes, ldh >= m), sigma (r doubles, device
   memory, descending), V = V_r (n x r planes, ldv >= n).  The first call
   allocates an n x k FP64 buffer for X^* that the context keeps.
   Stream-ordered. */
qsk_status qsketch_truncate(qsk_ctx *ctx, double *const Q[4], int64_t ldq, double *const X[4],
                            int64_t ldx, int32_t r, double *const HU[4], int64_t ldh,
                            double *sigma, double *const V[4], int64_t ldv);

/* Copy the current sketches out (Y: m x k, W: l x n) as FP64 planes, for
   tests and checkpoints.  Y or W may be NULL to skip it. */
qsk_status qsketch_sketches(qsk_ctx *ctx, double *const Y[4], int64_t ldy,
                            double *const W[4], int64_t ldw);

/* Y = 0, W = 0, columns_seen = 0 (stream-ordered). */
qsk_status qsketch_reset(qsk_ctx *ctx);

/* Relative error ||A - Q X||_F / ||A||_F (Section 5.1) of an approximation,
   with A given as planes in input_dtype format of ctx (ld >= m) and Q, X as
   FP64 planes from qsketch_finalize.  A measurement pass, not part of the
   one-pass method (it reads A again).  Synchronous; result in *err. */
qsk_status qsketch_rel_error(qsk_ctx *ctx, const void *const A[4], int64_t lda,
                             double *const Q[4], int64_t ldq,
                             double *const X[4], int64_t ldx, double *err);

/* Per-kernel timing of qsketch_update: with enable != 0, every later update
   brackets each of its kernel launches with HIP events on the context
   stream.  qsketch_get_timing synchronises the stream and returns, for
   `kernel` = 0 (test-matrix staging), 1 (Y product), 2 (W product) or
   3 (W split-K reduction), the summed duration in milliseconds and the
   number of launches since timing was enabled (or last reset by enabling
   again).  For measurement only: the events add a few microseconds per
   update. */
qsk_status qsketch_set_timing(qsk_ctx *ctx, int enable);
qsk_status qsketch_get_timing(qsk_ctx *ctx, int kernel, double *total_ms, int64_t *launches);

/* Stream (hipStream_t) of the context. */
void *qsketch_stream(const qsk_ctx *ctx);

/* ---------------------------------------------------------------------------
   Batches of independent problems.  Each problem i is a whole matrix A_i
   (cfgs[i].m x cfgs[i].n) whose one-pass approximation A_i ~ Q_i X_i
   (Alg. 4: both sketches of all columns, the rangefinder, the core solve) is
   computed for all problems together: the two sketch products of every
   problem run in one grouped launch each, and every step of the QB stage is
   one launch over all problems (one workgroup per problem for the small
   k x k algebra).  Randomness, rangefinders and results per problem are
   those of a single context with the same configuration.

   All configurations must share embedding, input_dtype, sketch_dtype (QSK_BF16
   or QSK_F32: the matrix-core path), pure, split_terms, n_correction and
   n_power; m, n, k, l and seed may differ.  max_block_cols is ignored;
   y_only, embedding_round and coalesce_cols must be 0.  Test matrices are drawn and staged
   once, at init. */
typedef struct qsk_batch qsk_batch;

/* Validate the configurations and allocate every problem's workspace on the
   current device (count >= 1).  Synchronous.  QSK_E_ARG for an invalid or
   inconsistent set, QSK_E_UNSUPPORTED for a sketch_dtype other than BF16 or
   F32, QSK_E_NOMEM if device memory is short. */
qsk_status qsketch_batch_init(int32_t count, const qsk_config *cfgs, void *hip_stream,
                              qsk_batch **out);

/* One-pass approximation of every problem with rangefinder rf.  Problem i
   reads A_i from planes[4 i + p] (input_dtype, column-major, leading
   dimension ld[i] >= m_i; planes[4 i] may be NULL when pure) and writes
   Q_i (m_i x k_i, FP64 planes Q[4 i + p], leading dimension ldq[i]) and
   X_i (k_i x n_i, FP64 planes X[4 i + p], leading dimension ldx[i]).  All
   arrays are host arrays of device pointers.  reports (count entries) may
   be NULL.  Allocates no device buffers (a graph capture, below, makes the
   runtime instantiate the graph); synchronises the stream before returning.
   QSK_E_NUMERIC if some problem's sketch is zero or non-finite (the other
   problems' outputs are still written).

   By default (execution mode 2, see qsketch_batch_set_exec) the run is
   first tried optimistically, every Cholesky factorisation assumed to
   succeed: the whole sequence of launches is captured once per rangefinder
   into a HIP graph on an internal stream (ordered after the caller's stream
   and before its later work) and replayed on later calls with the same
   pointer and leading-dimension arrays; a changed array recaptures.  If any
   factorisation failed, the run is repeated with a host check after every
   factorisation and the fallbacks of the single-problem driver.  Concurrent
   runs on one batch handle race. */
qsk_status qsketch_batch_run(qsk_batch *b, qsk_rangefinder rf, const void *const *planes,
                             const int64_t *ld, double *const *Q, const int64_t *ldq,
                             double *const *X, const int64_t *ldx, qsk_report *reports);

/* ||A_i - Q_i X_i||_F / ||A_i||_F for every problem into err[i] (a second
   pass over the inputs, for measurement).  Synchronous. */
qsk_status qsketch_batch_rel_error(qsk_batch *b, const void *const *planes, const int64_t *ld,
                                   double *const *Q, const int64_t *ldq, double *const *X,
                                   const int64_t *ldx, double *err);

/* Autotuner of the batch's launch shapes.  For every candidate (row tiles of
   W per block: 4, 7, 8 or 13, the last two with BF16 operands only; column
   tiles of Y per block: 4 or 7; the number of W blocks the row splits of the
   contraction aim at over all problems: 512, 2048 or 8192) it lays the
   staged test matrices out for that shape, times reps grouped sketch
   launches (Y and W of every problem, inputs as in qsketch_batch_run) after
   one untimed launch, and keeps the fastest.  The choice is remembered for
   the process under the device (architecture name and compute-unit count)
   and the batch's signature (operand format, split terms, input format,
   purity, every problem's m, n, k, l); a batch with the same signature takes
   it without timing; reps = 0 only applies a remembered choice.  When the
   environment variable QSK_TUNE_CACHE names a file, its entries are read
   once per process and every new choice is appended to it, one line each:
   "<arch> <CUs> <format>,<terms>,<input>,<pure>,<m>,<n>,<k>,<l>,... <W row
   tiles> <Y column tiles> <W blocks>"; lines that do not parse or hold
   shapes outside the candidates are ignored, and a file that cannot be
   opened is not an error.  Without a call the shapes come from a padding
   rule and 2048 W blocks.  Results of runs do not depend on the shapes
   beyond rounding order.  Leaves the sketch buffers with meaningless values
   (every run starts from zero).  Synchronous.  *nmt_out, *nj_out,
   *wblocks_out (each may be NULL) receive the shapes in use.  QSK_E_ARG for
   a NULL or short input array or reps outside 0..100. */
qsk_status qsketch_batch_autotune(qsk_batch *b, const void *const *planes, const int64_t *ld,
                                  int32_t reps, int32_t *nmt_out, int32_t *nj_out, int32_t *wblocks_out);

/* Execution mode of qsketch_batch_run: 0 careful only (a host check after
   every factorisation), 1 optimistic stream-ordered launches, 2 optimistic
   as a replayed HIP graph (the default).  Modes give the same results when
   no factorisation fails.  QSK_E_ARG for another value. */
qsk_status qsketch_batch_set_exec(qsk_batch *b, int32_t mode);

void qsketch_batch_destroy(qsk_batch *b);
const char *qsketch_batch_last_error(const qsk_batch *b);

/* Free everything.  Always valid, also on a poisoned context; NULL is a no-op. */
void qsketch_destroy(qsk_ctx *ctx);

const char *qsketch_strerror(qsk_status s);
const char *qsketch_last_error(const qsk_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* QSKETCH_H */
