// Host runtime behind the C ABI of include/qsketch.h: context, workspace,
// stream-ordered launches of the sketch update and of the FP64 QB stage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/qsketch.h"
#include "qsk_kernels.hpp"

// Scratch of the allocation-free projection (qsketch_project_noalloc): the
// zeroed real plane of a pure-quaternion block, then the partial sums of the
// split contraction.  The module holds one copy per device until the process
// ends; host code reaches it only through the address hipGetSymbolAddress
// returns on that device (the array's name is a host-side stand-in).
constexpr size_t QSK_NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[QSK_NOALLOC_SCRATCH_BYTES];

namespace {

using qsk::SmallStatus;

// Device address of `scratch` per device, looked up once per device with
// that device current.
constexpr int QSK_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[QSK_MAX_DEVICES] = {};

hipError_t scratch_address(int dev, void **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= QSK_MAX_DEVICES) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Workspace of one QB stage: the stream it runs on, the two side streams of
// its kappa estimates with their fork/join events, its device status words
// and its FP64 scratch.  Lane 0 is a view of the context's own fields; a
// second lane, allocated on the first paired finalize, lets another QB
// stage of the same sketch run beside it.
struct QbLane {
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr, side2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_fork2 = nullptr, ev_join2 = nullptr;
  double *u[2] = {nullptr, nullptr};   // m x k planar, two alternating buffers
  double *small = nullptr;             // k x k AoS matrices (SmallSlot)
  double *work = nullptr;              // driver scratch
  double *partials = nullptr;          // split-contraction partial sums
  int64_t partial_elems = 0;
  double *pbuf = nullptr, *p1buf = nullptr, *sbuf = nullptr;   // l x k planar each
  double *pinv_work = nullptr;         // (l + k) x k quaternions
  double *kwork = nullptr, *kwork2 = nullptr;
  SmallStatus *status = nullptr, *kstatus = nullptr;
};

}  // namespace

struct qsk_ctx {
  qsk_config cfg{};
  hipStream_t stream = nullptr;
  int device = 0;
  std::atomic<bool> poisoned{false};
  std::mutex err_mu;                   // last_error (a paired finalize launches from two threads)
  std::string last_error;
  int mode = 0;            // qsk::MODE_*
  int emode = 0;           // qsk::MODE_* of the test-matrix values
  size_t ts = 8;           // bytes per Y/W element
  int64_t maxcols = 0;
  int64_t columns_seen = 0;
  uint32_t k0 = 0, k1 = 0;
  // sketches; the matrix-core path keeps y_copies partial copies of Y whose
  // sum is Y (folded into copy 0 before Y is read)
  void *y = nullptr, *w = nullptr;
  int y_copies = 1;
  int y_dirty = 1;                     // copies 0 .. y_dirty - 1 may be nonzero
  // finalize workspace (FP64)
  double *u[2] = {nullptr, nullptr};   // m x k planar, two alternating buffers
  double *small = nullptr;             // k x k AoS matrices
  double *work = nullptr;              // driver scratch
  double *partials = nullptr;
  int64_t partial_elems = 0;
  double *pbuf = nullptr, *p1buf = nullptr, *sbuf = nullptr;   // l x k planar each
  double *err_acc = nullptr;
  double *pinv_work = nullptr;         // (l + k) x k quaternions
  SmallStatus *status = nullptr;
  // kappa estimates only feed the report, so they run on side streams that
  // fork from and join back into the context stream within each finalize:
  // kappa of H0 (pseudo-QR) on `side`, kappa of Q on `side2`, so that the
  // second need not wait for the first
  hipStream_t side = nullptr, side2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_fork2 = nullptr, ev_join2 = nullptr;
  double *kwork = nullptr, *kwork2 = nullptr;   // workspaces of the two kappa kernels
  SmallStatus *kstatus = nullptr;
  void *w_scratch = nullptr;           // split-K partials of the matrix-core W kernel
  int64_t w_scratch_bytes = 0;
  float *fp8_scales = nullptr;         // fp8 tile scales of the current block
  int64_t fp8_scale_elems = 0;
  qsk::MfmaStage stage{};              // transient test-matrix slices (matrix-core path)
  // optional per-kernel timing of updates
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;     // 8 events per recorded update
  size_t ev_used = 0;
  double t_ms[4] = {0, 0, 0, 0};
  int64_t t_count[4] = {0, 0, 0, 0};
  int use_mfma = 1;
  int gen_rad = 1;                     // Rademacher tiles generated in the product kernels
  bool psi_staged = false;             // stage.psi holds Psi as the sketch used it
  bool psi8_staged = false;            // f8.psi holds Psi (FP8X)
  qsk::Fp8xStage f8;                   // FP8X buffers
  void *zero_plane = nullptr;          // zeroed real plane for qsketch_project on pure input
  size_t zero_plane_bytes = 0;
  double *xt = nullptr;                // X^* (n x k planes) for qsketch_truncate
  size_t xt_bytes = 0;
  double *proj_part = nullptr;         // split-contraction partial sums of qsketch_project
  size_t proj_part_bytes = 0;
  void *pad = nullptr;                 // full-height block (4 planes, m x max_block_cols) for
  size_t pad_bytes = 0;                // qsketch_update_block
  void *noalloc_scratch = nullptr;     // this device's `scratch` (qsketch_project_noalloc)
  // coalescing of thin updates (cfg.coalesce_cols > 0): pending columns
  // pend_col0 .. pend_col0 + pend_ncols - 1, one plane of m x coalesce_cols
  // input elements after another (ld = m)
  void *pend = nullptr;
  int64_t pend_col0 = 0, pend_ncols = 0;
  int64_t work_cols = 0;               // widest block the sketch products see
  // Gram Y^* Y of the current sketch (S_YG), kept between finalize calls
  // until the sketch changes (both rangefinders start from it)
  bool gram_valid = false;
  // qsketch_finalize_pair: the second QB lane (its own streams and
  // workspace) and the events that fork it from and join it into `stream`
  QbLane lane1;
  bool lane1_ready = false;
  hipEvent_t ev_pair_fork = nullptr, ev_pair_join = nullptr;
  // qsketch_update_many: a sequence of updates captured once into a HIP
  // graph on its own stream and replayed while the arguments repeat
  hipStream_t gstream = nullptr;
  hipEvent_t gev_in = nullptr, gev_out = nullptr;
  hipGraphExec_t uexec = nullptr;
  std::vector<uint64_t> ukey;
  int64_t u_pend_col0 = 0, u_pend_ncols = 0, u_cols = 0;   // host state after the sequence
  int u_y_dirty = 1;
};

namespace {

const char *status_str(qsk_status s) {
  switch (s) {
    case QSK_OK: return "ok";
    case QSK_E_ARG: return "invalid argument";
    case QSK_E_STATE: return "context poisoned or destroyed";
    case QSK_E_NOMEM: return "device memory allocation failed";
    case QSK_E_HIP: return "HIP runtime error";
    case QSK_E_NUMERIC: return "numerical failure: no Q/X could be formed";
    case QSK_E_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

qsk_status fail_arg(qsk_ctx *c, const char *msg) {
  if (c) {
    std::lock_guard<std::mutex> lock(c->err_mu);
    c->last_error = msg;
  }
  return QSK_E_ARG;
}

qsk_status hip_fail(qsk_ctx *c, hipError_t e, const char *where) {
  c->poisoned = true;
  std::lock_guard<std::mutex> lock(c->err_mu);
  c->last_error = std::string(where) + ": " + hipGetErrorString(e);
  return QSK_E_HIP;
}

#define HIPCHK(ctx, expr)                                   \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr); \
  } while (0)

// A buffer the context grows on demand (kept until qsketch_destroy): at
// least `need` bytes in *p.  The stream is drained before an old buffer is
// freed.  A shortage of device memory returns QSK_E_NOMEM and leaves the
// context usable.
qsk_status grow_buffer(qsk_ctx *ctx, void **p, size_t *bytes, size_t need) {
  if (need <= *bytes) return QSK_OK;
  if (*p) {
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipFree(*p));
    *p = nullptr;
    *bytes = 0;
  }
  const hipError_t e = hipMalloc(p, need);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    *p = nullptr;
    ctx->last_error = "out of device memory for a work buffer";
    return QSK_E_NOMEM;
  }
  HIPCHK(ctx, e);
  *bytes = need;
  return QSK_OK;
}

void resolve_timing(qsk_ctx *c) {
  for (size_t u = 0; u + 8 <= c->ev_used; u += 8) {
    for (int kk = 0; kk < 4; ++kk) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->ev_pool[u + 2 * kk], c->ev_pool[u + 2 * kk + 1]) == hipSuccess) {
        c->t_ms[kk] += ms;
        c->t_count[kk] += 1;
      } else {
        (void)hipGetLastError();
      }
    }
  }
  c->ev_used = 0;
}

void free_events(qsk_ctx *c) {
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  c->ev_pool.clear();
  c->ev_used = 0;
}

void free_lane(QbLane &L) {
  if (L.stream) (void)hipStreamSynchronize(L.stream);
  if (L.side) (void)hipStreamSynchronize(L.side);
  if (L.side2) (void)hipStreamSynchronize(L.side2);
  for (hipEvent_t e : {L.ev_fork, L.ev_join, L.ev_fork2, L.ev_join2})
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t t : {L.stream, L.side, L.side2})
    if (t) (void)hipStreamDestroy(t);
  void *ptrs[] = {L.u[0], L.u[1], L.small, L.work, L.partials, L.pbuf, L.p1buf, L.sbuf,
                  L.pinv_work, L.kwork, L.kwork2, L.status, L.kstatus};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  L = QbLane{};
}

void free_all(qsk_ctx *c) {
  free_events(c);
  free_lane(c->lane1);
  c->lane1_ready = false;
  if (c->ev_pair_fork) (void)hipEventDestroy(c->ev_pair_fork);
  if (c->ev_pair_join) (void)hipEventDestroy(c->ev_pair_join);
  c->ev_pair_fork = c->ev_pair_join = nullptr;
  if (c->side) (void)hipStreamSynchronize(c->side);
  if (c->side2) (void)hipStreamSynchronize(c->side2);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->ev_fork2) (void)hipEventDestroy(c->ev_fork2);
  if (c->ev_join2) (void)hipEventDestroy(c->ev_join2);
  if (c->side) (void)hipStreamDestroy(c->side);
  if (c->side2) (void)hipStreamDestroy(c->side2);
  if (c->uexec) (void)hipGraphExecDestroy(c->uexec);
  if (c->gstream) (void)hipStreamSynchronize(c->gstream);
  if (c->gev_in) (void)hipEventDestroy(c->gev_in);
  if (c->gev_out) (void)hipEventDestroy(c->gev_out);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  c->uexec = nullptr;
  c->gev_in = c->gev_out = nullptr;
  c->gstream = nullptr;
  c->ev_fork = c->ev_join = c->ev_fork2 = c->ev_join2 = nullptr;
  c->side = c->side2 = nullptr;
  void *ptrs[] = {c->y, c->w, c->u[0], c->u[1], c->small, c->work, c->partials, c->pbuf,
                  c->p1buf, c->sbuf, c->err_acc, c->status, c->w_scratch, c->pinv_work,
                  c->stage.omega, c->stage.psi, c->kwork, c->kwork2, c->kstatus, c->fp8_scales, c->zero_plane, c->xt, c->proj_part, c->pad, c->pend,
                  c->f8.qw, c->f8.qy, c->f8.psi, c->f8.om};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  c->y = c->w = nullptr;
  c->u[0] = c->u[1] = nullptr;
  c->small = c->work = c->partials = c->pbuf = c->p1buf = c->sbuf = c->err_acc = nullptr;
  c->status = nullptr;
  c->w_scratch = nullptr;
  c->pinv_work = nullptr;
  c->stage.omega = c->stage.psi = nullptr;
  c->kwork = c->kwork2 = nullptr;
  c->fp8_scales = nullptr;
  c->kstatus = nullptr;
  c->f8.qw = c->f8.qy = c->f8.psi = c->f8.om = nullptr;
}

bool alloc(void **p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return false;
  }
  return true;
}

// Offsets of the k x k matrices inside ctx->small.
enum SmallSlot { S_G1 = 0, S_GU, S_R, S_T, S_RPROD, S_RTMP, S_G0, S_TMP, S_C, S_F, S_GP, S_RP,
                 S_TP1, S_TP2, S_TPT, S_Z, S_CR, S_CT, S_GI, S_M, S_TMP2, S_GH, S_GK0, S_YG, S_COUNT };

double *slot(qsk_ctx *c, int s) { return c->small + (size_t)s * c->cfg.k * c->cfg.k * 4; }
double *slot(const QbLane &L, int k, int s) { return L.small + (size_t)s * k * k * 4; }

// Lane 0: the context's own finalize workspace on the context stream.
QbLane lane0(qsk_ctx *c) {
  QbLane L;
  L.stream = c->stream;
  L.side = c->side; L.side2 = c->side2;
  L.ev_fork = c->ev_fork; L.ev_join = c->ev_join; L.ev_fork2 = c->ev_fork2; L.ev_join2 = c->ev_join2;
  L.u[0] = c->u[0]; L.u[1] = c->u[1];
  L.small = c->small; L.work = c->work;
  L.partials = c->partials; L.partial_elems = c->partial_elems;
  L.pbuf = c->pbuf; L.p1buf = c->p1buf; L.sbuf = c->sbuf; L.pinv_work = c->pinv_work;
  L.kwork = c->kwork; L.kwork2 = c->kwork2;
  L.status = c->status; L.kstatus = c->kstatus;
  return L;
}

// Sum the split-K copies of Y into copy 0 (stream-ordered).
// Only the copies an update added into since the last fold are read.
hipError_t fold_y(qsk_ctx *c) {
  if (c->y_copies <= 1 || c->y_dirty <= 1) return hipSuccess;
  const hipError_t e = qsk::launch_y_fold(c->stream, (float *)c->y, 4 * c->cfg.m * (int64_t)c->cfg.k, c->y_dirty);
  if (e == hipSuccess) c->y_dirty = 1;
  return e;
}

}  // namespace

extern "C" {

void qsketch_config_default(qsk_config *cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->embedding = QSK_GAUSSIAN;
  cfg->input_dtype = QSK_F64;
  cfg->sketch_dtype = QSK_F64;
  cfg->split_terms = 1;
  cfg->n_correction = 3;
  cfg->n_power = 3;
}

const char *qsketch_strerror(qsk_status s) { return status_str(s); }

const char *qsketch_last_error(const qsk_ctx *ctx) {
  if (!ctx) return "null context";
  return ctx->last_error.c_str();
}

void *qsketch_stream(const qsk_ctx *ctx) { return ctx ? (void *)ctx->stream : nullptr; }

qsk_status qsketch_set_timing(qsk_ctx *ctx, int enable) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->ev_used = 0;
  for (int i = 0; i < 4; ++i) { ctx->t_ms[i] = 0.0; ctx->t_count[i] = 0; }
  ctx->timing = enable != 0;
  return QSK_OK;
}

qsk_status qsketch_get_timing(qsk_ctx *ctx, int kernel, double *total_ms, int64_t *launches) {
  if (!ctx || kernel < 0 || kernel > 3 || !total_ms || !launches) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  resolve_timing(ctx);
  *total_ms = ctx->t_ms[kernel];
  *launches = ctx->t_count[kernel];
  return QSK_OK;
}

qsk_status qsketch_init(const qsk_config *cfg, void *hip_stream, qsk_ctx **out) {
  if (!cfg || !out) return QSK_E_ARG;
  *out = nullptr;
  const qsk_config &c = *cfg;
  if (c.m < 1 || c.n < 1 || c.m >= (1ll << 31) || c.n >= (1ll << 31)) return QSK_E_ARG;
  if (c.k < 1 || c.l < c.k || c.l > c.m || c.l > c.n || c.k > 256 || c.l > 1024) return QSK_E_ARG;
  if (c.embedding != QSK_GAUSSIAN && c.embedding != QSK_RADEMACHER) return QSK_E_ARG;
  if (c.input_dtype < QSK_F64 || c.input_dtype > QSK_BF16) return QSK_E_ARG;
  if (c.sketch_dtype < QSK_F64 || c.sketch_dtype > QSK_FP8_MFMA) return QSK_E_ARG;
  if (c.n_correction < 0 || c.n_correction > 8 || c.n_power < 1 || c.n_power > 64) return QSK_E_ARG;
  if (c.max_block_cols < 0) return QSK_E_ARG;
  if (c.y_only != 0 && c.y_only != 1) return QSK_E_ARG;
  if (c.coalesce_cols < 0 || c.coalesce_cols > c.n) return QSK_E_ARG;
  if (c.sketch_dtype == QSK_BF16 && (c.split_terms < 1 || c.split_terms > 3)) return QSK_E_ARG;
  if (c.sketch_dtype == QSK_FP8_E4M3 && (c.split_terms < 1 || c.split_terms > 2)) return QSK_E_ARG;
  if (c.sketch_dtype == QSK_FP8_MFMA && (c.split_terms < 1 || c.split_terms > 4)) return QSK_E_ARG;
  if (c.sketch_dtype != QSK_F64 && c.input_dtype == QSK_F64) return QSK_E_UNSUPPORTED;
  if (c.embedding_round < QSK_F64 || c.embedding_round > QSK_FP8_E4M3) return QSK_E_ARG;
  if (c.embedding_round != QSK_F64 && c.sketch_dtype != QSK_F64) return QSK_E_ARG;

  qsk_ctx *ctx = new (std::nothrow) qsk_ctx;
  if (!ctx) return QSK_E_NOMEM;
  ctx->cfg = c;
  if (ctx->cfg.max_block_cols == 0 || ctx->cfg.max_block_cols > c.n) ctx->cfg.max_block_cols = c.n;
  ctx->work_cols = std::max<int64_t>(ctx->cfg.max_block_cols, c.coalesce_cols);
  if (ctx->cfg.sketch_dtype != QSK_BF16 && ctx->cfg.sketch_dtype != QSK_FP8_E4M3 &&
      ctx->cfg.sketch_dtype != QSK_FP8_MFMA)
    ctx->cfg.split_terms = 1;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->mode = c.sketch_dtype;     // MODE_* and QSK dtypes share the numbering
  ctx->emode = c.sketch_dtype == QSK_F64 ? c.embedding_round
              : c.sketch_dtype == QSK_FP8_MFMA ? (int)qsk::MODE_FP8 : c.sketch_dtype;
  ctx->ts = c.sketch_dtype == QSK_F64 ? 8 : 4;
  ctx->k0 = (uint32_t)(c.seed & 0xFFFFFFFFull);
  ctx->k1 = (uint32_t)(c.seed >> 32);
  const char *env = std::getenv("QSK_NO_MFMA");
  ctx->use_mfma = (env && env[0] == '1') ? 0 : 1;
  const char *genv = std::getenv("QSK_STAGE_RADEMACHER");
  ctx->gen_rad = (genv && genv[0] == '1') ? 0 : 1;
  if (hipGetDevice(&ctx->device) != hipSuccess ||
      scratch_address(ctx->device, &ctx->noalloc_scratch) != hipSuccess) {
    (void)hipGetLastError();
    delete ctx;
    return QSK_E_HIP;
  }

  const int64_t m = c.m, n = c.n, k = c.k, l = c.l;
  const size_t kk = (size_t)k * k * 4;
  bool ok = true;
  const bool mfma_mode = c.sketch_dtype == QSK_BF16 || c.sketch_dtype == QSK_F32 ||
                         c.sketch_dtype == QSK_FP8_E4M3 || c.sketch_dtype == QSK_FP8_MFMA;
  ctx->y_copies = mfma_mode ? qsk::Y_COPIES : 1;
  ok = ok && alloc(&ctx->y, (size_t)ctx->y_copies * 4 * m * k * ctx->ts);
  if (!c.y_only) ok = ok && alloc(&ctx->w, 4 * (size_t)l * n * ctx->ts);
  ok = ok && alloc((void **)&ctx->u[0], 4 * (size_t)m * k * 8);
  ok = ok && alloc((void **)&ctx->u[1], 4 * (size_t)m * k * 8);
  ok = ok && alloc((void **)&ctx->small, S_COUNT * kk * 8);
  ok = ok && alloc((void **)&ctx->work, (12 * kk + 64 * (size_t)k) * 8);
  const int64_t maxk = l > k ? l : k;
  // split-contraction partial sums: room for 64 chunks of the largest
  // product and for 4096 chunk tiles (16 x 16, 4 planes) of any product
  ctx->partial_elems = std::max<int64_t>(64 * maxk * k * 4, 4096 * 1024);
  ok = ok && alloc((void **)&ctx->partials, (size_t)ctx->partial_elems * 8);
  ok = ok && alloc((void **)&ctx->pbuf, 4 * (size_t)l * k * 8);
  ok = ok && alloc((void **)&ctx->p1buf, 4 * (size_t)l * k * 8);
  ok = ok && alloc((void **)&ctx->sbuf, 4 * (size_t)l * k * 8);
  ok = ok && alloc((void **)&ctx->err_acc, 2 * 8);
  ok = ok && alloc((void **)&ctx->pinv_work, 4 * (size_t)(l + k) * k * 8);
  ok = ok && alloc((void **)&ctx->status, sizeof(SmallStatus));
  ok = ok && alloc((void **)&ctx->kstatus, sizeof(SmallStatus));
  ok = ok && alloc((void **)&ctx->kwork, kk * 8);
  ok = ok && alloc((void **)&ctx->kwork2, kk * 8);
  ok = ok && hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&ctx->side2, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&ctx->ev_fork2, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&ctx->ev_join2, hipEventDisableTiming) == hipSuccess;
  // matrix-core path: staging of Omega_J / Psi and the W split-K partials
  if (mfma_mode) {
    qsk::MfmaStage &g = ctx->stage;
    const bool op16 = c.sketch_dtype != QSK_F32;     // bf16 operands (BF16, FP8 data)
    qsk::stage_geometry(m, (int)l, (int)k, ctx->work_cols, op16, &g.LP, &g.MP, &g.KP, &g.NP);
    const size_t es = op16 ? 2 : 4;
    if (c.sketch_dtype == QSK_FP8_E4M3 || c.sketch_dtype == QSK_FP8_MFMA) {
      ctx->fp8_scale_elems = 4 * ((m + 31) / 32) * ((ctx->work_cols + 31) / 32);
      ok = ok && alloc((void **)&ctx->fp8_scales, (size_t)ctx->fp8_scale_elems * 4);
    }
    if (c.sketch_dtype == QSK_FP8_MFMA) {
      // the quantised block in both layouts and the e4m3 test matrices (the
      // bf16 staging below keeps Psi's e4m3 values for the QB stage)
      qsk::fp8x_geometry(m, (int)l, (int)k, ctx->work_cols, c.split_terms, c.pure, &ctx->f8);
      ok = ok && alloc((void **)&ctx->f8.qw, (size_t)ctx->f8.qw_bytes);
      ok = ok && alloc((void **)&ctx->f8.qy, (size_t)ctx->f8.qy_bytes);
      ok = ok && alloc((void **)&ctx->f8.psi, (size_t)ctx->f8.psi_bytes);
      ok = ok && alloc((void **)&ctx->f8.om, (size_t)ctx->f8.om_bytes);
    }
    ok = ok && alloc(&g.omega, 4 * (size_t)g.KP * g.NP * es);
    ok = ok && alloc(&g.psi, 4 * (size_t)g.LP * g.MP * es);
    // W split-K partials: 16 splits of the widest block, or, for thin
    // blocks (whose few column tiles need many row chunks to fill the
    // chip), as many splits of 256 rows as fit in 64 MiB
    const int64_t per_split = (int64_t)4 * ctx->work_cols * g.LP * 4;
    ctx->w_scratch_bytes = std::max<int64_t>(16 * per_split,
                                             std::min<int64_t>((int64_t)64 << 20, (m / 256) * per_split));
    ok = ok && alloc(&ctx->w_scratch, (size_t)ctx->w_scratch_bytes);
  }
  if (c.coalesce_cols > 0) {
    const size_t es = c.input_dtype == QSK_F64 ? 8 : c.input_dtype == QSK_F32 ? 4 : 2;
    ok = ok && alloc(&ctx->pend, 4 * (size_t)m * c.coalesce_cols * es);
  }
  if (!ok) {
    free_all(ctx);
    delete ctx;
    return QSK_E_NOMEM;
  }
  hipError_t e = hipMemsetAsync(ctx->y, 0, (size_t)ctx->y_copies * 4 * m * k * ctx->ts, ctx->stream);
  if (e == hipSuccess && ctx->w) e = hipMemsetAsync(ctx->w, 0, 4 * (size_t)l * n * ctx->ts, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    free_all(ctx);
    delete ctx;
    return QSK_E_HIP;
  }
  *out = ctx;
  return QSK_OK;
}

void qsketch_destroy(qsk_ctx *ctx) {
  if (!ctx) return;
  if (ctx->stream || true) (void)hipStreamSynchronize(ctx->stream);
  free_all(ctx);
  delete ctx;
}

qsk_status qsketch_reset(qsk_ctx *ctx) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  const qsk_config &c = ctx->cfg;
  HIPCHK(ctx, hipMemsetAsync(ctx->y, 0, (size_t)ctx->y_copies * 4 * c.m * c.k * ctx->ts, ctx->stream));
  if (ctx->w) HIPCHK(ctx, hipMemsetAsync(ctx->w, 0, 4 * (size_t)c.l * c.n * ctx->ts, ctx->stream));
  ctx->columns_seen = 0;
  ctx->pend_ncols = 0;
  ctx->gram_valid = false;
  ctx->y_dirty = 1;
  return QSK_OK;
}

static qsk_status check_block(qsk_ctx *ctx, int64_t col0, int64_t ncols, const void *const planes[4],
                              int64_t ld) {
  const qsk_config &c = ctx->cfg;
  if (!planes) return fail_arg(ctx, "planes is NULL");
  if (col0 < 0 || ncols < 1 || ncols > c.max_block_cols || col0 + ncols > c.n)
    return fail_arg(ctx, "column block out of range");
  if (ld < c.m) return fail_arg(ctx, "ld < m");
  for (int p = c.pure ? 1 : 0; p < 4; ++p)
    if (!planes[p]) return fail_arg(ctx, "NULL plane");
  return QSK_OK;
}

// Y += eta H Omega_J, W[:, J] += eta Psi H for a checked block.
static qsk_status sketch_block(qsk_ctx *ctx, int64_t col0, int64_t ncols, const void *const planes[4],
                               int64_t ld, double eta) {
  const qsk_config &c = ctx->cfg;
  ctx->gram_valid = false;
  qsk::SketchArgs s{};
  s.eta = eta;
  s.skip_w = c.y_only;
  s.stream = ctx->stream;
  s.mode = ctx->mode;
  s.emode = ctx->emode;
  s.in_dtype = c.input_dtype;
  for (int p = 0; p < 4; ++p) s.planes[p] = planes[p];
  if (c.pure) s.planes[0] = planes[1];
  s.lda = ld;
  s.pure = c.pure;
  s.m = c.m; s.col0 = col0; s.ncols = ncols;
  s.k = c.k; s.l = c.l;
  s.y = ctx->y; s.ldy = c.m; s.psy = c.m * (int64_t)c.k;
  s.pss = 4 * c.m * (int64_t)c.k;
  s.y_copies = ctx->y_copies;
  s.w = ctx->w; s.ldw = c.l; s.psw = c.l * (int64_t)c.n;
  s.rad = c.embedding == QSK_RADEMACHER;
  s.terms = c.split_terms;
  s.k0 = ctx->k0; s.k1 = ctx->k1;
  s.scratch = ctx->w_scratch;
  s.scratch_bytes = ctx->w_scratch_bytes;
  s.fp8_scales = ctx->fp8_scales;
  s.fp8_scale_elems = ctx->fp8_scale_elems;
  s.psi_ready = (ctx->mode == qsk::MODE_FP8X ? ctx->psi8_staged : ctx->psi_staged) ? 1 : 0;
  s.gen_rad = ctx->gen_rad;
  if (ctx->mode == qsk::MODE_FP8X) s.f8 = &ctx->f8;
  int splits = 1;
  s.y_splits = &splits;
  s.events = nullptr;
  if (ctx->timing && ctx->use_mfma && ctx->mode != qsk::MODE_F64) {
    if (ctx->ev_used + 8 > ctx->ev_pool.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t ev;
        HIPCHK(ctx, hipEventCreate(&ev));
        ctx->ev_pool.push_back(ev);
      }
    }
    s.events = &ctx->ev_pool[ctx->ev_used];
    ctx->ev_used += 8;
  }
  hipError_t e = hipErrorNotSupported;
  if (ctx->use_mfma && ctx->mode != qsk::MODE_F64) {
    e = qsk::launch_sketch_mfma(s, ctx->stage);
    if (e == hipSuccess && !c.y_only && ctx->mode == qsk::MODE_FP8X) ctx->psi8_staged = true;
    else if (e == hipSuccess && !c.y_only && !qsk::gen_in_kernel(s)) ctx->psi_staged = true;
    if (e == hipSuccess && splits > ctx->y_dirty) ctx->y_dirty = splits;
  }
  if (e == hipErrorNotSupported && (ctx->mode == qsk::MODE_FP8 || ctx->mode == qsk::MODE_FP8X)) {
    ctx->last_error = "fp8 sketch: block too large for the matrix-core path (32-bit offsets) or "
                      "matrix-core path disabled";
    return QSK_E_UNSUPPORTED;
  }
  if (e == hipErrorNotSupported) e = qsk::launch_sketch_generic(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "sketch update");
  return QSK_OK;
}

// Coalescing of thin updates: the pending columns' planes in ctx->pend.
static size_t input_size(const qsk_config &c) {
  return c.input_dtype == QSK_F64 ? 8 : c.input_dtype == QSK_F32 ? 4 : 2;
}

static void pending_planes(qsk_ctx *ctx, const void *pl[4]) {
  const qsk_config &c = ctx->cfg;
  const size_t plane = (size_t)c.m * c.coalesce_cols * input_size(c);
  for (int p = 0; p < 4; ++p) pl[p] = (const char *)ctx->pend + p * plane;
}

// Run the sketch products on the pending columns (if any).
static qsk_status flush_pending(qsk_ctx *ctx) {
  if (ctx->pend_ncols == 0) return QSK_OK;
  const void *pl[4];
  pending_planes(ctx, pl);
  const int64_t c0 = ctx->pend_col0, nc = ctx->pend_ncols;
  ctx->pend_ncols = 0;
  return sketch_block(ctx, c0, nc, pl, ctx->cfg.m, 1.0);
}

// Copy a checked block behind the pending columns (stream-ordered).
static qsk_status append_pending(qsk_ctx *ctx, int64_t col0, int64_t ncols, const void *const planes[4],
                                 int64_t ld) {
  const qsk_config &c = ctx->cfg;
  const size_t es = input_size(c);
  const void *pl[4];
  pending_planes(ctx, pl);
  if (ctx->pend_ncols == 0) ctx->pend_col0 = col0;
  for (int p = c.pure ? 1 : 0; p < 4; ++p) {
    char *dst = (char *)pl[p] + (size_t)ctx->pend_ncols * c.m * es;
    HIPCHK(ctx, hipMemcpy2DAsync(dst, (size_t)c.m * es, planes[p], (size_t)ld * es, (size_t)c.m * es,
                                 (size_t)ncols, hipMemcpyDeviceToDevice, ctx->stream));
  }
  ctx->pend_ncols += ncols;
  return QSK_OK;
}

// One checked column-block update (qsketch_update without the checks).
static qsk_status update_body(qsk_ctx *ctx, int64_t col0, int64_t ncols, const void *const planes[4],
                              int64_t ld) {
  const qsk_config &c = ctx->cfg;
  qsk_status st = QSK_OK;
  if (c.coalesce_cols > 0 && ncols < c.coalesce_cols) {
    if (ctx->pend_ncols > 0 &&
        (col0 != ctx->pend_col0 + ctx->pend_ncols || ctx->pend_ncols + ncols > c.coalesce_cols))
      st = flush_pending(ctx);
    if (st == QSK_OK) st = append_pending(ctx, col0, ncols, planes, ld);
    if (st == QSK_OK && ctx->pend_ncols == c.coalesce_cols) st = flush_pending(ctx);
  } else {
    st = flush_pending(ctx);
    if (st == QSK_OK) st = sketch_block(ctx, col0, ncols, planes, ld, 1.0);
  }
  if (st == QSK_OK) ctx->columns_seen += ncols;
  return st;
}

qsk_status qsketch_update(qsk_ctx *ctx, int64_t col0, int64_t ncols, const void *const planes[4],
                          int64_t ld) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  const qsk_status st = check_block(ctx, col0, ncols, planes, ld);
  if (st != QSK_OK) return st;
  return update_body(ctx, col0, ncols, planes, ld);
}

qsk_status qsketch_update_many(qsk_ctx *ctx, int32_t count, const int64_t *col0, const int64_t *ncols,
                               const void *const *planes, const int64_t *ld) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  if (count < 1 || !col0 || !ncols || !planes || !ld) return fail_arg(ctx, "bad update_many arguments");
  for (int32_t i = 0; i < count; ++i) {
    const qsk_status st = check_block(ctx, col0[i], ncols[i], planes + 4 * (size_t)i, ld[i]);
    if (st != QSK_OK) return st;
  }
  const qsk_config &c = ctx->cfg;
  if (!ctx->gstream) {
    HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->gev_in, hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->gev_out, hipEventDisableTiming));
  }
  // Psi is staged (once per context) outside the graph, so that replays do
  // not stage it again
  if (ctx->use_mfma && ctx->mode == qsk::MODE_FP8X && !c.y_only && !ctx->psi8_staged) {
    qsk::SketchArgs sa{};
    sa.stream = ctx->stream; sa.mode = ctx->mode; sa.l = c.l; sa.m = c.m; sa.k = c.k;
    sa.rad = c.embedding == QSK_RADEMACHER; sa.k0 = ctx->k0; sa.k1 = ctx->k1;
    HIPCHK(ctx, qsk::stage_psi8(sa, ctx->f8));
    ctx->psi8_staged = true;
  } else if (ctx->use_mfma && ctx->mode != qsk::MODE_F64 && !c.y_only && !ctx->psi_staged) {
    qsk::SketchArgs sa{};
    sa.stream = ctx->stream; sa.mode = ctx->mode; sa.l = c.l; sa.m = c.m; sa.k = c.k;
    sa.rad = c.embedding == QSK_RADEMACHER; sa.k0 = ctx->k0; sa.k1 = ctx->k1;
    sa.gen_rad = ctx->gen_rad;
    if (!qsk::gen_in_kernel(sa)) {
      HIPCHK(ctx, qsk::stage_psi(sa, ctx->stage));
      ctx->psi_staged = true;
    }
  }
  // the sequence, with the pending-column state it starts from
  std::vector<uint64_t> key;
  key.reserve(8 * (size_t)count + 4);
  key.push_back((uint64_t)count);
  key.push_back((uint64_t)ctx->pend_col0);
  key.push_back((uint64_t)ctx->pend_ncols);
  key.push_back((uint64_t)ctx->psi_staged | ((uint64_t)ctx->psi8_staged << 1));
  for (int32_t i = 0; i < count; ++i) {
    key.push_back((uint64_t)col0[i]);
    key.push_back((uint64_t)ncols[i]);
    key.push_back((uint64_t)ld[i]);
    for (int p = 0; p < 4; ++p) key.push_back((uint64_t)(uintptr_t)planes[4 * (size_t)i + p]);
  }
  if (!ctx->uexec || key != ctx->ukey) {
    if (ctx->uexec) {
      HIPCHK(ctx, hipStreamSynchronize(ctx->gstream));
      (void)hipGraphExecDestroy(ctx->uexec);
      ctx->uexec = nullptr;
    }
    // capture the updates on the graph stream (the host state they change
    // is recorded for the replays)
    hipStream_t user = ctx->stream;
    const bool timing = ctx->timing;
    ctx->stream = ctx->gstream;
    ctx->timing = false;
    int64_t cols = 0;
    hipError_t e = hipStreamBeginCapture(ctx->gstream, hipStreamCaptureModeThreadLocal);
    qsk_status r = e == hipSuccess ? QSK_OK : QSK_E_HIP;
    for (int32_t i = 0; i < count && r == QSK_OK; ++i) {
      r = update_body(ctx, col0[i], ncols[i], planes + 4 * (size_t)i, ld[i]);
      cols += ncols[i];
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(ctx->gstream, &graph) : e;
    ctx->stream = user;
    ctx->timing = timing;
    if (r != QSK_OK || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (r != QSK_OK) return r;
      return hip_fail(ctx, e2, "capture of the updates");
    }
    const hipError_t e3 = hipGraphInstantiate(&ctx->uexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) {
      ctx->uexec = nullptr;
      return hip_fail(ctx, e3, "hipGraphInstantiate");
    }
    ctx->ukey = key;
    ctx->u_pend_col0 = ctx->pend_col0;
    ctx->u_pend_ncols = ctx->pend_ncols;
    ctx->u_y_dirty = ctx->y_dirty;
    ctx->u_cols = cols;
    // the capture ran nothing: the state it left is what the launch makes
    ctx->columns_seen -= cols;
  }
  HIPCHK(ctx, hipEventRecord(ctx->gev_in, ctx->stream));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->gstream, ctx->gev_in, 0));
  HIPCHK(ctx, hipGraphLaunch(ctx->uexec, ctx->gstream));
  HIPCHK(ctx, hipEventRecord(ctx->gev_out, ctx->gstream));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->gev_out, 0));
  ctx->pend_col0 = ctx->u_pend_col0;
  ctx->pend_ncols = ctx->u_pend_ncols;
  if (ctx->u_y_dirty > ctx->y_dirty) ctx->y_dirty = ctx->u_y_dirty;
  ctx->gram_valid = false;
  ctx->columns_seen += ctx->u_cols;
  return QSK_OK;
}

qsk_status qsketch_update_block(qsk_ctx *ctx, int64_t row0, int64_t nrows, int64_t col0, int64_t ncols,
                                const void *const planes[4], int64_t ld) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  const qsk_config &c = ctx->cfg;
  if (row0 < 0 || nrows < 1 || row0 + nrows > c.m) return fail_arg(ctx, "row block out of range");
  if (!planes) return fail_arg(ctx, "planes is NULL");
  if (col0 < 0 || ncols < 1 || ncols > c.max_block_cols || col0 + ncols > c.n)
    return fail_arg(ctx, "column block out of range");
  if (ld < nrows) return fail_arg(ctx, "ld < nrows");
  for (int p = c.pure ? 1 : 0; p < 4; ++p)
    if (!planes[p]) return fail_arg(ctx, "NULL plane");
  const size_t es = c.input_dtype == QSK_F64 ? 8 : c.input_dtype == QSK_F32 ? 4 : 2;
  const size_t plane = (size_t)c.m * c.max_block_cols * es;
  {
    const qsk_status gs = grow_buffer(ctx, &ctx->pad, &ctx->pad_bytes, 4 * plane);
    if (gs != QSK_OK) return gs;
  }
  {
    const qsk_status fs = flush_pending(ctx);
    if (fs != QSK_OK) return fs;
  }
  // the full-height block: zero outside rows row0 .. row0 + nrows - 1
  const void *full[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int p = c.pure ? 1 : 0; p < 4; ++p) {
    char *dst = (char *)ctx->pad + p * plane;
    HIPCHK(ctx, hipMemsetAsync(dst, 0, (size_t)c.m * ncols * es, ctx->stream));
    HIPCHK(ctx, hipMemcpy2DAsync(dst + (size_t)row0 * es, (size_t)c.m * es, planes[p], (size_t)ld * es,
                                 (size_t)nrows * es, (size_t)ncols, hipMemcpyDeviceToDevice, ctx->stream));
    full[p] = dst;
  }
  if (c.pure) full[0] = full[1];
  qsk_status st = sketch_block(ctx, col0, ncols, full, c.m, 1.0);
  if (st == QSK_OK) ctx->columns_seen += ncols;
  return st;
}

// A <- theta A: both sketches are linear in A, so Y <- theta Y, W <- theta W
// (every split-K copy of Y scales with the sum).
static qsk_status scale_sketches(qsk_ctx *ctx, double theta) {
  if (theta == 1.0) return QSK_OK;
  ctx->gram_valid = false;
  const qsk_config &c = ctx->cfg;
  const int t = ctx->mode == qsk::MODE_F64 ? 0 : 1;
  HIPCHK(ctx, qsk::launch_scale(ctx->stream, t, ctx->y, (int64_t)ctx->y_copies * 4 * c.m * (int64_t)c.k, theta));
  if (ctx->w) HIPCHK(ctx, qsk::launch_scale(ctx->stream, t, ctx->w, 4 * (int64_t)c.l * c.n, theta));
  return QSK_OK;
}

qsk_status qsketch_scale(qsk_ctx *ctx, double theta) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  if (!std::isfinite(theta)) return fail_arg(ctx, "theta is not finite");
  const qsk_status fs = flush_pending(ctx);
  if (fs != QSK_OK) return fs;
  return scale_sketches(ctx, theta);
}

qsk_status qsketch_update_linear(qsk_ctx *ctx, double theta, double eta, int64_t col0, int64_t ncols,
                                 const void *const planes[4], int64_t ld) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  if (!std::isfinite(theta) || !std::isfinite(eta)) return fail_arg(ctx, "theta or eta is not finite");
  qsk_status st = check_block(ctx, col0, ncols, planes, ld);
  if (st == QSK_OK) st = flush_pending(ctx);
  if (st == QSK_OK) st = scale_sketches(ctx, theta);
  if (st == QSK_OK && eta != 0.0) st = sketch_block(ctx, col0, ncols, planes, ld, eta);
  if (st == QSK_OK) ctx->columns_seen += ncols;
  return st;
}

qsk_status qsketch_set_sketches(qsk_ctx *ctx, const double *const Y[4], int64_t ldy,
                                const double *const W[4], int64_t ldw, int64_t columns_seen) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  const qsk_config &c = ctx->cfg;
  if (columns_seen < 0) return fail_arg(ctx, "columns_seen < 0");
  if (Y) {
    if (ldy < c.m) return fail_arg(ctx, "ldy < m");
    for (int p = 0; p < 4; ++p)
      if (!Y[p]) return fail_arg(ctx, "NULL Y plane");
  }
  if (W) {
    if (!ctx->w) return fail_arg(ctx, "the context keeps no W (y_only)");
    if (ldw < c.l) return fail_arg(ctx, "ldw < l");
    for (int p = 0; p < 4; ++p)
      if (!W[p]) return fail_arg(ctx, "NULL W plane");
  }
  const int t = ctx->mode == qsk::MODE_F64 ? 0 : 1;
  ctx->pend_ncols = 0;                   // the new state replaces pending columns too
  ctx->gram_valid = false;
  if (Y) {
    const int64_t per_copy = 4 * c.m * (int64_t)c.k;
    if (ctx->y_copies > 1)
      HIPCHK(ctx, hipMemsetAsync((char *)ctx->y + per_copy * ctx->ts, 0,
                                 (size_t)(ctx->y_copies - 1) * per_copy * ctx->ts, ctx->stream));
    HIPCHK(ctx, qsk::launch_narrow(ctx->stream, t, Y, ldy, ctx->y, c.m, c.m * (int64_t)c.k, c.m, c.k));
    ctx->y_dirty = 1;
  }
  if (W) HIPCHK(ctx, qsk::launch_narrow(ctx->stream, t, W, ldw, ctx->w, c.l, c.l * (int64_t)c.n, c.l, c.n));
  ctx->columns_seen = columns_seen;
  return QSK_OK;
}

qsk_status qsketch_sketches(qsk_ctx *ctx, double *const Y[4], int64_t ldy, double *const W[4],
                            int64_t ldw) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  const qsk_config &c = ctx->cfg;
  const int t = ctx->mode == qsk::MODE_F64 ? 0 : 1;
  {
    const qsk_status fs = flush_pending(ctx);
    if (fs != QSK_OK) return fs;
  }
  if (Y) {
    if (ldy < c.m) return fail_arg(ctx, "ldy < m");
    HIPCHK(ctx, fold_y(ctx));
    HIPCHK(ctx, qsk::launch_widen(ctx->stream, t, ctx->y, c.m, c.m * (int64_t)c.k, c.m, c.k, Y, ldy));
  }
  if (W) {
    if (!ctx->w) return fail_arg(ctx, "the context keeps no W (y_only)");
    if (ldw < c.l) return fail_arg(ctx, "ldw < l");
    HIPCHK(ctx, qsk::launch_widen(ctx->stream, t, ctx->w, c.l, c.l * (int64_t)c.n, c.l, c.n, W, ldw));
  }
  return QSK_OK;
}

// One QB stage.  optimistic: no host synchronisation after the Cholesky
// factorisations (every one is assumed to succeed); a failure anywhere is
// recorded in the status's sticky fail_any and the call returns
// QSK_RETRY_CAREFUL, after which the caller runs the careful version, which
// checks each factorisation and takes the fallbacks.
static const qsk_status QSK_RETRY_CAREFUL = static_cast<qsk_status>(-1);

// What one enqueued QB stage leaves for its collection.
struct QbRun {
  qsk_rangefinder rf = QSK_PSEUDO_QR;   // QSK_PSEUDO_SVD_GS folded into QSK_PSEUDO_SVD
  int passes = 0;
  int flags = 0;
  bool kappa0 = false;                  // kappa of H0 launched on the lane's `side`
};

static qsk_status qb_check(qsk_ctx *ctx, qsk_rangefinder rf, double *const Q[4], int64_t ldq,
                           double *const X[4], int64_t ldx) {
  const qsk_config &c = ctx->cfg;
  if (rf != QSK_PSEUDO_QR && rf != QSK_PSEUDO_SVD && rf != QSK_PSEUDO_SVD_GS)
    return fail_arg(ctx, "unknown rangefinder");
  if (!Q) return fail_arg(ctx, "Q NULL");
  if (X && !ctx->w) return fail_arg(ctx, "the context keeps no W (y_only): call with X = NULL");
  for (int p = 0; p < 4; ++p)
    if (!Q[p] || (X && !X[p])) return fail_arg(ctx, "NULL output plane");
  if (ldq < c.m || (X && ldx < c.k)) return fail_arg(ctx, "leading dimension too small");
  return QSK_OK;
}

// Pending columns into the sketches, the split-K copies of Y summed.
static qsk_status qb_prepare(qsk_ctx *ctx) {
  const qsk_status fs = flush_pending(ctx);
  if (fs != QSK_OK) return fs;
  HIPCHK(ctx, fold_y(ctx));
  return QSK_OK;
}

// Y^* Y into dst on the lane's stream (with the lane's partial sums).
static qsk_status y_gram(qsk_ctx *ctx, const QbLane &L, double *dst) {
  const qsk_config &c = ctx->cfg;
  const int ty = ctx->mode == qsk::MODE_F64 ? 0 : 1;
  const void *yp[4];
  for (int p = 0; p < 4; ++p) yp[p] = (const char *)ctx->y + (size_t)p * c.m * c.k * ctx->ts;
  HIPCHK(ctx, qsk::launch_crossprod(L.stream, ty, yp, c.m, ty, yp, c.m, c.m, c.k, c.k, L.partials,
                                    L.partial_elems, dst));
  return QSK_OK;
}

// Psi as the sketch used it, for the core solve: the matrix-core path's
// staging holds exactly those values (rounded to the operand format); when
// the update kernels generated Psi in place, it is regenerated into the
// staging buffer once (the FP64 matrix-core product reads it there).
static qsk_status stage_psi_for_solve(qsk_ctx *ctx, hipStream_t st) {
  const qsk_config &c = ctx->cfg;
  if (!ctx->psi_staged && ctx->use_mfma && ctx->stage.psi && ctx->mode != qsk::MODE_F64) {
    qsk::SketchArgs sa{};
    sa.stream = st; sa.mode = ctx->mode; sa.l = c.l; sa.m = c.m; sa.k = c.k;
    sa.rad = c.embedding == QSK_RADEMACHER; sa.k0 = ctx->k0; sa.k1 = ctx->k1;
    HIPCHK(ctx, qsk::stage_psi(sa, ctx->stage));
    ctx->psi_staged = true;
  }
  return QSK_OK;
}

// The QB stage's launches on lane L (arguments checked, sketch prepared).
// The optimistic run makes no host synchronisation: its results, status
// and kappa estimates are read by qb_collect.  The careful run reads the
// status after each factorisation.
static qsk_status qb_enqueue(qsk_ctx *ctx, const QbLane &L, qsk_rangefinder rf, double *const Q[4],
                             int64_t ldq, double *const X[4], int64_t ldx, bool opt, QbRun *run) {
  const qsk_config &c = ctx->cfg;
  const int gs = rf == QSK_PSEUDO_SVD_GS;
  if (gs) rf = QSK_PSEUDO_SVD;
  run->rf = rf;
  hipStream_t st = L.stream;
  const int k = c.k, l = c.l;
  const int64_t m = c.m, n = c.n;
  const int ty = ctx->mode == qsk::MODE_F64 ? 0 : 1;
  const int complex_only = rf == QSK_PSEUDO_QR;
  const size_t kk = (size_t)k * k * 4;
  SmallStatus hs{};
  int flags = 0;
  bool kappa0 = false;                 // kappa of H0 launched on `side`

  if (opt) HIPCHK(ctx, qsk::launch_status_reset(st, L.status, 0));
  const void *yp[4];
  for (int p = 0; p < 4; ++p) yp[p] = (const char *)ctx->y + (size_t)p * m * k * ctx->ts;

  // ---- CholeskyQR of Y: complex QR of Y_c for pseudo-QR (the j-part of the
  // quaternion Gram is dropped), quaternion QR for pseudo-SVD.  A Cholesky
  // breakdown switches that pass to a shifted factorisation (Fukaya et al.,
  // shifted CholeskyQR3) and asks for two more clean passes; repeated shifted
  // passes lift an exactly rank-deficient sketch to a full orthonormal basis
  // whose extra directions are arbitrary.
  const void *zsrc[4] = {yp[0], yp[1], yp[2], yp[3]};
  int tz = ty;
  double *gz = slot(L, k, S_G1);
  const double rows_c = complex_only ? 2.0 * m : 4.0 * m;
  int passes = 0, need = 2;
  const int max_passes = 8;
  for (;;) {
    if (passes == 0 && ctx->gram_valid) {
      // Y^* Y of this sketch, kept from the previous finalize
      HIPCHK(ctx, hipMemcpyAsync(gz, slot(ctx, S_YG), kk * 8, hipMemcpyDeviceToDevice, st));
    } else {
      HIPCHK(ctx, qsk::launch_crossprod(st, tz, zsrc, m, tz, zsrc, m, m, k, k, L.partials,
                                        L.partial_elems, gz));
      if (passes == 0) {
        HIPCHK(ctx, hipMemcpyAsync(slot(ctx, S_YG), gz, kk * 8, hipMemcpyDeviceToDevice, st));
        ctx->gram_valid = true;
      }
    }
    HIPCHK(ctx, qsk::launch_chol_inv(st, gz, k, complex_only, 0.0, 1e-13, slot(L, k, S_R),
                                     slot(L, k, S_T), L.status));
    if (!opt) {
      HIPCHK(ctx, hipMemcpyAsync(&hs, L.status, sizeof(hs), hipMemcpyDeviceToHost, st));
      HIPCHK(ctx, hipStreamSynchronize(st));
    }
    ++passes;
    if (hs.fail) {
      if (!(hs.trace > 0.0) || !std::isfinite(hs.trace)) {
        ctx->last_error = "sketch Y is zero or non-finite";
        return QSK_E_NUMERIC;
      }
      const double shift = 11.0 * (rows_c * k + (double)k * (k + 1)) * 0x1p-53 * hs.trace;
      HIPCHK(ctx, qsk::launch_chol_inv(st, gz, k, complex_only, shift, 0.0, slot(L, k, S_R),
                                       slot(L, k, S_T), L.status));
      HIPCHK(ctx, hipMemcpyAsync(&hs, L.status, sizeof(hs), hipMemcpyDeviceToHost, st));
      HIPCHK(ctx, hipStreamSynchronize(st));
      if (hs.fail) {
        ctx->last_error = "Cholesky of the shifted Gram failed";
        return QSK_E_NUMERIC;
      }
      flags |= QSK_FLAG_CHOL_FALLBACK;
      if (need < passes + 2) need = passes + 2;
    }
    if (passes == 1) {
      HIPCHK(ctx, hipMemcpyAsync(slot(L, k, S_RPROD), slot(L, k, S_R), kk * 8, hipMemcpyDeviceToDevice, st));
    } else {
      HIPCHK(ctx, qsk::launch_small_gemm(st, k, slot(L, k, S_R), 0, slot(L, k, S_RPROD), 0, slot(L, k, S_RTMP)));
      HIPCHK(ctx, hipMemcpyAsync(slot(L, k, S_RPROD), slot(L, k, S_RTMP), kk * 8, hipMemcpyDeviceToDevice, st));
    }
    if (passes >= need || passes >= max_passes) break;
    double *ub = L.u[(passes - 1) & 1];
    double *up[4] = {ub, ub + (size_t)m * k, ub + 2 * (size_t)m * k, ub + 3 * (size_t)m * k};
    HIPCHK(ctx, qsk::launch_apply(st, tz, zsrc, m, m, k, slot(L, k, S_T), k, up, m, 1));
    for (int p = 0; p < 4; ++p) zsrc[p] = up[p];
    tz = 0;
    gz = slot(L, k, S_GU);
  }
  // Now H0 (pseudo-QR) or Q_Y (pseudo-SVD) = Z T with G_Z = gz.  (The
  // optimistic run keeps the sticky failure flag of the passes above.)
  if (opt) {
    HIPCHK(ctx, qsk::launch_status_reset(st, L.status, 1));
  } else {
    HIPCHK(ctx, hipMemsetAsync(L.status, 0, sizeof(SmallStatus), st));
  }
  HIPCHK(ctx, hipMemsetAsync(L.kstatus, 0, sizeof(SmallStatus), st));
  if (rf == QSK_PSEUDO_QR) {
    // G0 = H0^* H0 = T^* G_Z T; kappa of the raw factor
    HIPCHK(ctx, qsk::launch_small_gemm(st, k, gz, 0, slot(L, k, S_T), 0, slot(L, k, S_TMP)));
    HIPCHK(ctx, qsk::launch_small_gemm(st, k, slot(L, k, S_T), 1, slot(L, k, S_TMP), 0, slot(L, k, S_G0)));
    HIPCHK(ctx, hipMemcpyAsync(slot(L, k, S_GK0), slot(L, k, S_G0), kk * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(ctx, hipEventRecord(L.ev_fork, st));
    HIPCHK(ctx, hipStreamWaitEvent(L.side, L.ev_fork, 0));
    HIPCHK(ctx, qsk::launch_kappa(L.side, k, slot(L, k, S_GK0), L.kwork, 1, L.kstatus));
    HIPCHK(ctx, hipEventRecord(L.ev_join, L.side));
    kappa0 = true;
    // correction steps (eq. CondNumReductionIter) in the k x k space: with
    // H_j = H0 C_j and G_j = H_j^* H_j, H_{j+1} = (1 - eps) H_j + eps (H_j^dagger)^*
    // = H_j M_j with M_j = (1 - eps) I + eps G_j^{-1}  ((H^dagger)^* = H G^{-1});
    // C_{j+1} = C_j M_j, G_{j+1} = M_j^* G_j M_j.
    HIPCHK(ctx, qsk::launch_identity(st, k, slot(L, k, S_C)));
    for (int j = 0; j < c.n_correction; ++j) {
      HIPCHK(ctx, qsk::launch_chol_inv(st, slot(L, k, S_G0), k, 0, 0.0, 1e-13, slot(L, k, S_CR),
                                       slot(L, k, S_CT), L.status));
      int fail = 0;
      if (!opt) {
        HIPCHK(ctx, hipMemcpyAsync(&fail, &L.status->fail, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
      }
      if (fail) {
        flags |= QSK_FLAG_RANK_DEFICIENT;      // G_j singular: no further correction
        break;
      }
      HIPCHK(ctx, qsk::launch_small_gemm(st, k, slot(L, k, S_CT), 0, slot(L, k, S_CT), 1, slot(L, k, S_GI)));
      HIPCHK(ctx, qsk::launch_power_m(st, k, slot(L, k, S_GI), j, c.n_power, ctx->k0, ctx->k1,
                                      slot(L, k, S_M), L.status));
      HIPCHK(ctx, qsk::launch_small_gemm(st, k, slot(L, k, S_C), 0, slot(L, k, S_M), 0, slot(L, k, S_TMP)));
      HIPCHK(ctx, hipMemcpyAsync(slot(L, k, S_C), slot(L, k, S_TMP), kk * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(ctx, qsk::launch_small_gemm(st, k, slot(L, k, S_G0), 0, slot(L, k, S_M), 0, slot(L, k, S_TMP)));
      HIPCHK(ctx, qsk::launch_small_gemm(st, k, slot(L, k, S_M), 1, slot(L, k, S_TMP), 0, slot(L, k, S_G0)));
    }
  } else {
    // G_L = R_Y R_Y^*
    HIPCHK(ctx, qsk::launch_small_gemm(st, k, slot(L, k, S_RPROD), 0, slot(L, k, S_RPROD), 1, slot(L, k, S_TMP)));
    HIPCHK(ctx, qsk::launch_psvd_select(st, k, slot(L, k, S_TMP), ctx->k0, ctx->k1, slot(L, k, S_C),
                                        L.work, L.status, gs));
  }
  HIPCHK(ctx, qsk::launch_small_gemm(st, k, slot(L, k, S_T), 0, slot(L, k, S_C), 0, slot(L, k, S_F)));
  // kappa(Q) from G_Q = F^* G_Z F
  HIPCHK(ctx, qsk::launch_small_gemm(st, k, gz, 0, slot(L, k, S_F), 0, slot(L, k, S_TMP2)));
  HIPCHK(ctx, qsk::launch_small_gemm(st, k, slot(L, k, S_F), 1, slot(L, k, S_TMP2), 0, slot(L, k, S_GH)));
  HIPCHK(ctx, hipEventRecord(L.ev_fork2, st));
  HIPCHK(ctx, hipStreamWaitEvent(L.side2, L.ev_fork2, 0));
  HIPCHK(ctx, qsk::launch_kappa(L.side2, k, slot(L, k, S_GH), L.kwork2, 0, L.kstatus));
  HIPCHK(ctx, hipEventRecord(L.ev_join2, L.side2));
  HIPCHK(ctx, qsk::launch_apply(st, tz, zsrc, m, m, k, slot(L, k, S_F), k, Q, ldq));

  // ---- core solve X = (Psi Q)^dagger W (Alg. 2 through the normal form of
  // a CholeskyQR2 factorisation of P = Psi Q); skipped when X is NULL
  if (X) {
  double *pp[4], *p1[4], *sp[4];
  for (int p = 0; p < 4; ++p) {
    pp[p] = L.pbuf + (size_t)p * l * k;
    p1[p] = L.p1buf + (size_t)p * l * k;
    sp[p] = L.sbuf + (size_t)p * l * k;
  }
  {
    const qsk_status ss = stage_psi_for_solve(ctx, st);
    if (ss != QSK_OK) return ss;
  }
  const int psi_st_type = !ctx->psi_staged ? 0 : (ctx->mode == qsk::MODE_F32 ? 2 : 1);
  HIPCHK(ctx, qsk::launch_psi_apply(st, ctx->emode, c.embedding == QSK_RADEMACHER, ctx->k0, ctx->k1, l,
                                    m, Q, ldq, k, L.partials, L.partial_elems, pp, l,
                                    ctx->stage.psi, psi_st_type, ctx->stage.MP,
                                    (int64_t)ctx->stage.LP * ctx->stage.MP));
  SmallStatus ps{};
  HIPCHK(ctx, qsk::launch_crossprod(st, 0, (const void *const *)pp, l, 0, (const void *const *)pp, l,
                                    l, k, k, L.partials, L.partial_elems, slot(L, k, S_GP)));
  HIPCHK(ctx, qsk::launch_chol_inv(st, slot(L, k, S_GP), k, 0, 0.0, 1e-13, slot(L, k, S_RP),
                                   slot(L, k, S_TP1), L.status));
  if (!opt) {
    HIPCHK(ctx, hipMemcpyAsync(&ps, L.status, sizeof(ps), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
  }
  bool have_sstar = false;
  if (ps.fail) {
    // (Psi Q)^*(Psi Q) singular: minimum-norm least squares through a Jacobi
    // SVD of Psi Q (the reading of Alg. 2's backslash for a rank-deficient
    // system).
    flags |= QSK_FLAG_RANK_DEFICIENT;
    HIPCHK(ctx, qsk::launch_pinv_sstar(st, l, k, pp, l, 1e-13, L.pinv_work, sp, l));
    have_sstar = true;
  } else {
    // R^{-1} = TP1 alone when kappa_F(R_1)^2 = trace(G_P) ||TP1||_F^2 (an
    // upper bound on kappa_2(P)^2) is small enough for the normal-form
    // solve below; else a second CholeskyQR pass, R^{-1} = TP1 TP2.  The
    // optimistic run decides on the device: the second pass's launches are
    // given the gate status and return at once when the gate passes.
    HIPCHK(ctx, qsk::launch_core_gate(st, k, slot(L, k, S_TP1), slot(L, k, S_TPT), L.status));
    bool second = true;
    const SmallStatus *gate = nullptr;
    if (opt) {
      gate = L.status;
    } else {
      HIPCHK(ctx, hipMemcpyAsync(&ps, L.status, sizeof(ps), hipMemcpyDeviceToHost, st));
      HIPCHK(ctx, hipStreamSynchronize(st));
      second = !(ps.gate > 0.0 && ps.gate <= qsk::ONE_PASS_KAPPA2);
    }
    if (second) {
      HIPCHK(ctx, qsk::launch_apply(st, 0, (const void *const *)pp, l, l, k, slot(L, k, S_TP1), k, p1, l, 1,
                                    gate));
      HIPCHK(ctx, qsk::launch_crossprod(st, 0, (const void *const *)p1, l, 0, (const void *const *)p1,
                                        l, l, k, k, L.partials, L.partial_elems, slot(L, k, S_GP), gate));
      HIPCHK(ctx, qsk::launch_chol_inv(st, slot(L, k, S_GP), k, 0, 0.0, 1e-13, slot(L, k, S_RP),
                                       slot(L, k, S_TP2), L.status, gate));
      if (!opt) {
        HIPCHK(ctx, hipMemcpyAsync(&ps, L.status, sizeof(ps), hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
      }
      if (ps.fail) {
        flags |= QSK_FLAG_RANK_DEFICIENT;
        HIPCHK(ctx, qsk::launch_pinv_sstar(st, l, k, pp, l, 1e-13, L.pinv_work, sp, l));
        have_sstar = true;
      } else {
        HIPCHK(ctx, qsk::launch_small_gemm(st, k, slot(L, k, S_TP1), 0, slot(L, k, S_TP2), 0, slot(L, k, S_TPT),
                                           gate));
      }
    }
  }
  // Z = R^{-1} R^{-*} with R^{-1} = TPT; S^* = P Z; X = S W = (S^*)^* W
  if (!have_sstar) {
    HIPCHK(ctx, qsk::launch_small_gemm(st, k, slot(L, k, S_TPT), 0, slot(L, k, S_TPT), 1, slot(L, k, S_Z)));
    HIPCHK(ctx, qsk::launch_apply(st, 0, (const void *const *)pp, l, l, k, slot(L, k, S_Z), k, sp, l));
  }
  const void *wp[4];
  for (int p = 0; p < 4; ++p) wp[p] = (const char *)ctx->w + (size_t)p * l * n * ctx->ts;
  HIPCHK(ctx, qsk::launch_crossprod_planar(st, sp, l, ty, wp, l, l, k, (int)n, X, ldx));
  }

  // join the side streams (kappa estimates) into the lane's stream before
  // their results are read (the two kernels write different fields of kstatus)
  if (kappa0) HIPCHK(ctx, hipStreamWaitEvent(st, L.ev_join, 0));
  HIPCHK(ctx, hipStreamWaitEvent(st, L.ev_join2, 0));
  run->passes = passes;
  run->flags = flags;
  run->kappa0 = kappa0;
  return QSK_OK;
}

// Status and kappa estimates of an enqueued QB stage, read once its lane
// has drained; the optimistic run returns QSK_RETRY_CAREFUL when any
// factorisation failed.
static qsk_status qb_collect(qsk_ctx *ctx, const QbLane &L, const QbRun &run, qsk_report *report,
                             bool opt) {
  hipStream_t st = L.stream;
  SmallStatus ks{}, hs2{};
  HIPCHK(ctx, hipMemcpyAsync(&ks, L.kstatus, sizeof(ks), hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(&hs2, L.status, sizeof(hs2), hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  if (opt && hs2.fail_any) return QSK_RETRY_CAREFUL;
  if (report) {
    qsk_report r{};
    r.kappa = ks.kappa;
    r.kappa_initial = run.rf == QSK_PSEUDO_QR ? ks.kappa_initial : ks.kappa;
    r.n_eps = hs2.n_eps;
    for (int i = 0; i < 8; ++i) r.eps[i] = hs2.eps[i];
    r.t_bad = hs2.t_bad;
    r.flags = run.flags | hs2.flags;
    r.passes = run.passes;
    r.columns_seen = ctx->columns_seen;
    r.orth_defect = run.rf == QSK_PSEUDO_SVD ? ks.orth_defect : 0.0;
    *report = r;
  }
  return QSK_OK;
}

static qsk_status finalize_impl(qsk_ctx *ctx, qsk_rangefinder rf, double *const Q[4], int64_t ldq,
                                double *const X[4], int64_t ldx, qsk_report *report, bool opt) {
  qsk_status r = qb_check(ctx, rf, Q, ldq, X, ldx);
  if (r == QSK_OK) r = qb_prepare(ctx);
  if (r != QSK_OK) return r;
  const QbLane L = lane0(ctx);
  QbRun run;
  r = qb_enqueue(ctx, L, rf, Q, ldq, X, ldx, opt, &run);
  if (r != QSK_OK) return r;
  return qb_collect(ctx, L, run, report, opt);
}

// The second QB lane, with the sizes of the context's own workspace.
static qsk_status alloc_lane1(qsk_ctx *ctx) {
  if (ctx->lane1_ready) return QSK_OK;
  const int64_t m = ctx->cfg.m, k = ctx->cfg.k, l = ctx->cfg.l;
  const size_t kk = (size_t)k * k * 4;
  QbLane &L = ctx->lane1;
  bool ok = true;
  ok = ok && alloc((void **)&L.u[0], 4 * (size_t)m * k * 8);
  ok = ok && alloc((void **)&L.u[1], 4 * (size_t)m * k * 8);
  ok = ok && alloc((void **)&L.small, S_COUNT * kk * 8);
  ok = ok && alloc((void **)&L.work, (12 * kk + 64 * (size_t)k) * 8);
  L.partial_elems = ctx->partial_elems;
  ok = ok && alloc((void **)&L.partials, (size_t)L.partial_elems * 8);
  ok = ok && alloc((void **)&L.pbuf, 4 * (size_t)l * k * 8);
  ok = ok && alloc((void **)&L.p1buf, 4 * (size_t)l * k * 8);
  ok = ok && alloc((void **)&L.sbuf, 4 * (size_t)l * k * 8);
  ok = ok && alloc((void **)&L.pinv_work, 4 * (size_t)(l + k) * k * 8);
  ok = ok && alloc((void **)&L.status, sizeof(SmallStatus));
  ok = ok && alloc((void **)&L.kstatus, sizeof(SmallStatus));
  ok = ok && alloc((void **)&L.kwork, kk * 8);
  ok = ok && alloc((void **)&L.kwork2, kk * 8);
  // one stream of its own: its kappa estimates run on the first lane's side
  // streams (see qsketch_finalize_pair)
  ok = ok && hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess;
  for (hipEvent_t *e : {&L.ev_fork, &L.ev_join, &L.ev_fork2, &L.ev_join2, &ctx->ev_pair_fork,
                        &ctx->ev_pair_join})
    ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_lane(L);
    if (ctx->ev_pair_fork) (void)hipEventDestroy(ctx->ev_pair_fork);
    if (ctx->ev_pair_join) (void)hipEventDestroy(ctx->ev_pair_join);
    ctx->ev_pair_fork = ctx->ev_pair_join = nullptr;
    ctx->last_error = "out of device memory (or streams) for the second QB lane";
    return QSK_E_NOMEM;
  }
  ctx->lane1_ready = true;
  return QSK_OK;
}

static bool planes_overlap(double *const A[4], double *const B[4]) {
  if (!A || !B) return false;
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q)
      if (A[p] == B[q]) return true;
  return false;
}

qsk_status qsketch_finalize(qsk_ctx *ctx, qsk_rangefinder rf, double *const Q[4], int64_t ldq,
                            double *const X[4], int64_t ldx, qsk_report *report) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  const qsk_status r = finalize_impl(ctx, rf, Q, ldq, X, ldx, report, true);
  if (r != QSK_RETRY_CAREFUL) return r;
  return finalize_impl(ctx, rf, Q, ldq, X, ldx, report, false);
}

qsk_status qsketch_finalize_pair(qsk_ctx *ctx, qsk_rangefinder rf_a, double *const Qa[4], int64_t ldqa,
                                 double *const Xa[4], int64_t ldxa, qsk_report *report_a,
                                 qsk_rangefinder rf_b, double *const Qb[4], int64_t ldqb,
                                 double *const Xb[4], int64_t ldxb, qsk_report *report_b) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  qsk_status r = qb_check(ctx, rf_a, Qa, ldqa, Xa, ldxa);
  if (r == QSK_OK) r = qb_check(ctx, rf_b, Qb, ldqb, Xb, ldxb);
  if (r != QSK_OK) return r;
  if (planes_overlap(Qa, Qb) || planes_overlap(Xa, Xb) || planes_overlap(Qa, Xb) ||
      planes_overlap(Xa, Qb))
    return fail_arg(ctx, "the two results share an output plane");
  // a pseudo-QR stage goes to the context stream and the calling thread:
  // its early kappa of H0 and later kappa of Q then share the side streams
  // with a pseudo-SVD stage's late kappa of Q as arranged below (the other
  // way round the pair took 4.5 instead of 4.0 ms at m = 20000, k = 100)
  if (rf_a != QSK_PSEUDO_QR && rf_b == QSK_PSEUDO_QR) {
    std::swap(rf_a, rf_b);
    std::swap(Qa, Qb);
    std::swap(ldqa, ldqb);
    std::swap(Xa, Xb);
    std::swap(ldxa, ldxb);
    std::swap(report_a, report_b);
  }
  r = alloc_lane1(ctx);
  if (r == QSK_OK) r = qb_prepare(ctx);
  if (r != QSK_OK) return r;
  const QbLane La = lane0(ctx);
  // The second stage's kappa estimates go to the first stage's side streams,
  // crosswise: pseudo-QR launches its kappa of H0 early on `side` and its
  // kappa of Q later on `side2`, pseudo-SVD only a late kappa of Q on `side2`,
  // so the crossing keeps the two late estimates apart.  Streams beyond the
  // device's hardware queues would share a queue, where a stream waiting for
  // the other stage holds back every launch queued behind it.
  QbLane Lb = ctx->lane1;
  Lb.side = La.side2;
  Lb.side2 = La.side;
  // what both stages read and would otherwise write first: the Gram of Y
  // and, for a core solve, the staged Psi (on the context stream, before
  // the fork)
  if (!ctx->gram_valid) {
    r = y_gram(ctx, La, slot(ctx, S_YG));
    if (r != QSK_OK) return r;
    ctx->gram_valid = true;
  }
  if (Xa || Xb) {
    r = stage_psi_for_solve(ctx, La.stream);
    if (r != QSK_OK) return r;
  }
  HIPCHK(ctx, hipEventRecord(ctx->ev_pair_fork, La.stream));
  HIPCHK(ctx, hipStreamWaitEvent(Lb.stream, ctx->ev_pair_fork, 0));
  // The two stages are launched from two host threads: a stage is about a
  // hundred short launches, and launched one after the other the second
  // stage would reach the device only when the host has issued the first.
  // The optimistic launches write no host state of the context (the Gram
  // and Psi are ready; a launch failure is recorded under err_mu).
  // The worker makes the context's device current first (HIP's current
  // device is per thread); if no thread can be started, the second stage is
  // launched after the first from this thread.
  QbRun run_a, run_b;
  qsk_status rb_launch = QSK_OK;
  auto launch_b = [&] {
    const hipError_t e = hipSetDevice(ctx->device);
    rb_launch = e == hipSuccess ? qb_enqueue(ctx, Lb, rf_b, Qb, ldqb, Xb, ldxb, true, &run_b)
                                : hip_fail(ctx, e, "hipSetDevice in the second QB lane");
  };
  std::thread tb;
  bool threaded = true;
  try {
    tb = std::thread(launch_b);
  } catch (...) {
    threaded = false;
  }
  r = qb_enqueue(ctx, La, rf_a, Qa, ldqa, Xa, ldxa, true, &run_a);
  if (threaded) tb.join();
  else launch_b();
  if (r == QSK_OK) r = rb_launch;
  // the context stream continues after both stages
  HIPCHK(ctx, hipEventRecord(ctx->ev_pair_join, Lb.stream));
  HIPCHK(ctx, hipStreamWaitEvent(La.stream, ctx->ev_pair_join, 0));
  if (r != QSK_OK) return r;
  qsk_status ra = qb_collect(ctx, La, run_a, report_a, true);
  qsk_status rb = qb_collect(ctx, Lb, run_b, report_b, true);
  // a stage whose optimistic run failed a factorisation is run again, the
  // careful way, on the context stream
  if (ra == QSK_RETRY_CAREFUL) ra = finalize_impl(ctx, rf_a, Qa, ldqa, Xa, ldxa, report_a, false);
  if (rb == QSK_RETRY_CAREFUL) rb = finalize_impl(ctx, rf_b, Qb, ldqb, Xb, ldxb, report_b, false);
  return ra != QSK_OK ? ra : rb;
}

qsk_status qsketch_project(qsk_ctx *ctx, double *const Q[4], int64_t ldq, int64_t col0, int64_t ncols,
                           const void *const planes[4], int64_t ld, double *const X[4], int64_t ldx) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  const qsk_config &c = ctx->cfg;
  qsk_status st = check_block(ctx, col0, ncols, planes, ld);
  if (st != QSK_OK) return st;
  if (!Q || !X) return fail_arg(ctx, "Q/X NULL");
  for (int p = 0; p < 4; ++p)
    if (!Q[p] || !X[p]) return fail_arg(ctx, "NULL Q/X plane");
  if (ldq < c.m || ldx < c.k) return fail_arg(ctx, "leading dimension too small");
  const size_t es = c.input_dtype == QSK_F64 ? 8 : c.input_dtype == QSK_F32 ? 4 : 2;
  const void *b[4];
  for (int p = 0; p < 4; ++p) b[p] = planes[p];
  if (c.pure) {
    // the real plane of a pure quaternion block is zero: a zeroed plane of
    // the block's shape stands in for it
    const size_t need = ((size_t)(ncols - 1) * ld + c.m) * es;
    if (need > ctx->zero_plane_bytes) {
      const qsk_status gs = grow_buffer(ctx, &ctx->zero_plane, &ctx->zero_plane_bytes, need);
      if (gs != QSK_OK) return gs;
      HIPCHK(ctx, hipMemsetAsync(ctx->zero_plane, 0, need, ctx->stream));
    }
    b[0] = ctx->zero_plane;
  }
  const int64_t nch = qsk::project_chunks(c.m, c.k, ncols);
  const size_t pneed = nch > 1 ? (size_t)nch * c.k * ncols * 4 * 8 : 0;
  {
    const qsk_status gs = grow_buffer(ctx, (void **)&ctx->proj_part, &ctx->proj_part_bytes, pneed);
    if (gs != QSK_OK) return gs;
  }
  double *xo[4];
  for (int p = 0; p < 4; ++p) xo[p] = X[p] + col0 * ldx;
  HIPCHK(ctx, qsk::launch_project(ctx->stream, Q, ldq, c.input_dtype, b, ld, c.m, c.k, ncols, xo, ldx,
                                  ctx->proj_part, (int64_t)(ctx->proj_part_bytes / 8)));
  return QSK_OK;
}

qsk_status qsketch_project_noalloc(qsk_ctx *ctx, double *const Q[4], int64_t ldq, int64_t col0,
                                   int64_t ncols, const void *const planes[4], int64_t ld,
                                   double *const X[4], int64_t ldx) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  const qsk_config &c = ctx->cfg;
  qsk_status st = check_block(ctx, col0, ncols, planes, ld);
  if (st != QSK_OK) return st;
  if (!Q || !X) return fail_arg(ctx, "Q/X NULL");
  for (int p = 0; p < 4; ++p)
    if (!Q[p] || !X[p]) return fail_arg(ctx, "NULL Q/X plane");
  if (ldq < c.m || ldx < c.k) return fail_arg(ctx, "leading dimension too small");
  const size_t es = c.input_dtype == QSK_F64 ? 8 : c.input_dtype == QSK_F32 ? 4 : 2;
  unsigned char *base = (unsigned char *)ctx->noalloc_scratch;
  size_t used = 0;
  const void *b[4];
  for (int p = 0; p < 4; ++p) b[p] = planes[p];
  if (c.pure) {
    // the real plane of a pure quaternion block is zero: a zeroed stretch of
    // the scratch of the block's shape stands in for it (cleared on every
    // call: the previous call may have left partial sums there)
    const size_t need = ((size_t)(ncols - 1) * ld + c.m) * es;
    const size_t rounded = (need + 255) / 256 * 256;
    if (rounded > QSK_NOALLOC_SCRATCH_BYTES)
      return fail_arg(ctx, "qsketch_project_noalloc: a pure-quaternion block needs a zero real plane of "
                           "((ncols - 1) ld + m) elements, more than the 32 MiB static scratch holds");
    HIPCHK(ctx, qsk::launch_scale(ctx->stream, 0, base, (int64_t)(rounded / 8), 0.0));
    b[0] = base;
    used = rounded;
  }
  // partial sums of the split contraction in the rest of the scratch (the
  // split shrinks to what fits, down to none)
  double *part = (double *)(base + used);
  const int64_t part_elems = (int64_t)((QSK_NOALLOC_SCRATCH_BYTES - used) / 8);
  double *xo[4];
  for (int p = 0; p < 4; ++p) xo[p] = X[p] + col0 * ldx;
  HIPCHK(ctx, qsk::launch_project(ctx->stream, Q, ldq, c.input_dtype, b, ld, c.m, c.k, ncols, xo, ldx, part,
                                  part_elems));
  return QSK_OK;
}

qsk_status qsketch_truncate(qsk_ctx *ctx, double *const Q[4], int64_t ldq, double *const X[4], int64_t ldx,
                            int32_t r, double *const HU[4], int64_t ldh, double *sigma,
                            double *const V[4], int64_t ldv) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  const qsk_config &c = ctx->cfg;
  const int k = c.k;
  const int64_t m = c.m, n = c.n;
  if (r < 1 || r > k) return fail_arg(ctx, "need 1 <= r <= k");
  if (!Q || !X || !HU || !V || !sigma) return fail_arg(ctx, "NULL argument");
  for (int p = 0; p < 4; ++p)
    if (!Q[p] || !X[p] || !HU[p] || !V[p]) return fail_arg(ctx, "NULL plane");
  if (ldq < m || ldx < k || ldh < m || ldv < n) return fail_arg(ctx, "leading dimension too small");
  hipStream_t st = ctx->stream;
  // Z = X^* (n x k); the Gram Z^* Z = X X^* = U Sigma^2 U^*
  const size_t need = 4 * (size_t)n * k * 8;
  {
    const qsk_status gs = grow_buffer(ctx, (void **)&ctx->xt, &ctx->xt_bytes, need);
    if (gs != QSK_OK) return gs;
  }
  double *z[4];
  for (int p = 0; p < 4; ++p) z[p] = ctx->xt + (size_t)p * n * k;
  HIPCHK(ctx, qsk::launch_conj_transpose(st, X, ldx, n, k, z, n));
  HIPCHK(ctx, qsk::launch_crossprod(st, 0, (const void *const *)z, n, 0, (const void *const *)z, n, n, k, k,
                                    ctx->partials, ctx->partial_elems, slot(ctx, S_TMP)));
  HIPCHK(ctx, qsk::launch_herm_eig(st, k, slot(ctx, S_TMP), ctx->work, ctx->status));
  HIPCHK(ctx, qsk::launch_trunc_select(st, ctx->work, k, r, slot(ctx, S_C), slot(ctx, S_F), sigma));
  // H U_r (m x r) and V_r = X^* U_r Sigma_r^{-1} (n x r)
  HIPCHK(ctx, qsk::launch_apply(st, 0, (const void *const *)Q, ldq, m, k, slot(ctx, S_C), r, HU, ldh));
  HIPCHK(ctx, qsk::launch_apply(st, 0, (const void *const *)z, n, n, k, slot(ctx, S_F), r, V, ldv));
  return QSK_OK;
}

qsk_status qsketch_rel_error(qsk_ctx *ctx, const void *const A[4], int64_t lda, double *const Q[4],
                             int64_t ldq, double *const X[4], int64_t ldx, double *err) {
  if (!ctx) return QSK_E_ARG;
  if (ctx->poisoned) return QSK_E_STATE;
  const qsk_config &c = ctx->cfg;
  if (!A || !Q || !X || !err || lda < c.m) return fail_arg(ctx, "bad argument to rel_error");
  HIPCHK(ctx, hipMemsetAsync(ctx->err_acc, 0, 16, ctx->stream));
  HIPCHK(ctx, qsk::launch_error(ctx->stream, c.input_dtype, A, lda, c.pure, c.m, c.n, Q, ldq, X, ldx,
                                c.k, ctx->err_acc));
  double h[2];
  HIPCHK(ctx, hipMemcpyAsync(h, ctx->err_acc, 16, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  *err = h[1] > 0 ? std::sqrt(h[0] / h[1]) : 0.0;
  return QSK_OK;
}

}  // extern "C"
