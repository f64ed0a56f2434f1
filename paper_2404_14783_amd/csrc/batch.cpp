// Batches of independent problems behind qsketch_batch_* (include/qsketch.h):
// every problem's one-pass approximation (Alg. 4) with each step launched
// once for all problems.  The per-problem arithmetic is that of qsketch.cpp
// (same kernels, same argument structs); only the launches are grouped:
// a table of per-problem argument structs goes to the device and each block
// finds its problem from the prefix sums of the block counts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/qsketch.h"
#include "qsk_kernels.hpp"

namespace qsk {

void *arena_push(ArgArena &a, hipStream_t st, const void *src, size_t bytes) {
  const size_t off = (a.used + 255) & ~(size_t)255;
  if (off + bytes > a.cap) return nullptr;
  std::memcpy(a.host + off, src, bytes);
  if (!a.defer && hipMemcpyAsync(a.dev + off, a.host + off, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
    return nullptr;
  a.used = off + bytes;
  return a.dev + off;
}

}  // namespace qsk

namespace {

using qsk::GroupRef;
using qsk::SmallStatus;

// k x k slots per problem (same roles as in the single-problem driver)
enum BSlot { B_G1 = 0, B_GU, B_R, B_T, B_RPROD, B_RTMP, B_G0, B_TMP, B_C, B_F, B_GP, B_RP, B_TP1,
             B_TP2, B_TPT, B_Z, B_CR, B_CT, B_GI, B_M, B_TMP2, B_GH, B_GK0, B_COUNT };

struct Prob {
  qsk_config cfg{};
  int64_t m = 0, n = 0;
  int k = 0, l = 0;
  uint32_t k0 = 0, k1 = 0;
  float *y = nullptr, *w = nullptr;
  double *u[2] = {nullptr, nullptr};
  double *small = nullptr, *work = nullptr, *kwork = nullptr, *partials = nullptr;
  int64_t partial_elems = 0;
  double *pbuf = nullptr, *p1buf = nullptr, *sbuf = nullptr, *pinv_work = nullptr;
  float *wpart = nullptr;                 // partial sums of a split W product
  int64_t wpart_bytes = 0;
  qsk::MfmaStage stage{};
  // per-run state
  int passes = 0, need = 2, flags = 0;
  bool z_is_u = false;
  double *zsrc[4] = {nullptr, nullptr, nullptr, nullptr};
  double *gz = nullptr;
  double *slot(int s) const { return small + (size_t)s * k * k * 4; }
};

}  // namespace

struct qsk_batch {
  int count = 0;
  hipStream_t stream = nullptr, side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<Prob> p;
  int mode = 0, nmt = 4, nj = 4;       // tile shapes of the grouped sketch launches
  int wblocks = qsk::BATCH_W_BLOCKS;   // W blocks the row splits aim at
  void *pool = nullptr;
  SmallStatus *status = nullptr, *kstatus = nullptr;
  double *err_acc = nullptr;
  qsk::ArgArena arena{};
  bool poisoned = false;
  bool numeric_fail = false;
  std::string last_error;
  // execution: 0 careful (a host check after every factorisation), 1
  // optimistic stream-ordered, 2 optimistic as one captured graph per
  // rangefinder (replayed while the caller's pointers stay the same)
  int exec_mode = 2;
  hipStream_t gstream = nullptr;       // the graphs' stream (the caller's may be the null stream)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  qsk::ArgArena garena[2] = {};        // argument tables of each graph, written once per capture
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  std::vector<uintptr_t> gkey[2];
};

namespace {

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }
int64_t rup_i(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// Tile shapes of the grouped sketch launches: row tiles of W per block
// (13 only with bf16 operands) and column tiles of Y per block.
const int kNmt[4] = {4, 7, 8, 13}, kNj[2] = {4, 7};
// the largest of rup(x, 16 t) over the first n tile counts t
int64_t max_pad(int64_t x, const int *t, int n) {
  int64_t r = 0;
  for (int i = 0; i < n; ++i) r = std::max(r, rup_i(x, 16 * (int64_t)t[i]));
  return r;
}

qsk_status bfail(qsk_batch *b, hipError_t e, const char *where) {
  b->poisoned = true;
  b->last_error = std::string(where) + ": " + hipGetErrorString(e);
  return QSK_E_HIP;
}

#define BCHK(b, expr)                                      \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return bfail((b), e_, #expr);    \
  } while (0)

// Push per-problem argument structs and the prefix of their block counts.
template <typename A>
bool push_group(qsk_batch *b, const std::vector<A> &args, const std::vector<int64_t> &blocks,
                GroupRef *g, int64_t *total) {
  std::vector<int64_t> pre(args.size() + 1, 0);
  for (size_t i = 0; i < args.size(); ++i) pre[i + 1] = pre[i] + blocks[i];
  g->tab = qsk::arena_push(b->arena, b->stream, args.data(), args.size() * sizeof(A));
  g->prefix = (const int64_t *)qsk::arena_push(b->arena, b->stream, pre.data(), pre.size() * sizeof(int64_t));
  g->count = (int)args.size();
  *total = pre.back();
  return g->tab && g->prefix;
}

qsk_status arena_full(qsk_batch *b) {
  b->poisoned = true;
  b->last_error = "argument arena exhausted";
  return QSK_E_HIP;
}

// C_i = opA(A_i) opB(B_i) over the problems in ids; slots given as
// functions of the problem.
template <typename FA, typename FB, typename FC>
qsk_status gemm_all(qsk_batch *b, hipStream_t st, const std::vector<int> &ids, FA fa, int opa, FB fb,
                    int opb, FC fc) {
  if (ids.empty()) return QSK_OK;
  std::vector<qsk::GemmArgs> a(ids.size());
  std::vector<int64_t> nb(ids.size());
  for (size_t i = 0; i < ids.size(); ++i) {
    const Prob &q = b->p[ids[i]];
    a[i].k = q.k; a[i].a = fa(q); a[i].opa = opa; a[i].b = fb(q); a[i].opb = opb; a[i].c = fc(q);
    a[i].gx = (q.k + 15) / 16; a[i].gy = a[i].gx;
    nb[i] = (int64_t)a[i].gx * a[i].gy;
  }
  GroupRef g;
  int64_t tot;
  if (!push_group(b, a, nb, &g, &tot)) return arena_full(b);
  BCHK(b, qsk::launch_gemm_k(st, a[0], g, tot));
  return QSK_OK;
}

template <typename FA, typename FC>
qsk_status copy_all(qsk_batch *b, const std::vector<int> &ids, FA fa, FC fc) {
  if (ids.empty()) return QSK_OK;
  std::vector<qsk::GemmArgs> a(ids.size());
  std::vector<int64_t> nb(ids.size(), 1);
  for (size_t i = 0; i < ids.size(); ++i) {
    const Prob &q = b->p[ids[i]];
    a[i].k = q.k; a[i].a = fa(q); a[i].c = fc(q); a[i].gx = 1; a[i].gy = 1;
  }
  GroupRef g;
  int64_t tot;
  if (!push_group(b, a, nb, &g, &tot)) return arena_full(b);
  BCHK(b, qsk::launch_copy_small_k(b->stream, a[0], g, (int)ids.size()));
  return QSK_OK;
}

// Cholesky (+ inverse) of the k x k matrices g(q) into r(q), t(q); statuses
// per problem.  only_failed: the shifted retry of the problems whose last
// factorisation failed.
template <typename FG, typename FR, typename FT, typename FS>
qsk_status chol_all(qsk_batch *b, const std::vector<int> &ids, FG fg, int complex_only, FS fshift,
                    double tol, FR fr, FT ft, int only_failed) {
  if (ids.empty()) return QSK_OK;
  std::vector<qsk::CholArgs> a(ids.size());
  std::vector<int64_t> one(ids.size(), 1), kb(ids.size());
  for (size_t i = 0; i < ids.size(); ++i) {
    const Prob &q = b->p[ids[i]];
    a[i].g = fg(q); a[i].k = q.k; a[i].complex_only = complex_only; a[i].shift = fshift(ids[i]);
    a[i].tol = tol; a[i].r = fr(q); a[i].t = ft(q); a[i].status = b->status + ids[i];
    a[i].only_failed = only_failed; a[i].gx = q.k; a[i].gy = 1;
    kb[i] = q.k;
  }
  GroupRef g1, g2;
  int64_t t1, t2;
  if (!push_group(b, a, one, &g1, &t1) || !push_group(b, a, kb, &g2, &t2)) return arena_full(b);
  BCHK(b, qsk::launch_chol_k(b->stream, a[0], g1, (int)ids.size()));
  BCHK(b, qsk::launch_triinv_k(b->stream, a[0], g2, t2));
  return QSK_OK;
}

// Rows per K chunk of a grouped split-K product: one length for all
// problems, so that the waves (one 16 x 16 tile each) get equal work and
// about 4096 of them run in all.
int64_t group_chunk(const std::vector<int64_t> &rows, const std::vector<int64_t> &tiles) {
  double work = 0.0;
  for (size_t i = 0; i < rows.size(); ++i) work += (double)rows[i] * (double)tiles[i];
  int64_t c = (int64_t)(work / 4096.0);
  c = (c + 15) / 16 * 16;
  return c < 64 ? 64 : c;
}

// C_i = Z1_i^* Z2_i (AoS k x k) on the FP64 matrix cores through row-chunk
// partial sums.
template <typename FZ1, typename FZ2, typename FO>
qsk_status crossprod_all(qsk_batch *b, const std::vector<int> &ids, int t1, int t2, FZ1 fz1, FZ2 fz2,
                         FO fo, bool tall_l) {
  if (ids.empty()) return QSK_OK;
  std::vector<qsk::Gemm64Args> a(ids.size());
  std::vector<qsk::ReduceArgs> r(ids.size());
  std::vector<int64_t> nb(ids.size()), rb(ids.size()), rows_v, tiles_v;
  for (int id : ids) {
    const Prob &q = b->p[id];
    rows_v.push_back(tall_l ? q.l : q.m);
    tiles_v.push_back((int64_t)((q.k + 15) / 16) * ((q.k + 15) / 16));
  }
  const int64_t budget = group_chunk(rows_v, tiles_v);
  for (size_t i = 0; i < ids.size(); ++i) {
    const Prob &q = b->p[ids[i]];
    const int64_t rows = tall_l ? q.l : q.m;
    const void *z1[4], *z2[4];
    int64_t ld1, ld2;
    fz1(q, z1, &ld1);
    fz2(q, z2, &ld2);
    if (!qsk::g64_plan_crossprod(z1, ld1, z2, ld2, rows, q.k, q.k, q.partials, q.partial_elems, budget,
                                 fo(q), &a[i], &r[i])) {
      b->last_error = "crossprod partial buffer too small";
      return QSK_E_HIP;
    }
    nb[i] = (int64_t)a[i].gx * a[i].gy;
    rb[i] = r[i].gx;
  }
  GroupRef g1, g2;
  int64_t n1, n2;
  if (!push_group(b, a, nb, &g1, &n1) || !push_group(b, r, rb, &g2, &n2)) return arena_full(b);
  BCHK(b, qsk::launch_qgemm64_k(b->stream, t1, t2, true, a[0], g1, n1));
  BCHK(b, qsk::launch_reduce_k(b->stream, r[0], g2, n2));
  return QSK_OK;
}

// Out_i = Z_i C_i (planar FP64) on the FP64 matrix cores.
template <typename FZ, typename FC, typename FO>
qsk_status apply_all(qsk_batch *b, const std::vector<int> &ids, int tz, FZ fz, FC fc, FO fo,
                     bool tall_l, bool c_upper = false) {
  if (ids.empty()) return QSK_OK;
  std::vector<qsk::Gemm64Args> a(ids.size());
  std::vector<int64_t> nb(ids.size());
  for (size_t i = 0; i < ids.size(); ++i) {
    const Prob &q = b->p[ids[i]];
    const void *z[4];
    int64_t ldz, ldo;
    double *o[4];
    fz(q, z, &ldz);
    fo(q, o, &ldo);
    a[i] = qsk::g64_plan_apply(z, ldz, tall_l ? q.l : q.m, q.k, fc(q), q.k, o, ldo, c_upper ? 1 : 0);
    nb[i] = (int64_t)a[i].gx * a[i].gy;
  }
  GroupRef g;
  int64_t tot;
  if (!push_group(b, a, nb, &g, &tot)) return arena_full(b);
  BCHK(b, qsk::launch_qgemm64_k(b->stream, tz, 0, false, a[0], g, tot));
  return QSK_OK;
}

qsk_status read_status(qsk_batch *b, std::vector<SmallStatus> &hs) {
  hs.resize(b->count);
  BCHK(b, hipMemcpyAsync(hs.data(), b->status, sizeof(SmallStatus) * b->count, hipMemcpyDeviceToHost, b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  return QSK_OK;
}

void planes_of(double *base, int64_t rows, int k, double *out[4]) {
  for (int p = 0; p < 4; ++p) out[p] = base + (size_t)p * rows * k;
}

}  // namespace

// Y = A Omega and W = Psi A of every problem (accumulated into Y and W) in
// one grouped launch each, with the batch's current tile shapes.
static qsk_status launch_sketches(qsk_batch *b, const void *const *planes, const int64_t *ld) {
  const int n_all = b->count;
  hipStream_t st = b->stream;
  std::vector<qsk::SketchArgs> sa(n_all);
  std::vector<qsk::MfmaStage> sg(n_all);
  for (int i = 0; i < n_all; ++i) {
    Prob &q = b->p[i];
    qsk::SketchArgs &s = sa[i];
    s.stream = st; s.mode = b->mode; s.in_dtype = q.cfg.input_dtype;
    for (int p = 0; p < 4; ++p) s.planes[p] = planes[4 * i + p];
    if (q.cfg.pure) s.planes[0] = planes[4 * i + 1];
    s.lda = ld[i]; s.pure = q.cfg.pure; s.m = q.m; s.col0 = 0; s.ncols = q.n; s.k = q.k; s.l = q.l;
    s.y = q.y; s.ldy = q.m; s.psy = q.m * (int64_t)q.k; s.pss = 0; s.y_copies = 1;
    s.w = q.w; s.ldw = q.l; s.psw = q.l * (int64_t)q.n;
    s.rad = q.cfg.embedding == QSK_RADEMACHER; s.terms = q.cfg.split_terms; s.k0 = q.k0; s.k1 = q.k1;
    s.scratch = q.wpart; s.scratch_bytes = q.wpart_bytes;
    sg[i] = q.stage;
  }
  BCHK(b, qsk::launch_sketch_mfma_batch(sa.data(), sg.data(), n_all, b->nmt, b->nj, b->arena, b->wblocks));
  return QSK_OK;
}

// Every step of one batched run, stream-ordered on b->stream.  opt: no host
// synchronisation (every factorisation assumed to succeed, failures only
// recorded in the sticky status flag); the caller prepares the arena.
static qsk_status batch_body(qsk_batch *b, qsk_rangefinder rf, const void *const *planes,
                             const int64_t *ld, double *const *Q, const int64_t *ldq,
                             double *const *X, const int64_t *ldx, bool opt) {
  hipStream_t st = b->stream;
  if (!opt) {
    BCHK(b, hipStreamSynchronize(st));      // previous users of the arena are done
    b->arena.used = 0;
  }
  const int n_all = b->count;
  std::vector<int> all(n_all);
  for (int i = 0; i < n_all; ++i) all[i] = i;

  // ---- sketches (Section 4.1): Y = A Omega, W = Psi A of every problem
  b->numeric_fail = false;
  {
    // Y, W and the statuses start at zero (by kernel: no memset nodes in a graph)
    std::vector<qsk::ZeroArgs> za(2 * n_all + 1);
    std::vector<int64_t> zb(2 * n_all + 1);
    for (int i = 0; i < n_all; ++i) {
      Prob &q = b->p[i];
      q.passes = 0; q.need = 2; q.flags = 0; q.z_is_u = false;
      za[2 * i].p = q.y; za[2 * i].n16 = (int64_t)q.m * q.k;          // 4 planes x 4 bytes
      za[2 * i + 1].p = q.w; za[2 * i + 1].n16 = (int64_t)q.l * q.n;
    }
    // status and kstatus are adjacent, each padded to 256 bytes
    za[2 * n_all].p = b->status;
    za[2 * n_all].n16 = (int64_t)(((char *)b->kstatus - (char *)b->status) + sizeof(SmallStatus) * n_all) / 16;
    for (size_t i = 0; i < za.size(); ++i) {
      za[i].gx = (int)((za[i].n16 + qsk::ZERO_UNITS_PER_BLOCK - 1) / qsk::ZERO_UNITS_PER_BLOCK);
      za[i].gy = 1;
      zb[i] = za[i].gx;
    }
    GroupRef g;
    int64_t tot;
    if (!push_group(b, za, zb, &g, &tot)) return arena_full(b);
    BCHK(b, qsk::launch_zero_k(st, za[0], g, tot));
  }
  {
    qsk_status r = launch_sketches(b, planes, ld);
    if (r != QSK_OK) return r;
  }

  // ---- CholeskyQR of Y (as in the single-problem driver)
  const int complex_only = rf == QSK_PSEUDO_QR;
  for (int i = 0; i < n_all; ++i) {
    Prob &q = b->p[i];
    for (int p = 0; p < 4; ++p) q.zsrc[p] = nullptr;
    q.gz = q.slot(B_G1);
  }
  std::vector<SmallStatus> hs(n_all);     // all-successful unless read (careful mode)
  std::vector<int> active = all;
  bool numeric_fail = false;
  const int max_passes = 8;
  while (!active.empty()) {
    const bool first = !b->p[active[0]].z_is_u;
    qsk_status r = crossprod_all(
        b, active, first ? 1 : 0, first ? 1 : 0,
        [](const Prob &q, const void *z[4], int64_t *ldz) {
          for (int p = 0; p < 4; ++p)
            z[p] = q.z_is_u ? (const void *)q.zsrc[p] : (const void *)(q.y + (size_t)p * q.m * q.k);
          *ldz = q.m;
        },
        [](const Prob &q, const void *z[4], int64_t *ldz) {
          for (int p = 0; p < 4; ++p)
            z[p] = q.z_is_u ? (const void *)q.zsrc[p] : (const void *)(q.y + (size_t)p * q.m * q.k);
          *ldz = q.m;
        },
        [](const Prob &q) { return q.gz; }, false);
    if (r != QSK_OK) return r;
    r = chol_all(b, active, [](const Prob &q) { return (const double *)q.gz; }, complex_only,
                 [](int) { return 0.0; }, 1e-13, [](const Prob &q) { return q.slot(B_R); },
                 [](const Prob &q) { return q.slot(B_T); }, 0);
    if (r != QSK_OK) return r;
    if (!opt && (r = read_status(b, hs)) != QSK_OK) return r;
    std::vector<int> failed;
    std::vector<double> shifts(n_all, 0.0);
    for (int i : active) {
      if (!hs[i].fail) continue;
      if (!(hs[i].trace > 0.0) || !std::isfinite(hs[i].trace)) {
        numeric_fail = true;
        b->p[i].need = -1;          // dropped
        continue;
      }
      const Prob &q = b->p[i];
      const double rows_c = complex_only ? 2.0 * q.m : 4.0 * q.m;
      shifts[i] = 11.0 * (rows_c * q.k + (double)q.k * (q.k + 1)) * 0x1p-53 * hs[i].trace;
      failed.push_back(i);
    }
    if (!failed.empty()) {
      r = chol_all(b, failed, [](const Prob &q) { return (const double *)q.gz; }, complex_only,
                   [&](int i) { return shifts[i]; }, 0.0, [](const Prob &q) { return q.slot(B_R); },
                   [](const Prob &q) { return q.slot(B_T); }, 1);
      if (r != QSK_OK) return r;
      if (!opt && (r = read_status(b, hs)) != QSK_OK) return r;
      for (int i : failed) {
        Prob &q = b->p[i];
        if (hs[i].fail) { numeric_fail = true; q.need = -1; continue; }
        q.flags |= QSK_FLAG_CHOL_FALLBACK;
        if (q.need < q.passes + 3) q.need = q.passes + 3;
      }
    }
    std::vector<int> live;
    for (int i : active)
      if (b->p[i].need >= 0) live.push_back(i);
    for (int i : live) b->p[i].passes += 1;
    // R_prod <- R (first pass) or R R_prod
    std::vector<int> first_ids, later_ids;
    for (int i : live) (b->p[i].passes == 1 ? first_ids : later_ids).push_back(i);
    if ((r = copy_all(b, first_ids, [](const Prob &q) { return (const double *)q.slot(B_R); },
                      [](const Prob &q) { return q.slot(B_RPROD); })) != QSK_OK)
      return r;
    if ((r = gemm_all(b, st, later_ids, [](const Prob &q) { return (const double *)q.slot(B_R); }, 0,
                      [](const Prob &q) { return (const double *)q.slot(B_RPROD); }, 0,
                      [](const Prob &q) { return q.slot(B_RTMP); })) != QSK_OK)
      return r;
    if ((r = copy_all(b, later_ids, [](const Prob &q) { return (const double *)q.slot(B_RTMP); },
                      [](const Prob &q) { return q.slot(B_RPROD); })) != QSK_OK)
      return r;
    std::vector<int> next;
    for (int i : live) {
      const Prob &q = b->p[i];
      if (q.passes < q.need && q.passes < max_passes) next.push_back(i);
    }
    if (next.empty()) break;
    // Z <- Z T into the alternating buffer
    const bool from_y = !b->p[next[0]].z_is_u;
    r = apply_all(
        b, next, from_y ? 1 : 0,
        [](const Prob &q, const void *z[4], int64_t *ldz) {
          for (int p = 0; p < 4; ++p)
            z[p] = q.z_is_u ? (const void *)q.zsrc[p] : (const void *)(q.y + (size_t)p * q.m * q.k);
          *ldz = q.m;
        },
        [](const Prob &q) { return (const double *)q.slot(B_T); },
        [](const Prob &q, double *o[4], int64_t *ldo) {
          planes_of(q.u[(q.passes - 1) & 1], q.m, q.k, o);
          *ldo = q.m;
        }, false, true);
    if (r != QSK_OK) return r;
    for (int i : next) {
      Prob &q = b->p[i];
      planes_of(q.u[(q.passes - 1) & 1], q.m, q.k, q.zsrc);
      q.z_is_u = true;
      q.gz = q.slot(B_GU);
    }
    active = next;
  }
  std::vector<int> ok_ids;
  for (int i : all)
    if (b->p[i].need >= 0) ok_ids.push_back(i);

  // the optimistic run keeps the sticky failure flag of the passes above
  BCHK(b, qsk::launch_status_reset_n(st, b->status, n_all, opt ? 1 : 0));
  BCHK(b, qsk::launch_status_reset_n(st, b->kstatus, n_all, 0));
  qsk_status r = QSK_OK;
  auto S = [](int s) { return [s](const Prob &q) { return q.slot(s); }; };
  auto SC = [](int s) { return [s](const Prob &q) { return (const double *)q.slot(s); }; };
  auto GZ = [](const Prob &q) { return (const double *)q.gz; };
  auto kappa_all = [&](int which, int src_slot) -> qsk_status {
    if (ok_ids.empty()) return QSK_OK;
    std::vector<qsk::KappaArgs> a(ok_ids.size());
    std::vector<int64_t> one(ok_ids.size(), 1);
    for (size_t i = 0; i < ok_ids.size(); ++i) {
      const Prob &q = b->p[ok_ids[i]];
      a[i].k = q.k; a[i].gh = q.slot(src_slot); a[i].work = q.kwork; a[i].which = which;
      a[i].status = b->kstatus + ok_ids[i]; a[i].gx = 1; a[i].gy = 1;
    }
    GroupRef g;
    int64_t tot;
    if (!push_group(b, a, one, &g, &tot)) return arena_full(b);
    BCHK(b, hipEventRecord(b->ev_fork, st));
    BCHK(b, hipStreamWaitEvent(b->side, b->ev_fork, 0));
    BCHK(b, qsk::launch_kappa_k(b->side, a[0], g, (int)ok_ids.size()));
    return QSK_OK;
  };
  if (rf == QSK_PSEUDO_QR) {
    if ((r = gemm_all(b, st, ok_ids, GZ, 0, SC(B_T), 0, S(B_TMP))) != QSK_OK) return r;
    if ((r = gemm_all(b, st, ok_ids, SC(B_T), 1, SC(B_TMP), 0, S(B_G0))) != QSK_OK) return r;
    if ((r = copy_all(b, ok_ids, SC(B_G0), S(B_GK0))) != QSK_OK) return r;
    if ((r = kappa_all(1, B_GK0)) != QSK_OK) return r;
    {
      std::vector<qsk::GemmArgs> a(ok_ids.size());
      std::vector<int64_t> one(ok_ids.size(), 1);
      for (size_t i = 0; i < ok_ids.size(); ++i) {
        a[i].k = b->p[ok_ids[i]].k; a[i].c = b->p[ok_ids[i]].slot(B_C); a[i].gx = 1; a[i].gy = 1;
      }
      GroupRef g;
      int64_t tot;
      if (!ok_ids.empty()) {
        if (!push_group(b, a, one, &g, &tot)) return arena_full(b);
        BCHK(b, qsk::launch_identity_k(st, a[0], g, (int)ok_ids.size()));
      }
    }
    std::vector<int> corr = ok_ids;
    for (int j = 0; j < b->p[0].cfg.n_correction && !corr.empty(); ++j) {
      if ((r = chol_all(b, corr, SC(B_G0), 0, [](int) { return 0.0; }, 1e-13, S(B_CR), S(B_CT), 0)) != QSK_OK)
        return r;
      if (!opt && (r = read_status(b, hs)) != QSK_OK) return r;
      std::vector<int> go;
      for (int i : corr) {
        if (hs[i].fail) b->p[i].flags |= QSK_FLAG_RANK_DEFICIENT;
        else go.push_back(i);
      }
      corr = go;
      if (corr.empty()) break;
      if ((r = gemm_all(b, st, corr, SC(B_CT), 0, SC(B_CT), 1, S(B_GI))) != QSK_OK) return r;
      {
        std::vector<qsk::PowerArgs> a(corr.size());
        std::vector<int64_t> one(corr.size(), 1);
        for (size_t i = 0; i < corr.size(); ++i) {
          const Prob &q = b->p[corr[i]];
          a[i].k = q.k; a[i].gi = q.slot(B_GI); a[i].step = j; a[i].n_power = q.cfg.n_power;
          a[i].k0 = q.k0; a[i].k1 = q.k1; a[i].m_out = q.slot(B_M); a[i].status = b->status + corr[i];
          a[i].gx = 1; a[i].gy = 1;
        }
        GroupRef g;
        int64_t tot;
        if (!push_group(b, a, one, &g, &tot)) return arena_full(b);
        BCHK(b, qsk::launch_power_k(st, a[0], g, (int)corr.size()));
      }
      if ((r = gemm_all(b, st, corr, SC(B_C), 0, SC(B_M), 0, S(B_TMP))) != QSK_OK) return r;
      if ((r = copy_all(b, corr, SC(B_TMP), S(B_C))) != QSK_OK) return r;
      if ((r = gemm_all(b, st, corr, SC(B_G0), 0, SC(B_M), 0, S(B_TMP))) != QSK_OK) return r;
      if ((r = gemm_all(b, st, corr, SC(B_M), 1, SC(B_TMP), 0, S(B_G0))) != QSK_OK) return r;
    }
  } else {
    if ((r = gemm_all(b, st, ok_ids, SC(B_RPROD), 0, SC(B_RPROD), 1, S(B_TMP))) != QSK_OK) return r;
    if (!ok_ids.empty()) {
      for (int stage = 0; stage < 5; ++stage) {
        std::vector<qsk::PsvdArgs> a(ok_ids.size());
        std::vector<int64_t> nb(ok_ids.size());
        for (size_t i = 0; i < ok_ids.size(); ++i) {
          const Prob &q = b->p[ok_ids[i]];
          a[i].k = q.k; a[i].gl = q.slot(B_TMP); a[i].k0 = q.k0; a[i].k1 = q.k1; a[i].c = q.slot(B_C);
          a[i].work = q.work; a[i].status = b->status + ok_ids[i];
          a[i].gx = qsk::psvd_blocks(q.k, stage); a[i].gy = 1;
          nb[i] = a[i].gx;
        }
        GroupRef g;
        int64_t tot;
        if (!push_group(b, a, nb, &g, &tot)) return arena_full(b);
        BCHK(b, qsk::launch_psvd_stage(st, stage, a[0], g, tot));
      }
    }
  }
  if ((r = gemm_all(b, st, ok_ids, SC(B_T), 0, SC(B_C), 0, S(B_F))) != QSK_OK) return r;
  if ((r = gemm_all(b, st, ok_ids, GZ, 0, SC(B_F), 0, S(B_TMP2))) != QSK_OK) return r;
  if ((r = gemm_all(b, st, ok_ids, SC(B_F), 1, SC(B_TMP2), 0, S(B_GH))) != QSK_OK) return r;
  if ((r = kappa_all(0, B_GH)) != QSK_OK) return r;
  BCHK(b, hipEventRecord(b->ev_join, b->side));
  // Q = Z F
  if ((r = apply_all(
           b, ok_ids, 0,
           [](const Prob &q, const void *z[4], int64_t *ldz) {
             for (int p = 0; p < 4; ++p) z[p] = q.zsrc[p];
             *ldz = q.m;
           },
           SC(B_F),
           [&](const Prob &q, double *o[4], int64_t *ldo) {
             const int i = (int)(&q - b->p.data());
             for (int p = 0; p < 4; ++p) o[p] = Q[4 * i + p];
             *ldo = ldq[i];
           }, false)) != QSK_OK)
    return r;
  // ---- core solve: P = Psi Q, X = (P^dagger) W through CholeskyQR2 of P
  if (!ok_ids.empty()) {
    // P = Psi Q from the staged Psi (exactly the values that formed W)
    std::vector<qsk::Gemm64Args> a(ok_ids.size());
    std::vector<qsk::ReducePlanarArgs> rr(ok_ids.size());
    std::vector<int64_t> nb(ok_ids.size()), rb(ok_ids.size()), rows_v, tiles_v;
    for (int id : ok_ids) {
      const Prob &q = b->p[id];
      rows_v.push_back(q.m);
      tiles_v.push_back((int64_t)((q.l + 15) / 16) * ((q.k + 15) / 16));
    }
    const int64_t budget = group_chunk(rows_v, tiles_v);
    const int es = b->mode == qsk::MODE_BF16 ? 2 : 4;
    for (size_t i = 0; i < ok_ids.size(); ++i) {
      const int id = ok_ids[i];
      const Prob &q = b->p[id];
      const double *h[4] = {Q[4 * id], Q[4 * id + 1], Q[4 * id + 2], Q[4 * id + 3]};
      double *pout[4];
      planes_of(q.pbuf, q.l, q.k, pout);
      if (!qsk::g64_plan_psi(q.stage.psi, es, q.stage.MP, (int64_t)q.stage.LP * q.stage.MP, h, ldq[id],
                             q.l, q.m, q.k, q.partials, q.partial_elems, budget, pout, q.l, &a[i],
                             &rr[i])) {
        b->last_error = "psi product partial buffer too small";
        return QSK_E_HIP;
      }
      nb[i] = (int64_t)a[i].gx * a[i].gy;
      rb[i] = rr[i].gx;
    }
    GroupRef g1, g2;
    int64_t n1, n2;
    if (!push_group(b, a, nb, &g1, &n1) || !push_group(b, rr, rb, &g2, &n2)) return arena_full(b);
    BCHK(b, qsk::launch_qgemm64_k(st, es == 2 ? 2 : 1, 0, false, a[0], g1, n1));
    BCHK(b, qsk::launch_reduce_planar_k(st, rr[0], g2, n2));
  }
  auto PZ = [](double *Prob::*buf) {
    return [buf](const Prob &q, const void *z[4], int64_t *ldz) {
      for (int p = 0; p < 4; ++p) z[p] = (q.*buf) + (size_t)p * q.l * q.k;
      *ldz = q.l;
    };
  };
  auto PO = [](double *Prob::*buf) {
    return [buf](const Prob &q, double *o[4], int64_t *ldo) {
      planes_of(q.*buf, q.l, q.k, o);
      *ldo = q.l;
    };
  };
  auto pinv_all = [&](const std::vector<int> &ids) -> qsk_status {
    if (ids.empty()) return QSK_OK;
    std::vector<qsk::PinvArgs> a(ids.size());
    std::vector<int64_t> one(ids.size(), 1);
    for (size_t i = 0; i < ids.size(); ++i) {
      Prob &q = b->p[ids[i]];
      q.flags |= QSK_FLAG_RANK_DEFICIENT;
      a[i].l = q.l; a[i].k = q.k;
      for (int p = 0; p < 4; ++p) a[i].p[p] = q.pbuf + (size_t)p * q.l * q.k;
      a[i].ldp = q.l; a[i].tol = 1e-13; a[i].work = q.pinv_work;
      planes_of(q.sbuf, q.l, q.k, a[i].out);
      a[i].ldo = q.l; a[i].gx = 1; a[i].gy = 1;
    }
    GroupRef g;
    int64_t tot;
    if (!push_group(b, a, one, &g, &tot)) return arena_full(b);
    BCHK(b, qsk::launch_pinv_k(st, a[0], g, (int)ids.size()));
    return QSK_OK;
  };
  if ((r = crossprod_all(b, ok_ids, 0, 0, PZ(&Prob::pbuf), PZ(&Prob::pbuf), S(B_GP), true)) != QSK_OK) return r;
  if ((r = chol_all(b, ok_ids, SC(B_GP), 0, [](int) { return 0.0; }, 1e-13, S(B_RP), S(B_TP1), 0)) != QSK_OK)
    return r;
  if (!opt && (r = read_status(b, hs)) != QSK_OK) return r;
  std::vector<int> p_ok, p_bad;
  for (int i : ok_ids) (hs[i].fail ? p_bad : p_ok).push_back(i);
  if ((r = pinv_all(p_bad)) != QSK_OK) return r;
  if ((r = apply_all(b, p_ok, 0, PZ(&Prob::pbuf), SC(B_TP1), PO(&Prob::p1buf), true, true)) != QSK_OK)
    return r;
  if ((r = crossprod_all(b, p_ok, 0, 0, PZ(&Prob::p1buf), PZ(&Prob::p1buf), S(B_GP), true)) != QSK_OK) return r;
  if ((r = chol_all(b, p_ok, SC(B_GP), 0, [](int) { return 0.0; }, 1e-13, S(B_RP), S(B_TP2), 0)) != QSK_OK)
    return r;
  if (!opt && (r = read_status(b, hs)) != QSK_OK) return r;
  std::vector<int> p_ok2, p_bad2;
  for (int i : p_ok) (hs[i].fail ? p_bad2 : p_ok2).push_back(i);
  if ((r = pinv_all(p_bad2)) != QSK_OK) return r;
  if ((r = gemm_all(b, st, p_ok2, SC(B_TP1), 0, SC(B_TP2), 0, S(B_TPT))) != QSK_OK) return r;
  if ((r = gemm_all(b, st, p_ok2, SC(B_TPT), 0, SC(B_TPT), 1, S(B_Z))) != QSK_OK) return r;
  if ((r = apply_all(b, p_ok2, 0, PZ(&Prob::pbuf), SC(B_Z), PO(&Prob::sbuf), true)) != QSK_OK) return r;
  // X = (S^*)^* W
  if (!ok_ids.empty()) {
    std::vector<qsk::Gemm64Args> a(ok_ids.size());
    std::vector<int64_t> nb(ok_ids.size());
    for (size_t i = 0; i < ok_ids.size(); ++i) {
      const int id = ok_ids[i];
      const Prob &q = b->p[id];
      const void *z1[4], *z2[4];
      double *o[4];
      for (int p = 0; p < 4; ++p) {
        z1[p] = q.sbuf + (size_t)p * q.l * q.k;
        z2[p] = q.w + (size_t)p * q.l * q.n;
        o[p] = X[4 * id + p];
      }
      a[i] = qsk::g64_plan_crossprod_planar(z1, q.l, z2, q.l, q.l, q.k, (int)q.n, o, ldx[id]);
      nb[i] = (int64_t)a[i].gx * a[i].gy;
    }
    GroupRef g;
    int64_t tot;
    if (!push_group(b, a, nb, &g, &tot)) return arena_full(b);
    BCHK(b, qsk::launch_qgemm64_k(st, 0, 1, true, a[0], g, tot));
  }
  // join the kappa side stream
  BCHK(b, hipStreamWaitEvent(st, b->ev_join, 0));
  b->numeric_fail = numeric_fail;
  return QSK_OK;
}

// Read the statuses of the run just issued (one synchronisation) and fill
// the reports.  After an optimistic run *retry says whether any
// factorisation failed, in which case nothing is reported.
static qsk_status batch_collect(qsk_batch *b, qsk_rangefinder rf, qsk_report *reports, bool opt,
                                bool *retry) {
  const int n_all = b->count;
  hipStream_t st = b->stream;
  *retry = false;
  std::vector<SmallStatus> hs(n_all), ks(n_all);
  BCHK(b, hipMemcpyAsync(hs.data(), b->status, sizeof(SmallStatus) * n_all, hipMemcpyDeviceToHost, st));
  BCHK(b, hipMemcpyAsync(ks.data(), b->kstatus, sizeof(SmallStatus) * n_all, hipMemcpyDeviceToHost, st));
  BCHK(b, hipStreamSynchronize(st));
  if (opt) {
    for (int i = 0; i < n_all; ++i)
      if (hs[i].fail_any) *retry = true;
    if (*retry) return QSK_OK;
  }
  if (reports) {
    for (int i = 0; i < n_all; ++i) {
      const Prob &q = b->p[i];
      qsk_report rep{};
      rep.kappa = ks[i].kappa;
      rep.kappa_initial = rf == QSK_PSEUDO_QR ? ks[i].kappa_initial : ks[i].kappa;
      rep.n_eps = hs[i].n_eps;
      for (int e = 0; e < 8; ++e) rep.eps[e] = hs[i].eps[e];
      rep.t_bad = hs[i].t_bad;
      rep.flags = opt ? hs[i].flags : (q.flags | hs[i].flags | (q.need < 0 ? QSK_FLAG_NONFINITE : 0));
      rep.passes = opt ? 2 : q.passes;
      rep.columns_seen = q.n;
      rep.orth_defect = rf == QSK_PSEUDO_SVD ? ks[i].orth_defect : 0.0;
      reports[i] = rep;
    }
  }
  if (!opt && b->numeric_fail) {
    b->last_error = "a problem's sketch Y is zero or non-finite";
    return QSK_E_NUMERIC;
  }
  return QSK_OK;
}

// The optimistic run as a graph on b->gstream: captured on first use (and
// again when the caller's pointers change), then replayed.  The argument
// tables go to the graph's own arena once, after the capture, so the graph
// holds kernel nodes only.
static qsk_status batch_graph(qsk_batch *b, qsk_rangefinder rf, const void *const *planes,
                              const int64_t *ld, double *const *Q, const int64_t *ldq,
                              double *const *X, const int64_t *ldx) {
  const int n_all = b->count;
  const int gi = rf == QSK_PSEUDO_SVD ? 1 : 0;
  std::vector<uintptr_t> key;
  key.reserve(16 * (size_t)n_all);
  for (int i = 0; i < n_all; ++i) {
    for (int p = 0; p < 4; ++p) {
      key.push_back((uintptr_t)planes[4 * i + p]);
      key.push_back((uintptr_t)Q[4 * i + p]);
      key.push_back((uintptr_t)X[4 * i + p]);
    }
    key.push_back((uintptr_t)ld[i]);
    key.push_back((uintptr_t)ldq[i]);
    key.push_back((uintptr_t)ldx[i]);
  }
  hipStream_t user = b->stream;
  BCHK(b, hipEventRecord(b->ev_in, user));
  BCHK(b, hipStreamWaitEvent(b->gstream, b->ev_in, 0));
  if (!b->gexec[gi] || key != b->gkey[gi]) {
    if (b->gexec[gi]) {
      BCHK(b, hipStreamSynchronize(b->gstream));
      (void)hipGraphExecDestroy(b->gexec[gi]);
      b->gexec[gi] = nullptr;
    }
    std::swap(b->arena, b->garena[gi]);
    b->arena.used = 0;
    b->arena.defer = true;
    b->stream = b->gstream;
    hipError_t e = hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal);
    qsk_status r = e == hipSuccess ? batch_body(b, rf, planes, ld, Q, ldq, X, ldx, true) : QSK_E_HIP;
    hipGraph_t graph = nullptr;
    const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(b->gstream, &graph) : e;
    b->stream = user;
    b->arena.defer = false;
    std::swap(b->arena, b->garena[gi]);
    if (r != QSK_OK || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (r != QSK_OK) return r;
      return bfail(b, e2, "graph capture");
    }
    const hipError_t e3 = hipGraphInstantiate(&b->gexec[gi], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) {
      b->gexec[gi] = nullptr;
      return bfail(b, e3, "hipGraphInstantiate");
    }
    BCHK(b, hipMemcpyAsync(b->garena[gi].dev, b->garena[gi].host, b->garena[gi].used,
                           hipMemcpyHostToDevice, b->gstream));
    b->gkey[gi] = key;
  }
  BCHK(b, hipGraphLaunch(b->gexec[gi], b->gstream));
  BCHK(b, hipEventRecord(b->ev_out, b->gstream));
  BCHK(b, hipStreamWaitEvent(user, b->ev_out, 0));
  return QSK_OK;
}

// The captured graphs hold the launch shapes they were recorded with.
static void drop_graphs(qsk_batch *b) {
  for (int r = 0; r < 2; ++r) {
    if (b->gexec[r]) (void)hipGraphExecDestroy(b->gexec[r]);
    b->gexec[r] = nullptr;
    b->gkey[r].clear();
  }
}

// Lay the staged test matrices out for tile shapes (nmt, nj) and regenerate
// them; the captured graphs hold the old layout and are dropped.
static qsk_status restage(qsk_batch *b, int nmt, int nj) {
  for (int i = 0; i < b->count; ++i) {
    Prob &q = b->p[i];
    qsk::stage_geometry_tiles(q.m, q.l, q.k, q.n, nmt, nj, &q.stage.LP, &q.stage.MP, &q.stage.KP,
                              &q.stage.NP);
    qsk::SketchArgs s{};
    s.stream = b->stream; s.mode = b->mode; s.m = q.m; s.col0 = 0; s.ncols = q.n; s.k = q.k; s.l = q.l;
    s.rad = q.cfg.embedding == QSK_RADEMACHER; s.k0 = q.k0; s.k1 = q.k1;
    BCHK(b, qsk::stage_test_matrices(s, q.stage));
  }
  b->nmt = nmt;
  b->nj = nj;
  BCHK(b, hipStreamSynchronize(b->stream));
  drop_graphs(b);
  return QSK_OK;
}

// Tuned launch shapes by device and batch signature (operand format and
// every problem's m, n, k, l), shared by the batches of this process and,
// when QSK_TUNE_CACHE names a file, kept there across processes: one line
// per entry, "<arch> <CUs> <key, comma-separated> <nmt> <nj> <wblocks>"
// (lines that do not parse, or name another device, are ignored).
struct TuneChoice {
  int nmt, nj, wblocks;
};
static std::mutex g_tune_mu;
static std::map<std::string, TuneChoice> g_tuned;
static bool g_tune_file_read = false;

static std::string tune_key(const qsk_batch *b) {
  std::string key;
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    std::string arch = prop.gcnArchName;
    for (char &ch : arch)
      if (ch == ' ' || ch == '\t') ch = '_';
    key = arch + " " + std::to_string(prop.multiProcessorCount) + " ";
  } else {
    key = "unknown 0 ";
  }
  std::vector<int64_t> v = {b->mode, b->p[0].cfg.split_terms, b->p[0].cfg.input_dtype, b->p[0].cfg.pure};
  for (const Prob &q : b->p) {
    v.push_back(q.m); v.push_back(q.n); v.push_back(q.k); v.push_back(q.l);
  }
  for (size_t i = 0; i < v.size(); ++i) key += (i ? "," : "") + std::to_string(v[i]);
  return key;
}

static bool valid_choice(const TuneChoice &c, int mode) {
  const int n_nmt = mode == qsk::MODE_BF16 ? 4 : 2;
  bool ok_nmt = false, ok_nj = false;
  for (int a = 0; a < n_nmt; ++a) ok_nmt = ok_nmt || c.nmt == kNmt[a];
  for (int a = 0; a < 2; ++a) ok_nj = ok_nj || c.nj == kNj[a];
  return ok_nmt && ok_nj && c.wblocks >= 64 && c.wblocks <= (1 << 16);
}

// Called with g_tune_mu held: the cache file's entries, once per process.
static void read_tune_file() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char *path = std::getenv("QSK_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  char line[8192];
  while (std::fgets(line, sizeof(line), f)) {
    char arch[256], key[7000];
    int cus = 0;
    TuneChoice c{};
    if (std::sscanf(line, "%255s %d %6999s %d %d %d", arch, &cus, key, &c.nmt, &c.nj, &c.wblocks) != 6) continue;
    g_tuned[std::string(arch) + " " + std::to_string(cus) + " " + key] = c;
  }
  std::fclose(f);
}

// Called with g_tune_mu held: appends an entry to the cache file.
static void append_tune_file(const std::string &key, const TuneChoice &c) {
  const char *path = std::getenv("QSK_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d\n", key.c_str(), c.nmt, c.nj, c.wblocks);
  std::fclose(f);
}

extern "C" {

qsk_status qsketch_batch_init(int32_t count, const qsk_config *cfgs, void *hip_stream,
                              qsk_batch **out) {
  if (!out || !cfgs || count < 1) return QSK_E_ARG;
  *out = nullptr;
  const qsk_config &c0 = cfgs[0];
  for (int i = 0; i < count; ++i) {
    const qsk_config &c = cfgs[i];
    if (c.m < 1 || c.n < 1 || c.m >= (1ll << 31) || c.n >= (1ll << 31)) return QSK_E_ARG;
    if (c.k < 1 || c.l < c.k || c.l > c.m || c.l > c.n || c.k > 256 || c.l > 1024) return QSK_E_ARG;
    if (c.embedding != QSK_GAUSSIAN && c.embedding != QSK_RADEMACHER) return QSK_E_ARG;
    if (c.input_dtype < QSK_F64 || c.input_dtype > QSK_BF16) return QSK_E_ARG;
    if (c.sketch_dtype < QSK_F64 || c.sketch_dtype > QSK_FP8_MFMA) return QSK_E_ARG;
    if (c.n_correction < 0 || c.n_correction > 8 || c.n_power < 1 || c.n_power > 64) return QSK_E_ARG;
    if (c.sketch_dtype == QSK_BF16 && (c.split_terms < 1 || c.split_terms > 3)) return QSK_E_ARG;
    if (c.y_only || c.embedding_round != QSK_F64 || c.coalesce_cols != 0) return QSK_E_ARG;
    if (c.embedding != c0.embedding || c.input_dtype != c0.input_dtype ||
        c.sketch_dtype != c0.sketch_dtype || c.pure != c0.pure ||
        (c.sketch_dtype == QSK_BF16 && c.split_terms != c0.split_terms) ||
        c.n_correction != c0.n_correction || c.n_power != c0.n_power)
      return QSK_E_ARG;
  }
  if (c0.sketch_dtype != QSK_BF16 && c0.sketch_dtype != QSK_F32) return QSK_E_UNSUPPORTED;
  if (c0.input_dtype == QSK_F64) return QSK_E_UNSUPPORTED;

  qsk_batch *b = new (std::nothrow) qsk_batch;
  if (!b) return QSK_E_NOMEM;
  b->count = count;
  b->stream = (hipStream_t)hip_stream;
  b->mode = c0.sketch_dtype;
  b->p.resize(count);
  std::vector<int> ls(count), ks(count);
  for (int i = 0; i < count; ++i) { ls[i] = cfgs[i].l; ks[i] = cfgs[i].k; }
  qsk::batch_tiles(ls.data(), ks.data(), count, c0.sketch_dtype == QSK_BF16, &b->nmt, &b->nj);

  // carve every problem's workspace out of one allocation
  const size_t es = c0.sketch_dtype == QSK_BF16 ? 2 : 4;
  size_t total = 0;
  std::vector<std::vector<size_t>> off(count);
  for (int i = 0; i < count; ++i) {
    Prob &q = b->p[i];
    q.cfg = cfgs[i];
    if (c0.sketch_dtype != QSK_BF16) q.cfg.split_terms = 1;
    q.m = cfgs[i].m; q.n = cfgs[i].n; q.k = cfgs[i].k; q.l = cfgs[i].l;
    q.k0 = (uint32_t)(cfgs[i].seed & 0xFFFFFFFFull);
    q.k1 = (uint32_t)(cfgs[i].seed >> 32);
    qsk::stage_geometry_tiles(q.m, q.l, q.k, q.n, b->nmt, b->nj, &q.stage.LP, &q.stage.MP, &q.stage.KP,
                              &q.stage.NP);
    const size_t kk = (size_t)q.k * q.k * 4;
    const int64_t maxk = q.l > q.k ? q.l : q.k;
    q.partial_elems = 16 * maxk * q.k * 4;
    const size_t sizes[] = {
        4 * (size_t)q.m * q.k * 4,                 // y
        4 * (size_t)q.l * q.n * 4,                 // w
        4 * (size_t)q.m * q.k * 8,                 // u0
        4 * (size_t)q.m * q.k * 8,                 // u1
        (size_t)B_COUNT * kk * 8,                  // small
        (12 * kk + 64 * (size_t)q.k) * 8,          // work
        kk * 8,                                    // kwork
        (size_t)q.partial_elems * 8,               // partials
        4 * (size_t)q.l * q.k * 8,                 // pbuf
        4 * (size_t)q.l * q.k * 8,                 // p1buf
        4 * (size_t)q.l * q.k * 8,                 // sbuf
        4 * (size_t)(q.l + q.k) * q.k * 8,         // pinv_work
        // staging sized for the largest padding of any tile shape the
        // autotuner may pick
        4 * (size_t)max_pad(q.k, kNj, 2) * q.stage.NP * es,                            // omega staging
        4 * (size_t)max_pad(q.l, kNmt, c0.sketch_dtype == QSK_BF16 ? 4 : 2) * q.stage.MP * es,  // psi
        // W partial sums: up to 8 row chunks of 4 planes x n x the padded l
        8 * 4 * (size_t)q.n * max_pad(q.l, kNmt, c0.sketch_dtype == QSK_BF16 ? 4 : 2) * 4,
    };
    for (size_t s : sizes) {
      off[i].push_back(total);
      total += al(s);
    }
  }
  const size_t st_off = total;
  total += al(sizeof(SmallStatus) * count) * 2 + al(16 * (size_t)count);
  bool ok = hipMalloc(&b->pool, total) == hipSuccess;
  const size_t arena_cap = 8u << 20;
  ok = ok && hipHostMalloc((void **)&b->arena.host, arena_cap, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipMalloc((void **)&b->arena.dev, arena_cap) == hipSuccess;
  b->arena.cap = arena_cap;
  ok = ok && hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) == hipSuccess;
  for (int r = 0; r < 2; ++r) {
    ok = ok && hipHostMalloc((void **)&b->garena[r].host, arena_cap, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMalloc((void **)&b->garena[r].dev, arena_cap) == hipSuccess;
    b->garena[r].cap = arena_cap;
  }
  if (!ok) {
    (void)hipGetLastError();
    qsketch_batch_destroy(b);
    return QSK_E_NOMEM;
  }
  char *base = (char *)b->pool;
  for (int i = 0; i < count; ++i) {
    Prob &q = b->p[i];
    const std::vector<size_t> &o = off[i];
    q.y = (float *)(base + o[0]);
    q.w = (float *)(base + o[1]);
    q.u[0] = (double *)(base + o[2]);
    q.u[1] = (double *)(base + o[3]);
    q.small = (double *)(base + o[4]);
    q.work = (double *)(base + o[5]);
    q.kwork = (double *)(base + o[6]);
    q.partials = (double *)(base + o[7]);
    q.pbuf = (double *)(base + o[8]);
    q.p1buf = (double *)(base + o[9]);
    q.sbuf = (double *)(base + o[10]);
    q.pinv_work = (double *)(base + o[11]);
    q.stage.omega = base + o[12];
    q.stage.psi = base + o[13];
    q.wpart = (float *)(base + o[14]);
    q.wpart_bytes = (int64_t)(8 * 4 * (size_t)q.n * max_pad(q.l, kNmt, c0.sketch_dtype == QSK_BF16 ? 4 : 2) * 4);
  }
  b->status = (SmallStatus *)(base + st_off);
  b->kstatus = (SmallStatus *)(base + st_off + al(sizeof(SmallStatus) * count));
  b->err_acc = (double *)(base + st_off + 2 * al(sizeof(SmallStatus) * count));
  // the test matrices are fixed per problem: stage them once
  for (int i = 0; i < count; ++i) {
    Prob &q = b->p[i];
    qsk::SketchArgs s{};
    s.stream = b->stream; s.mode = b->mode; s.m = q.m; s.col0 = 0; s.ncols = q.n; s.k = q.k; s.l = q.l;
    s.rad = q.cfg.embedding == QSK_RADEMACHER; s.k0 = q.k0; s.k1 = q.k1;
    hipError_t e = qsk::stage_test_matrices(s, q.stage);
    if (e != hipSuccess) {
      qsketch_batch_destroy(b);
      return QSK_E_HIP;
    }
  }
  if (hipStreamSynchronize(b->stream) != hipSuccess) {
    qsketch_batch_destroy(b);
    return QSK_E_HIP;
  }
  *out = b;
  return QSK_OK;
}

void qsketch_batch_destroy(qsk_batch *b) {
  if (!b) return;
  if (b->stream || true) (void)hipStreamSynchronize(b->stream);
  if (b->side) (void)hipStreamSynchronize(b->side);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
  if (b->gstream) (void)hipStreamSynchronize(b->gstream);
  for (int r = 0; r < 2; ++r) {
    if (b->gexec[r]) (void)hipGraphExecDestroy(b->gexec[r]);
    if (b->garena[r].dev) (void)hipFree(b->garena[r].dev);
    if (b->garena[r].host) (void)hipHostFree(b->garena[r].host);
  }
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->gstream) (void)hipStreamDestroy(b->gstream);
  if (b->side) (void)hipStreamDestroy(b->side);
  if (b->pool) (void)hipFree(b->pool);
  if (b->arena.dev) (void)hipFree(b->arena.dev);
  if (b->arena.host) (void)hipHostFree(b->arena.host);
  delete b;
}

const char *qsketch_batch_last_error(const qsk_batch *b) {
  if (!b) return "null batch";
  return b->last_error.c_str();
}

qsk_status qsketch_batch_run(qsk_batch *b, qsk_rangefinder rf, const void *const *planes,
                             const int64_t *ld, double *const *Q, const int64_t *ldq,
                             double *const *X, const int64_t *ldx, qsk_report *reports) {
  if (!b) return QSK_E_ARG;
  if (b->poisoned) return QSK_E_STATE;
  if (rf != QSK_PSEUDO_QR && rf != QSK_PSEUDO_SVD) return QSK_E_ARG;
  if (!planes || !ld || !Q || !ldq || !X || !ldx) return QSK_E_ARG;
  const int n_all = b->count;
  for (int i = 0; i < n_all; ++i) {
    const Prob &q = b->p[i];
    if (ld[i] < q.m || ldq[i] < q.m || ldx[i] < q.k) return QSK_E_ARG;
    for (int p = q.cfg.pure ? 1 : 0; p < 4; ++p)
      if (!planes[4 * i + p]) return QSK_E_ARG;
    for (int p = 0; p < 4; ++p)
      if (!Q[4 * i + p] || !X[4 * i + p]) return QSK_E_ARG;
  }
  qsk_status r;
  bool retry = false;
  if (b->exec_mode == 2) {
    if ((r = batch_graph(b, rf, planes, ld, Q, ldq, X, ldx)) != QSK_OK) return r;
    if ((r = batch_collect(b, rf, reports, true, &retry)) != QSK_OK) return r;
    if (!retry) return QSK_OK;
  } else if (b->exec_mode == 1) {
    BCHK(b, hipStreamSynchronize(b->stream));
    b->arena.used = 0;
    if ((r = batch_body(b, rf, planes, ld, Q, ldq, X, ldx, true)) != QSK_OK) return r;
    if ((r = batch_collect(b, rf, reports, true, &retry)) != QSK_OK) return r;
    if (!retry) return QSK_OK;
  }
  if ((r = batch_body(b, rf, planes, ld, Q, ldq, X, ldx, false)) != QSK_OK) return r;
  return batch_collect(b, rf, reports, false, &retry);
}

qsk_status qsketch_batch_autotune(qsk_batch *b, const void *const *planes, const int64_t *ld,
                                  int32_t reps, int32_t *nmt_out, int32_t *nj_out, int32_t *wblocks_out) {
  if (!b || !planes || !ld || reps < 0 || reps > 100) return QSK_E_ARG;
  if (b->poisoned) return QSK_E_STATE;
  for (int i = 0; i < b->count; ++i) {
    const Prob &q = b->p[i];
    if (ld[i] < q.m) return QSK_E_ARG;
    for (int p = q.cfg.pure ? 1 : 0; p < 4; ++p)
      if (!planes[4 * i + p]) return QSK_E_ARG;
  }
  const std::string key = tune_key(b);
  TuneChoice best_c{-1, -1, -1};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    read_tune_file();
    auto it = g_tuned.find(key);
    if (it != g_tuned.end() && valid_choice(it->second, b->mode)) best_c = it->second;
  }
  if (best_c.nmt < 0 && reps > 0) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BCHK(b, hipEventCreate(&e0));
    BCHK(b, hipEventCreate(&e1));
    float best = -1.0f;
    qsk_status r = QSK_OK;
    const int n_nmt = b->mode == qsk::MODE_BF16 ? 4 : 2;
    // W row splits: fewer, longer chunks (fewer partial sums to reduce) or
    // more, shorter ones (more blocks in flight)
    const int wcand[3] = {qsk::BATCH_W_BLOCKS / 4, qsk::BATCH_W_BLOCKS, qsk::BATCH_W_BLOCKS * 4};
    for (int a = 0; a < n_nmt && r == QSK_OK; ++a) {
      for (int c = 0; c < 2 && r == QSK_OK; ++c) {
        if ((r = restage(b, kNmt[a], kNj[c])) != QSK_OK) break;
        for (int wb : wcand) {
          b->wblocks = wb;
          b->arena.used = 0;
          // one untimed launch, then reps timed ones; Y and W only accumulate
          if ((r = launch_sketches(b, planes, ld)) != QSK_OK) break;
          if (hipEventRecord(e0, b->stream) != hipSuccess) { r = QSK_E_HIP; break; }
          for (int t = 0; t < reps && r == QSK_OK; ++t) r = launch_sketches(b, planes, ld);
          if (r != QSK_OK) break;
          float ms = 0.0f;
          if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            r = QSK_E_HIP;
            break;
          }
          if (best < 0.0f || ms < best) { best = ms; best_c = {kNmt[a], kNj[c], wb}; }
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != QSK_OK) return r;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = best_c;
    append_tune_file(key, best_c);
  }
  if (best_c.nmt > 0) {
    qsk_status r = restage(b, best_c.nmt, best_c.nj);
    if (r != QSK_OK) return r;
    b->wblocks = best_c.wblocks;
  }
  if (nmt_out) *nmt_out = b->nmt;
  if (nj_out) *nj_out = b->nj;
  if (wblocks_out) *wblocks_out = b->wblocks;
  return QSK_OK;
}

qsk_status qsketch_batch_set_exec(qsk_batch *b, int32_t mode) {
  if (!b || mode < 0 || mode > 2) return QSK_E_ARG;
  if (b->poisoned) return QSK_E_STATE;
  b->exec_mode = mode;
  return QSK_OK;
}

qsk_status qsketch_batch_rel_error(qsk_batch *b, const void *const *planes, const int64_t *ld,
                                   double *const *Q, const int64_t *ldq, double *const *X,
                                   const int64_t *ldx, double *err) {
  if (!b || !planes || !ld || !Q || !ldq || !X || !ldx || !err) return QSK_E_ARG;
  if (b->poisoned) return QSK_E_STATE;
  hipStream_t st = b->stream;
  BCHK(b, hipStreamSynchronize(st));
  b->arena.used = 0;
  const int n_all = b->count;
  BCHK(b, hipMemsetAsync(b->err_acc, 0, 16 * (size_t)n_all, st));
  std::vector<qsk::ErrorArgs> a(n_all);
  std::vector<int64_t> nb(n_all);
  for (int i = 0; i < n_all; ++i) {
    const Prob &q = b->p[i];
    qsk::ErrorArgs &e = a[i];
    e.a[0] = planes[4 * i] ? planes[4 * i] : planes[4 * i + 1];
    for (int p = 1; p < 4; ++p) e.a[p] = planes[4 * i + p];
    e.lda = ld[i]; e.pure = q.cfg.pure; e.m = q.m; e.n = q.n;
    for (int p = 0; p < 4; ++p) { e.q[p] = Q[4 * i + p]; e.x[p] = X[4 * i + p]; }
    e.ldq = ldq[i]; e.ldx = ldx[i]; e.k = q.k; e.acc = b->err_acc + 2 * i;
    e.gx = (int)((q.m + 63) / 64); e.gy = (int)((q.n + 63) / 64);
    nb[i] = (int64_t)e.gx * e.gy;
  }
  GroupRef g;
  int64_t tot;
  if (!push_group(b, a, nb, &g, &tot)) return arena_full(b);
  BCHK(b, qsk::launch_error_k(st, b->p[0].cfg.input_dtype, a[0], g, tot));
  std::vector<double> h(2 * (size_t)n_all);
  BCHK(b, hipMemcpyAsync(h.data(), b->err_acc, 16 * (size_t)n_all, hipMemcpyDeviceToHost, st));
  BCHK(b, hipStreamSynchronize(st));
  for (int i = 0; i < n_all; ++i) err[i] = h[2 * i + 1] > 0 ? std::sqrt(h[2 * i] / h[2 * i + 1]) : 0.0;
  return QSK_OK;
}

}  // extern "C"
