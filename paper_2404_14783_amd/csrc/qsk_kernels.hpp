// Launch interfaces between the host runtime (qsketch.cpp) and the kernel
// translation units.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsk {

struct SmallStatus;
struct SketchArgs;

enum : int { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_FP8 = 3 };
enum : int { MODE_F64 = 0, MODE_F32 = 1, MODE_BF16 = 2, MODE_FP8 = 3, MODE_FP8X = 4 };

template <typename T> struct PlanesC { const T *p[4]; };
template <typename T> struct Planes { T *p[4]; };

// One column-block update of the sketches.
// Buffers of the FP8X format (e4m3 terms on the fp8 matrix cores): the
// update block quantised into T e4m3 terms, [q][t][column < CPW][row < RP]
// (qw, for the W product) and [q][t][row < RP][column < CP] (qy, for the Y
// product), and the test matrices as e4m3 bytes, Psi [4][LP][MPF] and
// Omega_J [4][KP][NPF].
struct Fp8xStage {
  uint8_t *qw = nullptr, *qy = nullptr, *psi = nullptr, *om = nullptr;
  int64_t RP = 0, CPW = 0, CP = 0, MPF = 0, NPF = 0;
  int LP = 0, KP = 0, NMT = 0, NJ = 0, T = 0, planes = 0;
  int64_t qw_bytes = 0, qy_bytes = 0, psi_bytes = 0, om_bytes = 0;
};
void fp8x_geometry(int64_t m, int l, int k, int64_t maxcols, int terms, int pure, Fp8xStage *f);
// Psi into the e4m3 staging of the FP8X format (done by the first update).
hipError_t stage_psi8(const SketchArgs &s, const Fp8xStage &f);
int fp8x_nmt(int l);

struct SketchArgs {
  hipStream_t stream;
  int mode;              // MODE_*
  int in_dtype;          // DT_* of the input planes
  const void *planes[4];
  int64_t lda;
  int pure;
  int64_t m, col0, ncols;
  int k, l;
  void *y; int64_t ldy, psy;   // Y planes: y + p * psy, element (i, j) at i + j * ldy
  int64_t pss;           // stride between the split-K copies of Y (matrix-core path)
  int y_copies;          // number of Y copies the matrix-core path may add into
  void *w; int64_t ldw, psw;
  int rad;               // 1 = Rademacher, 0 = Gaussian
  int terms;
  uint32_t k0, k1;       // Philox key
  void *scratch;         // split-K partial buffer for W (matrix-core path)
  int64_t scratch_bytes;
  float *fp8_scales;     // fp8 tile scales of the block, [4][ceil(m/32)][ceil(ncols/32)]
  int64_t fp8_scale_elems;
  int psi_ready;         // the staging buffer already holds Psi (it does not change)
  double eta = 1.0;      // scale of the products: Y += eta H Omega_J, W[:, J] += eta Psi H
  int skip_w = 0;        // Y only: no Psi staging, no W product
  int emode = -1;        // format of the test-matrix values (MODE_*); -1: that of `mode`
  int gen_rad = 1;       // matrix-core path: Rademacher tiles generated in the kernels (not staged)
  int *y_splits = nullptr;  // out (may be null): copies of Y the update added into
  const Fp8xStage *f8 = nullptr;  // FP8X buffers
  // optional timing: events[2 * kernel] before, [2 * kernel + 1] after (may be null)
  hipEvent_t *events;
};

hipError_t launch_sketch_generic(const SketchArgs &s);

// Transient staging buffers of the matrix-core path: this update's Omega_J
// ([4][KP][NP]) and Psi ([4][LP][MP]) in the operand format, regenerated from
// the Philox stream on every update.
struct MfmaStage {
  void *omega;
  void *psi;
  int LP, KP;
  int64_t MP, NP;
};
void stage_geometry(int64_t m, int l, int k, int64_t maxcols, int op_bf16, int *LP, int64_t *MP,
                    int *KP, int64_t *NP);
// Device copies of small argument tables (grouped launches).  `host` is
// pinned; push copies `bytes` to the next free slot and enqueues its upload
// on `st`, returning the device address (nullptr when full).  Reset `used`
// only after the stream has passed every launch that reads the tables.
struct ArgArena {
  char *host;
  char *dev;
  size_t cap, used;
  bool defer;          // tables only written to host; the caller copies [0, used) later
};
void *arena_push(ArgArena &a, hipStream_t st, const void *src, size_t bytes);

// Batches of problems on the matrix-core path (see batch.cpp).
void batch_tiles(const int *l, const int *k, int count, int op_bf16, int *nmt, int *nj);
void stage_geometry_tiles(int64_t m, int l, int k, int64_t maxcols, int nmt, int nj, int *LP,
                          int64_t *MP, int *KP, int64_t *NP);
// Omega (all s.ncols columns) and Psi of one problem into its staging buffers.
hipError_t stage_test_matrices(const SketchArgs &s, const MfmaStage &g);
// Y = A Omega and W = Psi A of `count` problems (s[i].col0 = 0, s[i].ncols = n)
// in one grouped launch per product.  wblocks: the number of W blocks the
// row splits aim at over all problems (more blocks: shorter row chunks).
constexpr int BATCH_W_BLOCKS = 2048;
hipError_t launch_sketch_mfma_batch(const SketchArgs *s, const MfmaStage *g, int count, int nmt,
                                    int nj, ArgArena &ar, int wblocks = BATCH_W_BLOCKS);

// Copies of Y the matrix-core Y kernel splits its columns over; Y is their sum.
constexpr int Y_COPIES = 4;
// copy 0 += copies 1 .. S-1 (each n_per_copy floats), which are cleared.
hipError_t launch_y_fold(hipStream_t st, float *y, int64_t n_per_copy, int S);
// Matrix-core path; returns hipErrorNotSupported for shapes it does not take.
hipError_t launch_sketch_mfma(const SketchArgs &s, const MfmaStage &g);
// Whether launch_sketch_mfma generates the update's test-matrix tiles in its
// kernels (then nothing is staged, and Psi must be regenerated for Psi Q).
bool gen_in_kernel(const SketchArgs &s);
// Psi alone into g.psi as a sketch of s.mode uses it.
hipError_t stage_psi(const SketchArgs &s, const MfmaStage &g);

// ---------------------------------------------------------------------------
// FP64 finalize building blocks (finalize.hip).  Small k x k quaternion
// matrices are stored as interleaved quaternions (w, x, y, z) column-major
// with leading dimension k ("AoS"); tall matrices as four planes.

// C (k1 x k2) = Z1^* Z2 over `rows` rows; Z1, Z2 planar (element types T1/T2:
// 0 = double, 1 = float).  Result written as AoS (ldc = k1) into out, using
// `partials` (size >= nchunks * k1 * k2 * 4 doubles) when rows > chunk.
hipError_t launch_crossprod(hipStream_t st, int t1, const void *const z1[4], int64_t ld1,
                            int t2, const void *const z2[4], int64_t ld2, int64_t rows, int k1,
                            int k2, double *partials, int64_t partial_elems, double *out_aos,
                            const SmallStatus *gate = nullptr);
// Same product written to planar FP64 output (used for X = S^* W).
hipError_t launch_crossprod_planar(hipStream_t st, const double *const z1[4], int64_t ld1,
                                   int t2, const void *const z2[4], int64_t ld2, int64_t rows,
                                   int k1, int k2, double *const out[4], int64_t ldo);
// Out (rows x kc, planar FP64) = Z (rows x k, planar, type tz) * C (k x kc, AoS, ldc = k).
hipError_t launch_apply(hipStream_t st, int tz, const void *const z[4], int64_t ldz, int64_t rows,
                        int k, const double *c_aos, int kc, double *const out[4], int64_t ldo,
                        int c_upper = 0, const SmallStatus *gate = nullptr);
// P (l x k, planar FP64) = Psi H with Psi regenerated as the sketch of `mode` used it.
hipError_t launch_psi_apply(hipStream_t st, int mode, int rad, uint32_t k0, uint32_t k1, int l,
                            int64_t m, const double *const h[4], int64_t ldh, int k,
                            double *partials, int64_t partial_elems, double *const p[4],
                            int64_t ldp, const void *psi_st = nullptr, int psi_st_type = 0,
                            int64_t psi_ld = 0, int64_t psi_ps = 0);
// Convert sketch planes (float or double) to FP64 planes.
// p[0 .. n) *= theta in place (T = float when tsrc != 0, else double);
// theta == 0 stores zeros.
hipError_t launch_scale(hipStream_t st, int tsrc, void *p, int64_t n, double theta);
// dst plane p (rows x cols, leading dimension ldd, planes pss apart) = the
// FP64 planes src rounded to the destination type (float when tdst != 0).
hipError_t launch_narrow(hipStream_t st, int tdst, const double *const src[4], int64_t lds,
                         void *dst, int64_t ldd, int64_t pss, int64_t rows, int64_t cols);
// X[:, 0 : ncols) (planar, ldx) = Q^* B with Q (m x k FP64 planes) and B
// the m x ncols block (element type tb: 0 double, 1 float, 2 bf16 bits).
// The m-long contraction is split in up to PROJECT_MAX_CHUNKS chunks whose
// partial sums (k x ncols AoS each) go to `partials` (partial_elems doubles)
// and are then summed; project_chunks gives the split for a shape.
constexpr int PROJECT_MAX_CHUNKS = 12;
int64_t project_chunks(int64_t m, int k, int64_t ncols);
hipError_t launch_project(hipStream_t st, const double *const q[4], int64_t ldq, int tb,
                          const void *const b[4], int64_t ldb, int64_t m, int k, int64_t ncols,
                          double *const x[4], int64_t ldx, double *partials, int64_t partial_elems);
// Rank-r truncation factors from those eigenpairs of X X^*: cu, cv (AoS
// k x r) = leading eigenvectors and the same over sigma; sigma (r).
hipError_t launch_trunc_select(hipStream_t st, const double *work, int k, int r, double *cu, double *cv,
                               double *sigma);
// Z (rows x cols, ldz) = X^* for X (cols x rows, ldx), FP64 planes.
hipError_t launch_conj_transpose(hipStream_t st, const double *const x[4], int64_t ldx, int64_t rows, int64_t cols,
                                 double *const z[4], int64_t ldz);
hipError_t launch_widen(hipStream_t st, int tsrc, const void *src, int64_t lds, int64_t pss,
                        int64_t rows, int64_t cols, double *const dst[4], int64_t ldd);
// sum over planes/columns of ||A - Q X||^2 and ||A||^2 (into acc[0], acc[1]).
hipError_t launch_error(hipStream_t st, int tin, const void *const a[4], int64_t lda, int pure,
                        int64_t m, int64_t n, const double *const q[4], int64_t ldq,
                        const double *const x[4], int64_t ldx, int k, double *acc);

// Single-workgroup small dense drivers.
struct SmallStatus {
  int fail;            // Cholesky met a non-positive pivot
  int flags;
  double min_pivot2;   // smallest pivot^2 / max diagonal
  double trace;
  int t_bad;
  int n_eps;
  double eps[8];
  double kappa;
  double kappa_initial;
  double orth_defect;
  int good_count;
  int fail_any;        // sticky: some Cholesky since the last full reset failed
  double gate;         // core solve: trace(G_P) ||R_1^{-1}||_F^2 (0: not formed)
};

// The core solve's second CholeskyQR pass is skipped when the first factor
// R_1 of P = Psi Q has kappa_F(R_1)^2 = trace(G_P) ||R_1^{-1}||_F^2 (an upper
// bound on kappa_2(P)^2) at most this: the normal-form solve with R_1 then
// has relative error below about 1e6 u.  Kernels given a gate status return
// at once when its gate lies in (0, ONE_PASS_KAPPA2].
constexpr double ONE_PASS_KAPPA2 = 1e6;

// ---------------------------------------------------------------------------
// Argument structs of the FP64 finalize kernels.  Every kernel takes its
// struct by value plus a GroupRef: with tab == nullptr it is a plain launch
// for one problem (block indices from the grid); otherwise tab points to
// `count` structs in device memory, prefix[p] is the first linear block of
// problem p (prefix[count] = total blocks), and each block finds its problem
// and its (bx, by, bz) within that problem's gx x gy x gz grid.
struct GroupRef {
  const void *tab;
  const int64_t *prefix;
  int count;
};

// Step-tile layout of the staged Psi on the matrix-core path (ES bytes per
// element): element (o, t) of a plane with 16 lp16 rows (o) and a multiple of
// 32 columns (t, the contraction index of W = Psi A) lies in the 512-element
// tile of step t / 32 and row tile o / 16, ordered [sub][g][o mod 16][e] with
// g = (t mod 32) / 8, CE = 16 / ES elements per 16 bytes, sub = (t mod 8) /
// CE and e = t mod CE.  A lane L = (o mod 16) + 16 g of the W kernel's
// direct-to-LDS load takes 16 bytes at 16 L (+ 1 KB per sub), so each load
// instruction reads 1 KB of consecutive bytes; four consecutive t from a
// multiple of 4 stay consecutive.
template <int ES>
__host__ __device__ __forceinline__ int64_t psi_tiled_index(int64_t o, int64_t t, int64_t lp16) {
  constexpr int CE = 16 / ES;
  const int64_t tt = t & 31;
  return (((t >> 5) * lp16 + (o >> 4)) << 9) + ((tt & 7) / CE) * (64 * CE) + (tt >> 3) * (16 * CE) +
         (o & 15) * CE + (tt % CE);
}

struct Gemm64Args {         // C = opA(A) B, quaternion, FP64 matrix cores (16 x 16 tiles)
  const void *a[4]; int64_t sa_i, sa_t;   // A(i, t) of plane p: a[p][i * sa_i + t * sa_t]
  const void *b[4]; int64_t sb_t, sb_j;   // B(t, j): b[p][t * sb_t + j * sb_j]
  int64_t M, N, K, kchunk;                // K split in chunks of kchunk (blockIdx.y)
  int mt, nt;                             // 16-wide tiles in M and N
  double *out[4]; int64_t ldo; int accumulate;
  double *partial;                        // split K: [chunk][N][M] AoS partial sums
  int herm;                               // C Hermitian (A = B, conj): tiles tm <= tn only
  int b_upper;                            // B upper triangular: t < 16 (tn + 1) only
  const SmallStatus *gate;                // skip when its gate passes (see ONE_PASS_KAPPA2)
  int a_tiled;                            // A is a staged Psi in the step-tile layout
  int64_t a_lp16;                         // (its rows / 16; sa_i, sa_t unused)
  int gx, gy;
};
struct ReduceArgs {
  const double *partial; int nchunks; int64_t elems; double *out;
  int herm, m;              // herm: tiles below the diagonal (16 x 16, m rows) mirror the ones above
  const SmallStatus *gate;
  int gx, gy;
};
struct ReducePlanarArgs {
  const double *partial; int nchunks, r, c;
  double *out[4]; int64_t ldo;
  int gx, gy;
};
struct PsiApplyArgs {       // partial sums of Psi H
  int mode, rad;
  uint32_t k0, k1;
  int l;
  int64_t m;
  const double *h[4]; int64_t ldh;
  int k;
  int64_t chunk;
  double *partial;
  // optional: Psi as the sketch staged it (0 none: regenerate; 1 bf16;
  // 2 fp32), element (row o, column t) of plane p at o * psi_ld + t + p * psi_ps
  const void *psi_st;
  int psi_st_type;
  int64_t psi_ld, psi_ps;
  int gx, gy;
};
struct ErrorArgs {
  const void *a[4]; int64_t lda;
  int pure;
  int64_t m, n;
  const double *q[4]; int64_t ldq;
  const double *x[4]; int64_t ldx;
  int k;
  double *acc;
  int gx, gy;
};
struct CholArgs {           // R = chol(G'), T = R^{-1}
  const double *g;
  int k, complex_only;
  double shift, tol;
  double *r, *t;
  SmallStatus *status;
  int only_failed;          // factor only where status->fail is set (the shifted retry)
  const SmallStatus *gate;
  int gx, gy;
};
struct GemmArgs {
  int k; const double *a; int opa; const double *b; int opb; double *c;
  const SmallStatus *gate;
  int gx, gy;
};
struct PowerArgs {
  int k; const double *gi; int step, n_power; uint32_t k0, k1; double *m_out; SmallStatus *status;
  int gx, gy;
};
struct PsvdArgs {
  int k; double *gl; uint32_t k0, k1; double *c, *work; SmallStatus *status; int gx, gy;
  int gs;                   // bad part through Alg. 3's Gram-Schmidt branch (else the second SVD)
};
struct PinvArgs {
  int l, k; const double *p[4]; int64_t ldp; double tol; double *work; double *out[4]; int64_t ldo;
  int gx, gy;
};
struct KappaArgs { int k; const double *gh; double *work; int which; SmallStatus *status; int gx, gy; };

// R = chol(G') with G' = G (full quaternion) or its complex part (j-part
// zeroed) when complex_only; plus `shift` * I when shift > 0; T = R^{-1}.
// A pivot^2 <= tol * max diagonal counts as a failure.
hipError_t launch_chol_inv(hipStream_t st, const double *g, int k, int complex_only, double shift,
                           double tol, double *r, double *t, SmallStatus *status,
                           const SmallStatus *gate = nullptr);
// C = opA(A) * opB(B) (k x k AoS; op = 0 none, 1 conjugate transpose).
hipError_t launch_small_gemm(hipStream_t st, int k, const double *a, int opa, const double *b,
                             int opb, double *c, const SmallStatus *gate = nullptr);
// C = T (k x k AoS copy) and status->gate = status->trace * ||T||_F^2 (the
// core solve's one-pass test, after the Cholesky of G_P wrote the trace).
hipError_t launch_core_gate(hipStream_t st, int k, const double *t, double *c, SmallStatus *status);
// One pseudo-QR correction step's eps (power iteration on G^{-1}, recorded
// in status->eps) and M = (1 - eps) I + eps G^{-1}, given gi = G^{-1}.
hipError_t launch_power_m(hipStream_t st, int k, const double *gi, int step, int n_power,
                          uint32_t k0, uint32_t k1, double *m_out, SmallStatus *status);
// pseudo-SVD selection from G_L = R_Y R_Y^* (k x k, destroyed): quaternion
// eigensolver, pair rule, bad-part repair; writes the k x k combination C
// (H = Q_Y C).  work: >= 17 k^2 + 8 k quaternion-sized doubles.
hipError_t launch_psvd_select(hipStream_t st, int k, double *gl, uint32_t k0, uint32_t k1,
                              double *c, double *work, SmallStatus *status, int gs = 0);
// kappa of H from G_H = H^* H: chol, Jacobi singular values.
// Eigenpairs of a k x k quaternion Hermitian matrix (AoS, destroyed), in
// the pseudo-SVD work layout (eigenvalues ascending).
hipError_t launch_herm_eig(hipStream_t st, int k, double *g, double *work, SmallStatus *status);
hipError_t launch_kappa(hipStream_t st, int k, const double *gh, double *work, int which,
                        SmallStatus *status);
// S^* = (P^dagger)^* (l x k planar) for a rank-deficient P by a Jacobi SVD
// of [P; I]; work holds (l + k) k quaternions.
hipError_t launch_pinv_sstar(hipStream_t st, int l, int k, const double *const p[4], int64_t ldp,
                             double tol, double *work, double *const out[4], int64_t ldo);
// identity into a k x k AoS buffer
hipError_t launch_identity(hipStream_t st, int k, double *c);

// Kernel launches taking an argument struct and a GroupRef (batched form:
// `blocks` / `count` = total linear blocks / problems of the table).
bool plan_psi_apply(int l, int64_t m, int k, int64_t partial_elems, int64_t *chunk, int64_t *nch);
// ta / tb: 0 double, 1 float, 2 bf16 bits; conj_a conjugates A's entries.
hipError_t launch_qgemm64_k(hipStream_t st, int ta, int tb, bool conj_a, const Gemm64Args &a, GroupRef g,
                            int64_t blocks);
// Arguments of the FP64 matrix-core products for one problem of a grouped
// launch; K is split in chunks of chunk_hint rows (longer where the
// partial-sum buffer is short).
//   C (AoS k1 x k2) = Z1^* Z2 through split-K partials and *r;
bool g64_plan_crossprod(const void *const z1[4], int64_t ld1, const void *const z2[4], int64_t ld2,
                        int64_t rows, int k1, int k2, double *partials, int64_t partial_elems,
                        int64_t chunk_hint, double *out_aos, Gemm64Args *g, ReduceArgs *r);
//   Out (planar) = Z1^* Z2 without a split;
Gemm64Args g64_plan_crossprod_planar(const void *const z1[4], int64_t ld1, const void *const z2[4],
                                     int64_t ld2, int64_t rows, int k1, int k2, double *const out[4],
                                     int64_t ldo);
//   Out (planar) = Z C with C AoS k x kc;
Gemm64Args g64_plan_apply(const void *const z[4], int64_t ldz, int64_t rows, int k, const double *c_aos,
                          int kc, double *const out[4], int64_t ldo, int c_upper);
//   P (planar l x k) = Psi H from the staged Psi (element size es) through
//   split-K partials and *r.
bool g64_plan_psi(const void *psi_st, int es, int64_t psi_ld, int64_t psi_ps, const double *const h[4],
                  int64_t ldh, int l, int64_t m, int k, double *partials, int64_t partial_elems,
                  int64_t chunk_hint, double *const p[4], int64_t ldp, Gemm64Args *g,
                  ReducePlanarArgs *r);
hipError_t launch_reduce_k(hipStream_t st, const ReduceArgs &a, GroupRef g, int64_t blocks);
hipError_t launch_reduce_planar_k(hipStream_t st, const ReducePlanarArgs &a, GroupRef g, int64_t blocks);
hipError_t launch_psi_apply_k(hipStream_t st, const PsiApplyArgs &a, GroupRef g, int64_t blocks);
hipError_t launch_error_k(hipStream_t st, int tin, const ErrorArgs &a, GroupRef g, int64_t blocks);
// Zero a status; keep_fail_any = 1 leaves the sticky fail_any as it is.
hipError_t launch_status_reset(hipStream_t st, SmallStatus *s, int keep_fail_any);
// count consecutive statuses, the same way
hipError_t launch_status_reset_n(hipStream_t st, SmallStatus *s, int count, int keep_fail_any);
// Zero a buffer of n16 16-byte units (grouped: one entry per buffer).
struct ZeroArgs { void *p; int64_t n16; int gx, gy; };
constexpr int ZERO_UNITS_PER_BLOCK = 1024;
hipError_t launch_zero_k(hipStream_t st, const ZeroArgs &a, GroupRef g, int64_t blocks);
hipError_t launch_chol_k(hipStream_t st, const CholArgs &a, GroupRef g, int count);
hipError_t launch_triinv_k(hipStream_t st, const CholArgs &a, GroupRef g, int64_t blocks);
hipError_t launch_gemm_k(hipStream_t st, const GemmArgs &a, GroupRef g, int64_t blocks);
hipError_t launch_power_k(hipStream_t st, const PowerArgs &a, GroupRef g, int count);
hipError_t launch_identity_k(hipStream_t st, const GemmArgs &a, GroupRef g, int count);
hipError_t launch_copy_small_k(hipStream_t st, const GemmArgs &a, GroupRef g, int count);
// The pseudo-SVD pipeline: stage 0 eigenvalues, 1 inverse iteration, 2
// re-orthogonalisation, 3 back-transformation, 4 selection; stage s uses
// psvd_blocks(k, s) workgroups per problem (the args' gx).
int psvd_blocks(int k, int stage);
hipError_t launch_psvd_stage(hipStream_t st, int stage, const PsvdArgs &a, GroupRef g, int64_t blocks);
hipError_t launch_pinv_k(hipStream_t st, const PinvArgs &a, GroupRef g, int count);
hipError_t launch_kappa_k(hipStream_t st, const KappaArgs &a, GroupRef g, int count);

}  // namespace qsk
