// Launch interfaces between the host runtime (qsketch.cpp) and the kernel
// translation units.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsk {

enum : int { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_FP8 = 3 };
enum : int { MODE_F64 = 0, MODE_F32 = 1, MODE_BF16 = 2, MODE_FP8 = 3 };

template <typename T> struct PlanesC { const T *p[4]; };
template <typename T> struct Planes { T *p[4]; };

// One column-block update of the sketches.
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
// Copies of Y the matrix-core Y kernel splits its columns over; Y is their sum.
constexpr int Y_COPIES = 4;
// copy 0 += copies 1 .. S-1 (each n_per_copy floats), which are cleared.
hipError_t launch_y_fold(hipStream_t st, float *y, int64_t n_per_copy, int S);
// Matrix-core path; returns hipErrorNotSupported for shapes it does not take.
hipError_t launch_sketch_mfma(const SketchArgs &s, const MfmaStage &g);

// ---------------------------------------------------------------------------
// FP64 finalize building blocks (finalize.hip).  Small k x k quaternion
// matrices are stored as interleaved quaternions (w, x, y, z) column-major
// with leading dimension k ("AoS"); tall matrices as four planes.

// C (k1 x k2) = Z1^* Z2 over `rows` rows; Z1, Z2 planar (element types T1/T2:
// 0 = double, 1 = float).  Result written as AoS (ldc = k1) into out, using
// `partials` (size >= nchunks * k1 * k2 * 4 doubles) when rows > chunk.
hipError_t launch_crossprod(hipStream_t st, int t1, const void *const z1[4], int64_t ld1,
                            int t2, const void *const z2[4], int64_t ld2, int64_t rows, int k1,
                            int k2, double *partials, int64_t partial_elems, double *out_aos);
// Same product written to planar FP64 output (used for X = S^* W).
hipError_t launch_crossprod_planar(hipStream_t st, const double *const z1[4], int64_t ld1,
                                   int t2, const void *const z2[4], int64_t ld2, int64_t rows,
                                   int k1, int k2, double *const out[4], int64_t ldo);
// Out (rows x kc, planar FP64) = Z (rows x k, planar, type tz) * C (k x kc, AoS, ldc = k).
hipError_t launch_apply(hipStream_t st, int tz, const void *const z[4], int64_t ldz, int64_t rows,
                        int k, const double *c_aos, int kc, double *const out[4], int64_t ldo);
// P (l x k, planar FP64) = Psi H with Psi regenerated as the sketch of `mode` used it.
hipError_t launch_psi_apply(hipStream_t st, int mode, int rad, uint32_t k0, uint32_t k1, int l,
                            int64_t m, const double *const h[4], int64_t ldh, int k,
                            double *partials, int64_t partial_elems, double *const p[4],
                            int64_t ldp);
// Convert sketch planes (float or double) to FP64 planes.
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
  int pad;
};

// R = chol(G') with G' = G (full quaternion) or its complex part (j-part
// zeroed) when complex_only; plus `shift` * I when shift > 0; T = R^{-1}.
// A pivot^2 <= tol * max diagonal counts as a failure.
hipError_t launch_chol_inv(hipStream_t st, const double *g, int k, int complex_only, double shift,
                           double tol, double *r, double *t, SmallStatus *status);
// C = opA(A) * opB(B) (k x k AoS; op = 0 none, 1 conjugate transpose).
hipError_t launch_small_gemm(hipStream_t st, int k, const double *a, int opa, const double *b,
                             int opb, double *c);
// One pseudo-QR correction step's eps (power iteration on G^{-1}, recorded
// in status->eps) and M = (1 - eps) I + eps G^{-1}, given gi = G^{-1}.
hipError_t launch_power_m(hipStream_t st, int k, const double *gi, int step, int n_power,
                          uint32_t k0, uint32_t k1, double *m_out, SmallStatus *status);
// pseudo-SVD selection from G_L = R_Y R_Y^* (k x k, destroyed): quaternion
// eigensolver, pair rule, bad-part repair; writes the k x k combination C
// (H = Q_Y C).  work: >= 17 k^2 + 8 k quaternion-sized doubles.
hipError_t launch_psvd_select(hipStream_t st, int k, double *gl, uint32_t k0, uint32_t k1,
                              double *c, double *work, SmallStatus *status);
// kappa of H from G_H = H^* H: chol, Jacobi singular values.
hipError_t launch_kappa(hipStream_t st, int k, const double *gh, double *work, int which,
                        SmallStatus *status);
// S^* = (P^dagger)^* (l x k planar) for a rank-deficient P by a Jacobi SVD
// of [P; I]; work holds (l + k) k quaternions.
hipError_t launch_pinv_sstar(hipStream_t st, int l, int k, const double *const p[4], int64_t ldp,
                             double tol, double *work, double *const out[4], int64_t ldo);
// identity into a k x k AoS buffer
hipError_t launch_identity(hipStream_t st, int k, double *c);

}  // namespace qsk
