// FP64 finalize kernels for the QB stage (Alg. 4): CholeskyQR passes over the
// sketch Y (its quaternion Gram and the right-multiplication by small factors),
// Psi H with Psi regenerated, the cross product for the least-squares core
// solve, the error measurement pass, and single-workgroup drivers for the
// small dense k x k quaternion algebra (Cholesky, triangular inverse,
// products, the pseudo-QR corrections, one-sided Jacobi SVD, pseudo-SVD pair
// selection and repair).
#include <algorithm>

#include "qsk_device.hpp"
#include "qsk_kernels.hpp"

namespace qsk {

template <typename T> __device__ __forceinline__ double ldv(const T *p, int64_t i) { return (double)gp(p)[i]; }

template <typename T>
__device__ __forceinline__ qd load_q(const PlanesC<T> &z, int64_t idx) {
  return {ldv(z.p[0], idx), ldv(z.p[1], idx), ldv(z.p[2], idx), ldv(z.p[3], idx)};
}

template <typename T, typename P>
__device__ __forceinline__ PlanesC<T> mkc_d(const P (&z)[4]) {
  PlanesC<T> r;
  for (int q = 0; q < 4; ++q) r.p[q] = (const T *)z[q];
  return r;
}

// A launch given a gate status whose core-solve gate passes does nothing.
__device__ __forceinline__ bool gate_skip(const SmallStatus *g) {
  if (!g) return false;
  const double v = *(const volatile double *)&g->gate;
  return v > 0.0 && v <= ONE_PASS_KAPPA2;
}

// The problem and block indices of this block (see GroupRef).
template <typename A>
__device__ __forceinline__ bool group_select(const A &a0, const GroupRef &g, A &a, int &bx, int &by,
                                             int &bz) {
  if (!g.tab) {
    a = a0;
    bx = blockIdx.x; by = blockIdx.y; bz = blockIdx.z;
    return true;
  }
  int p;
  int64_t local;
  group_find(g, &p, &local);
  a = ((const A *)g.tab)[p];
  bx = (int)(local % a.gx);
  by = (int)((local / a.gx) % a.gy);
  bz = (int)(local / ((int64_t)a.gx * a.gy));
  return true;
}

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Quaternion FP64 products on the matrix cores: C = opA(A) B with
// opA(A)(i, t) = A(i, t) or its conjugate, as 16 real products per 16 x 16
// output tile (v_mfma_f64_16x16x4_f64, K = 4 per instruction).  Element
// (i, t) of plane p of A is a[p][i * sa_i + t * sa_t] (types double, float
// or bf16 bits), element (t, j) of B is b[p][t * sb_t + j * sb_j]; so the
// same kernel serves Z1^* Z2 (Gram matrices), Z T, Psi Q and S^* W.  One
// wave per output tile, four tiles per workgroup, one chunk of K per
// blockIdx.y; the operands of the next K step are loaded while the matrix
// cores work on this one.  Lane l supplies A(i0 + l mod 16, t0 + l / 16) and
// B(t0 + l / 16, j0 + l mod 16) and holds C(i0 + l / 16 + 4 u, j0 + l mod 16),
// u = 0..3.  Output: planar (out, ldo; accumulate adds) or, for a split K,
// AoS partial sums partial[((chunk * N + j) * M + i) * 4 + p].
typedef __attribute__((ext_vector_type(4))) double v4d;
template <typename T> __device__ __forceinline__ double ld64(const void *p, int64_t i);
template <> __device__ __forceinline__ double ld64<double>(const void *p, int64_t i) { return gp((const double *)p)[i]; }
template <> __device__ __forceinline__ double ld64<float>(const void *p, int64_t i) { return gp((const float *)p)[i]; }
template <> __device__ __forceinline__ double ld64<uint16_t>(const void *p, int64_t i) {
  return __uint_as_float(((uint32_t)gp((const uint16_t *)p)[i]) << 16);
}

// Hamilton product a b: plane p of the result takes sign * a_q * b_{qsel(p, q)}
__device__ constexpr int hp_b(int p, int q) {
  constexpr int t[4][4] = {{0, 1, 2, 3}, {1, 0, 3, 2}, {2, 3, 0, 1}, {3, 2, 1, 0}};
  return t[p][q];
}
__device__ constexpr int hp_s(int p, int q) {   // +1 / -1
  constexpr int t[4][4] = {{1, -1, -1, -1}, {1, 1, 1, -1}, {1, -1, 1, 1}, {1, 1, -1, 1}};
  return t[p][q];
}

// Loads of 4 operand values at t, t + 1, t + 2, t + 3: one vector load when
// t is the contiguous index (CONT), else four strided loads.
template <typename T, bool CONT>
__device__ __forceinline__ void ld64x4(const void *p, int64_t base, int64_t st, double (&v)[4]) {
  if constexpr (CONT && sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2), aligned(8)));   // element alignment only
    const QSK_GLOBAL d2 *q = (const QSK_GLOBAL d2 *)((const double *)p + base);
    const d2 x = q[0], y = q[1];
    v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
  } else if constexpr (CONT && sizeof(T) == 4) {
    typedef float f4 __attribute__((ext_vector_type(4), aligned(4)));
    const f4 x = *(const QSK_GLOBAL f4 *)((const float *)p + base);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else if constexpr (CONT && sizeof(T) == 2) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2), aligned(2)));
    const u2 x = *(const QSK_GLOBAL u2 *)((const uint16_t *)p + base);
    v[0] = __uint_as_float(x.x << 16); v[1] = __uint_as_float(x.x & 0xFFFF0000u);
    v[2] = __uint_as_float(x.y << 16); v[3] = __uint_as_float(x.y & 0xFFFF0000u);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = ld64<T>(p, base + s * st);
  }
}

// Output tile of a wave: column-major over the mt x nt tiles, or over the
// tiles on and above the diagonal (tm <= tn, column by column) for a
// Hermitian product.
__device__ __forceinline__ bool g64_tile(const Gemm64Args &A, int tile, int *tm, int *tn) {
  if (A.herm) {
    if (tile >= A.mt * (A.mt + 1) / 2) return false;
    int c = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((c + 1) * (c + 2) / 2 <= tile) ++c;
    while (c * (c + 1) / 2 > tile) --c;
    *tn = c;
    *tm = tile - c * (c + 1) / 2;
    return true;
  }
  if (tile >= A.mt * A.nt) return false;
  *tm = tile % A.mt;
  *tn = tile / A.mt;
  return true;
}

// ATILE: A is a staged Psi in the step-tile layout (psi_tiled_index)
template <typename TA, typename TB, bool CONJ_A, bool ACONT, bool BCONT, bool ATILE = false>
__global__ __launch_bounds__(256) void qgemm64_k(Gemm64Args args, GroupRef grp) {
  Gemm64Args A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  if (gate_skip(A.gate)) return;
  const int lane = threadIdx.x & 63;
  const int tile = bx * 4 + (threadIdx.x >> 6);
  int tm, tn;
  if (!g64_tile(A, tile, &tm, &tn)) return;              // whole wave
  const int64_t i = (int64_t)tm * 16 + (lane & 15);      // A row of this lane
  const int64_t j = (int64_t)tn * 16 + (lane & 15);      // B column of this lane
  const int kq = lane >> 4;
  const int64_t kb = (int64_t)by * A.kchunk;
  const int64_t ke = min(A.b_upper ? min(A.K, (int64_t)tn * 16 + 16) : A.K, kb + A.kchunk);
  const bool iok = i < A.M, jok = j < A.N;
  const int64_t ai = (iok ? i : 0) * A.sa_i, bj = (jok ? j : 0) * A.sb_j;
#define QSK_G64_AIDX(T_) (ATILE ? psi_tiled_index<(int)sizeof(TA)>(iok ? i : 0, (T_), A.a_lp16) : ai + (T_) * A.sa_t)
  v4d acc[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) acc[p] = {0.0, 0.0, 0.0, 0.0};
  // super-steps of 16 values of t: K slot kq of the s-th instruction is
  // t = t0 + 4 kq + s, so each lane reads 4 consecutive t per operand
  double na[4][4], nb[4][4];
#define QSK_G64_LOAD(T0)                                                               \
  do {                                                                                 \
    const int64_t t_ = (T0) + 4 * kq;                                                  \
    if ((T0) + 16 <= ke) {                                                             \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                  \
        ld64x4<TA, ACONT>(A.a[q], QSK_G64_AIDX(t_), A.sa_t, na[q]);                    \
        ld64x4<TB, BCONT>(A.b[q], t_ * A.sb_t + bj, A.sb_t, nb[q]);                    \
      }                                                                                \
    } else {                                                                           \
      _Pragma("unroll") for (int q = 0; q < 4; ++q)                                    \
        _Pragma("unroll") for (int s = 0; s < 4; ++s) {                                \
          const bool in_ = t_ + s < ke;                                                \
          const int64_t tc_ = in_ ? t_ + s : kb;                                       \
          const double x_ = ld64<TA>(A.a[q], QSK_G64_AIDX(tc_));                       \
          const double y_ = ld64<TB>(A.b[q], tc_ * A.sb_t + bj);                       \
          na[q][s] = in_ ? x_ : 0.0;                                                   \
          nb[q][s] = in_ ? y_ : 0.0;                                                   \
        }                                                                              \
    }                                                                                  \
    if (!iok) _Pragma("unroll") for (int q = 0; q < 4; ++q) _Pragma("unroll") for (int s = 0; s < 4; ++s) na[q][s] = 0.0; \
    if (!jok) _Pragma("unroll") for (int q = 0; q < 4; ++q) _Pragma("unroll") for (int s = 0; s < 4; ++s) nb[q][s] = 0.0; \
  } while (0)
  QSK_G64_LOAD(kb);
  for (int64_t t0 = kb; t0 < ke; t0 += 16) {
    double xa[4][4], xb[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) { xa[q][s] = CONJ_A && q > 0 ? -na[q][s] : na[q][s]; xb[q][s] = nb[q][s]; }
    if (t0 + 16 < ke) QSK_G64_LOAD(t0 + 16);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double aq = xa[q][s], naq = -xa[q][s];
#pragma unroll
        for (int p = 0; p < 4; ++p)
          acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(hp_s(p, q) > 0 ? aq : naq, xb[hp_b(p, q)][s], acc[p], 0, 0, 0);
      }
  }
#undef QSK_G64_LOAD
#undef QSK_G64_AIDX
  if (!jok) return;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t r = (int64_t)tm * 16 + kq + 4 * u;
    if (r >= A.M) continue;
    if (A.partial) {
      QSK_GLOBAL double *q = gpw(A.partial) + 4 * (((int64_t)by * A.N + j) * A.M + r);
      q[0] = acc[0][u]; q[1] = acc[1][u]; q[2] = acc[2][u]; q[3] = acc[3][u];
    } else {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        QSK_GLOBAL double *o = gpw(A.out[p]) + r + j * A.ldo;
        *o = A.accumulate ? *o + acc[p][u] : acc[p][u];
      }
    }
  }
}

// Strided operands (t not contiguous): one K step of 4 per iteration, one
// value per lane and plane.
template <typename TA, typename TB, bool CONJ_A>
__global__ __launch_bounds__(256) void qgemm64s_k(Gemm64Args args, GroupRef grp) {
  Gemm64Args A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  if (gate_skip(A.gate)) return;
  const int lane = threadIdx.x & 63;
  const int tile = bx * 4 + (threadIdx.x >> 6);
  int tm, tn;
  if (!g64_tile(A, tile, &tm, &tn)) return;              // whole wave
  const int64_t i = (int64_t)tm * 16 + (lane & 15);      // A row of this lane
  const int64_t j = (int64_t)tn * 16 + (lane & 15);      // B column of this lane
  const int kq = lane >> 4;
  const int64_t kb = (int64_t)by * A.kchunk;
  const int64_t ke = min(A.b_upper ? min(A.K, (int64_t)tn * 16 + 16) : A.K, kb + A.kchunk);
  const bool iok = i < A.M, jok = j < A.N;
  const int64_t ai = (iok ? i : 0) * A.sa_i, bj = (jok ? j : 0) * A.sb_j;
  v4d acc[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) acc[p] = {0.0, 0.0, 0.0, 0.0};
  double na[4], nb[4];
#define QSK_G64_LOAD(T0)                                                               \
  do {                                                                                 \
    const int64_t t_ = (T0) + kq;                                                      \
    const bool ta_ = iok && t_ < ke, tb_ = jok && t_ < ke;                              \
    const int64_t tc_ = t_ < ke ? t_ : kb;                                             \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                    \
      const double x_ = ld64<TA>(A.a[q], ai + tc_ * A.sa_t);                          \
      const double y_ = ld64<TB>(A.b[q], tc_ * A.sb_t + bj);                           \
      na[q] = ta_ ? x_ : 0.0;                                                          \
      nb[q] = tb_ ? y_ : 0.0;                                                          \
    }                                                                                  \
  } while (0)
  QSK_G64_LOAD(kb);
  for (int64_t t0 = kb; t0 < ke; t0 += 4) {
    double xa[4], xb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) { xa[q] = CONJ_A && q > 0 ? -na[q] : na[q]; xb[q] = nb[q]; }
    if (t0 + 4 < ke) QSK_G64_LOAD(t0 + 4);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double aq = xa[q], naq = -xa[q];
#pragma unroll
      for (int p = 0; p < 4; ++p)
        acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(hp_s(p, q) > 0 ? aq : naq, xb[hp_b(p, q)], acc[p], 0, 0, 0);
    }
  }
#undef QSK_G64_LOAD
  if (!jok) return;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t r = (int64_t)tm * 16 + kq + 4 * u;
    if (r >= A.M) continue;
    if (A.partial) {
      QSK_GLOBAL double *q = gpw(A.partial) + 4 * (((int64_t)by * A.N + j) * A.M + r);
      q[0] = acc[0][u]; q[1] = acc[1][u]; q[2] = acc[2][u]; q[3] = acc[3][u];
    } else {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        QSK_GLOBAL double *o = gpw(A.out[p]) + r + j * A.ldo;
        *o = A.accumulate ? *o + acc[p][u] : acc[p][u];
      }
    }
  }
}

// Out = Z C for a tall Z (A(i, t) = z[p][i + t sa_t], rows contiguous) and a
// small C stored AoS (B(t, j) = the four planes at b[0] + t sb_t + j sb_j,
// consecutive): one wave per 16 rows and up to four 16-wide column tiles,
// so each value of Z is loaded once per four output tiles; one K step of 4
// per iteration, the next step's operands loaded while the matrix cores
// work.  blockIdx.x: four 16-row tiles, blockIdx.y: a group of four column
// tiles.
template <typename TA>
__global__ __launch_bounds__(256) void qgemm64w_k(Gemm64Args A) {
  if (gate_skip(A.gate)) return;
  const int lane = threadIdx.x & 63;
  const int tm = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tm >= A.mt) return;                                // whole wave
  const int tn0 = blockIdx.y * 4;
  const int ntl = min(4, A.nt - tn0);
  const int64_t i = (int64_t)tm * 16 + (lane & 15);
  const int kq = lane >> 4;
  const bool iok = i < A.M;
  const int64_t ai = (iok ? i : 0) * A.sa_i;
  const int64_t ke = A.b_upper ? min(A.K, (int64_t)(tn0 + ntl) * 16) : A.K;
  const double *bq = (const double *)A.b[0];
  int64_t bj[4];
  bool jok[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t j = (int64_t)(tn0 + u) * 16 + (lane & 15);
    jok[u] = u < ntl && j < A.N;
    bj[u] = (jok[u] ? j : 0) * A.sb_j;
  }
  v4d acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[u][p] = {0.0, 0.0, 0.0, 0.0};
  // A (the tall operand, from HBM) is loaded one step ahead; B (small,
  // cached) when its step comes
  double na[4];
  typedef double d2 __attribute__((ext_vector_type(2), aligned(8)));
#define QSK_G64W_LOAD_A(T0)                                                            \
  do {                                                                                 \
    const int64_t t_ = (T0) + kq;                                                      \
    const bool tin_ = t_ < ke;                                                         \
    const int64_t tc_ = tin_ ? t_ : 0;                                                 \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                    \
      const double x_ = ld64<TA>(A.a[q], ai + tc_ * A.sa_t);                          \
      na[q] = (tin_ && iok) ? x_ : 0.0;                                                \
    }                                                                                  \
  } while (0)
  QSK_G64W_LOAD_A(0);
  for (int64_t t0 = 0; t0 < ke; t0 += 4) {
    double xa[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) xa[q] = na[q];
    if (t0 + 4 < ke) QSK_G64W_LOAD_A(t0 + 4);
    const int64_t t = t0 + kq;
    const bool tin = t < ke;
    const int64_t tc = tin ? t : 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      // column tile u takes part while t is inside it (B upper triangular:
      // rows below 16 (tn + 1) only); wave-uniform
      if (u >= ntl || (A.b_upper && t0 >= (int64_t)(tn0 + u + 1) * 16)) continue;
      const QSK_GLOBAL d2 *bp = (const QSK_GLOBAL d2 *)(bq + tc * A.sb_t + bj[u]);
      const d2 v0 = bp[0], v1 = bp[1];
      const bool ok = tin && jok[u];
      const double xb[4] = {ok ? v0.x : 0.0, ok ? v0.y : 0.0, ok ? v1.x : 0.0, ok ? v1.y : 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double aq = xa[q], naq = -xa[q];
#pragma unroll
        for (int p = 0; p < 4; ++p)
          acc[u][p] = __builtin_amdgcn_mfma_f64_16x16x4f64(hp_s(p, q) > 0 ? aq : naq, xb[hp_b(p, q)],
                                                          acc[u][p], 0, 0, 0);
      }
    }
  }
#undef QSK_G64W_LOAD_A
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (!jok[u]) continue;
    const int64_t j = (int64_t)(tn0 + u) * 16 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = (int64_t)tm * 16 + kq + 4 * v;
      if (r >= A.M) continue;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        QSK_GLOBAL double *o = gpw(A.out[p]) + r + j * A.ldo;
        *o = A.accumulate ? *o + acc[u][p][v] : acc[u][p][v];
      }
    }
  }
}

hipError_t launch_qgemm64_k(hipStream_t st, int ta, int tb, bool conj_a, const Gemm64Args &a, GroupRef g,
                            int64_t blocks) {
  const dim3 grid = g.tab ? dim3((unsigned)blocks) : dim3((unsigned)a.gx, (unsigned)a.gy);
  // ta / tb: 0 double, 1 float, 2 bf16; vector loads where t is contiguous
  const bool ac = a.sa_t == 1, bc = a.sb_t == 1;
#define QSK_G64(TA, TB, CJ)                                                                       \
  do {                                                                                             \
    if (ac && bc) hipLaunchKernelGGL((qgemm64_k<TA, TB, CJ, true, true>), grid, dim3(256), 0, st, a, g);   \
    else hipLaunchKernelGGL((qgemm64s_k<TA, TB, CJ>), grid, dim3(256), 0, st, a, g);                      \
  } while (0)
  if (conj_a) {
    if (ta == 0 && tb == 0) QSK_G64(double, double, true);
    else if (ta == 0 && tb == 1) QSK_G64(double, float, true);
    else if (ta == 0 && tb == 2) QSK_G64(double, uint16_t, true);
    else if (ta == 1 && tb == 1) QSK_G64(float, float, true);
    else return hipErrorInvalidValue;
  } else if (a.a_tiled) {
    // a staged Psi (contiguous in t within its step tiles) times H
    if (!bc) return hipErrorInvalidValue;
    if (ta == 1 && tb == 0) hipLaunchKernelGGL((qgemm64_k<float, double, false, true, true, true>), grid, dim3(256), 0, st, a, g);
    else if (ta == 2 && tb == 0) hipLaunchKernelGGL((qgemm64_k<uint16_t, double, false, true, true, true>), grid, dim3(256), 0, st, a, g);
    else return hipErrorInvalidValue;
  } else {
    if (ta == 0 && tb == 0) QSK_G64(double, double, false);
    else if (ta == 1 && tb == 0) QSK_G64(float, double, false);
    else if (ta == 2 && tb == 0) QSK_G64(uint16_t, double, false);
    else return hipErrorInvalidValue;
  }
#undef QSK_G64
  return hipGetLastError();
}

__global__ void reduce_chunks_k(ReduceArgs args, GroupRef grp) {
  ReduceArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  if (gate_skip(A.gate)) return;
  const double *partial = A.partial;
  const int nchunks = A.nchunks;
  const int64_t elems = A.elems;
  double *out = A.out;
  const int64_t e = (int64_t)bx * blockDim.x + threadIdx.x;
  if (e >= elems) return;
  int64_t src = e;
  double sg = 1.0;
  if (A.herm) {
    // element (i, j), plane p of an m x m AoS matrix; tiles below the
    // diagonal were not computed: C(i, j) = conj(C(j, i))
    const int p = (int)(e & 3);
    const int64_t ij = e >> 2, i = ij % A.m, j = ij / A.m;
    if (i / 16 > j / 16) {
      src = 4 * (i * A.m + j) + p;
      if (p > 0) sg = -1.0;
    }
  }
  // sixteen loads in flight at a time, added in chunk order
  double s = 0.0;
  int c = 0;
  for (; c + 16 <= nchunks; c += 16) {
    double a[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) a[u] = gp(partial)[(int64_t)(c + u) * elems + src];
#pragma unroll
    for (int u = 0; u < 16; ++u) s += a[u];
  }
  for (; c < nchunks; ++c) s += gp(partial)[(int64_t)c * elems + src];
  gpw(out)[e] = sg * s;
}

// AoS (r x c, ld = r) partial sums -> planar output.
__global__ void reduce_chunks_planar_k(ReducePlanarArgs args, GroupRef grp) {
  ReducePlanarArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  const double *partial = A.partial;
  const int nchunks = A.nchunks, r = A.r, c = A.c;
  Planes<double> out;
  for (int q = 0; q < 4; ++q) out.p[q] = A.out[q];
  const int64_t ldo = A.ldo;
  const int64_t e = (int64_t)bx * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)r * c;
  if (e >= n) return;
  const int i = (int)(e % r), j = (int)(e / r);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int ch = 0;
  for (; ch + 4 <= nchunks; ch += 4) {           // four chunks' loads in flight, added in order
    double a[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int p = 0; p < 4; ++p) a[u][p] = gp(partial)[((int64_t)(ch + u) * n + e) * 4 + p];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int p = 0; p < 4; ++p) s[p] += a[u][p];
  }
  for (; ch < nchunks; ++ch)
    for (int p = 0; p < 4; ++p) s[p] += gp(partial)[((int64_t)ch * n + e) * 4 + p];
  for (int p = 0; p < 4; ++p) gpw(out.p[p])[i + (int64_t)j * ldo] = s[p];
}

static int64_t chunk_rows(int64_t rows, int tiles, int64_t max_chunks) {
  // aim for >= ~1024 blocks; chunk a multiple of 32 rows
  int64_t want = (1024 + tiles - 1) / tiles;
  if (want < 1) want = 1;
  if (want > max_chunks) want = max_chunks;
  int64_t chunk = (rows + want - 1) / want;
  chunk = ((chunk + 31) / 32) * 32;
  if (chunk < 256) chunk = 256;
  return chunk;
}

static void set_planes(double *dst[4], double *const src[4]) {
  for (int q = 0; q < 4; ++q) dst[q] = src[q];
}
static void set_planes(const double *dst[4], const double *const src[4]) {
  for (int q = 0; q < 4; ++q) dst[q] = src[q];
}

hipError_t launch_reduce_k(hipStream_t st, const ReduceArgs &a, GroupRef g, int64_t blocks) {
  hipLaunchKernelGGL(reduce_chunks_k, dim3((unsigned)(g.tab ? blocks : a.gx)), dim3(256), 0, st, a, g);
  return hipGetLastError();
}

hipError_t launch_reduce_planar_k(hipStream_t st, const ReducePlanarArgs &a, GroupRef g,
                                  int64_t blocks) {
  hipLaunchKernelGGL(reduce_chunks_planar_k, dim3((unsigned)(g.tab ? blocks : a.gx)), dim3(256), 0,
                     st, a, g);
  return hipGetLastError();
}

// Split of K for the matrix-core products: about 4096 waves in all (four
// per SIMD), chunks a multiple of 16, at most max_chunks of them.
static int64_t g64_chunk(int64_t K, int64_t tiles, int64_t max_chunks, int64_t *nch) {
  int64_t want = (4096 + tiles - 1) / tiles;
  if (want > max_chunks) want = max_chunks;
  if (want < 1) want = 1;
  int64_t chunk = (K + want - 1) / want;
  chunk = (chunk + 15) / 16 * 16;
  if (chunk < 64) chunk = 64;
  *nch = (K + chunk - 1) / chunk;
  return chunk;
}

static bool same_planes(const void *const a[4], const void *const b[4]) {
  return a[0] == b[0] && a[1] == b[1] && a[2] == b[2] && a[3] == b[3];
}
static int64_t g64_tiles(const Gemm64Args &g) {
  return g.herm ? (int64_t)g.mt * (g.mt + 1) / 2 : (int64_t)g.mt * g.nt;
}
// Hermitian product: only the tiles on and above the diagonal
static void g64_set_herm(Gemm64Args &g, bool herm) {
  g.herm = herm ? 1 : 0;
  g.gx = (int)((g64_tiles(g) + 3) / 4);
}

static Gemm64Args g64_args(const void *const a[4], int64_t sa_i, int64_t sa_t, const void *const b[4],
                           int64_t sb_t, int64_t sb_j, int64_t M, int64_t N, int64_t K) {
  Gemm64Args g{};
  for (int p = 0; p < 4; ++p) { g.a[p] = a[p]; g.b[p] = b[p]; }
  g.sa_i = sa_i; g.sa_t = sa_t; g.sb_t = sb_t; g.sb_j = sb_j;
  g.M = M; g.N = N; g.K = K; g.kchunk = K;
  g.mt = (int)((M + 15) / 16); g.nt = (int)((N + 15) / 16);
  g.gx = (g.mt * g.nt + 3) / 4; g.gy = 1;
  return g;
}

hipError_t launch_crossprod(hipStream_t st, int t1, const void *const z1[4], int64_t ld1, int t2,
                            const void *const z2[4], int64_t ld2, int64_t rows, int k1, int k2,
                            double *partials, int64_t partial_elems, double *out_aos,
                            const SmallStatus *gate) {
  // C(i, j) = sum_t conj(Z1(t, i)) Z2(t, j) on the FP64 matrix cores, K split
  const int64_t max_chunks = partial_elems / ((int64_t)k1 * k2 * 4);
  if (max_chunks < 1) return hipErrorInvalidValue;
  Gemm64Args g = g64_args(z1, ld1, 1, z2, 1, ld2, k1, k2, rows);
  g.gate = gate;
  g64_set_herm(g, t1 == t2 && ld1 == ld2 && k1 == k2 && same_planes(z1, z2));
  int64_t nch;
  g.kchunk = g64_chunk(rows, g64_tiles(g), max_chunks, &nch);
  g.gy = (int)nch;
  g.partial = partials;
  hipError_t e = launch_qgemm64_k(st, t1, t2, true, g, GroupRef{}, 0);
  if (e != hipSuccess) return e;
  ReduceArgs r{};
  r.partial = partials; r.nchunks = (int)nch; r.elems = (int64_t)k1 * k2 * 4; r.out = out_aos;
  r.herm = g.herm; r.m = k1; r.gate = gate;
  r.gx = (int)((r.elems + 255) / 256); r.gy = 1;
  return launch_reduce_k(st, r, GroupRef{}, r.gx);
}

hipError_t launch_crossprod_planar(hipStream_t st, const double *const z1[4], int64_t ld1, int t2,
                                   const void *const z2[4], int64_t ld2, int64_t rows, int k1,
                                   int k2, double *const out[4], int64_t ldo) {
  const void *zz[4] = {z1[0], z1[1], z1[2], z1[3]};
  Gemm64Args g = g64_args(zz, ld1, 1, z2, 1, ld2, k1, k2, rows);
  for (int p = 0; p < 4; ++p) g.out[p] = out[p];
  g.ldo = ldo;
  return launch_qgemm64_k(st, 0, t2, true, g, GroupRef{}, 0);
}

int64_t project_chunks(int64_t m, int k, int64_t ncols) {
  // about 8 waves per SIMD over the output tiles and the chunks of the
  // m-long contraction, chunks of at least 256 rows
  const int64_t tiles = ((k + 15) / 16) * ((ncols + 15) / 16);
  int64_t want = (8192 + tiles - 1) / tiles;
  want = std::min<int64_t>(want, std::max<int64_t>(1, m / 256));
  return std::max<int64_t>(1, std::min<int64_t>(want, PROJECT_MAX_CHUNKS));
}

hipError_t launch_project(hipStream_t st, const double *const q[4], int64_t ldq, int tb,
                          const void *const b[4], int64_t ldb, int64_t m, int k, int64_t ncols,
                          double *const x[4], int64_t ldx, double *partials, int64_t partial_elems) {
  if ((int64_t)(int)ncols != ncols) return hipErrorInvalidValue;
  const int64_t per_chunk = (int64_t)k * ncols * 4;
  int64_t want = project_chunks(m, k, ncols);
  if (!partials) want = 1;
  want = std::min<int64_t>(want, partial_elems / per_chunk);
  if (want < 2) return launch_crossprod_planar(st, q, ldq, tb, b, ldb, m, k, (int)ncols, x, ldx);
  const void *qq[4] = {q[0], q[1], q[2], q[3]};
  Gemm64Args g = g64_args(qq, ldq, 1, b, 1, ldb, k, ncols, m);
  int64_t chunk = ((m + want - 1) / want + 15) / 16 * 16;
  const int64_t nch = (m + chunk - 1) / chunk;
  g.kchunk = chunk;
  g.gy = (int)nch;
  g.partial = partials;
  hipError_t e = launch_qgemm64_k(st, 0, tb, true, g, GroupRef{}, 0);
  if (e != hipSuccess) return e;
  ReducePlanarArgs r{};
  r.partial = partials; r.nchunks = (int)nch; r.r = k; r.c = (int)ncols;
  set_planes(r.out, x); r.ldo = ldx;
  r.gx = (int)((per_chunk / 4 + 255) / 256); r.gy = 1;
  return launch_reduce_planar_k(st, r, GroupRef{}, r.gx);
}

// Split of K for one problem of a grouped launch: chunks of chunk_hint rows
// (the same for every problem, so that all waves get about the same work),
// fewer and longer where the partial-sum buffer holds fewer.
static int64_t g64_group_chunk(int64_t K, int64_t chunk_hint, int64_t max_chunks, int64_t *nch) {
  int64_t chunk = chunk_hint < 16 ? 16 : (chunk_hint + 15) / 16 * 16;
  const int64_t least = ((K + max_chunks - 1) / max_chunks + 15) / 16 * 16;
  if (chunk < least) chunk = least;
  *nch = (K + chunk - 1) / chunk;
  return chunk;
}

bool g64_plan_crossprod(const void *const z1[4], int64_t ld1, const void *const z2[4], int64_t ld2,
                        int64_t rows, int k1, int k2, double *partials, int64_t partial_elems,
                        int64_t chunk_hint, double *out_aos, Gemm64Args *g, ReduceArgs *r) {
  const int64_t max_chunks = partial_elems / ((int64_t)k1 * k2 * 4);
  if (max_chunks < 1) return false;
  *g = g64_args(z1, ld1, 1, z2, 1, ld2, k1, k2, rows);
  g64_set_herm(*g, ld1 == ld2 && k1 == k2 && same_planes(z1, z2));
  int64_t nch;
  g->kchunk = g64_group_chunk(rows, chunk_hint, max_chunks, &nch);
  g->gy = (int)nch;
  g->partial = partials;
  *r = ReduceArgs{};
  r->partial = partials; r->nchunks = (int)nch; r->elems = (int64_t)k1 * k2 * 4; r->out = out_aos;
  r->herm = g->herm; r->m = k1;
  r->gx = (int)((r->elems + 255) / 256); r->gy = 1;
  return true;
}

Gemm64Args g64_plan_crossprod_planar(const void *const z1[4], int64_t ld1, const void *const z2[4],
                                     int64_t ld2, int64_t rows, int k1, int k2, double *const out[4],
                                     int64_t ldo) {
  Gemm64Args g = g64_args(z1, ld1, 1, z2, 1, ld2, k1, k2, rows);
  for (int p = 0; p < 4; ++p) g.out[p] = out[p];
  g.ldo = ldo;
  return g;
}

Gemm64Args g64_plan_apply(const void *const z[4], int64_t ldz, int64_t rows, int k, const double *c_aos,
                          int kc, double *const out[4], int64_t ldo, int c_upper) {
  const void *cp[4] = {c_aos, c_aos + 1, c_aos + 2, c_aos + 3};
  Gemm64Args g = g64_args(z, 1, ldz, cp, 4, 4 * (int64_t)k, rows, kc, k);
  g.b_upper = c_upper;
  for (int p = 0; p < 4; ++p) g.out[p] = out[p];
  g.ldo = ldo;
  return g;
}

bool g64_plan_psi(const void *psi_st, int es, int64_t psi_ld, int64_t psi_ps, const double *const h[4],
                  int64_t ldh, int l, int64_t m, int k, double *partials, int64_t partial_elems,
                  int64_t chunk_hint, double *const p[4], int64_t ldp, Gemm64Args *g,
                  ReducePlanarArgs *r) {
  const int64_t max_chunks = partial_elems / ((int64_t)l * k * 4);
  if (max_chunks < 1) return false;
  const void *pp[4];
  for (int q = 0; q < 4; ++q) pp[q] = (const char *)psi_st + (size_t)q * psi_ps * es;
  const void *hh[4] = {h[0], h[1], h[2], h[3]};
  *g = g64_args(pp, psi_ld, 1, hh, 1, ldh, l, k, m);
  g->a_tiled = 1;
  g->a_lp16 = psi_ps / psi_ld / 16;
  int64_t nch;
  g->kchunk = g64_group_chunk(m, chunk_hint, max_chunks, &nch);
  g->gy = (int)nch;
  g->partial = partials;
  *r = ReducePlanarArgs{};
  r->partial = partials; r->nchunks = (int)nch; r->r = l; r->c = k;
  set_planes(r->out, p); r->ldo = ldp;
  r->gx = (int)(((int64_t)l * k + 255) / 256); r->gy = 1;
  return true;
}

// ---------------------------------------------------------------------------
hipError_t launch_apply(hipStream_t st, int tz, const void *const z[4], int64_t ldz, int64_t rows,
                        int k, const double *c_aos, int kc, double *const out[4], int64_t ldo,
                        int c_upper, const SmallStatus *gate) {
  // Out(i, j) = sum_t Z(i, t) C(t, j), C AoS with leading dimension k
  const void *cp[4] = {c_aos, c_aos + 1, c_aos + 2, c_aos + 3};
  Gemm64Args g = g64_args(z, 1, ldz, cp, 4, 4 * (int64_t)k, rows, kc, k);
  g.b_upper = c_upper;
  g.gate = gate;
  for (int p = 0; p < 4; ++p) g.out[p] = out[p];
  g.ldo = ldo;
  // the wide kernel: Z read once per four column tiles
  const dim3 grid((unsigned)((g.mt + 3) / 4), (unsigned)((g.nt + 3) / 4));
  if (tz == 0) hipLaunchKernelGGL(qgemm64w_k<double>, grid, dim3(256), 0, st, g);
  else if (tz == 1) hipLaunchKernelGGL(qgemm64w_k<float>, grid, dim3(256), 0, st, g);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// P = Psi H, Psi (l x m) regenerated as the sketch of `mode` used it.  A
// block owns 16 rows of Psi and every column of H (up to 16 tiles of 16), so
// each entry of Psi is regenerated once per chunk of rows of H.
__global__ __launch_bounds__(256) void psi_apply_k(PsiApplyArgs args, GroupRef grp) {
  PsiApplyArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  const int mode = A.mode, rad = A.rad, l = A.l, k = A.k;
  const uint32_t k0 = A.k0, k1 = A.k1;
  const int64_t m = A.m, ldh = A.ldh, chunk = A.chunk;
  const PlanesC<double> h = mkc_d<double>(A.h);
  double *partial = A.partial;
  __shared__ qd sp[16][33];
  __shared__ qd sh[32][17];
  const int tid = threadIdx.x;
  const int rr = tid & 15, bb = tid >> 4;
  const int r0 = bx * 16;
  const int nbt = (k + 15) / 16;
  const int64_t is = (int64_t)by * chunk;
  const int64_t ie = min(m, is + chunk);
  qd acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = qzero();
  for (int64_t i0 = is; i0 < ie; i0 += 32) {
    for (int e = tid; e < 512; e += 256) {
      const int ii = e & 31, q = e >> 5;
      const int64_t gi = i0 + ii;
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      if (gi < ie && r0 + q < l) {
        if (A.psi_st_type == 1) {          // bf16 staging of the sketch (step tiles)
          const QSK_GLOBAL uint16_t *ps = gp((const uint16_t *)A.psi_st) + psi_tiled_index<2>(r0 + q, gi, A.psi_ps / A.psi_ld / 16);
#pragma unroll
          for (int p = 0; p < 4; ++p) v[p] = (double)__uint_as_float(((uint32_t)ps[p * A.psi_ps]) << 16);
        } else if (A.psi_st_type == 2) {   // fp32 staging
          const QSK_GLOBAL float *ps = gp((const float *)A.psi_st) + psi_tiled_index<4>(r0 + q, gi, A.psi_ps / A.psi_ld / 16);
#pragma unroll
          for (int p = 0; p < 4; ++p) v[p] = (double)ps[p * A.psi_ps];
        } else {
          embed_entry_as_used(mode, rad, (uint32_t)gi, (uint32_t)(r0 + q), STREAM_PSI, k0, k1, v);
        }
      }
      sp[q][ii] = {v[0], v[1], v[2], v[3]};
    }
#pragma unroll
    for (int bt = 0; bt < 16; ++bt) {
      if (bt < nbt) {
        __syncthreads();
        for (int e = tid; e < 512; e += 256) {
          const int ii = e & 31, q = e >> 5;
          const int64_t gi = i0 + ii;
          const int b = bt * 16 + q;
          sh[ii][q] = (gi < ie && b < k) ? load_q(h, gi + (int64_t)b * ldh) : qzero();
        }
        __syncthreads();
#pragma unroll 8
        for (int ii = 0; ii < 32; ++ii) qfma(acc[bt], sp[rr][ii], sh[ii][bb]);
      }
    }
    __syncthreads();
  }
  const int gr = r0 + rr;
  if (gr < l) {
#pragma unroll
    for (int bt = 0; bt < 16; ++bt) {
      const int gb = bt * 16 + bb;
      if (bt < nbt && gb < k) {
        QSK_GLOBAL double *q = gpw(partial) + 4 * (((int64_t)by * k + gb) * l + gr);
        q[0] = acc[bt].w; q[1] = acc[bt].x; q[2] = acc[bt].y; q[3] = acc[bt].z;
      }
    }
  }
}

bool plan_psi_apply(int l, int64_t m, int k, int64_t partial_elems, int64_t *chunk, int64_t *nch) {
  if (k > 256) return false;
  const int tiles = (l + 15) / 16;
  const int64_t per = (int64_t)l * k * 4;
  const int64_t max_chunks = partial_elems / per;
  if (max_chunks < 1) return false;
  *chunk = chunk_rows(m, tiles, max_chunks);
  *nch = (m + *chunk - 1) / *chunk;
  return *nch <= max_chunks;
}

hipError_t launch_psi_apply_k(hipStream_t st, const PsiApplyArgs &a, GroupRef g, int64_t blocks) {
  dim3 grid = g.tab ? dim3((unsigned)blocks) : dim3(a.gx, a.gy);
  hipLaunchKernelGGL(psi_apply_k, grid, dim3(256), 0, st, a, g);
  return hipGetLastError();
}

hipError_t launch_psi_apply(hipStream_t st, int mode, int rad, uint32_t k0, uint32_t k1, int l,
                            int64_t m, const double *const h[4], int64_t ldh, int k,
                            double *partials, int64_t partial_elems, double *const p[4],
                            int64_t ldp, const void *psi_st, int psi_st_type, int64_t psi_ld,
                            int64_t psi_ps) {
  int64_t chunk, nch;
  if (psi_st && (psi_st_type == 1 || psi_st_type == 2)) {
    // staged Psi: P(i, j) = sum_t Psi(i, t) H(t, j) on the FP64 matrix cores
    const int64_t max_chunks = partial_elems / ((int64_t)l * k * 4);
    if (max_chunks < 1) return hipErrorInvalidValue;
    const size_t es = psi_st_type == 1 ? 2 : 4;
    const void *pp[4];
    for (int q = 0; q < 4; ++q) pp[q] = (const char *)psi_st + (size_t)q * psi_ps * es;
    const void *hh[4] = {h[0], h[1], h[2], h[3]};
    Gemm64Args g = g64_args(pp, psi_ld, 1, hh, 1, ldh, l, k, m);
    g.a_tiled = 1;                       // the step-tile layout of the staging
    g.a_lp16 = psi_ps / psi_ld / 16;
    g.kchunk = g64_chunk(m, (int64_t)g.mt * g.nt, max_chunks, &nch);
    g.gy = (int)nch;
    g.partial = partials;
    hipError_t e = launch_qgemm64_k(st, psi_st_type == 1 ? 2 : 1, 0, false, g, GroupRef{}, 0);
    if (e != hipSuccess) return e;
    ReducePlanarArgs r{};
    r.partial = partials; r.nchunks = (int)nch; r.r = l; r.c = k;
    set_planes(r.out, p); r.ldo = ldp;
    r.gx = (int)(((int64_t)l * k + 255) / 256); r.gy = 1;
    return launch_reduce_planar_k(st, r, GroupRef{}, r.gx);
  }
  if (!plan_psi_apply(l, m, k, partial_elems, &chunk, &nch)) return hipErrorInvalidValue;
  PsiApplyArgs a{};
  a.mode = mode; a.rad = rad; a.k0 = k0; a.k1 = k1; a.l = l; a.m = m;
  set_planes(a.h, h);
  a.ldh = ldh; a.k = k; a.chunk = chunk; a.partial = partials;
  a.psi_st = psi_st; a.psi_st_type = psi_st_type; a.psi_ld = psi_ld; a.psi_ps = psi_ps;
  a.gx = (l + 15) / 16; a.gy = (int)nch;
  hipError_t e = launch_psi_apply_k(st, a, GroupRef{}, 0);
  if (e != hipSuccess) return e;
  ReducePlanarArgs r{};
  r.partial = partials; r.nchunks = (int)nch; r.r = l; r.c = k;
  set_planes(r.out, p); r.ldo = ldp;
  r.gx = (int)(((int64_t)l * k + 255) / 256); r.gy = 1;
  return launch_reduce_planar_k(st, r, GroupRef{}, r.gx);
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void widen_k(const T *src, int64_t lds, int64_t pss, int64_t rows, int64_t cols,
                        Planes<double> dst, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e % rows, j = e / rows;
  for (int p = 0; p < 4; ++p) dst.p[p][i + j * ldd] = (double)src[p * pss + i + j * lds];
}

hipError_t launch_widen(hipStream_t st, int tsrc, const void *src, int64_t lds, int64_t pss,
                        int64_t rows, int64_t cols, double *const dst[4], int64_t ldd) {
  Planes<double> d;
  for (int p = 0; p < 4; ++p) d.p[p] = dst[p];
  const int64_t n = rows * cols;
  if (tsrc == 0)
    hipLaunchKernelGGL((widen_k<double>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (const double *)src, lds, pss, rows, cols, d, ldd);
  else
    hipLaunchKernelGGL((widen_k<float>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (const float *)src, lds, pss, rows, cols, d, ldd);
  return hipGetLastError();
}

template <typename T>
__global__ void scale_k(T *p, int64_t n, T theta) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = theta == T(0) ? T(0) : p[e] * theta;
}

hipError_t launch_scale(hipStream_t st, int tsrc, void *p, int64_t n, double theta) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 16384);
  if (tsrc == 0)
    hipLaunchKernelGGL((scale_k<double>), dim3((unsigned)blocks), dim3(256), 0, st, (double *)p, n, theta);
  else
    hipLaunchKernelGGL((scale_k<float>), dim3((unsigned)blocks), dim3(256), 0, st, (float *)p, n, (float)theta);
  return hipGetLastError();
}

template <typename T>
__global__ void narrow_k(PlanesC<double> src, int64_t lds, T *dst, int64_t ldd, int64_t pss, int64_t rows,
                         int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % rows, j = e / rows;
    for (int p = 0; p < 4; ++p) dst[p * pss + i + j * ldd] = (T)src.p[p][i + j * lds];
  }
}

hipError_t launch_narrow(hipStream_t st, int tdst, const double *const src[4], int64_t lds,
                         void *dst, int64_t ldd, int64_t pss, int64_t rows, int64_t cols) {
  PlanesC<double> s;
  for (int p = 0; p < 4; ++p) s.p[p] = src[p];
  const int64_t blocks = std::min<int64_t>((rows * cols + 255) / 256, 16384);
  if (blocks <= 0) return hipSuccess;
  if (tdst == 0)
    hipLaunchKernelGGL((narrow_k<double>), dim3((unsigned)blocks), dim3(256), 0, st, s, lds, (double *)dst, ldd,
                       pss, rows, cols);
  else
    hipLaunchKernelGGL((narrow_k<float>), dim3((unsigned)blocks), dim3(256), 0, st, s, lds, (float *)dst, ldd,
                       pss, rows, cols);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Error pass: 64 x 64 tiles of H X, accumulated against A in FP64.
template <typename T> __device__ __forceinline__ double lda_val(const T *p, int64_t i);
template <> __device__ __forceinline__ double lda_val<double>(const double *p, int64_t i) { return gp(p)[i]; }
template <> __device__ __forceinline__ double lda_val<float>(const float *p, int64_t i) { return gp(p)[i]; }
template <> __device__ __forceinline__ double lda_val<uint16_t>(const uint16_t *p, int64_t i) {
  return (double)__uint_as_float(((uint32_t)gp(p)[i]) << 16);
}

template <typename TIN>
__global__ __launch_bounds__(256) void error_k(ErrorArgs args, GroupRef grp) {
  ErrorArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  const PlanesC<TIN> a = mkc_d<TIN>(A.a);
  const PlanesC<double> q = mkc_d<double>(A.q), x = mkc_d<double>(A.x);
  const int64_t lda = A.lda, m = A.m, n = A.n, ldq = A.ldq, ldx = A.ldx;
  const int pure = A.pure, k = A.k;
  double *acc = A.acc;
  __shared__ qd sq[64][9];
  __shared__ qd sx[8][65];
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;      // 4 x 4 outputs per thread
  const int64_t i0 = (int64_t)bx * 64, j0 = (int64_t)by * 64;
  qd c[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) c[u][v] = qzero();
  for (int b0 = 0; b0 < k; b0 += 8) {
    for (int e = tid; e < 512; e += 256) {
      const int ii = e & 63, bb = e >> 6;
      const int64_t gi = i0 + ii;
      sq[ii][bb] = (gi < m && b0 + bb < k) ? load_q(q, gi + (int64_t)(b0 + bb) * ldq) : qzero();
      const int jj = e & 63, b2 = e >> 6;
      const int64_t gj = j0 + jj;
      sx[b2][jj] = (gj < n && b0 + b2 < k) ? load_q(x, (b0 + b2) + gj * ldx) : qzero();
    }
    __syncthreads();
#pragma unroll
    for (int bb = 0; bb < 8; ++bb) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const qd qv = sq[tr + 16 * u][bb];
#pragma unroll
        for (int v = 0; v < 4; ++v) qfma(c[u][v], qv, sx[bb][tc + 16 * v]);
      }
    }
    __syncthreads();
  }
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t gi = i0 + tr + 16 * u, gj = j0 + tc + 16 * v;
      if (gi < m && gj < n) {
        const int64_t idx = gi + gj * lda;
        const double aw = pure ? 0.0 : lda_val<TIN>(a.p[0], idx);
        const double ax = lda_val<TIN>(a.p[1], idx), ay = lda_val<TIN>(a.p[2], idx),
                     az = lda_val<TIN>(a.p[3], idx);
        const double dw = aw - c[u][v].w, dx = ax - c[u][v].x, dy = ay - c[u][v].y, dz = az - c[u][v].z;
        num += dw * dw + dx * dx + dy * dy + dz * dz;
        den += aw * aw + ax * ax + ay * ay + az * az;
      }
    }
  red[0][tid] = num;
  red[1][tid] = den;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) { red[0][tid] += red[0][tid + s]; red[1][tid] += red[1][tid + s]; }
    __syncthreads();
  }
  if (tid == 0) { atomicAdd(&acc[0], red[0][0]); atomicAdd(&acc[1], red[1][0]); }
}

hipError_t launch_error_k(hipStream_t st, int tin, const ErrorArgs &a, GroupRef g, int64_t blocks) {
  dim3 grid = g.tab ? dim3((unsigned)blocks) : dim3(a.gx, a.gy);
  if (tin == DT_F64) hipLaunchKernelGGL((error_k<double>), grid, dim3(256), 0, st, a, g);
  else if (tin == DT_F32) hipLaunchKernelGGL((error_k<float>), grid, dim3(256), 0, st, a, g);
  else hipLaunchKernelGGL((error_k<uint16_t>), grid, dim3(256), 0, st, a, g);
  return hipGetLastError();
}

hipError_t launch_error(hipStream_t st, int tin, const void *const a[4], int64_t lda, int pure,
                        int64_t m, int64_t n, const double *const q[4], int64_t ldq,
                        const double *const x[4], int64_t ldx, int k, double *acc) {
  ErrorArgs e{};
  e.a[0] = a[0] ? a[0] : a[1];
  for (int p = 1; p < 4; ++p) e.a[p] = a[p];
  e.lda = lda; e.pure = pure; e.m = m; e.n = n;
  set_planes(e.q, q); e.ldq = ldq;
  set_planes(e.x, x); e.ldx = ldx;
  e.k = k; e.acc = acc;
  e.gx = (int)((m + 63) / 64); e.gy = (int)((n + 63) / 64);
  return launch_error_k(st, tin, e, GroupRef{}, 0);
}

// ===========================================================================
// Single-workgroup small dense algebra on k x k AoS quaternion matrices in
// global memory (one CU; all waves of the block share its L1, so a
// __syncthreads() makes a block's global writes visible to the block).

__device__ __forceinline__ qd gq(const double *a, int i, int j, int ld) {
  const QSK_GLOBAL double *p = gp(a) + 4 * ((int64_t)i + (int64_t)j * ld);
  return {p[0], p[1], p[2], p[3]};
}
__device__ __forceinline__ void sq_(double *a, int i, int j, int ld, qd v) {
  QSK_GLOBAL double *p = gpw(a) + 4 * ((int64_t)i + (int64_t)j * ld);
  p[0] = v.w; p[1] = v.x; p[2] = v.y; p[3] = v.z;
}

__device__ void sm_identity(double *c, int k) {
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e % k, j = e / k;
    sq_(c, i, j, k, {i == j ? 1.0 : 0.0, 0.0, 0.0, 0.0});
  }
  __syncthreads();
}

__device__ void sm_copy(double *dst, const double *src, int n_doubles) {
  for (int e = threadIdx.x; e < n_doubles; e += blockDim.x) dst[e] = src[e];
  __syncthreads();
}

// C = opA(A) opB(B); op 1 = conjugate transpose.  C must not alias A or B.
__device__ void sm_gemm(int k, const double *a, int opa, const double *b, int opb, double *c) {
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e % k, j = e / k;
    qd s = qzero();
    for (int t = 0; t < k; ++t) {
      const qd av = opa ? qconj(gq(a, t, i, k)) : gq(a, i, t, k);
      const qd bv = opb ? qconj(gq(b, j, t, k)) : gq(b, t, j, k);
      qfma(s, av, bv);
    }
    sq_(c, i, j, k, s);
  }
  __syncthreads();
}

// Upper Cholesky G' = R^* R (right-looking, blocked by CB pivot rows held in
// LDS); returns in shared `fail` whether a pivot fell below tol * max
// diagonal.  k <= 256.  The trailing matrix is updated in r (global memory)
// until its upper triangle fits in the LDS pool beside the panel buffers;
// from then on it lives there, packed by columns (column c of the block
// holds rows 0 .. c), and only the finished rows are written to r.
constexpr int CHOL_POOL = 4992;       // quaternions of LDS (156 KB)
__device__ __forceinline__ int chol_pk(int a, int c) { return ((c * (c + 1)) >> 1) + a; }

// Trailing update of sm_chol after a panel of jb pivot rows (rows j0 ..,
// finished and scaled in `done`, row stride w): G'[a, c] -= sum over the
// panel rows of conj(done[rr][a]) done[rr][c] for b0 <= a <= c < b0 + nr, in
// the packed LDS block T (INLDS) or in r.  Thread t takes the entries t,
// t + nt, t + 2 nt, ... (column by column), CH at a time: their loads are
// issued together, then the updates and the stores, so that a load never
// waits for the store of the previous entry (each entry's arithmetic is the
// same as one at a time).
template <bool INLDS, int CH>
__device__ __forceinline__ void chol_trailing(qd *T, int o, double *r, int k, const qd *done, int w, int j0,
                                              int jb, int b0, int nr) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int tot = (nr * (nr + 1)) >> 1;
  for (int e0 = tid; e0 < tot; e0 += CH * nt) {
    int ga_[CH], gc_[CH];
    qd v[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int e = e0 + u * nt;
      int ga = b0, gc = b0;
      if (e < tot) {
        int cc = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (cc > 0 && ((cc * (cc + 1)) >> 1) > e) --cc;
        while ((((cc + 1) * (cc + 2)) >> 1) <= e) ++cc;
        ga = b0 + e - ((cc * (cc + 1)) >> 1);
        gc = b0 + cc;
      }
      ga_[u] = ga;
      gc_[u] = gc;
      if (e < tot) v[u] = INLDS ? T[chol_pk(ga - o, gc - o)] : gq(r, ga, gc, k);
      else v[u] = qzero();
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (e0 + u * nt >= tot) break;
      qd x = v[u];
      for (int rr = 0; rr < jb; ++rr)
        x = qsub(x, qmul(qconj(done[rr * w + ga_[u] - j0]), done[rr * w + gc_[u] - j0]));
      if (INLDS) T[chol_pk(ga_[u] - o, gc_[u] - o)] = x;
      else sq_(r, ga_[u], gc_[u], k, x);
    }
  }
}
// The same update dealt out in 2 x 2 blocks of entries (rows a0, a0 + 1,
// columns c0, c0 + 1 of the trailing triangle, block (A, C) with A <= C
// packed by columns): the four panel values of a block's rows and columns
// are loaded once per panel row for up to four entries, half the LDS reads
// per entry of one entry at a time.  Each entry's arithmetic is the same as
// one at a time.
template <bool INLDS>
__device__ __forceinline__ void chol_trailing2(qd *T, int o, double *r, int k, const qd *done, int w, int j0,
                                               int jb, int b0, int nr) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nb = (nr + 1) >> 1;
  const int tot = (nb * (nb + 1)) >> 1;
  const int end = b0 + nr;
  for (int e = tid; e < tot; e += nt) {
    int cc = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (cc > 0 && ((cc * (cc + 1)) >> 1) > e) --cc;
    while ((((cc + 1) * (cc + 2)) >> 1) <= e) ++cc;
    const int ab = e - ((cc * (cc + 1)) >> 1);
    const int a0 = b0 + 2 * ab, c0 = b0 + 2 * cc, a1 = a0 + 1, c1 = c0 + 1;
    // entries of the block inside the upper triangle and the trailing block
    const bool v01 = c1 < end, v10 = ab < cc && a1 < end, v11 = a1 < end && c1 < end;
    qd x00 = INLDS ? T[chol_pk(a0 - o, c0 - o)] : gq(r, a0, c0, k);
    qd x01 = v01 ? (INLDS ? T[chol_pk(a0 - o, c1 - o)] : gq(r, a0, c1, k)) : qzero();
    qd x10 = v10 ? (INLDS ? T[chol_pk(a1 - o, c0 - o)] : gq(r, a1, c0, k)) : qzero();
    qd x11 = v11 ? (INLDS ? T[chol_pk(a1 - o, c1 - o)] : gq(r, a1, c1, k)) : qzero();
    const int ia0 = a0 - j0, ic0 = c0 - j0;
    const int ia1 = a1 < end ? ia0 + 1 : ia0, ic1 = c1 < end ? ic0 + 1 : ic0;
    for (int rr = 0; rr < jb; ++rr) {
      const qd *dr = done + rr * w;
      const qd da0 = qconj(dr[ia0]), da1 = qconj(dr[ia1]), dc0 = dr[ic0], dc1 = dr[ic1];
      x00 = qsub(x00, qmul(da0, dc0));
      x01 = qsub(x01, qmul(da0, dc1));
      x10 = qsub(x10, qmul(da1, dc0));
      x11 = qsub(x11, qmul(da1, dc1));
    }
    if (INLDS) {
      T[chol_pk(a0 - o, c0 - o)] = x00;
      if (v01) T[chol_pk(a0 - o, c1 - o)] = x01;
      if (v10) T[chol_pk(a1 - o, c0 - o)] = x10;
      if (v11) T[chol_pk(a1 - o, c1 - o)] = x11;
    } else {
      sq_(r, a0, c0, k, x00);
      if (v01) sq_(r, a0, c1, k, x01);
      if (v10) sq_(r, a1, c0, k, x10);
      if (v11) sq_(r, a1, c1, k, x11);
    }
  }
}
__device__ void sm_chol(const double *g, double *r, int k, int complex_only, double shift,
                        double tol, int *fail, double *minp, double *trace) {
  // Panels of CB pivot rows live in LDS twice: `panel` holds the rows as
  // updated so far (read by the elimination), `done` the finished, scaled
  // rows (read by the trailing update), so each pivot costs one barrier.
  // Both are CB x w (row stride w = k - j0) at the front of the pool.
  constexpr int CB = 8;
  __shared__ qd pool[CHOL_POOL];
  __shared__ double s_maxd;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < k * k; e += nt) {
    const int i = e % k, j = e / k;
    qd v = qzero();
    if (i <= j) {
      v = gq(g, i, j, k);
      if (complex_only) { v.y = 0.0; v.z = 0.0; }
      if (i == j) { v.x = 0.0; v.y = 0.0; v.z = 0.0; v.w += shift; }
    }
    sq_(r, i, j, k, v);
  }
  // the diagonal goes to LDS in parallel; one thread then takes its maximum
  // and its sum in index order
  double *diag = (double *)pool;
  for (int i = tid; i < k; i += nt) diag[i] = gq(g, i, i, k).w + shift;
  __syncthreads();
  if (tid == 0) {
    double md = 0.0, tr = 0.0;
    for (int i = 0; i < k; ++i) { const double d = diag[i]; md = fmax(md, d); tr += d; }
    s_maxd = md;
    *trace = tr;
    *fail = 0;
    *minp = 1.0;
  }
  __syncthreads();
  qd *T = nullptr;                    // LDS trailing block, rows and columns o ..
  int o = 0;
#define QSK_CHOL_GET(A_, C_) (T ? T[chol_pk((A_) - o, (C_) - o)] : gq(r, (A_), (C_), k))
  for (int j0 = 0; j0 < k; j0 += CB) {
    const int jb = min(CB, k - j0), w = k - j0;
    qd *panel = pool, *done = pool + CB * w;
    if (!T && 2 * CB * w + ((w * (w + 1)) >> 1) <= CHOL_POOL) {
      // move the upper triangle of rows and columns j0 .. k-1 into LDS
      T = pool + 2 * CB * w;
      o = j0;
      for (int e = tid; e < ((w * (w + 1)) >> 1); e += nt) {
        int c = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (c > 0 && ((c * (c + 1)) >> 1) > e) --c;
        while ((((c + 1) * (c + 2)) >> 1) <= e) ++c;
        const int a = e - ((c * (c + 1)) >> 1);
        T[e] = gq(r, o + a, o + c, k);
      }
      __syncthreads();
    }
    for (int e = tid; e < jb * w; e += nt) {
      const int rr = e / w, cc = e % w;
      panel[rr * w + cc] = cc >= rr ? QSK_CHOL_GET(j0 + rr, j0 + cc) : qzero();
    }
    __syncthreads();
    for (int rr = 0; rr < jb; ++rr) {
      // every thread reads the pivot; a pivot below tol * max diagonal marks
      // failure (the factor is then discarded by the caller)
      const double d = panel[rr * w + rr].w;
      const double rel = s_maxd > 0.0 ? d / s_maxd : 0.0;
      if (tid == 0) {
        if (rel < *minp) *minp = rel;
        if (!(rel > tol)) *fail = 1;
      }
      const double sd = sqrt(fmax(d, 0.0));
      const double inv_d = d > 0.0 ? 1.0 / d : 0.0, inv_s = sd > 0.0 ? 1.0 / sd : 0.0;
      const int rows = jb - rr - 1;
      for (int e = tid; e < rows * w; e += nt) {
        const int r2 = rr + 1 + e / w, cc = e % w;
        if (cc >= r2)
          panel[r2 * w + cc] = qsub(panel[r2 * w + cc],
                                    qscale(qmul(qconj(panel[rr * w + r2]), panel[rr * w + cc]), inv_d));
      }
      for (int cc = tid; cc < w; cc += nt)
        done[rr * w + cc] = cc < rr ? qzero() : (cc == rr ? qd{sd, 0.0, 0.0, 0.0} : qscale(panel[rr * w + cc], inv_s));
      __syncthreads();
    }
    if (*fail) return;
    for (int e = tid; e < jb * w; e += nt) {
      const int rr = e / w, cc = e % w;
      if (cc >= rr) sq_(r, j0 + rr, j0 + cc, k, done[rr * w + cc]);
    }
    // trailing update of the upper triangle, its entries dealt to the
    // threads in turn (packed by columns)
    const int nr = k - j0 - jb, b0 = j0 + jb;
    // (in LDS one entry at a time; in global memory 2 x 2 blocks, whose
    // halved panel reads shorten the memory-bound update)
    if (T) chol_trailing<true, 4>(T, o, r, k, done, w, j0, jb, b0, nr);
    else chol_trailing2<false>(T, o, r, k, done, w, j0, jb, b0, nr);
    __syncthreads();
  }
#undef QSK_CHOL_GET
}

// T = R^{-1} for upper triangular R with real positive diagonal (single
// workgroup version, used inside drivers).
__device__ void sm_triinv(const double *r, double *t, int k) {
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    for (int a = k - 1; a > c; --a) sq_(t, a, c, k, qzero());
    sq_(t, c, c, k, {1.0 / r[4 * (c + (int64_t)c * k)], 0.0, 0.0, 0.0});
    for (int a = c - 1; a >= 0; --a) {
      qd s = qzero();
      for (int b = a + 1; b <= c; ++b) qfma(s, gq(r, a, b, k), gq(t, b, c, k));
      sq_(t, a, c, k, qscale(s, -1.0 / r[4 * (a + (int64_t)a * k)]));
    }
  }
  __syncthreads();
}

// Wave-level sum of a double across 64 lanes.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One-sided (Hestenes) Jacobi on the columns of a rows x cols quaternion
// matrix: quaternion inner products are made real by a unit-quaternion
// column scaling, then a real plane rotation orthogonalises the pair.
// Round-robin pair order; stops after a sweep without rotations.
__device__ void sm_jacobi(double *a, int rows, int cols, int lda, int max_sweeps, double tol,
                          int rows_rot = -1) {
  if (rows_rot < 0) rows_rot = rows;
  __shared__ int s_rot;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int n = cols + (cols & 1);
  if (n < 2) return;
  // below ~rows * u the inner products are rounding noise: rotating on them
  // never terminates
  tol = fmax(tol, 4.0 * rows * 0x1p-53);
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) s_rot = 0;
    __syncthreads();
    for (int round = 0; round < n - 1; ++round) {
      for (int pi = wave; pi < n / 2; pi += nw) {
        int p, q;
        if (pi == 0) { p = n - 1; q = round; }
        else { p = (round + pi) % (n - 1); q = (round - pi + (n - 1)) % (n - 1); }
        if (p >= cols || q >= cols) continue;
        double al = 0.0, be = 0.0;
        qd ga = qzero();
        for (int i = lane; i < rows; i += 64) {
          const qd ap = gq(a, i, p, lda), aq = gq(a, i, q, lda);
          al += qnorm2(ap);
          be += qnorm2(aq);
          qfma_cj(ga, ap, aq);
        }
        al = wave_sum(al); be = wave_sum(be);
        ga.w = wave_sum(ga.w); ga.x = wave_sum(ga.x); ga.y = wave_sum(ga.y); ga.z = wave_sum(ga.z);
        const double gn = sqrt(qnorm2(ga));
        if (!(gn > tol * sqrt(al * be)) || al == 0.0 || be == 0.0) continue;
        const qd mu_c = qscale(qconj(ga), 1.0 / gn);           // conj(mu), mu = gamma / |gamma|
        const double zeta = (be - al) / (2.0 * gn);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int i = lane; i < rows_rot; i += 64) {
          const qd ap = gq(a, i, p, lda);
          const qd aq = qmul(gq(a, i, q, lda), mu_c);
          sq_(a, i, p, lda, qsub(qscale(ap, c), qscale(aq, s)));
          sq_(a, i, q, lda, qadd(qscale(ap, s), qscale(aq, c)));
        }
        if (lane == 0) atomicAdd(&s_rot, 1);
      }
      __syncthreads();
    }
    const int rot = s_rot;
    __syncthreads();
    if (rot == 0) break;
  }
}

// Column norms, descending order, normalised columns into u (rows x cols).
__device__ void sm_sorted_columns(const double *a, int rows, int cols, int lda, double *sig,
                                  int *order, double *u, int ldu) {
  for (int j = threadIdx.x; j < cols; j += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < rows; ++i) s += qnorm2(gq(a, i, j, lda));
    sig[j] = sqrt(s);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 0; j < cols; ++j) order[j] = j;
    for (int j = 1; j < cols; ++j) {            // insertion sort, descending
      const int key = order[j];
      int x = j - 1;
      while (x >= 0 && sig[order[x]] < sig[key]) { order[x + 1] = order[x]; --x; }
      order[x + 1] = key;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rows * cols; e += blockDim.x) {
    const int i = e % rows, j = e / rows;
    const int src = order[j];
    const double s = sig[src];
    sq_(u, i, j, ldu, s > 0.0 ? qscale(gq(a, i, src, lda), 1.0 / s) : qzero());
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void chol_kernel(CholArgs args, GroupRef grp) {
  CholArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  if (gate_skip(A.gate)) return;
  const double *g = A.g;
  const int k = A.k, complex_only = A.complex_only;
  const double shift = A.shift, tol = A.tol;
  double *r = A.r;
  SmallStatus *status = A.status;
  if (A.only_failed && !status->fail) return;
  __shared__ int fail;
  __shared__ double minp, trace;
  sm_chol(g, r, k, complex_only, shift, tol, &fail, &minp, &trace);
  __syncthreads();
  if (threadIdx.x == 0) {
    status->fail = fail;
    if (fail) status->fail_any = 1;
    status->min_pivot2 = minp;
    status->trace = trace;
  }
}

// T = R^{-1}, one workgroup per column c, by a column sweep of R T = I:
// for b = c, c-1, ..., 0: T[b, c] = (delta_bc - s_b) / R[b, b], then
// s_a += R[a, b] T[b, c] for a < b (no reductions, one barrier per b).
// Skipped when the Cholesky failed.
__global__ __launch_bounds__(256) void triinv_kernel(CholArgs args, GroupRef grp) {
  CholArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  if (gate_skip(A.gate)) return;
  const double *r = A.r;
  double *t = A.t;
  const int k = A.k;
  const SmallStatus *status = A.status;
  __shared__ qd acc[256];
  __shared__ qd col[256];
  if (status && status->fail) return;
  if (bx >= k) return;
  const int c = bx, tid = threadIdx.x;
  // k <= 256: thread a owns row a.  The pivots' reciprocals are read once,
  // and column b - 1 of R is loaded while step b runs.
  __shared__ double dinv[256];
  for (int a = tid; a < k; a += 256) {
    acc[a] = qzero();
    col[a] = qzero();
    if (a <= c) dinv[a] = 1.0 / gp(r)[4 * (a + (int64_t)a * k)];
  }
  __syncthreads();
  qd rcur = tid < c ? gq(r, tid, c, k) : qzero();
  for (int b = c; b >= 0; --b) {
    const qd rnext = tid + 1 < b ? gq(r, tid, b - 1, k) : qzero();
    qd tb = qsub(b == c ? qd{1.0, 0.0, 0.0, 0.0} : qzero(), acc[b]);
    tb = qscale(tb, dinv[b]);
    if (tid == 0) col[b] = tb;
    if (tid < b) qfma(acc[tid], rcur, tb);
    rcur = rnext;
    __syncthreads();
  }
  for (int a = tid; a < k; a += 256) sq_(t, a, c, k, col[a]);
}

__global__ void status_reset_kernel(SmallStatus *s, int keep_fail_any) {
  if (threadIdx.x == 0) {
    const int fa = keep_fail_any ? s->fail_any : 0;
    *s = SmallStatus{};
    s->fail_any = fa;
  }
}
hipError_t launch_status_reset(hipStream_t st, SmallStatus *s, int keep_fail_any) {
  hipLaunchKernelGGL(status_reset_kernel, dim3(1), dim3(64), 0, st, s, keep_fail_any);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void status_reset_n_kernel(SmallStatus *s, int count, int keep_fail_any) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    const int fa = keep_fail_any ? s[i].fail_any : 0;
    s[i] = SmallStatus{};
    s[i].fail_any = fa;
  }
}
hipError_t launch_status_reset_n(hipStream_t st, SmallStatus *s, int count, int keep_fail_any) {
  hipLaunchKernelGGL(status_reset_n_kernel, dim3(1), dim3(256), 0, st, s, count, keep_fail_any);
  return hipGetLastError();
}

// Zeroing by a kernel instead of a memset command, so that a captured graph
// holds kernel nodes only.
__global__ __launch_bounds__(256) void zero_kernel(ZeroArgs args, GroupRef grp) {
  ZeroArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  uint4 *p = (uint4 *)A.p;
  const int64_t base = (int64_t)bx * ZERO_UNITS_PER_BLOCK;
  for (int j = threadIdx.x; j < ZERO_UNITS_PER_BLOCK; j += 256)
    if (base + j < A.n16) p[base + j] = make_uint4(0u, 0u, 0u, 0u);
}
hipError_t launch_zero_k(hipStream_t st, const ZeroArgs &a, GroupRef g, int64_t blocks) {
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)(g.tab ? blocks : a.gx)), dim3(256), 0, st, a, g);
  return hipGetLastError();
}

hipError_t launch_chol_k(hipStream_t st, const CholArgs &a, GroupRef g, int count) {
  hipLaunchKernelGGL(chol_kernel, dim3(g.tab ? count : 1), dim3(1024), 0, st, a, g);
  return hipGetLastError();
}
hipError_t launch_triinv_k(hipStream_t st, const CholArgs &a, GroupRef g, int64_t blocks) {
  hipLaunchKernelGGL(triinv_kernel, dim3((unsigned)(g.tab ? blocks : a.k)), dim3(256), 0, st, a, g);
  return hipGetLastError();
}


hipError_t launch_chol_inv(hipStream_t st, const double *g, int k, int complex_only, double shift,
                           double tol, double *r, double *t, SmallStatus *status, const SmallStatus *gate) {
  CholArgs a{};
  a.g = g; a.k = k; a.complex_only = complex_only; a.shift = shift; a.tol = tol;
  a.r = r; a.t = t; a.status = status; a.only_failed = 0; a.gate = gate;
  a.gx = k; a.gy = 1;
  hipError_t e = launch_chol_k(st, a, GroupRef{}, 1);
  if (e != hipSuccess) return e;
  return launch_triinv_k(st, a, GroupRef{}, 0);
}

// C = opA(A) opB(B) for k x k AoS matrices: 16 x 16 output tiles per block,
// 16-wide slabs of A and B staged in LDS.
__global__ __launch_bounds__(256) void qgemm_small_kernel(GemmArgs args, GroupRef grp) {
  GemmArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  if (gate_skip(A.gate)) return;
  const int k = A.k, opa = A.opa, opb = A.opb;
  const double *a = A.a, *b = A.b;
  double *c = A.c;
  __shared__ qd sa[16][17];
  __shared__ qd sb[16][17];
  const int tid = threadIdx.x, ti = tid & 15, tj = tid >> 4;
  const int i0 = bx * 16, j0 = by * 16;
  if (i0 >= k || j0 >= k) return;
  qd acc = qzero();
  // the operands of the next 16-wide step are loaded while this one is
  // multiplied
  auto load_a = [&](int t0) {
    const int gi = i0 + ti, gt = t0 + tj;
    return (gi < k && gt < k) ? (opa ? qconj(gq(a, gt, gi, k)) : gq(a, gi, gt, k)) : qzero();
  };
  auto load_b = [&](int t0) {
    const int gt2 = t0 + ti, gj = j0 + tj;
    return (gt2 < k && gj < k) ? (opb ? qconj(gq(b, gj, gt2, k)) : gq(b, gt2, gj, k)) : qzero();
  };
  qd va = load_a(0), vb = load_b(0);
  for (int t0 = 0; t0 < k; t0 += 16) {
    sa[ti][tj] = va;
    sb[ti][tj] = vb;
    __syncthreads();
    if (t0 + 16 < k) { va = load_a(t0 + 16); vb = load_b(t0 + 16); }
#pragma unroll
    for (int tt = 0; tt < 16; ++tt) qfma(acc, sa[ti][tt], sb[tt][tj]);
    __syncthreads();
  }
  if (i0 + ti < k && j0 + tj < k) sq_(c, i0 + ti, j0 + tj, k, acc);
}

hipError_t launch_gemm_k(hipStream_t st, const GemmArgs &a, GroupRef g, int64_t blocks) {
  dim3 grid = g.tab ? dim3((unsigned)blocks) : dim3(a.gx, a.gy);
  hipLaunchKernelGGL(qgemm_small_kernel, grid, dim3(256), 0, st, a, g);
  return hipGetLastError();
}

hipError_t launch_small_gemm(hipStream_t st, int k, const double *a, int opa, const double *b,
                             int opb, double *c, const SmallStatus *gate) {
  GemmArgs x{};
  x.k = k; x.a = a; x.opa = opa; x.b = b; x.opb = opb; x.c = c; x.gate = gate;
  x.gx = (k + 15) / 16; x.gy = (k + 15) / 16;
  return launch_gemm_k(st, x, GroupRef{}, 0);
}

// One correction step's eps and M (eq. CondNumReductionIter in the k x k
// space): n_power normalised power iterates v <- G^{-1} v from the Philox
// stream-2 start vector of step `step`, eps = (v^* G^{-1} v)^{-1/2}, and
// M = (1 - eps) I + eps G^{-1}.
__global__ __launch_bounds__(1024) void power_m_kernel(PowerArgs args, GroupRef grp) {
  PowerArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  const int k = A.k, step = A.step, n_power = A.n_power;
  const double *gi = A.gi;
  const uint32_t k0 = A.k0, k1 = A.k1;
  double *m_out = A.m_out;
  SmallStatus *status = A.status;
  __shared__ double v[4 * 256], w[4 * 256];
  __shared__ qd part[4][256];
  __shared__ double s_red[16];
  __shared__ double s_eps;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // sum of one value per thread over the block
  auto block_sum = [&](double x) -> double {
    x = wave_sum(x);
    if (lane == 0) s_red[wave] = x;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < 16; ++i) t += s_red[i];
    __syncthreads();
    return t;
  };
  for (int i = tid; i < k; i += blockDim.x) {
    double e[4];
    gauss_entry_f64((uint32_t)i, (uint32_t)step, STREAM_POWER, k0, k1, e);
    v[4 * i] = e[0]; v[4 * i + 1] = e[1]; v[4 * i + 2] = e[2]; v[4 * i + 3] = e[3];
  }
  __syncthreads();
  // w = G^{-1} v: row i = tid mod 256, the columns split over 4 parts
  const int row = tid & 255, prt = tid >> 8;
  for (int it = 0; it <= n_power; ++it) {
    double sq = 0.0;
    for (int i = tid; i < 4 * k; i += blockDim.x) sq += v[i] * v[i];
    const double inv_nrm = 1.0 / sqrt(block_sum(sq));
    for (int i = tid; i < 4 * k; i += blockDim.x) v[i] *= inv_nrm;
    __syncthreads();
    if (row < k) {
      qd acc = qzero();
      for (int t2 = prt; t2 < k; t2 += 4)
        qfma(acc, gq(gi, row, t2, k), {v[4 * t2], v[4 * t2 + 1], v[4 * t2 + 2], v[4 * t2 + 3]});
      part[prt][row] = acc;
    }
    __syncthreads();
    for (int i = tid; i < k; i += blockDim.x) {
      qd s2 = part[0][i];
      for (int p = 1; p < 4; ++p) s2 = qadd(s2, part[p][i]);
      w[4 * i] = s2.w; w[4 * i + 1] = s2.x; w[4 * i + 2] = s2.y; w[4 * i + 3] = s2.z;
    }
    __syncthreads();
    if (it == n_power) {
      double rl = 0.0;
      for (int i = tid; i < 4 * k; i += blockDim.x) rl += v[i] * w[i];      // Re(v^* w)
      const double rho = block_sum(rl);
      if (tid == 0) {
        s_eps = 1.0 / sqrt(rho);
        status->eps[status->n_eps] = s_eps;
        status->n_eps += 1;
      }
      __syncthreads();
    } else {
      for (int i = tid; i < 4 * k; i += blockDim.x) v[i] = w[i];
      __syncthreads();
    }
  }
  const double eps = s_eps;
  for (int e = tid; e < k * k; e += blockDim.x) {
    const int i = e % k, j = e / k;
    qd gv = qscale(gq(gi, i, j, k), eps);
    if (i == j) gv.w += 1.0 - eps;
    sq_(m_out, i, j, k, gv);
  }
}

hipError_t launch_power_k(hipStream_t st, const PowerArgs &a, GroupRef g, int count) {
  hipLaunchKernelGGL(power_m_kernel, dim3(g.tab ? count : 1), dim3(1024), 0, st, a, g);
  return hipGetLastError();
}

hipError_t launch_power_m(hipStream_t st, int k, const double *gi, int step, int n_power,
                          uint32_t k0, uint32_t k1, double *m_out, SmallStatus *status) {
  PowerArgs a{};
  a.k = k; a.gi = gi; a.step = step; a.n_power = n_power; a.k0 = k0; a.k1 = k1;
  a.m_out = m_out; a.status = status; a.gx = 1; a.gy = 1;
  return launch_power_k(st, a, GroupRef{}, 1);
}

__global__ __launch_bounds__(1024) void identity_kernel(GemmArgs args, GroupRef grp) {
  GemmArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  sm_identity(A.c, A.k);
}

// C = A (k x k AoS copy)
__global__ __launch_bounds__(1024) void copy_small_kernel(GemmArgs args, GroupRef grp) {
  GemmArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  const int64_t n = 4 * (int64_t)A.k * A.k;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) A.c[e] = A.a[e];
}

hipError_t launch_identity_k(hipStream_t st, const GemmArgs &a, GroupRef g, int count) {
  hipLaunchKernelGGL(identity_kernel, dim3(g.tab ? count : 1), dim3(1024), 0, st, a, g);
  return hipGetLastError();
}
hipError_t launch_copy_small_k(hipStream_t st, const GemmArgs &a, GroupRef g, int count) {
  hipLaunchKernelGGL(copy_small_kernel, dim3(g.tab ? count : 1), dim3(1024), 0, st, a, g);
  return hipGetLastError();
}

// C = T and the core-solve gate: trace(G_P) ||T||_F^2, ||T||_F^2 summed in a
// fixed order (strided per thread, then over the threads in index order).
__global__ __launch_bounds__(1024) void core_gate_kernel(int k, const double *t, double *c, SmallStatus *status) {
  __shared__ double part[1024];
  const int64_t n = 4 * (int64_t)k * k;
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const double v = t[e];
    c[e] = v;
    s += v * v;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) tot += part[i];
    status->gate = status->trace * tot;
  }
}
hipError_t launch_core_gate(hipStream_t st, int k, const double *t, double *c, SmallStatus *status) {
  hipLaunchKernelGGL(core_gate_kernel, dim3(1), dim3(1024), 0, st, k, t, c, status);
  return hipGetLastError();
}

hipError_t launch_identity(hipStream_t st, int k, double *c) {
  GemmArgs a{};
  a.k = k; a.c = c; a.gx = 1; a.gy = 1;
  return launch_identity_k(st, a, GroupRef{}, 1);
}

// LDS pool (doubles) of the tridiagonalisation and of the eigenvector clean-up.
constexpr int TRI_POOL = 19200;

// Work layout of the pseudo-SVD pipeline (doubles; kq = k * k):
//   U  [0, 4kq)           eigenvectors of G_L (AoS k x k), then the bad-pair
//   B  [4kq, 12kq)        matrices of the repair (B, UB as in the kernel);
//   E = work + 20 kq:     the eigensolver's state between its kernels:
//     HV [0, 4kq)         Householder vectors (column j: rows j+1..k-1)
//     X  [4kq, 5kq)       eigenvectors of the tridiagonal T (column i at i k)
//     HA [5kq, 5kq + 4k)  alpha_j of the reflectors
//     DD, EE, LAM, HB     4 arrays of k: diagonal, off-diagonal, eigenvalues
//                         (ascending), reflector betas
//     CQ [.., + 4k)       diagonal unitary scaling delta_r (quaternions)
//     TN                  ||T|| (max row sum)
struct PsvdLayout {
  double *U, *B, *UB, *HV, *X, *HA, *DD, *EE, *LAM, *HB, *CQ, *TN;
  __host__ __device__ PsvdLayout(double *work, int k) {
    const int64_t kq = (int64_t)k * k;
    U = work; B = work + 4 * kq; UB = work + 12 * kq;
    double *e = work + 20 * kq;
    HV = e; X = e + 4 * kq; HA = e + 5 * kq;
    DD = HA + 4 * k; EE = DD + k; LAM = EE + k; HB = LAM + k; CQ = HB + k; TN = CQ + 4 * k;
  }
};

// pseudo-SVD (Alg. 3) with Y = Q_Y R_Y, Q_Y orthonormal: the complex SVD of
// chi_Y is chi_{Q_Y} times that of chi_{R_Y}, whose left singular vectors
// are the eigenvectors of G_L = R_Y R_Y^* (computed by the structure-
// preserving quaternion eigensolver above, so every singular value comes
// paired).  Pair rule: pair i is good iff sigma_i > TAU_S sigma_0 and it is
// separated from its neighbours by more than tau_p sigma_0 (tau_p = 64 * 2k *
// 2^-53).  Bad part: B = [u_b..., -u_b j ...] (the two members of each bad
// pair), B diag(f) with f from Philox stream 3, Jacobi SVD, one column per
// pair of the leading 2t.  Output C (k x k): H = Q_Y C = [H_g, H_b~].
// (Last kernel of the pipeline: the eigenvectors are in U, the eigenvalues
// in LAM.)
__global__ __launch_bounds__(1024) void psvd_finish_kernel(PsvdArgs args, GroupRef grp) {
  PsvdArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  const int k = A.k;
  double *c = A.c, *work = A.work;
  const uint32_t k0 = A.k0, k1 = A.k1;
  SmallStatus *status = A.status;
  __shared__ int order[512];
  __shared__ double sig[512];
  __shared__ double lam[256];
  __shared__ int good[256];
  __shared__ int n_good, n_bad;
  const PsvdLayout L(work, k);
  double *U = L.U, *B = L.B, *UB = L.UB;
  for (int i = threadIdx.x; i < k; i += blockDim.x) lam[i] = gp(L.LAM)[i];
  __syncthreads();
  // descending order of sigma = sqrt(max(lambda, 0))
  for (int i = threadIdx.x; i < k; i += blockDim.x) sig[i] = sqrt(fmax(lam[k - 1 - i], 0.0));
  __syncthreads();
  if (threadIdx.x == 0) {
    const double s0 = sig[0];
    const double tau_p = 64.0 * 2.0 * k * 0x1p-53;
    int ng = 0;
    for (int i = 0; i < k; ++i) {
      const double si = sig[i];
      bool ok = si > 1e-13 * s0;
      if (ok && i > 0) ok = (sig[i - 1] - si) > tau_p * s0;
      if (ok && i < k - 1) ok = (si - sig[i + 1]) > tau_p * s0;
      good[i] = ok ? 1 : 0;
      ng += ok ? 1 : 0;
    }
    n_good = ng;
    n_bad = k - ng;
    status->t_bad = k - ng;
    status->good_count = ng;
    if (k - ng > 0) status->flags |= 8;
    int g = 0, b = 0;
    for (int i = 0; i < k; ++i) order[i] = good[i] ? g++ : -(1 + b++);
  }
  __syncthreads();
  const int t = n_bad;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e % k, j = e / k;            // j: descending singular value index
    const int dst = order[j];
    const qd uv = gq(U, i, k - 1 - j, k);
    if (dst >= 0) {
      sq_(c, i, dst, k, uv);
    } else {
      const int bi = -dst - 1;
      // f_j = 1 + u_j, u_j = (x0 + 1/2) 2^-32 from counter (j, 0, 3, 0)
      const u32x4 xa = philox((uint32_t)bi, 0u, STREAM_DIAGF, 0u, k0, k1);
      const u32x4 xb = philox((uint32_t)(t + bi), 0u, STREAM_DIAGF, 0u, k0, k1);
      const double fa = 1.0 + ((double)xa.x0 + 0.5) * 0x1p-32;
      const double fb = 1.0 + ((double)xb.x0 + 0.5) * 0x1p-32;
      // first member u, second member -u j (J conj(u_c) is the compact
      // representation of -u j)
      sq_(B, i, bi, k, qscale(uv, fa));
      sq_(B, i, t + bi, k, qscale(qmul(uv, {0.0, 0.0, 1.0, 0.0}), -fb));
    }
  }
  __syncthreads();
  if (t > 0 && A.gs) {
    // Gram-Schmidt branch: the candidates in U_b's column order (the first
    // members u of the bad pairs, then the second members -u j), each
    // orthogonalised twice against the columns taken so far (a quaternion
    // projection q (q^* x) removes a column and its J-partner at once), kept
    // when more than 1e-8 of its norm remains, until t are taken
    __shared__ int badj[256];
    __shared__ qd xs[256], coef[256];
    __shared__ double s_red[16];
    for (int j = threadIdx.x; j < k; j += blockDim.x)
      if (order[j] < 0) badj[-order[j] - 1] = j;
    __syncthreads();
    int taken = 0;
    for (int cand = 0; cand < 2 * t && taken < t; ++cand) {
      const int j = badj[cand % t];
      for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const qd uv = gq(U, i, k - 1 - j, k);
        xs[i] = cand < t ? uv : qscale(qmul(uv, {0.0, 0.0, 1.0, 0.0}), -1.0);
      }
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass) {
        for (int s2 = threadIdx.x; s2 < taken; s2 += blockDim.x) {
          qd a = qzero();
          for (int i = 0; i < k; ++i) qfma_cj(a, gq(c, i, n_good + s2, k), xs[i]);
          coef[s2] = a;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < k; i += blockDim.x) {
          qd x = xs[i];
          for (int s2 = 0; s2 < taken; ++s2) x = qsub(x, qmul(gq(c, i, n_good + s2, k), coef[s2]));
          xs[i] = x;
        }
        __syncthreads();
      }
      double part = 0.0;
      for (int i = threadIdx.x; i < k; i += blockDim.x) part += qnorm2(xs[i]);
      part = wave_sum(part);
      if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = part;
      __syncthreads();
      double nrm2 = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) nrm2 += s_red[w];
      const double nrm = sqrt(nrm2);                      // the candidate had norm 1
      if (nrm > 1e-8) {
        for (int i = threadIdx.x; i < k; i += blockDim.x) sq_(c, i, n_good + taken, k, qscale(xs[i], 1.0 / nrm));
        ++taken;
      }
      __syncthreads();
    }
  } else if (t > 0) {
    sm_jacobi(B, k, 2 * t, k, 60, 1e-15);
    __syncthreads();
    sm_sorted_columns(B, k, 2 * t, k, sig, order, UB, k);
    // chi_{B diag f} has each of B's t nonzero quaternion singular values
    // twice; one column per pair of its leading 2t columns is, in quaternion
    // terms, the leading t columns of the sorted Jacobi result.
    for (int e = threadIdx.x; e < k * t; e += blockDim.x) {
      const int i = e % k, j = e / k;
      sq_(c, i, n_good + j, k, gq(UB, i, j, k));
    }
    __syncthreads();
  }
}


// Minimum-norm least squares for a rank-deficient P (l x k, planar):
// one-sided Jacobi on [P; I] (inner products over the P rows only) gives
// P V = B with orthogonal columns and V accumulated; with sigma_i = ||b_i||,
// P^dagger = V diag(1/sigma_i^2) B^* over sigma_i > tol sigma_max, so
// S^* = (P^dagger)^* = B diag(w) V^*, written planar (l x k).
__global__ __launch_bounds__(1024) void pinv_sstar_kernel(PinvArgs args, GroupRef grp) {
  PinvArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  const int l = A.l, k = A.k;
  const PlanesC<double> p = mkc_d<double>(A.p);
  const int64_t ldp = A.ldp, ldo = A.ldo;
  const double tol = A.tol;
  double *work = A.work;
  Planes<double> out;
  for (int q = 0; q < 4; ++q) out.p[q] = A.out[q];
  __shared__ double sig[256];
  __shared__ double s_max;
  const int rows = l + k;
  double *M = work;                       // rows x k, AoS, ld = rows
  for (int e = threadIdx.x; e < rows * k; e += blockDim.x) {
    const int i = e % rows, j = e / rows;
    qd v;
    if (i < l) v = {p.p[0][i + j * ldp], p.p[1][i + j * ldp], p.p[2][i + j * ldp], p.p[3][i + j * ldp]};
    else v = {(i - l) == j ? 1.0 : 0.0, 0.0, 0.0, 0.0};
    sq_(M, i, j, rows, v);
  }
  __syncthreads();
  sm_jacobi(M, l, k, rows, 60, 1e-15, rows);
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < l; ++i) s += qnorm2(gq(M, i, j, rows));
    sig[j] = sqrt(s);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int j = 0; j < k; ++j) mx = fmax(mx, sig[j]);
    s_max = mx;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < l * k; e += blockDim.x) {
    const int r = e % l, c = e / l;
    qd acc = qzero();
    for (int i = 0; i < k; ++i) {
      const double si = sig[i];
      if (!(si > tol * s_max)) continue;
      const double w = 1.0 / (si * si);
      qfma(acc, qscale(gq(M, r, i, rows), w), qconj(gq(M, l + c, i, rows)));
    }
    const int64_t o = r + (int64_t)c * ldo;
    out.p[0][o] = acc.w; out.p[1][o] = acc.x; out.p[2][o] = acc.y; out.p[3][o] = acc.z;
  }
}

hipError_t launch_pinv_k(hipStream_t st, const PinvArgs &a, GroupRef g, int count) {
  hipLaunchKernelGGL(pinv_sstar_kernel, dim3(g.tab ? count : 1), dim3(1024), 0, st, a, g);
  return hipGetLastError();
}

hipError_t launch_pinv_sstar(hipStream_t st, int l, int k, const double *const p[4], int64_t ldp,
                             double tol, double *work, double *const out[4], int64_t ldo) {
  PinvArgs a{};
  a.l = l; a.k = k; set_planes(a.p, p); a.ldp = ldp; a.tol = tol; a.work = work;
  set_planes(a.out, out); a.ldo = ldo; a.gx = 1; a.gy = 1;
  return launch_pinv_k(st, a, GroupRef{}, 1);
}

// Householder reduction of a k x k quaternion Hermitian matrix to a real
// symmetric tridiagonal with the same eigenvalues: for column j,
// x = G[j+1:, j], alpha = -(x_0 / |x_0|) ||x||, v = x - alpha e_1,
// beta = 2 / ||v||^2 (the reflector I - beta v v^* is unitary and Hermitian
// over the quaternions), p = beta G' v, w = p - (beta / 2) Re(v^* p) v,
// G' <- G' - v w^* - w v^*.  Diagonal d_j = Re G[j, j], off-diagonal
// magnitudes e_j = |alpha_j| (a diagonal unitary scaling makes them real).
//
// The first steps work on G in global memory (G is destroyed); once the
// trailing matrix fits, its lower triangle moves to LDS (packed by columns)
// and the remaining steps run there.  pool: TRI_POOL doubles of LDS.

// packed lower storage of an n0 x n0 block: column s holds rows s..n0-1
__device__ __forceinline__ int pk(int r, int s, int n0) { return s * n0 - ((s * (s - 1)) >> 1) + (r - s); }

// Element (r, c), r >= c, of the lower triangle: packed in LDS (L) or in the
// full matrix in global memory.
template <bool L>
__device__ __forceinline__ qd tri_get(const qd *P, const double *g, int r, int c, int o0, int n0, int k) {
  if constexpr (L) return P[pk(r - o0, c - o0, n0)];
  else return gq(g, r, c, k);
}
template <bool L>
__device__ __forceinline__ void tri_set(qd *P, double *g, int r, int c, int o0, int n0, int k, qd x) {
  if constexpr (L) P[pk(r - o0, c - o0, n0)] = x;
  else sq_(g, r, c, k, x);
}

// One Householder step j of sm_tridiag; the storage (LDS or global) is a
// template parameter so that no access pays for the other's branch or waits.
template <bool L>
__device__ __forceinline__ void tri_step(int j, int k, double *g, qd *P, int o0, int n0, qd *v, qd *pv,
                                         double *d, double *e, double *hv, double *hbeta, double *halpha,
                                         double *s_beta) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = k - j - 1, o = j + 1;
  // (A) one wave forms the reflector of column j: x = G[o.., j], alpha =
  // -|x| x0 / |x0|, v = x - alpha e_0, beta = 2 / |v|^2
  if (wave == 0) {
    qd x[4];
    double loc = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int aa = lane + 64 * t;
      x[t] = aa < n ? tri_get<L>(P, g, o + aa, j, o0, n0, k) : qzero();
      loc += qnorm2(x[t]);
    }
    const double xn2 = wave_sum(loc), xn = sqrt(xn2);
    const qd x0 = {__shfl(x[0].w, 0, 64), __shfl(x[0].x, 0, 64), __shfl(x[0].y, 0, 64), __shfl(x[0].z, 0, 64)};
    const double ax0 = sqrt(qnorm2(x0));
    double beta = 0.0;
    qd alpha = qzero();
    if (xn != 0.0) {
      const qd u = ax0 > 0.0 ? qscale(x0, 1.0 / ax0) : qd{1.0, 0.0, 0.0, 0.0};
      alpha = qscale(u, -xn);
      beta = 1.0 / (xn2 + xn * ax0);
    }
    if (lane == 0) {
      d[j] = tri_get<L>(P, g, j, j, o0, n0, k).w;
      e[j] = xn;
      s_beta[j & 1] = beta;
      if (halpha) { halpha[4 * j] = alpha.w; halpha[4 * j + 1] = alpha.x; halpha[4 * j + 2] = alpha.y; halpha[4 * j + 3] = alpha.z; }
      if (hbeta) hbeta[j] = beta;
    }
    if (beta != 0.0) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int aa = lane + 64 * t;
        if (aa < n) v[aa] = aa == 0 ? qsub(x0, alpha) : x[t];
      }
    }
  }
  __syncthreads();
  const double beta = s_beta[j & 1];
  if (beta == 0.0) return;                         // uniform; G unchanged
  if (hv)
    for (int aa = tid; aa < n; aa += blockDim.x) sq_(hv, aa, j, k, v[aa]);
  // (B) p = beta G' v: lpr lanes per row a (c congruent to sub mod lpr);
  // lower entries G[a, c] (c <= a) and conj(G[c, a]) above, without branches
  {
    const int lpr = n <= 128 ? 8 : 4;
    const int aa = tid / lpr, sub = tid % lpr;
    qd sacc = qzero();
    if (aa < n) {
#pragma unroll 4
      for (int c = sub; c < n; c += lpr) {
        const bool lo = c <= aa;
        qd x = tri_get<L>(P, g, o + (lo ? aa : c), o + (lo ? c : aa), o0, n0, k);
        const double sg = lo ? 1.0 : -1.0;
        x.x *= sg; x.y *= sg; x.z *= sg;
        qfma(sacc, x, v[c]);
      }
    }
    for (int off = 1; off < lpr; off <<= 1) {
      sacc.w += __shfl_xor(sacc.w, off, 64); sacc.x += __shfl_xor(sacc.x, off, 64);
      sacc.y += __shfl_xor(sacc.y, off, 64); sacc.z += __shfl_xor(sacc.z, off, 64);
    }
    if (aa < n && sub == 0) pv[aa] = qscale(sacc, beta);
  }
  __syncthreads();
  // (C) every wave forms s_k = beta/2 Re(v^* p) itself (same order, same
  // value), then the rank-2 update of the lower triangle with w = p - s_k v:
  // G'[a, c] -= v_a conj(w_c) + w_a conj(v_c).  The n (n + 1) / 2 entries
  // are numbered pair of columns by pair of columns and dealt to the threads
  // in turn, so that no thread takes more than one more entry than any other
  // and consecutive threads mostly touch consecutive rows of one column.
  {
    double kl = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int aa = lane + 64 * t;
      if (aa < n) {
        const qd pa = pv[aa], va = v[aa];
        kl += va.w * pa.w + va.x * pa.x + va.y * pa.y + va.z * pa.z;
      }
    }
    const double sk = 0.5 * beta * wave_sum(kl);
    // entries dealt by column pairs: pair p holds column p (rows p .. n - 1)
    // and column n - 1 - p (rows n - 1 - p .. n - 1), n + 1 entries in all
    // (the middle column of an odd n alone); entry E is (pair E / (n + 1),
    // offset E mod (n + 1)), so no square root is needed
    const int np1 = n + 1;
    const int tot = ((n + 1) >> 1) * np1 - ((n & 1) ? (np1 >> 1) : 0);
    const float inv = 1.0f / (float)np1;
    // CH entries per thread at a time: their loads go out together, then the
    // updates and stores (a load never waits for the previous entry's store)
    constexpr int CH = 4;
    const int nt = blockDim.x;
    for (int e0 = tid; e0 < tot; e0 += CH * nt) {
      int ia[CH], ic[CH];
      qd gvs[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int e = e0 + u * nt;
        int cc = 0, aa = 0;
        if (e < tot) {
          int pq = (int)((float)e * inv);
          if (pq * np1 > e) --pq;
          if ((pq + 1) * np1 <= e) ++pq;
          const int off = e - pq * np1;
          const int len1 = n - pq;                 // entries of column pq
          if (off < len1) { cc = pq; aa = pq + off; }
          else { cc = n - 1 - pq; aa = cc + (off - len1); }
        }
        ia[u] = aa;
        ic[u] = cc;
        gvs[u] = e < tot ? tri_get<L>(P, g, o + aa, o + cc, o0, n0, k) : qzero();
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        if (e0 + u * nt >= tot) break;
        const int aa = ia[u], cc = ic[u];
        const qd va = v[aa], vc = v[cc];
        const qd wa = qsub(pv[aa], qscale(va, sk));
        const qd wc = qsub(pv[cc], qscale(vc, sk));
        qd gv = gvs[u];
        gv = qsub(gv, qmul(va, qconj(wc)));
        gv = qsub(gv, qmul(wa, qconj(vc)));
        tri_set<L>(P, g, o + aa, o + cc, o0, n0, k, gv);
      }
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void sm_tridiag(double *g, int k, double *d, double *e, double *pool,
                           double *hv = nullptr, double *hbeta = nullptr, double *halpha = nullptr) {
  __shared__ double s_beta[2];        // by parity of j: a step that skips has no closing barrier
  qd *v = (qd *)pool;                 // up to 256
  qd *pv = v + 256;                   // up to 256
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  int n0 = 0, o0 = 0;                 // LDS block: rows/cols o0 .. o0 + n0 - 1
  qd *P = nullptr;
  #pragma unroll 1
  for (int j = 0; j + 1 < k; ++j) {
    const int n = k - j - 1;
    if (!P && 2 * (n + 1) + (n + 1) * (n + 2) / 2 <= TRI_POOL / 4) {
      // move the lower triangle of G[j:, j:] to LDS (v, pv then sit at its front)
      n0 = n + 1;
      o0 = j;
      v = (qd *)pool;
      pv = v + n0;
      P = pv + n0;
      #pragma unroll 1
      for (int s = wave; s < n0; s += nw)
        #pragma unroll 1
        for (int r = s + lane; r < n0; r += 64) P[pk(r, s, n0)] = gq(g, o0 + r, o0 + s, k);
      __syncthreads();
    }
    if (P) tri_step<true>(j, k, g, P, o0, n0, v, pv, d, e, hv, hbeta, halpha, s_beta);
    else tri_step<false>(j, k, g, P, o0, n0, v, pv, d, e, hv, hbeta, halpha, s_beta);
  }
  if (tid == 0) d[k - 1] = P ? P[pk(k - 1 - o0, k - 1 - o0, n0)].w : gq(g, k - 1, k - 1, k).w;
  __syncthreads();
}

// Number of eigenvalues of the real symmetric tridiagonal (d, e) below x
// (Sturm count through the LDL^T pivots of T - x I).
// The pivot recurrence needs 1/q only to full working precision, not
// correctly rounded: the hardware reciprocal estimate plus one Newton step
// (error ~ the square of the estimate's) replaces the division, and a pivot
// of magnitude below 1e-300 is replaced by +-1e-300 (keeping its sign), so
// that no reciprocal overflows.
__device__ int sturm_count(const double *d, const double *e, int k, double x) {
  int c = 0;
  double q = d[0] - x;
  if (q < 0.0) ++c;
  for (int i = 1; i < k; ++i) {
    if (fabs(q) < 1e-300) q = q < 0.0 ? -1e-300 : 1e-300;
    double r = __builtin_amdgcn_rcp(q);
    r = fma(r, fma(-q, r, 1.0), r);
    const double ei = e[i - 1];
    q = (d[i] - x) - ei * ei * r;
    if (q < 0.0) ++c;
  }
  return c;
}

// Selected eigenvalues of the real symmetric tridiagonal (d, e) by
// multisection: the eigenvalue of ascending index idx[g] (idx == nullptr:
// index g) for g < cnt goes to lam[g].  A group of P threads (P a power of
// two <= 64, so a group never spans two waves) evaluates P Sturm counts per
// round on an even grid of the bracket and keeps the sub-interval where the
// count passes the index; P + 1 times narrower per round.  Stops at full
// precision (bracket within a few ulps of its end points) or below
// u^2 ||T||.
__device__ __forceinline__ void sm_bisect_sel(const double *d, const double *e, int k, const int *idx, int cnt,
                              double *lam) {
  __shared__ double s_lo, s_hi;
  if (threadIdx.x == 0) {
    double lo = d[0], hi = d[0];
    for (int i = 0; i < k; ++i) {
      const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < k ? fabs(e[i]) : 0.0);
      lo = fmin(lo, d[i] - r);
      hi = fmax(hi, d[i] + r);
    }
    const double pad = 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300;
    s_lo = lo - pad;
    s_hi = hi + pad;
  }
  __syncthreads();
  int P = 64;
  while (P > 1 && P * cnt > (int)blockDim.x) P >>= 1;
  const int ngroups = blockDim.x / P;
  const int grp = threadIdx.x / P, sub = threadIdx.x % P;
  const int lane_base = (threadIdx.x & 63) & ~(P - 1);
  const uint64_t gmask = P == 64 ? ~0ull : ((1ull << P) - 1ull);
  const double floor_w = 0x1p-106 * fmax(fabs(s_lo), fabs(s_hi));
  // every lane of a wave runs the same number of rounds (the ballot needs the
  // whole wave): groups past cnt work on a dummy index and store nothing
  const int rounds_groups = (cnt + ngroups - 1) / ngroups;
  for (int rg = 0; rg < rounds_groups; ++rg) {
    const int g = grp + rg * ngroups;
    const bool active = g < cnt;
    const int i = active ? (idx ? idx[g] : g) : 0;
    double lo = s_lo, hi = active ? s_hi : s_lo;     // inactive groups start done
    for (int it = 0; it < 120; ++it) {
      const double w = hi - lo;
      const bool done = w <= 4.0 * 0x1p-53 * fmax(fabs(lo), fabs(hi)) || w <= floor_w;
      // the wave keeps iterating until all its groups are done
      if (__ballot(!done) == 0ull) break;
      const double h = w / (double)(P + 1);
      const double x = lo + (double)(sub + 1) * h;
      const bool above = sturm_count(d, e, k, x) > i;    // lambda_i < x
      const uint64_t bits = (__ballot(above) >> lane_base) & gmask;
      if (!done) {
        if (bits == 0ull) {
          lo = lo + (double)P * h;
        } else {
          const int s = __builtin_ctzll(bits);
          const double nhi = lo + (double)(s + 1) * h;
          const double nlo = s > 0 ? lo + (double)s * h : lo;
          lo = nlo;
          hi = nhi;
        }
      }
    }
    if (active && sub == 0) lam[g] = 0.5 * (lo + hi);
  }
  __syncthreads();
}

// Sturm count of sturm_count with (d, e^2) in LDS (e2[i - 1] = e[i - 1]^2,
// the product the recurrence forms), four steps per loop trip so that the
// loads run ahead of the dependent pivot chain.
__device__ __forceinline__ int sturm_count_lds(const QSK_LDS double *d, const QSK_LDS double *e2, int k,
                                               double x) {
  int c = 0;
  double q = d[0] - x;
  if (q < 0.0) ++c;
  int i = 1;
  for (; i + 3 < k; i += 4) {
    const double d0 = d[i], d1 = d[i + 1], d2 = d[i + 2], d3 = d[i + 3];
    const double f0 = e2[i - 1], f1 = e2[i], f2 = e2[i + 1], f3 = e2[i + 2];
#define QSK_STURM_STEP(DI, FI)                                  \
    {                                                           \
      if (fabs(q) < 1e-300) q = q < 0.0 ? -1e-300 : 1e-300;     \
      double r = __builtin_amdgcn_rcp(q);                       \
      r = fma(r, fma(-q, r, 1.0), r);                           \
      q = ((DI) - x) - (FI) * r;                                \
      if (q < 0.0) ++c;                                         \
    }
    QSK_STURM_STEP(d0, f0) QSK_STURM_STEP(d1, f1) QSK_STURM_STEP(d2, f2) QSK_STURM_STEP(d3, f3)
  }
  for (; i < k; ++i) QSK_STURM_STEP(d[i], e2[i - 1])
#undef QSK_STURM_STEP
  return c;
}

// Eigenvalue i (ascending) of the real symmetric tridiagonal (d, e) by one
// wave: multisection of the Gershgorin bracket with 64 Sturm counts per
// round (65 times narrower per round), with the stopping rule of
// sm_bisect_sel.  e2 holds e^2.  Every lane returns the value.
__device__ double wave_bisect(const QSK_LDS double *d, const QSK_LDS double *e, const QSK_LDS double *e2,
                              int k, int i) {
  const int lane = threadIdx.x & 63;
  double lo = INFINITY, hi = -INFINITY;
  for (int j = lane; j < k; j += 64) {
    const double r = (j > 0 ? fabs(e[j - 1]) : 0.0) + (j + 1 < k ? fabs(e[j]) : 0.0);
    lo = fmin(lo, d[j] - r);
    hi = fmax(hi, d[j] + r);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
  }
  const double pad = 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300;
  lo -= pad;
  hi += pad;
  const double floor_w = 0x1p-106 * fmax(fabs(lo), fabs(hi));
  for (int it = 0; it < 120; ++it) {
    const double w = hi - lo;                   // the same in every lane
    if (w <= 4.0 * 0x1p-53 * fmax(fabs(lo), fabs(hi)) || w <= floor_w) break;
    const double h = w / 65.0;
    const double x = lo + (double)(lane + 1) * h;
    const uint64_t bits = __ballot(sturm_count_lds(d, e2, k, x) > i);     // lambda_i < x
    if (bits == 0ull) {
      lo = lo + 64.0 * h;
    } else {
      const int s = __builtin_ctzll(bits);
      const double nhi = lo + (double)(s + 1) * h;
      lo = s > 0 ? lo + (double)s * h : lo;
      hi = nhi;
    }
  }
  return 0.5 * (lo + hi);
}

// One vector of cgs2_block: x_i (at xi) loses its components along x_0 ..
// x_{i-1} (in xs) twice, then is normalised.
template <typename P, typename PI>
__device__ __forceinline__ void cgs2_vec(P xs, PI xi, int i, int k, double *coef, double *s_nrm,
                                         QSK_LDS double *red) {
  // inner products: 16 lanes per pair (j, i), 64 pairs at a time; the
  // update x_i -= sum_j coef_j x_j: rows over rb threads, the sum over j
  // split in np partial sums (short serial chains) that meet in red
  // (blockDim.x doubles of LDS).  The loops are unrolled so that several
  // loads are in flight (the sums keep their order).
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nt = blockDim.x, grp = tid >> 4, sl = tid & 15, ngrp = nt >> 4;
  const int rb = k <= 128 ? 128 : 256, np = nt / rb, row = tid % rb, part = tid / rb;
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = grp; j < i; j += ngrp) {
      P xj = xs + (int64_t)j * k;
      double s = 0.0;
#pragma unroll 4
      for (int r = sl; r < k; r += 16) s += xj[r] * xi[r];
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (sl == 0) coef[j] = s;
    }
    __syncthreads();
    if (part < np) {
      double acc = 0.0;
      if (row < k)
#pragma unroll 8
        for (int j = part; j < i; j += np) acc += coef[j] * xs[(int64_t)j * k + row];
      red[part * rb + row] = acc;
    }
    __syncthreads();
    if (part == 0 && row < k) {
      double s = 0.0;
      for (int p = 0; p < np; ++p) s += red[p * rb + row];
      xi[row] -= s;
    }
    __syncthreads();
  }
  if (wave == 0) {
    double s = 0.0;
    for (int r = lane; r < k; r += 64) s += xi[r] * xi[r];
    s = wave_sum(s);
    if (lane == 0) *s_nrm = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  }
  __syncthreads();
  const double sc = *s_nrm;
  for (int r = tid; r < k; r += blockDim.x) xi[r] *= sc;
  __syncthreads();
}

// Classical Gram-Schmidt, twice, over the c vectors xs[0..c) (length k,
// stride k; LDS or global), in order: each vector loses its components along
// the earlier ones and is normalised.  With xl (k doubles of LDS) the vector
// being orthogonalised is worked on there and copied back when done.
template <typename P>
__device__ __forceinline__ void cgs2_block(P xs, int k, int c, double *coef, double *s_nrm,
                                           QSK_LDS double *red, QSK_LDS double *xl = nullptr) {
  const int tid = threadIdx.x;
  for (int i = 1; i < c; ++i) {
    P xi = xs + (int64_t)i * k;
    if (xl) {
      for (int r = tid; r < k; r += blockDim.x) xl[r] = xi[r];
      __syncthreads();
      cgs2_vec(xs, xl, i, k, coef, s_nrm, red);
      for (int r = tid; r < k; r += blockDim.x) xi[r] = xl[r];
      __syncthreads();
    } else {
      cgs2_vec(xs, xi, i, k, coef, s_nrm, red);
    }
  }
}

// Full eigendecomposition of the k x k quaternion Hermitian G_L for the
// pseudo-SVD, as a pipeline of kernels (state in the PsvdLayout arrays):
//   psvd_eig_kernel      tridiagonalisation, one workgroup;
//   psvd_invit_kernel    eigenvalues of T by multisection, one wave each,
//                        then their eigenvectors by inverse iteration, four
//                        per workgroup, each lane with its LU factors in LDS;
//   psvd_orth_kernel     Gram-Schmidt twice inside clusters of eigenvalues
//                        closer than 1e-3 ||T|| and the diagonal unitary
//                        scaling, one workgroup;
//   psvd_bt_kernel       back-transformation through the Householder
//                        reflectors, one wave per column, four columns per
//                        workgroup;
//   psvd_finish_kernel   pair rule and bad-pair repair (above).
__global__ __launch_bounds__(1024) void psvd_eig_kernel(PsvdArgs args, GroupRef grp) {
  PsvdArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  const int k = A.k;
  const PsvdLayout L(A.work, k);
  __shared__ double dd[256], ee[256], hb[256];
  __shared__ double pool[TRI_POOL];
  sm_tridiag(A.gl, k, dd, ee, pool, L.HV, hb, L.HA);
  const int tid = threadIdx.x;
  if (tid == 0) {
    double tn = 0.0;
    for (int i = 0; i < k; ++i) tn = fmax(tn, fabs(dd[i]) + (i > 0 ? ee[i - 1] : 0.0) + (i + 1 < k ? ee[i] : 0.0));
    gpw(L.TN)[0] = tn;
  }
  for (int i = tid; i < k; i += blockDim.x) {
    gpw(L.DD)[i] = dd[i];
    gpw(L.EE)[i] = ee[i];
    gpw(L.HB)[i] = hb[i];
  }
}

// Eigenvector of the real symmetric tridiagonal (d, e) for eigenvalue lam:
// three solves with the partial-pivoting LU of T - lam I from a
// pseudo-random start (Philox, fixed key, counter (seq, j)), so that equal or
// nearly equal eigenvalues still give independent vectors.  The LU factors
// and x are private LDS arrays of length k; the pivots' reciprocals are
// formed once.
__device__ void invit_lds(const QSK_LDS double *d, const QSK_LDS double *e, int k, double lam, double tnorm,
                          uint32_t seq, QSK_LDS double *x, QSK_LDS double *dl, QSK_LDS double *dd,
                          QSK_LDS double *du, QSK_LDS double *du2, QSK_LDS double *pv) {
  const double tiny = 0x1p-52 * tnorm + 1e-300;
  for (int j = 0; j < k; ++j) {
    const u32x4 r = philox(seq, (uint32_t)j, 0x51u, 0u, 0x2545F491u, 0x9E3779B9u);
    x[j] = ((double)r.x0 + 0.5) * 0x1p-31 - 1.0;
  }
  for (int j = 0; j < k; ++j) {
    dd[j] = d[j] - lam;
    if (j + 1 < k) { dl[j] = e[j]; du[j] = e[j]; }
    du2[j] = 0.0;
    pv[j] = 0.0;
  }
  double dj = dd[0];
  for (int j = 0; j + 1 < k; ++j) {
    const double lj = dl[j], uj = du[j], dn = dd[j + 1];
    if (fabs(dj) >= fabs(lj)) {
      if (dj == 0.0) dj = tiny;
      const double f = lj / dj;
      dd[j] = dj;
      dl[j] = f;
      dj = dn - f * uj;
    } else {
      const double f = dj / lj;
      dd[j] = lj;
      dl[j] = f;
      du[j] = dn;
      dj = uj - f * dn;
      if (j + 2 < k) {
        const double u1 = du[j + 1];
        du2[j] = u1;
        du[j + 1] = -f * u1;
      }
      pv[j] = 1.0;
    }
  }
  if (dj == 0.0) dj = tiny;
  dd[k - 1] = dj;
  for (int j = 0; j < k; ++j) dd[j] = 1.0 / dd[j];        // reciprocals of the pivots
  for (int it = 0; it < 3; ++it) {
    double xj = x[0];
    for (int j = 0; j + 1 < k; ++j) {
      double xn = x[j + 1];
      if (pv[j] != 0.0) { const double t = xj; xj = xn; xn = t; }
      x[j] = xj;
      xj = xn - dl[j] * xj;
    }
    x[k - 1] = xj;
    double x2 = xj * dd[k - 1];
    x[k - 1] = x2;
    double x1 = 0.0;
    if (k > 1) { x1 = (x[k - 2] - du[k - 2] * x2) * dd[k - 2]; x[k - 2] = x1; }
    for (int j = k - 3; j >= 0; --j) {
      const double xv = (x[j] - du[j] * x1 - du2[j] * x2) * dd[j];
      x[j] = xv;
      x2 = x1;
      x1 = xv;
    }
    double nrm = 0.0;
    for (int j = 0; j < k; ++j) nrm += x[j] * x[j];
    nrm = sqrt(nrm);
    if (!(nrm > 0.0) || !isfinite(nrm)) { for (int j = 0; j < k; ++j) x[j] = (j == 0); nrm = 1.0; }
    const double inv = 1.0 / nrm;
    for (int j = 0; j < k; ++j) x[j] *= inv;
  }
}

constexpr int INVIT_EPB = 4;          // eigenpairs per workgroup
// Eigenvalues INVIT_EPB bx .. + INVIT_EPB - 1 of T, one wave each (written
// to LAM), then their eigenvectors, one lane of the first wave each.
__global__ __launch_bounds__(64 * INVIT_EPB) void psvd_invit_kernel(PsvdArgs args, GroupRef grp) {
  PsvdArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  const int k = A.k;
  const PsvdLayout L(A.work, k);
  __shared__ double sd[256], se[256], se2[256], slam[INVIT_EPB];
  __shared__ double lu[INVIT_EPB][6][258];     // padded: lanes hit different banks
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = tid; j < k; j += blockDim.x) {
    const double ej = gp(L.EE)[j];
    sd[j] = gp(L.DD)[j];
    se[j] = ej;
    se2[j] = ej * ej;
  }
  __syncthreads();
  const int iw = bx * INVIT_EPB + wave;
  if (iw < k) {                                 // the whole wave
    const double lv = wave_bisect((const QSK_LDS double *)sd, (const QSK_LDS double *)se,
                                  (const QSK_LDS double *)se2, k, iw);
    if (lane == 0) {
      slam[wave] = lv;
      gpw(L.LAM)[iw] = lv;
    }
  }
  __syncthreads();
  const int i = bx * INVIT_EPB + lane;
  if (wave == 0 && lane < INVIT_EPB && i < k) {
    QSK_LDS double(*b)[258] = (QSK_LDS double(*)[258])lu[lane];
    invit_lds((const QSK_LDS double *)sd, (const QSK_LDS double *)se, k, slam[lane], gp(L.TN)[0],
              (uint32_t)i, b[0], b[1], b[2], b[3], b[4], b[5]);
    QSK_GLOBAL double *xo = gpw(L.X) + (int64_t)i * k;
    for (int j = 0; j < k; ++j) xo[j] = b[0][j];
  }
}

__global__ __launch_bounds__(1024) void psvd_orth_kernel(PsvdArgs args, GroupRef grp) {
  PsvdArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  const int k = A.k;
  const PsvdLayout L(A.work, k);
  __shared__ double lam[256], coef[256];
  __shared__ double s_nrm;
  __shared__ double pool[TRI_POOL];
  const int tid = threadIdx.x;
  for (int i = tid; i < k; i += blockDim.x) lam[i] = gp(L.LAM)[i];
  __syncthreads();
  const double tn = gp(L.TN)[0];
  // re-orthogonalise within clusters (ascending order), in LDS when they fit
  for (int c0 = 0; c0 < k;) {
    int c1 = c0 + 1;
    while (c1 < k && lam[c1] - lam[c1 - 1] <= 1e-3 * tn) ++c1;
    const int c = c1 - c0;
    if (c > 1) {
      QSK_GLOBAL double *xg = gpw(L.X) + (int64_t)c0 * k;
      if ((int64_t)c * k + 1024 <= TRI_POOL) {
        QSK_LDS double *xs = (QSK_LDS double *)pool;
        for (int q = tid; q < c * k; q += blockDim.x) xs[q] = xg[q];
        __syncthreads();
        cgs2_block(xs, k, c, coef, &s_nrm, (QSK_LDS double *)(pool + (int64_t)c * k));
        for (int q = tid; q < c * k; q += blockDim.x) xg[q] = xs[q];
        __syncthreads();
      } else {
        cgs2_block(xg, k, c, coef, &s_nrm, (QSK_LDS double *)pool, (QSK_LDS double *)pool + 1024);
      }
    }
    c0 = c1;
  }
  // diagonal unitary scaling: delta_0 = 1, delta_{j+1} = alpha_j delta_j / |alpha_j|
  // (the alpha_j staged in LDS in parallel, the running product formed by
  // one thread, the result copied out in parallel)
  __syncthreads();
  qd *als = (qd *)pool;
  qd *dls = als + k;
  for (int j = tid; j + 1 < k; j += blockDim.x)
    als[j] = qd{gp(L.HA)[4 * j], gp(L.HA)[4 * j + 1], gp(L.HA)[4 * j + 2], gp(L.HA)[4 * j + 3]};
  __syncthreads();
  if (tid == 0) {
    qd delta = {1.0, 0.0, 0.0, 0.0};
    dls[0] = delta;
    for (int j = 0; j + 1 < k; ++j) {
      const qd al = als[j];
      const double aa = sqrt(qnorm2(al));
      if (aa > 0.0) delta = qmul(qscale(al, 1.0 / aa), delta);
      dls[j + 1] = delta;
    }
  }
  __syncthreads();
  QSK_GLOBAL double *cq = gpw(L.CQ);
  for (int j = tid; j < k; j += blockDim.x) {
    const qd dj = dls[j];
    cq[4 * j] = dj.w; cq[4 * j + 1] = dj.x; cq[4 * j + 2] = dj.y; cq[4 * j + 3] = dj.z;
  }
}

// u = H_0 H_1 ... H_{k-2} D x for each column: lane r of the column's wave
// owns rows r, r + 64, ... (in registers); only the inner products v^* u
// cross lanes.  The reflector of the next step is loaded while this one is
// applied.
constexpr int BT_COLS = 4;             // columns (waves) per workgroup
__global__ __launch_bounds__(64 * BT_COLS) void psvd_bt_kernel(PsvdArgs args, GroupRef grp) {
  PsvdArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  const int k = A.k;
  const PsvdLayout L(A.work, k);
  const int lane = threadIdx.x & 63;
  const int col = bx * BT_COLS + (threadIdx.x >> 6);
  if (col >= k) return;                         // whole wave
  constexpr int R = 4;                          // rows per lane (k <= 256)
  qd u[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int r = lane + 64 * t;
    u[t] = qzero();
    if (r < k) {
      const QSK_GLOBAL double *cq = gp(L.CQ) + 4 * r;
      u[t] = qscale(qd{cq[0], cq[1], cq[2], cq[3]}, gp(L.X)[(int64_t)col * k + r]);
    }
  }
  qd vn[R];
  double bn = 0.0;
#define QSK_BT_LOAD(J)                                                               \
  do {                                                                               \
    bn = (J) >= 0 ? gp(L.HB)[(J)] : 0.0;                                             \
    _Pragma("unroll") for (int t = 0; t < R; ++t) {                                  \
      const int r = lane + 64 * t;                                                   \
      vn[t] = ((J) >= 0 && r > (J) && r < k) ? gq(L.HV, r - (J) - 1, (J), k) : qzero(); \
    }                                                                                \
  } while (0)
  QSK_BT_LOAD(k - 2);
  for (int j = k - 2; j >= 0; --j) {
    qd v[R];
#pragma unroll
    for (int t = 0; t < R; ++t) v[t] = vn[t];
    const double beta = bn;
    QSK_BT_LOAD(j - 1);
    if (beta == 0.0) continue;                  // uniform
    qd s = qzero();
#pragma unroll
    for (int t = 0; t < R; ++t) qfma_cj(s, v[t], u[t]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s.w += __shfl_xor(s.w, off, 64);
      s.x += __shfl_xor(s.x, off, 64);
      s.y += __shfl_xor(s.y, off, 64);
      s.z += __shfl_xor(s.z, off, 64);
    }
    s = qscale(s, beta);
#pragma unroll
    for (int t = 0; t < R; ++t) u[t] = qsub(u[t], qmul(v[t], s));
  }
#undef QSK_BT_LOAD
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int r = lane + 64 * t;
    if (r < k) sq_(L.U, r, col, k, u[t]);
  }
}

static int psvd_invit_blocks(int k) { return (k + INVIT_EPB - 1) / INVIT_EPB; }
static int psvd_bt_blocks(int k) { return (k + BT_COLS - 1) / BT_COLS; }
int psvd_blocks(int k, int stage) { return stage == 1 ? psvd_invit_blocks(k) : stage == 3 ? psvd_bt_blocks(k) : 1; }

hipError_t launch_psvd_stage(hipStream_t st, int stage, const PsvdArgs &a, GroupRef g, int64_t blocks) {
  const dim3 grid((unsigned)(g.tab ? blocks : psvd_blocks(a.k, stage)));
  switch (stage) {
    case 0: hipLaunchKernelGGL(psvd_eig_kernel, grid, dim3(1024), 0, st, a, g); break;
    case 1: hipLaunchKernelGGL(psvd_invit_kernel, grid, dim3(64 * INVIT_EPB), 0, st, a, g); break;
    case 2: hipLaunchKernelGGL(psvd_orth_kernel, grid, dim3(1024), 0, st, a, g); break;
    case 3: hipLaunchKernelGGL(psvd_bt_kernel, grid, dim3(64 * BT_COLS), 0, st, a, g); break;
    default: hipLaunchKernelGGL(psvd_finish_kernel, grid, dim3(1024), 0, st, a, g); break;
  }
  return hipGetLastError();
}

hipError_t launch_psvd_select(hipStream_t st, int k, double *gl, uint32_t k0, uint32_t k1,
                              double *c, double *work, SmallStatus *status, int gs) {
  for (int stage = 0; stage < 5; ++stage) {
    PsvdArgs a{};
    a.k = k; a.gl = gl; a.k0 = k0; a.k1 = k1; a.c = c; a.work = work; a.status = status; a.gs = gs;
    a.gx = psvd_blocks(k, stage); a.gy = 1;
    const hipError_t e = launch_psvd_stage(st, stage, a, GroupRef{}, 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Eigen-decomposition of a k x k quaternion Hermitian matrix g (AoS, destroyed):
// the first four stages of the pseudo-SVD pipeline (tridiagonalisation and
// bisection, inverse iteration, re-orthogonalisation, back-transformation).
// Eigenvalues ascending in PsvdLayout(work, k).LAM, eigenvectors in .U (AoS,
// column i for eigenvalue i).
hipError_t launch_herm_eig(hipStream_t st, int k, double *g, double *work, SmallStatus *status) {
  for (int stage = 0; stage < 4; ++stage) {
    PsvdArgs a{};
    a.k = k; a.gl = g; a.work = work; a.status = status;
    a.gx = psvd_blocks(k, stage); a.gy = 1;
    const hipError_t e = launch_psvd_stage(st, stage, a, GroupRef{}, 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Truncation (Alg. 5) from the eigenpairs of X X^* = U Sigma^2 U^*: column c
// of cu is the eigenvector of the c-th largest eigenvalue, cv the same
// column over sigma_c = sqrt(max(lambda, 0)) (zero when sigma_c is zero),
// sigma[c] = sigma_c.  cu, cv: AoS k x r.
__global__ __launch_bounds__(256) void trunc_select_kernel(const double *work, int k, int r, double *cu,
                                                           double *cv, double *sigma) {
  const PsvdLayout L(const_cast<double *>(work), k);
  for (int e = threadIdx.x; e < k * r; e += blockDim.x) {
    const int i = e % k, c = e / k, src = k - 1 - c;
    const double s = sqrt(fmax(gp(L.LAM)[src], 0.0));
    const qd u = gq(L.U, i, src, k);
    sq_(cu, i, c, k, u);
    sq_(cv, i, c, k, s > 0.0 ? qscale(u, 1.0 / s) : qzero());
  }
  for (int c = threadIdx.x; c < r; c += blockDim.x) sigma[c] = sqrt(fmax(gp(L.LAM)[k - 1 - c], 0.0));
}

hipError_t launch_trunc_select(hipStream_t st, const double *work, int k, int r, double *cu, double *cv,
                               double *sigma) {
  hipLaunchKernelGGL(trunc_select_kernel, dim3(1), dim3(256), 0, st, work, k, r, cu, cv, sigma);
  return hipGetLastError();
}

// Z (rows x cols planar, ldz) = X^* for X (cols x rows planar, ldx).
__global__ void conj_transpose_k(PlanesC<double> x, int64_t ldx, int64_t rows, int64_t cols, Planes<double> z,
                                 int64_t ldz) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e % rows, i = e / rows;
    const int64_t src = i + t * ldx;
    z.p[0][t + i * ldz] = x.p[0][src];
    z.p[1][t + i * ldz] = -x.p[1][src];
    z.p[2][t + i * ldz] = -x.p[2][src];
    z.p[3][t + i * ldz] = -x.p[3][src];
  }
}

hipError_t launch_conj_transpose(hipStream_t st, const double *const x[4], int64_t ldx, int64_t rows, int64_t cols,
                                 double *const z[4], int64_t ldz) {
  PlanesC<double> a;
  Planes<double> b;
  for (int p = 0; p < 4; ++p) { a.p[p] = x[p]; b.p[p] = z[p]; }
  const int64_t blocks = std::min<int64_t>((rows * cols + 255) / 256, 16384);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(conj_transpose_k, dim3((unsigned)blocks), dim3(256), 0, st, a, ldx, rows, cols, b, ldz);
  return hipGetLastError();
}

// kappa of H from its Gram G_H = H^* H: the eigenvalues of G_H are the
// squared singular values of H, so kappa(H) = sqrt(lambda_max / lambda_min)
// (Section 3.1, after Remark 3.1).  which: 0 -> status->kappa (and the
// orthonormality defect max|G_H - I|), 1 -> status->kappa_initial.
__global__ __launch_bounds__(1024) void kappa_kernel(KappaArgs args, GroupRef grp) {
  KappaArgs A;
  int bx, by, bz;
  if (!group_select(args, grp, A, bx, by, bz)) return;
  const int k = A.k, which = A.which;
  const double *gh = A.gh;
  double *work = A.work;
  SmallStatus *status = A.status;
  __shared__ double dd[256], ee[256], lam[256];
  __shared__ double s_def;
  const int64_t kk = (int64_t)k * k * 4;
  double *G = work;
  {
    __shared__ double s_w[16];
    double dft = 0.0;
    for (int q = threadIdx.x; q < k * k; q += blockDim.x) {
      const int i = q % k, j = q / k;
      qd v = gq(gh, i, j, k);
      if (i == j) v.w -= 1.0;
      dft = fmax(dft, sqrt(qnorm2(v)));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dft = fmax(dft, __shfl_xor(dft, off, 64));
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = dft;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t = fmax(t, s_w[q]);
      s_def = t;
    }
  }
  __shared__ int ends[2];
  __shared__ double pool[TRI_POOL];
  sm_copy(G, gh, (int)kk);
  sm_tridiag(G, k, dd, ee, pool);
  if (threadIdx.x == 0) { ends[0] = 0; ends[1] = k - 1; }
  __syncthreads();
  sm_bisect_sel(dd, ee, k, ends, 2, lam);
  if (threadIdx.x == 0) {
    const double lmin = lam[0], lmax = lam[1];
    const double kap = lmin > 0.0 ? sqrt(lmax / lmin) : INFINITY;
    if (which == 0) { status->kappa = kap; status->orth_defect = s_def; }
    else status->kappa_initial = kap;
  }
}

hipError_t launch_kappa_k(hipStream_t st, const KappaArgs &a, GroupRef g, int count) {
  hipLaunchKernelGGL(kappa_kernel, dim3(g.tab ? count : 1), dim3(1024), 0, st, a, g);
  return hipGetLastError();
}

hipError_t launch_kappa(hipStream_t st, int k, const double *gh, double *work, int which,
                        SmallStatus *status) {
  KappaArgs a{};
  a.k = k; a.gh = gh; a.work = work; a.which = which; a.status = status; a.gx = 1; a.gy = 1;
  return launch_kappa_k(st, a, GroupRef{}, 1);
}

}  // namespace qsk
