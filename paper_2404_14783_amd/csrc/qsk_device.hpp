// Device-side building blocks shared by the qsketch kernels: Philox4x32-10,
// the quaternion Gaussian / Rademacher test-matrix entries, exact rounding to
// the operand formats, and FP64 quaternion arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qsk_kernels.hpp"

// Global-memory views of generic pointers: loads and stores through them are
// global_* instructions (counted by vmcnt only), so waits for LDS results do
// not also wait for global loads in flight, as they must for flat_* ones.
#define QSK_GLOBAL __attribute__((address_space(1)))
#define QSK_LDS __attribute__((address_space(3)))
template <typename T>
__device__ __forceinline__ const QSK_GLOBAL T *gp(const T *p) { return (const QSK_GLOBAL T *)p; }
template <typename T>
__device__ __forceinline__ QSK_GLOBAL T *gpw(T *p) { return (QSK_GLOBAL T *)p; }

namespace qsk {

enum : int { STREAM_OMEGA = 0, STREAM_PSI = 1, STREAM_POWER = 2, STREAM_DIAGF = 3 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the Philox S-box,
// key advanced by the Weyl constants between rounds.
struct u32x4 { uint32_t x0, x1, x2, x3; };

__device__ __forceinline__ u32x4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

// ---------------------------------------------------------------------------
// Rounding helpers.  All produce the value of the target format held in a
// float (bf16 and e4m3 values are exactly representable in FP32).

__device__ __forceinline__ float bf16_rne(float f) {     // RNE, finite inputs
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

__device__ __forceinline__ float bf16_rne_d(double d) {  // single rounding from FP64
  uint64_t u = (uint64_t)__double_as_longlong(d);
  u += 0x00000FFFFFFFFFFFull + ((u >> 45) & 1ull);
  u &= ~0x00001FFFFFFFFFFFull;
  return (float)__longlong_as_double((long long)u);
}

// OCP e4m3fn: 3 mantissa bits, normals down to 2^-6, subnormal quantum 2^-9,
// saturate at 448.
__device__ __forceinline__ float e4m3_rne(float f) {
  const float a = fabsf(f);
  if (a == 0.f) return f;
  int e;
  (void)frexpf(a, &e);                       // a = m 2^e, 0.5 <= m < 1
  const int lead = max(e - 1, -6);
  const float q = ldexpf(1.f, lead - 3);
  float r = rintf(a / q) * q;
  r = fminf(r, 448.f);
  return copysignf(r, f);
}

__device__ __forceinline__ float e4m3_rne_d(double d) {
  const double a = fabs(d);
  if (a == 0.0) return (float)d;
  int e;
  (void)frexp(a, &e);
  const int lead = max(e - 1, -6);
  const double q = ldexp(1.0, lead - 3);
  double r = rint(a / q) * q;
  r = fmin(r, 448.0);
  return (float)copysign(r, d);
}

template <int MODE> __device__ __forceinline__ float round_mode(float f) {
  if constexpr (MODE == MODE_BF16) return bf16_rne(f);
  else if constexpr (MODE == MODE_FP8) return e4m3_rne(f);
  else return f;
}
template <int MODE> __device__ __forceinline__ float round_mode_d(double d) {
  if constexpr (MODE == MODE_BF16) return bf16_rne_d(d);
  else if constexpr (MODE == MODE_FP8) return e4m3_rne_d(d);
  else return (float)d;
}

// ---------------------------------------------------------------------------
// Quaternion Gaussian entry from one Philox output (Box-Muller on the pairs
// (x0, x1) and (x2, x3), u = (x + 1/2) 2^-32).

__device__ __forceinline__ void gauss_f64(const u32x4 &x, double out[4]) {
  const double s = 0x1p-32;
  const double u0 = ((double)x.x0 + 0.5) * s, u1 = ((double)x.x1 + 0.5) * s;
  const double u2 = ((double)x.x2 + 0.5) * s, u3 = ((double)x.x3 + 0.5) * s;
  const double ra = sqrt(-2.0 * log(u0)), rb = sqrt(-2.0 * log(u2));
  double sa, ca, sb, cb;
  sincospi(2.0 * u1, &sa, &ca);
  sincospi(2.0 * u3, &sb, &cb);
  out[0] = ra * ca; out[1] = ra * sa; out[2] = rb * cb; out[3] = rb * sb;
}

// FP32 evaluation with relative accuracy everywhere: ln u through log1p near
// u = 1, and the angle reduced to the nearest quarter turn in integer
// arithmetic before the float sine/cosine.
__device__ __forceinline__ float ln_uniform_f32(uint32_t x) {
  if (x < 0x80000000u) return logf((float)(2u * x + 1u) * 0x1p-33f);
  const uint32_t w = 2u * (0xFFFFFFFFu - x) + 1u;            // 2^33 (1 - u)
  return log1pf(-(float)w * 0x1p-33f);
}

__device__ __forceinline__ void sincos_turn_f32(uint32_t x, float *s, float *c) {
  // theta = 2 pi v / 2^33 with v = 2x + 1; quarter turn = 2^31.
  const uint64_t v = 2ull * x + 1ull;
  const uint64_t q = (v + (1ull << 30)) >> 31;
  const long long d = (long long)v - (long long)(q << 31);    // |d| <= 2^30
  const float phi = (float)d * (float)(6.283185307179586476925 * 0x1p-33);   // 2 pi / 2^33
  float sp, cp;
  sincosf(phi, &sp, &cp);
  switch ((int)(q & 3ull)) {
    case 0: *c = cp; *s = sp; break;
    case 1: *c = -sp; *s = cp; break;
    case 2: *c = -cp; *s = -sp; break;
    default: *c = sp; *s = -cp; break;
  }
}

__device__ __forceinline__ void gauss_f32(const u32x4 &x, float out[4]) {
  const float ra = sqrtf(-2.f * ln_uniform_f32(x.x0));
  const float rb = sqrtf(-2.f * ln_uniform_f32(x.x2));
  float sa, ca, sb, cb;
  sincos_turn_f32(x.x1, &sa, &ca);
  sincos_turn_f32(x.x3, &sb, &cb);
  out[0] = ra * ca; out[1] = ra * sa; out[2] = rb * cb; out[3] = rb * sb;
}

// Relative margin that covers the FP32 evaluation error of gauss_f32.
#define QSK_GUARD_REL 0x1p-20f

template <int MODE> __device__ __forceinline__ bool near_tie(float z) {
  const float lo = z * (1.f - QSK_GUARD_REL), hi = z * (1.f + QSK_GUARD_REL);
  return round_mode<MODE>(lo) != round_mode<MODE>(hi);
}

// One quaternion test-matrix entry in the operand format of MODE, equal to
// the FP64 value rounded once (for BF16 / FP8 a component whose FP32 value is
// within the guard band of a rounding tie is recomputed in FP64).
template <int MODE>
__device__ __forceinline__ void gauss_entry(uint32_t t, uint32_t o, uint32_t stream, uint32_t k0,
                                            uint32_t k1, float out[4]) {
  const u32x4 x = philox(t, o, stream, 0u, k0, k1);
  gauss_f32(x, out);
  if constexpr (MODE == MODE_BF16 || MODE == MODE_FP8) {
    const bool tie = near_tie<MODE>(out[0]) || near_tie<MODE>(out[1]) || near_tie<MODE>(out[2]) ||
               near_tie<MODE>(out[3]);
    if (tie) {
      double d[4];
      gauss_f64(x, d);
#pragma unroll
      for (int p = 0; p < 4; ++p) out[p] = round_mode_d<MODE>(d[p]);
    } else {
#pragma unroll
      for (int p = 0; p < 4; ++p) out[p] = round_mode<MODE>(out[p]);
    }
  }
}

__device__ __forceinline__ void gauss_entry_f64(uint32_t t, uint32_t o, uint32_t stream,
                                                uint32_t k0, uint32_t k1, double out[4]) {
  gauss_f64(philox(t, o, stream, 0u, k0, k1), out);
}

// Rademacher: counter (t >> 5, o, stream, 1); 4 bits per entry.
__device__ __forceinline__ uint32_t rademacher_nibble(uint32_t t, uint32_t o, uint32_t stream,
                                                      uint32_t k0, uint32_t k1) {
  const u32x4 x = philox(t >> 5, o, stream, 1u, k0, k1);
  const uint32_t b = t & 31u;
  const uint32_t w = b >> 3;
  const uint32_t word = w == 0 ? x.x0 : (w == 1 ? x.x1 : (w == 2 ? x.x2 : x.x3));
  return (word >> (4u * (b & 7u))) & 0xFu;
}

__device__ __forceinline__ void nibble_to_signs(uint32_t nib, float out[4]) {
#pragma unroll
  for (int p = 0; p < 4; ++p) out[p] = ((nib >> p) & 1u) ? -1.f : 1.f;
}

// Entry in the operand format of MODE (FP64 mode uses the double overload).
template <int MODE>
__device__ __forceinline__ void embed_entry(int rademacher, uint32_t t, uint32_t o, uint32_t stream,
                                            uint32_t k0, uint32_t k1, float out[4]) {
  if (rademacher) nibble_to_signs(rademacher_nibble(t, o, stream, k0, k1), out);
  else gauss_entry<MODE>(t, o, stream, k0, k1, out);
}

__device__ __forceinline__ void embed_entry_f64(int rademacher, uint32_t t, uint32_t o,
                                                uint32_t stream, uint32_t k0, uint32_t k1,
                                                double out[4]) {
  if (rademacher) {
    const uint32_t nib = rademacher_nibble(t, o, stream, k0, k1);
#pragma unroll
    for (int p = 0; p < 4; ++p) out[p] = ((nib >> p) & 1u) ? -1.0 : 1.0;
  } else {
    gauss_entry_f64(t, o, stream, k0, k1, out);
  }
}

// Value of an entry exactly as the sketch of MODE used it, widened to FP64.
__device__ __forceinline__ void embed_entry_as_used(int mode, int rademacher, uint32_t t,
                                                    uint32_t o, uint32_t stream, uint32_t k0,
                                                    uint32_t k1, double out[4]) {
  if (mode == MODE_F64) { embed_entry_f64(rademacher, t, o, stream, k0, k1, out); return; }
  float f[4];
  if (mode == MODE_F32) embed_entry<MODE_F32>(rademacher, t, o, stream, k0, k1, f);
  else if (mode == MODE_BF16) embed_entry<MODE_BF16>(rademacher, t, o, stream, k0, k1, f);
  else embed_entry<MODE_FP8>(rademacher, t, o, stream, k0, k1, f);
#pragma unroll
  for (int p = 0; p < 4; ++p) out[p] = (double)f[p];
}

// ---------------------------------------------------------------------------
// Grouped launches (see GroupRef): the problem p of this block and the
// block's linear index within that problem.
__device__ __forceinline__ void group_find(const GroupRef &g, int *p, int64_t *local) {
  const int64_t b = blockIdx.x;
  int lo = 0, hi = g.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.prefix[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  *p = lo;
  *local = b - g.prefix[lo];
}

// ---------------------------------------------------------------------------
// FP64 quaternion arithmetic (Hamilton product, Section 2).
struct qd { double w, x, y, z; };

__device__ __forceinline__ qd qzero() { return {0.0, 0.0, 0.0, 0.0}; }
__device__ __forceinline__ qd qadd(qd a, qd b) { return {a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ qd qsub(qd a, qd b) { return {a.w - b.w, a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ qd qscale(qd a, double s) { return {a.w * s, a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ qd qconj(qd a) { return {a.w, -a.x, -a.y, -a.z}; }
__device__ __forceinline__ double qnorm2(qd a) { return a.w * a.w + a.x * a.x + a.y * a.y + a.z * a.z; }
__device__ __forceinline__ qd qmul(qd a, qd b) {
  return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
          a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
          a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
          a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
// acc += a b
__device__ __forceinline__ void qfma(qd &acc, qd a, qd b) {
  acc.w = fma(a.w, b.w, fma(-a.x, b.x, fma(-a.y, b.y, fma(-a.z, b.z, acc.w))));
  acc.x = fma(a.w, b.x, fma(a.x, b.w, fma(a.y, b.z, fma(-a.z, b.y, acc.x))));
  acc.y = fma(a.w, b.y, fma(-a.x, b.z, fma(a.y, b.w, fma(a.z, b.x, acc.y))));
  acc.z = fma(a.w, b.z, fma(a.x, b.y, fma(-a.y, b.x, fma(a.z, b.w, acc.z))));
}
// acc += conj(a) b
__device__ __forceinline__ void qfma_cj(qd &acc, qd a, qd b) { qfma(acc, qconj(a), b); }

}  // namespace qsk
