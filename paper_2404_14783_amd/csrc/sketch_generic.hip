// Direct-FMA sketch kernels, Y += H Omega_J and W[:, J] += Psi H for one
// column block J (Section 4.1 sketches with the linear update of Section 4).
// They accumulate in FP64 whatever the operand format, so their only
// difference from an exact evaluation on the operand values is FP64 rounding:
// they are the FP64 sketch path and the fallback for shapes the matrix-core
// kernels do not take.
#include "qsk_device.hpp"
#include "qsk_kernels.hpp"

namespace qsk {

template <typename T> __device__ __forceinline__ float load_f(const T *p, int64_t idx);
template <> __device__ __forceinline__ float load_f<float>(const float *p, int64_t idx) { return p[idx]; }
template <> __device__ __forceinline__ float load_f<uint16_t>(const uint16_t *p, int64_t idx) {
  return __uint_as_float(((uint32_t)p[idx]) << 16);
}
template <> __device__ __forceinline__ float load_f<double>(const double *p, int64_t idx) {
  return (float)p[idx];
}
template <typename T> __device__ __forceinline__ double load_d(const T *p, int64_t idx) {
  return (double)load_f<T>(p, idx);
}
template <> __device__ __forceinline__ double load_d<double>(const double *p, int64_t idx) { return p[idx]; }

// Operand value of one data element as the sketch of MODE multiplies it.
template <int MODE, typename TIN>
__device__ __forceinline__ double operand(const TIN *p, int64_t idx, int terms) {
  if constexpr (MODE == MODE_F64) {
    return load_d<TIN>(p, idx);
  } else if constexpr (MODE == MODE_F32) {
    return (double)load_f<TIN>(p, idx);
  } else {   // BF16 split
    const float a = load_f<TIN>(p, idx);
    const float hi = bf16_rne(a);
    double s = hi;
    if (terms > 1) {
      const float r1 = a - hi;
      const float mid = bf16_rne(r1);
      s += mid;
      if (terms > 2) s += bf16_rne(r1 - mid);
    }
    return s;
  }
}

template <int MODE>
__device__ __forceinline__ void entry_d(int rad, uint32_t t, uint32_t o, uint32_t stream,
                                        uint32_t k0, uint32_t k1, double e[4]) {
  if constexpr (MODE == MODE_F64) {
    embed_entry_f64(rad, t, o, stream, k0, k1, e);
  } else {
    float f[4];
    embed_entry<MODE>(rad, t, o, stream, k0, k1, f);
#pragma unroll
    for (int p = 0; p < 4; ++p) e[p] = f[p];
  }
}

template <typename TO> __device__ __forceinline__ void add_out(TO *p, double v) { *p = (TO)((double)*p + v); }

// Y[i, j] += sum_t H[i, t] Omega[col0 + t, j]; 64 rows x 8 columns per block.
template <int MODE, int EMODE, typename TIN, typename TY>
__global__ __launch_bounds__(256) void sketch_y_generic(PlanesC<TIN> a, int64_t lda, int pure,
                                                        int64_t m, int64_t col0, int64_t ncols,
                                                        int k, TY *y, int64_t ldy, int64_t psy,
                                                        int rad, int terms, uint32_t k0, uint32_t k1,
                                                        double eta) {
  __shared__ double om[32][8][4];
  const int r = threadIdx.x & 63, c = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + r;
  const int j0 = blockIdx.y * 8;
  qd acc0 = qzero(), acc1 = qzero();
  for (int64_t t0 = 0; t0 < ncols; t0 += 32) {
    {
      const int tt = threadIdx.x >> 3, jj = threadIdx.x & 7;
      double e[4] = {0.0, 0.0, 0.0, 0.0};
      if (t0 + tt < ncols && j0 + jj < k)
        entry_d<EMODE>(rad, (uint32_t)(col0 + t0 + tt), (uint32_t)(j0 + jj), STREAM_OMEGA, k0, k1, e);
#pragma unroll
      for (int p = 0; p < 4; ++p) om[tt][jj][p] = e[p];
    }
    __syncthreads();
    if (i < m) {
      const int tmax = (int)min((int64_t)32, ncols - t0);
      for (int tt = 0; tt < tmax; ++tt) {
        const int64_t idx = i + (t0 + tt) * lda;
        qd av;
        av.w = pure ? 0.0 : operand<MODE, TIN>(a.p[0], idx, terms);
        av.x = operand<MODE, TIN>(a.p[1], idx, terms);
        av.y = operand<MODE, TIN>(a.p[2], idx, terms);
        av.z = operand<MODE, TIN>(a.p[3], idx, terms);
        const qd o0 = {om[tt][c][0], om[tt][c][1], om[tt][c][2], om[tt][c][3]};
        const qd o1 = {om[tt][c + 4][0], om[tt][c + 4][1], om[tt][c + 4][2], om[tt][c + 4][3]};
        qfma(acc0, av, o0);
        qfma(acc1, av, o1);
      }
    }
    __syncthreads();
  }
  if (i < m) {
    const int ja = j0 + c, jb = j0 + c + 4;
    if (ja < k) {
      TY *q = y + i + ja * ldy;
      add_out(q, eta * acc0.w); add_out(q + psy, eta * acc0.x); add_out(q + 2 * psy, eta * acc0.y); add_out(q + 3 * psy, eta * acc0.z);
    }
    if (jb < k) {
      TY *q = y + i + jb * ldy;
      add_out(q, eta * acc1.w); add_out(q + psy, eta * acc1.x); add_out(q + 2 * psy, eta * acc1.y); add_out(q + 3 * psy, eta * acc1.z);
    }
  }
}

// W[r, col0 + j] += sum_i Psi[r, i] H[i, j]; 64 columns x 8 rows per block.
template <int MODE, int EMODE, typename TIN, typename TW>
__global__ __launch_bounds__(256) void sketch_w_generic(PlanesC<TIN> a, int64_t lda, int pure,
                                                        int64_t m, int64_t col0, int64_t ncols,
                                                        int l, TW *w, int64_t ldw, int64_t psw,
                                                        int rad, int terms, uint32_t k0, uint32_t k1,
                                                        double eta) {
  __shared__ double ps[8][32][4];
  const int jc = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + jc;
  const int r0 = blockIdx.y * 8;
  qd acc0 = qzero(), acc1 = qzero();
  for (int64_t i0 = 0; i0 < m; i0 += 32) {
    {
      const int rr = threadIdx.x >> 5, ii = threadIdx.x & 31;
      double e[4] = {0.0, 0.0, 0.0, 0.0};
      if (i0 + ii < m && r0 + rr < l)
        entry_d<EMODE>(rad, (uint32_t)(i0 + ii), (uint32_t)(r0 + rr), STREAM_PSI, k0, k1, e);
#pragma unroll
      for (int p = 0; p < 4; ++p) ps[rr][ii][p] = e[p];
    }
    __syncthreads();
    if (j < ncols) {
      const int imax = (int)min((int64_t)32, m - i0);
      for (int ii = 0; ii < imax; ++ii) {
        const int64_t idx = (i0 + ii) + j * lda;
        qd av;
        av.w = pure ? 0.0 : operand<MODE, TIN>(a.p[0], idx, terms);
        av.x = operand<MODE, TIN>(a.p[1], idx, terms);
        av.y = operand<MODE, TIN>(a.p[2], idx, terms);
        av.z = operand<MODE, TIN>(a.p[3], idx, terms);
        const qd p0 = {ps[rg][ii][0], ps[rg][ii][1], ps[rg][ii][2], ps[rg][ii][3]};
        const qd p1 = {ps[rg + 4][ii][0], ps[rg + 4][ii][1], ps[rg + 4][ii][2], ps[rg + 4][ii][3]};
        qfma(acc0, p0, av);
        qfma(acc1, p1, av);
      }
    }
    __syncthreads();
  }
  if (j < ncols) {
    const int ra = r0 + rg, rb = r0 + rg + 4;
    if (ra < l) {
      TW *q = w + ra + (col0 + j) * ldw;
      add_out(q, eta * acc0.w); add_out(q + psw, eta * acc0.x); add_out(q + 2 * psw, eta * acc0.y); add_out(q + 3 * psw, eta * acc0.z);
    }
    if (rb < l) {
      TW *q = w + rb + (col0 + j) * ldw;
      add_out(q, eta * acc1.w); add_out(q + psw, eta * acc1.x); add_out(q + 2 * psw, eta * acc1.y); add_out(q + 3 * psw, eta * acc1.z);
    }
  }
}

// EMODE: the format of the test-matrix values (an FP64 sketch may take the
// rounded values of a low-precision one)
template <int MODE, int EMODE, typename TIN, typename TS>
static hipError_t launch_generic_t(const SketchArgs &s) {
  PlanesC<TIN> a;
  for (int p = 0; p < 4; ++p) a.p[p] = (const TIN *)s.planes[p];
  if (s.pure || !a.p[0]) a.p[0] = a.p[1];
  dim3 gy((unsigned)((s.m + 63) / 64), (unsigned)((s.k + 7) / 8));
  hipLaunchKernelGGL((sketch_y_generic<MODE, EMODE, TIN, TS>), gy, dim3(256), 0, s.stream, a, s.lda, s.pure,
                     s.m, s.col0, s.ncols, s.k, (TS *)s.y, s.ldy, s.psy, s.rad, s.terms, s.k0, s.k1, s.eta);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (s.skip_w) return hipSuccess;
  dim3 gw((unsigned)((s.ncols + 63) / 64), (unsigned)((s.l + 7) / 8));
  hipLaunchKernelGGL((sketch_w_generic<MODE, EMODE, TIN, TS>), gw, dim3(256), 0, s.stream, a, s.lda, s.pure,
                     s.m, s.col0, s.ncols, s.l, (TS *)s.w, s.ldw, s.psw, s.rad, s.terms, s.k0, s.k1, s.eta);
  return hipGetLastError();
}

template <int MODE, typename TIN, typename TS>
static hipError_t launch_generic_e(const SketchArgs &s) {
  const int em = s.emode < 0 ? MODE : s.emode;
  if constexpr (MODE == MODE_F64) {
    switch (em) {
      case MODE_F64: return launch_generic_t<MODE, MODE_F64, TIN, TS>(s);
      case MODE_F32: return launch_generic_t<MODE, MODE_F32, TIN, TS>(s);
      case MODE_BF16: return launch_generic_t<MODE, MODE_BF16, TIN, TS>(s);
      case MODE_FP8: return launch_generic_t<MODE, MODE_FP8, TIN, TS>(s);
      default: return hipErrorInvalidValue;
    }
  } else {
    if (em != MODE) return hipErrorInvalidValue;
    return launch_generic_t<MODE, MODE, TIN, TS>(s);
  }
}

hipError_t launch_sketch_generic(const SketchArgs &s) {
  switch (s.mode) {
    case MODE_F64:
      if (s.in_dtype == DT_F64) return launch_generic_e<MODE_F64, double, double>(s);
      if (s.in_dtype == DT_F32) return launch_generic_e<MODE_F64, float, double>(s);
      return launch_generic_e<MODE_F64, uint16_t, double>(s);
    case MODE_F32:
      if (s.in_dtype == DT_F32) return launch_generic_e<MODE_F32, float, float>(s);
      return launch_generic_e<MODE_F32, uint16_t, float>(s);
    case MODE_BF16:
      if (s.in_dtype == DT_F32) return launch_generic_e<MODE_BF16, float, float>(s);
      return launch_generic_e<MODE_BF16, uint16_t, float>(s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace qsk
