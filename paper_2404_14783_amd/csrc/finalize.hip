// FP64 finalize kernels for the QB stage (Alg. 4): CholeskyQR passes over the
// sketch Y (its quaternion Gram and the right-multiplication by small factors),
// Psi H with Psi regenerated, the cross product for the least-squares core
// solve, the error measurement pass, and single-workgroup drivers for the
// small dense k x k quaternion algebra (Cholesky, triangular inverse,
// products, the pseudo-QR corrections, one-sided Jacobi SVD, pseudo-SVD pair
// selection and repair).
#include "qsk_device.hpp"
#include "qsk_kernels.hpp"

namespace qsk {

template <typename T> __device__ __forceinline__ double ldv(const T *p, int64_t i) { return (double)p[i]; }

template <typename T>
__device__ __forceinline__ qd load_q(const PlanesC<T> &z, int64_t idx) {
  return {ldv(z.p[0], idx), ldv(z.p[1], idx), ldv(z.p[2], idx), ldv(z.p[3], idx)};
}

// ---------------------------------------------------------------------------
// C = Z1^* Z2 (k1 x k2) over a chunk of rows per block.z.
template <typename T1, typename T2>
__global__ __launch_bounds__(256) void crossprod_k(PlanesC<T1> z1, int64_t ld1, PlanesC<T2> z2,
                                                   int64_t ld2, int64_t rows, int64_t chunk, int k1,
                                                   int k2, double *partial, Planes<double> outp,
                                                   int64_t ldo, int planar) {
  __shared__ qd s1[32][17];
  __shared__ qd s2[32][17];
  const int tid = threadIdx.x;
  const int a = tid & 15, b = tid >> 4;
  const int a0 = blockIdx.x * 16, b0 = blockIdx.y * 16;
  const int64_t rs = (int64_t)blockIdx.z * chunk;
  const int64_t re = min(rows, rs + chunk);
  qd acc = qzero();
  for (int64_t r0 = rs; r0 < re; r0 += 32) {
    for (int e = tid; e < 512; e += 256) {
      const int rr = e & 31, cc = e >> 5;
      const int64_t row = r0 + rr;
      const int c1 = a0 + cc, c2 = b0 + cc;
      s1[rr][cc] = (row < re && c1 < k1) ? load_q(z1, row + (int64_t)c1 * ld1) : qzero();
      s2[rr][cc] = (row < re && c2 < k2) ? load_q(z2, row + (int64_t)c2 * ld2) : qzero();
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < 32; ++rr) qfma_cj(acc, s1[rr][a], s2[rr][b]);
    __syncthreads();
  }
  const int ga = a0 + a, gb = b0 + b;
  if (ga < k1 && gb < k2) {
    if (planar) {
      const int64_t o = ga + (int64_t)gb * ldo;
      outp.p[0][o] = acc.w; outp.p[1][o] = acc.x; outp.p[2][o] = acc.y; outp.p[3][o] = acc.z;
    } else {
      double *q = partial + 4 * (((int64_t)blockIdx.z * k2 + gb) * k1 + ga);
      q[0] = acc.w; q[1] = acc.x; q[2] = acc.y; q[3] = acc.z;
    }
  }
}

__global__ void reduce_chunks_k(const double *partial, int nchunks, int64_t elems, double *out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= elems) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += partial[(int64_t)c * elems + e];
  out[e] = s;
}

// AoS (r x c, ld = r) partial sums -> planar output.
__global__ void reduce_chunks_planar_k(const double *partial, int nchunks, int r, int c,
                                       Planes<double> out, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)r * c;
  if (e >= n) return;
  const int i = (int)(e % r), j = (int)(e / r);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int ch = 0; ch < nchunks; ++ch)
    for (int p = 0; p < 4; ++p) s[p] += partial[((int64_t)ch * n + e) * 4 + p];
  for (int p = 0; p < 4; ++p) out.p[p][i + (int64_t)j * ldo] = s[p];
}

template <typename T> static PlanesC<T> mkc(const void *const z[4]) {
  PlanesC<T> r;
  for (int p = 0; p < 4; ++p) r.p[p] = (const T *)z[p];
  return r;
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

hipError_t launch_crossprod(hipStream_t st, int t1, const void *const z1[4], int64_t ld1, int t2,
                            const void *const z2[4], int64_t ld2, int64_t rows, int k1, int k2,
                            double *partials, int64_t partial_elems, double *out_aos) {
  const int tiles = ((k1 + 15) / 16) * ((k2 + 15) / 16);
  const int64_t per = (int64_t)k1 * k2 * 4;
  int64_t max_chunks = partial_elems / per;
  if (max_chunks < 1) return hipErrorInvalidValue;
  const int64_t chunk = chunk_rows(rows, tiles, max_chunks);
  const int64_t nch = (rows + chunk - 1) / chunk;
  if (nch > max_chunks) return hipErrorInvalidValue;
  dim3 g((k1 + 15) / 16, (k2 + 15) / 16, (unsigned)nch);
  Planes<double> none{};
  if (t1 == 0 && t2 == 0)
    hipLaunchKernelGGL((crossprod_k<double, double>), g, dim3(256), 0, st, mkc<double>(z1), ld1,
                       mkc<double>(z2), ld2, rows, chunk, k1, k2, partials, none, 0, 0);
  else if (t1 == 1 && t2 == 1)
    hipLaunchKernelGGL((crossprod_k<float, float>), g, dim3(256), 0, st, mkc<float>(z1), ld1,
                       mkc<float>(z2), ld2, rows, chunk, k1, k2, partials, none, 0, 0);
  else if (t1 == 0 && t2 == 1)
    hipLaunchKernelGGL((crossprod_k<double, float>), g, dim3(256), 0, st, mkc<double>(z1), ld1,
                       mkc<float>(z2), ld2, rows, chunk, k1, k2, partials, none, 0, 0);
  else
    return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_chunks_k, dim3((unsigned)((per + 255) / 256)), dim3(256), 0, st,
                     partials, (int)nch, per, out_aos);
  return hipGetLastError();
}

hipError_t launch_crossprod_planar(hipStream_t st, const double *const z1[4], int64_t ld1, int t2,
                                   const void *const z2[4], int64_t ld2, int64_t rows, int k1,
                                   int k2, double *const out[4], int64_t ldo) {
  dim3 g((k1 + 15) / 16, (k2 + 15) / 16, 1);
  Planes<double> o;
  for (int p = 0; p < 4; ++p) o.p[p] = out[p];
  const void *zz1[4] = {z1[0], z1[1], z1[2], z1[3]};
  if (t2 == 1)
    hipLaunchKernelGGL((crossprod_k<double, float>), g, dim3(256), 0, st, mkc<double>(zz1), ld1,
                       mkc<float>(z2), ld2, rows, rows, k1, k2, (double *)nullptr, o, ldo, 1);
  else
    hipLaunchKernelGGL((crossprod_k<double, double>), g, dim3(256), 0, st, mkc<double>(zz1), ld1,
                       mkc<double>(z2), ld2, rows, rows, k1, k2, (double *)nullptr, o, ldo, 1);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Out = Z C: one row per thread, 16 output columns per block.y, C staged in
// LDS 64 rows at a time.
template <typename TZ>
__global__ __launch_bounds__(256) void apply_k(PlanesC<TZ> z, int64_t ldz, int64_t rows, int k,
                                               const double *__restrict__ c, int kc,
                                               Planes<double> out, int64_t ldo) {
  __shared__ qd sc[64][16];
  const int tid = threadIdx.x;
  const int b0 = blockIdx.y * 16;
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
  qd acc[16];
#pragma unroll
  for (int b = 0; b < 16; ++b) acc[b] = qzero();
  for (int a0 = 0; a0 < k; a0 += 64) {
    for (int e = tid; e < 64 * 16; e += 256) {
      const int aa = e >> 4, bb = e & 15;
      const int ga = a0 + aa, gb = b0 + bb;
      if (ga < k && gb < kc) {
        const double *q = c + 4 * ((int64_t)ga + (int64_t)gb * k);
        sc[aa][bb] = {q[0], q[1], q[2], q[3]};
      } else {
        sc[aa][bb] = qzero();
      }
    }
    __syncthreads();
    if (i < rows) {
      const int amax = min(64, k - a0);
      for (int aa = 0; aa < amax; ++aa) {
        const qd zi = load_q(z, i + (int64_t)(a0 + aa) * ldz);
#pragma unroll
        for (int b = 0; b < 16; ++b) qfma(acc[b], zi, sc[aa][b]);
      }
    }
    __syncthreads();
  }
  if (i < rows) {
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      const int gb = b0 + b;
      if (gb < kc) {
        const int64_t o = i + (int64_t)gb * ldo;
        out.p[0][o] = acc[b].w; out.p[1][o] = acc[b].x; out.p[2][o] = acc[b].y; out.p[3][o] = acc[b].z;
      }
    }
  }
}

hipError_t launch_apply(hipStream_t st, int tz, const void *const z[4], int64_t ldz, int64_t rows,
                        int k, const double *c_aos, int kc, double *const out[4], int64_t ldo) {
  dim3 g((unsigned)((rows + 255) / 256), (kc + 15) / 16);
  Planes<double> o;
  for (int p = 0; p < 4; ++p) o.p[p] = out[p];
  if (tz == 0)
    hipLaunchKernelGGL((apply_k<double>), g, dim3(256), 0, st, mkc<double>(z), ldz, rows, k, c_aos,
                       kc, o, ldo);
  else
    hipLaunchKernelGGL((apply_k<float>), g, dim3(256), 0, st, mkc<float>(z), ldz, rows, k, c_aos,
                       kc, o, ldo);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// P = Psi H, Psi (l x m) regenerated as the sketch of `mode` used it.
__global__ __launch_bounds__(256) void psi_apply_k(int mode, int rad, uint32_t k0, uint32_t k1,
                                                   int l, int64_t m, PlanesC<double> h,
                                                   int64_t ldh, int k, int64_t chunk,
                                                   double *partial) {
  __shared__ qd sp[16][33];
  __shared__ qd sh[32][17];
  const int tid = threadIdx.x;
  const int rr = tid & 15, bb = tid >> 4;
  const int r0 = blockIdx.x * 16, b0 = blockIdx.y * 16;
  const int64_t is = (int64_t)blockIdx.z * chunk;
  const int64_t ie = min(m, is + chunk);
  qd acc = qzero();
  for (int64_t i0 = is; i0 < ie; i0 += 32) {
    for (int e = tid; e < 512; e += 256) {
      const int ii = e & 31, q = e >> 5;
      const int64_t gi = i0 + ii;
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      if (gi < ie && r0 + q < l)
        embed_entry_as_used(mode, rad, (uint32_t)gi, (uint32_t)(r0 + q), STREAM_PSI, k0, k1, v);
      sp[q][ii] = {v[0], v[1], v[2], v[3]};
      sh[ii][q] = (gi < ie && b0 + q < k) ? load_q(h, gi + (int64_t)(b0 + q) * ldh) : qzero();
    }
    __syncthreads();
#pragma unroll 8
    for (int ii = 0; ii < 32; ++ii) qfma(acc, sp[rr][ii], sh[ii][bb]);
    __syncthreads();
  }
  const int gr = r0 + rr, gb = b0 + bb;
  if (gr < l && gb < k) {
    double *q = partial + 4 * (((int64_t)blockIdx.z * k + gb) * l + gr);
    q[0] = acc.w; q[1] = acc.x; q[2] = acc.y; q[3] = acc.z;
  }
}

hipError_t launch_psi_apply(hipStream_t st, int mode, int rad, uint32_t k0, uint32_t k1, int l,
                            int64_t m, const double *const h[4], int64_t ldh, int k,
                            double *partials, int64_t partial_elems, double *const p[4],
                            int64_t ldp) {
  const int tiles = ((l + 15) / 16) * ((k + 15) / 16);
  const int64_t per = (int64_t)l * k * 4;
  const int64_t max_chunks = partial_elems / per;
  if (max_chunks < 1) return hipErrorInvalidValue;
  const int64_t chunk = chunk_rows(m, tiles, max_chunks);
  const int64_t nch = (m + chunk - 1) / chunk;
  if (nch > max_chunks) return hipErrorInvalidValue;
  PlanesC<double> hh;
  for (int q = 0; q < 4; ++q) hh.p[q] = h[q];
  dim3 g((l + 15) / 16, (k + 15) / 16, (unsigned)nch);
  hipLaunchKernelGGL(psi_apply_k, g, dim3(256), 0, st, mode, rad, k0, k1, l, m, hh, ldh, k, chunk,
                     partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  Planes<double> o;
  for (int q = 0; q < 4; ++q) o.p[q] = p[q];
  const int64_t n = (int64_t)l * k;
  hipLaunchKernelGGL(reduce_chunks_planar_k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     partials, (int)nch, l, k, o, ldp);
  return hipGetLastError();
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

// ---------------------------------------------------------------------------
// Error pass: 64 x 64 tiles of H X, accumulated against A in FP64.
template <typename T> __device__ __forceinline__ double lda_val(const T *p, int64_t i);
template <> __device__ __forceinline__ double lda_val<double>(const double *p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ double lda_val<float>(const float *p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ double lda_val<uint16_t>(const uint16_t *p, int64_t i) {
  return (double)__uint_as_float(((uint32_t)p[i]) << 16);
}

template <typename TIN>
__global__ __launch_bounds__(256) void error_k(PlanesC<TIN> a, int64_t lda, int pure, int64_t m,
                                               int64_t n, PlanesC<double> q, int64_t ldq,
                                               PlanesC<double> x, int64_t ldx, int k, double *acc) {
  __shared__ qd sq[64][9];
  __shared__ qd sx[8][65];
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;      // 4 x 4 outputs per thread
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
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

hipError_t launch_error(hipStream_t st, int tin, const void *const a[4], int64_t lda, int pure,
                        int64_t m, int64_t n, const double *const q[4], int64_t ldq,
                        const double *const x[4], int64_t ldx, int k, double *acc) {
  PlanesC<double> qq, xx;
  for (int p = 0; p < 4; ++p) { qq.p[p] = q[p]; xx.p[p] = x[p]; }
  const void *aa[4] = {a[0] ? a[0] : a[1], a[1], a[2], a[3]};
  dim3 g((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64));
  if (tin == DT_F64)
    hipLaunchKernelGGL((error_k<double>), g, dim3(256), 0, st, mkc<double>(aa), lda, pure, m, n, qq,
                       ldq, xx, ldx, k, acc);
  else if (tin == DT_F32)
    hipLaunchKernelGGL((error_k<float>), g, dim3(256), 0, st, mkc<float>(aa), lda, pure, m, n, qq,
                       ldq, xx, ldx, k, acc);
  else
    hipLaunchKernelGGL((error_k<uint16_t>), g, dim3(256), 0, st, mkc<uint16_t>(aa), lda, pure, m,
                       n, qq, ldq, xx, ldx, k, acc);
  return hipGetLastError();
}

// ===========================================================================
// Single-workgroup small dense algebra on k x k AoS quaternion matrices in
// global memory (one CU; all waves of the block share its L1, so a
// __syncthreads() makes a block's global writes visible to the block).

__device__ __forceinline__ qd gq(const double *a, int i, int j, int ld) {
  const double *p = a + 4 * ((int64_t)i + (int64_t)j * ld);
  return {p[0], p[1], p[2], p[3]};
}
__device__ __forceinline__ void sq_(double *a, int i, int j, int ld, qd v) {
  double *p = a + 4 * ((int64_t)i + (int64_t)j * ld);
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

// Upper Cholesky G' = R^* R; returns in shared `fail` whether a pivot fell
// below tol * max diagonal.
__device__ void sm_chol(const double *g, double *r, int k, int complex_only, double shift,
                        double tol, int *fail, double *minp, double *trace) {
  __shared__ double s_piv;
  __shared__ double s_maxd;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e % k, j = e / k;
    qd v = qzero();
    if (i <= j) {
      v = gq(g, i, j, k);
      if (complex_only) { v.y = 0.0; v.z = 0.0; }
      if (i == j) { v.x = 0.0; v.y = 0.0; v.z = 0.0; v.w += shift; }
    }
    sq_(r, i, j, k, v);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double md = 0.0, tr = 0.0;
    for (int i = 0; i < k; ++i) { const double d = r[4 * (i + (int64_t)i * k)]; md = fmax(md, d); tr += d; }
    s_maxd = md;
    *trace = tr;
    *fail = 0;
    *minp = 1.0;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (threadIdx.x == 0) {
      const double d = r[4 * (j + (int64_t)j * k)];
      const double rel = s_maxd > 0.0 ? d / s_maxd : 0.0;
      if (rel < *minp) *minp = rel;
      if (!(rel > tol)) *fail = 1;
      s_piv = sqrt(fmax(d, 0.0));
      r[4 * (j + (int64_t)j * k)] = s_piv;
    }
    __syncthreads();
    if (*fail) return;
    const double inv = 1.0 / s_piv;
    for (int c = j + 1 + threadIdx.x; c < k; c += blockDim.x) sq_(r, j, c, k, qscale(gq(r, j, c, k), inv));
    __syncthreads();
    const int nrem = k - j - 1;
    for (int e = threadIdx.x; e < nrem * nrem; e += blockDim.x) {
      const int aa = e % nrem, cc = e / nrem;
      if (aa <= cc) {
        const int ga = j + 1 + aa, gc = j + 1 + cc;
        qd v = gq(r, ga, gc, k);
        const qd ra = qconj(gq(r, j, ga, k)), rc = gq(r, j, gc, k);
        const qd prod = qmul(ra, rc);
        v = qsub(v, prod);
        sq_(r, ga, gc, k, v);
      }
    }
    __syncthreads();
  }
}

// T = R^{-1} for upper triangular R with real positive diagonal.
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
__global__ __launch_bounds__(1024) void chol_inv_kernel(const double *g, int k, int complex_only,
                                                        double shift, double tol, double *r,
                                                        double *t, SmallStatus *status) {
  __shared__ int fail;
  __shared__ double minp, trace;
  sm_chol(g, r, k, complex_only, shift, tol, &fail, &minp, &trace);
  __syncthreads();
  if (threadIdx.x == 0) {
    status->fail = fail;
    status->min_pivot2 = minp;
    status->trace = trace;
  }
  if (!fail) sm_triinv(r, t, k);
}

hipError_t launch_chol_inv(hipStream_t st, const double *g, int k, int complex_only, double shift,
                           double tol, double *r, double *t, SmallStatus *status) {
  hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(1024), 0, st, g, k, complex_only, shift, tol, r,
                     t, status);
  return hipGetLastError();
}

__global__ __launch_bounds__(1024) void small_gemm_kernel(int k, const double *a, int opa,
                                                          const double *b, int opb, double *c) {
  sm_gemm(k, a, opa, b, opb, c);
}

hipError_t launch_small_gemm(hipStream_t st, int k, const double *a, int opa, const double *b,
                             int opb, double *c) {
  hipLaunchKernelGGL(small_gemm_kernel, dim3(1), dim3(1024), 0, st, k, a, opa, b, opb, c);
  return hipGetLastError();
}

__global__ __launch_bounds__(1024) void identity_kernel(int k, double *c) { sm_identity(c, k); }

hipError_t launch_identity(hipStream_t st, int k, double *c) {
  hipLaunchKernelGGL(identity_kernel, dim3(1), dim3(1024), 0, st, k, c);
  return hipGetLastError();
}

// pseudo-QR correction steps in the k x k space.  With H_j = H0 C_j and
// G_j = H_j^* H_j, one step (eq. CondNumReductionIter) is
//   H_{j+1} = (1 - eps) H_j + eps (H_j^dagger)^* = H_j M_j,
//   M_j = (1 - eps) I + eps G_j^{-1}    ((H^dagger)^* = H G^{-1}),
// so C_{j+1} = C_j M_j and G_{j+1} = M_j^* G_j M_j.  eps comes from n_power
// normalised power iterates v <- G_j^{-1} v started from Philox stream 2,
// eps = (v^* G_j^{-1} v)^{-1/2}.
__global__ __launch_bounds__(1024) void pqr_corrections_kernel(int k, const double *g0, int n_corr,
                                                               int n_power, uint32_t k0,
                                                               uint32_t k1, double *c,
                                                               double *work, SmallStatus *status) {
  __shared__ int fail;
  __shared__ double minp, trace, s_eps, s_nrm;
  const int64_t kk = (int64_t)k * k * 4;
  double *G = work, *R = work + kk, *T = work + 2 * kk, *Gi = work + 3 * kk, *M = work + 4 * kk,
         *tmp = work + 5 * kk, *v = work + 6 * kk, *w = v + 4 * k;
  sm_copy(G, g0, (int)kk);
  sm_identity(c, k);
  if (threadIdx.x == 0) { status->n_eps = 0; status->flags = 0; }
  for (int j = 0; j < n_corr; ++j) {
    sm_chol(G, R, k, 0, 0.0, 1e-13, &fail, &minp, &trace);
    __syncthreads();
    if (fail) {
      if (threadIdx.x == 0) status->flags |= 2;        // QSK_FLAG_RANK_DEFICIENT
      break;
    }
    sm_triinv(R, T, k);
    sm_gemm(k, T, 0, T, 1, Gi);                        // G^{-1} = T T^*
    // start vector
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
      double e[4];
      gauss_entry_f64((uint32_t)i, (uint32_t)j, STREAM_POWER, k0, k1, e);
      v[4 * i] = e[0]; v[4 * i + 1] = e[1]; v[4 * i + 2] = e[2]; v[4 * i + 3] = e[3];
    }
    __syncthreads();
    for (int it = 0; it <= n_power; ++it) {
      // normalise v
      if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < 4 * k; ++i) s += v[i] * v[i];
        s_nrm = sqrt(s);
      }
      __syncthreads();
      for (int i = threadIdx.x; i < 4 * k; i += blockDim.x) v[i] /= s_nrm;
      __syncthreads();
      // w = G^{-1} v
      for (int i = threadIdx.x; i < k; i += blockDim.x) {
        qd s = qzero();
        for (int t2 = 0; t2 < k; ++t2) qfma(s, gq(Gi, i, t2, k), {v[4 * t2], v[4 * t2 + 1], v[4 * t2 + 2], v[4 * t2 + 3]});
        w[4 * i] = s.w; w[4 * i + 1] = s.x; w[4 * i + 2] = s.y; w[4 * i + 3] = s.z;
      }
      __syncthreads();
      if (it == n_power) {
        if (threadIdx.x == 0) {
          double rho = 0.0;
          for (int i = 0; i < 4 * k; ++i) rho += v[i] * w[i];     // Re(v^* w)
          s_eps = 1.0 / sqrt(rho);
        }
        __syncthreads();
      } else {
        for (int i = threadIdx.x; i < 4 * k; i += blockDim.x) v[i] = w[i];
        __syncthreads();
      }
    }
    const double eps = s_eps;
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
      const int i = e % k, jj = e / k;
      qd gv = qscale(gq(Gi, i, jj, k), eps);
      if (i == jj) gv.w += 1.0 - eps;
      sq_(M, i, jj, k, gv);
    }
    __syncthreads();
    sm_gemm(k, c, 0, M, 0, tmp);                       // C <- C M
    sm_copy(c, tmp, (int)kk);
    sm_gemm(k, G, 0, M, 0, tmp);                       // G <- M^* (G M)
    sm_gemm(k, M, 1, tmp, 0, G);
    if (threadIdx.x == 0) {
      status->eps[status->n_eps] = eps;
      status->n_eps += 1;
    }
    __syncthreads();
  }
}

hipError_t launch_pqr_corrections(hipStream_t st, int k, const double *g0, int n_corr, int n_power,
                                  uint32_t k0, uint32_t k1, double *c, double *work,
                                  SmallStatus *status) {
  hipLaunchKernelGGL(pqr_corrections_kernel, dim3(1), dim3(1024), 0, st, k, g0, n_corr, n_power, k0,
                     k1, c, work, status);
  return hipGetLastError();
}

// pseudo-SVD (Alg. 3) on R_Y, with Y = Q_Y R_Y and Q_Y orthonormal: the
// complex SVD of chi_Y is chi_{Q_Y} times the SVD of chi_{R_Y}, which the
// quaternion one-sided Jacobi returns with every singular value paired.
// Pair rule: pair i is good iff sigma_i > TAU_S sigma_0 and it is separated
// from its neighbours by more than tau_p sigma_0 (tau_p = 64 * 2k * 2^-53).
// Bad part: B = [u_b..., -u_b j ...] (the two members of each bad pair),
// B diag(f) with f from Philox stream 3, Jacobi SVD, one column per pair of
// the leading 2t.  Output C (k x k): H = Q_Y C = [H_g, H_b~].
__global__ __launch_bounds__(1024) void psvd_select_kernel(int k, const double *ry, uint32_t k0,
                                                           uint32_t k1, double *c, double *work,
                                                           SmallStatus *status) {
  __shared__ int order[512];
  __shared__ double sig[512];
  __shared__ int good[256];
  __shared__ int n_good, n_bad;
  const int64_t kk = (int64_t)k * k * 4;
  double *A = work, *U = work + kk, *B = work + 2 * kk, *UB = work + 2 * kk + 2 * kk;
  sm_copy(A, ry, (int)kk);
  sm_jacobi(A, k, k, k, 60, 1e-15);
  __syncthreads();
  sm_sorted_columns(A, k, k, k, sig, order, U, k);
  if (threadIdx.x == 0) {
    const double s0 = sig[order[0]];
    const double tau_p = 64.0 * 2.0 * k * 0x1p-53;
    int ng = 0;
    for (int i = 0; i < k; ++i) {
      const double si = sig[order[i]];
      bool ok = si > 1e-13 * s0;
      if (ok && i > 0) ok = (sig[order[i - 1]] - si) > tau_p * s0;
      if (ok && i < k - 1) ok = (si - sig[order[i + 1]]) > tau_p * s0;
      good[i] = ok ? 1 : 0;
      ng += ok ? 1 : 0;
    }
    n_good = ng;
    n_bad = k - ng;
    status->t_bad = k - ng;
    status->good_count = ng;
    if (k - ng > 0) status->flags |= 8;
  }
  __syncthreads();
  // good columns first
  if (threadIdx.x == 0) {
    int g = 0, b = 0;
    for (int i = 0; i < k; ++i) {
      if (good[i]) order[i] = g++;
      else order[i] = -(1 + b++);
    }
  }
  __syncthreads();
  const int t = n_bad;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e % k, j = e / k;
    const int dst = order[j];
    const qd uv = gq(U, i, j, k);
    if (dst >= 0) {
      sq_(c, i, dst, k, uv);
    } else {
      const int bi = -dst - 1;
      double f1[4], f2[4];
      (void)f2;
      // f_j = 1 + u_j, u_j = (x0 + 1/2) 2^-32 from counter (j, 0, 3, 0)
      const u32x4 xa = philox((uint32_t)bi, 0u, STREAM_DIAGF, 0u, k0, k1);
      const u32x4 xb = philox((uint32_t)(t + bi), 0u, STREAM_DIAGF, 0u, k0, k1);
      f1[0] = 1.0 + ((double)xa.x0 + 0.5) * 0x1p-32;
      f2[0] = 1.0 + ((double)xb.x0 + 0.5) * 0x1p-32;
      // first member u, second member -u j (the partner of u's compact
      // representation, J conj(u_c), is the compact representation of -u j)
      sq_(B, i, bi, k, qscale(uv, f1[0]));
      const qd uj = qmul(uv, {0.0, 0.0, 1.0, 0.0});
      sq_(B, i, t + bi, k, qscale(uj, -f2[0]));
    }
  }
  __syncthreads();
  if (t > 0) {
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

hipError_t launch_psvd_select(hipStream_t st, int k, const double *ry, uint32_t k0, uint32_t k1,
                              double *c, double *work, SmallStatus *status) {
  hipLaunchKernelGGL(psvd_select_kernel, dim3(1), dim3(1024), 0, st, k, ry, k0, k1, c, work, status);
  return hipGetLastError();
}

// Minimum-norm least squares for a rank-deficient P (l x k, planar):
// one-sided Jacobi on [P; I] (inner products over the P rows only) gives
// P V = B with orthogonal columns and V accumulated; with sigma_i = ||b_i||,
// P^dagger = V diag(1/sigma_i^2) B^* over sigma_i > tol sigma_max, so
// S^* = (P^dagger)^* = B diag(w) V^*, written planar (l x k).
__global__ __launch_bounds__(1024) void pinv_sstar_kernel(int l, int k, PlanesC<double> p,
                                                          int64_t ldp, double tol, double *work,
                                                          Planes<double> out, int64_t ldo) {
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

hipError_t launch_pinv_sstar(hipStream_t st, int l, int k, const double *const p[4], int64_t ldp,
                             double tol, double *work, double *const out[4], int64_t ldo) {
  PlanesC<double> pp;
  Planes<double> oo;
  for (int q = 0; q < 4; ++q) { pp.p[q] = p[q]; oo.p[q] = out[q]; }
  hipLaunchKernelGGL(pinv_sstar_kernel, dim3(1), dim3(1024), 0, st, l, k, pp, ldp, tol, work, oo, ldo);
  return hipGetLastError();
}

// kappa of H = Z F from G_Z = Z^* Z: G_H = F^* G_Z F; R = chol(G_H);
// singular values of R (Jacobi) are those of H.  which: 0 -> status->kappa,
// 1 -> status->kappa_initial.  Also the orthonormality defect max|G_H - I|.
__global__ __launch_bounds__(1024) void kappa_kernel(int k, const double *gz, const double *f,
                                                     double *work, int which, SmallStatus *status) {
  __shared__ int fail;
  __shared__ double minp, trace;
  __shared__ int order[512];
  __shared__ double sig[512];
  __shared__ double s_def;
  const int64_t kk = (int64_t)k * k * 4;
  double *tmp = work, *GH = work + kk, *R = work + 2 * kk, *U = work + 3 * kk;
  sm_gemm(k, gz, 0, f, 0, tmp);
  sm_gemm(k, f, 1, tmp, 0, GH);
  if (threadIdx.x == 0) {
    double d = 0.0;
    for (int e = 0; e < k * k; ++e) {
      const int i = e % k, j = e / k;
      qd v = gq(GH, i, j, k);
      if (i == j) v.w -= 1.0;
      d = fmax(d, sqrt(qnorm2(v)));
    }
    s_def = d;
  }
  sm_chol(GH, R, k, 0, 0.0, 1e-300, &fail, &minp, &trace);
  __syncthreads();
  double kap = INFINITY;
  if (!fail) {
    sm_jacobi(R, k, k, k, 60, 1e-15);
    __syncthreads();
    sm_sorted_columns(R, k, k, k, sig, order, U, k);
    const double smax = sig[order[0]], smin = sig[order[k - 1]];
    kap = smin > 0.0 ? smax / smin : INFINITY;
  }
  if (threadIdx.x == 0) {
    if (which == 0) { status->kappa = kap; status->orth_defect = s_def; }
    else status->kappa_initial = kap;
  }
}

hipError_t launch_kappa(hipStream_t st, int k, const double *gz, const double *f, double *work,
                        int which, SmallStatus *status) {
  hipLaunchKernelGGL(kappa_kernel, dim3(1), dim3(1024), 0, st, k, gz, f, work, which, status);
  return hipGetLastError();
}

}  // namespace qsk
