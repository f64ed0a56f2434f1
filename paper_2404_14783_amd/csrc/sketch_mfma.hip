// Matrix-core (MFMA) sketch kernels for gfx950.
//
// One column-block update J adds, for each output plane p,
//   Y_p      += sum_q A_q[:, J] R_qp(Omega_J)      (Y = A Omega, Section 4.1)
//   W_p[:,J] += sum_q S_pq(Psi)  A_q[:, J]          (W = Psi A)
// where R(Omega) and S(Psi) are the signed plane permutations of the
// Hamilton product (the real representation of Appendix B.1):
//   R: row q=w (Ow, Ox, Oy, Oz), q=x (-Ox, Ow, -Oz, Oy), q=y (-Oy, Oz, Ow, -Ox), q=z (-Oz, -Oy, Ox, Ow)
//   S: row p=w (Pw, -Px, -Py, -Pz), p=x (Px, Pw, -Pz, Py), p=y (Py, Pz, Pw, -Px), p=z (Pz, -Py, Px, Pw)
// Every (p, q) pair is one 16 x 16 matrix-core product per tile; the four
// planes of a fragment of A and of the test matrix feed 16 products.
//
// Operands: BF16 (v_mfma_f32_16x16x32_bf16, the data split into 1-3 bf16
// terms) or FP32 (v_mfma_f32_16x16x4_f32); FP32 accumulation either way.  The
// K order inside a 32-wide step is permuted so that every lane holds 8
// consecutive contraction indices: lane group g = lane / 16 owns indices
// 8g .. 8g + 7, which keeps both the A-column reads (W) and the staged test
// matrix reads contiguous.
//
// The test-matrix slices this update needs (Omega_J, Psi) are regenerated
// from the Philox stream into a transient staging buffer by gen_stage_kernel,
// already rounded to the operand format, then read by the GEMMs.
#include <type_traits>

#include "qsk_device.hpp"
#include "qsk_kernels.hpp"

namespace qsk {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(4))) float floatx4;

enum : int { OP_BF16 = 0, OP_F32 = 1 };

// ---------------------------------------------------------------------------
// Staging of the test matrices.  Layout [plane][o][t] with t (the contraction
// index) fastest; entries outside (o < n_o, t < n_t) are zero.
template <int MODE, typename OPT>
__global__ __launch_bounds__(256) void gen_stage_kernel(OPT *dst, int n_o, int o_pad, int64_t t0,
                                                        int64_t n_t, int64_t t_pad, uint32_t stream,
                                                        int rad, uint32_t k0, uint32_t k1) {
  const int64_t total = (int64_t)o_pad * t_pad;
  const int64_t ps = total;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e % t_pad;
    const int o = (int)(e / t_pad);
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (o < n_o && t < n_t) embed_entry<MODE>(rad, (uint32_t)(t0 + t), (uint32_t)o, stream, k0, k1, v);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      if constexpr (sizeof(OPT) == 2) {
        dst[p * ps + e] = (OPT)(__float_as_uint(v[p]) >> 16);   // exact: v is a bf16 value
      } else {
        dst[p * ps + e] = v[p];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Fragments.
struct FragB { uint32_t v[4]; };          // 8 bf16
struct FragF { float v[8]; };             // 8 fp32

__device__ __forceinline__ FragB negB(const FragB &a) {
  FragB r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r.v[i] = a.v[i] ^ 0x80008000u;
  return r;
}
__device__ __forceinline__ FragF negF(const FragF &a) {
  FragF r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r.v[i] = -a.v[i];
  return r;
}

__device__ __forceinline__ floatx4 mma(const FragB &a, const FragB &b, floatx4 c) {
  bf16x8_t av, bv;
  __builtin_memcpy(&av, a.v, 16);
  __builtin_memcpy(&bv, b.v, 16);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mma(const FragF &a, const FragF &b, floatx4 c) {
#pragma unroll
  for (int s = 0; s < 8; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[s], b.v[s], c, 0, 0, 0);
  return c;
}

// Split 8 fp32 data values into TERMS bf16 fragments (hi, mid, lo).
template <int TERMS>
__device__ __forceinline__ void split_terms(const float (&x)[8], FragB (&out)[3]) {
  float r[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = x[i];
#pragma unroll
  for (int tm = 0; tm < 3; ++tm) {
    if (tm < TERMS) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float a0 = bf16_rne(r[2 * i]), a1 = bf16_rne(r[2 * i + 1]);
        out[tm].v[i] = (__float_as_uint(a0) >> 16) | (__float_as_uint(a1) & 0xFFFF0000u);
        r[2 * i] -= a0;
        r[2 * i + 1] -= a1;
      }
    }
  }
}

template <typename TIN> __device__ __forceinline__ float ldin(const TIN *p, int64_t i);
template <> __device__ __forceinline__ float ldin<float>(const float *p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ float ldin<uint16_t>(const uint16_t *p, int64_t i) {
  return __uint_as_float(((uint32_t)p[i]) << 16);
}

// Signed plane selection of R(Omega) (Y) and S(Psi) (W): index into
// {+w, +x, +y, +z, -x, -y, -z} = {0, 1, 2, 3, 4, 5, 6}.  Used inside fully
// unrolled loops so that every index is a compile-time constant.
__device__ constexpr int rsel(int q, int p) {      // R(Omega)[q][p]
  constexpr int t[4][4] = {{0, 1, 2, 3}, {4, 0, 6, 2}, {5, 3, 0, 4}, {6, 5, 1, 0}};
  return t[q][p];
}
__device__ constexpr int ssel(int p, int q) {      // S(Psi)[p][q]
  constexpr int t[4][4] = {{0, 4, 5, 6}, {1, 0, 6, 2}, {2, 3, 0, 4}, {3, 5, 1, 0}};
  return t[p][q];
}

// ---------------------------------------------------------------------------
// W kernel.  Block = 4 waves; blockIdx.x -> 64 columns of the update block
// (16 per wave), blockIdx.y -> NMT row tiles of W (16 rows each), blockIdx.z
// -> a chunk of the rows of A (split K).  Psi's tile is staged in LDS; each
// wave reads its own A fragments straight from HBM (8 contiguous rows per
// lane).
struct WArgs {
  const void *a[4];
  int64_t lda, m, ncols, col0;
  const void *psi;            // staged [4][LP][MP]
  int LP;
  int64_t MP;
  int l, terms, pure, S;
  int64_t kchunk;
  float *w;
  int64_t ldw, psw;
  float *part;                // [S][4][ncols][LP]
};

template <int OP, typename TIN, int NMT, int TERMS>
__global__ __launch_bounds__(256) void w_mfma_kernel(WArgs a) {
  using OPT = typename std::conditional<OP == OP_BF16, uint16_t, float>::type;
  using Frag = typename std::conditional<OP == OP_BF16, FragB, FragF>::type;
  constexpr int LDK = 32 + (OP == OP_BF16 ? 8 : 4);        // padded K stride in LDS
  __shared__ OPT s_psi[4][NMT * 16][LDK];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int64_t j = (int64_t)blockIdx.x * 64 + wave * 16 + c16;
  const int rbase = blockIdx.y * NMT * 16;
  const int64_t ib = (int64_t)blockIdx.z * a.kchunk;
  const int64_t ie = min(a.m, ib + a.kchunk);
  const OPT *psi = (const OPT *)a.psi;
  const int64_t pps = (int64_t)a.LP * a.MP;
  const TIN *ap[4] = {(const TIN *)a.a[0], (const TIN *)a.a[1], (const TIN *)a.a[2], (const TIN *)a.a[3]};
  const bool jok = j < a.ncols;

  floatx4 acc[NMT][4];
#pragma unroll
  for (int r = 0; r < NMT; ++r)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[r][p] = {0.f, 0.f, 0.f, 0.f};

  for (int64_t i0 = ib; i0 < ie; i0 += 32) {
    // stage Psi[rbase .. rbase + 16 NMT, i0 .. i0 + 32) for the four planes
    constexpr int EPV = 16 / sizeof(OPT);                  // elements per 16-byte vector
    constexpr int VPR = 32 / EPV;                          // vectors per row
    for (int e = tid; e < 4 * NMT * 16 * VPR; e += 256) {
      const int v = e % VPR, rr = (e / VPR) % (NMT * 16), pl = e / (VPR * NMT * 16);
      const uint4 val = *(const uint4 *)(psi + pl * pps + (int64_t)(rbase + rr) * a.MP + i0 + v * EPV);
      *(uint4 *)&s_psi[pl][rr][v * EPV] = val;
    }
    // this wave's A fragments: rows i0 + 8g .. +7 of column j, four planes
    float x[4][8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int64_t i = i0 + 8 * g + s;
        x[q][s] = (jok && i < ie && !(q == 0 && a.pure)) ? ldin<TIN>(ap[q], i + j * a.lda) : 0.f;
      }
    }
    __syncthreads();
    Frag af[4][3];
    if constexpr (OP == OP_BF16) {
#pragma unroll
      for (int q = 0; q < 4; ++q) split_terms<TERMS>(x[q], af[q]);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int s = 0; s < 8; ++s) af[q][0].v[s] = x[q][s];
    }
#pragma unroll
    for (int rt = 0; rt < NMT; ++rt) {
      Frag pf[7];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const OPT *src = &s_psi[s][rt * 16 + c16][8 * g];
        if constexpr (OP == OP_BF16) {
          const uint4 u = *(const uint4 *)src;
          pf[s].v[0] = u.x; pf[s].v[1] = u.y; pf[s].v[2] = u.z; pf[s].v[3] = u.w;
        } else {
#pragma unroll
          for (int t = 0; t < 8; ++t) pf[s].v[t] = src[t];
        }
      }
      if constexpr (OP == OP_BF16) { pf[4] = negB(pf[1]); pf[5] = negB(pf[2]); pf[6] = negB(pf[3]); }
      else { pf[4] = negF(pf[1]); pf[5] = negF(pf[2]); pf[6] = negF(pf[3]); }
#pragma unroll
      for (int p = 0; p < 4; ++p) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (q == 0 && a.pure) continue;
          const Frag &ps = pf[ssel(p, q)];
#pragma unroll
          for (int tm = 0; tm < TERMS; ++tm) acc[rt][p] = mma(ps, af[q][tm], acc[rt][p]);
        }
      }
    }
    __syncthreads();
  }
  // epilogue: lane holds column j, rows rbase + rt*16 + 4g + (0..3)
  if (!jok) return;
#pragma unroll
  for (int rt = 0; rt < NMT; ++rt) {
    const int r0 = rbase + rt * 16 + 4 * g;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      if (a.S == 1) {
        float *dst = a.w + p * a.psw + (a.col0 + j) * a.ldw;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (r0 + t < a.l) dst[r0 + t] += acc[rt][p][t];
      } else {
        float *dst = a.part + (((int64_t)blockIdx.z * 4 + p) * a.ncols + j) * a.LP + r0;
        *(floatx4 *)dst = acc[rt][p];
      }
    }
  }
}

__global__ void w_reduce_kernel(const float *part, int S, int LP, int64_t ncols, int l, int64_t col0,
                                float *w, int64_t ldw, int64_t psw) {
  const int64_t total = 4 * ncols * (int64_t)l;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % l);
    const int64_t jp = e / l;
    const int64_t j = jp % ncols;
    const int p = (int)(jp / ncols);
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += part[(((int64_t)z * 4 + p) * ncols + j) * LP + r];
    w[p * psw + (col0 + j) * ldw + r] += s;
  }
}

// ---------------------------------------------------------------------------
// Y kernel.  Block = WAVES waves covering 16 WAVES rows of A; wave w owns row
// tile w and NJ column tiles of Y (16 columns each) for all four planes;
// blockIdx.y selects the group of NJ column tiles.  The A tile is staged in
// LDS in the operand format (transposed so each lane reads 8 consecutive
// columns of A); Omega fragments come from the staging buffer.
struct YArgs {
  const void *a[4];
  int64_t lda, m, ncols;
  const void *om;             // staged [4][KP][NP]
  int KP;
  int64_t NP;
  int k, terms, pure;
  float *y;
  int64_t ldy, psy;
};

template <int OP, typename TIN, int NJ, int WAVES, int TERMS>
__global__ __launch_bounds__(64 * WAVES) void y_mfma_kernel(YArgs a) {
  using OPT = typename std::conditional<OP == OP_BF16, uint16_t, float>::type;
  using Frag = typename std::conditional<OP == OP_BF16, FragB, FragF>::type;
  constexpr int NT = TERMS;
  constexpr int ROWS = 16 * WAVES;
  constexpr int LDK = 32 + (OP == OP_BF16 ? 8 : 4);
  __shared__ OPT s_a[NT][4][ROWS][LDK];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int64_t rb = (int64_t)blockIdx.x * ROWS;
  const int jt0 = blockIdx.y * NJ;
  const OPT *om = (const OPT *)a.om;
  const int64_t ops = (int64_t)a.KP * a.NP;
  const TIN *ap[4] = {(const TIN *)a.a[0], (const TIN *)a.a[1], (const TIN *)a.a[2], (const TIN *)a.a[3]};
  // loader role: row lr of the tile, column group lg (8 columns)
  const int lr = tid % ROWS, lg = tid / ROWS;                // lg in 0..3
  const int64_t grow = rb + lr;

  floatx4 acc[NJ][4];
#pragma unroll
  for (int t = 0; t < NJ; ++t)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[t][p] = {0.f, 0.f, 0.f, 0.f};

  for (int64_t t0 = 0; t0 < a.ncols; t0 += 32) {
    {
      float x[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int64_t t = t0 + 8 * lg + s;
          x[s] = (grow < a.m && t < a.ncols && !(q == 0 && a.pure)) ? ldin<TIN>(ap[q], grow + t * a.lda) : 0.f;
        }
        if constexpr (OP == OP_BF16) {
          FragB f[3];
          split_terms<TERMS>(x, f);
#pragma unroll
          for (int tm = 0; tm < TERMS; ++tm)
            *(uint4 *)&s_a[tm][q][lr][8 * lg] = make_uint4(f[tm].v[0], f[tm].v[1], f[tm].v[2], f[tm].v[3]);
        } else {
#pragma unroll
          for (int s = 0; s < 8; ++s) s_a[0][q][lr][8 * lg + s] = x[s];
        }
      }
    }
    __syncthreads();
    Frag af[4][NT];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int tm = 0; tm < NT; ++tm) {
        {
          const OPT *src = &s_a[tm][q][wave * 16 + c16][8 * g];
          if constexpr (OP == OP_BF16) {
            const uint4 u = *(const uint4 *)src;
            af[q][tm].v[0] = u.x; af[q][tm].v[1] = u.y; af[q][tm].v[2] = u.z; af[q][tm].v[3] = u.w;
          } else {
#pragma unroll
            for (int s = 0; s < 8; ++s) af[q][tm].v[s] = src[s];
          }
        }
      }
    }
#pragma unroll
    for (int jt = 0; jt < NJ; ++jt) {
      const int jj = (jt0 + jt) * 16 + c16;                 // column of Y this lane reads Omega for
      Frag of[7];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const OPT *src = om + s * ops + (int64_t)jj * a.NP + t0 + 8 * g;
        if constexpr (OP == OP_BF16) {
          const uint4 u = *(const uint4 *)src;
          of[s].v[0] = u.x; of[s].v[1] = u.y; of[s].v[2] = u.z; of[s].v[3] = u.w;
        } else {
          const float4 u0 = *(const float4 *)src, u1 = *(const float4 *)(src + 4);
          of[s].v[0] = u0.x; of[s].v[1] = u0.y; of[s].v[2] = u0.z; of[s].v[3] = u0.w;
          of[s].v[4] = u1.x; of[s].v[5] = u1.y; of[s].v[6] = u1.z; of[s].v[7] = u1.w;
        }
      }
      if constexpr (OP == OP_BF16) { of[4] = negB(of[1]); of[5] = negB(of[2]); of[6] = negB(of[3]); }
      else { of[4] = negF(of[1]); of[5] = negF(of[2]); of[6] = negF(of[3]); }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q == 0 && a.pure) continue;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const Frag &os = of[rsel(q, p)];
#pragma unroll
          for (int tm = 0; tm < TERMS; ++tm) acc[jt][p] = mma(af[q][tm], os, acc[jt][p]);
        }
      }
    }
    __syncthreads();
  }
  // epilogue: lane holds column (jt0 + jt) * 16 + c16 of Y, rows rb + 16 wave + 4g + (0..3)
  const int64_t r0 = rb + wave * 16 + 4 * g;
#pragma unroll
  for (int jt = 0; jt < NJ; ++jt) {
    const int jj = (jt0 + jt) * 16 + c16;
    if (jj >= a.k) continue;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      float *dst = a.y + p * a.psy + (int64_t)jj * a.ldy;
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (r0 + t < a.m) dst[r0 + t] += acc[jt][p][t];
    }
  }
}

// ---------------------------------------------------------------------------
static inline int64_t rup(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// Staging geometry shared with the host's allocation.
void stage_geometry(int64_t m, int l, int k, int64_t maxcols, int *LP, int64_t *MP, int *KP,
                    int64_t *NP) {
  *LP = (int)rup(l, 112);
  *MP = rup(m, 32);
  *KP = (int)rup(k, 16 * 7);
  *NP = rup(maxcols, 32);
}

template <int MODE, typename OPT>
static hipError_t gen_stage(hipStream_t st, OPT *dst, int n_o, int o_pad, int64_t t0, int64_t n_t,
                            int64_t t_pad, uint32_t stream, int rad, uint32_t k0, uint32_t k1) {
  const int64_t total = (int64_t)o_pad * t_pad;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((gen_stage_kernel<MODE, OPT>), dim3((unsigned)blocks), dim3(256), 0, st, dst,
                     n_o, o_pad, t0, n_t, t_pad, stream, rad, k0, k1);
  return hipGetLastError();
}

static inline void mark(const SketchArgs &s, int idx) {
  if (s.events) (void)hipEventRecord(s.events[idx], s.stream);
}

template <int OP, typename TIN, int TERMS>
static hipError_t launch_t(const SketchArgs &s, const MfmaStage &g) {
  using OPT = typename std::conditional<OP == OP_BF16, uint16_t, float>::type;
  hipError_t e;
  mark(s, 0);
  // regenerate Omega_J and Psi in the operand format
  OPT *om = (OPT *)g.omega;
  OPT *ps = (OPT *)g.psi;
  const int64_t NPu = rup(s.ncols, 32);
  if (s.mode == MODE_BF16) {
    e = gen_stage<MODE_BF16, OPT>(s.stream, om, s.k, g.KP, s.col0, s.ncols, NPu, STREAM_OMEGA, s.rad, s.k0, s.k1);
    if (e != hipSuccess) return e;
    {
      e = gen_stage<MODE_BF16, OPT>(s.stream, ps, s.l, g.LP, 0, s.m, g.MP, STREAM_PSI, s.rad, s.k0, s.k1);
      if (e != hipSuccess) return e;
    }
  } else {
    e = gen_stage<MODE_F32, OPT>(s.stream, om, s.k, g.KP, s.col0, s.ncols, NPu, STREAM_OMEGA, s.rad, s.k0, s.k1);
    if (e != hipSuccess) return e;
    {
      e = gen_stage<MODE_F32, OPT>(s.stream, ps, s.l, g.LP, 0, s.m, g.MP, STREAM_PSI, s.rad, s.k0, s.k1);
      if (e != hipSuccess) return e;
    }
  }
  mark(s, 1);
  // ---- Y
  {
    mark(s, 2);
    YArgs y{};
    for (int p = 0; p < 4; ++p) y.a[p] = s.planes[p];
    y.lda = s.lda; y.m = s.m; y.ncols = s.ncols;
    y.om = om; y.KP = g.KP; y.NP = NPu;
    y.k = s.k; y.terms = s.terms; y.pure = s.pure;
    y.y = (float *)s.y; y.ldy = s.ldy; y.psy = s.psy;
    constexpr int WAVES = 4, NJ = 7;
    const int ntiles = (s.k + 15) / 16;
    dim3 grid((unsigned)((s.m + 16 * WAVES - 1) / (16 * WAVES)), (unsigned)((ntiles + NJ - 1) / NJ));
    hipLaunchKernelGGL((y_mfma_kernel<OP, TIN, NJ, WAVES, TERMS>), grid, dim3(64 * WAVES), 0, s.stream, y);
    e = hipGetLastError();
    mark(s, 3);
    if (e != hipSuccess) return e;
  }
  // ---- W
  {
    WArgs w{};
    for (int p = 0; p < 4; ++p) w.a[p] = s.planes[p];
    w.lda = s.lda; w.m = s.m; w.ncols = s.ncols; w.col0 = s.col0;
    w.psi = ps; w.LP = g.LP; w.MP = g.MP;
    w.l = s.l; w.terms = s.terms; w.pure = s.pure;
    w.w = (float *)s.w; w.ldw = s.ldw; w.psw = s.psw;
    constexpr int NMT = 7;
    const int mgroups = (s.l + 16 * NMT - 1) / (16 * NMT);
    const int64_t ctiles = (s.ncols + 63) / 64;
    // split the rows of A so that there are >= ~2 blocks per CU
    int64_t S = (512 + ctiles * mgroups - 1) / (ctiles * mgroups);
    if (S > 16) S = 16;
    int64_t kchunk = rup((s.m + S - 1) / S, 32);
    if (kchunk < 256) kchunk = 256;
    S = (s.m + kchunk - 1) / kchunk;
    const int64_t need = S * 4 * s.ncols * (int64_t)g.LP * 4;
    if (S > 1 && need > s.scratch_bytes) { S = 1; kchunk = rup(s.m, 32); }
    w.S = (int)S; w.kchunk = kchunk; w.part = (float *)s.scratch;
    dim3 grid((unsigned)ctiles, (unsigned)mgroups, (unsigned)S);
    mark(s, 4);
    hipLaunchKernelGGL((w_mfma_kernel<OP, TIN, NMT, TERMS>), grid, dim3(256), 0, s.stream, w);
    e = hipGetLastError();
    mark(s, 5);
    if (e != hipSuccess) return e;
    mark(s, 6);
    if (S > 1) {
      const int64_t total = 4 * s.ncols * (int64_t)s.l;
      int64_t blocks = (total + 255) / 256;
      if (blocks > 65536) blocks = 65536;
      hipLaunchKernelGGL(w_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s.stream,
                         (const float *)s.scratch, (int)S, g.LP, s.ncols, s.l, s.col0, (float *)s.w,
                         s.ldw, s.psw);
      e = hipGetLastError();
    }
    mark(s, 7);
  }
  return e;
}

hipError_t launch_sketch_mfma(const SketchArgs &s, const MfmaStage &g) {
  if (s.mode != MODE_BF16 && s.mode != MODE_F32) return hipErrorNotSupported;
  if (!g.omega || !g.psi) return hipErrorNotSupported;
  if (s.mode == MODE_BF16) {
    if (s.in_dtype == DT_F32) {
      if (s.terms == 1) return launch_t<OP_BF16, float, 1>(s, g);
      if (s.terms == 2) return launch_t<OP_BF16, float, 2>(s, g);
      return launch_t<OP_BF16, float, 3>(s, g);
    }
    if (s.in_dtype == DT_BF16) return launch_t<OP_BF16, uint16_t, 1>(s, g);   // bf16 data: exact in one term
  } else {
    if (s.in_dtype == DT_F32) return launch_t<OP_F32, float, 1>(s, g);
    if (s.in_dtype == DT_BF16) return launch_t<OP_F32, uint16_t, 1>(s, g);
  }
  return hipErrorNotSupported;
}

}  // namespace qsk
