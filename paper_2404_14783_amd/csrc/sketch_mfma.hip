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
#include <vector>

#include "qsk_device.hpp"
#include "qsk_kernels.hpp"

namespace qsk {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(4))) float floatx4;
// native 16-byte vector for the register-staged tiles (HIP's uint4 is a
// struct that keeps arrays of it out of registers)
typedef __attribute__((ext_vector_type(4))) unsigned int u32v4;

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

// Split 8 fp32 data values into TERMS bf16 fragments (hi, mid, lo): each
// term is the round-to-nearest-even bf16 value of what the previous terms
// left (the hardware conversion v_cvt_pk_bf16_f32 rounds to nearest even).
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2_t;
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
        const bf16x2_t h = {(__bf16)r[2 * i], (__bf16)r[2 * i + 1]};
        uint32_t u;
        __builtin_memcpy(&u, &h, 4);
        out[tm].v[i] = u;
        if (tm + 1 < TERMS) {
          r[2 * i] -= __uint_as_float(u << 16);
          r[2 * i + 1] -= __uint_as_float(u & 0xFFFF0000u);
        }
      }
    }
  }
}

template <typename TIN> __device__ __forceinline__ float ldin(const TIN *p, int64_t i);
template <> __device__ __forceinline__ float ldin<float>(const float *p, int64_t i) { return gp(p)[i]; }
template <> __device__ __forceinline__ float ldin<uint16_t>(const uint16_t *p, int64_t i) {
  return __uint_as_float(((uint32_t)gp(p)[i]) << 16);
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
// Block-to-tile mapping.  Workgroups are dispatched to the eight XCDs in
// turn (block b runs on XCD b mod 8), so the linear tile index is taken as
// (b mod 8) * (total / 8) + b / 8: consecutive tiles, which share a slice of
// the staged test matrix, then run on one XCD and hit its L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t total) {
  if ((total & 7) != 0) return b;
  return (b & 7) * (total >> 3) + (b >> 3);
}

// Loads of 8 consecutive input values (rows i .. i+7 of one column) for the
// operand conversion; vector loads when the column segment is aligned.
template <typename TIN>
__device__ __forceinline__ void load8(const TIN *p, int64_t idx, int64_t navail, bool vec, float (&x)[8]);
template <>
__device__ __forceinline__ void load8<float>(const float *p, int64_t idx, int64_t navail, bool vec,
                                             float (&x)[8]) {
  if (vec && navail >= 8) {
    const QSK_GLOBAL floatx4 *v = (const QSK_GLOBAL floatx4 *)(p + idx);
    const floatx4 u0 = v[0], u1 = v[1];
    x[0] = u0.x; x[1] = u0.y; x[2] = u0.z; x[3] = u0.w;
    x[4] = u1.x; x[5] = u1.y; x[6] = u1.z; x[7] = u1.w;
  } else {
#pragma unroll
    for (int s = 0; s < 8; ++s) x[s] = s < navail ? gp(p)[idx + s] : 0.f;
  }
}
template <>
__device__ __forceinline__ void load8<uint16_t>(const uint16_t *p, int64_t idx, int64_t navail,
                                                bool vec, float (&x)[8]) {
  if (vec && navail >= 8) {
    const u32v4 u = *(const QSK_GLOBAL u32v4 *)(p + idx);
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      x[2 * s] = __uint_as_float(w[s] << 16);
      x[2 * s + 1] = __uint_as_float(w[s] & 0xFFFF0000u);
    }
  } else {
#pragma unroll
    for (int s = 0; s < 8; ++s) x[s] = s < navail ? __uint_as_float(((uint32_t)gp(p)[idx + s]) << 16) : 0.f;
  }
}

// One input element at a byte address (global).
template <typename TIN> __device__ __forceinline__ float ld_elem(const QSK_GLOBAL char *p);
template <> __device__ __forceinline__ float ld_elem<float>(const QSK_GLOBAL char *p) {
  return *(const QSK_GLOBAL float *)p;
}
template <> __device__ __forceinline__ float ld_elem<uint16_t>(const QSK_GLOBAL char *p) {
  return __uint_as_float(((uint32_t)*(const QSK_GLOBAL uint16_t *)p) << 16);
}

// The negated copies of planes x, y, z of a test-matrix fragment set.
__device__ __forceinline__ void neg3(FragB (&f)[7]) { f[4] = negB(f[1]); f[5] = negB(f[2]); f[6] = negB(f[3]); }
__device__ __forceinline__ void neg3(FragF (&f)[7]) { f[4] = negF(f[1]); f[5] = negF(f[2]); f[6] = negF(f[3]); }

template <typename Frag, typename OPT>
__device__ __forceinline__ void lds_frag(const OPT *src, Frag &f);
template <>
__device__ __forceinline__ void lds_frag<FragB, uint16_t>(const uint16_t *src, FragB &f) {
  const uint4 u = *(const uint4 *)src;
  f.v[0] = u.x; f.v[1] = u.y; f.v[2] = u.z; f.v[3] = u.w;
}
template <>
__device__ __forceinline__ void lds_frag<FragF, float>(const float *src, FragF &f) {
  const float4 u0 = *(const float4 *)src, u1 = *(const float4 *)(src + 4);
  f.v[0] = u0.x; f.v[1] = u0.y; f.v[2] = u0.z; f.v[3] = u0.w;
  f.v[4] = u1.x; f.v[5] = u1.y; f.v[6] = u1.z; f.v[7] = u1.w;
}

// The data operand of one lane: 8 values per plane -> TERMS fragments.
template <int OP, int TERMS>
__device__ __forceinline__ void to_frags(const float (&x)[8], FragB (&out)[3]) { split_terms<TERMS>(x, out); }
template <int OP, int TERMS>
__device__ __forceinline__ void to_frags(const float (&x)[8], FragF (&out)[3]) {
#pragma unroll
  for (int s = 0; s < 8; ++s) out[0].v[s] = x[s];
}

// ---------------------------------------------------------------------------
// W kernel.  Tiles: 64 columns of the update block x NMT row tiles of W
// (16 rows each) x one chunk of the rows of A (split K over S chunks).
// Block = 4 waves; wave w owns columns 16 w .. 16 w + 15 of the tile, all NMT
// row tiles and all four planes.  Per 32-row step the Psi tile (4 planes x
// 16 NMT rows x 32) goes through LDS; each lane's A values (8 consecutive
// rows of its column, four planes) go straight from HBM into registers.  Both
// are fetched one step ahead (software pipelining).
struct WArgs {
  const void *a[4];
  int64_t lda, m, ncols, col0;
  const void *psi;            // staged [4][LP][MP]
  int LP;
  int64_t MP;
  int l, pure, S, ctiles, rgroups, vec;
  int64_t kchunk;
  float *w;
  int64_t ldw, psw;
  float *part;                // [S][4][ncols][LP]
};

template <int OP, typename TIN, int NMT, int TERMS, bool PURE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void w_mfma_kernel(WArgs a0, GroupRef grp) {
  WArgs a;
  int64_t t;
  if (grp.tab) {
    int p;
    group_find(grp, &p, &t);
    a = ((const WArgs *)grp.tab)[p];
  } else {
    a = a0;
    t = xcd_tile(blockIdx.x, (int64_t)a.ctiles * a.rgroups * a.S);
  }
  using OPT = typename std::conditional<OP == OP_BF16, uint16_t, float>::type;
  using Frag = typename std::conditional<OP == OP_BF16, FragB, FragF>::type;
  constexpr int LDK = 32 + (OP == OP_BF16 ? 8 : 4);        // padded K stride in LDS
  constexpr int EPV = 16 / sizeof(OPT);                    // elements per 16-byte vector
  constexpr int VPR = 32 / EPV;                            // vectors per tile row
  constexpr int NV = 4 * NMT * 16 * VPR;                   // vectors per Psi tile
  constexpr int VPT = NV / 256;
  static_assert(NV % 256 == 0, "Psi tile must split evenly over the block");
  __shared__ OPT s_psi[2][4][NMT * 16][LDK];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int bx = (int)(t % a.ctiles);
  const int by = (int)((t / a.ctiles) % a.rgroups);
  const int bz = (int)(t / ((int64_t)a.ctiles * a.rgroups));
  const int64_t j = (int64_t)bx * 64 + wave * 16 + c16;
  const int rbase = by * NMT * 16;
  const int64_t ib = (int64_t)bz * a.kchunk;
  const int64_t ie = min(a.m, ib + a.kchunk);
  const OPT *psi = (const OPT *)a.psi;
  const int64_t pps = (int64_t)a.LP * a.MP;
  const TIN *ap[4] = {(const TIN *)a.a[0], (const TIN *)a.a[1], (const TIN *)a.a[2], (const TIN *)a.a[3]};
  const bool jok = j < a.ncols;
  const bool vec = a.vec != 0;

  floatx4 acc[NMT][4];
#pragma unroll
  for (int r = 0; r < NMT; ++r)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[r][p] = {0.f, 0.f, 0.f, 0.f};

  float xa[4][8];
  u32v4 pr[VPT];
#define QSK_W_FETCH(I0)                                                                         \
  do {                                                                                          \
    const int64_t i_ = (I0) + 8 * g;                                                            \
    const int64_t nav_ = jok ? min((int64_t)8, ie - i_) : 0;                                    \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                             \
      if (q == 0 && PURE) {                                                                   \
        _Pragma("unroll") for (int s = 0; s < 8; ++s) xa[q][s] = 0.f;                           \
      } else {                                                                                  \
        load8<TIN>(ap[q], i_ + j * a.lda, nav_, vec, xa[q]);                                    \
      }                                                                                         \
    }                                                                                           \
    _Pragma("unroll") for (int u = 0; u < VPT; ++u) {                                           \
      const int e = tid + u * 256;                                                              \
      const int v = e % VPR, rr = (e / VPR) % (NMT * 16), pl = e / (VPR * NMT * 16);            \
      pr[u] = *(const QSK_GLOBAL u32v4 *)(psi + pl * pps + (int64_t)(rbase + rr) * a.MP + (I0) + v * EPV);   \
    }                                                                                           \
  } while (0)

#define QSK_W_STORE_PSI(BUF)                                                                    \
  do {                                                                                          \
    _Pragma("unroll") for (int u = 0; u < VPT; ++u) {                                           \
      const int e = tid + u * 256;                                                              \
      const int v = e % VPR, rr = (e / VPR) % (NMT * 16), pl = e / (VPR * NMT * 16);            \
      *(u32v4 *)&s_psi[BUF][pl][rr][v * EPV] = pr[u];                                           \
    }                                                                                           \
  } while (0)

  QSK_W_FETCH(ib);
  QSK_W_STORE_PSI(0);
  __syncthreads();
  int buf = 0;
  for (int64_t i0 = ib; i0 < ie; i0 += 32) {
    Frag af[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q) to_frags<OP, TERMS>(xa[q], af[q]);
    const bool more = i0 + 32 < ie;
    if (more) QSK_W_FETCH(i0 + 32);
    // Psi fragments of row tile rt + 1 are read from LDS while the matrix
    // cores work on row tile rt
    Frag pnext[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) lds_frag<Frag, OPT>(&s_psi[buf][s][c16][8 * g], pnext[s]);
#pragma unroll
    for (int rt = 0; rt < NMT; ++rt) {
      Frag pf[7];
#pragma unroll
      for (int s = 0; s < 4; ++s) pf[s] = pnext[s];
      if (rt + 1 < NMT) {
#pragma unroll
        for (int s = 0; s < 4; ++s) lds_frag<Frag, OPT>(&s_psi[buf][s][(rt + 1) * 16 + c16][8 * g], pnext[s]);
      }
      if constexpr (OP == OP_BF16) { pf[4] = negB(pf[1]); pf[5] = negB(pf[2]); pf[6] = negB(pf[3]); }
      else { pf[4] = negF(pf[1]); pf[5] = negF(pf[2]); pf[6] = negF(pf[3]); }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q == 0 && PURE) continue;
#pragma unroll
        for (int tm = 0; tm < TERMS; ++tm)
#pragma unroll
          for (int p = 0; p < 4; ++p) acc[rt][p] = mma(pf[ssel(p, q)], af[q][tm], acc[rt][p]);
      }
    }
    if (more) QSK_W_STORE_PSI(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // epilogue: lane holds column j, rows rbase + rt*16 + 4g + (0..3)
  if (!jok) return;
#pragma unroll
  for (int rt = 0; rt < NMT; ++rt) {
    const int r0 = rbase + rt * 16 + 4 * g;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      if (a.S == 1) {
        QSK_GLOBAL float *dst = gpw(a.w + p * a.psw + (a.col0 + j) * a.ldw);
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
          if (r0 + tt < a.l) dst[r0 + tt] += acc[rt][p][tt];
      } else {
        float *dst = a.part + (((int64_t)bz * 4 + p) * a.ncols + j) * a.LP + r0;
        *(QSK_GLOBAL floatx4 *)dst = acc[rt][p];
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
    for (int z = 0; z < S; ++z) s += gp(part)[(((int64_t)z * 4 + p) * ncols + j) * LP + r];
    gpw(w)[p * psw + (col0 + j) * ldw + r] += s;
  }
}

// ---------------------------------------------------------------------------
// Y kernel.  Tiles: 64 rows of A x NJ column tiles of Y (16 columns each) x
// one chunk of the update's columns (split K over S chunks; chunk s adds into
// its own copy s of Y, and the copies are summed when the sketch is read).
// Block = 4 waves; wave w owns rows 16 w .. 16 w + 15 of the tile, all NJ
// column tiles and all four planes.  No other wave needs a wave's rows of A,
// so each lane loads its own operand values (row c16, columns 8 g .. 8 g + 7
// of the step) straight from HBM; only the Omega tile, which all four waves
// share, goes through LDS (two buffers, one barrier per step).  Both are
// fetched one step ahead.
struct YArgs {
  const void *a[4];
  int64_t lda, m, ncols;
  const void *om;             // staged [4][KP][NP]
  int KP;
  int64_t NP;
  int k, pure, S, rblocks, cgroups;
  int64_t tchunk;
  float *y;
  int64_t ldy, psy, pss;      // copy s of plane p: y + s * pss + p * psy
};

template <int OP, typename TIN, int NJ, int TERMS, bool PURE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void y_mfma_kernel(YArgs a0, GroupRef grp) {
  YArgs a;
  int64_t t;
  if (grp.tab) {
    int p;
    group_find(grp, &p, &t);
    a = ((const YArgs *)grp.tab)[p];
  } else {
    a = a0;
    t = xcd_tile(blockIdx.x, (int64_t)a.rblocks * a.cgroups * a.S);
  }
  using OPT = typename std::conditional<OP == OP_BF16, uint16_t, float>::type;
  using Frag = typename std::conditional<OP == OP_BF16, FragB, FragF>::type;
  constexpr int LDK = 32 + (OP == OP_BF16 ? 8 : 4);
  constexpr int EPV = 16 / sizeof(OPT);
  constexpr int VPR = 32 / EPV;
  constexpr int NV = 4 * NJ * 16 * VPR;                     // vectors per Omega tile
  constexpr int VPT = NV / 256;
  static_assert(NV % 256 == 0, "Omega tile must split evenly over the block");
  __shared__ OPT s_om[2][4][NJ * 16][LDK];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int64_t bx = t % a.rblocks;
  const int by = (int)((t / a.rblocks) % a.cgroups);
  const int bz = (int)(t / ((int64_t)a.rblocks * a.cgroups));
  const int64_t rb = bx * 64;
  const int jt0 = by * NJ;
  const int64_t tb = (int64_t)bz * a.tchunk;
  const int64_t te = min(a.ncols, tb + a.tchunk);
  const OPT *om = (const OPT *)a.om;
  const int64_t ops = (int64_t)a.KP * a.NP;
  // plane bases (uniform) and this lane's byte offsets into them: the update
  // block of every plane spans < 4 GiB (checked on the host), so a 32-bit
  // offset from a scalar base addresses it
  const QSK_GLOBAL char *ab[4] = {(const QSK_GLOBAL char *)a.a[0], (const QSK_GLOBAL char *)a.a[1],
                                  (const QSK_GLOBAL char *)a.a[2], (const QSK_GLOBAL char *)a.a[3]};
  const int64_t row = rb + wave * 16 + c16;                 // this lane's row of A
  const bool rok = row < a.m;
  const int64_t rowc = rok ? row : a.m - 1;

  floatx4 acc[NJ][4];
#pragma unroll
  for (int u = 0; u < NJ; ++u)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[u][p] = {0.f, 0.f, 0.f, 0.f};

  // A values of two steps in flight: X[q][s] = A_q[row, T + 8 g + s]
  float xa0[4][8], xa1[4][8];
  u32v4 orr[VPT];
#define QSK_Y_FETCH_A(T0, X)                                                                    \
  do {                                                                                          \
    /* out-of-range elements load a valid address and are zeroed (no branches) */              \
    _Pragma("unroll") for (int s = 0; s < 8; ++s) {                                             \
      const int64_t tt = (T0) + 8 * g + s;                                                      \
      const bool ok_ = rok && tt < te;                                                          \
      const uint32_t off_ = (uint32_t)((rowc + (ok_ ? tt : tb) * a.lda) * (int64_t)sizeof(TIN)); \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                           \
        if (q == 0 && PURE) { X[q][s] = 0.f; continue; }                                        \
        const float v_ = ld_elem<TIN>(ab[q] + off_);                                            \
        X[q][s] = ok_ ? v_ : 0.f;                                                               \
      }                                                                                         \
    }                                                                                           \
  } while (0)
#define QSK_Y_FETCH_OM(T0)                                                                      \
  do {                                                                                          \
    _Pragma("unroll") for (int u = 0; u < VPT; ++u) {                                           \
      const int e = tid + u * 256;                                                              \
      const int v = e % VPR, oo = (e / VPR) % (NJ * 16), pl = e / (VPR * NJ * 16);              \
      orr[u] = *(const QSK_GLOBAL u32v4 *)(om + pl * ops + (int64_t)(jt0 * 16 + oo) * a.NP + (T0) + v * EPV); \
    }                                                                                           \
  } while (0)
#define QSK_Y_STORE_OM(BUF)                                                                     \
  do {                                                                                          \
    _Pragma("unroll") for (int u = 0; u < VPT; ++u) {                                           \
      const int e = tid + u * 256;                                                              \
      const int v = e % VPR, oo = (e / VPR) % (NJ * 16), pl = e / (VPR * NJ * 16);              \
      *(u32v4 *)&s_om[BUF][pl][oo][v * EPV] = orr[u];                                           \
    }                                                                                           \
  } while (0)
  // one 32-column step from the A values in X: convert, refetch X two steps
  // ahead, fetch the next Omega tile, run the matrix cores, stage Omega
#define QSK_Y_STEP(T0, X)                                                                       \
  do {                                                                                          \
    Frag af[4][3];                                                                              \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) to_frags<OP, TERMS>(X[q], af[q]);             \
    if ((T0) + 64 < te) QSK_Y_FETCH_A((T0) + 64, X);                                            \
    const bool more_ = (T0) + 32 < te;                                                          \
    if (more_) QSK_Y_FETCH_OM((T0) + 32);                                                       \
    Frag onext[4];                                                                              \
    _Pragma("unroll") for (int s = 0; s < 4; ++s)                                               \
      lds_frag<Frag, OPT>(&s_om[buf][s][c16][8 * g], onext[s]);                                 \
    _Pragma("unroll") for (int jt = 0; jt < NJ; ++jt) {                                         \
      Frag of[7];                                                                               \
      _Pragma("unroll") for (int s = 0; s < 4; ++s) of[s] = onext[s];                           \
      if (jt + 1 < NJ) {                                                                        \
        _Pragma("unroll") for (int s = 0; s < 4; ++s)                                           \
          lds_frag<Frag, OPT>(&s_om[buf][s][(jt + 1) * 16 + c16][8 * g], onext[s]);             \
      }                                                                                         \
      neg3(of);                                                                                 \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                           \
        if (q == 0 && PURE) continue;                                                         \
        _Pragma("unroll") for (int tm = 0; tm < TERMS; ++tm)                                    \
          _Pragma("unroll") for (int p = 0; p < 4; ++p)                                         \
            acc[jt][p] = mma(af[q][tm], of[rsel(q, p)], acc[jt][p]);                            \
      }                                                                                         \
    }                                                                                           \
    if (more_) QSK_Y_STORE_OM(buf ^ 1);                                                         \
    __syncthreads();                                                                            \
    buf ^= 1;                                                                                   \
  } while (0)

  QSK_Y_FETCH_A(tb, xa0);
  if (tb + 32 < te) QSK_Y_FETCH_A(tb + 32, xa1);
  QSK_Y_FETCH_OM(tb);
  QSK_Y_STORE_OM(0);
  __syncthreads();
  int buf = 0;
  for (int64_t t0 = tb; t0 < te; t0 += 64) {
    QSK_Y_STEP(t0, xa0);
    if (t0 + 32 < te) QSK_Y_STEP(t0 + 32, xa1);
  }
  // epilogue: lane holds column (jt0 + jt) * 16 + c16 of Y, rows rb + 16 wave + 4g + (0..3)
  const int64_t r0 = rb + wave * 16 + 4 * g;
  float *ys = a.y + bz * a.pss;
#pragma unroll
  for (int jt = 0; jt < NJ; ++jt) {
    const int jj = (jt0 + jt) * 16 + c16;
    if (jj >= a.k) continue;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      QSK_GLOBAL float *dst = gpw(ys + p * a.psy + (int64_t)jj * a.ldy);
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
        if (r0 + tt < a.m) dst[r0 + tt] += acc[jt][p][tt];
    }
  }
}

#undef QSK_W_FETCH
#undef QSK_W_STORE_PSI
#undef QSK_Y_FETCH_A
#undef QSK_Y_FETCH_OM
#undef QSK_Y_STORE_OM
#undef QSK_Y_STEP

// Y = sum of its split-K copies: copy 0 += copies 1 .. S-1, which are cleared.
__global__ void y_fold_kernel(float *y, int64_t n_per_copy, int S) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_per_copy;
       e += (int64_t)gridDim.x * blockDim.x) {
    float s = y[e];
    for (int c = 1; c < S; ++c) {
      s += y[c * n_per_copy + e];
      y[c * n_per_copy + e] = 0.f;
    }
    y[e] = s;
  }
}

hipError_t launch_y_fold(hipStream_t st, float *y, int64_t n_per_copy, int S) {
  if (S <= 1) return hipSuccess;
  int64_t blocks = (n_per_copy + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(y_fold_kernel, dim3((unsigned)blocks), dim3(256), 0, st, y, n_per_copy, S);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
static inline int64_t rup(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// Tile choices: NMT row tiles of W per block (from {4, 7, 13}; 13 only for
// bf16 operands, whose Psi tile is half the size) and NJ column tiles of Y
// per block (from {4, 7}), each minimising the padded tile count (ties go to
// the larger tile).
static int pick_tiles(int tiles, const int *cand, int nc) {
  int best = cand[0], best_pad = 1 << 30;
  for (int i = 0; i < nc; ++i) {
    const int c = cand[i];
    const int pad = (tiles + c - 1) / c * c;
    if (pad < best_pad || (pad == best_pad && c > best)) { best = c; best_pad = pad; }
  }
  return best;
}
static int w_nmt(int l, int op_bf16) {
  static const int cb[3] = {4, 7, 13}, cf[2] = {4, 7};
  return op_bf16 ? pick_tiles((l + 15) / 16, cb, 3) : pick_tiles((l + 15) / 16, cf, 2);
}
static int y_nj(int k) {
  static const int c[2] = {4, 7};
  return pick_tiles((k + 15) / 16, c, 2);
}

// Staging geometry shared with the host's allocation.
void stage_geometry(int64_t m, int l, int k, int64_t maxcols, int op_bf16, int *LP, int64_t *MP,
                    int *KP, int64_t *NP) {
  *LP = (int)rup(l, 16 * w_nmt(l, op_bf16));
  *MP = rup(m, 32);
  *KP = (int)rup(k, 16 * y_nj(k));
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

// `pure` (no real plane) is a template parameter so that the product
// sequences have no branches
template <int OP, typename TIN, int TERMS, int NMT>
static void launch_w(const WArgs &w, int64_t blocks, hipStream_t st, GroupRef g = GroupRef{}) {
  if (w.pure)
    hipLaunchKernelGGL((w_mfma_kernel<OP, TIN, NMT, TERMS, true>), dim3((unsigned)blocks), dim3(256), 0, st, w, g);
  else
    hipLaunchKernelGGL((w_mfma_kernel<OP, TIN, NMT, TERMS, false>), dim3((unsigned)blocks), dim3(256), 0, st, w, g);
}
template <int OP, typename TIN, int TERMS, int NJ>
static void launch_y(const YArgs &y, int64_t blocks, hipStream_t st, GroupRef g = GroupRef{}) {
  if (y.pure)
    hipLaunchKernelGGL((y_mfma_kernel<OP, TIN, NJ, TERMS, true>), dim3((unsigned)blocks), dim3(256), 0, st, y, g);
  else
    hipLaunchKernelGGL((y_mfma_kernel<OP, TIN, NJ, TERMS, false>), dim3((unsigned)blocks), dim3(256), 0, st, y, g);
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

template <int OP, typename TIN, int TERMS>
static hipError_t launch_t(const SketchArgs &s, const MfmaStage &g) {
  using OPT = typename std::conditional<OP == OP_BF16, uint16_t, float>::type;
  // the Y kernel addresses each plane's update block with 32-bit byte offsets
  if ((uint64_t)((s.m - 1) + (s.ncols - 1) * s.lda) * sizeof(TIN) >= (1ull << 32)) return hipErrorNotSupported;
  hipError_t e;
  mark(s, 0);
  // regenerate Omega_J and Psi in the operand format
  OPT *om = (OPT *)g.omega;
  OPT *ps = (OPT *)g.psi;
  const int64_t NPu = rup(s.ncols, 32);
  if (s.mode == MODE_BF16) {
    e = gen_stage<MODE_BF16, OPT>(s.stream, om, s.k, g.KP, s.col0, s.ncols, NPu, STREAM_OMEGA, s.rad, s.k0, s.k1);
    if (e != hipSuccess) return e;
    e = gen_stage<MODE_BF16, OPT>(s.stream, ps, s.l, g.LP, 0, s.m, g.MP, STREAM_PSI, s.rad, s.k0, s.k1);
    if (e != hipSuccess) return e;
  } else {
    e = gen_stage<MODE_F32, OPT>(s.stream, om, s.k, g.KP, s.col0, s.ncols, NPu, STREAM_OMEGA, s.rad, s.k0, s.k1);
    if (e != hipSuccess) return e;
    e = gen_stage<MODE_F32, OPT>(s.stream, ps, s.l, g.LP, 0, s.m, g.MP, STREAM_PSI, s.rad, s.k0, s.k1);
    if (e != hipSuccess) return e;
  }
  mark(s, 1);
  // vector loads of the input need 16-byte aligned column segments
  bool vec = (s.lda % (16 / (int64_t)sizeof(TIN))) == 0;
  for (int p = s.pure ? 1 : 0; p < 4; ++p) vec = vec && aligned16(s.planes[p]);
  // ---- Y
  {
    mark(s, 2);
    YArgs y{};
    for (int p = 0; p < 4; ++p) y.a[p] = s.planes[p];
    y.lda = s.lda; y.m = s.m; y.ncols = s.ncols;
    y.om = om; y.KP = g.KP; y.NP = NPu;
    y.k = s.k; y.pure = s.pure;
    y.y = (float *)s.y; y.ldy = s.ldy; y.psy = s.psy; y.pss = s.pss;
    const int nj = y_nj(s.k);
    const int ntiles = (s.k + 15) / 16;
    y.rblocks = (int)((s.m + 63) / 64);
    y.cgroups = (ntiles + nj - 1) / nj;
    // split the update's columns over the Y copies so that the grid holds
    // about four blocks per CU
    int64_t S = (1024 + (int64_t)y.rblocks * y.cgroups - 1) / ((int64_t)y.rblocks * y.cgroups);
    if (S > s.y_copies) S = s.y_copies;
    if (S < 1) S = 1;
    int64_t tchunk = rup((s.ncols + S - 1) / S, 32);
    S = (s.ncols + tchunk - 1) / tchunk;
    y.S = (int)S; y.tchunk = tchunk;
    const int64_t blocks = (int64_t)y.rblocks * y.cgroups * S;
    if (nj == 7) launch_y<OP, TIN, TERMS, 7>(y, blocks, s.stream);
    else launch_y<OP, TIN, TERMS, 4>(y, blocks, s.stream);
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
    w.l = s.l; w.pure = s.pure; w.vec = vec ? 1 : 0;
    w.w = (float *)s.w; w.ldw = s.ldw; w.psw = s.psw;
    const int nmt = w_nmt(s.l, OP == OP_BF16);
    w.rgroups = (int)(g.LP / (16 * nmt));
    w.ctiles = (int)((s.ncols + 63) / 64);
    // split the rows of A so that there are >= ~2 blocks per CU
    const int64_t base = (int64_t)w.ctiles * w.rgroups;
    int64_t S = (512 + base - 1) / base;
    if (S > 16) S = 16;
    int64_t kchunk = rup((s.m + S - 1) / S, 32);
    if (kchunk < 256) kchunk = 256;
    S = (s.m + kchunk - 1) / kchunk;
    const int64_t need = S * 4 * s.ncols * (int64_t)g.LP * 4;
    if (S > 1 && need > s.scratch_bytes) { S = 1; kchunk = rup(s.m, 32); }
    w.S = (int)S; w.kchunk = kchunk; w.part = (float *)s.scratch;
    const int64_t blocks = base * S;
    mark(s, 4);
    if (nmt == 13) launch_w<OP, TIN, TERMS, (OP == OP_BF16 ? 13 : 7)>(w, blocks, s.stream);
    else if (nmt == 7) launch_w<OP, TIN, TERMS, 7>(w, blocks, s.stream);
    else launch_w<OP, TIN, TERMS, 4>(w, blocks, s.stream);
    e = hipGetLastError();
    mark(s, 5);
    if (e != hipSuccess) return e;
    mark(s, 6);
    if (S > 1) {
      const int64_t total = 4 * s.ncols * (int64_t)s.l;
      int64_t rblocks = (total + 255) / 256;
      if (rblocks > 65536) rblocks = 65536;
      hipLaunchKernelGGL(w_reduce_kernel, dim3((unsigned)rblocks), dim3(256), 0, s.stream,
                         (const float *)s.scratch, (int)S, g.LP, s.ncols, s.l, s.col0, (float *)s.w,
                         s.ldw, s.psw);
      e = hipGetLastError();
    }
    mark(s, 7);
  }
  return e;
}

// ---------------------------------------------------------------------------
// Batches: one tile choice for all problems, the test matrices staged once
// (all n columns of Omega), and the Y and W products of every problem in one
// grouped launch each (no split K: each problem's tiles write its own Y and
// W directly).
void batch_tiles(const int *l, const int *k, int count, int op_bf16, int *nmt, int *nj) {
  static const int cb[3] = {4, 7, 13}, cf[2] = {4, 7}, cy[2] = {4, 7};
  const int *cw = op_bf16 ? cb : cf;
  const int ncw = op_bf16 ? 3 : 2;
  int64_t best = -1;
  for (int i = 0; i < ncw; ++i) {
    int64_t pad = 0;
    for (int p = 0; p < count; ++p) {
      const int t = (l[p] + 15) / 16;
      pad += (t + cw[i] - 1) / cw[i] * cw[i];
    }
    if (best < 0 || pad < best || (pad == best && cw[i] > *nmt)) { best = pad; *nmt = cw[i]; }
  }
  best = -1;
  for (int i = 0; i < 2; ++i) {
    int64_t pad = 0;
    for (int p = 0; p < count; ++p) {
      const int t = (k[p] + 15) / 16;
      pad += (t + cy[i] - 1) / cy[i] * cy[i];
    }
    if (best < 0 || pad < best || (pad == best && cy[i] > *nj)) { best = pad; *nj = cy[i]; }
  }
}

void stage_geometry_tiles(int64_t m, int l, int k, int64_t maxcols, int nmt, int nj, int *LP,
                          int64_t *MP, int *KP, int64_t *NP) {
  *LP = (int)rup(l, 16 * nmt);
  *MP = rup(m, 32);
  *KP = (int)rup(k, 16 * nj);
  *NP = rup(maxcols, 32);
}

hipError_t stage_test_matrices(const SketchArgs &s, const MfmaStage &g) {
  if (s.mode == MODE_BF16) {
    hipError_t e = gen_stage<MODE_BF16, uint16_t>(s.stream, (uint16_t *)g.omega, s.k, g.KP, 0, s.ncols,
                                                  g.NP, STREAM_OMEGA, s.rad, s.k0, s.k1);
    if (e != hipSuccess) return e;
    return gen_stage<MODE_BF16, uint16_t>(s.stream, (uint16_t *)g.psi, s.l, g.LP, 0, s.m, g.MP,
                                          STREAM_PSI, s.rad, s.k0, s.k1);
  }
  if (s.mode == MODE_F32) {
    hipError_t e = gen_stage<MODE_F32, float>(s.stream, (float *)g.omega, s.k, g.KP, 0, s.ncols, g.NP,
                                              STREAM_OMEGA, s.rad, s.k0, s.k1);
    if (e != hipSuccess) return e;
    return gen_stage<MODE_F32, float>(s.stream, (float *)g.psi, s.l, g.LP, 0, s.m, g.MP, STREAM_PSI,
                                      s.rad, s.k0, s.k1);
  }
  return hipErrorNotSupported;
}

template <int OP, typename TIN, int TERMS>
static hipError_t launch_batch_t(const SketchArgs *s, const MfmaStage *g, int count, int nmt, int nj,
                                 ArgArena &ar) {
  std::vector<YArgs> ys(count);
  std::vector<WArgs> ws(count);
  std::vector<int64_t> py(count + 1, 0), pw(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    const SketchArgs &q = s[i];
    if ((uint64_t)((q.m - 1) + (q.ncols - 1) * q.lda) * sizeof(TIN) >= (1ull << 32)) return hipErrorNotSupported;
    bool vec = (q.lda % (16 / (int64_t)sizeof(TIN))) == 0;
    for (int p = q.pure ? 1 : 0; p < 4; ++p) vec = vec && aligned16(q.planes[p]);
    YArgs &y = ys[i];
    for (int p = 0; p < 4; ++p) y.a[p] = q.planes[p];
    y.lda = q.lda; y.m = q.m; y.ncols = q.ncols;
    y.om = g[i].omega; y.KP = g[i].KP; y.NP = g[i].NP;
    y.k = q.k; y.pure = q.pure;
    y.y = (float *)q.y; y.ldy = q.ldy; y.psy = q.psy; y.pss = 0;
    y.rblocks = (int)((q.m + 63) / 64);
    y.cgroups = g[i].KP / (16 * nj);
    y.S = 1; y.tchunk = rup(q.ncols, 32);
    py[i + 1] = py[i] + (int64_t)y.rblocks * y.cgroups;
    WArgs &w = ws[i];
    for (int p = 0; p < 4; ++p) w.a[p] = q.planes[p];
    w.lda = q.lda; w.m = q.m; w.ncols = q.ncols; w.col0 = 0;
    w.psi = g[i].psi; w.LP = g[i].LP; w.MP = g[i].MP;
    w.l = q.l; w.pure = q.pure; w.vec = vec ? 1 : 0;
    w.w = (float *)q.w; w.ldw = q.ldw; w.psw = q.psw;
    w.rgroups = g[i].LP / (16 * nmt);
    w.ctiles = (int)((q.ncols + 63) / 64);
    w.S = 1; w.kchunk = rup(q.m, 32); w.part = nullptr;
    pw[i + 1] = pw[i] + (int64_t)w.ctiles * w.rgroups;
  }
  hipStream_t st = s[0].stream;
  GroupRef gy{arena_push(ar, st, ys.data(), ys.size() * sizeof(YArgs)),
              (const int64_t *)arena_push(ar, st, py.data(), py.size() * sizeof(int64_t)), count};
  GroupRef gw{arena_push(ar, st, ws.data(), ws.size() * sizeof(WArgs)),
              (const int64_t *)arena_push(ar, st, pw.data(), pw.size() * sizeof(int64_t)), count};
  if (!gy.tab || !gy.prefix || !gw.tab || !gw.prefix) return hipErrorOutOfMemory;
  if (nj == 7) launch_y<OP, TIN, TERMS, 7>(ys[0], py[count], st, gy);
  else launch_y<OP, TIN, TERMS, 4>(ys[0], py[count], st, gy);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nmt == 13) launch_w<OP, TIN, TERMS, (OP == OP_BF16 ? 13 : 7)>(ws[0], pw[count], st, gw);
  else if (nmt == 7) launch_w<OP, TIN, TERMS, 7>(ws[0], pw[count], st, gw);
  else launch_w<OP, TIN, TERMS, 4>(ws[0], pw[count], st, gw);
  return hipGetLastError();
}

hipError_t launch_sketch_mfma_batch(const SketchArgs *s, const MfmaStage *g, int count, int nmt,
                                    int nj, ArgArena &ar) {
  if (count < 1) return hipSuccess;
  const SketchArgs &a = s[0];
  if (a.mode == MODE_BF16) {
    if (a.in_dtype == DT_F32) {
      if (a.terms == 1) return launch_batch_t<OP_BF16, float, 1>(s, g, count, nmt, nj, ar);
      if (a.terms == 2) return launch_batch_t<OP_BF16, float, 2>(s, g, count, nmt, nj, ar);
      return launch_batch_t<OP_BF16, float, 3>(s, g, count, nmt, nj, ar);
    }
    if (a.in_dtype == DT_BF16) return launch_batch_t<OP_BF16, uint16_t, 1>(s, g, count, nmt, nj, ar);
  } else if (a.mode == MODE_F32) {
    if (a.in_dtype == DT_F32) return launch_batch_t<OP_F32, float, 1>(s, g, count, nmt, nj, ar);
    if (a.in_dtype == DT_BF16) return launch_batch_t<OP_F32, uint16_t, 1>(s, g, count, nmt, nj, ar);
  }
  return hipErrorNotSupported;
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
