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
#include <algorithm>
#include <cmath>
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

// Operand formats of the products: bf16 (data split into bf16 terms), fp32,
// and fp8-quantised data: e4m3 with a power-of-two scale per 32 x 32 tile,
// whose dequantised values are exact in bf16, plus the exact residual as
// further bf16 terms (all three run on the bf16 matrix-core instruction).
enum : int { OP_BF16 = 0, OP_F32 = 1, OP_FP8 = 2 };
constexpr bool op_f32(int op) { return op == OP_F32; }

// ---------------------------------------------------------------------------
// Staging of the test matrices.  Layout [plane][o][t] with t (the contraction
// index) fastest; entries outside (o < n_o, t < n_t) are zero.
template <int MODE, typename OPT>
__global__ __launch_bounds__(256) void gen_stage_kernel(OPT *dst, int n_o, int o_pad, int64_t t0,
                                                        int64_t n_t, int64_t t_pad, uint32_t stream,
                                                        int rad, uint32_t k0, uint32_t k1, int tiled) {
  const int64_t total = (int64_t)o_pad * t_pad;
  const int64_t ps = total;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e % t_pad;
    const int o = (int)(e / t_pad);
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (o < n_o && t < n_t) embed_entry<MODE>(rad, (uint32_t)(t0 + t), (uint32_t)o, stream, k0, k1, v);
    const int64_t d = tiled ? psi_tiled_index<sizeof(OPT)>(o, t, o_pad >> 4) : e;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      if constexpr (sizeof(OPT) == 2) {
        dst[p * ps + d] = (OPT)(__float_as_uint(v[p]) >> 16);   // exact: v is a bf16 value
      } else {
        dst[p * ps + d] = v[p];
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

// The same tables read by test-matrix plane: the data plane q whose product
// with plane s of Psi (W) or of Omega (Y) lands in output plane p, and
// whether that term carries a minus sign.  Each output plane takes each
// test-matrix plane exactly once.
__device__ constexpr int w_q_of(int p, int s) {
  for (int q = 0; q < 4; ++q)
    if (ssel(p, q) == s || (s > 0 && ssel(p, q) == s + 3)) return q;
  return -1;
}
__device__ constexpr bool w_neg(int p, int s) { return ssel(p, w_q_of(p, s)) >= 4; }
__device__ constexpr int y_q_of(int p, int s) {
  for (int q = 0; q < 4; ++q)
    if (rsel(q, p) == s || (s > 0 && rsel(q, p) == s + 3)) return q;
  return -1;
}
__device__ constexpr bool y_neg(int p, int s) { return rsel(y_q_of(p, s), p) >= 4; }

// ---------------------------------------------------------------------------
// Block-to-tile mapping.  Workgroups are dispatched to the eight XCDs in
// turn (block b runs on XCD b mod 8), so the linear tile index is taken as
// (b mod 8) * (total / 8) + b / 8: consecutive tiles, which share a slice of
// the staged test matrix, then run on one XCD and hit its L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t total) {
  if ((total & 7) != 0) return b;
  return (b & 7) * (total >> 3) + (b >> 3);
}

// The negated copies of planes x, y, z of a test-matrix fragment set.
__device__ __forceinline__ FragB negx(const FragB &a) { return negB(a); }
__device__ __forceinline__ FragF negx(const FragF &a) { return negF(a); }
// The sign of a product term goes on the data operand when it has at most
// two terms: its planes x, y, z are negated once per step (the test-matrix
// fragments of every tile would need it once per tile), and a signed
// selection 4..6 multiplies the plain test-matrix plane 1..3 with the
// negated data.  With three terms the registers are short, and the
// test-matrix fragments are negated instead.
template <int TERMS> constexpr bool neg_on_data() { return TERMS <= 2; }
template <typename Frag, int TERMS>
__device__ __forceinline__ void neg_data(const Frag (&af)[4][3], Frag (&naf)[4][3]) {
  if constexpr (neg_on_data<TERMS>()) {
#pragma unroll
    for (int q = 1; q < 4; ++q)
#pragma unroll
      for (int tm = 0; tm < TERMS; ++tm) naf[q][tm] = negx(af[q][tm]);
  }
}

// fp8 operand split of 8 data values sharing the tile scale sc (a power of
// two): term 0 is q * sc with q = e4m3(x / sc) (round to nearest even, as
// the tile scale keeps |x / sc| <= 448 no saturation occurs), exact in bf16;
// the residual x - q * sc is exact in fp32 and follows as TERMS - 1 bf16
// terms.
template <int TERMS>
__device__ __forceinline__ void split_fp8(const float (&x)[8], float sc, FragB (&out)[3]) {
  const float inv = 1.0f / sc;                       // exact: sc is a power of two
  float r[8];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float d0 = e4m3_rne(x[2 * i] * inv) * sc, d1 = e4m3_rne(x[2 * i + 1] * inv) * sc;
    out[0].v[i] = (__float_as_uint(d0) >> 16) | (__float_as_uint(d1) & 0xFFFF0000u);
    r[2 * i] = x[2 * i] - d0;
    r[2 * i + 1] = x[2 * i + 1] - d1;
  }
  if constexpr (TERMS > 1) {
    FragB rest[3];
    split_terms<TERMS - 1>(r, rest);
#pragma unroll
    for (int tm = 1; tm < TERMS; ++tm) out[tm] = rest[tm - 1];
  }
}

// The data operand of one lane: 8 values per plane -> TERMS fragments.
template <int OP, int TERMS>
__device__ __forceinline__ void to_frags(const float (&x)[8], float sc, FragB (&out)[3]) {
  if constexpr (OP == OP_FP8) split_fp8<TERMS>(x, sc, out);
  else split_terms<TERMS>(x, out);
}
template <int OP, int TERMS>
__device__ __forceinline__ void to_frags(const float (&x)[8], float sc, FragF (&out)[3]) {
#pragma unroll
  for (int s = 0; s < 8; ++s) out[0].v[s] = x[s];
}

// ---------------------------------------------------------------------------
// Operand access shared by both kernels.
//
// The data planes are read through buffer resources that span one plane of
// the update block, [0, ((ncols - 1) lda + m) elements): a load at an offset
// past the end returns zero instead of faulting, so the loads need no
// predicates and never split the instruction stream into branches.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
// 8 consecutive values of one column (W's data operand); byte offset voff
template <typename TIN> __device__ __forceinline__ void bload8(rsrc_t r, uint32_t voff, float (&x)[8]);
template <> __device__ __forceinline__ void bload8<float>(rsrc_t r, uint32_t voff, float (&x)[8]) {
  const u32v4 u0 = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
  const u32v4 u1 = __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16, 0, 0);
  x[0] = __uint_as_float(u0.x); x[1] = __uint_as_float(u0.y); x[2] = __uint_as_float(u0.z); x[3] = __uint_as_float(u0.w);
  x[4] = __uint_as_float(u1.x); x[5] = __uint_as_float(u1.y); x[6] = __uint_as_float(u1.z); x[7] = __uint_as_float(u1.w);
}
template <> __device__ __forceinline__ void bload8<uint16_t>(rsrc_t r, uint32_t voff, float (&x)[8]) {
  const u32v4 u = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    x[2 * s] = __uint_as_float(w[s] << 16);
    x[2 * s + 1] = __uint_as_float(w[s] & 0xFFFF0000u);
  }
}
// one value (Y's data operand); the column stride goes in the scalar offset
template <typename TIN> __device__ __forceinline__ float bload1(rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ float bload1<float>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <> __device__ __forceinline__ float bload1<uint16_t>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __uint_as_float(((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)) << 16);
}

// ---------------------------------------------------------------------------
// fp8 tile scales of one update block: for plane p and the 32 x 32 tile
// (rt, ct) of the block (rows from 0, columns from the block's first), the
// smallest power of two sc with amax / sc <= 448, 1 for an all-zero tile;
// sc[(p * RT + rt) * CT + ct].  One wave per tile: lane L reads rows
// 4 (L mod 8) .. + 3 of columns L / 8 + 8 j, j = 0..3, so that each load
// instruction covers eight 128-byte column segments; reads past the block
// return zero and rows past m are masked.
template <typename TIN>
__global__ __launch_bounds__(256) void fp8_scale_kernel(const void *a0, const void *a1, const void *a2,
                                                        const void *a3, int64_t lda, int64_t m,
                                                        int64_t ncols, int pure, int RT, int CT,
                                                        float *sc) {
  const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t ntiles = 4 * (int64_t)RT * CT;
  if (tile >= ntiles) return;
  const int p = (int)(tile / ((int64_t)RT * CT));
  const int rt = (int)((tile / CT) % RT), ct = (int)(tile % CT);
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)rt * 32 + 4 * (lane & 7);
  const void *a = p == 0 ? a0 : p == 1 ? a1 : p == 2 ? a2 : a3;
  float mx = 0.f;
  if (!(p == 0 && pure)) {
    const rsrc_t rs = make_rsrc(a, (uint32_t)(((ncols - 1) * lda + m) * (int64_t)sizeof(TIN)));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t c = (int64_t)ct * 32 + (lane >> 3) + 8 * j;
      const uint32_t voff = (uint32_t)((r + c * lda) * (int64_t)sizeof(TIN));
      float x[4];
      if constexpr (sizeof(TIN) == 4) {
        const u32v4 u = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, 0, 0);
        x[0] = __uint_as_float(u.x); x[1] = __uint_as_float(u.y);
        x[2] = __uint_as_float(u.z); x[3] = __uint_as_float(u.w);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = bload1<uint16_t>(rs, voff + 2 * i, 0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) mx = fmaxf(mx, r + i < m ? fabsf(x[i]) : 0.f);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) {
    float s = 1.f;
    if (mx > 0.f) {
      // mx = f 2^E with 0.5 <= f < 1, and 448 = 0.875 2^9: the smallest e with
      // mx <= 448 2^e is E - 9, or E - 8 when f > 0.875
      int E;
      const float f = frexpf(mx, &E);
      s = ldexpf(1.f, E - 9 + (f > 0.875f ? 1 : 0));
    }
    sc[tile] = s;
  }
}

// The staged test-matrix tiles go from HBM straight into LDS (no register
// staging): one instruction moves 16 bytes per lane into 1 KB of LDS, lane L
// writing bytes 16 L .. 16 L + 15 of the block.  A (plane, 16-row tile) block
// of a 32-wide step is laid out in the order the fragment reads want it:
// lane L = 16 g + c holds row c, contraction indices 8 g .. 8 g + 7 (bf16:
// one block; fp32: two blocks, indices 8g..8g+3 and 8g+4..8g+7), so a
// fragment read is one contiguous, conflict-free 1 KB wave access per block.
__device__ __forceinline__ void dma16(const void *src, void *lds_block) {
  __builtin_amdgcn_global_load_lds((const QSK_GLOBAL void *)src, (QSK_LDS void *)lds_block, 16, 0, 0);
}
// wait until this wave's loads (direct-to-LDS ones included) have landed
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }
// wait until at most N (< 64) of this wave's vector memory instructions are
// outstanding: they complete in issue order, so everything issued before the
// last N has landed
template <int N> __device__ __forceinline__ void wait_vm_but() {
  static_assert(N >= 0 && N < 64, "vmcnt");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0F70);
}
// vector memory instructions of one step's operand fetch of a lane
template <int OP, typename TIN, bool PURE> constexpr int a_fetch_loads(int per_plane) {
  return (PURE ? 3 : 4) * (per_plane + (OP == OP_FP8 ? 1 : 0));
}

template <typename Frag> __device__ __forceinline__ void dma_frag(const char *blk, int lane, Frag &f);
template <> __device__ __forceinline__ void dma_frag<FragB>(const char *blk, int lane, FragB &f) {
  const u32v4 u = *(const QSK_LDS u32v4 *)(blk + lane * 16);
  f.v[0] = u.x; f.v[1] = u.y; f.v[2] = u.z; f.v[3] = u.w;
}
template <> __device__ __forceinline__ void dma_frag<FragF>(const char *blk, int lane, FragF &f) {
  const floatx4 u0 = *(const QSK_LDS floatx4 *)(blk + lane * 16);
  const floatx4 u1 = *(const QSK_LDS floatx4 *)(blk + 1024 + lane * 16);
  f.v[0] = u0.x; f.v[1] = u0.y; f.v[2] = u0.z; f.v[3] = u0.w;
  f.v[4] = u1.x; f.v[5] = u1.y; f.v[6] = u1.z; f.v[7] = u1.w;
}

// ---------------------------------------------------------------------------
// Rademacher test-matrix tiles generated in place of the staged ones.  A
// step's tile holds rows o0 .. o0 + 16 ntiles - 1 of the test matrix (rows of
// Psi for W, columns of Omega for Y) at 32 consecutive contraction indices
// from tb, in the 1 KB LDS blocks [plane][tile] of the fragment layout (lane
// 16 g + c: row c of the tile, indices 8 g .. 8 g + 7 as bf16 +-1).  One
// Philox call serves 32 contraction indices of a row, 4 bits per entry (bit
// p: the sign of plane p), so one thread makes a whole row of the tile: one
// call when tb is a multiple of 32, two when the step straddles two calls
// (the entries tb .. tb + 31 are bits 4 (tb mod 32) .. of the two calls'
// 256 bits).  Rows at or past n_o are zero.  Row r goes to wave r mod 4,
// lane r / 4, so the four SIMDs share the work (waves 4 .. have none).

// bf16 +-1 pair of entries 2d, 2d + 1 of a plane whose sign bits sit at
// bits 8d and 8d + 4 of y
// The four words of bf16 +-1 pairs of one 32-bit sign word y: word d holds
// (-1)^bit(8d) in its low half and (-1)^bit(8d + 4) in its high half.  The
// sign bits are moved to bit 7 of each byte (s, t), then one byte permute
// per word places byte d of s and of t at the two sign positions.
__device__ __forceinline__ u32v4 rad_quad(uint32_t y) {
  const uint32_t s = (y << 7) & 0x80808080u, t = (y << 3) & 0x80808080u;
  u32v4 v;
  // selector bytes: 0x0c = zero byte, 0..3 = bytes of s, 4..7 = bytes of t
  v.x = __builtin_amdgcn_perm(t, s, 0x040c000cu) | 0x3F803F80u;
  v.y = __builtin_amdgcn_perm(t, s, 0x050c010cu) | 0x3F803F80u;
  v.z = __builtin_amdgcn_perm(t, s, 0x060c020cu) | 0x3F803F80u;
  v.w = __builtin_amdgcn_perm(t, s, 0x070c030cu) | 0x3F803F80u;
  return v;
}

__device__ __forceinline__ uint32_t pick_word(int wd, int i, const uint32_t (&z)[8]) {
  // z[wd + i] for wd in 0 .. 3, i in 0 .. 4, as selects (no indexed registers)
  const uint32_t a = i < 8 ? z[i] : 0u;
  const uint32_t b = i + 1 < 8 ? z[i + 1] : 0u;
  const uint32_t c = i + 2 < 8 ? z[i + 2] : 0u;
  const uint32_t d = i + 3 < 8 ? z[i + 3] : 0u;
  return wd == 0 ? a : (wd == 1 ? b : (wd == 2 ? c : d));
}

template <int NT>
__device__ __forceinline__ void rad_tile(char *lds, int64_t o0, int64_t n_o, int64_t tb, uint32_t stream,
                                         uint32_t k0, uint32_t k1, int wave, int lane) {
  if (wave >= 4) return;
  const int r = 4 * lane + wave;
  if (r >= 16 * NT) return;
  const int64_t o = o0 + r;
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  if (o < n_o) {
    const uint32_t c0 = (uint32_t)(tb >> 5), off = (uint32_t)(tb & 31);
    const u32x4 x = philox(c0, (uint32_t)o, stream, 1u, k0, k1);
    if (off == 0) {
      w[0] = x.x0; w[1] = x.x1; w[2] = x.x2; w[3] = x.x3;
    } else {
      const u32x4 y = philox(c0 + 1u, (uint32_t)o, stream, 1u, k0, k1);
      const uint32_t z[8] = {x.x0, x.x1, x.x2, x.x3, y.x0, y.x1, y.x2, y.x3};
      const int bit = (int)(4 * off), wd = bit >> 5, sh = bit & 31;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const uint32_t lo = pick_word(wd, g, z), hi = pick_word(wd, g + 1, z);
        w[g] = sh ? (lo >> sh) | (hi << (32 - sh)) : lo;
      }
    }
  }
  const int tile = r >> 4, c = r & 15;
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
      *(QSK_LDS u32v4 *)(lds + (pl * NT + tile) * 1024 + (16 * g + c) * 16) = rad_quad(w[g] >> pl);
    }
}

// ---------------------------------------------------------------------------
// W kernel.  Tiles: 64 columns of the update block x NMT row tiles of W
// (16 rows each) x one chunk of the rows of A (split K over S chunks).
// Block = 4H waves, H per SIMD: wave w owns columns 16 (w mod 4) .. + 15 of
// the tile and the w / 4-th of H slices of the NMT row tiles, all four
// planes.  With H = 2 one wave's loads, conversions and barrier waits overlap
// the other's matrix-core work.  Per 32-row step the Psi tile (4 planes x 16
// NMT rows x 32) goes HBM -> LDS directly (two buffers, one barrier per
// step); each lane's A values (8 consecutive rows of its column, four planes)
// come from HBM into registers.  Both are fetched one step ahead.
struct WArgs {
  const void *a[4];
  int64_t lda, m, ncols, col0;
  const void *psi;            // staged [4][LP][MP]
  int LP;
  int64_t MP;
  int l, pure, S, ctiles, rgroups;
  int64_t kchunk;
  float *w;
  int64_t ldw, psw;
  float *part;                // [S][4][ncols][LP]
  const float *fsc;           // fp8 tile scales [4][RT][CT] (OP_FP8)
  int RT, CT;
  float eta = 1.f;            // W += eta Psi H
  uint32_t k0 = 0, k1 = 0;    // Philox key (Psi tiles generated in the kernel)
};

// GEN: the Rademacher Psi tiles are generated in the kernel (rad_tile)
// instead of read from the staging buffer
template <int OP, typename TIN, int NMT, int TERMS, bool PURE, int H, bool GEN>
__global__ __launch_bounds__(256 * H) __attribute__((amdgpu_waves_per_eu(H, H))) void w_mfma_kernel(WArgs a0, GroupRef grp) {
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
  using OPT = typename std::conditional<!op_f32(OP), uint16_t, float>::type;
  using Frag = typename std::conditional<!op_f32(OP), FragB, FragF>::type;
  constexpr int NH = (NMT + H - 1) / H;                    // row tiles per wave
  constexpr int SUB = !op_f32(OP) ? 1 : 2;               // 1 KB blocks per (plane, row tile)
  constexpr int NBLK = 4 * NMT * SUB;                      // 1 KB blocks per step
  constexpr int NW = 4 * H;                                // waves per block
  __shared__ __attribute__((aligned(1024))) char s_psi[2][NBLK][1024];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c16 = lane & 15, g = lane >> 4;
  const int cg = wave & 3, hf = wave >> 2;
  const int bx = (int)(t % a.ctiles);
  const int by = (int)((t / a.ctiles) % a.rgroups);
  const int bz = (int)(t / ((int64_t)a.ctiles * a.rgroups));
  const int64_t j = (int64_t)bx * 64 + cg * 16 + c16;
  const int rbase = by * NMT * 16;
  const int rt0 = hf * NH;                                 // first row tile of this wave
  const int64_t ib = (int64_t)bz * a.kchunk;
  const int64_t ie = min(a.m, ib + a.kchunk);
  const OPT *psi = (const OPT *)a.psi;
  const int64_t pps = (int64_t)a.LP * a.MP;
  const uint32_t abytes = (uint32_t)(((a.ncols - 1) * a.lda + a.m) * (int64_t)sizeof(TIN));
  rsrc_t ar[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) ar[q] = make_rsrc(a.a[q], abytes);
  // byte offset of rows ib + 8g .. of column j (the host keeps every offset
  // of the block below 2^32; columns j >= ncols read zeros or other
  // columns' values and are never stored)
  uint32_t voff = (uint32_t)((ib + 8 * g + j * a.lda) * (int64_t)sizeof(TIN));
  const uint32_t vstep = 32u * (uint32_t)sizeof(TIN);
  // DMA sources: the step tile of row tile rt at step i is 1 KB (2 KB for
  // FP32) of contiguous staging, lane L takes 16 bytes at 16 L
  constexpr int CE = 16 / (int)sizeof(OPT);                // elements per lane and load
  const int lp16 = a.LP >> 4;
  const OPT *psrc = psi + (int64_t)(rbase >> 4) * 512 + lane * CE;

  floatx4 acc[NH][4];
#pragma unroll
  for (int r = 0; r < NH; ++r)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[r][p] = {0.f, 0.f, 0.f, 0.f};

  // The range check of a 16-byte load works per dword: with bf16 data the
  // dword that holds the block's last element, A[m-1, ncols-1], may reach
  // past the end of the buffer and read as zero.  That element is loaded on
  // its own once and put back where it belongs.
  float last[4] = {0.f, 0.f, 0.f, 0.f};
  const bool fix_last = sizeof(TIN) == 2 && j == a.ncols - 1 && ie == a.m;
  if constexpr (sizeof(TIN) == 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (!(q == 0 && PURE)) last[q] = bload1<TIN>(ar[q], abytes - 2, 0);
  }

  float xa[4][8];
  // fp8: the scales of this lane's tiles (rows of the step, column j)
  float scn[4] = {1.f, 1.f, 1.f, 1.f};
  const int sct = OP == OP_FP8 ? (int)min(j >> 5, (int64_t)a.CT - 1) : 0;
#define QSK_W_FETCH_A(I0)                                                                       \
  do {                                                                                          \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                             \
      if (q == 0 && PURE) {                                                                     \
        _Pragma("unroll") for (int s = 0; s < 8; ++s) xa[q][s] = 0.f;                           \
      } else {                                                                                  \
        bload8<TIN>(ar[q], voff, xa[q]);                                                        \
        if constexpr (OP == OP_FP8)                                                             \
          scn[q] = gp(a.fsc)[((int64_t)q * a.RT + min((int64_t)(I0) >> 5, (int64_t)a.RT - 1)) * a.CT + sct]; \
      }                                                                                         \
    }                                                                                           \
  } while (0)
#define QSK_W_DMA(I0, B)                                                                        \
  do {                                                                                          \
    if constexpr (GEN) {                                                                        \
      rad_tile<NMT>(&s_psi[B][0][0], rbase, a.l, (I0), STREAM_PSI, a.k0, a.k1, wave, lane);     \
      break;                                                                                    \
    }                                                                                           \
    _Pragma("unroll") for (int k_ = 0; k_ < (NBLK + NW - 1) / NW; ++k_) {                       \
      const int u_ = wave + k_ * NW;                                                            \
      if (u_ < NBLK) {                                                                          \
        const int sb_ = u_ % SUB, rt_ = (u_ / SUB) % NMT, pl_ = u_ / (SUB * NMT);               \
        dma16(psrc + pl_ * pps + ((I0) >> 5) * lp16 * 512 + rt_ * 512 + 64 * CE * sb_, &s_psi[B][u_][0]); \
      }                                                                                         \
    }                                                                                           \
  } while (0)

  QSK_W_FETCH_A(ib);
  QSK_W_DMA(ib, 0);
  wait_vm();
  __syncthreads();
  int buf = 0;
  for (int64_t i0 = ib; i0 < ie; i0 += 32) {
    // rows past the end hold other columns' values (or zeros): drop them
    const int64_t rem = ie - (i0 + 8 * g);
    Frag af[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        xa[q][s] = s < rem ? xa[q][s] : 0.f;
        if constexpr (sizeof(TIN) == 2) xa[q][s] = (fix_last && s == rem - 1) ? last[q] : xa[q][s];
      }
      to_frags<OP, TERMS>(xa[q], scn[q], af[q]);
    }
    Frag naf[4][3];
    neg_data<Frag, TERMS>(af, naf);
    voff += vstep;
    // the next step's test-matrix tile first, then its operand values, so
    // that the wait before the barrier can leave the latter in flight
    if (i0 + 32 < ie) QSK_W_DMA(i0 + 32, buf ^ 1);
    __builtin_amdgcn_sched_barrier(0);
    QSK_W_FETCH_A(i0 + 32);                                // next step (past the end: unused)
    __builtin_amdgcn_sched_barrier(0);
    // The products of a 16-row tile run grouped by Psi plane s; once group s
    // is issued the tile's plane-s fragment is dead, and plane s of the next
    // tile is read from LDS into the same registers while groups s + 1 ..
    // run, so the LDS latency stays hidden behind the matrix cores.  Tiles
    // that lie below NMT in every wave carry no branch.
    Frag pf[4];
    if ((H - 1) * NH < NMT || rt0 < NMT) {
#pragma unroll
      for (int s = 0; s < 4; ++s) dma_frag<Frag>(&s_psi[buf][(s * NMT + rt0) * SUB][0], lane, pf[s]);
    }
#pragma unroll
    for (int i = 0; i < NH; ++i) {
      const int rt = rt0 + i;
      if ((H - 1) * NH + i < NMT || rt < NMT) {
        const bool next = i + 1 < NH && ((H - 1) * NH + i + 1 < NMT || rt + 1 < NMT);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          Frag nps;
          if constexpr (!neg_on_data<TERMS>()) nps = negx(pf[s]);
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            const int q = w_q_of(p, s);
            if (q == 0 && PURE) continue;
            const bool ng = w_neg(p, s);
#pragma unroll
            for (int tm = 0; tm < TERMS; ++tm) {
              if constexpr (neg_on_data<TERMS>()) acc[i][p] = mma(pf[s], ng ? naf[q][tm] : af[q][tm], acc[i][p]);
              else acc[i][p] = mma(ng ? nps : pf[s], af[q][tm], acc[i][p]);
            }
          }
          if (next) dma_frag<Frag>(&s_psi[buf][(s * NMT + rt + 1) * SUB][0], lane, pf[s]);
        }
      }
    }
    wait_vm_but<a_fetch_loads<OP, TIN, PURE>(sizeof(TIN) == 4 ? 2 : 1)>();
    __syncthreads();
    buf ^= 1;
  }
  // epilogue: lane holds column j, rows rbase + rt*16 + 4g + (0..3)
  if (j >= a.ncols) return;
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    const int rt = rt0 + i;
    if (rt >= NMT) continue;
    const int r0 = rbase + rt * 16 + 4 * g;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      if (a.S == 1) {
        QSK_GLOBAL float *dst = gpw(a.w + p * a.psw + (a.col0 + j) * a.ldw);
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
          if (r0 + tt < a.l) dst[r0 + tt] += a.eta * acc[i][p][tt];
      } else {
        float *dst = a.part + (((int64_t)bz * 4 + p) * a.ncols + j) * a.LP + r0;
        *(QSK_GLOBAL floatx4 *)dst = acc[i][p];
      }
    }
  }
}

__global__ void w_reduce_kernel(const float *part, int S, int LP, int64_t ncols, int l, int64_t col0,
                                float *w, int64_t ldw, int64_t psw, float eta) {
  const int64_t total = 4 * ncols * (int64_t)l;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % l);
    const int64_t jp = e / l;
    const int64_t j = jp % ncols;
    const int p = (int)(jp / ncols);
    // four partials' loads in flight at a time, added in order
    float s = 0.f;
    int z = 0;
    for (; z + 4 <= S; z += 4) {
      float a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = gp(part)[(((int64_t)(z + u) * 4 + p) * ncols + j) * LP + r];
#pragma unroll
      for (int u = 0; u < 4; ++u) s += a[u];
    }
    for (; z < S; ++z) s += gp(part)[(((int64_t)z * 4 + p) * ncols + j) * LP + r];
    gpw(w)[p * psw + (col0 + j) * ldw + r] += eta * s;
  }
}

// The same sum for the problems of a batch whose W product was split:
// 256 entries of W per block.
struct WRedArgs {
  const float *part;
  int S, LP;
  int64_t ncols;
  int l;
  float *w;
  int64_t ldw, psw;
};
__global__ __launch_bounds__(256) void w_reduce_group_kernel(WRedArgs a0, GroupRef grp) {
  (void)a0;
  int pi;
  int64_t t;
  group_find(grp, &pi, &t);
  const WRedArgs a = ((const WRedArgs *)grp.tab)[pi];
  const int64_t e = t * 256 + threadIdx.x;
  if (e >= 4 * a.ncols * (int64_t)a.l) return;
  const int r = (int)(e % a.l);
  const int64_t jp = e / a.l;
  const int64_t j = jp % a.ncols;
  const int p = (int)(jp / a.ncols);
  float s = 0.f;
  for (int z = 0; z < a.S; ++z) s += gp(a.part)[(((int64_t)z * 4 + p) * a.ncols + j) * a.LP + r];
  gpw(a.w)[p * a.psw + j * a.ldw + r] += s;
}

// ---------------------------------------------------------------------------
// Y kernel.  Tiles: 64 H rows of A x NJ column tiles of Y (16 columns each)
// x one chunk of the update's columns (split K over S chunks; chunk s adds
// into its own copy s of Y, and the copies are summed when the sketch is
// read).  Block = 4H waves, H per SIMD: wave w owns rows 16 w .. 16 w + 15 of
// the tile and all NJ column tiles, all four planes.  Each lane loads its
// own operand values (row c16, columns 8 g .. 8 g + 7 of the step) from HBM;
// the Omega tile, which all waves share, goes HBM -> LDS directly (two
// buffers, one barrier per step).  Both are fetched one step ahead.
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
  const float *fsc;           // fp8 tile scales [4][RT][CT] (OP_FP8)
  int RT, CT;
  float eta = 1.f;            // Y += eta H Omega
  int64_t col0 = 0;           // first column of the block (Omega tiles generated in the kernel)
  uint32_t k0 = 0, k1 = 0;
};

// GEN: the Rademacher Omega tiles are generated in the kernel (rad_tile)
template <int OP, typename TIN, int NJ, int TERMS, bool PURE, int H, bool GEN>
__global__ __launch_bounds__(256 * H) __attribute__((amdgpu_waves_per_eu(H, H))) void y_mfma_kernel(YArgs a0, GroupRef grp) {
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
  using OPT = typename std::conditional<!op_f32(OP), uint16_t, float>::type;
  using Frag = typename std::conditional<!op_f32(OP), FragB, FragF>::type;
  constexpr int SUB = !op_f32(OP) ? 1 : 2;
  constexpr int NBLK = 4 * NJ * SUB;
  constexpr int NW = 4 * H;
  __shared__ __attribute__((aligned(1024))) char s_om[2][NBLK][1024];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c16 = lane & 15, g = lane >> 4;
  const int64_t bx = t % a.rblocks;
  const int by = (int)((t / a.rblocks) % a.cgroups);
  const int bz = (int)(t / ((int64_t)a.rblocks * a.cgroups));
  const int64_t rb = bx * 64 * H;
  const int jt0 = by * NJ;                                  // first column tile of the block
  const int64_t tb = (int64_t)bz * a.tchunk;
  const int64_t te = min(a.ncols, tb + a.tchunk);
  const OPT *om = (const OPT *)a.om;
  const int64_t ops = (int64_t)a.KP * a.NP;
  const uint32_t abytes = (uint32_t)(((a.ncols - 1) * a.lda + a.m) * (int64_t)sizeof(TIN));
  rsrc_t ar[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) ar[q] = make_rsrc(a.a[q], abytes);
  // this lane's row; rows >= m read other columns' values (or zeros) and
  // only feed rows of Y that are never stored; columns >= ncols lie past the
  // end of the buffer and read zeros (the host keeps every offset < 2^32)
  const int64_t row = rb + wave * 16 + c16;
  const uint32_t col_bytes = (uint32_t)(a.lda * (int64_t)sizeof(TIN));
  uint32_t voff = (uint32_t)((row + (tb + 8 * g) * a.lda) * (int64_t)sizeof(TIN));
  const uint32_t vstep = 32u * col_bytes;
  // DMA sources: the step tile of column tile jt at step t is 1 KB (2 KB for
  // FP32) of contiguous staging, lane L takes 16 bytes at 16 L
  constexpr int CE = 16 / (int)sizeof(OPT);                // elements per lane and load
  const int kp16 = a.KP >> 4;
  const OPT *osrc = om + (int64_t)jt0 * 512 + lane * CE;

  floatx4 acc[NJ][4];
#pragma unroll
  for (int u = 0; u < NJ; ++u)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[u][p] = {0.f, 0.f, 0.f, 0.f};

  // A values of the next step: xa[q][s] = A_q[row, T + 8 g + s]
  float xa[4][8];
  // fp8: the scales of this lane's tiles (its row, columns of the step)
  float scn[4] = {1.f, 1.f, 1.f, 1.f};
  const int64_t srt = OP == OP_FP8 ? min(row >> 5, (int64_t)a.RT - 1) : 0;
#define QSK_Y_FETCH_A(T0)                                                                       \
  do {                                                                                          \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                             \
      _Pragma("unroll") for (int s = 0; s < 8; ++s)                                             \
        xa[q][s] = (q == 0 && PURE) ? 0.f : bload1<TIN>(ar[q], voff, (uint32_t)s * col_bytes);  \
      if constexpr (OP == OP_FP8)                                                               \
        if (!(q == 0 && PURE))                                                                  \
          scn[q] = gp(a.fsc)[((int64_t)q * a.RT + srt) * a.CT + min((int64_t)(T0) >> 5, (int64_t)a.CT - 1)]; \
    }                                                                                           \
  } while (0)
#define QSK_Y_DMA(T0, B)                                                                        \
  do {                                                                                          \
    if constexpr (GEN) {                                                                        \
      rad_tile<NJ>(&s_om[B][0][0], (int64_t)jt0 * 16, a.k, a.col0 + (T0), STREAM_OMEGA, a.k0, a.k1, wave, lane); \
      break;                                                                                    \
    }                                                                                           \
    _Pragma("unroll") for (int k_ = 0; k_ < (NBLK + NW - 1) / NW; ++k_) {                       \
      const int u_ = wave + k_ * NW;                                                            \
      if (u_ < NBLK) {                                                                          \
        const int sb_ = u_ % SUB, jt_ = (u_ / SUB) % NJ, pl_ = u_ / (SUB * NJ);                 \
        dma16(osrc + pl_ * ops + ((T0) >> 5) * kp16 * 512 + jt_ * 512 + 64 * CE * sb_, &s_om[B][u_][0]); \
      }                                                                                         \
    }                                                                                           \
  } while (0)

  QSK_Y_FETCH_A(tb);
  QSK_Y_DMA(tb, 0);
  wait_vm();
  __syncthreads();
  int buf = 0;
  for (int64_t t0 = tb; t0 < te; t0 += 32) {
    Frag af[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q) to_frags<OP, TERMS>(xa[q], scn[q], af[q]);
    Frag naf[4][3];
    neg_data<Frag, TERMS>(af, naf);
    voff += vstep;
    QSK_Y_FETCH_A(t0 + 32);                                 // next step (past the end: unused)
    if (t0 + 32 < te) QSK_Y_DMA(t0 + 32, buf ^ 1);
    // grouped by Omega plane, the next column tile's fragments read during
    // the current tile's products (as in the W kernel)
    Frag of[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) dma_frag<Frag>(&s_om[buf][(s * NJ) * SUB][0], lane, of[s]);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        Frag nof;
        if constexpr (!neg_on_data<TERMS>()) nof = negx(of[s]);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int q = y_q_of(p, s);
          if (q == 0 && PURE) continue;
          const bool ng = y_neg(p, s);
#pragma unroll
          for (int tm = 0; tm < TERMS; ++tm) {
            if constexpr (neg_on_data<TERMS>()) acc[i][p] = mma(ng ? naf[q][tm] : af[q][tm], of[s], acc[i][p]);
            else acc[i][p] = mma(af[q][tm], ng ? nof : of[s], acc[i][p]);
          }
        }
        if (i + 1 < NJ) dma_frag<Frag>(&s_om[buf][(s * NJ + i + 1) * SUB][0], lane, of[s]);
      }
    }
    wait_vm();
    __syncthreads();
    buf ^= 1;
  }
  // epilogue: lane holds column (jt0 + i) * 16 + c16 of Y, rows rb + 16 wave + 4g + (0..3)
  const int64_t r0 = rb + wave * 16 + 4 * g;
  float *ys = a.y + bz * a.pss;
  const bool full = rb + 64 * H <= a.m && ((a.ldy | a.psy | a.pss) & 3) == 0;
  if (full) {
    // whole tile inside Y: 16-byte read-modify-writes through one buffer per
    // plane; columns past k get an offset past the end, so their loads read
    // zeros and their stores are dropped (no branches)
    rsrc_t yr[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) yr[p] = make_rsrc(ys + p * a.psy, (uint32_t)(a.psy * 4));
    floatx4 old[NJ][4];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
      const int jj = (jt0 + i) * 16 + c16;
      const uint32_t o = jj < a.k ? (uint32_t)((jj * a.ldy + r0) * 4) : 0xFFFFFFF0u;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const u32v4 u = __builtin_amdgcn_raw_buffer_load_b128(yr[p], o, 0, 0);
        old[i][p] = {__uint_as_float(u.x), __uint_as_float(u.y), __uint_as_float(u.z), __uint_as_float(u.w)};
      }
    }
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
      const int jj = (jt0 + i) * 16 + c16;
      const uint32_t o = jj < a.k ? (uint32_t)((jj * a.ldy + r0) * 4) : 0xFFFFFFF0u;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const floatx4 v = old[i][p] + a.eta * acc[i][p];
        const u32v4 u = {__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z), __float_as_uint(v.w)};
        __builtin_amdgcn_raw_buffer_store_b128(u, yr[p], o, 0, 0);
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    const int jj = (jt0 + i) * 16 + c16;
    if (jj >= a.k) continue;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      QSK_GLOBAL float *dst = gpw(ys + p * a.psy + (int64_t)jj * a.ldy);
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
        if (r0 + tt < a.m) dst[r0 + tt] += a.eta * acc[i][p][tt];
    }
  }
}

#undef QSK_W_FETCH_A
#undef QSK_W_DMA
#undef QSK_Y_FETCH_A
#undef QSK_Y_DMA

// Y = sum of its split-K copies: copy 0 += copies 1 .. S-1, which are cleared.
__global__ void y_fold_kernel(float *y, int64_t n_per_copy, int S) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_per_copy;
       e += (int64_t)gridDim.x * blockDim.x) {
    // the copies are read before any is cleared, and added in order
    float s = y[e];
    int c = 1;
    for (; c + 2 <= S; c += 2) {
      const float a0 = y[c * n_per_copy + e], a1 = y[(c + 1) * n_per_copy + e];
      y[c * n_per_copy + e] = 0.f;
      y[(c + 1) * n_per_copy + e] = 0.f;
      s += a0;
      s += a1;
    }
    for (; c < S; ++c) {
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

// Tile choices: NMT row tiles of W per block (from {4, 7, 8, 13}; 8 and 13
// only for bf16 operands, whose Psi tile is half the size) and NJ column tiles of Y
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
  static const int cb[4] = {4, 7, 8, 13}, cf[2] = {4, 7};
  return op_bf16 ? pick_tiles((l + 15) / 16, cb, 4) : pick_tiles((l + 15) / 16, cf, 2);
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

// tiled: the step-tile layout (psi_tiled_index; t_pad a multiple of 32,
// o_pad of 16) that the product kernels' direct-to-LDS loads read, else
// [plane][o][t] with t fastest
template <int MODE, typename OPT>
static hipError_t gen_stage(hipStream_t st, OPT *dst, int n_o, int o_pad, int64_t t0, int64_t n_t,
                            int64_t t_pad, uint32_t stream, int rad, uint32_t k0, uint32_t k1,
                            bool tiled = false) {
  const int64_t total = (int64_t)o_pad * t_pad;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((gen_stage_kernel<MODE, OPT>), dim3((unsigned)blocks), dim3(256), 0, st, dst,
                     n_o, o_pad, t0, n_t, t_pad, stream, rad, k0, k1, tiled ? 1 : 0);
  return hipGetLastError();
}

static inline void mark(const SketchArgs &s, int idx) {
  if (s.events) (void)hipEventRecord(s.events[idx], s.stream);
}

// Waves per SIMD of the two kernels (the block has 4 H waves).
#ifndef QSK_W_WAVES
#define QSK_W_WAVES 2
#endif
#ifndef QSK_Y_WAVES
#define QSK_Y_WAVES 2
#endif
template <int OP> constexpr int w_waves() { return !op_f32(OP) ? QSK_W_WAVES : 1; }
template <int OP> constexpr int y_waves() { return !op_f32(OP) ? QSK_Y_WAVES : 1; }

// `pure` (no real plane) is a template parameter so that the product
// sequences have no branches
// gen: Rademacher test-matrix tiles generated in the kernel (bf16 operands)
template <int OP, typename TIN, int TERMS, int NMT>
static void launch_w(const WArgs &w, int64_t blocks, hipStream_t st, GroupRef g = GroupRef{}, bool gen = false) {
  constexpr int H = w_waves<OP>();
  if constexpr (!op_f32(OP)) {
    if (gen) {
      if (w.pure)
        hipLaunchKernelGGL((w_mfma_kernel<OP, TIN, NMT, TERMS, true, H, true>), dim3((unsigned)blocks), dim3(256 * H), 0, st, w, g);
      else
        hipLaunchKernelGGL((w_mfma_kernel<OP, TIN, NMT, TERMS, false, H, true>), dim3((unsigned)blocks), dim3(256 * H), 0, st, w, g);
      return;
    }
  }
  if (w.pure)
    hipLaunchKernelGGL((w_mfma_kernel<OP, TIN, NMT, TERMS, true, H, false>), dim3((unsigned)blocks), dim3(256 * H), 0, st, w, g);
  else
    hipLaunchKernelGGL((w_mfma_kernel<OP, TIN, NMT, TERMS, false, H, false>), dim3((unsigned)blocks), dim3(256 * H), 0, st, w, g);
}
template <int OP, typename TIN, int TERMS, int NJ>
static void launch_y(const YArgs &y, int64_t blocks, hipStream_t st, GroupRef g = GroupRef{}, bool gen = false) {
  constexpr int H = y_waves<OP>();
  if constexpr (!op_f32(OP)) {
    if (gen) {
      if (y.pure)
        hipLaunchKernelGGL((y_mfma_kernel<OP, TIN, NJ, TERMS, true, H, true>), dim3((unsigned)blocks), dim3(256 * H), 0, st, y, g);
      else
        hipLaunchKernelGGL((y_mfma_kernel<OP, TIN, NJ, TERMS, false, H, true>), dim3((unsigned)blocks), dim3(256 * H), 0, st, y, g);
      return;
    }
  }
  if (y.pure)
    hipLaunchKernelGGL((y_mfma_kernel<OP, TIN, NJ, TERMS, true, H, false>), dim3((unsigned)blocks), dim3(256 * H), 0, st, y, g);
  else
    hipLaunchKernelGGL((y_mfma_kernel<OP, TIN, NJ, TERMS, false, H, false>), dim3((unsigned)blocks), dim3(256 * H), 0, st, y, g);
}
// Blocks of 4 H waves resident at once on the device: every CU holds two
// waves per SIMD of these kernels (their register budget).
static int64_t resident_blocks(int H) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cus = n;
    else
      cus = 256;
  }
  return (int64_t)cus * std::max(1, 2 / H);
}

// Split count S in [1, smax] of a grid of base * S blocks: the largest
// fraction of busy slots in the last round of `slots` resident blocks; among
// equal fractions the fewest splits that still fill every slot once.
static int64_t pick_split(int64_t base, int64_t smax, int64_t slots) {
  int64_t best = 1;
  double best_u = -1.0;
  bool best_full = false;
  for (int64_t S = 1; S <= smax; ++S) {
    const int64_t b = base * S;
    const int64_t rounds = (b + slots - 1) / slots;
    const double u = std::floor(100.0 * (double)b / (double)(rounds * slots)) / 100.0;
    const bool full = b >= slots;
    if (u > best_u || (u == best_u && full && !best_full)) {
      best = S;
      best_u = u;
      best_full = full;
    }
  }
  return best;
}

// Rows of A per Y block.
template <int OP> constexpr int y_rows() { return 64 * y_waves<OP>(); }

// The Y epilogue addresses a plane of Y (m x k fp32) with 32-bit offsets.
static bool y_plane_fits(int64_t m, int64_t k) { return (uint64_t)m * k * 4 < 0xFFFFFFF0ull; }

// Both kernels address a plane of the update block with 32-bit byte offsets,
// including the rows and columns that whole tiles and steps run past the
// end (which read zeros or values that are never used).
template <typename TIN>
static bool offsets_fit(int64_t m, int64_t ncols, int64_t lda) {
  return (uint64_t)((ncols + 64) * lda + rup(m, 128) + 64) * sizeof(TIN) < (1ull << 32);
}

// Whether an update's test-matrix tiles are generated inside the product
// kernels (Rademacher with bf16 operands) rather than staged.
bool gen_in_kernel(const SketchArgs &s) {
  return s.rad && s.gen_rad && (s.mode == MODE_BF16 || s.mode == MODE_FP8);
}

template <int OP, typename TIN, int TERMS>
static hipError_t launch_t(const SketchArgs &s, const MfmaStage &g) {
  using OPT = typename std::conditional<!op_f32(OP), uint16_t, float>::type;
  if (!offsets_fit<TIN>(s.m, s.ncols, s.lda) || !y_plane_fits(s.m, s.k)) return hipErrorNotSupported;
  hipError_t e;
  mark(s, 0);
  // Rademacher test matrices with bf16 operands are generated inside the
  // product kernels; otherwise regenerate Omega_J in the operand format,
  // and Psi once (it is the same for every block)
  const bool gen = gen_in_kernel(s);
  OPT *om = (OPT *)g.omega;
  OPT *ps = (OPT *)g.psi;
  const int64_t NPu = rup(s.ncols, 32);
  if (gen) {
    // nothing staged
  } else if (s.mode == MODE_BF16) {
    e = gen_stage<MODE_BF16, OPT>(s.stream, om, s.k, g.KP, s.col0, s.ncols, NPu, STREAM_OMEGA, s.rad, s.k0, s.k1, true);
    if (e != hipSuccess) return e;
    if (!s.psi_ready && !s.skip_w) e = gen_stage<MODE_BF16, OPT>(s.stream, ps, s.l, g.LP, 0, s.m, g.MP, STREAM_PSI, s.rad, s.k0, s.k1, true);
    if (e != hipSuccess) return e;
  } else if (s.mode == MODE_FP8) {
    // e4m3 test-matrix values, staged as (exact) bf16
    e = gen_stage<MODE_FP8, OPT>(s.stream, om, s.k, g.KP, s.col0, s.ncols, NPu, STREAM_OMEGA, s.rad, s.k0, s.k1, true);
    if (e != hipSuccess) return e;
    if (!s.psi_ready && !s.skip_w) e = gen_stage<MODE_FP8, OPT>(s.stream, ps, s.l, g.LP, 0, s.m, g.MP, STREAM_PSI, s.rad, s.k0, s.k1, true);
    if (e != hipSuccess) return e;
  } else {
    e = gen_stage<MODE_F32, OPT>(s.stream, om, s.k, g.KP, s.col0, s.ncols, NPu, STREAM_OMEGA, s.rad, s.k0, s.k1, true);
    if (e != hipSuccess) return e;
    if (!s.psi_ready && !s.skip_w) e = gen_stage<MODE_F32, OPT>(s.stream, ps, s.l, g.LP, 0, s.m, g.MP, STREAM_PSI, s.rad, s.k0, s.k1, true);
    if (e != hipSuccess) return e;
  }
  // fp8: the tile scales of this block
  const int RT = (int)((s.m + 31) / 32), CT = (int)((s.ncols + 31) / 32);
  if constexpr (OP == OP_FP8) {
    if (!s.fp8_scales || 4 * (int64_t)RT * CT > s.fp8_scale_elems) return hipErrorInvalidValue;
    const int64_t tiles = 4 * (int64_t)RT * CT;
    hipLaunchKernelGGL(fp8_scale_kernel<TIN>, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s.stream,
                       s.planes[0], s.planes[1], s.planes[2], s.planes[3], s.lda, s.m, s.ncols, s.pure,
                       RT, CT, s.fp8_scales);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  mark(s, 1);
  // ---- Y
  {
    mark(s, 2);
    YArgs y{};
    y.fsc = s.fp8_scales; y.RT = RT; y.CT = CT;
    for (int p = 0; p < 4; ++p) y.a[p] = s.planes[p];
    y.lda = s.lda; y.m = s.m; y.ncols = s.ncols;
    y.om = om; y.KP = g.KP; y.NP = NPu;
    y.k = s.k; y.pure = s.pure; y.eta = (float)s.eta;
    y.col0 = s.col0; y.k0 = s.k0; y.k1 = s.k1;
    y.y = (float *)s.y; y.ldy = s.ldy; y.psy = s.psy; y.pss = s.pss;
    const int nj = y_nj(s.k);
    const int ntiles = (s.k + 15) / 16;
    y.rblocks = (int)((s.m + y_rows<OP>() - 1) / y_rows<OP>());
    y.cgroups = (ntiles + nj - 1) / nj;
    // split the update's columns over the Y copies, the grid's last round
    // of resident blocks as full as possible
    int64_t S = pick_split((int64_t)y.rblocks * y.cgroups, std::min<int64_t>(s.y_copies, (s.ncols + 31) / 32),
                           resident_blocks(y_waves<OP>()));
    int64_t tchunk = rup((s.ncols + S - 1) / S, 32);
    S = (s.ncols + tchunk - 1) / tchunk;
    y.S = (int)S; y.tchunk = tchunk;
    if (s.y_splits) *s.y_splits = (int)S;
    const int64_t blocks = (int64_t)y.rblocks * y.cgroups * S;
    if (nj == 7) launch_y<OP, TIN, TERMS, 7>(y, blocks, s.stream, GroupRef{}, gen);
    else launch_y<OP, TIN, TERMS, 4>(y, blocks, s.stream, GroupRef{}, gen);
    e = hipGetLastError();
    mark(s, 3);
    if (e != hipSuccess) return e;
  }
  // ---- W
  if (!s.skip_w) {
    WArgs w{};
    w.fsc = s.fp8_scales; w.RT = RT; w.CT = CT;
    for (int p = 0; p < 4; ++p) w.a[p] = s.planes[p];
    w.lda = s.lda; w.m = s.m; w.ncols = s.ncols; w.col0 = s.col0;
    w.psi = ps; w.LP = g.LP; w.MP = g.MP;
    w.l = s.l; w.pure = s.pure; w.eta = (float)s.eta;
    w.k0 = s.k0; w.k1 = s.k1;
    w.w = (float *)s.w; w.ldw = s.ldw; w.psw = s.psw;
    const int nmt = w_nmt(s.l, !op_f32(OP));
    w.rgroups = (int)(g.LP / (16 * nmt));
    w.ctiles = (int)((s.ncols + 63) / 64);
    // split the rows of A (chunks of at least 256 rows, partials within the
    // scratch buffer), the grid's last round of resident blocks as full as
    // possible
    const int64_t base = (int64_t)w.ctiles * w.rgroups;
    const int64_t per_split = 4 * s.ncols * (int64_t)g.LP * 4;
    const int64_t smax = std::max<int64_t>(1, std::min<int64_t>(s.m / 256, s.scratch_bytes / per_split));
    int64_t S = pick_split(base, smax, resident_blocks(w_waves<OP>()));
    int64_t kchunk = rup((s.m + S - 1) / S, 32);
    if (kchunk < 256) kchunk = 256;
    S = (s.m + kchunk - 1) / kchunk;
    const int64_t need = S * 4 * s.ncols * (int64_t)g.LP * 4;
    if (S > 1 && need > s.scratch_bytes) { S = 1; kchunk = rup(s.m, 32); }
    w.S = (int)S; w.kchunk = kchunk; w.part = (float *)s.scratch;
    const int64_t blocks = base * S;
    mark(s, 4);
    if (nmt == 13) launch_w<OP, TIN, TERMS, (!op_f32(OP) ? 13 : 7)>(w, blocks, s.stream, GroupRef{}, gen);
    else if (nmt == 8) launch_w<OP, TIN, TERMS, (!op_f32(OP) ? 8 : 7)>(w, blocks, s.stream, GroupRef{}, gen);
    else if (nmt == 7) launch_w<OP, TIN, TERMS, 7>(w, blocks, s.stream, GroupRef{}, gen);
    else launch_w<OP, TIN, TERMS, 4>(w, blocks, s.stream, GroupRef{}, gen);
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
                         s.ldw, s.psw, (float)s.eta);
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
  static const int cb[4] = {4, 7, 8, 13}, cf[2] = {4, 7}, cy[2] = {4, 7};
  const int *cw = op_bf16 ? cb : cf;
  const int ncw = op_bf16 ? 4 : 2;
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

// Psi alone into its staging buffer, with the values a sketch of s.mode uses
// (P = Psi Q reads it there when the update kernels generated Psi in place).
hipError_t stage_psi(const SketchArgs &s, const MfmaStage &g) {
  if (s.mode == MODE_BF16)
    return gen_stage<MODE_BF16, uint16_t>(s.stream, (uint16_t *)g.psi, s.l, g.LP, 0, s.m, g.MP, STREAM_PSI,
                                          s.rad, s.k0, s.k1, true);
  if (s.mode == MODE_FP8 || s.mode == MODE_FP8X)
    return gen_stage<MODE_FP8, uint16_t>(s.stream, (uint16_t *)g.psi, s.l, g.LP, 0, s.m, g.MP, STREAM_PSI,
                                         s.rad, s.k0, s.k1, true);
  if (s.mode == MODE_F32)
    return gen_stage<MODE_F32, float>(s.stream, (float *)g.psi, s.l, g.LP, 0, s.m, g.MP, STREAM_PSI, s.rad,
                                      s.k0, s.k1, true);
  return hipErrorNotSupported;
}

hipError_t stage_test_matrices(const SketchArgs &s, const MfmaStage &g) {
  if (s.mode == MODE_BF16) {
    hipError_t e = gen_stage<MODE_BF16, uint16_t>(s.stream, (uint16_t *)g.omega, s.k, g.KP, 0, s.ncols,
                                                  g.NP, STREAM_OMEGA, s.rad, s.k0, s.k1, true);
    if (e != hipSuccess) return e;
    return gen_stage<MODE_BF16, uint16_t>(s.stream, (uint16_t *)g.psi, s.l, g.LP, 0, s.m, g.MP,
                                          STREAM_PSI, s.rad, s.k0, s.k1, true);
  }
  if (s.mode == MODE_F32) {
    hipError_t e = gen_stage<MODE_F32, float>(s.stream, (float *)g.omega, s.k, g.KP, 0, s.ncols, g.NP,
                                              STREAM_OMEGA, s.rad, s.k0, s.k1, true);
    if (e != hipSuccess) return e;
    return gen_stage<MODE_F32, float>(s.stream, (float *)g.psi, s.l, g.LP, 0, s.m, g.MP, STREAM_PSI,
                                      s.rad, s.k0, s.k1, true);
  }
  return hipErrorNotSupported;
}

template <int OP, typename TIN, int TERMS>
static hipError_t launch_batch_t(const SketchArgs *s, const MfmaStage *g, int count, int nmt, int nj,
                                 ArgArena &ar, int wblocks) {
  std::vector<YArgs> ys(count);
  std::vector<WArgs> ws(count);
  std::vector<int64_t> py(count + 1, 0), pw(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    const SketchArgs &q = s[i];
    if (!offsets_fit<TIN>(q.m, q.ncols, q.lda) || !y_plane_fits(q.m, q.k)) return hipErrorNotSupported;
    YArgs &y = ys[i];
    for (int p = 0; p < 4; ++p) y.a[p] = q.planes[p];
    y.lda = q.lda; y.m = q.m; y.ncols = q.ncols;
    y.om = g[i].omega; y.KP = g[i].KP; y.NP = g[i].NP;
    y.k = q.k; y.pure = q.pure;
    y.y = (float *)q.y; y.ldy = q.ldy; y.psy = q.psy; y.pss = 0;
    y.rblocks = (int)((q.m + y_rows<OP>() - 1) / y_rows<OP>());
    y.cgroups = g[i].KP / (16 * nj);
    y.S = 1; y.tchunk = rup(q.ncols, 32);
    py[i + 1] = py[i] + (int64_t)y.rblocks * y.cgroups;
    WArgs &w = ws[i];
    for (int p = 0; p < 4; ++p) w.a[p] = q.planes[p];
    w.lda = q.lda; w.m = q.m; w.ncols = q.ncols; w.col0 = 0;
    w.psi = g[i].psi; w.LP = g[i].LP; w.MP = g[i].MP;
    w.l = q.l; w.pure = q.pure;
    w.w = (float *)q.w; w.ldw = q.ldw; w.psw = q.psw;
    w.rgroups = g[i].LP / (16 * nmt);
    w.ctiles = (int)((q.ncols + 63) / 64);
    w.S = 1; w.kchunk = rup(q.m, 32); w.part = nullptr;
  }
  // W: the rows of A split so that the blocks of all problems cover about
  // the same number of rows (about `wblocks` blocks in all, at least 256
  // rows, at most 8 splits, partial sums within the problem's scratch)
  int64_t work = 0;
  for (int i = 0; i < count; ++i) work += (int64_t)ws[i].ctiles * ws[i].rgroups * ws[i].m;
  const int64_t wchunk = std::max<int64_t>(256, rup(work / std::max(wblocks, 1), 32));
  std::vector<WRedArgs> rs;
  std::vector<int64_t> rb;
  for (int i = 0; i < count; ++i) {
    WArgs &w = ws[i];
    const SketchArgs &q = s[i];
    const int64_t per_split = 4 * q.ncols * (int64_t)w.LP * 4;
    int64_t S = std::min<int64_t>(8, (w.m + wchunk - 1) / wchunk);
    if (!q.scratch) S = 1;
    S = std::min<int64_t>(S, std::max<int64_t>(1, q.scratch_bytes / per_split));
    if (S > 1) {
      w.kchunk = rup((w.m + S - 1) / S, 32);
      S = (w.m + w.kchunk - 1) / w.kchunk;
    }
    if (S > 1) {
      w.S = (int)S;
      w.part = (float *)q.scratch;
      WRedArgs r{};
      r.part = w.part; r.S = w.S; r.LP = w.LP; r.ncols = q.ncols; r.l = q.l;
      r.w = (float *)q.w; r.ldw = q.ldw; r.psw = q.psw;
      rs.push_back(r);
      rb.push_back((4 * q.ncols * (int64_t)q.l + 255) / 256);
    } else {
      w.S = 1; w.kchunk = rup(w.m, 32); w.part = nullptr;
    }
    pw[i + 1] = pw[i] + (int64_t)w.ctiles * w.rgroups * w.S;
  }
  // Blocks are dispatched in table order; the problems whose blocks run
  // longest (most columns for Y, the longest row chunk for W) go first so
  // that they do not form the tail of the launch.
  std::vector<int> oy(count), ow(count);
  for (int i = 0; i < count; ++i) oy[i] = ow[i] = i;
  std::stable_sort(oy.begin(), oy.end(), [&](int a, int b) { return ys[a].ncols > ys[b].ncols; });
  std::stable_sort(ow.begin(), ow.end(), [&](int a, int b) { return ws[a].kchunk > ws[b].kchunk; });
  std::vector<YArgs> ys2(count);
  std::vector<WArgs> ws2(count);
  for (int i = 0; i < count; ++i) {
    ys2[i] = ys[oy[i]];
    ws2[i] = ws[ow[i]];
    py[i + 1] = py[i] + (int64_t)ys2[i].rblocks * ys2[i].cgroups;
    pw[i + 1] = pw[i] + (int64_t)ws2[i].ctiles * ws2[i].rgroups * ws2[i].S;
  }
  ys.swap(ys2);
  ws.swap(ws2);
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
  if (nmt == 13) launch_w<OP, TIN, TERMS, (!op_f32(OP) ? 13 : 7)>(ws[0], pw[count], st, gw);
  else if (nmt == 8) launch_w<OP, TIN, TERMS, (!op_f32(OP) ? 8 : 7)>(ws[0], pw[count], st, gw);
  else if (nmt == 7) launch_w<OP, TIN, TERMS, 7>(ws[0], pw[count], st, gw);
  else launch_w<OP, TIN, TERMS, 4>(ws[0], pw[count], st, gw);
  e = hipGetLastError();
  if (e != hipSuccess || rs.empty()) return e;
  std::vector<int64_t> pr(rs.size() + 1, 0);
  for (size_t i = 0; i < rs.size(); ++i) pr[i + 1] = pr[i] + rb[i];
  GroupRef gr{arena_push(ar, st, rs.data(), rs.size() * sizeof(WRedArgs)),
              (const int64_t *)arena_push(ar, st, pr.data(), pr.size() * sizeof(int64_t)), (int)rs.size()};
  if (!gr.tab || !gr.prefix) return hipErrorOutOfMemory;
  hipLaunchKernelGGL(w_reduce_group_kernel, dim3((unsigned)pr.back()), dim3(256), 0, st, rs[0], gr);
  return hipGetLastError();
}

hipError_t launch_sketch_mfma_batch(const SketchArgs *s, const MfmaStage *g, int count, int nmt,
                                    int nj, ArgArena &ar, int wblocks) {
  if (count < 1) return hipSuccess;
  const SketchArgs &a = s[0];
  if (a.mode == MODE_BF16) {
    if (a.in_dtype == DT_F32) {
      if (a.terms == 1) return launch_batch_t<OP_BF16, float, 1>(s, g, count, nmt, nj, ar, wblocks);
      if (a.terms == 2) return launch_batch_t<OP_BF16, float, 2>(s, g, count, nmt, nj, ar, wblocks);
      return launch_batch_t<OP_BF16, float, 3>(s, g, count, nmt, nj, ar, wblocks);
    }
    if (a.in_dtype == DT_BF16) return launch_batch_t<OP_BF16, uint16_t, 1>(s, g, count, nmt, nj, ar, wblocks);
  } else if (a.mode == MODE_F32) {
    if (a.in_dtype == DT_F32) return launch_batch_t<OP_F32, float, 1>(s, g, count, nmt, nj, ar, wblocks);
    if (a.in_dtype == DT_BF16) return launch_batch_t<OP_F32, uint16_t, 1>(s, g, count, nmt, nj, ar, wblocks);
  }
  return hipErrorNotSupported;
}

// ===========================================================================
// FP8X: the data as T e4m3 terms with the 32 x 32 tile scales, all terms on
// the fp8 matrix cores (v_mfma_scale_f32_16x16x128_f8f6f4, E8M0 block
// scales, FP32 accumulation).  Term t of a value x quantises what the
// earlier terms left at scale sc 16^-t (sc: the tile scale), so the operand
// is sum_t q_t sc 16^-t with every q_t an e4m3 value.
//
// The update block is quantised once per update (fp8x_quant_kernel) into
// bytes in two layouts: columns of rows (rows contiguous) for the W product,
// whose contraction runs over the rows of A, and rows of columns (columns
// contiguous) for the Y product, whose contraction runs over the columns;
// the products then only move bytes and issue matrix-core instructions.
// The test matrices are staged as e4m3 bytes.
//
// Operand layout of the instruction (16 x 128 A, 128 x 16 B; checked on the
// device): lane L = r + 16 g (r: row of A, column of B) holds 32 bytes,
// bytes 0-15 the contraction indices 16 g .. 16 g + 15 and bytes 16-31 the
// indices 64 + 16 g .. 64 + 16 g + 15; the E8M0 scale of indices
// 32 b .. 32 b + 31 is byte 0 of the scale operand of lane r + 16 b.  With
// the 128 indices of a step in order, scale block b is rows (W) or columns
// (Y) 32 b .. 32 b + 31 of the step: one tile of the data scales, whose
// exponent lane r + 16 b supplies.
typedef __attribute__((ext_vector_type(8))) int i32x8;

__device__ __forceinline__ uint32_t e4m3_byte(float e4m3_value) {   // exact for e4m3 values
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(e4m3_value, 0.f, 0, false) & 0xFFu;
}

// Fragment-ordered 2 KB blocks of e4m3 bytes (the layout of the quantised
// data and of the staged test matrices): 16 indices r (rows of an A operand,
// columns of a B operand) x 128 contraction indices kk, byte (r, kk) at
// (kk / 64) 1024 + (r + 16 ((kk mod 64) / 16)) 16 + kk mod 16.  Lane
// L = r + 16 g of the fp8 instruction takes its 32 operand bytes as the 16
// bytes at 16 L and at 1024 + 16 L, so each load or direct-to-LDS copy of a
// block moves 1 KB of consecutive bytes; a staged tile keeps this order in
// LDS.  Blocks follow each other along kk (the contraction) fastest.
__host__ __device__ constexpr int frag8_off(int r, int kk) {
  return (kk >> 6) * 1024 + (r + 16 * ((kk & 63) >> 4)) * 16 + (kk & 15);
}

struct QuantArgs {
  const void *a[4];
  int64_t lda, m, ncols;
  int pure, RT, CT, T;
  float *fsc;                 // out: tile scales [4][RT][CT]
  uint8_t *qw;                // [q][t]: blocks (16 columns, 128 rows), rows fastest
  uint8_t *qy;                // [q][t]: blocks (16 rows, 128 columns), columns fastest
  int64_t RP, CPW, CP;
};

// Value of an e4m3 byte (OCP e4m3fn; the quantisation never produces NaN).
__device__ __forceinline__ float e4m3_value(uint32_t b) {
  const uint32_t e = (b >> 3) & 15u, mt = b & 7u;
  const float v = e ? __uint_as_float(((e + 120u) << 23) | (mt << 20)) : (float)mt * 0x1p-9f;
  return (b & 0x80u) ? -v : v;
}

// One block per 128 x 128 piece of one plane of the padded block (4 x 4
// tiles of 32 x 32): the tile scales (the smallest power of two sc with
// amax / sc <= 448, 1 for an all-zero tile), then the T e4m3 terms of every
// value, one term at a time staged in LDS in both byte layouts and written
// out column by column (qw: 128 bytes of each column) and row by row (qy:
// 128 bytes of each row).  Every global access instruction covers whole 128-byte runs:
// thread t loads 4 consecutive rows (16 bytes of FP32) of column
// (t / 8) + 32 j at rows 32 s + 4 (t mod 8), j, s = 0..3, so 8 lanes read one
// 32-row run of a column; the stores move 16 bytes per lane, 8 lanes per
// column (qw) or row (qy).  Values outside the block are zero.  The e4m3
// rounding is the hardware's round-to-nearest-even conversion; the inputs
// are within range (|x / sc| <= 448 for term 0, <= 256 after it).
constexpr int QLD = 144;                 // LDS row of 128 bytes, padded
template <typename TIN>
__global__ __launch_bounds__(256) void fp8x_quant_kernel(QuantArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t s_qw[128][QLD];      // [column][row]
  __shared__ __attribute__((aligned(16))) uint8_t s_qy[128][QLD];      // [row][column]
  __shared__ float s_red[4][16];
  __shared__ float s_sc[16];
  const int q = blockIdx.z;
  if (q == 0 && a.pure) return;
  const int64_t r0 = (int64_t)blockIdx.x * 128, c0 = (int64_t)blockIdx.y * 128;
  const int tid = threadIdx.x, l8 = tid & 7, cg = tid >> 3, lane = tid & 63, wave = tid >> 6;
  const rsrc_t rs = make_rsrc(a.a[q], (uint32_t)(((a.ncols - 1) * a.lda + a.m) * (int64_t)sizeof(TIN)));
  // x[j][s][i]: row r0 + 32 s + 4 l8 + i of column c0 + cg + 32 j
  float x[4][4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t c = c0 + cg + 32 * j;
    const bool colok = c < a.ncols;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t r = r0 + 32 * s + 4 * l8;
      const uint32_t off = (uint32_t)(((colok ? c : 0) * a.lda + r) * (int64_t)sizeof(TIN));
      float v[4];
      if constexpr (sizeof(TIN) == 4) {
        const u32v4 u = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        v[0] = __uint_as_float(u.x); v[1] = __uint_as_float(u.y); v[2] = __uint_as_float(u.z); v[3] = __uint_as_float(u.w);
      } else {
        // 2-byte loads: exact range checks and no alignment requirement
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = bload1<uint16_t>(rs, off + 2u * i, 0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) x[j][s][i] = (colok && r + i < a.m) ? v[i] : 0.f;
    }
  }
  // tile maxima: tile (s, j) over this thread's 4 values, the wave, then the
  // four waves
  float mx[16];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int s = 0; s < 4; ++s)
      mx[4 * s + j] = fmaxf(fmaxf(fabsf(x[j][s][0]), fabsf(x[j][s][1])), fmaxf(fabsf(x[j][s][2]), fabsf(x[j][s][3])));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int u = 0; u < 16; ++u) mx[u] = fmaxf(mx[u], __shfl_xor(mx[u], off, 64));
  if (lane < 16) {
    float v = mx[0];
#pragma unroll
    for (int u = 1; u < 16; ++u) v = lane == u ? mx[u] : v;
    s_red[wave][lane] = v;
  }
  __syncthreads();
  if (tid < 16) {
    const float m4 = fmaxf(fmaxf(s_red[0][tid], s_red[1][tid]), fmaxf(s_red[2][tid], s_red[3][tid]));
    float sc = 1.f;
    if (m4 > 0.f) {
      // m4 = f 2^E with 0.5 <= f < 1 and 448 = 0.875 2^9: the smallest e with
      // m4 <= 448 2^e is E - 9, or E - 8 when f > 0.875
      int E;
      const float f = frexpf(m4, &E);
      sc = ldexpf(1.f, E - 9 + (f > 0.875f ? 1 : 0));
    }
    s_sc[tid] = sc;
    const int rt = tid >> 2, ct = tid & 3;
    const int64_t grt = r0 / 32 + rt, gct = c0 / 32 + ct;
    if (grt < a.RT && gct < a.CT) gpw(a.fsc)[((int64_t)q * a.RT + grt) * a.CT + gct] = sc;
  }
  __syncthreads();
  // terms: 4 bytes per (j, s) and term, one word into the column layout and
  // four bytes into the row layout; then the stores, 16 bytes per lane:
  // piece id = tid + 256 v of the eight 2 KB blocks of the piece, block
  // id / 128, 16 bytes w = id mod 128 at (r, kk) = (w mod 16, 64 (w / 64) +
  // 16 ((w mod 64) / 16))
  for (int t = 0; t < a.T; ++t) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float sc = s_sc[4 * s + j];
        const float st = ldexpf(sc, -4 * t), inv = ldexpf(1.f / sc, 4 * t);   // powers of two
        const uint32_t p01 = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x[j][s][0] * inv, x[j][s][1] * inv, 0, false);
        const uint32_t p23 = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x[j][s][2] * inv, x[j][s][3] * inv, 0, false);
        const uint32_t b[4] = {p01 & 0xFFu, (p01 >> 8) & 0xFFu, p23 & 0xFFu, (p23 >> 8) & 0xFFu};
#pragma unroll
        for (int i = 0; i < 4; ++i) x[j][s][i] -= e4m3_value(b[i]) * st;                // exact
        const int col = cg + 32 * j, row = 32 * s + 4 * l8;
        *(QSK_LDS uint32_t *)&s_qw[col][row] = b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24);
#pragma unroll
        for (int i = 0; i < 4; ++i) s_qy[row + i][col] = (uint8_t)b[i];
      }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int id = tid + 256 * v, blk = id >> 7, w = id & 127;
      const int r = w & 15, kk = 64 * (w >> 6) + 16 * ((w & 63) >> 4);
      if (c0 + 16 * blk < a.CPW) {
        QSK_GLOBAL u32v4 *dst = (QSK_GLOBAL u32v4 *)(gpw(a.qw) + ((int64_t)q * a.T + t) * a.CPW * a.RP +
                                                     ((c0 / 16 + blk) * (a.RP / 128) + r0 / 128) * 2048 + 16 * w);
        *dst = *(const QSK_LDS u32v4 *)&s_qw[16 * blk + r][kk];
      }
      QSK_GLOBAL u32v4 *dst = (QSK_GLOBAL u32v4 *)(gpw(a.qy) + ((int64_t)q * a.T + t) * a.RP * a.CP +
                                                   ((r0 / 16 + blk) * (a.CP / 128) + c0 / 128) * 2048 + 16 * w);
      *dst = *(const QSK_LDS u32v4 *)&s_qy[16 * blk + r][kk];
    }
    __syncthreads();                           // the buffers are written again for the next term
  }
}

// Test-matrix staging as e4m3 bytes: per plane, fragment-ordered blocks
// (16 o x 128 t, frag8_off) with t fastest, zero outside (o < n_o,
// t < n_t); four consecutive t per thread (o_pad a multiple of 16, t_pad of
// 128).
__global__ __launch_bounds__(256) void gen_stage8_kernel(uint8_t *dst, int n_o, int o_pad, int64_t t0,
                                                         int64_t n_t, int64_t t_pad, uint32_t stream, int rad,
                                                         uint32_t k0, uint32_t k1) {
  const int64_t words = (int64_t)o_pad * (t_pad / 4);
  const int64_t ps = (int64_t)o_pad * t_pad;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words;
       w += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(w / (t_pad / 4));
    const int64_t t = 4 * (w % (t_pad / 4));
    uint32_t out[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (o < n_o && t + i < n_t) embed_entry<MODE_FP8>(rad, (uint32_t)(t0 + t + i), (uint32_t)o, stream, k0, k1, v);
#pragma unroll
      for (int p = 0; p < 4; ++p) out[p] |= e4m3_byte(v[p]) << (8 * i);
    }
    const int64_t d = ((t >> 7) * (o_pad >> 4) + (o >> 4)) * 2048 + frag8_off(o & 15, (int)(t & 127));
#pragma unroll
    for (int p = 0; p < 4; ++p) *(QSK_GLOBAL uint32_t *)(gpw(dst) + p * ps + d) = out[p];
  }
}

// Negation of the 32 e4m3 values of a fragment (sign bits).
__device__ __forceinline__ i32x8 neg8(const i32x8 &a) {
  i32x8 r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = a[i] ^ (int)0x80808080;
  return r;
}
// The fragment of 16-row tile `tile` of an LDS tile set: lane (c, g) reads
// chunks g and 4 + g of row c.  A (plane, tile) block holds 128 chunks of
// 16 bytes, chunk (kc, row) at kc * 16 + row, so that eight consecutive
// lanes read eight different bank groups.
__device__ __forceinline__ i32x8 lds_frag8(const char *tile, int c16, int g) {
  const u32v4 lo = *(const QSK_LDS u32v4 *)(tile + (g * 16 + c16) * 16);
  const u32v4 hi = *(const QSK_LDS u32v4 *)(tile + ((4 + g) * 16 + c16) * 16);
  i32x8 r;
  r[0] = (int)lo.x; r[1] = (int)lo.y; r[2] = (int)lo.z; r[3] = (int)lo.w;
  r[4] = (int)hi.x; r[5] = (int)hi.y; r[6] = (int)hi.z; r[7] = (int)hi.w;
  return r;
}
__device__ __forceinline__ i32x8 bload_frag8(rsrc_t rs, uint32_t off) {
  const u32v4 lo = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
  const u32v4 hi = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 1024, 0, 0);
  i32x8 r;
  r[0] = (int)lo.x; r[1] = (int)lo.y; r[2] = (int)lo.z; r[3] = (int)lo.w;
  r[4] = (int)hi.x; r[5] = (int)hi.y; r[6] = (int)hi.z; r[7] = (int)hi.w;
  return r;
}
// E8M0 exponent byte of a power-of-two float scale
__device__ __forceinline__ int e8m0_of(float sc) { return (int)((__float_as_uint(sc) >> 23) & 0xFFu); }

struct W8Args {
  const uint8_t *qw;
  int64_t RP, CPW;
  const uint8_t *psi;         // [4][LP][MPF] e4m3 bytes
  int LP;
  int64_t MPF;
  const float *fsc;
  int RT, CT;
  int64_t ncols, col0;
  int l, S, ctiles, rgroups;
  int64_t kchunk;
  float *w;
  int64_t ldw, psw;
  float *part;                // [S][4][ncols][LP]
  float eta;
};

// W = Psi A on the fp8 matrix cores: a block of 4 waves owns 64 columns of
// the update block (16 per wave) and NMT 16-row tiles of W, over one chunk
// of the rows of A; 128 rows per step, the Psi tile HBM -> LDS directly (two
// buffers), the data fragments (2 x 16 bytes per plane and term) from HBM
// into registers one step ahead.
template <int NMT, int T, bool PURE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void w_fp8x_kernel(W8Args a) {
  constexpr int TB = 2048;                                 // bytes of a (plane, row tile) per step
  constexpr int NBLK = 4 * NMT * 2;                        // 1 KB DMA blocks per step
  __shared__ __attribute__((aligned(1024))) char s_psi[2][4 * NMT * TB];
  const int64_t tl = xcd_tile(blockIdx.x, (int64_t)a.ctiles * a.rgroups * a.S);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c16 = lane & 15, g = lane >> 4;
  const int bx = (int)(tl % a.ctiles);
  const int by = (int)((tl / a.ctiles) % a.rgroups);
  const int bz = (int)(tl / ((int64_t)a.ctiles * a.rgroups));
  const int64_t j = (int64_t)bx * 64 + wave * 16 + c16;
  const int rbase = by * NMT * 16;
  const int64_t ib = (int64_t)bz * a.kchunk;
  const int64_t ie = min(a.RP, ib + a.kchunk);
  const int sct = (int)min(j >> 5, (int64_t)a.CT - 1);
  // data: one resource per (plane, term) over its CPW x RP bytes
  rsrc_t dr[4][T];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < T; ++t)
      dr[q][t] = make_rsrc(a.qw + ((int64_t)(PURE ? (q > 0 ? q : 1) : q) * T + t) * a.CPW * a.RP,
                           (uint32_t)(a.CPW * a.RP));
  // this lane's data bytes: block (column tile, row step), 16 bytes at 16 lane
  uint32_t voff = (uint32_t)((((int64_t)bx * 4 + wave) * (a.RP / 128) + ib / 128) * 2048 + 16 * lane);
  // DMA source of this lane for 1 KB block half hh of a (plane, tile): chunk
  // c = 64 hh + lane is (kc = c / 16, row c mod 16)
  floatx4 acc[NMT][4];
#pragma unroll
  for (int i = 0; i < NMT; ++i)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[i][p] = {0.f, 0.f, 0.f, 0.f};
  i32x8 df[4][T];
  int e8[4] = {127, 127, 127, 127};
#define QSK_W8_FETCH(I0)                                                                         \
  do {                                                                                           \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                              \
      if (q == 0 && PURE) continue;                                                              \
      _Pragma("unroll") for (int t = 0; t < T; ++t) df[q][t] = bload_frag8(dr[q][t], voff);     \
      e8[q] = e8m0_of(gp(a.fsc)[((int64_t)q * a.RT + min((int64_t)(I0) / 32 + g, (int64_t)a.RT - 1)) * a.CT + sct]); \
    }                                                                                            \
  } while (0)
#define QSK_W8_DMA(I0, B)                                                                        \
  do {                                                                                           \
    _Pragma("unroll") for (int k_ = 0; k_ < NBLK / 4; ++k_) {                                    \
      const int u_ = wave + 4 * k_;                                                              \
      const int hh_ = u_ & 1, rt_ = (u_ >> 1) % NMT, pl_ = (u_ >> 1) / NMT;                      \
      dma16(a.psi + (((int64_t)pl_ * (a.MPF / 128) + (I0) / 128) * (a.LP / 16) + rbase / 16 + rt_) * 2048 + \
                hh_ * 1024 + 16 * lane, &s_psi[B][(pl_ * NMT + rt_) * TB + hh_ * 1024]);       \
    }                                                                                            \
  } while (0)
  QSK_W8_FETCH(ib);
  QSK_W8_DMA(ib, 0);
  wait_vm();
  __syncthreads();
  int buf = 0;
  for (int64_t i0 = ib; i0 < ie; i0 += 128) {
    i32x8 cur[4][T];
    int ce[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ce[q] = e8[q];
#pragma unroll
      for (int t = 0; t < T; ++t) cur[q][t] = df[q][t];
    }
    voff += 2048;
    if (i0 + 128 < ie) {
      QSK_W8_DMA(i0 + 128, buf ^ 1);
      __builtin_amdgcn_sched_barrier(0);
      QSK_W8_FETCH(i0 + 128);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < NMT; ++i) {
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        const i32x8 pf = lds_frag8(&s_psi[buf][(sp * NMT + i) * TB], c16, g);
        const i32x8 npf = neg8(pf);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int q = w_q_of(p, sp);
          if (q == 0 && PURE) continue;
          const bool ng = w_neg(p, sp);
#pragma unroll
          for (int t = 0; t < T; ++t)
            acc[i][p] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(ng ? npf : pf, cur[q][t], acc[i][p], 0, 0, 0,
                                                                          127, 0, max(ce[q] - 4 * t, 0));
        }
      }
    }
    wait_vm();
    __syncthreads();
    buf ^= 1;
  }
#undef QSK_W8_FETCH
#undef QSK_W8_DMA
  // epilogue: lane holds column j, rows rbase + i * 16 + 4g + (0..3)
  if (j >= a.ncols) return;
#pragma unroll
  for (int i = 0; i < NMT; ++i) {
    const int r0 = rbase + i * 16 + 4 * g;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      if (a.S == 1) {
        QSK_GLOBAL float *dst = gpw(a.w + p * a.psw + (a.col0 + j) * a.ldw);
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
          if (r0 + tt < a.l) dst[r0 + tt] += a.eta * acc[i][p][tt];
      } else {
        float *dst = a.part + (((int64_t)bz * 4 + p) * a.ncols + j) * a.LP + r0;
        *(QSK_GLOBAL floatx4 *)dst = acc[i][p];
      }
    }
  }
}

struct Y8Args {
  const uint8_t *qy;
  int64_t RP, CP;
  const uint8_t *om;          // [4][KP][NPF] e4m3 bytes
  int KP;
  int64_t NPF;
  const float *fsc;
  int RT, CT;
  int64_t m, ncols;
  int k, S, rblocks, cgroups;
  int64_t tchunk;
  float *y;
  int64_t ldy, psy, pss;
  float eta;
};

// Y = A Omega on the fp8 matrix cores: a block of 4 waves owns 64 rows of A
// (16 per wave) and NJ 16-column tiles of Y, over one chunk of the update's
// columns (copy bz of Y); 128 columns per step, the Omega tile HBM -> LDS
// directly (two buffers), the data fragments from HBM one step ahead.
template <int NJ, int T, bool PURE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void y_fp8x_kernel(Y8Args a) {
  constexpr int TB = 2048;
  constexpr int NBLK = 4 * NJ * 2;
  __shared__ __attribute__((aligned(1024))) char s_om[2][4 * NJ * TB];
  const int64_t tl = xcd_tile(blockIdx.x, (int64_t)a.rblocks * a.cgroups * a.S);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c16 = lane & 15, g = lane >> 4;
  const int64_t bx = tl % a.rblocks;
  const int by = (int)((tl / a.rblocks) % a.cgroups);
  const int bz = (int)(tl / ((int64_t)a.rblocks * a.cgroups));
  const int64_t rb = bx * 64;
  const int jt0 = by * NJ;
  const int64_t tb = (int64_t)bz * a.tchunk;
  const int64_t te = min(a.CP, tb + a.tchunk);
  const int64_t row = rb + wave * 16 + c16;
  const int srt = (int)min(row >> 5, (int64_t)a.RT - 1);
  rsrc_t dr[4][T];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < T; ++t)
      dr[q][t] = make_rsrc(a.qy + ((int64_t)(PURE ? (q > 0 ? q : 1) : q) * T + t) * a.RP * a.CP,
                           (uint32_t)(a.RP * a.CP));
  // this lane's data bytes: block (row tile, column step), 16 bytes at 16 lane
  uint32_t voff = (uint32_t)((((rb + wave * 16) / 16) * (a.CP / 128) + tb / 128) * 2048 + 16 * lane);
  floatx4 acc[NJ][4];
#pragma unroll
  for (int i = 0; i < NJ; ++i)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[i][p] = {0.f, 0.f, 0.f, 0.f};
  i32x8 df[4][T];
  int e8[4] = {127, 127, 127, 127};
#define QSK_Y8_FETCH(T0)                                                                         \
  do {                                                                                           \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                              \
      if (q == 0 && PURE) continue;                                                              \
      _Pragma("unroll") for (int t = 0; t < T; ++t) df[q][t] = bload_frag8(dr[q][t], voff);     \
      e8[q] = e8m0_of(gp(a.fsc)[((int64_t)q * a.RT + srt) * a.CT + min((int64_t)(T0) / 32 + g, (int64_t)a.CT - 1)]); \
    }                                                                                            \
  } while (0)
#define QSK_Y8_DMA(T0, B)                                                                        \
  do {                                                                                           \
    _Pragma("unroll") for (int k_ = 0; k_ < NBLK / 4; ++k_) {                                    \
      const int u_ = wave + 4 * k_;                                                              \
      const int hh_ = u_ & 1, jt_ = (u_ >> 1) % NJ, pl_ = (u_ >> 1) / NJ;                        \
      dma16(a.om + (((int64_t)pl_ * (a.NPF / 128) + (T0) / 128) * (a.KP / 16) + jt0 + jt_) * 2048 + \
                hh_ * 1024 + 16 * lane, &s_om[B][(pl_ * NJ + jt_) * TB + hh_ * 1024]);         \
    }                                                                                            \
  } while (0)
  QSK_Y8_FETCH(tb);
  QSK_Y8_DMA(tb, 0);
  wait_vm();
  __syncthreads();
  int buf = 0;
  for (int64_t t0 = tb; t0 < te; t0 += 128) {
    i32x8 cur[4][T];
    int ce[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ce[q] = e8[q];
#pragma unroll
      for (int t = 0; t < T; ++t) cur[q][t] = df[q][t];
    }
    voff += 2048;
    if (t0 + 128 < te) {
      QSK_Y8_DMA(t0 + 128, buf ^ 1);
      __builtin_amdgcn_sched_barrier(0);
      QSK_Y8_FETCH(t0 + 128);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        const i32x8 of = lds_frag8(&s_om[buf][(sp * NJ + i) * TB], c16, g);
        const i32x8 nof = neg8(of);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int q = y_q_of(p, sp);
          if (q == 0 && PURE) continue;
          const bool ng = y_neg(p, sp);
#pragma unroll
          for (int t = 0; t < T; ++t)
            acc[i][p] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(cur[q][t], ng ? nof : of, acc[i][p], 0, 0, 0,
                                                                          max(ce[q] - 4 * t, 0), 0, 127);
        }
      }
    }
    wait_vm();
    __syncthreads();
    buf ^= 1;
  }
#undef QSK_Y8_FETCH
#undef QSK_Y8_DMA
  // epilogue: lane holds column (jt0 + i) * 16 + c16 of Y, rows rb + 16 wave + 4g + (0..3)
  const int64_t r0 = rb + wave * 16 + 4 * g;
  float *ys = a.y + bz * a.pss;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    const int jj = (jt0 + i) * 16 + c16;
    if (jj >= a.k) continue;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      QSK_GLOBAL float *dst = gpw(ys + p * a.psy + (int64_t)jj * a.ldy);
      if (r0 + 3 < a.m && ((a.ldy | a.psy | a.pss) & 3) == 0) {
        QSK_GLOBAL floatx4 *d4 = (QSK_GLOBAL floatx4 *)(dst + r0);
        *d4 = *d4 + a.eta * acc[i][p];
      } else {
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
          if (r0 + tt < a.m) dst[r0 + tt] += a.eta * acc[i][p][tt];
      }
    }
  }
}

// Y for a block of at most 128 columns (one step): the Omega tile of the
// workgroup's column group stays in LDS while the workgroup walks over row
// blocks of 64 (bx, bx + G, bx + 2 G, ...); the data fragments of the next
// row block and the old Y values of the current one are fetched before the
// products, so their latency hides behind the matrix cores.
template <int NJ, int T, bool PURE, int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void y_fp8x_rows_kernel(Y8Args a) {
  // NS 128-column steps of the gathered block (CP = 128 NS), their Omega
  // tiles all resident
  constexpr int TB = 2048;
  constexpr int NBLK = 4 * NJ * 2;
  __shared__ __attribute__((aligned(1024))) char s_om[NS][4 * NJ * TB];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c16 = lane & 15, g = lane >> 4;
  const int G = (int)gridDim.x;
  const int by = (int)blockIdx.y;
  const int jt0 = by * NJ;
  rsrc_t dr[4][T];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < T; ++t)
      dr[q][t] = make_rsrc(a.qy + ((int64_t)(PURE ? (q > 0 ? q : 1) : q) * T + t) * a.RP * a.CP,
                           (uint32_t)(a.RP * a.CP));
  // the Omega tiles (128 NS columns of the block x NJ tiles x 4 planes)
#pragma unroll
  for (int ks = 0; ks < NS; ++ks)
#pragma unroll
    for (int k_ = 0; k_ < NBLK / 4; ++k_) {
      const int u_ = wave + 4 * k_;
      const int hh_ = u_ & 1, jt_ = (u_ >> 1) % NJ, pl_ = (u_ >> 1) / NJ;
      dma16(a.om + (((int64_t)pl_ * (a.NPF / 128) + ks) * (a.KP / 16) + jt0 + jt_) * 2048 + hh_ * 1024 + 16 * lane,
            &s_om[ks][(pl_ * NJ + jt_) * TB + hh_ * 1024]);
    }
  // one (row block, column step) at a time: the next one's data terms are
  // loaded while the matrix cores work on this one; Y is read at the first
  // step of a row block and written after its last
  i32x8 df[4][T];
  int e8[4] = {127, 127, 127, 127};
  int64_t bx = blockIdx.x;
  int ks = 0;
#define QSK_YR_FETCH(BX, KS)                                                                     \
  do {                                                                                           \
    const int64_t row_ = (BX) * 64 + wave * 16 + c16;                                            \
    const uint32_t off_ = (uint32_t)((((BX) * 4 + wave) * (a.CP / 128) + (KS)) * 2048 + 16 * lane); \
    const int srt_ = (int)min(row_ >> 5, (int64_t)a.RT - 1);                                     \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                              \
      if (q == 0 && PURE) continue;                                                              \
      _Pragma("unroll") for (int t = 0; t < T; ++t) df[q][t] = bload_frag8(dr[q][t], off_);      \
      e8[q] = e8m0_of(gp(a.fsc)[((int64_t)q * a.RT + srt_) * a.CT + min(4 * (KS) + g, a.CT - 1)]); \
    }                                                                                            \
  } while (0)
  if (bx * 64 < a.m) QSK_YR_FETCH(bx, 0);
  wait_vm();
  __syncthreads();
  floatx4 acc[NJ][4];
#pragma unroll
  for (int i = 0; i < NJ; ++i)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[i][p] = {0.f, 0.f, 0.f, 0.f};
  floatx4 old[NJ][4];
  while (bx * 64 < a.m) {
    i32x8 cur[4][T];
    int ce[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ce[q] = e8[q];
#pragma unroll
      for (int t = 0; t < T; ++t) cur[q][t] = df[q][t];
    }
    const int64_t r0 = bx * 64 + wave * 16 + 4 * g;
    const bool full = r0 + 3 < a.m && ((a.ldy | a.psy) & 3) == 0;
    if (ks == 0) {
      // old Y values of this row block
#pragma unroll
      for (int i = 0; i < NJ; ++i) {
        const int jj = (jt0 + i) * 16 + c16;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          old[i][p] = {0.f, 0.f, 0.f, 0.f};
          if (jj < a.k && full) old[i][p] = *(const QSK_GLOBAL floatx4 *)gp(a.y + p * a.psy + (int64_t)jj * a.ldy + r0);
        }
      }
    }
    const int64_t nbx = ks + 1 < NS ? bx : bx + G;
    const int nks = ks + 1 < NS ? ks + 1 : 0;
    if (nbx * 64 < a.m) QSK_YR_FETCH(nbx, nks);
    __builtin_amdgcn_sched_barrier(0);
    const char *om = &s_om[ks][0];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        const i32x8 of = lds_frag8(om + (sp * NJ + i) * TB, c16, g);
        const i32x8 nof = neg8(of);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int q = y_q_of(p, sp);
          if (q == 0 && PURE) continue;
          const bool ng = y_neg(p, sp);
#pragma unroll
          for (int t = 0; t < T; ++t)
            acc[i][p] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(cur[q][t], ng ? nof : of, acc[i][p], 0, 0, 0,
                                                                          max(ce[q] - 4 * t, 0), 0, 127);
        }
      }
    }
    if (ks == NS - 1) {
#pragma unroll
      for (int i = 0; i < NJ; ++i) {
        const int jj = (jt0 + i) * 16 + c16;
        if (jj >= a.k) continue;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          QSK_GLOBAL float *dst = gpw(a.y + p * a.psy + (int64_t)jj * a.ldy);
          if (full) {
            *(QSK_GLOBAL floatx4 *)(dst + r0) = old[i][p] + a.eta * acc[i][p];
          } else {
#pragma unroll
            for (int tt = 0; tt < 4; ++tt)
              if (r0 + tt < a.m) dst[r0 + tt] += a.eta * acc[i][p][tt];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < NJ; ++i)
#pragma unroll
        for (int p = 0; p < 4; ++p) acc[i][p] = {0.f, 0.f, 0.f, 0.f};
    }
    bx = nbx;
    ks = nks;
  }
#undef QSK_YR_FETCH
}

int fp8x_nmt(int l) {
  static const int c[3] = {4, 7, 8};        // LDS: 16 KB per tile for the two buffers
  return pick_tiles((l + 15) / 16, c, 3);
}

// Geometry of the FP8X buffers (bytes): the quantised block in both layouts
// and the e4m3 test matrices.
void fp8x_geometry(int64_t m, int l, int k, int64_t maxcols, int terms, int pure, Fp8xStage *f) {
  f->RP = rup(m, 128);
  f->CPW = rup(maxcols, 64);
  f->CP = rup(maxcols, 128);
  f->T = terms;
  f->planes = pure ? 3 : 4;
  f->NMT = fp8x_nmt(l);
  f->NJ = y_nj(k);
  f->LP = (int)rup(l, 16 * f->NMT);
  f->MPF = rup(m, 128);
  f->KP = (int)rup(k, 16 * f->NJ);
  f->NPF = f->CP;
  f->qw_bytes = (int64_t)4 * terms * f->CPW * f->RP;
  f->qy_bytes = (int64_t)4 * terms * f->RP * f->CP;
  f->psi_bytes = (int64_t)4 * f->LP * f->MPF;
  f->om_bytes = (int64_t)4 * f->KP * f->NPF;
}

template <int T, bool PURE>
static void launch_w8(const W8Args &w, int nmt, int64_t blocks, hipStream_t st) {
  if (nmt == 8) hipLaunchKernelGGL((w_fp8x_kernel<8, T, PURE>), dim3((unsigned)blocks), dim3(256), 0, st, w);
  else if (nmt == 7) hipLaunchKernelGGL((w_fp8x_kernel<7, T, PURE>), dim3((unsigned)blocks), dim3(256), 0, st, w);
  else hipLaunchKernelGGL((w_fp8x_kernel<4, T, PURE>), dim3((unsigned)blocks), dim3(256), 0, st, w);
}
template <int T, bool PURE>
static void launch_y8(const Y8Args &y, int nj, int64_t blocks, hipStream_t st) {
  if (nj == 7) hipLaunchKernelGGL((y_fp8x_kernel<7, T, PURE>), dim3((unsigned)blocks), dim3(256), 0, st, y);
  else hipLaunchKernelGGL((y_fp8x_kernel<4, T, PURE>), dim3((unsigned)blocks), dim3(256), 0, st, y);
}
template <int T>
static void launch_w8_t(const W8Args &w, int pure, int nmt, int64_t blocks, hipStream_t st) {
  if (pure) launch_w8<T, true>(w, nmt, blocks, st); else launch_w8<T, false>(w, nmt, blocks, st);
}
template <int T>
static void launch_y8_t(const Y8Args &y, int pure, int nj, int64_t blocks, hipStream_t st) {
  if (pure) launch_y8<T, true>(y, nj, blocks, st); else launch_y8<T, false>(y, nj, blocks, st);
}
template <int T, bool PURE>
static void launch_y8r(const Y8Args &y, dim3 grid, hipStream_t st) {
  if (y.CP == 256) hipLaunchKernelGGL((y_fp8x_rows_kernel<4, T, PURE, 2>), grid, dim3(256), 0, st, y);
  else hipLaunchKernelGGL((y_fp8x_rows_kernel<4, T, PURE, 1>), grid, dim3(256), 0, st, y);
}
template <int T>
static void launch_y8r_t(const Y8Args &y, int pure, dim3 grid, hipStream_t st) {
  if (pure) launch_y8r<T, true>(y, grid, st); else launch_y8r<T, false>(y, grid, st);
}

// Psi alone into the e4m3 staging of the FP8X format.
hipError_t stage_psi8(const SketchArgs &s, const Fp8xStage &f) {
  if (!f.psi) return hipErrorInvalidValue;
  const int64_t words = (int64_t)f.LP * (f.MPF / 4);
  hipLaunchKernelGGL(gen_stage8_kernel, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 65536)), dim3(256), 0,
                     s.stream, f.psi, s.l, f.LP, (int64_t)0, s.m, f.MPF, STREAM_PSI, s.rad, s.k0, s.k1);
  return hipGetLastError();
}

static hipError_t launch_fp8x(const SketchArgs &s, const Fp8xStage &f) {
  if (!f.qw || !f.qy || !f.psi || !f.om || s.ncols > f.CPW || !s.fp8_scales) return hipErrorInvalidValue;
  if (s.terms < 1 || s.terms > 4 || s.terms != f.T) return hipErrorInvalidValue;
  if ((uint64_t)f.CPW * f.RP >= (1ull << 32) || (uint64_t)f.RP * f.CP >= (1ull << 32)) return hipErrorNotSupported;
  if (s.in_dtype == DT_F32 ? !offsets_fit<float>(s.m, s.ncols, s.lda) : !offsets_fit<uint16_t>(s.m, s.ncols, s.lda))
    return hipErrorNotSupported;
  hipError_t e;
  mark(s, 0);
  // test matrices as e4m3 bytes: Omega_J per update, Psi once per sketch
  {
    const int64_t NPu = rup(s.ncols, 128);
    int64_t words = (int64_t)f.KP * (NPu / 4);
    hipLaunchKernelGGL(gen_stage8_kernel, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 65536)), dim3(256), 0,
                       s.stream, f.om, s.k, f.KP, s.col0, s.ncols, NPu, STREAM_OMEGA, s.rad, s.k0, s.k1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!s.psi_ready && !s.skip_w && (e = stage_psi8(s, f)) != hipSuccess) return e;
  }
  // tile scales and the e4m3 terms in both layouts, one pass over the block
  const int RT = (int)((s.m + 31) / 32), CT = (int)((s.ncols + 31) / 32);
  if (4 * (int64_t)RT * CT > s.fp8_scale_elems) return hipErrorInvalidValue;
  {
    QuantArgs qa{};
    for (int p = 0; p < 4; ++p) qa.a[p] = s.planes[p];
    qa.lda = s.lda; qa.m = s.m; qa.ncols = s.ncols; qa.pure = s.pure; qa.RT = RT; qa.CT = CT; qa.T = f.T;
    qa.fsc = s.fp8_scales; qa.qw = f.qw; qa.qy = f.qy; qa.RP = f.RP; qa.CPW = f.CPW;
    qa.CP = rup(s.ncols, 128);
    const dim3 grid((unsigned)(f.RP / 128), (unsigned)(qa.CP / 128), 4);
    if (s.in_dtype == DT_F32) hipLaunchKernelGGL(fp8x_quant_kernel<float>, grid, dim3(256), 0, s.stream, qa);
    else hipLaunchKernelGGL(fp8x_quant_kernel<uint16_t>, grid, dim3(256), 0, s.stream, qa);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  mark(s, 1);
  const int64_t CPu = rup(s.ncols, 128);
  // ---- Y
  {
    mark(s, 2);
    Y8Args y{};
    y.qy = f.qy; y.RP = f.RP; y.CP = CPu;
    y.om = f.om; y.KP = f.KP; y.NPF = CPu;
    y.fsc = s.fp8_scales; y.RT = RT; y.CT = CT;
    y.m = s.m; y.ncols = s.ncols; y.k = s.k;
    y.y = (float *)s.y; y.ldy = s.ldy; y.psy = s.psy; y.pss = s.pss; y.eta = (float)s.eta;
    const int nj = f.NJ;
    const int ntiles = (s.k + 15) / 16;
    y.rblocks = (int)((s.m + 63) / 64);
    y.cgroups = (ntiles + nj - 1) / nj;
    if ((CPu == 128 || CPu == 256) && nj == 4 && !(f.T == 4 && !s.pure)) {
      // one or two 128-column steps: row-walking blocks with the Omega tiles
      // kept in LDS and Y read and written once per row block (four column
      // tiles: the registers of seven do not fit)
      y.S = 1; y.tchunk = CPu;
      if (s.y_splits) *s.y_splits = 1;
      const int64_t G = std::min<int64_t>(y.rblocks, std::max<int64_t>(1, 2 * resident_blocks(2) / y.cgroups));
      const dim3 grid((unsigned)G, (unsigned)y.cgroups);
      switch (f.T) {
        case 1: launch_y8r_t<1>(y, s.pure, grid, s.stream); break;
        case 2: launch_y8r_t<2>(y, s.pure, grid, s.stream); break;
        case 3: launch_y8r_t<3>(y, s.pure, grid, s.stream); break;
        default: launch_y8r_t<4>(y, s.pure, grid, s.stream); break;
      }
    } else {
      int64_t S = pick_split((int64_t)y.rblocks * y.cgroups, std::min<int64_t>(s.y_copies, CPu / 128),
                             resident_blocks(2));
      int64_t tchunk = rup((CPu + S - 1) / S, 128);
      S = (CPu + tchunk - 1) / tchunk;
      y.S = (int)S; y.tchunk = tchunk;
      if (s.y_splits) *s.y_splits = (int)S;
      const int64_t blocks = (int64_t)y.rblocks * y.cgroups * S;
      switch (f.T) {
        case 1: launch_y8_t<1>(y, s.pure, nj, blocks, s.stream); break;
        case 2: launch_y8_t<2>(y, s.pure, nj, blocks, s.stream); break;
        case 3: launch_y8_t<3>(y, s.pure, nj, blocks, s.stream); break;
        default: launch_y8_t<4>(y, s.pure, nj, blocks, s.stream); break;
      }
    }
    e = hipGetLastError();
    mark(s, 3);
    if (e != hipSuccess) return e;
  }
  // ---- W
  if (!s.skip_w) {
    W8Args w{};
    w.qw = f.qw; w.RP = f.RP; w.CPW = f.CPW;
    w.psi = f.psi; w.LP = f.LP; w.MPF = f.MPF;
    w.fsc = s.fp8_scales; w.RT = RT; w.CT = CT;
    w.ncols = s.ncols; w.col0 = s.col0; w.l = s.l; w.eta = (float)s.eta;
    w.w = (float *)s.w; w.ldw = s.ldw; w.psw = s.psw;
    const int nmt = f.NMT;
    w.rgroups = f.LP / (16 * nmt);
    w.ctiles = (int)((s.ncols + 63) / 64);
    const int64_t base = (int64_t)w.ctiles * w.rgroups;
    const int64_t per_split = 4 * s.ncols * (int64_t)f.LP * 4;
    const int64_t smax = std::max<int64_t>(1, std::min<int64_t>(f.RP / 256, s.scratch_bytes / per_split));
    int64_t S = pick_split(base, smax, resident_blocks(2));
    int64_t kchunk = rup((f.RP + S - 1) / S, 128);
    if (kchunk < 256) kchunk = 256;
    S = (f.RP + kchunk - 1) / kchunk;
    if (S > 1 && S * per_split > s.scratch_bytes) { S = 1; kchunk = f.RP; }
    w.S = (int)S; w.kchunk = kchunk; w.part = (float *)s.scratch;
    const int64_t blocks = base * S;
    mark(s, 4);
    switch (f.T) {
      case 1: launch_w8_t<1>(w, s.pure, nmt, blocks, s.stream); break;
      case 2: launch_w8_t<2>(w, s.pure, nmt, blocks, s.stream); break;
      case 3: launch_w8_t<3>(w, s.pure, nmt, blocks, s.stream); break;
      default: launch_w8_t<4>(w, s.pure, nmt, blocks, s.stream); break;
    }
    e = hipGetLastError();
    mark(s, 5);
    if (e != hipSuccess) return e;
    mark(s, 6);
    if (S > 1) {
      const int64_t total = 4 * s.ncols * (int64_t)s.l;
      int64_t rblocks = (total + 255) / 256;
      if (rblocks > 65536) rblocks = 65536;
      hipLaunchKernelGGL(w_reduce_kernel, dim3((unsigned)rblocks), dim3(256), 0, s.stream, (const float *)s.scratch,
                         (int)S, f.LP, s.ncols, s.l, s.col0, (float *)s.w, s.ldw, s.psw, (float)s.eta);
      e = hipGetLastError();
    }
    mark(s, 7);
  }
  return e;
}

hipError_t launch_sketch_mfma(const SketchArgs &s, const MfmaStage &g) {
  if (s.mode == MODE_FP8X) return s.f8 ? launch_fp8x(s, *s.f8) : hipErrorInvalidValue;
  if (s.mode != MODE_BF16 && s.mode != MODE_F32 && s.mode != MODE_FP8) return hipErrorNotSupported;
  if (!g.omega || !g.psi) return hipErrorNotSupported;
  if (s.mode == MODE_FP8) {
    // split_terms 1: the e4m3 term alone; 2: plus the residual (two bf16 terms)
    if (s.in_dtype == DT_F32)
      return s.terms == 1 ? launch_t<OP_FP8, float, 1>(s, g) : launch_t<OP_FP8, float, 3>(s, g);
    if (s.in_dtype == DT_BF16)
      return s.terms == 1 ? launch_t<OP_FP8, uint16_t, 1>(s, g) : launch_t<OP_FP8, uint16_t, 3>(s, g);
    return hipErrorNotSupported;
  }
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
