// Device code of the fused MFMA passes (binary trees, 16-point leaves, rank 16).
//
// A pass applies K consecutive butterfly levels (plus, at the ends of the
// product, the leaf blocks or the middle weights) to one tile of 2^K slots.
// In k_fused_pass one wavefront owns COLS right-hand-side columns of the tile
// and keeps all of its 2^K slots in registers for the whole pass; in
// k_fused_pass_x2 (four-level passes) a pair of wavefronts shares the tile's
// slots and swaps half of them through LDS once.  Two lane geometries:
//
//   COLS = 32 (v_mfma_*_32x32):  lane l -> column l % 32, half e = l / 32;
//            the lane holds slot rows {4e..4e+3, 8+4e..11+4e} (8 complex).
//   COLS = 16 (v_mfma_*_16x16):  lane l -> column l % 16, quarter e = l / 16;
//            the lane holds slot rows {4e..4e+3} (4 complex).
//
// A butterfly (two input slots -> two output slots, one 32 x 32 complex block;
// Sec. 3.2.1 and 3.2.2: G^l_{2i+c,j} acting on [z_{i,2j}; z_{i,2j+1}], and the
// H analogue) is computed as real contractions on the matrix cores:
//   Re(out) = [Re M, -Im M] . [Re x; Im x],  Im(out) = [Re M, -Im M] . [Im x; -Re x].
// The accumulator layout of one level holds, in each lane, exactly the rows
// that the next level's B operand needs from that lane, so the interleaving of
// slots between levels is register renaming: no LDS, no cross-lane traffic.
// The A operands (the blocks) are packed in per-lane order, 8 KB per block
// (4 KB per leaf pair in the 16-column geometry); every wavefront of a
// workgroup works on the same tile, so the workgroup copies each stage of
// blocks from L2 into LDS once (global -> LDS loads, one stage ahead).
//
// Precisions: FP32, and split BF16 / FP16 (x = hi + lo, three MFMA products
// lo*hi + hi*lo + hi*hi with FP32 accumulation; FP16 also scales each block and
// each column by a power of two to stay inside the FP16 range).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

namespace bfly {
namespace fused {

// f(std::integral_constant<int, 0>{}) ... f(std::integral_constant<int, N-1>{}):
// every tile-local index is a compile-time constant, so the slot arrays stay
// in registers.
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kRank = 16;          // r == n0 == 16
constexpr int kBlockBytes = 8192;  // packed A operands of one 32 x 32 complex block
constexpr int kBlockBytes64 = 16384;  // the same, FP64 (Re M and Im M as doubles)
constexpr int kLeafBytes64 = 8192;    // FP64 leaf pair (two 16 x 16 blocks)
constexpr int kDefaultCols = 16;   // columns per wavefront unless BF_FUSED_COLS says otherwise

enum InKind : int { kInAct = 0, kInUser = 1, kInMiddle = 2 };
enum OutKind : int { kOutAct = 0, kOutUser = 1 };
enum Prec : int { kF32 = 0, kBF16 = 1, kF16 = 2, kF64 = 3 };

struct FusedArgs {
  const void *in;
  void *out;
  const char *fac;      // [K][ntiles][2^(K-1)] blocks
  const char *leaf;     // [ntiles][2^(K-1)] blocks (leaf in or leaf out)
  const float *fscale;  // FP16: power-of-two scale per block, same order as fac
  const float *lscale;  // FP16: same for leaf blocks
  const float *Sm;      // middle weights in natural slot order (kInMiddle)
  const double *Sm64;   // the same in FP64 (FP64 passes)
  int64_t ld, nrhs, nchunks, nslots, ntiles, m;
  int log_slo, mode_si, in_kind, out_kind, ngroups, log_m;
  // optional per-depth copies of the state in the activation layout (used by the
  // backward pass): lvl[0] after the leaf blocks or the middle weights, lvl[d]
  // after d levels (d < K, or d = K before the leaf-out blocks); nullptr: none
  void *lvl[5];
};

// Slot (in the global slot order of the level-by-level chain) of tile-local slot
// q after d of the pass's K levels.  A level that reads strided slots moves the
// paired bit to the bottom of the low bits; one that reads contiguous slots moves
// the bottom bit up: after d levels the first d output bits sit next to the tile's
// lo bits and the K - d unprocessed input bits keep their places.
template <int K>
__device__ __forceinline__ int64_t slot_at_depth(const FusedArgs &a, int64_t base, int64_t lo, int64_t q,
                                                 int d) {
  const int64_t dm = (int64_t(1) << d) - 1;
  if (a.mode_si)
    return base + ((q >> d) << (d + a.log_slo)) + (lo << d) + (q & dm);
  return base + ((q & dm) << (K - d + a.log_slo)) + (lo << (K - d)) + (q >> d);
}

struct BlockA {
  u32x4 v[8];  // this lane's 128 bytes of one packed block
};

// Component j of a 4-vector.  The element is copied to a scalar before any
// reinterpretation: hipcc for gfx950 reads element 0 when __builtin_bit_cast
// is applied to a vector-element expression directly.
__device__ __forceinline__ float as_f32(const u32x4 w, int j) {
  const unsigned e = j == 0 ? w.x : j == 1 ? w.y : j == 2 ? w.z : w.w;
  return __builtin_bit_cast(float, e);
}
__device__ __forceinline__ float pick4(const f32x4 w, int j) {
  return j == 0 ? w.x : j == 1 ? w.y : j == 2 ? w.z : w.w;
}

__device__ __forceinline__ BlockA load_block(const char *A, int lane) {
  const u32x4 *p = reinterpret_cast<const u32x4 *>(A) + lane;
  BlockA b;
#pragma unroll
  for (int v = 0; v < 8; ++v) b.v[v] = p[v * 64];
  return b;
}

// x * s = hi + lo with hi = RNE(x * s) and lo = RNE(x * s - hi), two values per
// conversion (one packed convert yields both halves of a 32-bit register)
template <class H8, class Hs>
__device__ __forceinline__ void split8(const float *x, float s, H8 &hi, H8 &lo) {
  typedef Hs h2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int j = 0; j < 8; j += 2) {
    const f32x2 v = {x[j] * s, x[j + 1] * s};
    const h2 h = __builtin_convertvector(v, h2);
    const f32x2 r = v - __builtin_convertvector(h, f32x2);
    const h2 l = __builtin_convertvector(r, h2);
    hi[j] = h.x;
    hi[j + 1] = h.y;
    lo[j] = l.x;
    lo[j + 1] = l.y;
  }
}

// flip the sign bit of eight 16-bit values
template <class H8>
__device__ __forceinline__ H8 neg8(const H8 &x) {
  u32x4 u = __builtin_bit_cast(u32x4, x);
  u ^= 0x80008000u;
  return __builtin_bit_cast(H8, u);
}

__device__ __forceinline__ floatx16 mfma32(const bf16x8 &a, const bf16x8 &b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx16 mfma32(const halfx8 &a, const halfx8 &b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma16(const bf16x8 &a, const bf16x8 &b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma16(const halfx8 &a, const halfx8 &b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Power-of-two scale for one column from this lane's values and the lanes
// holding the other rows of the same column.
template <int COLS>
__device__ __forceinline__ void column_scale(float mx, float bscale, float &cs, float &inv) {
  mx = fmaxf(mx, __shfl_xor(mx, 32));
  if (COLS == 16) mx = fmaxf(mx, __shfl_xor(mx, 16));
  int e = 0;
  if (mx > 0.f) (void)frexpf(mx, &e);
  cs = ldexpf(1.f, -e);
  inv = ldexpf(bscale, e);
}

// ---- COLS = 32: slot = x[16] (8 real parts, 8 imaginary parts) ------------------
//
// FP32, v_mfma_f32_32x32x2_f32: K step s = 16 part + 8 c' + rho takes row
// row_of(e, rho) of input slot c' from this lane (part 0: real, 1: imaginary);
// the A value for lane (i, e) is [Re M, -Im M][i][that K index].
// Split, v_mfma_f32_32x32x16: K step t = 2 part + c' takes the 8 rows of input
// slot c' in this lane; A.v[t] holds the hi halves, A.v[4 + t] the lo halves.
__device__ __forceinline__ void block32_f32(const BlockA &A, const float *x0, const float *x1,
                                            float *y0, float *y1) {
  floatx16 dr = {}, di = {};
#pragma unroll
  for (int s = 0; s < 32; ++s) {
    const float a = as_f32(A.v[s >> 2], s & 3);
    const int part = s >> 4, cp = (s >> 3) & 1, rho = s & 7;
    const float *x = cp ? x1 : x0;
    const float xre = x[rho], xim = x[8 + rho];
    if (part == 0) {
      dr = __builtin_amdgcn_mfma_f32_32x32x2f32(a, xre, dr, 0, 0, 0);
      di = __builtin_amdgcn_mfma_f32_32x32x2f32(a, xim, di, 0, 0, 0);
    } else {
      dr = __builtin_amdgcn_mfma_f32_32x32x2f32(a, xim, dr, 0, 0, 0);
      di = __builtin_amdgcn_mfma_f32_32x32x2f32(a, -xre, di, 0, 0, 0);
    }
  }
#pragma unroll
  for (int rho = 0; rho < 8; ++rho) {
    y0[rho] = dr[rho];
    y1[rho] = dr[8 + rho];
    y0[8 + rho] = di[rho];
    y1[8 + rho] = di[8 + rho];
  }
}

template <class H8, class Hs, bool kScale>
__device__ __forceinline__ void block32_split(const BlockA &A, float bscale, const float *x0,
                                              const float *x1, float *y0, float *y1) {
  float cs = 1.f, inv = 1.f;
  if (kScale) {
    float mx = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) mx = fmaxf(mx, fmaxf(fabsf(x0[j]), fabsf(x1[j])));
    column_scale<32>(mx, bscale, cs, inv);
  }
  H8 xh[4], xl[4];
  split8<H8, Hs>(x0, cs, xh[0], xl[0]);      // t = 0: real parts of slot 0
  split8<H8, Hs>(x1, cs, xh[1], xl[1]);      // t = 1: real parts of slot 1
  split8<H8, Hs>(x0 + 8, cs, xh[2], xl[2]);  // t = 2: imaginary parts of slot 0
  split8<H8, Hs>(x1 + 8, cs, xh[3], xl[3]);  // t = 3: imaginary parts of slot 1
  floatx16 dr = {}, di = {};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const H8 ahi = __builtin_bit_cast(H8, A.v[t]);
    const H8 alo = __builtin_bit_cast(H8, A.v[4 + t]);
    dr = mfma32(alo, xh[t], dr);
    dr = mfma32(ahi, xl[t], dr);
    dr = mfma32(ahi, xh[t], dr);
    const H8 yh = t < 2 ? xh[t + 2] : neg8(xh[t - 2]);
    const H8 yl = t < 2 ? xl[t + 2] : neg8(xl[t - 2]);
    di = mfma32(alo, yh, di);
    di = mfma32(ahi, yl, di);
    di = mfma32(ahi, yh, di);
  }
#pragma unroll
  for (int rho = 0; rho < 8; ++rho) {
    y0[rho] = dr[rho] * inv;
    y1[rho] = dr[8 + rho] * inv;
    y0[8 + rho] = di[rho] * inv;
    y1[8 + rho] = di[8 + rho] * inv;
  }
}

// ---- COLS = 16: slot = x[8] (4 real parts, 4 imaginary parts) -------------------
//
// Output tile T (16 rows) is output slot c = T.
// FP32, v_mfma_f32_16x16x4_f32, three real products per complex product (Gauss):
// with a = Re M, b = Im M, x = Re in, y = Im in,
//   P1 = a x,  P2 = b y,  P3 = (a + b)(x + y);   Re out = P1 - P2,  Im out = P3 - P1 - P2.
// K step k = 4 c' + rho takes row 4e + rho of input slot c'; the lane's A values for
// output row 16 T + i are Re M at float 16 T + k and Im M at float 16 T + 8 + k of
// its 32.
// Split, v_mfma_f32_16x16x32: K step t = part; this lane's 8 values are rows
// 4e..4e+3 of slot 0 then of slot 1; A.v[2T + t] hi, A.v[4 + 2T + t] lo (of
// [Re M, -Im M]).
// The block is read from LDS (blk: its packed 8 KB) one output slot at a time, so
// only half of it and three accumulators are live.
__device__ __forceinline__ void block16_f32(const char *blk, int lane, const float *x0, const float *x1,
                                            float *y0, float *y1) {
#pragma unroll
  for (int T = 0; T < 2; ++T) {
    // keep the compiler from hoisting the second half's operands (it spills then)
    __builtin_amdgcn_sched_barrier(0);
    u32x4 av[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) av[j] = reinterpret_cast<const u32x4 *>(blk + (4 * T + j) * 1024)[lane];
    floatx4 p1 = {}, p2 = {}, p3 = {};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int cp = k >> 2, rho = k & 3;
      const float *x = cp ? x1 : x0;
      const float xre = x[rho], xim = x[4 + rho];
      const float a = as_f32(av[k >> 2], k & 3), b = as_f32(av[2 + (k >> 2)], k & 3);
      p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, xre, p1, 0, 0, 0);
      p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(b, xim, p2, 0, 0, 0);
      p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a + b, xre + xim, p3, 0, 0, 0);
    }
    float *y = T ? y1 : y0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      y[v] = p1[v] - p2[v];
      y[4 + v] = p3[v] - p1[v] - p2[v];
    }
  }
}

template <class H8, class Hs, bool kScale>
__device__ __forceinline__ void block16_split(const BlockA &A, float bscale, const float *x0,
                                              const float *x1, float *y0, float *y1) {
  float cs = 1.f, inv = 1.f;
  if (kScale) {
    float mx = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) mx = fmaxf(mx, fmaxf(fabsf(x0[j]), fabsf(x1[j])));
    column_scale<16>(mx, bscale, cs, inv);
  }
  float re[8], im[8];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    re[j] = x0[j];
    re[4 + j] = x1[j];
    im[j] = x0[4 + j];
    im[4 + j] = x1[4 + j];
  }
  H8 xh[2], xl[2];
  split8<H8, Hs>(re, cs, xh[0], xl[0]);
  split8<H8, Hs>(im, cs, xh[1], xl[1]);
  const H8 nh = neg8(xh[0]), nl = neg8(xl[0]);
  floatx4 dr[2] = {{}, {}}, di[2] = {{}, {}};
#pragma unroll
  for (int T = 0; T < 2; ++T) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const H8 ahi = __builtin_bit_cast(H8, A.v[2 * T + t]);
      const H8 alo = __builtin_bit_cast(H8, A.v[4 + 2 * T + t]);
      dr[T] = mfma16(alo, xh[t], dr[T]);
      dr[T] = mfma16(ahi, xl[t], dr[T]);
      dr[T] = mfma16(ahi, xh[t], dr[T]);
      const H8 yh = t == 0 ? xh[1] : nh;
      const H8 yl = t == 0 ? xl[1] : nl;
      di[T] = mfma16(alo, yh, di[T]);
      di[T] = mfma16(ahi, yl, di[T]);
      di[T] = mfma16(ahi, yh, di[T]);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    y0[v] = dr[0][v] * inv;
    y0[4 + v] = di[0][v] * inv;
    y1[v] = dr[1][v] * inv;
    y1[4 + v] = di[1][v] * inv;
  }
}

template <int COLS, int PREC>
__device__ __forceinline__ void block_op(const BlockA &A, float bscale, const float *x0,
                                         const float *x1, float *y0, float *y1) {
  if constexpr (COLS == 32) {
    if constexpr (PREC == kF32)
      block32_f32(A, x0, x1, y0, y1);
    else if constexpr (PREC == kBF16)
      block32_split<bf16x8, __bf16, false>(A, 1.f, x0, x1, y0, y1);
    else
      block32_split<halfx8, _Float16, true>(A, bscale, x0, x1, y0, y1);
  } else {
    if constexpr (PREC == kBF16)
      block16_split<bf16x8, __bf16, false>(A, 1.f, x0, x1, y0, y1);
    else
      block16_split<halfx8, _Float16, true>(A, bscale, x0, x1, y0, y1);
  }
}

// ---- leaf blocks, 16-column geometry: one 16 x 16 product per slot ----------------
//
// A leaf pair is block diagonal, so each slot is multiplied by its own 16 x 16
// block: one K step of 32 = (real parts, imaginary parts) of this lane's rows
// 4e .. 4e+3.  Per slot c the packed block holds two 16-byte pieces per lane:
// split precisions: hi, lo of [Re M, -Im M][i][(part, 4e + rho)];
// FP32: the same 8 values as floats (K step s = 4 part + rho of v_mfma 16x16x4).
template <class H8, class Hs, bool kScale>
__device__ __forceinline__ void leaf16_split(const u32x4 ahi_u, const u32x4 alo_u, float bscale,
                                             const float *x, float *y) {
  float cs = 1.f, inv = 1.f;
  if (kScale) {
    float mx = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) mx = fmaxf(mx, fabsf(x[j]));
    column_scale<16>(mx, bscale, cs, inv);
  }
  H8 xh, xl;
  split8<H8, Hs>(x, cs, xh, xl);  // re rows, then im rows
  // operand of the imaginary part: (im rows, -re rows)
  const u32x4 uh = __builtin_bit_cast(u32x4, xh), ul = __builtin_bit_cast(u32x4, xl);
  const H8 yh = __builtin_bit_cast(H8, u32x4{uh.z, uh.w, uh.x ^ 0x80008000u, uh.y ^ 0x80008000u});
  const H8 yl = __builtin_bit_cast(H8, u32x4{ul.z, ul.w, ul.x ^ 0x80008000u, ul.y ^ 0x80008000u});
  const H8 ahi = __builtin_bit_cast(H8, ahi_u), alo = __builtin_bit_cast(H8, alo_u);
  floatx4 dr = {}, di = {};
  dr = mfma16(alo, xh, dr);
  dr = mfma16(ahi, xl, dr);
  dr = mfma16(ahi, xh, dr);
  di = mfma16(alo, yh, di);
  di = mfma16(ahi, yl, di);
  di = mfma16(ahi, yh, di);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    y[v] = dr[v] * inv;
    y[4 + v] = di[v] * inv;
  }
}

// FP32 leaf block, Gauss's three products as in block16_f32: a0 holds Re M, a1 Im M
// of this lane's K index rho (rows 4e + rho).
__device__ __forceinline__ void leaf16_f32(const u32x4 a0, const u32x4 a1, const float *x, float *y) {
  floatx4 p1 = {}, p2 = {}, p3 = {};
#pragma unroll
  for (int rho = 0; rho < 4; ++rho) {
    const float a = as_f32(a0, rho), b = as_f32(a1, rho);
    const float xre = x[rho], xim = x[4 + rho];
    p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, xre, p1, 0, 0, 0);
    p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(b, xim, p2, 0, 0, 0);
    p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a + b, xre + xim, p3, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    y[v] = p1[v] - p2[v];
    y[4 + v] = p3[v] - p1[v] - p2[v];
  }
}

// the two slots of a leaf pair; blk points at the pair's four pieces
template <int PREC>
__device__ __forceinline__ void leaf_pair16(const char *blk, int lane, float bscale, const float *x0,
                                            const float *x1, float *y0, float *y1) {
  const u32x4 *b = reinterpret_cast<const u32x4 *>(blk) + lane;
  const u32x4 p0 = b[0], p1 = b[64], p2 = b[128], p3 = b[192];
  if constexpr (PREC == kF32) {
    leaf16_f32(p0, p1, x0, y0);
    leaf16_f32(p2, p3, x1, y1);
  } else if constexpr (PREC == kBF16) {
    leaf16_split<bf16x8, __bf16, false>(p0, p1, 1.f, x0, y0);
    leaf16_split<bf16x8, __bf16, false>(p2, p3, 1.f, x1, y1);
  } else {
    leaf16_split<halfx8, _Float16, true>(p0, p1, bscale, x0, y0);
    leaf16_split<halfx8, _Float16, true>(p2, p3, bscale, x1, y1);
  }
}

// ---- geometry: which slot rows a lane holds ----------------------------------------
template <int COLS>
struct Geo;
template <>
struct Geo<32> {
  static constexpr int kSW = 16;  // floats per slot per lane
  static constexpr int kRows = 8;
  __device__ static int row(int e, int rho) { return rho < 4 ? 4 * e + rho : 8 + 4 * e + (rho - 4); }
  // activation pair j (rows 2 pair, 2 pair + 1) held by this lane
  __device__ static int pair(int e, int j) { return (j < 2) ? 2 * e + j : 4 + 2 * e + (j - 2); }
};
template <>
struct Geo<16> {
  static constexpr int kSW = 8;
  static constexpr int kRows = 4;
  __device__ static int row(int e, int rho) { return 4 * e + rho; }
  __device__ static int pair(int e, int j) { return 2 * e + j; }
};

// Launch shape per pass depth of k_fused_pass.  Every pass fits at least two
// resident wavefronts per SIMD (at most 256 registers).  Blocks are staged in
// LDS in groups of kStageBlocks (double buffered, 2 x kStageBlocks x 8 KB);
// four-level passes use half-level stages and four-wavefront workgroups so that
// two workgroups share a CU and overlap each other's loads and stores.
template <int COLS, int K>
struct PassTraits {
  static constexpr int kWavesPerEU = 2;
  static constexpr int kMaxWaves = K >= 4 ? 4 : 8;  // wavefronts per workgroup
  static constexpr int kStageBlocks = (1 << (K - 1)) < 4 ? (1 << (K - 1)) : 4;
};

// Packed bytes of one leaf pair: a block-diagonal 32 x 32 block (32 columns per
// wavefront) or two 16 x 16 blocks (16 columns per wavefront).
template <int COLS>
constexpr int kLeafBytes = COLS == 16 ? kBlockBytes / 2 : kBlockBytes;

// Block beta (0 .. 2^(K-1) - 1) of block group g: leaf-in (if LI), levels
// 0 .. K-1, leaf-out (if LO).  Returns its packed bytes and its FP16 scale slot.
template <int COLS, int K, bool LI>
__device__ __forceinline__ const char *group_block(const FusedArgs &a, int64_t tile, int g, int beta,
                                                   const float *&scale) {
  constexpr int NB = 1 << (K - 1);
  const int d = g - (LI ? 1 : 0);
  if (d < 0 || d >= K) {
    const int64_t bi = tile * NB + beta;
    scale = a.lscale ? a.lscale + bi : nullptr;
    return a.leaf + bi * kLeafBytes<COLS>;
  }
  const int64_t bi = ((int64_t)d * a.ntiles + tile) * NB + beta;
  scale = a.fscale ? a.fscale + bi : nullptr;
  return a.fac + bi * kBlockBytes;
}

template <int K, bool LI, bool LO>
__device__ __forceinline__ constexpr bool is_leaf_group(int g) {
  return (LI && g == 0) || (LO && g == (LI ? 1 : 0) + K);
}

// Workgroup -> (tile, group of column chunks).  Workgroups are dispatched to the
// eight XCDs round robin, so the groups of one tile are placed eight ids apart:
// they run on the same XCD at about the same time and share its L2.
__device__ __forceinline__ void tile_of_block(const FusedArgs &a, int64_t &tile, int64_t &group) {
  const int64_t gid = blockIdx.x;
  const int64_t G = a.ngroups;
  if (G == 1) {
    tile = gid;
    group = 0;
  } else if ((a.ntiles & 7) == 0) {
    const int64_t xcd = gid & 7, r = gid >> 3;
    group = r % G;
    tile = (r / G) * 8 + xcd;
  } else {
    tile = gid / G;
    group = gid - tile * G;
  }
}

template <int COLS, int K, int PREC, bool LI, bool LO>
__global__ __launch_bounds__((PassTraits<COLS, K>::kMaxWaves * 64))
__attribute__((amdgpu_waves_per_eu(PassTraits<COLS, K>::kWavesPerEU)))
void k_fused_pass(FusedArgs a) {
  using G = Geo<COLS>;
  constexpr int SW = G::kSW;
  constexpr int NR = G::kRows;
  constexpr int NS = 1 << K;
  constexpr int NB = NS / 2;
  constexpr int LOGC = COLS == 32 ? 5 : 4;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
  const int n = lane & (COLS - 1), e = lane / COLS;
  int64_t tile, group;
  tile_of_block(a, tile, group);
  const int64_t chunk = group * (blockDim.x >> 6) + wave;
  if (chunk >= a.nchunks) return;
  const int64_t slo = int64_t(1) << a.log_slo;
  const int64_t hi = tile >> a.log_slo, lo = tile & (slo - 1);
  const int64_t base = hi << (K + a.log_slo);
  const int64_t col = (chunk << LOGC) + n;
  const bool col_ok = col < a.nrhs;

  // Blocks of the stage being computed sit in one half of an LDS double buffer
  // while the next stage's blocks stream into the other half: every wavefront
  // of the workgroup copies its share with global -> LDS loads (16 bytes per
  // lane, no registers), one stage ahead.  Stage st = group g (leaf-in, a
  // level, leaf-out) times part: blocks part*HB .. part*HB + HB - 1 of g.
  constexpr int HB = PassTraits<COLS, K>::kStageBlocks;
  constexpr int NPART = NB / HB;
  constexpr int NST = ((LI ? 1 : 0) + K + (LO ? 1 : 0)) * NPART;
  __shared__ __attribute__((aligned(16))) char lds[2 * HB * kBlockBytes];
  const int W = (int)(blockDim.x >> 6);
  const int wact = (int)((a.nchunks - group * W) < W ? (a.nchunks - group * W) : W);
  auto issue_stage = [&](int sti) {
    char *dst = lds + (sti & 1) * (HB * kBlockBytes);
    const int g = sti / NPART, b0 = (sti % NPART) * HB;
    const int lp = is_leaf_group<K, LI, LO>(g) ? kLeafBytes<COLS> / 1024 : 8;  // pieces per block
    for (int c = wave; c < HB * lp; c += wact) {
      const int blk = c / lp, piece = c - blk * lp;
      const float *sp;
      const char *src = group_block<COLS, K, LI>(a, tile, g, b0 + blk, sp) + piece * 1024 + lane * 16;
      __builtin_amdgcn_global_load_lds(
          src, (__attribute__((address_space(3))) void *)(dst + blk * kBlockBytes + piece * 1024), 16, 0, 0);
    }
  };
  auto block_scale = [&](int g, int beta) {
    if constexpr (PREC != kF16) return 1.f;
    const float *sp;
    (void)group_block<COLS, K, LI>(a, tile, g, beta, sp);
    return *sp;
  };
  issue_stage(0);

  // st[q][0 .. NR-1] real, st[q][NR .. 2 NR - 1] imaginary parts of this lane's rows
  float st[NS][SW];

  // ---- inputs at depth 0
  static_for<NS>([&](auto Q) {
    constexpr int q = Q;
    const int64_t slot = a.mode_si ? base + ((int64_t)q << a.log_slo) + lo : base + (lo << K) + q;
    if constexpr (LI) {
      const f32x2 *g = static_cast<const f32x2 *>(a.in);
      static_for<NR>([&](auto RHO) {
        constexpr int rho = RHO;
        f32x2 v = {0.f, 0.f};
        if (col_ok) v = __builtin_nontemporal_load(&g[(slot * kRank + G::row(e, rho)) * a.ld + col]);
        st[q][rho] = v.x;
        st[q][NR + rho] = v.y;
      });
    } else {
      // the first pass after the middle level reads the transposed slot (M^h is a
      // block transpose of the m x m grid of slots; m is a power of two)
      const int64_t tr = ((slot & (a.m - 1)) << a.log_m) | (slot >> a.log_m);
      const int64_t src = a.in_kind == kInMiddle ? tr : slot;
      const f32x4 *p = static_cast<const f32x4 *>(a.in) + ((chunk * a.nslots + src) * 8) * COLS + n;
      static_for<NR / 2>([&](auto J) {
        constexpr int j = J;
        const f32x4 v = __builtin_nontemporal_load(p + G::pair(e, j) * COLS);
        st[q][2 * j] = v.x;
        st[q][NR + 2 * j] = v.y;
        st[q][2 * j + 1] = v.z;
        st[q][NR + 2 * j + 1] = v.w;
      });
    }
  });
  // middle weights S^h_{i,j}, in natural slot order, after every load is in flight
  if (!LI && a.in_kind == kInMiddle) {
    static_for<NS>([&](auto Q) {
      constexpr int q = Q;
      const int64_t slot = a.mode_si ? base + ((int64_t)q << a.log_slo) + lo : base + (lo << K) + q;
      const f32x4 *sp = reinterpret_cast<const f32x4 *>(a.Sm + slot * kRank);
      static_for<NR / 4>([&](auto J) {
        constexpr int j = J;
        const f32x4 s4 = sp[COLS == 32 ? (j == 0 ? e : 2 + e) : e];
        static_for<4>([&](auto V) {
          const float sc = pick4(s4, V);
          st[q][4 * j + V] *= sc;
          st[q][NR + 4 * j + V] *= sc;
        });
      });
    });
  }

  // one block operation: block beta of group g, staged in LDS
  auto step = [&](auto G, auto BETA, const float *x0, const float *x1, float *y0, float *y1) {
    constexpr int g = G, beta = BETA;
    constexpr int sti = g * NPART + beta / HB;
    const char *blk = lds + (sti & 1) * (HB * kBlockBytes) + (beta % HB) * kBlockBytes;
    if constexpr (COLS == 16 && is_leaf_group<K, LI, LO>(g)) {
      leaf_pair16<PREC>(blk, lane, block_scale(g, beta), x0, x1, y0, y1);
    } else if constexpr (COLS == 16 && PREC == kF32) {
      block16_f32(blk, lane, x0, x1, y0, y1);
    } else {
      BlockA A;
      static_for<8>([&](auto V) {
        A.v[V] = reinterpret_cast<const u32x4 *>(blk + V * 1024)[lane];
      });
      block_op<COLS, PREC>(A, block_scale(g, beta), x0, x1, y0, y1);
    }
  };
  // entering stage sti: its blocks have landed in LDS, the previous stage is done
  // everywhere, and the next stage's copy starts
  auto stage_begin = [&](auto STI) {
    constexpr int sti = STI;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if constexpr (sti + 1 < NST) issue_stage(sti + 1);
  };
  auto pair_group = [&](auto G) {
    constexpr int g = G;
    static_for<NB>([&](auto PP) {
      constexpr int pp = PP;
      if constexpr (pp % HB == 0) stage_begin(std::integral_constant<int, g * NPART + pp / HB>{});
      float t0[SW], t1[SW];
      step(G, PP, st[2 * pp], st[2 * pp + 1], t0, t1);
      static_for<SW>([&](auto J) {
        st[2 * pp][J] = t0[J];
        st[2 * pp + 1][J] = t1[J];
      });
    });
  };

  // copy of the state after d levels into a.lvl[d] (activation layout)
  auto store_depth = [&](int d) {
    f32x4 *dst = static_cast<f32x4 *>(a.lvl[d]);
    if (!dst) return;
    static_for<NS>([&](auto Q) {
      constexpr int q = Q;
      const int64_t slot = slot_at_depth<K>(a, base, lo, q, d);
      f32x4 *p = dst + ((chunk * a.nslots + slot) * 8) * COLS + n;
      static_for<NR / 2>([&](auto J) {
        constexpr int j = J;
        const f32x4 v = {st[q][2 * j], st[q][NR + 2 * j], st[q][2 * j + 1], st[q][NR + 2 * j + 1]};
        __builtin_nontemporal_store(v, p + G::pair(e, j) * COLS);
      });
    });
  };

  // ---- leaf blocks applied to slot pairs before the first level
  if constexpr (LI) pair_group(std::integral_constant<int, 0>{});
  if (LI || a.in_kind == kInMiddle) store_depth(0);

  // ---- K butterfly levels
  static_for<K>([&](auto D) {
    constexpr int d = D;
    constexpr int g = (LI ? 1 : 0) + d;
    float nx[NS][SW];
    static_for<NB>([&](auto BETA) {
      constexpr int beta = BETA;
      if constexpr (beta % HB == 0) stage_begin(std::integral_constant<int, g * NPART + beta / HB>{});
      constexpr int ap = beta >> d, b = beta & ((1 << d) - 1);
      constexpr int qi0 = (2 * ap) * (1 << d) + b, qi1 = (2 * ap + 1) * (1 << d) + b;
      constexpr int qo0 = ap * (2 << d) + 2 * b, qo1 = qo0 + 1;
      step(std::integral_constant<int, g>{}, BETA, st[qi0], st[qi1], nx[qo0], nx[qo1]);
    });
    static_for<NS>([&](auto Q) {
      static_for<SW>([&](auto J) { st[Q][J] = nx[Q][J]; });
    });
    if (d + 1 < K || LO) store_depth(d + 1);
  });

  // ---- leaf blocks after the last level
  if constexpr (LO) pair_group(std::integral_constant<int, (LI ? 1 : 0) + K>{});

  // ---- outputs at depth K (a.out == nullptr: only the per-depth copies are wanted)
  if (!a.out) return;
  static_for<NS>([&](auto Q) {
    constexpr int q = Q;
    const int64_t slot = a.mode_si ? base + (lo << K) + q : base + ((int64_t)q << a.log_slo) + lo;
    if constexpr (LO) {
      if (col_ok) {
        f32x2 *u = static_cast<f32x2 *>(a.out);
        static_for<NR>([&](auto RHO) {
          constexpr int rho = RHO;
          const f32x2 v = {st[q][rho], st[q][NR + rho]};
          __builtin_nontemporal_store(v, &u[(slot * kRank + G::row(e, rho)) * a.ld + col]);
        });
      }
    } else {
      f32x4 *p = static_cast<f32x4 *>(a.out) + ((chunk * a.nslots + slot) * 8) * COLS + n;
      static_for<NR / 2>([&](auto J) {
        constexpr int j = J;
        const f32x4 v = {st[q][2 * j], st[q][NR + 2 * j], st[q][2 * j + 1], st[q][NR + 2 * j + 1]};
        __builtin_nontemporal_store(v, p + G::pair(e, j) * COLS);
      });
    }
  });
}

// ---- split tiles: two wavefronts share one tile of one column chunk ----------------
//
// Wavefront h (0 or 1) of a pair holds the tile slots q = h 2^(K-1) + j,
// j < 2^(K-1), so its state is half that of the pass above and four wavefronts
// fit on a SIMD.  Levels 0 .. K-2 never pair slots of different halves (they
// keep the top bit of q), so each wavefront runs them alone on its 2^(K-1)
// slots, computing blocks h 2^(K-2) + beta'.  The last level pairs slot b with
// slot 2^(K-1) + b: before it the pair swaps half of its slots through LDS
// (wavefront 0 keeps the x0 operands of b < 2^(K-2), wavefront 1 the x1 operands
// of b >= 2^(K-2)), and wavefront h' then computes the blocks b = h' 2^(K-2) + k,
// whose outputs 2b, 2b + 1 are again slots of half h'.  Leaf blocks pair slots
// 2p, 2p + 1, so they stay inside one half too.
// Staging of the split passes: blocks stream into two LDS buffers of one stage
// each, one stage ahead of the stage being computed; the swap of halves has an
// LDS region of its own.  Workgroups hold 1, 2 or 4 column chunks (2, 4 or 8
// wavefronts); a wavefront pair past the last chunk stays resident, loading and
// storing nothing, and takes its share of the block copies.
#ifndef BF_SPLIT_MAX_PAIRS
#define BF_SPLIT_MAX_PAIRS 4
#endif
#ifndef BF_SPLIT_SWAP_KB
#define BF_SPLIT_SWAP_KB 16
#endif
// One block per wavefront per stage, four stage buffers (copies three stages ahead,
// 64 KB, plus the 16 KB swap region: two workgroups per CU).  At N = 2^20, 256
// columns: 4.59 ms split BF16 and 7.51 ms FP32, against 4.69 and 7.67 ms with two
// blocks per stage in two buffers.
#ifndef BF_SPLIT_PB
#define BF_SPLIT_PB 1
#endif
#ifndef BF_SPLIT_NBUF
#define BF_SPLIT_NBUF 4
#endif
template <int K>
struct SplitTraits {
  static constexpr int kHS = 1 << (K - 1);  // slots per wavefront
  static constexpr int kWB = kHS / 2;       // blocks per wavefront per level
  static constexpr int kPB = kWB < BF_SPLIT_PB ? kWB : BF_SPLIT_PB;  // blocks per wavefront per stage
  static constexpr int kHB = 2 * kPB;            // blocks per stage
  static constexpr int kNPART = kWB / kPB;       // stages per block group
  static constexpr int kMaxPairs = BF_SPLIT_MAX_PAIRS;  // column chunks per workgroup
  static constexpr int kSwapBytes = BF_SPLIT_SWAP_KB * 1024;
  static constexpr int kSR = kSwapBytes / (2 * kMaxPairs * 2048);  // slots per swap round
  static constexpr int kRounds = (kWB + kSR - 1) / kSR;
  static constexpr int kNBUF = BF_SPLIT_NBUF;      // stage buffers: copies run kNBUF - 1 stages ahead
  static constexpr int kLdsBytes = kNBUF * kHB * kBlockBytes + kSwapBytes;
};

// CP column chunks (wavefront pairs) per workgroup.
template <int K, int PREC, bool LI, bool LO, int CP, bool IO = false>
__global__ __launch_bounds__(CP * 128) __attribute__((amdgpu_waves_per_eu(4)))
void k_fused_pass_x2(FusedArgs a) {
  using T = SplitTraits<K>;
  using G = Geo<16>;
  constexpr int SW = G::kSW;
  constexpr int NR = G::kRows;
  constexpr int HS = T::kHS, WB = T::kWB, PB = T::kPB, HB = T::kHB, NPART = T::kNPART;
  constexpr int NST = ((LI ? 1 : 0) + K + (LO ? 1 : 0)) * NPART;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
  const int half = wave & 1;
  const int n = lane & 15, e = lane >> 4;
  int64_t tile, group;
  tile_of_block(a, tile, group);
  constexpr int W = 2 * CP;  // wavefronts
  const int64_t chunk = group * CP + (wave >> 1);
  const bool active = chunk < a.nchunks;
  const int64_t slo = int64_t(1) << a.log_slo;
  const int64_t hi = tile >> a.log_slo, lo = tile & (slo - 1);
  const int64_t base = hi << (K + a.log_slo);
  const int64_t col = (chunk << 4) + n;
  const bool col_ok = active && col < a.nrhs;
  const int qh = half * HS;  // first tile slot of this wavefront

  // Stage (g, part) holds blocks h WB + part PB + i of group g at position
  // h PB + i of its buffer, for both halves h.
  __shared__ __attribute__((aligned(16))) char lds[T::kLdsBytes];
  constexpr int NBUF = T::kNBUF;
  char *const swap = lds + NBUF * HB * kBlockBytes;
  // every wavefront copies HB lp / W of the stage's 1 KB pieces (W divides HB lp)
  auto issue_stage = [&](auto STI) {
    constexpr int sti = STI;
    char *dst = lds + (sti % NBUF) * (HB * kBlockBytes);
    constexpr int g = sti / NPART, part = sti % NPART;
    constexpr int lp = is_leaf_group<K, LI, LO>(g) ? kLeafBytes<16> / 1024 : 8;  // pieces per block
    static_assert((HB * lp) % W == 0, "pieces per wavefront");
    static_for<HB * lp / W>([&](auto I) {
      const int c = wave + (int)I * W;
      const int pos = c / lp, piece = c - pos * lp;
      const int beta = (pos / PB) * WB + part * PB + (pos % PB);
      const float *sp;
      const char *src = group_block<16, K, LI>(a, tile, g, beta, sp) + piece * 1024 + lane * 16;
      __builtin_amdgcn_global_load_lds(
          src, (__attribute__((address_space(3))) void *)(dst + pos * kBlockBytes + piece * 1024), 16, 0, 0);
    });
  };
  auto block_scale = [&](int g, int beta) {
    if constexpr (PREC != kF16) return 1.f;
    const float *sp;
    (void)group_block<16, K, LI>(a, tile, g, beta, sp);
    return *sp;
  };
  issue_stage(std::integral_constant<int, 0>{});

  float st[HS][SW];

  // ---- inputs at depth 0: tile slots qh .. qh + HS - 1, issued in slot order (the
  // order the first stages take them in)
  static_for<HS>([&](auto J) {
    constexpr int j = J;
    __builtin_amdgcn_sched_barrier(0);
    const int64_t q = qh + j;
    const int64_t slot = a.mode_si ? base + (q << a.log_slo) + lo : base + (lo << K) + q;
    if constexpr (LI) {
      // every lane loads (column 0 in place of a missing one), so each wavefront
      // issues the same number of loads and the first stage can wait for its blocks
      // alone (stage_begin); the leaf blocks' outputs of missing columns are zeroed
      const f32x2 *g = static_cast<const f32x2 *>(a.in);
      const int64_t cl = col_ok ? col : 0;
      static_for<NR>([&](auto RHO) {
        constexpr int rho = RHO;
        const f32x2 v = __builtin_nontemporal_load(&g[(slot * kRank + G::row(e, rho)) * a.ld + cl]);
        st[j][rho] = v.x;
        st[j][NR + rho] = v.y;
      });
    } else {
      const int64_t tr = ((slot & (a.m - 1)) << a.log_m) | (slot >> a.log_m);
      const int64_t src = a.in_kind == kInMiddle ? tr : slot;
      // an idle wavefront pair loads chunk 0 (see above) and stores nothing
      const int64_t ck = active ? chunk : 0;
      const f32x4 *p = static_cast<const f32x4 *>(a.in) + ((ck * a.nslots + src) * 8) * 16 + n;
      static_for<NR / 2>([&](auto JJ) {
        constexpr int jj = JJ;
        const f32x4 v = __builtin_nontemporal_load(p + G::pair(e, jj) * 16);
        st[j][2 * jj] = v.x;
        st[j][NR + 2 * jj] = v.y;
        st[j][2 * jj + 1] = v.z;
        st[j][NR + 2 * jj + 1] = v.w;
      });
    }
  });
  if (!LI && a.in_kind == kInMiddle) {
    static_for<HS>([&](auto J) {
      constexpr int j = J;
      const int64_t q = qh + j;
      const int64_t slot = a.mode_si ? base + (q << a.log_slo) + lo : base + (lo << K) + q;
      const f32x4 s4 = reinterpret_cast<const f32x4 *>(a.Sm + slot * kRank)[e];
      static_for<4>([&](auto V) {
        const float sc = pick4(s4, V);
        st[j][V] *= sc;
        st[j][NR + V] *= sc;
      });
    });
  }
  // the next NBUF - 2 stages follow the state loads, so the first stage's wait
  // leaves them in flight
  static_for<NBUF - 2>([&](auto I) {
    if constexpr (1 + (int)I < NST) issue_stage(std::integral_constant<int, 1 + (int)I>{});
  });

  // block h WB + bw of group g (bw < WB), staged in LDS
  auto step = [&](auto GG, auto BW, const float *x0, const float *x1, float *y0, float *y1) {
    constexpr int g = GG, bw = BW;
    constexpr int sti = g * NPART + bw / PB;
    const char *blk = lds + (sti % NBUF) * (HB * kBlockBytes) + (half * PB + bw % PB) * kBlockBytes;
    if constexpr (is_leaf_group<K, LI, LO>(g)) {
      leaf_pair16<PREC>(blk, lane, block_scale(g, half * WB + bw), x0, x1, y0, y1);
    } else if constexpr (PREC == kF32) {
      block16_f32(blk, lane, x0, x1, y0, y1);
    } else {
      BlockA A;
      static_for<8>([&](auto V) {
        A.v[V] = reinterpret_cast<const u32x4 *>(blk + V * 1024)[lane];
      });
      block_op<16, PREC>(A, block_scale(g, half * WB + bw), x0, x1, y0, y1);
    }
  };
  // Barriers are bare s_barriers between explicit waits: a workgroup fence would also
  // wait for every load in flight.  The empty asm statements keep the compiler from
  // moving LDS accesses across them.
  auto barrier_after = [&](auto VM) {
    constexpr int vm = VM;
    static_assert(vm >= 0 && vm <= 63, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((vm & 15) | (7 << 4) | ((vm >> 4) << 14));  // vmcnt(vm) lgkmcnt(0)
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  // Entering stage sti: its blocks have landed and every wavefront is done with stage
  // sti - 1, whose buffer now receives stage sti + NBUF - 1.  Only the copies of the
  // stages after sti (and, at the first stage, the tile's state loads: HS NR / 2, or
  // HS NR from the user vector) may still be in flight; loads complete in order, and
  // each level waits for the slots it takes.
  constexpr auto loads_of = [](int st) {
    return T::kHB * (is_leaf_group<K, LI, LO>(st / T::kNPART) ? kLeafBytes<16> / 1024 : 8) / (2 * CP);
  };
  constexpr auto pending = [loads_of](int sti) {
    constexpr int nst = ((LI ? 1 : 0) + K + (LO ? 1 : 0)) * T::kNPART;
    int c = 0;
    for (int st = sti + 1; st <= sti + T::kNBUF - 2 && st < nst; ++st) c += loads_of(st);
    return c;
  };
  auto stage_begin = [&](auto STI) {
    constexpr int sti = STI;
    constexpr int state_loads = LI ? HS * NR : HS * NR / 2;
    barrier_after(std::integral_constant<int, pending(sti) + (sti == 0 ? state_loads : 0)>{});
    if constexpr (sti + NBUF - 1 < NST) issue_stage(std::integral_constant<int, sti + NBUF - 1>{});
  };
  // leaf blocks: slots 2 bw, 2 bw + 1 of this half
  auto pair_group = [&](auto GG) {
    constexpr int g = GG;
    static_for<WB>([&](auto BW) {
      constexpr int bw = BW;
      if constexpr (bw % PB == 0) stage_begin(std::integral_constant<int, g * NPART + bw / PB>{});
      float t0[SW], t1[SW];
      step(GG, BW, st[2 * bw], st[2 * bw + 1], t0, t1);
      // leaf-in: columns past nrhs (loaded from column 0) become zeros, as every
      // activation buffer holds there
      const bool keep = !(LI && g == 0) || col_ok;
      static_for<SW>([&](auto JJ) {
        st[2 * bw][JJ] = keep ? t0[JJ] : 0.f;
        st[2 * bw + 1][JJ] = keep ? t1[JJ] : 0.f;
      });
    });
  };

  // copy of this half's state after d levels into a.lvl[d] (activation layout)
  auto store_depth = [&](int d) {
    f32x4 *dst = static_cast<f32x4 *>(a.lvl[d]);
    if (!dst || !active) return;
    static_for<HS>([&](auto J) {
      constexpr int j = J;
      const int64_t slot = slot_at_depth<K>(a, base, lo, qh + j, d);
      f32x4 *p = dst + ((chunk * a.nslots + slot) * 8) * 16 + n;
      static_for<NR / 2>([&](auto JJ) {
        constexpr int jj = JJ;
        const f32x4 v = {st[j][2 * jj], st[j][NR + 2 * jj], st[j][2 * jj + 1], st[j][NR + 2 * jj + 1]};
        __builtin_nontemporal_store(v, p + G::pair(e, jj) * 16);
      });
    });
  };

  if constexpr (LI) pair_group(std::integral_constant<int, 0>{});
  if (LI || a.in_kind == kInMiddle) store_depth(0);

  // ---- levels 0 .. K-2 inside the half
  static_for<K - 1>([&](auto D) {
    constexpr int d = D;
    constexpr int g = (LI ? 1 : 0) + d;
    float nx[HS][SW];
    static_for<WB>([&](auto BW) {
      constexpr int bw = BW;
      if constexpr (bw % PB == 0) stage_begin(std::integral_constant<int, g * NPART + bw / PB>{});
      constexpr int ap = bw >> d, b = bw & ((1 << d) - 1);
      constexpr int qi0 = (2 * ap) * (1 << d) + b, qi1 = qi0 + (1 << d);
      constexpr int qo0 = ap * (2 << d) + 2 * b, qo1 = qo0 + 1;
      step(std::integral_constant<int, g>{}, BW, st[qi0], st[qi1], nx[qo0], nx[qo1]);
    });
    static_for<HS>([&](auto Q) {
      static_for<SW>([&](auto JJ) { st[Q][JJ] = nx[Q][JJ]; });
    });
    store_depth(d + 1);
  });

  // a pass run only for the states inside it has stored them all; it ends once the
  // block copies still in flight have landed (none may land after the workgroup)
  if constexpr (IO) {
    __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));  // vmcnt(0)
    return;
  }

  // ---- swap halves through the swap region: kp[k] is the operand this
  // wavefront keeps for block half WB + k, rv[k] the one it receives
  constexpr int gl = (LI ? 1 : 0) + K - 1;  // group of the last level
  float kp[WB][SW], rv[WB][SW];
  static_for<WB>([&](auto KK) {
    constexpr int k = KK;
    static_for<SW>([&](auto JJ) {
      const float a0 = st[k][JJ], a1 = st[WB + k][JJ];
      kp[k][JJ] = half ? a1 : a0;
      st[k][JJ] = half ? a0 : a1;  // the operand sent to the other half
    });
  });
  static_for<T::kRounds>([&](auto R) {
    constexpr int r0 = R * T::kSR;
    if constexpr (R > 0) barrier_after(std::integral_constant<int, 63>{});  // the previous round's reads are done
    static_for<T::kSR>([&](auto S) {
      constexpr int k = r0 + S;
      if constexpr (k < WB) {
        f32x4 *w = reinterpret_cast<f32x4 *>(swap + ((wave * T::kSR + S) * 2) * 1024) + lane;
        w[0] = f32x4{st[k][0], st[k][1], st[k][2], st[k][3]};
        w[64] = f32x4{st[k][4], st[k][5], st[k][6], st[k][7]};
      }
    });
    barrier_after(std::integral_constant<int, 63>{});  // this round's writes are done
    static_for<T::kSR>([&](auto S) {
      constexpr int k = r0 + S;
      if constexpr (k < WB) {
        const f32x4 *rp =
            reinterpret_cast<const f32x4 *>(swap + (((wave ^ 1) * T::kSR + S) * 2) * 1024) + lane;
        const f32x4 u0 = rp[0], u1 = rp[64];
        rv[k][0] = u0.x; rv[k][1] = u0.y; rv[k][2] = u0.z; rv[k][3] = u0.w;
        rv[k][4] = u1.x; rv[k][5] = u1.y; rv[k][6] = u1.z; rv[k][7] = u1.w;
      }
    });
  });

  // ---- last level: blocks b = half WB + k, inputs slots b and HS + b
  static_for<WB>([&](auto BW) {
    constexpr int k = BW;
    if constexpr (k % PB == 0) stage_begin(std::integral_constant<int, gl * NPART + k / PB>{});
    float x0[SW], x1[SW];
    static_for<SW>([&](auto JJ) {
      x0[JJ] = half ? rv[k][JJ] : kp[k][JJ];
      x1[JJ] = half ? kp[k][JJ] : rv[k][JJ];
    });
    step(std::integral_constant<int, gl>{}, BW, x0, x1, st[2 * k], st[2 * k + 1]);
  });
  if constexpr (LO) store_depth(K);

  if constexpr (LO) pair_group(std::integral_constant<int, (LI ? 1 : 0) + K>{});

  // ---- outputs at depth K (a.out == nullptr: only the per-depth copies are wanted)
  if (!active || !a.out) return;
  static_for<HS>([&](auto J) {
    constexpr int j = J;
    const int64_t q = qh + j;
    const int64_t slot = a.mode_si ? base + (lo << K) + q : base + (q << a.log_slo) + lo;
    if constexpr (LO) {
      if (col_ok) {
        f32x2 *u = static_cast<f32x2 *>(a.out);
        static_for<NR>([&](auto RHO) {
          constexpr int rho = RHO;
          const f32x2 v = {st[j][rho], st[j][NR + rho]};
          __builtin_nontemporal_store(v, &u[(slot * kRank + G::row(e, rho)) * a.ld + col]);
        });
      }
    } else {
      f32x4 *p = static_cast<f32x4 *>(a.out) + ((chunk * a.nslots + slot) * 8) * 16 + n;
      static_for<NR / 2>([&](auto JJ) {
        constexpr int jj = JJ;
        const f32x4 v = {st[j][2 * jj], st[j][NR + 2 * jj], st[j][2 * jj + 1], st[j][NR + 2 * jj + 1]};
        __builtin_nontemporal_store(v, p + G::pair(e, jj) * 16);
      });
    }
  });
}

// One workgroup per (tile, group of up to kMaxWaves column chunks).
template <int COLS, int K>
inline int64_t waves_per_group(const FusedArgs &a) {
  const int64_t mw = PassTraits<COLS, K>::kMaxWaves;
  return a.nchunks < mw ? a.nchunks : mw;
}

// Launch one pass (defined in bf_fused_<prec>.hip).  inner_only: the pass runs only
// for its per-depth copies strictly inside it (no output, no copy after its last
// level); the passes with two wavefronts per tile then launch a variant that ends
// after the levels each wavefront holds on its own.
template <int PREC>
hipError_t launch_prec(FusedArgs a, int cols, int K, bool leaf_in, bool leaf_out, bool split,
                       hipStream_t s, bool inner_only = false);
// Launch one FP64 pass (bf_fused_f64.hip; 16 columns per wavefront, K <= 4).
hipError_t launch_f64(FusedArgs a, int K, bool leaf_in, bool leaf_out, hipStream_t s);

#define BF_FUSED_LAUNCH(COLS, KK, PREC, LI, LO)                                               \
  do {                                                                                        \
    const int64_t w = waves_per_group<COLS, KK>(a);                                           \
    a.ngroups = (int)((a.nchunks + w - 1) / w);                                               \
    hipLaunchKernelGGL((k_fused_pass<COLS, KK, PREC, LI, LO>),                                \
                       dim3((unsigned)(a.ntiles * a.ngroups)), dim3((unsigned)(w * 64)), 0, s, \
                       a);                                                                    \
  } while (0)

template <int K, int PREC, bool LI, bool LO, int CP, bool IO>
void launch_x2(FusedArgs a, hipStream_t s) {
  a.ngroups = (int)((a.nchunks + CP - 1) / CP);
  hipLaunchKernelGGL((k_fused_pass_x2<K, PREC, LI, LO, CP, IO>), dim3((unsigned)(a.ntiles * a.ngroups)),
                     dim3((unsigned)(CP * 128)), 0, s, a);
}

// column chunks per workgroup: the most (up to BF_SPLIT_MAX_PAIRS) that the column count fills
#define BF_FUSED_LAUNCH_X2(KK, PREC, LI, LO, IO)                                    \
  do {                                                                              \
    if (a.nchunks >= BF_SPLIT_MAX_PAIRS)                                            \
      launch_x2<KK, PREC, LI, LO, BF_SPLIT_MAX_PAIRS, IO>(a, s);                    \
    else if (a.nchunks >= 2)                                                        \
      launch_x2<KK, PREC, LI, LO, 2, IO>(a, s);                                     \
    else                                                                            \
      launch_x2<KK, PREC, LI, LO, 1, IO>(a, s);                                     \
  } while (0)

// keys 256 + ...: full passes; 512 + ...: passes run only for their inner states
#define BF_FUSED_CASES_X2(KK, PREC)                            \
  case 256 + KK * 4 + 0:                                       \
    BF_FUSED_LAUNCH_X2(KK, PREC, false, false, false);         \
    break;                                                     \
  case 256 + KK * 4 + 2:                                       \
    BF_FUSED_LAUNCH_X2(KK, PREC, true, false, false);          \
    break;                                                     \
  case 256 + KK * 4 + 1:                                       \
    BF_FUSED_LAUNCH_X2(KK, PREC, false, true, false);          \
    break;                                                     \
  case 512 + KK * 4 + 0:                                       \
    BF_FUSED_LAUNCH_X2(KK, PREC, false, false, true);          \
    break;                                                     \
  case 512 + KK * 4 + 2:                                       \
    BF_FUSED_LAUNCH_X2(KK, PREC, true, false, true);           \
    break;

#define BF_FUSED_CASES(COLS, KK, PREC)                         \
  case (COLS / 16) * 64 + KK * 4 + 0:                          \
    BF_FUSED_LAUNCH(COLS, KK, PREC, false, false);             \
    break;                                                     \
  case (COLS / 16) * 64 + KK * 4 + 2:                          \
    BF_FUSED_LAUNCH(COLS, KK, PREC, true, false);              \
    break;                                                     \
  case (COLS / 16) * 64 + KK * 4 + 1:                          \
    BF_FUSED_LAUNCH(COLS, KK, PREC, false, true);              \
    break;

#define BF_FUSED_DEFINE_LAUNCH(PREC)                                                        \
  template <>                                                                               \
  hipError_t launch_prec<PREC>(FusedArgs a, int cols, int K, bool li, bool lo, bool split, \
                               hipStream_t s, bool inner_only) {                            \
    const int key = split && cols == 16 ? (inner_only && !lo ? 512 : 256) : (cols / 16) * 64; \
    switch (key + K * 4 + (li ? 2 : 0) + (lo ? 1 : 0)) {                                    \
      BF_FUSED_CASES(32, 1, PREC)                                                           \
      BF_FUSED_CASES(32, 2, PREC)                                                           \
      BF_FUSED_CASES(32, 3, PREC)                                                           \
      BF_FUSED_CASES(16, 1, PREC)                                                           \
      BF_FUSED_CASES(16, 2, PREC)                                                           \
      BF_FUSED_CASES(16, 3, PREC)                                                           \
      BF_FUSED_CASES(16, 4, PREC)                                                           \
      BF_FUSED_CASES_X2(3, PREC)                                                            \
      BF_FUSED_CASES_X2(4, PREC)                                                            \
      default:                                                                              \
        return hipErrorInvalidValue;                                                        \
    }                                                                                       \
    return hipGetLastError();                                                               \
  }

}  // namespace fused
}  // namespace bfly
