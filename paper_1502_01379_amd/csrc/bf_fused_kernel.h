// Device code of the fused MFMA passes (binary trees, 16-point leaves, rank 16).
//
// A pass applies K consecutive butterfly levels (plus, at the ends of the
// product, the leaf blocks or the middle weights) to one tile of 2^K slots.
// One wavefront owns 32 right-hand-side columns of the tile and keeps all of
// its 2^K slots in registers for the whole pass:
//
//   lane l: column n = l % 32 of the chunk, half eta = l / 32;
//   slot q: 8 complex rows per lane, rows {4 eta .. 4 eta + 3, 8 + 4 eta .. 11 + 4 eta}
//           of the slot's r = 16 coefficients.
//
// A butterfly (two input slots -> two output slots, one 32 x 32 complex block;
// Sec. 3.2.1 and 3.2.2: G^l_{2i+c,j} acting on [z_{i,2j}; z_{i,2j+1}], and the
// H analogue) is two real 32 x 32 x 64 products on the matrix cores:
//   Re(out) = [Re M, -Im M] . [Re x; Im x],  Im(out) = [Re M, -Im M] . [Im x; -Re x].
// The 32 x 32 accumulator of v_mfma_*_32x32 leaves, in each lane, exactly the
// rows that the next level's B operand needs from that lane, so the
// interleaving of slots between levels is register renaming: no LDS, no
// cross-lane traffic.  The A operands (the blocks) are packed on the host in
// per-lane order, 8 KB per block, streamed through L2 one block ahead of use.
//
// Precisions: FP32 (v_mfma_f32_32x32x2_f32), and split BF16 / FP16
// (x = hi + lo, three v_mfma_f32_32x32x16 products lo*hi + hi*lo + hi*hi with
// FP32 accumulation; FP16 also scales each block and each column by a power
// of two to stay inside the FP16 range).
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
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kRank = 16;          // r == n0 == 16
constexpr int kBlockBytes = 8192;  // packed A operands of one 32 x 32 complex block
constexpr int kMaxK = 4;          // deepest compiled pass
constexpr int kDefaultK = 3;      // deepest pass used unless BF_FUSED_KMAX says otherwise
constexpr int kWaves = 8;          // most wavefronts (right-hand-side chunks) per workgroup

enum InKind : int { kInAct = 0, kInUser = 1, kInMiddle = 2 };
enum OutKind : int { kOutAct = 0, kOutUser = 1 };
enum Prec : int { kF32 = 0, kBF16 = 1, kF16 = 2 };

struct FusedArgs {
  const void *in;
  void *out;
  const char *fac;      // [K][ntiles][2^(K-1)] blocks
  const char *leaf;     // [ntiles][2^(K-1)] blocks (leaf in or leaf out)
  const float *fscale;  // FP16: power-of-two scale per block, same order as fac
  const float *lscale;  // FP16: same for leaf blocks
  const float *Sm;      // middle weights in natural slot order (kInMiddle)
  int64_t ld, nrhs, nchunks, nslots, ntiles, m;
  int log_slo, mode_si, in_kind, out_kind;
};

struct BlockA {
  u32x4 v[8];  // this lane's 128 bytes of one packed block
};

__device__ __forceinline__ int row_of(int eta, int rho) {
  return rho < 4 ? 4 * eta + rho : 8 + 4 * eta + (rho - 4);
}

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

// ---- one 32 x 32 complex block: (x0, x1) -> (y0, y1) ---------------------------
__device__ __forceinline__ void block_f32(const BlockA &A, const float *x0r, const float *x0i,
                                          const float *x1r, const float *x1i, float *y0r,
                                          float *y0i, float *y1r, float *y1i) {
  floatx16 dr = {}, di = {};
#pragma unroll
  for (int s = 0; s < 32; ++s) {
    const float a = as_f32(A.v[s >> 2], s & 3);
    const int part = s >> 4, cp = (s >> 3) & 1, rho = s & 7;
    const float xre = cp ? x1r[rho] : x0r[rho];
    const float xim = cp ? x1i[rho] : x0i[rho];
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
    y0r[rho] = dr[rho];
    y1r[rho] = dr[8 + rho];
    y0i[rho] = di[rho];
    y1i[rho] = di[8 + rho];
  }
}

template <class H8, class Hs>
__device__ __forceinline__ void split8(const float *x, float s, H8 &hi, H8 &lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float v = x[j] * s;
    const Hs h = (Hs)v;
    hi[j] = h;
    lo[j] = (Hs)(v - (float)h);
  }
}

// flip the sign bit of eight 16-bit values
template <class H8>
__device__ __forceinline__ H8 neg8(const H8 &x) {
  u32x4 u = __builtin_bit_cast(u32x4, x);
  u ^= 0x80008000u;
  return __builtin_bit_cast(H8, u);
}

__device__ __forceinline__ floatx16 mfma16(const bf16x8 &a, const bf16x8 &b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx16 mfma16(const halfx8 &a, const halfx8 &b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// Split precision: K step t = 2 part + c' covers the 8 rows of input slot c' in
// this lane (part 0: real parts, part 1: imaginary parts).  A.v[t] holds the hi
// halves of step t, A.v[4 + t] the lo halves.
template <class H8, class Hs, bool kScale>
__device__ __forceinline__ void block_split(const BlockA &A, float bscale, const float *x0r,
                                            const float *x0i, const float *x1r,
                                            const float *x1i, float *y0r, float *y0i, float *y1r,
                                            float *y1i) {
  float cs = 1.f, inv = 1.f;
  if (kScale) {
    // per-column power-of-two scale over both halves of the column
    float mx = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      mx = fmaxf(mx, fmaxf(fmaxf(fabsf(x0r[j]), fabsf(x0i[j])), fmaxf(fabsf(x1r[j]), fabsf(x1i[j]))));
    mx = fmaxf(mx, __shfl_xor(mx, 32));
    int e = 0;
    if (mx > 0.f) (void)frexpf(mx, &e);
    cs = ldexpf(1.f, -e);
    inv = ldexpf(bscale, e);
  }
  H8 xh[4], xl[4];
  split8<H8, Hs>(x0r, cs, xh[0], xl[0]);
  split8<H8, Hs>(x1r, cs, xh[1], xl[1]);
  split8<H8, Hs>(x0i, cs, xh[2], xl[2]);
  split8<H8, Hs>(x1i, cs, xh[3], xl[3]);
  floatx16 dr = {}, di = {};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const H8 ahi = __builtin_bit_cast(H8, A.v[t]);
    const H8 alo = __builtin_bit_cast(H8, A.v[4 + t]);
    dr = mfma16(alo, xh[t], dr);
    dr = mfma16(ahi, xl[t], dr);
    dr = mfma16(ahi, xh[t], dr);
    const H8 yh = t < 2 ? xh[t + 2] : neg8(xh[t - 2]);
    const H8 yl = t < 2 ? xl[t + 2] : neg8(xl[t - 2]);
    di = mfma16(alo, yh, di);
    di = mfma16(ahi, yl, di);
    di = mfma16(ahi, yh, di);
  }
#pragma unroll
  for (int rho = 0; rho < 8; ++rho) {
    y0r[rho] = dr[rho] * inv;
    y1r[rho] = dr[8 + rho] * inv;
    y0i[rho] = di[rho] * inv;
    y1i[rho] = di[8 + rho] * inv;
  }
}

template <int PREC>
__device__ __forceinline__ void block_op(const BlockA &A, float bscale, const float *x0r,
                                         const float *x0i, const float *x1r, const float *x1i,
                                         float *y0r, float *y0i, float *y1r, float *y1i) {
  if constexpr (PREC == kF32)
    block_f32(A, x0r, x0i, x1r, x1i, y0r, y0i, y1r, y1i);
  else if constexpr (PREC == kBF16)
    block_split<bf16x8, __bf16, false>(A, 1.f, x0r, x0i, x1r, x1i, y0r, y0i, y1r, y1i);
  else
    block_split<halfx8, _Float16, true>(A, bscale, x0r, x0i, x1r, x1i, y0r, y0i, y1r, y1i);
}

// Block operands in the order the pass consumes them: leaf-in pairs, then
// depth 0 .. K-1 butterflies, then leaf-out pairs.
template <int K, bool LI>
__device__ __forceinline__ int64_t op_block(const FusedArgs &a, int64_t tile, int o,
                                            const char *&base_ptr, const float *&scale_ptr) {
  constexpr int NB = 1 << (K - 1);
  if (LI && o < NB) {
    base_ptr = a.leaf;
    scale_ptr = a.lscale;
    return tile * NB + o;
  }
  const int o2 = o - (LI ? NB : 0);
  if (o2 < K * NB) {
    base_ptr = a.fac;
    scale_ptr = a.fscale;
    return ((int64_t)(o2 / NB) * a.ntiles + tile) * NB + (o2 % NB);
  }
  base_ptr = a.leaf;
  scale_ptr = a.lscale;
  return tile * NB + (o2 - K * NB);
}

// Passes of up to three levels are compiled for two resident wavefronts per
// SIMD (at most 256 registers) and fetch each block right before use; the
// other wavefront hides that latency.  Four-level passes need the whole SIMD
// register file for their 16 slots and prefetch one block ahead instead.
template <int K>
struct PassTraits {
  static constexpr bool kPrefetch = K >= 4;
  static constexpr int kWavesPerEU = K >= 4 ? 1 : 2;
  static constexpr int kMaxWaves = K >= 4 ? 4 : kWaves;  // wavefronts per workgroup
};

template <int K, int PREC, bool LI, bool LO>
__global__ __launch_bounds__(PassTraits<K>::kMaxWaves * 64)
__attribute__((amdgpu_waves_per_eu(PassTraits<K>::kWavesPerEU)))
void k_fused_pass(FusedArgs a) {
  constexpr int NS = 1 << K;
  constexpr int NB = NS / 2;
  constexpr int NOPS = (LI ? NB : 0) + K * NB + (LO ? NB : 0);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = lane & 31, eta = lane >> 5;
  const int64_t chunk = (int64_t)blockIdx.y * (blockDim.x >> 6) + wave;
  if (chunk >= a.nchunks) return;
  const int64_t tile = blockIdx.x;
  const int64_t slo = int64_t(1) << a.log_slo;
  const int64_t hi = tile >> a.log_slo, lo = tile & (slo - 1);
  const int64_t base = hi << (K + a.log_slo);
  const int64_t col = chunk * 32 + n;
  const bool col_ok = col < a.nrhs;

  auto fetch = [&](int o, float &bs) {
    const char *bp;
    const float *sp;
    const int64_t bi = op_block<K, LI>(a, tile, o, bp, sp);
    bs = (PREC == kF16) ? sp[bi] : 1.f;
    return load_block(bp + bi * kBlockBytes, lane);
  };
  float bs_cur;
  BlockA cur = fetch(0, bs_cur);

  // st[q][0..7] real, st[q][8..15] imaginary parts of this lane's rows of slot q
  float st[NS][16];

  // ---- inputs at depth 0
  static_for<NS>([&](auto Q) {
    constexpr int q = Q;
    const int64_t slot = a.mode_si ? base + ((int64_t)q << a.log_slo) + lo : base + (lo << K) + q;
    if constexpr (LI) {
      const f32x2 *g = static_cast<const f32x2 *>(a.in);
      static_for<8>([&](auto RHO) {
        constexpr int rho = RHO;
        f32x2 v = {0.f, 0.f};
        if (col_ok) v = __builtin_nontemporal_load(&g[(slot * kRank + row_of(eta, rho)) * a.ld + col]);
        st[q][rho] = v.x;
        st[q][8 + rho] = v.y;
      });
    } else {
      int64_t src = slot;
      if (a.in_kind == kInMiddle) {
        const int64_t sh = slot / a.m;
        src = (slot - sh * a.m) * a.m + sh;
      }
      const f32x4 *p = static_cast<const f32x4 *>(a.in) + ((chunk * a.nslots + src) * 8) * 32 + n;
      static_for<4>([&](auto J) {
        constexpr int j = J;
        const int pair = (j < 2) ? 2 * eta + j : 4 + 2 * eta + (j - 2);
        const f32x4 v = __builtin_nontemporal_load(p + pair * 32);
        st[q][2 * j] = v.x;
        st[q][8 + 2 * j] = v.y;
        st[q][2 * j + 1] = v.z;
        st[q][8 + 2 * j + 1] = v.w;
      });
      if (a.in_kind == kInMiddle) {
        const f32x4 *sp = reinterpret_cast<const f32x4 *>(a.Sm + slot * kRank);
        const f32x4 s0 = sp[eta], s1 = sp[2 + eta];
        static_for<8>([&](auto RHO) {
          constexpr int rho = RHO;
          const float sc = rho < 4 ? pick4(s0, rho & 3) : pick4(s1, rho & 3);
          st[q][rho] *= sc;
          st[q][8 + rho] *= sc;
        });
      }
    }
  });

  // one block operation (op index O) with the next block's operands in flight
  auto step = [&](auto O, const float *x0, const float *x1, float *y0, float *y1) {
    constexpr int o = O;
    if constexpr (PassTraits<K>::kPrefetch) {
      float bs_nxt = 1.f;
      BlockA nxt;
      if constexpr (o + 1 < NOPS) nxt = fetch(o + 1, bs_nxt);
      block_op<PREC>(cur, bs_cur, x0, x0 + 8, x1, x1 + 8, y0, y0 + 8, y1, y1 + 8);
      if constexpr (o + 1 < NOPS) {
        cur = nxt;
        bs_cur = bs_nxt;
      }
    } else {
      if constexpr (o > 0) cur = fetch(o, bs_cur);
      block_op<PREC>(cur, bs_cur, x0, x0 + 8, x1, x1 + 8, y0, y0 + 8, y1, y1 + 8);
    }
    __builtin_amdgcn_sched_barrier(0);
  };

  // ---- leaf blocks applied to slot pairs before the first level
  if constexpr (LI) {
    static_for<NB>([&](auto PP) {
      constexpr int pp = PP;
      float t0[16], t1[16];
      step(std::integral_constant<int, pp>{}, st[2 * pp], st[2 * pp + 1], t0, t1);
      static_for<16>([&](auto J) {
        st[2 * pp][J] = t0[J];
        st[2 * pp + 1][J] = t1[J];
      });
    });
  }

  // ---- K butterfly levels
  static_for<K>([&](auto D) {
    constexpr int d = D;
    float nx[NS][16];
    static_for<NB>([&](auto BETA) {
      constexpr int beta = BETA;
      constexpr int ap = beta >> d, b = beta & ((1 << d) - 1);
      constexpr int qi0 = (2 * ap) * (1 << d) + b, qi1 = (2 * ap + 1) * (1 << d) + b;
      constexpr int qo0 = ap * (2 << d) + 2 * b, qo1 = qo0 + 1;
      constexpr int o = (LI ? NB : 0) + d * NB + beta;
      step(std::integral_constant<int, o>{}, st[qi0], st[qi1], nx[qo0], nx[qo1]);
    });
    static_for<NS>([&](auto Q) {
      static_for<16>([&](auto J) { st[Q][J] = nx[Q][J]; });
    });
  });

  // ---- leaf blocks after the last level
  if constexpr (LO) {
    static_for<NB>([&](auto PP) {
      constexpr int pp = PP;
      constexpr int o = (LI ? NB : 0) + K * NB + pp;
      float t0[16], t1[16];
      step(std::integral_constant<int, o>{}, st[2 * pp], st[2 * pp + 1], t0, t1);
      static_for<16>([&](auto J) {
        st[2 * pp][J] = t0[J];
        st[2 * pp + 1][J] = t1[J];
      });
    });
  }

  // ---- outputs at depth K
  static_for<NS>([&](auto Q) {
    constexpr int q = Q;
    const int64_t slot = a.mode_si ? base + (lo << K) + q : base + ((int64_t)q << a.log_slo) + lo;
    if constexpr (LO) {
      if (col_ok) {
        f32x2 *u = static_cast<f32x2 *>(a.out);
        static_for<8>([&](auto RHO) {
          constexpr int rho = RHO;
          const f32x2 v = {st[q][rho], st[q][8 + rho]};
          __builtin_nontemporal_store(v, &u[(slot * kRank + row_of(eta, rho)) * a.ld + col]);
        });
      }
    } else {
      f32x4 *p = static_cast<f32x4 *>(a.out) + ((chunk * a.nslots + slot) * 8) * 32 + n;
      static_for<4>([&](auto J) {
        constexpr int j = J;
        const int pair = (j < 2) ? 2 * eta + j : 4 + 2 * eta + (j - 2);
        const f32x4 v = {st[q][2 * j], st[q][8 + 2 * j], st[q][2 * j + 1], st[q][8 + 2 * j + 1]};
        __builtin_nontemporal_store(v, p + pair * 32);
      });
    }
  });
}

// One workgroup per tile and group of up to kMaxWaves right-hand-side chunks.
template <int K>
inline dim3 launch_block(const FusedArgs &a) {
  const int64_t w = a.nchunks < PassTraits<K>::kMaxWaves ? a.nchunks : PassTraits<K>::kMaxWaves;
  return dim3((unsigned)(w * 64));
}
template <int K>
inline dim3 launch_grid(const FusedArgs &a) {
  const int64_t w = a.nchunks < PassTraits<K>::kMaxWaves ? a.nchunks : PassTraits<K>::kMaxWaves;
  return dim3((unsigned)a.ntiles, (unsigned)((a.nchunks + w - 1) / w));
}

// Launch one pass of precision PREC (defined in bf_fused_<prec>.hip).
template <int PREC>
hipError_t launch_prec(const FusedArgs &a, int K, bool leaf_in, bool leaf_out, hipStream_t s);

#define BF_FUSED_DEFINE_LAUNCH(PREC)                                                      \
  template <>                                                                             \
  hipError_t launch_prec<PREC>(const FusedArgs &a, int K, bool li, bool lo,              \
                               hipStream_t s) {                                           \
    switch (K * 4 + (li ? 2 : 0) + (lo ? 1 : 0)) {                                        \
      BF_FUSED_CASES(1, PREC)                                                             \
      BF_FUSED_CASES(2, PREC)                                                             \
      BF_FUSED_CASES(3, PREC)                                                             \
      BF_FUSED_CASES(4, PREC)                                                             \
      default:                                                                            \
        return hipErrorInvalidValue;                                                      \
    }                                                                                     \
    return hipGetLastError();                                                             \
  }

#define BF_FUSED_CASES(KK, PREC)                                                              \
  case KK * 4 + 0:                                                                            \
    hipLaunchKernelGGL((k_fused_pass<KK, PREC, false, false>), launch_grid<KK>(a),            \
                       launch_block<KK>(a), 0, s, a);                                         \
    break;                                                                                    \
  case KK * 4 + 2:                                                                            \
    hipLaunchKernelGGL((k_fused_pass<KK, PREC, true, false>), launch_grid<KK>(a),             \
                       launch_block<KK>(a), 0, s, a);                                         \
    break;                                                                                    \
  case KK * 4 + 1:                                                                            \
    hipLaunchKernelGGL((k_fused_pass<KK, PREC, false, true>), launch_grid<KK>(a),             \
                       launch_block<KK>(a), 0, s, a);                                         \
    break;

}  // namespace fused
}  // namespace bfly
