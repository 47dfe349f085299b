// FP64 fused passes (binary trees, 16-point leaves, rank 16, 16 columns per
// wavefront): the pass structure of bf_fused_kernel.h with FP64 state, FP64
// blocks and the FP64 matrix cores.
//
// Lane geometry: lane l holds column l % 16 and, of every slot, rows e, e + 4,
// e + 8, e + 12 (e = l / 16; rho-th value: row 4 rho + e), four complex values in
// eight doubles (real parts, then imaginary parts).  This is the accumulator
// layout of v_mfma_f64_16x16x4_f64 (value rho of lane (n, e) is row 4 rho + e of
// the 16 x 16 tile, unlike the 16 x 16 FP32 products, whose lanes hold four
// consecutive rows).  A butterfly (two input slots -> two output slots, one
// 32 x 32 complex block; Sec. 3.2.1 and 3.2.2) is computed on those products with
// Gauss's three real products per complex one: with a = Re M, b = Im M,
// x = Re in, y = Im in,
//   P1 = a x,  P2 = b y,  P3 = (a + b)(x + y);   Re out = P1 - P2,  Im out = P3 - P1 - P2.
// K step k = 4c' + rho of one 16-row output tile takes row 4 rho + e of input slot
// c' from lane (n, e), so the accumulator of one level again holds the rows the
// next level's operand needs from that lane: slots move between levels by
// register renaming.
//
// Tiles: passes of three or four levels give each tile to a pair of wavefronts
// (wavefront h holds the tile slots h 2^(K-1) + j), which swap half of their
// slots through LDS before the last level, as k_fused_pass_x2 does; shallower
// passes give the tile to one wavefront.  Blocks stream into LDS with
// global -> LDS loads, one block (or half block) per wavefront position and stage,
// one stage (or three half-block stages) ahead.  A workgroup holds up to two column
// chunks of one tile (80 KB of LDS, so two workgroups share a CU and overlap each
// other's loads; four chunks per workgroup, one workgroup per CU, were 5% slower at
// N = 2^20, 256 columns); workgroups of one tile get ids eight apart (same XCD,
// shared L2).
#include <hip/hip_runtime.h>

#include "bf_fused_kernel.h"

namespace bfly {
namespace fused {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

#ifndef BF_F64_MAX_CHUNKS
#define BF_F64_MAX_CHUNKS 2
#endif
#ifndef BF_F64_STAGE_BUFFERS
#define BF_F64_STAGE_BUFFERS 2
#endif
// Stages per block: whole blocks through two buffers (PARTS 1), or two halves, one
// per output tile, through four buffers in the same LDS (PARTS 2: the copies run
// one and a half blocks ahead).  Measured at N = 2^20, 256 columns, same box and
// process: halves take the leaf-out pass from 4.34 to 4.19 ms, whole blocks the
// middle passes from 3.88 to 3.82 ms; leaf-in passes are even.
#ifndef BF_F64_PARTS
#define BF_F64_PARTS 1
#endif
#ifndef BF_F64_PARTS_LO
#define BF_F64_PARTS_LO 2
#endif

// CW column chunks per workgroup; blocks stream through NBUF LDS stage buffers,
// NBUF - 1 stages ahead of the one being computed.
template <int K, int CW, int NBUF, int PARTS>
struct F64Traits {
  static constexpr int kW = K >= 3 ? 2 : 1;                 // wavefronts per tile of one chunk
  static constexpr int kHS = (1 << K) / kW;                 // slots per wavefront
  static constexpr int kWB = kHS / 2;                       // blocks per wavefront per level
  static constexpr int kWaves = CW * kW;                    // wavefronts per workgroup
  static constexpr int kParts = PARTS;                      // stages per block (1, or one per output tile)
  static constexpr int kStageBytes = kW * kBlockBytes64 / kParts;  // a block (part) per wavefront position
  static constexpr int kSlotBytes = 4096;                   // one slot of one wavefront (64 x 8 doubles)
  // the half-swap region (one slot per wavefront per round) also stages the middle
  // weights of each wavefront's slots (1 KB per wavefront) before the first level
  static constexpr int kSwapBytes = kW == 2 ? kWaves * kSlotBytes : kWaves * 1024;
  static constexpr int kLdsBytes = NBUF * kStageBytes + kSwapBytes;
};

// s_waitcnt immediate (gfx9 encoding): at most vm vector-memory operations of this
// wavefront outstanding, no LDS operation outstanding, any export count.
constexpr int waitcnt_vm(int vm) { return (vm & 15) | (7 << 4) | ((vm >> 4) << 14); }

// Block beta of group g (leaf-in, levels 0 .. K-1, leaf-out).
template <int K, bool LI>
__device__ __forceinline__ const char *block64(const FusedArgs &a, int64_t tile, int g, int beta) {
  constexpr int NB = 1 << (K - 1);
  const int d = g - (LI ? 1 : 0);
  if (d < 0 || d >= K) return a.leaf + (tile * NB + beta) * (int64_t)kLeafBytes64;
  return a.fac + (((int64_t)d * a.ntiles + tile) * NB + beta) * (int64_t)kBlockBytes64;
}

// One output tile T (rows 16T .. 16T + 15, i.e. output slot T) of a 32 x 32 block
// times the input slots x0 (c' = 0) and x1 (c' = 1).  Packed block: lane i + 16e holds
// M[16T + i][16c' + 4 rho + e] of K step k = 4c' + rho at double
// (((2T + part) 4 + k / 2) 64 + lane) 2 + k % 2 (part 0: Re M, 1: Im M); tile T's
// operands are the 8 KB at T * 8 KB, passed here as blkT.
__device__ __forceinline__ void tile16_f64(const char *blkT, int lane, const double *x0, const double *x1,
                                           double *y) {
  const f64x2 *bp = reinterpret_cast<const f64x2 *>(blkT) + lane;
  f64x4 p1 = {}, p2 = {}, p3 = {};
  // operands of two K steps at a time (the register budget holds the state)
  f64x2 av = bp[0], bv = bp[256];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    f64x2 an = av, bn = bv;
    if (kk < 3) {
      an = bp[(kk + 1) * 64];
      bn = bp[256 + (kk + 1) * 64];
    }
#pragma unroll
    for (int k = 2 * kk; k < 2 * kk + 2; ++k) {
      const double *x = (k >> 2) ? x1 : x0;
      const int rho = k & 3;
      const double xre = x[rho], xim = x[4 + rho];
      const double am = (k & 1) ? av.y : av.x;
      const double bm = (k & 1) ? bv.y : bv.x;
      p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(am, xre, p1, 0, 0, 0);
      p2 = __builtin_amdgcn_mfma_f64_16x16x4f64(bm, xim, p2, 0, 0, 0);
      p3 = __builtin_amdgcn_mfma_f64_16x16x4f64(am + bm, xre + xim, p3, 0, 0, 0);
    }
    av = an;
    bv = bn;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    y[v] = p1[v] - p2[v];
    y[4 + v] = p3[v] - p1[v] - p2[v];
  }
}

// A leaf pair: slot c times its own 16 x 16 block M_c.  Packed pair: lane i + 16e
// holds M_c[i][4 rho + e] at double (((2c + part) 2 + rho / 2) 64 + lane) 2 + rho % 2;
// slot c's operands are the 4 KB at c * 4 KB, passed here as blkc.
__device__ __forceinline__ void leaf16_f64(const char *blkc, int lane, const double *x, double *y) {
  const f64x2 *bp = reinterpret_cast<const f64x2 *>(blkc) + lane;
  const f64x2 a01 = bp[0], a23 = bp[64], b01 = bp[128], b23 = bp[192];
  f64x4 p1 = {}, p2 = {}, p3 = {};
#pragma unroll
  for (int rho = 0; rho < 4; ++rho) {
    const f64x2 ap = rho < 2 ? a01 : a23, bp2 = rho < 2 ? b01 : b23;
    const double am = (rho & 1) ? ap.y : ap.x, bm = (rho & 1) ? bp2.y : bp2.x;
    const double xre = x[rho], xim = x[4 + rho];
    p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(am, xre, p1, 0, 0, 0);
    p2 = __builtin_amdgcn_mfma_f64_16x16x4f64(bm, xim, p2, 0, 0, 0);
    p3 = __builtin_amdgcn_mfma_f64_16x16x4f64(am + bm, xre + xim, p3, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    y[v] = p1[v] - p2[v];
    y[4 + v] = p3[v] - p1[v] - p2[v];
  }
}

// Activations (FP64): [chunk][slot][row 16][column 16] complex128; user vectors
// g, u: [N][ld] complex128.
template <int K, bool LI, bool LO, int CW, int NBUF, int PARTS>
__global__ __launch_bounds__((F64Traits<K, CW, NBUF, PARTS>::kWaves * 64)) __attribute__((amdgpu_waves_per_eu(2)))
void k_fused_pass_f64(FusedArgs a) {
  using T = F64Traits<K, CW, NBUF, PARTS>;
  constexpr int W = T::kW, HS = T::kHS, WB = T::kWB, NW = T::kWaves;
  constexpr int NST = ((LI ? 1 : 0) + K + (LO ? 1 : 0)) * WB * PARTS;
  // global -> LDS loads of one wavefront for stage s (16 or 8 pieces of 1 KB per
  // block, over PARTS stages, spread over the workgroup's NW wavefronts), and those of
  // the stages after sti that are in flight when stage sti begins
  constexpr auto loads_of = [](int s) {
    return (is_leaf_group<K, LI, LO>(s / (WB * PARTS)) ? 8 : 16) / PARTS * W / NW;
  };
  constexpr auto pending = [loads_of](int sti) {
    int n = 0;
    for (int s = sti + 1; s <= sti + NBUF - 2 && s < NST; ++s) n += loads_of(s);
    return n;
  };
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
  const int half = W == 2 ? (wave & 1) : 0;
  const int n = lane & 15, e = lane >> 4;
  int64_t tile, group;
  tile_of_block(a, tile, group);
  const int64_t chunk = group * CW + wave / W;
  const bool active = chunk < a.nchunks;
  const int64_t slo = int64_t(1) << a.log_slo;
  const int64_t hi = tile >> a.log_slo, lo = tile & (slo - 1);
  const int64_t base = hi << (K + a.log_slo);
  const int64_t col = (chunk << 4) + n;
  const bool col_ok = active && col < a.nrhs;
  const int qh = half * HS;  // first tile slot of this wavefront

  // stage sti = (group g, block bw, part): that part of block half WB + bw of group g
  // for both halves, at position half of LDS buffer sti % NBUF
  __shared__ __attribute__((aligned(16))) char lds[T::kLdsBytes];
  auto issue_stage = [&](auto STI) {
    constexpr int sti = STI;
    char *dst = lds + (sti % NBUF) * T::kStageBytes;
    constexpr int bs = sti / PARTS, part = sti % PARTS;
    constexpr int g = bs / WB, bw = bs % WB;
    constexpr int pbytes = (is_leaf_group<K, LI, LO>(g) ? kLeafBytes64 : kBlockBytes64) / PARTS;
    constexpr int lp = pbytes / 1024;  // pieces per position
    static_for<loads_of(sti)>([&](auto I) {
      const int c = wave + (int)I * NW;
      const int pos = c / lp, piece = c - pos * lp;
      const char *src = block64<K, LI>(a, tile, g, pos * WB + bw) + part * pbytes + piece * 1024 + lane * 16;
      __builtin_amdgcn_global_load_lds(
          src, (__attribute__((address_space(3))) void *)(dst + pos * (kBlockBytes64 / PARTS) + piece * 1024),
          16, 0, 0);
    });
  };
  issue_stage(std::integral_constant<int, 0>{});
  // middle weights S^h_{i,j} (real, natural slot order) of this wavefront's slots, into
  // its 1 KB of the swap region: lane l copies 16 bytes of slot l / 8 (a whole slot row
  // of 16 values per 8 lanes); applied to the state after the first stage's barrier
  const bool mid = !LI && a.in_kind == kInMiddle;
  char *const sreg = lds + NBUF * T::kStageBytes + wave * 1024;
  if (mid) {
    const int j = (lane >> 3) < HS ? (lane >> 3) : 0;
    const int64_t q = qh + j;
    const int64_t slot = a.mode_si ? base + (q << a.log_slo) + lo : base + (lo << K) + q;
    const char *src = reinterpret_cast<const char *>(a.Sm64 + slot * kRank) + (lane & 7) * 16;
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)sreg, 16, 0, 0);
  }
  // the counted waits below assume this issue order (first stage and middle weights,
  // state loads, later stages): the empty asm statements keep the compiler from
  // interleaving them
  asm volatile("" ::: "memory");

  double st[HS][8];

  // ---- inputs at depth 0: tile slots qh .. qh + HS - 1
  static_for<HS>([&](auto J) {
    constexpr int j = J;
    const int64_t q = qh + j;
    const int64_t slot = a.mode_si ? base + (q << a.log_slo) + lo : base + (lo << K) + q;
    if constexpr (LI) {
      // every lane loads (column 0 in place of a missing one), so each wavefront
      // issues the same number of loads and the first stage can wait for its blocks
      // alone (stage_begin); the leaf blocks' outputs of missing columns are zeroed
      const f64x2 *g = static_cast<const f64x2 *>(a.in);
      const int64_t cl = col_ok ? col : 0;
      static_for<4>([&](auto RHO) {
        constexpr int rho = RHO;
        const f64x2 v = __builtin_nontemporal_load(&g[(slot * kRank + 4 * rho + e) * a.ld + cl]);
        st[j][rho] = v.x;
        st[j][4 + rho] = v.y;
      });
    } else {
      // the first pass after the middle level reads the transposed slot
      const int64_t tr = ((slot & (a.m - 1)) << a.log_m) | (slot >> a.log_m);
      const int64_t src = a.in_kind == kInMiddle ? tr : slot;
      // an idle wavefront pair loads chunk 0 (see above) and stores nothing
      const int64_t ck = active ? chunk : 0;
      const f64x2 *p = static_cast<const f64x2 *>(a.in) + ((ck * a.nslots + src) * kRank + e) * 16 + n;
      static_for<4>([&](auto RHO) {
        constexpr int rho = RHO;
        const f64x2 v = __builtin_nontemporal_load(p + rho * 64);
        st[j][rho] = v.x;
        st[j][4 + rho] = v.y;
      });
    }
  });
  // the next NBUF - 2 stages follow the state loads, so the first stage's wait
  // leaves them in flight
  asm volatile("" ::: "memory");
  static_for<NBUF - 2>([&](auto I) {
    if constexpr (1 + (int)I < NST) issue_stage(std::integral_constant<int, 1 + (int)I>{});
  });

  // Barriers are bare s_barriers after explicit waits (a workgroup fence would also
  // wait for every load in flight); the empty asm statements keep the compiler from
  // moving LDS accesses across them.
  auto barrier_after = [&](auto VM) {
    constexpr int vm = VM;
    static_assert(vm >= 0 && vm <= 63, "vmcnt range");
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(vm));
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  // entering stage sti: its blocks have landed (only the copies of the stages after it
  // may still be in flight; loads complete in order), every wavefront is done with
  // stage sti - 1, whose buffer now receives stage sti + NBUF - 1.  The first stage
  // also waits for the tile's state loads, and the empty asm statements after it keep
  // the compiler from moving work on the state above the barrier: a wait of the
  // compiler's own for a state register, with block copies in flight, would be a full
  // vmcnt(0) and drain the copies of the next stages (N = 2^20, 256 columns: 16.17-16.21
  // -> 16.06-16.09 ms per apply)
  auto stage_begin = [&](auto STI) {
    constexpr int sti = STI;
    barrier_after(std::integral_constant<int, pending(sti)>{});
    if constexpr (sti == 0) {
      static_for<HS>([&](auto J) {
        static_for<8>([&](auto V) {
          double &x = st[(int)J][(int)V];
          asm volatile("" : "+v"(x));
        });
      });
      // the middle weights landed with the first stage (they were issued before the
      // state loads); read before the next copy is issued, so no copy is in flight
      // that the reads could be taken to depend on
      if (!LI && mid) {
        static_for<HS>([&](auto J) {
          static_for<4>([&](auto RHO) {
            const double sc = *reinterpret_cast<const double *>(sreg + (int)J * 128 + (4 * (int)RHO + e) * 8);
            st[J][RHO] *= sc;
            st[J][4 + RHO] *= sc;
          });
        });
      }
    }
    if constexpr (sti + NBUF - 1 < NST) issue_stage(std::integral_constant<int, sti + NBUF - 1>{});
  };
  // block half WB + bw of group g, staged in LDS (one stage per block, or one per
  // output slot with PARTS = 2), applied to x0, x1
  auto butterfly = [&](auto GG, auto BW, const double *x0, const double *x1, double *y0, double *y1) {
    constexpr int g = GG, bw = BW;
    constexpr int bs = g * WB + bw;
    constexpr bool leaf = is_leaf_group<K, LI, LO>(g);
    static_for<PARTS>([&](auto P) {
      constexpr int part = P;
      stage_begin(std::integral_constant<int, bs * PARTS + part>{});
      const char *pb = lds + ((bs * PARTS + part) % NBUF) * T::kStageBytes + half * (kBlockBytes64 / PARTS);
      static_for<2 / PARTS>([&](auto Q) {
        constexpr int c = part + Q;  // output slot (tile) of this part
        const char *cb = pb + (int)Q * (leaf ? kLeafBytes64 : kBlockBytes64) / 2;
        if constexpr (leaf)
          leaf16_f64(cb, lane, c ? x1 : x0, c ? y1 : y0);
        else
          tile16_f64(cb, lane, x0, x1, c ? y1 : y0);
      });
    });
  };
  // leaf blocks: slots 2 bw, 2 bw + 1 of this wavefront
  auto pair_group = [&](auto GG) {
    constexpr int g = GG;
    static_for<WB>([&](auto BW) {
      constexpr int bw = BW;
      double t0[8], t1[8];
      butterfly(GG, BW, st[2 * bw], st[2 * bw + 1], t0, t1);
      // leaf-in: columns past nrhs (loaded from column 0) become zeros
      const bool keep = !(LI && g == 0) || col_ok;
      static_for<8>([&](auto V) {
        st[2 * bw][V] = keep ? t0[V] : 0.0;
        st[2 * bw + 1][V] = keep ? t1[V] : 0.0;
      });
    });
  };

  if constexpr (LI) pair_group(std::integral_constant<int, 0>{});

  // ---- levels inside the wavefront: all K (one wavefront per tile) or 0 .. K-2
  constexpr int LOCAL = W == 2 ? K - 1 : K;
  static_for<LOCAL>([&](auto D) {
    constexpr int d = D;
    constexpr int g = (LI ? 1 : 0) + d;
    double nx[HS][8];
    static_for<WB>([&](auto BW) {
      constexpr int bw = BW;
      constexpr int ap = bw >> d, b = bw & ((1 << d) - 1);
      constexpr int qi0 = (2 * ap) * (1 << d) + b, qi1 = qi0 + (1 << d);
      constexpr int qo0 = ap * (2 << d) + 2 * b, qo1 = qo0 + 1;
      butterfly(std::integral_constant<int, g>{}, BW, st[qi0], st[qi1], nx[qo0], nx[qo1]);
    });
    static_for<HS>([&](auto Q) {
      static_for<8>([&](auto V) { st[Q][V] = nx[Q][V]; });
    });
  });

  if constexpr (W == 2) {
    // ---- the last level pairs slot b with slot HS + b: wavefront h' computes the
    // blocks b = h' WB + k from slot b (held by wavefront 0) and slot HS + b (held
    // by wavefront 1); each wavefront keeps the operand it holds for its own blocks
    // and sends the other one through LDS, one slot per round
    constexpr int gl = (LI ? 1 : 0) + K - 1;
    char *const swap = lds + NBUF * T::kStageBytes;
    double kp[WB][8], rv[WB][8];
    static_for<WB>([&](auto KK) {
      constexpr int k = KK;
      static_for<8>([&](auto V) {
        const double a0 = st[k][V], a1 = st[WB + k][V];
        kp[k][V] = half ? a1 : a0;
        st[k][V] = half ? a0 : a1;  // the operand sent to the other wavefront
      });
    });
    static_for<WB>([&](auto KK) {
      constexpr int k = KK;
      if constexpr (k > 0) barrier_after(std::integral_constant<int, 63>{});  // the previous round's reads are done
      f64x2 *w = reinterpret_cast<f64x2 *>(swap + wave * T::kSlotBytes) + lane;
      static_for<4>([&](auto I) {
        constexpr int i = I;
        w[64 * i] = f64x2{st[k][2 * i], st[k][2 * i + 1]};
      });
      barrier_after(std::integral_constant<int, 63>{});  // this round's writes are done
      const f64x2 *rp = reinterpret_cast<const f64x2 *>(swap + (wave ^ 1) * T::kSlotBytes) + lane;
      static_for<4>([&](auto I) {
        constexpr int i = I;
        const f64x2 v = rp[64 * i];
        rv[k][2 * i] = v.x;
        rv[k][2 * i + 1] = v.y;
      });
    });
    static_for<WB>([&](auto KK) {
      constexpr int k = KK;
      double x0[8], x1[8];
      static_for<8>([&](auto V) {
        x0[V] = half ? rv[k][V] : kp[k][V];
        x1[V] = half ? kp[k][V] : rv[k][V];
      });
      butterfly(std::integral_constant<int, gl>{}, KK, x0, x1, st[2 * k], st[2 * k + 1]);
    });
  }

  if constexpr (LO) pair_group(std::integral_constant<int, (LI ? 1 : 0) + K>{});

  // ---- outputs at depth K
  if (!active) return;
  static_for<HS>([&](auto J) {
    constexpr int j = J;
    const int64_t q = qh + j;
    const int64_t slot = a.mode_si ? base + (lo << K) + q : base + (q << a.log_slo) + lo;
    if constexpr (LO) {
      if (col_ok) {
        f64x2 *u = static_cast<f64x2 *>(a.out);
        static_for<4>([&](auto RHO) {
          constexpr int rho = RHO;
          const f64x2 v = {st[j][rho], st[j][4 + rho]};
          __builtin_nontemporal_store(v, &u[(slot * kRank + 4 * rho + e) * a.ld + col]);
        });
      }
    } else {
      f64x2 *p = static_cast<f64x2 *>(a.out) + ((chunk * a.nslots + slot) * kRank + e) * 16 + n;
      static_for<4>([&](auto RHO) {
        constexpr int rho = RHO;
        const f64x2 v = {st[j][rho], st[j][4 + rho]};
        __builtin_nontemporal_store(v, p + rho * 64);
      });
    }
  });
}

template <int K, bool LI, bool LO, int CW>
void launch_f64_cw(FusedArgs a, hipStream_t s) {
  constexpr int PARTS = LO ? BF_F64_PARTS_LO : BF_F64_PARTS;
  constexpr int NBUF = PARTS == 2 ? 4 : CW >= 4 ? BF_F64_STAGE_BUFFERS : 2;
  using T = F64Traits<K, CW, NBUF, PARTS>;
  a.ngroups = (int)((a.nchunks + CW - 1) / CW);
  hipLaunchKernelGGL((k_fused_pass_f64<K, LI, LO, CW, NBUF, PARTS>), dim3((unsigned)(a.ntiles * a.ngroups)),
                     dim3((unsigned)(T::kWaves * 64)), 0, s, a);
}

// chunks per workgroup: the most that the column count fills
#define BF_F64_LAUNCH(KK, LI, LO)                                                     \
  do {                                                                                \
    if (BF_F64_MAX_CHUNKS >= 4 && a.nchunks >= 4)                                     \
      launch_f64_cw<KK, LI, LO, (BF_F64_MAX_CHUNKS >= 4 ? 4 : 1)>(a, s);              \
    else if (a.nchunks >= 2)                                                          \
      launch_f64_cw<KK, LI, LO, 2>(a, s);                                             \
    else                                                                              \
      launch_f64_cw<KK, LI, LO, 1>(a, s);                                             \
  } while (0)

#define BF_F64_CASES(KK)                 \
  case KK * 4 + 0:                       \
    BF_F64_LAUNCH(KK, false, false);     \
    break;                               \
  case KK * 4 + 2:                       \
    BF_F64_LAUNCH(KK, true, false);      \
    break;                               \
  case KK * 4 + 1:                       \
    BF_F64_LAUNCH(KK, false, true);      \
    break;

hipError_t launch_f64(FusedArgs a, int K, bool li, bool lo, hipStream_t s) {
  if (a.nchunks < 1) return hipErrorInvalidValue;
  switch (K * 4 + (li ? 2 : 0) + (lo ? 1 : 0)) {
    BF_F64_CASES(1)
    BF_F64_CASES(2)
    BF_F64_CASES(3)
    BF_F64_CASES(4)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fused
}  // namespace bfly
