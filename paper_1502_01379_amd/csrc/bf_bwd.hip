// Backward-pass kernels for handles on the fused path (radix 2, leaf 16, r 16).
//
//  * k_pack_pass / k_pack_leaf16: pack the blocks of a K-level FP32 fused pass
//    (butterfly blocks and leaf pairs) from the canonical factors on the device,
//    in the per-lane A-operand order of the 16-column block products, so the
//    backward pass runs the same fused passes as the apply in FP32.
//  * k_grad_leaf: the gradient of the leaf blocks (two leaves per wavefront).
//  * k_grad_middle: the gradient of the middle weights (one wavefront per slot).
//  * k_grad_level: the gradient of every block of one level,
//        grad[2 hi + cx][lo][rx][cy r + ry] = sum_n X[strided(b,cx)][rx][n] conj(Y[contig(b,cy)][ry][n]),
//    (grad_B = sum_n d_out x_in^* for G levels with X = d_out, Y = x_in;
//     grad_W = sum_n x_in d_out^* for H levels with X = x_in, Y = d_out),
//    as three 32 x 32 x nrhs real contractions on the matrix cores (Gauss's
//    three-product form of the complex sum).  One
//    wavefront per butterfly, columns in chunks of 16 staged through LDS
//    (transposed, padded rows: conflict-free reads), fixed summation order.
#include <hip/hip_runtime.h>

#include "bf_internal.h"

namespace bfly {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int kR = 16;  // rank == leaf size on this path

// value = [Re M, -Im M][o][(part, k)] for the block of butterfly b, with
//   direct: M[o][k] = Fb[2 hi + o / r][lo][o % r][k]
//   tconj:  M[o][k] = conj(Fb[2 hi + k / r][lo][k % r][o])
__device__ __forceinline__ float block_value(const float2 *__restrict__ Fb, int64_t hi, int64_t lo,
                                             int64_t blo, int tconj, int o, int k, int part) {
  float2 v;
  if (tconj)
    v = Fb[(((2 * hi + k / kR) * blo + lo) * kR + (k % kR)) * (2 * kR) + o];
  else
    v = Fb[(((2 * hi + o / kR) * blo + lo) * kR + (o % kR)) * (2 * kR) + k];
  if (tconj) v.y = -v.y;
  return part == 0 ? v.x : -v.y;
}

// Blocks of a K-level FP32 pass, [depth d][tile][beta], from the canonical
// factors: the butterfly at depth d takes tile-local slots qi0, qi0 + 2^d, whose
// place in the level-by-level slot order is fixed by the pass's slot mode (the
// same map the pass uses for its per-depth copies); the level's butterfly index
// follows from the slot pattern of that level (strided or contiguous input).
// RNE split of an FP32 value into BF16 hi + lo, as bit patterns
__device__ __forceinline__ void split_bf16(float v, uint16_t &hi, uint16_t &lo) {
  const __bf16 h = (__bf16)v;
  const __bf16 l = (__bf16)(v - (float)h);
  hi = __builtin_bit_cast(uint16_t, h);
  lo = __builtin_bit_cast(uint16_t, l);
}

// split = 0: FP32 layout, value 16 T + s of lane (i, e) at float (s / 4 ... ) as the
// 16-column FP32 product reads it; split = 1: BF16 hi / lo layout of the split
// product (piece w = 2 T + part holds this lane's 8 values j: input row 16 (j / 4)
// + 4 e + j % 4; hi in pieces 0 .. 3, lo in pieces 4 .. 7)
__global__ void k_pack_pass(PackPassArgs a, float *__restrict__ out, int split) {
  const int64_t NB = int64_t(1) << (a.K - 1);
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)a.K * a.ntiles * NB * 2048) return;
  const int f = (int)(t & 31);
  const int lane = (int)((t >> 5) & 63);
  const int64_t bi = t >> 11;
  const int d = (int)(bi / (a.ntiles * NB));
  const int64_t rem = bi - d * a.ntiles * NB;
  const int64_t tile = rem / NB;
  const int beta = (int)(rem - tile * NB);
  const int ap = beta >> d, bb = beta & ((1 << d) - 1);
  const int64_t q = ((int64_t)(2 * ap) << d) + bb;
  const int64_t lo = tile & ((int64_t(1) << a.log_slo) - 1);
  const int64_t base = (tile >> a.log_slo) << (a.K + a.log_slo);
  const int64_t dm = (int64_t(1) << d) - 1;
  const int64_t slot = a.mode_si ? base + ((q >> d) << (d + a.log_slo)) + (lo << d) + (q & dm)
                                 : base + ((q & dm) << (a.K - d + a.log_slo)) + (lo << (a.K - d)) + (q >> d);
  const PackDepth &pd = a.dep[d];
  const int64_t blo = int64_t(1) << pd.log_blo;
  const int64_t b = pd.contig ? (slot >> 1) : (((slot >> (pd.log_blo + 1)) << pd.log_blo) | (slot & (blo - 1)));
  const int i = lane & 15, e = lane >> 4;
  if (split) {
    const int w = f >> 3, j = f & 7;
    const int T = w >> 1, part = w & 1;
    const float v = block_value(static_cast<const float2 *>(pd.Fb), b / blo, b % blo, blo, pd.tconj,
                                16 * T + i, 16 * (j >> 2) + 4 * e + (j & 3), part);
    uint16_t hi, lo16;
    split_bf16(v, hi, lo16);
    uint16_t *o16 = reinterpret_cast<uint16_t *>(out) + bi * 4096;
    o16[(w * 64 + lane) * 8 + j] = hi;
    o16[((4 + w) * 64 + lane) * 8 + j] = lo16;
    return;
  }
  // FP32: Re M and +Im M, for Gauss's three products (block16_f32)
  const int T = f >> 4, sidx = f & 15;
  const int part = sidx >> 3, cp = (sidx >> 2) & 1, rho = sidx & 3;
  const float v = block_value(static_cast<const float2 *>(pd.Fb), b / blo, b % blo, blo, pd.tconj,
                              16 * T + i, 16 * cp + 4 * e + rho, part);
  out[bi * 2048 + ((f >> 2) * 64 + lane) * 4 + (f & 3)] = part ? -v : v;
}

// Leaf pairs of a pass (tile, q: leaves (tile << K) + 2q + c) as two 16 x 16 FP32
// blocks: in  M_c[a][p] = conj(W[j][p][a]),  out  M_c[p][a] = W[j][p][a];
// value j of lane i + 16 e is [Re M_c, -Im M_c][i][(j / 4, 4 e + j % 4)].
__global__ void k_pack_leaf16(const float2 *__restrict__ W, float *__restrict__ out, int64_t npairs,
                              int K, int in, int split) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= npairs * 1024) return;
  const int64_t bi = t >> 10;
  const int w = (int)(t & 1023);
  // FP32: 2 pieces of 4 floats per slot; split: this thread makes value jv's hi and lo
  const int c = w >> 9;
  const int lane = split ? (w >> 3) & 63 : (w >> 2) & 63;
  const int pc = split ? 0 : (w >> 8) & 1, jj = split ? 0 : w & 3;
  const int jv = split ? (w & 7) : pc * 4 + jj;  // value index 0..7
  const int i = lane & 15, e = lane >> 4;
  const int k = 4 * e + (jv & 3);
  const int64_t tile = bi >> (K - 1), qq = bi & ((int64_t(1) << (K - 1)) - 1);
  const int64_t leaf = (tile << K) + 2 * qq + c;
  float2 m = in ? W[(leaf * kR + k) * kR + i] : W[(leaf * kR + i) * kR + k];
  if (in) m.y = -m.y;
  const float v = (jv >> 2) == 0 ? m.x : -m.y;
  if (split) {
    uint16_t hi, lo;
    split_bf16(v, hi, lo);
    uint16_t *o16 = reinterpret_cast<uint16_t *>(out) + bi * 2048;
    o16[((c * 2 + 0) * 64 + lane) * 8 + jv] = hi;
    o16[((c * 2 + 1) * 64 + lane) * 8 + jv] = lo;
    return;
  }
  out[bi * 1024 + ((c * 2 + pc) * 64 + lane) * 4 + jj] = pc ? -v : v;  // FP32: +Im (Gauss)
}

constexpr int kRowPad = 272;  // bytes per column of a staged 32-row chunk (256 + 16)

// Rows (2 slots x 16 rows) x 16 columns [n0, n0 + 16) of one activation operand:
// this lane's four 16-byte pieces (two complex values of one column each) are
// loaded into registers, then written to LDS as [column][row] complex with row
// stride kRowPad bytes.
struct Chunk {
  f32x4 v[4];
};
__device__ __forceinline__ void load_chunk(const float2 *__restrict__ act, int64_t nslots,
                                           int64_t s0, int64_t s1, int64_t n0, int cs, int lane,
                                           Chunk &ch) {
  const int C = 1 << cs;
  const int64_t chunk = n0 >> cs;
  const int nb = (int)(n0 & (C - 1));
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int piece = v * 64 + lane;          // 256 pieces of 16 bytes (2 complex)
    const int c = piece >> 7;                 // slot 0 or 1
    const int p = (piece >> 4) & 7;           // row pair
    const int n = piece & 15;                 // column within the 16
    const int64_t slot = c ? s1 : s0;
    ch.v[v] = *reinterpret_cast<const f32x4 *>(act + ((chunk * nslots + slot) * 8 + p) * (2 * C) +
                                               (int64_t)(nb + n) * 2);
  }
}
__device__ __forceinline__ void store_chunk(const Chunk &ch, char *lds, int lane) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int piece = v * 64 + lane;
    const int c = piece >> 7, p = (piece >> 4) & 7, n = piece & 15;
    *reinterpret_cast<f32x4 *>(lds + n * kRowPad + (c * 16 + 2 * p) * 8) = ch.v[v];
  }
}
__device__ __forceinline__ void stage_chunk(const float2 *__restrict__ act, int64_t nslots,
                                            int64_t s0, int64_t s1, int64_t n0, int cs,
                                            char *lds, int lane) {
  Chunk ch;
  load_chunk(act, nslots, s0, s1, n0, cs, lane, ch);
  store_chunk(ch, lds, lane);
}

// Stage rows (2 leaves x 16 points) x 16 columns [n0, n0 + 16) of a user vector
// [N][ld] into LDS as [column][row] complex, row stride kRowPad bytes; columns
// at or past nrhs are zero.
__device__ __forceinline__ void stage_user(const float2 *__restrict__ u, int64_t ld, int64_t row0,
                                           int64_t n0, int64_t nrhs, char *lds, int lane) {
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int piece = v * 64 + lane;  // 512 complex: row = piece / 16, column = piece % 16
    const int row = piece >> 4, n = piece & 15;
    float2 val = make_float2(0.f, 0.f);
    if (n0 + n < nrhs) val = u[(row0 + row) * ld + n0 + n];
    *reinterpret_cast<float2 *>(lds + n * kRowPad + row * 8) = val;
  }
}

// Gradient of two leaf blocks (leaves 2 pr, 2 pr + 1):
//   grad[j][p][a] = sum_n U[(j n0 + p) ld + n] conj(act[j][a][n])
// (grad U^L with U = delta_u, act = z^L; grad V^L with U = g, act = delta y^L).
__global__ __launch_bounds__(256) void k_grad_leaf(const float2 *__restrict__ U, int64_t ld,
                                                    const float2 *__restrict__ act,
                                                    float2 *__restrict__ grad, int64_t npairs,
                                                    int64_t nslots, int64_t nrhs, int cs) {
  __shared__ __attribute__((aligned(16))) char lds[4][2][16 * kRowPad];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t pr = (int64_t)blockIdx.x * 4 + wave;
  if (pr >= npairs) return;
  char *lx = lds[wave][0], *ly = lds[wave][1];
  const int i = lane & 31, eta = lane >> 5;
  floatx16 t1 = {}, t2 = {}, t3 = {};
  const int64_t npad = ((nrhs + 15) >> 4) << 4;
  for (int64_t n0 = 0; n0 < npad; n0 += 16) {
    stage_user(U, ld, 2 * pr * kR, n0, nrhs, lx, lane);
    stage_chunk(act, nslots, 2 * pr, 2 * pr + 1, n0, cs, ly, lane);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int n = 8 * eta + s;
      const f32x2 xv = *reinterpret_cast<const f32x2 *>(lx + n * kRowPad + i * 8);
      const f32x2 yv = *reinterpret_cast<const f32x2 *>(ly + n * kRowPad + i * 8);
      // x conj(y) by Gauss's three products, as in k_grad_level
      t1 = __builtin_amdgcn_mfma_f32_32x32x2f32(xv.x, yv.x, t1, 0, 0, 0);
      t2 = __builtin_amdgcn_mfma_f32_32x32x2f32(xv.y, yv.y, t2, 0, 0, 0);
      t3 = __builtin_amdgcn_mfma_f32_32x32x2f32(xv.x + xv.y, yv.x - yv.y, t3, 0, 0, 0);
    }
    __builtin_amdgcn_wave_barrier();
  }
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int row = 8 * (reg >> 2) + 4 * eta + (reg & 3);
    const int c = row >> 4;
    if ((i >> 4) != c) continue;  // only the two diagonal 16 x 16 blocks
    float2 v;
    v.x = t1[reg] + t2[reg];
    v.y = t3[reg] - t1[reg] + t2[reg];
    grad[((2 * pr + c) * kR + (row & 15)) * kR + (i & 15)] = v;
  }
}

__global__ __launch_bounds__(256) void k_grad_level(const float2 *__restrict__ X,
                                                     const float2 *__restrict__ Y,
                                                     float2 *__restrict__ grad, int64_t nb,
                                                     int64_t blo, int64_t nslots, int64_t nrhs,
                                                     int cs) {
  __shared__ __attribute__((aligned(16))) char lds[4][2][16 * kRowPad];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * 4 + wave;
  if (b >= nb) return;
  const int64_t hi = b / blo, lo = b - hi * blo;
  const int64_t sx0 = hi * 2 * blo + lo, sx1 = sx0 + blo;        // strided slots
  const int64_t sy0 = hi * 2 * blo + 2 * lo, sy1 = sy0 + 1;      // contiguous slots
  char *lx = lds[wave][0], *ly = lds[wave][1];
  const int i = lane & 31, eta = lane >> 5;
  floatx16 t1 = {}, t2 = {}, t3 = {};
  const int64_t npad = ((nrhs + 15) >> 4) << 4;
  // the next chunk's loads are in flight while the current one is contracted
  Chunk cx, cy;
  load_chunk(X, nslots, sx0, sx1, 0, cs, lane, cx);
  load_chunk(Y, nslots, sy0, sy1, 0, cs, lane, cy);
  for (int64_t n0 = 0; n0 < npad; n0 += 16) {
    store_chunk(cx, lx, lane);
    store_chunk(cy, ly, lane);
    if (n0 + 16 < npad) {
      load_chunk(X, nslots, sx0, sx1, n0 + 16, cs, lane, cx);
      load_chunk(Y, nslots, sy0, sy1, n0 + 16, cs, lane, cy);
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wavefront's LDS writes are done
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int n = 8 * eta + s;
      const f32x2 xv = *reinterpret_cast<const f32x2 *>(lx + n * kRowPad + i * 8);
      const f32x2 yv = *reinterpret_cast<const f32x2 *>(ly + n * kRowPad + i * 8);
      // columns past nrhs hold zeros in every activation buffer; x conj(y) by Gauss's
      // three products: t1 = Re x Re y, t2 = Im x Im y, t3 = (Re x + Im x)(Re y - Im y),
      // Re = t1 + t2, Im = t3 - t1 + t2
      t1 = __builtin_amdgcn_mfma_f32_32x32x2f32(xv.x, yv.x, t1, 0, 0, 0);
      t2 = __builtin_amdgcn_mfma_f32_32x32x2f32(xv.y, yv.y, t2, 0, 0, 0);
      t3 = __builtin_amdgcn_mfma_f32_32x32x2f32(xv.x + xv.y, yv.x - yv.y, t3, 0, 0, 0);
    }
    __builtin_amdgcn_wave_barrier();
  }
  // lane (j, eta) holds D[8 q + 4 eta + v][j]: row (cx, rx), column j = cy r + ry
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int row = 8 * (reg >> 2) + 4 * eta + (reg & 3);
    const int cx = row >> 4, rx = row & 15;
    float2 v;
    v.x = t1[reg] + t2[reg];
    v.y = t3[reg] - t1[reg] + t2[reg];
    grad[(((2 * hi + cx) * blo + lo) * kR + rx) * (2 * kR) + i] = v;
  }
}

// grad_S[i][j][k] = Re sum_n dz[(i m + j)][k][n] conj(y[(j m + i)][k][n]) (the
// middle weights scale slot i m + j by S[i][j] after the block transpose).  One
// wavefront per slot s = i m + j: per 16-column chunk the two slots are 2 KB
// each, read as 128 pieces of (rows 2p, 2p + 1; column n); lane l takes pieces
// l and l + 64 (pairs p = l / 16 and 4 + l / 16), and the 16 columns are summed
// across lanes at the end.
__global__ __launch_bounds__(256) void k_grad_middle(const f32x4 *__restrict__ dz,
                                                      const f32x4 *__restrict__ y,
                                                      float *__restrict__ grad, int64_t nslots,
                                                      int64_t nchunks, int log_m) {
  const int lane = threadIdx.x & 63;
  const int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= nslots) return;
  const int64_t m = int64_t(1) << log_m;
  const int64_t tr = ((s & (m - 1)) << log_m) | (s >> log_m);
  float acc[4] = {0.f, 0.f, 0.f, 0.f};  // rows 2p, 2p + 1 for p = lane / 16 and 4 + lane / 16
  for (int64_t c = 0; c < nchunks; ++c) {
    const f32x4 *a = dz + (c * nslots + s) * 128 + lane;
    const f32x4 *b = y + (c * nslots + tr) * 128 + lane;
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const f32x4 x = a[v * 64], w = b[v * 64];
      acc[2 * v] += x.x * w.x + x.y * w.y;
      acc[2 * v + 1] += x.z * w.z + x.w * w.w;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) acc[q] += __shfl_xor(acc[q], off);
  if ((lane & 15) == 0) {
    const int p = lane >> 4;
    float *g = grad + s * kR;
    g[2 * p] = acc[0];
    g[2 * p + 1] = acc[1];
    g[8 + 2 * p] = acc[2];
    g[8 + 2 * p + 1] = acc[3];
  }
}

}  // namespace

hipError_t launch_grad_middle(const bf_plan *p, const void *dz, const void *y, void *grad,
                              int64_t nrhs, hipStream_t s) {
  int log_m = 0;
  while ((int64_t(1) << log_m) < p->m) ++log_m;
  const int64_t nchunks = (nrhs + 15) / 16;
  hipLaunchKernelGGL(k_grad_middle, dim3((unsigned)((p->P + 3) / 4)), dim3(256), 0, s,
                     (const f32x4 *)dz, (const f32x4 *)y, (float *)grad, p->P, nchunks, log_m);
  return hipGetLastError();
}

hipError_t launch_grad_leaf_mfma(const bf_plan *p, const void *user, int64_t ld, const void *act,
                                 void *grad, int64_t nrhs, hipStream_t s) {
  const int64_t npairs = p->P / 2;
  hipLaunchKernelGGL(k_grad_leaf, dim3((unsigned)((npairs + 3) / 4)), dim3(256), 0, s,
                     (const float2 *)user, ld, (const float2 *)act, (float2 *)grad, npairs, p->P,
                     nrhs, p->cs);
  return hipGetLastError();
}

hipError_t launch_pack_pass(const PackPassArgs &a, void *out, bool split, hipStream_t s) {
  const int bs = 256;
  const int64_t total = (int64_t)a.K * a.ntiles * (int64_t(1) << (a.K - 1)) * 2048;
  hipLaunchKernelGGL(k_pack_pass, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, s, a, (float *)out,
                     split ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_pack_leaf16(const void *canon_leaf, void *out, int64_t npairs, int K, bool in,
                              bool split, hipStream_t s) {
  const int bs = 256;
  const int64_t total = npairs * 1024;
  hipLaunchKernelGGL(k_pack_leaf16, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, s,
                     (const float2 *)canon_leaf, (float *)out, npairs, K, in ? 1 : 0, split ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_grad_level_mfma(const bf_plan *p, const LevelOp &op, const void *X, const void *Y,
                                  void *grad, int64_t nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_level, dim3((unsigned)((op.nb + 3) / 4)), dim3(256), 0, s,
                     (const float2 *)X, (const float2 *)Y, (float2 *)grad, op.nb, op.blo, p->P,
                     nrhs, p->cs);
  return hipGetLastError();
}

}  // namespace bfly
