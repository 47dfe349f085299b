// One butterfly level as an FP32 matrix-core product (per-level path, any radix R
// and rank r with R r = 32, 64 or 128 and r even).
//
// Butterfly b of a level combines R input slots into R output slots through one
// (R r) x (R r) complex block M (Sec. 3.2.1 and 3.2.2: the blocks of G^l, and of
// the conjugate transposes of H^l):
//   direct  M[co r + a][ci r + k] = Fb[R hi + co][lo][a][ci r + k]
//   tconj   M[co r + a][ci r + k] = conj(Fb[R hi + ci][lo][k][co r + a])
// with b = hi blo + lo.  The product is the real contraction
//   Re y = [Re M, -Im M] [Re x; Im x],  Im y = [Re M, -Im M] [Im x; -Re x]
// on v_mfma_f32_32x32x2_f32.  One workgroup per butterfly, R r / 32 wavefronts;
// wavefront w computes output rows 32 w .. 32 w + 31 and keeps its rows of the
// real block ([Re M, -Im M], 2 R r values per row) in registers; the workgroup
// walks the 32-column activation chunks, copying each chunk's R r x 32 complex
// inputs into LDS in their activation layout with global -> LDS loads, one chunk
// ahead of the one being contracted.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "bf_internal.h"

namespace bfly {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// A operand of step s (K indices 2 s, 2 s + 1) for lane (i, kk): real block row
// 32 w + i, K index 2 s + kk; stored as [b][w][s / 4][lane][s % 4].
__global__ void k_pack_level_mfma(const float2 *__restrict__ Fb, float *__restrict__ out, int64_t nb,
                                  int64_t blo, int R, int r, int tconj) {
  const int BR = R * r;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nb * (int64_t)BR * 2 * BR) return;
  const int sl = (int)(t & 3);
  const int lane = (int)((t >> 2) & 63);
  const int64_t q = t >> 8;             // (b, w, s / 4)
  const int s4 = (int)(q % (BR / 4));   // s / 4
  const int64_t bw = q / (BR / 4);      // b * (BR / 32) + w
  const int w = (int)(bw % (BR / 32));
  const int64_t b = bw / (BR / 32);
  const int s = 4 * s4 + sl;
  const int o = 32 * w + (lane & 31);
  const int k2 = 2 * s + (lane >> 5);   // 0 .. 2 BR - 1
  const int part = k2 >= BR ? 1 : 0, kin = k2 - part * BR;
  const int64_t hi = b / blo, lo = b - hi * blo;
  const int co = o / r, a = o - co * r, ci = kin / r, k = kin - ci * r;
  float2 m;
  if (tconj) {
    m = Fb[(((R * hi + ci) * blo + lo) * r + k) * BR + co * r + a];
    m.y = -m.y;
  } else {
    m = Fb[(((R * hi + co) * blo + lo) * r + a) * BR + ci * r + k];
  }
  out[t] = part == 0 ? m.x : -m.y;
}

template <int BR>
__global__ __launch_bounds__(BR * 2) void k_level_mfma(const f32x4 *__restrict__ Ap,
                                                        const f32x4 *__restrict__ x,
                                                        f32x4 *__restrict__ y, int64_t blo,
                                                        int64_t nslots, int64_t nchunks, int R,
                                                        int r, int strided_in) {
  constexpr int W = BR / 32;
  constexpr int kChunkBytes = BR * 32 * 8;  // R slots x r rows x 32 columns, complex64
  // two chunk buffers in the activation layout: [slot c][row pair p][column n] x 16 B
  // (rows 2p and 2p + 1 of column n, real and imaginary parts)
  __shared__ __attribute__((aligned(16))) char xs[2][kChunkBytes];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t b = blockIdx.x;
  const int64_t hi = b / blo, lo = b - hi * blo;
  const int half = r / 2;  // row pairs per slot
  auto slot = [&](int c, bool strided) {
    return strided ? hi * R * blo + c * blo + lo : hi * R * blo + R * lo + c;
  };
  // one chunk: R slots of half * 32 pieces, contiguous in global memory per slot
  auto issue = [&](int64_t ch) {
    char *dst = xs[ch & 1];
    for (int pc = threadIdx.x; pc < BR * 16; pc += BR * 2) {
      const int c = pc / (half * 32), rem = pc - c * half * 32;
      const f32x4 *src = x + (ch * nslots + slot(c, strided_in != 0)) * half * 32 + rem;
      __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)(dst + pc * 16),
                                       16, 0, 0);
    }
  };
  issue(0);
  // this wavefront's rows of the real block: a[s] = A[32 w + i][2 s + kk]
  float a[BR];
  {
    const f32x4 *src = Ap + (b * W + w) * (BR / 4) * 64 + lane;
#pragma unroll
    for (int s4 = 0; s4 < BR / 4; ++s4) {
      const f32x4 v = src[s4 * 64];
      a[4 * s4] = v.x;
      a[4 * s4 + 1] = v.y;
      a[4 * s4 + 2] = v.z;
      a[4 * s4 + 3] = v.w;
    }
  }
  const int j = lane & 31, kk = lane >> 5;
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    // this chunk's copies (and the block rows) have landed; the previous chunk's eight
    // output stores per lane, issued after them, may still be in flight
    if (ch == 0)
      __builtin_amdgcn_s_waitcnt(0);
    else
      __builtin_amdgcn_s_waitcnt(0xf78);  // vmcnt(8)
    // everyone's copies have; the other buffer is free (a bare barrier: __syncthreads
    // would also wait for the output stores still in flight)
    __builtin_amdgcn_s_barrier();
    if (ch + 1 < nchunks) issue(ch + 1);
    const float *xc = reinterpret_cast<const float *>(xs[ch & 1]);
    floatx16 dre = {}, dim = {};
#pragma unroll
    for (int s = 0; s < BR; ++s) {
      // K index k = 2 s + kk of [Re x; Im x] (and of [Im x; -Re x]): input row
      // 2 sp + kk with sp = s or s - BR / 2, i.e. row pair sp across the slots,
      // which the buffer stores at (sp * 32 + j) * 16 bytes
      const bool lo_half = 2 * s < BR;
      const int sp = lo_half ? s : s - BR / 2;
      const float *e = xc + (sp * 32 + j) * 4 + kk * 2;
      const float xr = e[0], xi = e[1];
      const float bre = lo_half ? xr : xi;
      const float bim = lo_half ? xi : -xr;
      dre = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], bre, dre, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], bim, dim, 0, 0, 0);
    }
    // lane (j, eta) holds rows 32 w + 8 q + 4 eta + v of column j
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int v = 0; v < 4; v += 2) {
        const int o = 32 * w + 8 * q + 4 * kk + v;
        const int co = o / r, row = o - co * r;
        const f32x4 val = {dre[4 * q + v], dim[4 * q + v], dre[4 * q + v + 1], dim[4 * q + v + 1]};
        y[((ch * nslots + slot(co, strided_in == 0)) * half + row / 2) * 32 + j] = val;
      }
  }
}

// As k_level_mfma, with the K range of the real block split over two wavefronts per
// row group (2 BR / 32 wavefronts): wavefront (w, kh) keeps steps kh BR/2 .. kh BR/2 +
// BR/2 - 1 of rows 32 w .. 32 w + 31, so it holds half the block rows and the register
// count allows two workgroups per CU (one workgroup's block load overlaps the other's
// products).  After each chunk the K-high wavefronts hand their partial sums to the
// K-low ones through the chunk buffer just consumed, which then store the outputs.
// Workgroup barrier without a memory fence (which would also wait for global stores and
// copies in flight); the empty asm statements keep the compiler from moving LDS
// accesses across it, since the barrier instruction itself does not order memory for
// the compiler.
__device__ __forceinline__ void wg_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int BR, int R>
__global__ __launch_bounds__(BR * 4) __attribute__((amdgpu_waves_per_eu(4))) void k_level_mfma_ks(
    const f32x4 *__restrict__ Ap, const f32x4 *__restrict__ x, f32x4 *__restrict__ y, int64_t blo,
    int64_t nslots, int64_t nchunks, int strided_in) {
  constexpr int r = BR / R;
  constexpr int W = BR / 32;
  constexpr int HS = BR / 2;                 // steps per K half
  constexpr int kChunkBytes = BR * 32 * 8;   // R slots x r rows x 32 columns, complex64
  static_assert(W * 64 * 32 * 4 <= kChunkBytes, "partial sums must fit in one chunk buffer");
  __shared__ __attribute__((aligned(16))) char xs[2][kChunkBytes];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int w = wv % W, kh = wv / W;
  const int64_t b = blockIdx.x;
  const int64_t hi = b / blo, lo = b - hi * blo;
  constexpr int half = r / 2;
  auto slot = [&](int c, bool strided) {
    return strided ? hi * R * blo + c * blo + lo : hi * R * blo + R * lo + c;
  };
  static_assert(r % 32 == 0, "a 32-row group of outputs must lie in one slot");
  // input slot c of this butterfly is s_in0 + c * dc_in (both uniform)
  const int64_t s_in0 = slot(0, strided_in != 0), dc_in = strided_in ? blo : 1;
  const int64_t s_out0 = slot(0, strided_in == 0), dc_out = strided_in ? 1 : blo;
  auto issue = [&](int64_t ch) {
    char *dst = xs[ch & 1];
    const f32x4 *xb = x + (ch * nslots + s_in0) * (half * 32);
#pragma unroll
    for (int k = 0; k < (BR * 16) / (BR * 4); ++k) {
      constexpr int kPerSlot = (half * 32) / (BR * 4);  // pieces of one slot per thread
      const int c = k / kPerSlot, part = k % kPerSlot;
      const f32x4 *src = xb + c * dc_in * (half * 32) + part * (BR * 4) + threadIdx.x;
      __builtin_amdgcn_global_load_lds(src,
                                       (__attribute__((address_space(3))) void *)(dst + (k * BR * 4 + threadIdx.x) * 16),
                                       16, 0, 0);
    }
  };
  issue(0);
  float a[HS];
  {
    const f32x4 *src = Ap + (b * W + w) * (BR / 4) * 64 + kh * (HS / 4) * 64 + lane;
#pragma unroll
    for (int s4 = 0; s4 < HS / 4; ++s4) {
      const f32x4 v = src[s4 * 64];
      a[4 * s4] = v.x;
      a[4 * s4 + 1] = v.y;
      a[4 * s4 + 2] = v.z;
      a[4 * s4 + 3] = v.w;
    }
  }
  const int j = lane & 31, kk = lane >> 5;
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    // this chunk's copies have landed: the K-low wavefronts may still have their eight
    // output stores of the previous chunk in flight, issued after the copies; the
    // K-high wavefronts store nothing
    if (ch == 0 || kh == 1)
      __builtin_amdgcn_s_waitcnt(0);
    else
      __builtin_amdgcn_s_waitcnt(0xf78);  // vmcnt(8)
    wg_barrier();
    if (ch + 1 < nchunks) issue(ch + 1);
    const float *xc = reinterpret_cast<const float *>(xs[ch & 1]);
    floatx16 dre = {}, dim = {};
#pragma unroll
    for (int s2 = 0; s2 < HS; ++s2) {
      // step s = kh HS + s2: the K-low half reads [Re x; Im x] rows, the K-high half
      // [Im x; -Re x], both at row pair s2 of the buffer
      const float *e = xc + (s2 * 32 + j) * 4 + kk * 2;
      const float xr = e[0], xi = e[1];
      const float bre = kh == 0 ? xr : xi;
      const float bim = kh == 0 ? xi : -xr;
      dre = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s2], bre, dre, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s2], bim, dim, 0, 0, 0);
      // keep the scheduler from hoisting every step's buffer reads (registers)
      if (s2 % 8 == 7) __builtin_amdgcn_sched_barrier(0);
    }
    // every wavefront is done reading this buffer; the K-high ones put their partial
    // sums there, the K-low ones add them
    wg_barrier();
    float *red = reinterpret_cast<float *>(xs[ch & 1]) + (w * 64 + lane) * 32;
    if (kh == 1) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        red[i] = dre[i];
        red[16 + i] = dim[i];
      }
    }
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    wg_barrier();
    if (kh == 0) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        dre[i] += red[i];
        dim[i] += red[16 + i];
        // a few partial sums in flight at a time (registers)
        if (i % 4 == 3) __builtin_amdgcn_sched_barrier(0);
      }
      // lane (j, eta) holds rows 32 w + 8 q + 4 eta + v of column j: output slot co =
      // 32 w / r, rows row0 + 8 q + 4 eta + v with row0 = 32 w - co r
      const int co = (32 * w) / r, row0 = 32 * w - co * r;
      f32x4 *yb = y + ((ch * nslots + s_out0 + co * dc_out) * half + row0 / 2 + 2 * kk) * 32 + j;
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; v += 2) {
          const f32x4 val = {dre[4 * q + v], dim[4 * q + v], dre[4 * q + v + 1], dim[4 * q + v + 1]};
          yb[(4 * q + v / 2) * 32] = val;
        }
    }
  }
}

}  // namespace

bool level_mfma_supported(int R, int r) {
  const int BR = R * r;
  return (BR == 32 || BR == 64 || BR == 128) && r % 2 == 0;
}

hipError_t launch_pack_level_mfma(const LevelOp &op, int R, int r, void *out, hipStream_t s) {
  const int BR = R * r;
  const int64_t total = op.nb * (int64_t)BR * 2 * BR;
  const int bs = 256;
  hipLaunchKernelGGL(k_pack_level_mfma, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, s,
                     (const float2 *)op.mat, (float *)out, op.nb, op.blo, R, r, op.tconj ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_level_mfma(const bf_plan *p, const LevelOp &op, const void *in, void *out,
                             int64_t nrhs, hipStream_t s) {
  const int BR = p->R * p->r;
  const int64_t nchunks = (nrhs + 31) / 32;
  const int strided = op.mode == kStridedIn ? 1 : 0;
  const f32x4 *A = static_cast<const f32x4 *>(op.packed);
  const f32x4 *x = static_cast<const f32x4 *>(in);
  f32x4 *y = static_cast<f32x4 *>(out);
  if (BR == 32)
    hipLaunchKernelGGL(k_level_mfma<32>, dim3((unsigned)op.nb), dim3(64), 0, s, A, x, y, op.blo, p->P,
                       nchunks, p->R, p->r, strided);
  else if (BR == 64)
    hipLaunchKernelGGL(k_level_mfma<64>, dim3((unsigned)op.nb), dim3(128), 0, s, A, x, y, op.blo, p->P,
                       nchunks, p->R, p->r, strided);
  else if (p->opt.level_ksplit < 0)
    hipLaunchKernelGGL(k_level_mfma<128>, dim3((unsigned)op.nb), dim3(256), 0, s, A, x, y, op.blo, p->P,
                       nchunks, p->R, p->r, strided);
  else if (p->R == 4)
    hipLaunchKernelGGL((k_level_mfma_ks<128, 4>), dim3((unsigned)op.nb), dim3(512), 0, s, A, x, y, op.blo,
                       p->P, nchunks, strided);
  else
    hipLaunchKernelGGL((k_level_mfma_ks<128, 2>), dim3((unsigned)op.nb), dim3(512), 0, s, A, x, y, op.blo,
                       p->P, nchunks, strided);
  return hipGetLastError();
}

}  // namespace bfly
