// Per-level kernels: one launch per factor of the product, any radix, rank and
// leaf size, FP64 or FP32.  These run the FP64 path, every shape the fused MFMA
// passes do not cover, and the per-level steps of the backward pass.
//
// Each factor is one of
//   leaf-in     y_j = W_j^* x_{leaf j}       W = V^L_j forward, U^L_j adjoint
//   butterfly   out[c_out r + a] = sum_k M_b[c_out r + a][k] in[k],  k = c_in r + b
//               (the R x R block relation of one butterfly, Sec. 3.2.1 / 3.2.2)
//   middle      y[(a m + b)] = S[a][b] .* x[(b m + a)]    (Sec. 3.1, M^h)
//   leaf-out    u_{leaf i} = W_i z_i          W = U^L_i forward, V^L_i adjoint
// Factors are read in the canonical layout of bf.h, converted to the compute
// precision, without any repacking.
#include <hip/hip_runtime.h>

#include "bf_internal.h"

namespace bfly {
namespace {

template <class T> struct Cx;
template <> struct Cx<float> { using type = float2; };
template <> struct Cx<double> { using type = double2; };

template <class C> __device__ __forceinline__ C cmul(C a, C b) {
  C o;
  o.x = a.x * b.x - a.y * b.y;
  o.y = a.x * b.y + a.y * b.x;
  return o;
}
// a * conj(b)
template <class C> __device__ __forceinline__ C cmulc(C a, C b) {
  C o;
  o.x = a.x * b.x + a.y * b.y;
  o.y = a.y * b.x - a.x * b.y;
  return o;
}

// Row-pair layout shared with the fused passes (see bf_internal.h).
__device__ __forceinline__ int64_t act_off(int64_t slot, int row, int64_t n, int64_t nslots, int r,
                                           int cs) {
  const int rp = (r + 1) >> 1;
  return (((n >> cs) * nslots + slot) * rp + (row >> 1)) * (int64_t(2) << cs) +
         (n & ((1 << cs) - 1)) * 2 + (row & 1);
}

__device__ __forceinline__ int64_t slot_of(int64_t b, int c, int64_t blo, int R, bool strided) {
  const int64_t hi = b / blo, lo = b - hi * blo;
  return strided ? hi * R * blo + c * blo + lo : hi * R * blo + R * lo + c;
}

// y[j][a][n] = sum_p conj(W[j][p][a]) x[(j n0 + p) ld + n] with W the canonical
// [P][n0][r] leaf array (V^L forward, U^L adjoint); padded columns get zeros.
template <class T>
__global__ void k_leaf_in(const typename Cx<T>::type *__restrict__ W,
                          const typename Cx<T>::type *__restrict__ x, int64_t ld,
                          typename Cx<T>::type *__restrict__ y, int64_t P, int n0, int r,
                          int64_t nrhs, int64_t npad, int cs) {
  using C = typename Cx<T>::type;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= P * r * npad) return;
  const int64_t n = t % npad;
  const int a = (int)((t / npad) % r);
  const int64_t j = t / (npad * r);
  C acc{0, 0};
  if (n < nrhs) {
    const C *w = W + j * n0 * r + a;
    for (int p = 0; p < n0; ++p) {
      const C v = x[(j * n0 + p) * ld + n];
      const C c = cmulc(v, w[p * r]);
      acc.x += c.x;
      acc.y += c.y;
    }
  }
  y[act_off(j, a, n, P, r, cs)] = acc;
}

// u[(i n0 + p) ld + n] = sum_a W[i][p][a] z[i][a][n]
template <class T>
__global__ void k_leaf_out(const typename Cx<T>::type *__restrict__ W,
                           const typename Cx<T>::type *__restrict__ z,
                           typename Cx<T>::type *__restrict__ u, int64_t ld, int64_t P, int n0,
                           int r, int64_t nrhs, int cs) {
  using C = typename Cx<T>::type;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= P * n0 * nrhs) return;
  const int64_t n = t % nrhs;
  const int p = (int)((t / nrhs) % n0);
  const int64_t i = t / (nrhs * n0);
  const C *w = W + (i * n0 + p) * r;
  C acc{0, 0};
  for (int a = 0; a < r; ++a) {
    const C c = cmul(w[a], z[act_off(i, a, n, P, r, cs)]);
    acc.x += c.x;
    acc.y += c.y;
  }
  u[(i * n0 + p) * ld + n] = acc;
}

// The same two leaf products with one thread per (leaf, column): the thread
// keeps the leaf's N0 input rows (leaf-in) or RR rank rows (leaf-out) of its
// column in registers and produces every output row, so each input is read once.
template <class T, int N0>
__global__ void k_leaf_in_col(const typename Cx<T>::type *__restrict__ W,
                              const typename Cx<T>::type *__restrict__ x, int64_t ld,
                              typename Cx<T>::type *__restrict__ y, int64_t P, int r, int64_t nrhs,
                              int64_t npad, int cs) {
  using C = typename Cx<T>::type;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= P * npad) return;
  const int64_t n = t % npad, j = t / npad;
  C v[N0];
#pragma unroll
  for (int p = 0; p < N0; ++p) v[p] = n < nrhs ? x[(j * N0 + p) * ld + n] : C{0, 0};
  const C *w = W + j * N0 * r;
  for (int a = 0; a < r; ++a) {
    C acc{0, 0};
#pragma unroll
    for (int p = 0; p < N0; ++p) {
      const C c = cmulc(v[p], w[p * r + a]);
      acc.x += c.x;
      acc.y += c.y;
    }
    y[act_off(j, a, n, P, r, cs)] = acc;
  }
}

// Leaf-in with the leaf index uniform across each wavefront (npad a multiple of 64, so
// the 64 columns of a wavefront share one leaf): the n0 x r leaf block is then read
// with scalar loads (read-only, uniform addresses), in order, instead of once per
// column through the vector memory path.
// The r outputs of a column are split over SPLIT wavefronts (RR / SPLIT accumulators
// per thread), which keeps the register count low enough for several wavefronts per
// SIMD; the column's n0 inputs are read by each of them.
template <class T, int N0, int RR, int SPLIT>
__global__ __launch_bounds__(256) void k_leaf_in_uni(const typename Cx<T>::type *__restrict__ W,
                                                     const typename Cx<T>::type *__restrict__ x,
                                                     int64_t ld, typename Cx<T>::type *__restrict__ y,
                                                     int64_t P, int64_t nrhs, int64_t npad, int cs) {
  using C = typename Cx<T>::type;
  constexpr int RS = RR / SPLIT;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= P * SPLIT * npad) return;
  const int64_t n = t % npad;
  const int q = __builtin_amdgcn_readfirstlane((int)(t / npad));
  const int64_t j = q / SPLIT;
  const int a0 = (q % SPLIT) * RS;
  C v[N0];
#pragma unroll
  for (int p = 0; p < N0; ++p) v[p] = n < nrhs ? x[(j * N0 + p) * ld + n] : C{0, 0};
  const C *w = W + j * N0 * RR + a0;
  C acc[RS];
#pragma unroll
  for (int a = 0; a < RS; ++a) acc[a] = C{0, 0};
#pragma unroll
  for (int p = 0; p < N0; ++p) {
#pragma unroll
    for (int a = 0; a < RS; ++a) {
      const C c = cmulc(v[p], w[p * RR + a]);
      acc[a].x += c.x;
      acc[a].y += c.y;
    }
  }
#pragma unroll
  for (int a = 0; a < RS; ++a) y[act_off(j, a0 + a, n, P, RR, cs)] = acc[a];
}

// Leaf-out with the leaf index uniform across each wavefront (nrhs a multiple of 64).
// The n0 output rows of a leaf are split over SPLIT wavefronts (n0 / SPLIT rows each),
// which shortens each wavefront and so the tail of the launch.
template <class T, int RR, int SPLIT>
__global__ __launch_bounds__(256) void k_leaf_out_uni(const typename Cx<T>::type *__restrict__ W,
                                                      const typename Cx<T>::type *__restrict__ z,
                                                      typename Cx<T>::type *__restrict__ u, int64_t ld,
                                                      int64_t P, int n0, int64_t nrhs, int cs) {
  using C = typename Cx<T>::type;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= P * SPLIT * nrhs) return;
  const int64_t n = t % nrhs;
  const int q = __builtin_amdgcn_readfirstlane((int)(t / nrhs));
  const int64_t i = q / SPLIT;
  const int rows = n0 / SPLIT, p0 = (q % SPLIT) * rows;
  C v[RR];
#pragma unroll
  for (int a = 0; a < RR; ++a) v[a] = z[act_off(i, a, n, P, RR, cs)];
  for (int p = p0; p < p0 + rows; ++p) {
    const C *w = W + (i * n0 + p) * RR;
    C acc{0, 0};
#pragma unroll
    for (int a = 0; a < RR; ++a) {
      const C c = cmul(w[a], v[a]);
      acc.x += c.x;
      acc.y += c.y;
    }
    u[(i * n0 + p) * ld + n] = acc;
  }
}

template <class T, int RR>
__global__ void k_leaf_out_col(const typename Cx<T>::type *__restrict__ W,
                               const typename Cx<T>::type *__restrict__ z,
                               typename Cx<T>::type *__restrict__ u, int64_t ld, int64_t P, int n0,
                               int64_t nrhs, int cs) {
  using C = typename Cx<T>::type;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= P * nrhs) return;
  const int64_t n = t % nrhs, i = t / nrhs;
  C v[RR];
#pragma unroll
  for (int a = 0; a < RR; ++a) v[a] = z[act_off(i, a, n, P, RR, cs)];
  for (int p = 0; p < n0; ++p) {
    const C *w = W + (i * n0 + p) * RR;
    C acc{0, 0};
#pragma unroll
    for (int a = 0; a < RR; ++a) {
      const C c = cmul(w[a], v[a]);
      acc.x += c.x;
      acc.y += c.y;
    }
    u[(i * n0 + p) * ld + n] = acc;
  }
}

// One butterfly level: thread per (butterfly, output row, column).  Fb is the
// canonical level array [R^(l+1)][blo][r][R r].  With o = c_out r + a_out and
// k = c_in r + b_in the block entry is
//   direct (tconj = 0):  Fb[R hi + c_out][lo][a_out][c_in r + b_in]
//                        (G forward, H adjoint)
//   tconj = 1:           conj(Fb[R hi + c_in][lo][b_in][c_out r + a_out])
//                        (H forward, G adjoint)
template <class T>
__global__ void k_butterfly(const typename Cx<T>::type *__restrict__ Fb,
                            const typename Cx<T>::type *__restrict__ x,
                            typename Cx<T>::type *__restrict__ y, int64_t nb, int64_t blo, int R,
                            int r, int strided_in, int tconj, int64_t nslots, int64_t npad,
                            int cs) {
  using C = typename Cx<T>::type;
  const int Rr = R * r;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nb * Rr * npad) return;
  const int64_t n = t % npad;
  const int o = (int)((t / npad) % Rr);
  const int64_t b = t / (npad * Rr);
  const int64_t hi = b / blo, lo = b - hi * blo;
  const int co = o / r, a = o - co * r;
  C acc{0, 0};
  for (int ci = 0; ci < R; ++ci) {
    const int64_t s_in = slot_of(b, ci, blo, R, strided_in != 0);
    if (tconj) {
      const C *blk = Fb + ((R * hi + ci) * blo + lo) * r * Rr;
      for (int k = 0; k < r; ++k) {
        const C c = cmulc(x[act_off(s_in, k, n, nslots, r, cs)], blk[k * Rr + co * r + a]);
        acc.x += c.x;
        acc.y += c.y;
      }
    } else {
      const C *row = Fb + (((R * hi + co) * blo + lo) * r + a) * Rr + ci * r;
      for (int k = 0; k < r; ++k) {
        const C c = cmul(row[k], x[act_off(s_in, k, n, nslots, r, cs)]);
        acc.x += c.x;
        acc.y += c.y;
      }
    }
  }
  const int64_t s_out = slot_of(b, co, blo, R, strided_in == 0);
  y[act_off(s_out, a, n, nslots, r, cs)] = acc;
}

// y[(a m + b)][k] = S[a][b][k] x[(b m + a)][k]  (forward, M^h)
// y[(a m + b)][k] = S[b][a][k] x[(b m + a)][k]  (adjoint, (M^h)^* = (M^h)^T, S real)
template <class T>
__global__ void k_middle(const T *__restrict__ S, const typename Cx<T>::type *__restrict__ x,
                         typename Cx<T>::type *__restrict__ y, int64_t m, int r, int transpose,
                         int64_t npad, int cs) {
  using C = typename Cx<T>::type;
  const int64_t nslots = m * m;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nslots * r * npad) return;
  const int64_t n = t % npad;
  const int k = (int)((t / npad) % r);
  const int64_t so = t / (npad * r);
  const int64_t a = so / m, b = so - a * m;
  const T s = S[(transpose ? b * m + a : so) * r + k];
  const C v = x[act_off(b * m + a, k, n, nslots, r, cs)];
  y[act_off(so, k, n, nslots, r, cs)] = C{s * v.x, s * v.y};
}

// As k_middle for FP32 and even r, one thread per (slot, row pair, column): rows 2kp and
// 2kp + 1 of a column are adjacent in the activation layout (16-byte aligned), so each
// thread moves them with one 16-byte load and store.
__global__ void k_middle_pairs(const float *__restrict__ S, const float4 *__restrict__ x,
                               float4 *__restrict__ y, int64_t m, int r, int transpose, int64_t npad,
                               int cs) {
  const int64_t nslots = m * m;
  const int rp = r >> 1;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nslots * rp * npad) return;
  const int64_t n = t % npad;
  const int kp = (int)((t / npad) % rp);
  const int64_t so = t / (npad * rp);
  const int64_t a = so / m, b = so - a * m;
  const float *sp = S + (transpose ? b * m + a : so) * r + 2 * kp;
  const float s0 = sp[0], s1 = sp[1];
  const float4 v = x[act_off(b * m + a, 2 * kp, n, nslots, r, cs) >> 1];
  y[act_off(so, 2 * kp, n, nslots, r, cs) >> 1] = float4{s0 * v.x, s0 * v.y, s1 * v.z, s1 * v.w};
}

// grad[R hi + cx][lo][rx][cy r + ry] = sum_n X[strided(b,cx)][rx][n] conj(Y[contig(b,cy)][ry][n])
template <class T>
__global__ void k_level_grad(const typename Cx<T>::type *__restrict__ X,
                             const typename Cx<T>::type *__restrict__ Y,
                             typename Cx<T>::type *__restrict__ grad, int64_t nb, int64_t blo,
                             int R, int r, int64_t nslots, int64_t nrhs, int cs) {
  using C = typename Cx<T>::type;
  const int Rr = R * r;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nb * Rr * Rr) return;
  const int e2 = (int)(t % Rr);           // cy r + ry
  const int e1 = (int)((t / Rr) % Rr);    // cx r + rx
  const int64_t b = t / (Rr * Rr);
  const int cx = e1 / r, rx = e1 - cx * r;
  const int cy = e2 / r, ry = e2 - cy * r;
  const int64_t sx = slot_of(b, cx, blo, R, true);
  const int64_t sy = slot_of(b, cy, blo, R, false);
  C acc{0, 0};
  for (int64_t n = 0; n < nrhs; ++n) {
    const C c = cmulc(X[act_off(sx, rx, n, nslots, r, cs)], Y[act_off(sy, ry, n, nslots, r, cs)]);
    acc.x += c.x;
    acc.y += c.y;
  }
  const int64_t hi = b / blo, lo = b - hi * blo;
  const int64_t p = R * hi + cx;
  grad[((p * blo + lo) * r + rx) * Rr + e2] = acc;
}

// grad[j][p][a] = sum_n user[(j n0 + p) ld + n] conj(act[j][a][n])
template <class T>
__global__ void k_leaf_grad(const typename Cx<T>::type *__restrict__ user, int64_t ld,
                            const typename Cx<T>::type *__restrict__ act,
                            typename Cx<T>::type *__restrict__ grad, int64_t P, int n0, int r,
                            int64_t nrhs, int cs) {
  using C = typename Cx<T>::type;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= P * n0 * r) return;
  const int a = (int)(t % r);
  const int p = (int)((t / r) % n0);
  const int64_t j = t / (r * n0);
  C acc{0, 0};
  for (int64_t n = 0; n < nrhs; ++n) {
    const C c = cmulc(user[(j * n0 + p) * ld + n], act[act_off(j, a, n, P, r, cs)]);
    acc.x += c.x;
    acc.y += c.y;
  }
  grad[t] = acc;
}

// grad_S[i][j][k] = Re sum_n dz[(i m + j)][k][n] conj(y[(j m + i)][k][n])
template <class T>
__global__ void k_middle_grad(const typename Cx<T>::type *__restrict__ dz,
                              const typename Cx<T>::type *__restrict__ y, T *__restrict__ grad,
                              int64_t m, int r, int64_t nrhs, int cs) {
  const int64_t nslots = m * m;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nslots * r) return;
  const int k = (int)(t % r);
  const int64_t s = t / r;
  const int64_t i = s / m, j = s - i * m;
  T acc = 0;
  for (int64_t n = 0; n < nrhs; ++n) {
    const auto a = dz[act_off(s, k, n, nslots, r, cs)];
    const auto b = y[act_off(j * m + i, k, n, nslots, r, cs)];
    acc += a.x * b.x + a.y * b.y;
  }
  grad[t] = acc;
}

inline unsigned blocks_for(int64_t total, int bs) { return (unsigned)((total + bs - 1) / bs); }

template <class T>
hipError_t level_op_t(const bf_plan *p, const LevelOp &op, const void *in, int64_t ld_in,
                      void *out, int64_t ld_out, int64_t nrhs, hipStream_t s) {
  using C = typename Cx<T>::type;
  const int cs = p->cs;
  const int64_t npad = ((nrhs + (1 << cs) - 1) >> cs) << cs;
  const int bs = 256;
  switch (op.kind) {
    case LevelOp::kLeafIn:
      if (npad % 64 == 0 && (p->n0 == 16 || p->n0 == 4) && (p->r == 32 || p->r == 16 || p->r == 8) &&
          p->P * 2 * npad < (int64_t(1) << 31)) {
#define BF_LEAF_IN_UNI(N0, RR)                                                                  \
  if (p->n0 == N0 && p->r == RR) {                                                              \
    constexpr int SP = RR == 32 ? 2 : 1;                                                        \
    hipLaunchKernelGGL((k_leaf_in_uni<T, N0, RR, SP>), dim3(blocks_for(p->P * SP * npad, bs)),  \
                       dim3(bs), 0, s, (const C *)op.mat, (const C *)in, ld_in, (C *)out, p->P, \
                       nrhs, npad, cs);                                                         \
  }
        BF_LEAF_IN_UNI(16, 32) BF_LEAF_IN_UNI(16, 16) BF_LEAF_IN_UNI(16, 8)
        BF_LEAF_IN_UNI(4, 32) BF_LEAF_IN_UNI(4, 16) BF_LEAF_IN_UNI(4, 8)
#undef BF_LEAF_IN_UNI
        break;
      }
      if (p->n0 == 16 || p->n0 == 4) {
        const dim3 grid(blocks_for(p->P * npad, bs));
        if (p->n0 == 16)
          hipLaunchKernelGGL((k_leaf_in_col<T, 16>), grid, dim3(bs), 0, s, (const C *)op.mat,
                             (const C *)in, ld_in, (C *)out, p->P, p->r, nrhs, npad, cs);
        else
          hipLaunchKernelGGL((k_leaf_in_col<T, 4>), grid, dim3(bs), 0, s, (const C *)op.mat,
                             (const C *)in, ld_in, (C *)out, p->P, p->r, nrhs, npad, cs);
        break;
      }
      hipLaunchKernelGGL(k_leaf_in<T>, dim3(blocks_for(p->P * p->r * npad, bs)), dim3(bs), 0, s,
                         (const C *)op.mat, (const C *)in, ld_in, (C *)out, p->P, p->n0, p->r,
                         nrhs, npad, cs);
      break;
    case LevelOp::kButterfly:
      hipLaunchKernelGGL(k_butterfly<T>, dim3(blocks_for(op.nb * p->R * p->r * npad, bs)),
                         dim3(bs), 0, s, (const C *)op.mat, (const C *)in, (C *)out, op.nb,
                         op.blo, p->R, p->r, op.mode == kStridedIn ? 1 : 0, op.tconj ? 1 : 0,
                         p->P, npad, cs);
      break;
    case LevelOp::kMiddle:
      if constexpr (sizeof(T) == 4) {
        if (p->r % 2 == 0) {
          hipLaunchKernelGGL(k_middle_pairs, dim3(blocks_for(p->m * p->m * (p->r / 2) * npad, bs)),
                             dim3(bs), 0, s, (const float *)op.mat, (const float4 *)in,
                             (float4 *)out, p->m, p->r, op.tconj ? 1 : 0, npad, cs);
          break;
        }
      }
      hipLaunchKernelGGL(k_middle<T>, dim3(blocks_for(p->m * p->m * p->r * npad, bs)), dim3(bs),
                         0, s, (const T *)op.mat, (const C *)in, (C *)out, p->m, p->r,
                         op.tconj ? 1 : 0, npad, cs);
      break;
    case LevelOp::kLeafOut:
      if (nrhs % 64 == 0 && (p->r == 32 || p->r == 16 || p->r == 8) &&
          p->P * 2 * nrhs < (int64_t(1) << 31)) {
        const bool two = p->n0 % 2 == 0;
        const dim3 grid(blocks_for(p->P * (two ? 2 : 1) * nrhs, bs));
#define BF_LEAF_OUT_UNI(RR)                                                                     \
  if (p->r == RR) {                                                                             \
    if (two)                                                                                    \
      hipLaunchKernelGGL((k_leaf_out_uni<T, RR, 2>), grid, dim3(bs), 0, s, (const C *)op.mat,   \
                         (const C *)in, (C *)out, ld_out, p->P, p->n0, nrhs, cs);               \
    else                                                                                        \
      hipLaunchKernelGGL((k_leaf_out_uni<T, RR, 1>), grid, dim3(bs), 0, s, (const C *)op.mat,   \
                         (const C *)in, (C *)out, ld_out, p->P, p->n0, nrhs, cs);               \
  }
        BF_LEAF_OUT_UNI(32) BF_LEAF_OUT_UNI(16) BF_LEAF_OUT_UNI(8)
#undef BF_LEAF_OUT_UNI
        break;
      }
      if (p->r == 32 || p->r == 16 || p->r == 8) {
        const dim3 grid(blocks_for(p->P * nrhs, bs));
        if (p->r == 32)
          hipLaunchKernelGGL((k_leaf_out_col<T, 32>), grid, dim3(bs), 0, s, (const C *)op.mat,
                             (const C *)in, (C *)out, ld_out, p->P, p->n0, nrhs, cs);
        else if (p->r == 16)
          hipLaunchKernelGGL((k_leaf_out_col<T, 16>), grid, dim3(bs), 0, s, (const C *)op.mat,
                             (const C *)in, (C *)out, ld_out, p->P, p->n0, nrhs, cs);
        else
          hipLaunchKernelGGL((k_leaf_out_col<T, 8>), grid, dim3(bs), 0, s, (const C *)op.mat,
                             (const C *)in, (C *)out, ld_out, p->P, p->n0, nrhs, cs);
        break;
      }
      hipLaunchKernelGGL(k_leaf_out<T>, dim3(blocks_for(p->P * p->n0 * nrhs, bs)), dim3(bs), 0,
                         s, (const C *)op.mat, (const C *)in, (C *)out, ld_out, p->P, p->n0,
                         p->r, nrhs, cs);
      break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_level_op(const bf_plan *p, const LevelOp &op, const void *in, int64_t ld_in,
                           void *out, int64_t ld_out, int64_t nrhs, hipStream_t s) {
  if (op.kind == LevelOp::kButterfly && op.packed && p->cs == 5)
    return launch_level_mfma(p, op, in, out, nrhs, s);
  if (p->prec == BF_PREC_F64) return level_op_t<double>(p, op, in, ld_in, out, ld_out, nrhs, s);
  return level_op_t<float>(p, op, in, ld_in, out, ld_out, nrhs, s);
}

hipError_t launch_level_grad(const bf_plan *p, const LevelOp &op, const void *X, const void *Y,
                             void *grad, int64_t nrhs, hipStream_t s) {
  const int bs = 256;
  const int64_t total = op.nb * (int64_t)(p->R * p->r) * (p->R * p->r);
  if (p->prec == BF_PREC_F64)
    hipLaunchKernelGGL(k_level_grad<double>, dim3(blocks_for(total, bs)), dim3(bs), 0, s,
                       (const double2 *)X, (const double2 *)Y, (double2 *)grad, op.nb, op.blo,
                       p->R, p->r, p->P, nrhs, p->cs);
  else
    hipLaunchKernelGGL(k_level_grad<float>, dim3(blocks_for(total, bs)), dim3(bs), 0, s,
                       (const float2 *)X, (const float2 *)Y, (float2 *)grad, op.nb, op.blo, p->R,
                       p->r, p->P, nrhs, p->cs);
  return hipGetLastError();
}

hipError_t launch_leaf_grad(const bf_plan *p, const void *user, int64_t ld, const void *act,
                            void *grad, int64_t nrhs, hipStream_t s) {
  const int bs = 256;
  const int64_t total = p->P * p->n0 * p->r;
  if (p->prec == BF_PREC_F64)
    hipLaunchKernelGGL(k_leaf_grad<double>, dim3(blocks_for(total, bs)), dim3(bs), 0, s,
                       (const double2 *)user, ld, (const double2 *)act, (double2 *)grad, p->P,
                       p->n0, p->r, nrhs, p->cs);
  else
    hipLaunchKernelGGL(k_leaf_grad<float>, dim3(blocks_for(total, bs)), dim3(bs), 0, s,
                       (const float2 *)user, ld, (const float2 *)act, (float2 *)grad, p->P,
                       p->n0, p->r, nrhs, p->cs);
  return hipGetLastError();
}

hipError_t launch_middle_grad(const bf_plan *p, const void *dz, const void *y, void *grad,
                              int64_t nrhs, hipStream_t s) {
  const int bs = 256;
  const int64_t total = p->m * p->m * p->r;
  if (p->prec == BF_PREC_F64)
    hipLaunchKernelGGL(k_middle_grad<double>, dim3(blocks_for(total, bs)), dim3(bs), 0, s,
                       (const double2 *)dz, (const double2 *)y, (double *)grad, p->m, p->r, nrhs,
                       p->cs);
  else
    hipLaunchKernelGGL(k_middle_grad<float>, dim3(blocks_for(total, bs)), dim3(bs), 0, s,
                       (const float2 *)dz, (const float2 *)y, (float *)grad, p->m, p->r, nrhs,
                       p->cs);
  return hipGetLastError();
}

}  // namespace bfly
