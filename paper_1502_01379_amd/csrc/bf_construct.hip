// Construction of the butterfly factorization on the GPU in FP64: the entry-
// sampling route (Sec. 3.1, second case: Algorithm 2.2 on every middle-level
// block, stored in the first form of Sec. 2) followed by the recursive
// factorization of Sec. 3.2.1 (U -> G) and 3.2.2 (V -> H), plus the batched
// linear algebra it is built from.  Declared in include/bf_construct.h.
//
// Work is batched over blocks: every middle-level block of a chunk, or every
// (node, child, column group) item of a recursion level, is one workgroup of
// the factorization kernels, so a launch covers thousands of small problems.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "bf_construct.h"
#include "bf_internal.h"

// Index and value checks of the host build that runs these kernels on the CPU
// (BF_CONSTRUCT_HOST_CHECK); nothing in the library build.
#ifdef BF_CONSTRUCT_HOST_CHECK
#define BFC_ASSERT(c) SIMT_CHECK((c), #c)
#else
#define BFC_ASSERT(c) ((void)0)
#endif

namespace {

// ---- complex helpers (double2 = (re, im)) --------------------------------------

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cjmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// Sum over the 64 lanes of a wavefront.  Every lane returns lane 0's value, so
// branches taken on the result are uniform across the wavefront.
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return __shfl(v, 0, 64);
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return __shfl(v, 0, 64);
}

// Sum over a 256-thread workgroup; every thread must call it.
__device__ __forceinline__ double block_sum(double v, double *red4) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red4[0] + red4[1]) + (red4[2] + red4[3]);
}

inline unsigned grid_for(int64_t total, int threads = 256) {
  int64_t g = (total + threads - 1) / threads;
#ifdef BF_CONSTRUCT_HOST_CHECK
  g = std::min<int64_t>(g, 4);  // host check: few workgroups, the loops stride over the rest
#endif
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

// ---- kernel entries (Sec. 4, Example 1; Sec. 1.1) -------------------------------

constexpr double kTwoPi = 6.283185307179586;

__device__ double2 kernel_entry(int kind, int64_t N, int64_t i, int64_t k) {
  const int64_t xi = k - N / 2;
  int64_t t = (i * xi) % N;  // x xi mod 1 = ((i xi) mod N) / N, exact
  if (t < 0) t += N;
  double f = (double)t / (double)N;
  if (kind == BF_KERNEL_FIO) {
    const double x = (double)i / (double)N;
    const double c = (2.0 + sin(kTwoPi * x)) / 8.0;
    double s = c * (double)(xi < 0 ? -xi : xi);
    s -= floor(s);
    f += s;
    f -= floor(f);
  }
  double sn, cs;
  sincospi(2.0 * f, &sn, &cs);
  return make_double2(cs, sn);
}

// out[z][x][y] (x < nx, y < ny) = K(row, col) with, for trans = 0, row from
// index x and col from index y (trans = 1 swaps them), optionally conjugated.
// Row index u maps to row0 + rl[z][u] (or row0 + u without a list), likewise for
// columns; block z of an m x m grid of b x b blocks has row0 = (g / m) b and
// col0 = (g % m) b with g = g0 + z (m = 0: row0 = col0 = 0).
struct EntArgs {
  int kind;
  int64_t N;
  int64_t nblk, g0, m, b;
  const int64_t *rl;
  int64_t rls;
  const int64_t *cl;
  int64_t cls;
  int64_t nx, ny;
  int trans, conj;
  double2 *out;
  int64_t ld, bs;
};

__global__ __launch_bounds__(256) void k_entries(EntArgs a) {
  const int64_t per = a.nx * a.ny, total = per * a.nblk;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t z = e / per, rem = e - z * per, x = rem / a.ny, y = rem - x * a.ny;
    const int64_t u = a.trans ? y : x, v = a.trans ? x : y;
    int64_t row0 = 0, col0 = 0;
    if (a.m > 0) {
      const int64_t g = a.g0 + z;
      row0 = (g / a.m) * a.b;
      col0 = (g % a.m) * a.b;
    }
    const int64_t i = row0 + (a.rl ? a.rl[z * a.rls + u] : u);
    const int64_t k = col0 + (a.cl ? a.cl[z * a.cls + v] : v);
    BFC_ASSERT(!a.rl || (a.rl[z * a.rls + u] >= 0 && (a.m == 0 || a.rl[z * a.rls + u] < a.b)));
    BFC_ASSERT(!a.cl || (a.cl[z * a.cls + v] >= 0 && (a.m == 0 || a.cl[z * a.cls + v] < a.b)));
    BFC_ASSERT(i >= 0 && i < a.N && k >= 0 && k < a.N);
    double2 val = kernel_entry(a.kind, a.N, i, k);
    if (a.conj) val.y = -val.y;
    a.out[z * a.bs + x * a.ld + y] = val;
  }
}

// ---- random index sets (Algorithm 2.2, steps 2, 3 and 6) ---------------------------

// SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
// generators", 2014): a Weyl sequence passed through a 64-bit mixer.
__device__ __forceinline__ uint64_t splitmix64(uint64_t &state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

constexpr int kMaxDim = 8192;  // b: rows or columns of one middle-level block

// out[z] = keep[z][0 .. nkeep) followed by min(count, dim - nkeep) distinct
// indices of [0, dim) not in keep, drawn uniformly (all of them, in increasing
// order, when no more than `count` remain).
struct SampArgs {
  int64_t g0, dim;
  const int64_t *keep;
  int64_t nkeep, kstride;
  int64_t count;
  uint64_t seed, stream_id;
  int64_t *out;
  int64_t ostride;
};

__global__ __launch_bounds__(64) void k_sample(SampArgs a) {
  __shared__ uint32_t used[kMaxDim / 32];
  const int64_t z = blockIdx.x;
  const int64_t words = (a.dim + 31) / 32;
  for (int64_t w = threadIdx.x; w < words; w += 64) used[w] = 0;
  __syncthreads();
  if (threadIdx.x != 0) return;
  int64_t *o = a.out + z * a.ostride;
  for (int64_t t = 0; t < a.nkeep; ++t) {
    const int64_t v = a.keep[z * a.kstride + t];
    BFC_ASSERT(v >= 0 && v < a.dim);
    BFC_ASSERT(!(used[v >> 5] >> (v & 31) & 1u));  // the kept indices are distinct
    o[t] = v;
    used[v >> 5] |= 1u << (v & 31);
  }
  const int64_t rest = a.dim - a.nkeep;
  const int64_t want = a.count < rest ? a.count : rest;
  int64_t got = 0;
  if (want < rest) {
    uint64_t st = a.seed;
    st = splitmix64(st) ^ (uint64_t)(a.g0 + z);
    st = splitmix64(st) ^ a.stream_id;
    const int64_t cap = 64 * a.dim + 1024;
    for (int64_t tries = 0; got < want && tries < cap; ++tries) {
      const int64_t v = (int64_t)__umul64hi(splitmix64(st), (uint64_t)a.dim);
      if (used[v >> 5] >> (v & 31) & 1u) continue;
      used[v >> 5] |= 1u << (v & 31);
      o[a.nkeep + got++] = v;
    }
  }
  for (int64_t v = 0; got < want && v < a.dim; ++v) {
    if (used[v >> 5] >> (v & 31) & 1u) continue;
    used[v >> 5] |= 1u << (v & 31);
    o[a.nkeep + got++] = v;
  }
  BFC_ASSERT(got == want);
}

// ---- column pivots of a pivoted QR (Algorithm 2.2, steps 2 and 3) ------------------

constexpr int kPivMaxP = 128;

struct PivArgs {
  double2 *A;  // [blk][n][p]: column j of the p x n matrix at A + j p
  int64_t bs;
  int p;
  int n;
  int npiv;
  int64_t *piv;
};

// One workgroup per matrix.  Step k takes the column of largest residual norm
// (the first on ties), normalizes it to q and removes q q^* from every other
// remaining column; residual norms are recomputed from the updated columns, so
// they never suffer the cancellation of norm downdating.
__global__ __launch_bounds__(256) void k_colpiv(PivArgs a) {
  __shared__ double nrm[kMaxDim];
  __shared__ double2 q[kPivMaxP];
  __shared__ double bv[4];
  __shared__ int bi[4];
  __shared__ int pick;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double2 *A = a.A + blockIdx.x * a.bs;
  const int p = a.p, n = a.n;
  const double2 zero = make_double2(0.0, 0.0);
  for (int j = wave; j < n; j += 4) {
    const double2 *col = A + (int64_t)j * p;
    double s = 0.0;
    for (int t = lane; t < p; t += 64) s += cabs2(col[t]);
    BFC_ASSERT(std::isfinite(s));
    s = wave_sum(s);
    if (lane == 0) nrm[j] = s;
  }
  __syncthreads();
  for (int k = 0; k < a.npiv; ++k) {
    double best = -2.0;
    int besti = n;
    for (int j = tid; j < n; j += 256) {
      const double v = nrm[j];
      if (v > best) {
        best = v;
        besti = j;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(besti, o, 64);
      if (ov > best || (ov == best && oi < besti)) {
        best = ov;
        besti = oi;
      }
    }
    if (lane == 0) {
      bv[wave] = best;
      bi[wave] = besti;
    }
    __syncthreads();
    if (tid == 0) {
      double b0 = bv[0];
      int i0 = bi[0];
      for (int w = 1; w < 4; ++w)
        if (bv[w] > b0 || (bv[w] == b0 && bi[w] < i0)) {
          b0 = bv[w];
          i0 = bi[w];
        }
      BFC_ASSERT(i0 >= 0 && i0 < n);
      if (i0 < 0 || i0 >= n) i0 = n - 1;  // only reachable with non-finite entries
      pick = i0;
      a.piv[blockIdx.x * (int64_t)a.npiv + k] = i0;
      nrm[i0] = -1.0;
    }
    __syncthreads();
    const int pk = pick;
    if (wave == 0) {
      const double2 *col = A + (int64_t)pk * p;
      const double2 v0 = lane < p ? col[lane] : zero;
      const double2 v1 = lane + 64 < p ? col[lane + 64] : zero;
      const double s = wave_sum(cabs2(v0) + cabs2(v1));
      const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
      if (lane < p) q[lane] = cscale(v0, inv);
      if (lane + 64 < p) q[lane + 64] = cscale(v1, inv);
    }
    __syncthreads();
    for (int j = wave; j < n; j += 4) {
      if (nrm[j] < 0.0) continue;  // already a pivot (same j on every lane)
      double2 *col = A + (int64_t)j * p;
      double2 v0 = zero, v1 = zero, q0 = zero, q1 = zero;
      if (lane < p) {
        v0 = col[lane];
        q0 = q[lane];
      }
      if (lane + 64 < p) {
        v1 = col[lane + 64];
        q1 = q[lane + 64];
      }
      double2 c = cadd(cjmul(q0, v0), cjmul(q1, v1));
      c.x = wave_sum(c.x);
      c.y = wave_sum(c.y);
      v0 = csub(v0, cmul(c, q0));
      v1 = csub(v1, cmul(c, q1));
      if (lane < p) col[lane] = v0;
      if (lane + 64 < p) col[lane + 64] = v1;
      const double s = wave_sum(cabs2(v0) + cabs2(v1));
      if (lane == 0) nrm[j] = s;
    }
    __syncthreads();
  }
}

// ---- QR of tall blocks by Gram-Schmidt with reorthogonalization --------------------

constexpr int kQrMaxK = 64;
constexpr double kQrDependent = 1e-12;

struct QrArgs {
  double2 *A;  // [blk][n][k], overwritten by Q
  int64_t bs, n;
  int k;
  double2 *R;  // [blk][k][k] or NULL
};

__global__ __launch_bounds__(256) void k_cgs_qr(QrArgs a) {
  __shared__ double red4[4];
  __shared__ double red[4][16];
  __shared__ double2 coef[kQrMaxK];
  __shared__ double2 rsum[kQrMaxK];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double2 *A = a.A + blockIdx.x * a.bs;
  const int k = a.k;
  const int64_t n = a.n;
  for (int l = 0; l < k; ++l) {
    double s = 0.0;
    for (int64_t row = tid; row < n; row += 256) s += cabs2(A[row * k + l]);
    BFC_ASSERT(std::isfinite(s));
    const double n0 = block_sum(s, red4);
    if (tid < k) rsum[tid] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int pass = 0; pass < 2 && l > 0; ++pass) {
      for (int i0 = 0; i0 < l; i0 += 8) {
        double2 acc[8];
#pragma unroll
        for (int ii = 0; ii < 8; ++ii) acc[ii] = make_double2(0.0, 0.0);
        for (int64_t row = tid; row < n; row += 256) {
          const double2 w = A[row * k + l];
          const double2 *qr = A + row * k + i0;
#pragma unroll
          for (int ii = 0; ii < 8; ++ii)
            if (i0 + ii < l) acc[ii] = cadd(acc[ii], cjmul(qr[ii], w));
        }
#pragma unroll
        for (int ii = 0; ii < 8; ++ii) {
          acc[ii].x = wave_sum(acc[ii].x);
          acc[ii].y = wave_sum(acc[ii].y);
        }
        if (lane == 0) {
#pragma unroll
          for (int ii = 0; ii < 8; ++ii) {
            red[wave][2 * ii] = acc[ii].x;
            red[wave][2 * ii + 1] = acc[ii].y;
          }
        }
        __syncthreads();
        if (tid < 8 && i0 + tid < l) {
          const double2 c =
              make_double2((red[0][2 * tid] + red[1][2 * tid]) + (red[2][2 * tid] + red[3][2 * tid]),
                           (red[0][2 * tid + 1] + red[1][2 * tid + 1]) +
                               (red[2][2 * tid + 1] + red[3][2 * tid + 1]));
          coef[i0 + tid] = c;
          rsum[i0 + tid] = cadd(rsum[i0 + tid], c);
        }
        __syncthreads();
      }
      for (int64_t row = tid; row < n; row += 256) {
        double2 w = A[row * k + l];
        const double2 *qr = A + row * k;
        for (int i = 0; i < l; ++i) w = csub(w, cmul(qr[i], coef[i]));
        A[row * k + l] = w;
      }
      __syncthreads();
    }
    s = 0.0;
    for (int64_t row = tid; row < n; row += 256) s += cabs2(A[row * k + l]);
    const double nr = sqrt(block_sum(s, red4));
    const bool dep = !(nr > kQrDependent * sqrt(n0));
    const double inv = dep ? 0.0 : 1.0 / nr;
    for (int64_t row = tid; row < n; row += 256) A[row * k + l] = cscale(A[row * k + l], inv);
    if (a.R) {
      double2 *R = a.R + blockIdx.x * (int64_t)k * k;
      for (int i = tid; i < k; i += 256)
        R[i * k + l] = i < l ? rsum[i] : make_double2(i == l && !dep ? nr : 0.0, 0.0);
    }
    __syncthreads();
  }
}

// ---- thin SVD of small matrices by one-sided Jacobi rotations ----------------------

struct SvdArgs {
  const double2 *A;  // [blk][m][n]
  int m, n;
  double2 *U;  // [blk][m][n] or NULL
  double *s;   // [blk][n]
  double2 *V;  // [blk][n][n]
};

constexpr double kJacobiTol = 2e-15;
constexpr int kJacobiSweeps = 40;

// Columns are orthogonalized pairwise (Hestenes): for columns a_p, a_q with
// alpha = |a_p|^2, beta = |a_q|^2, gamma = a_p^* a_q = |gamma| e, the unitary
// [[c, s], [-s conj(e), c conj(e)]] with t = tan = sign(zeta)/(|zeta| +
// sqrt(1 + zeta^2)), zeta = (beta - alpha)/(2|gamma|), makes them orthogonal; V
// accumulates the same rotations.  A sweep visits every pair once in a round-robin
// order (n/2 disjoint pairs per round, one wavefront per pair, one lane per row).
// The matrix is first divided by its largest entry (undone on the singular
// values), and a column below 1e-16 of the Frobenius norm is left alone: without
// both, rotations among numerically zero columns shrink them into the subnormal
// range, where e = gamma/|gamma| overflows.
template <int MM, int NN>
__global__ __launch_bounds__(256) void k_jacobi_svd(SvdArgs a) {
  __shared__ double2 Ac[NN * MM];
  __shared__ double2 Vc[NN * NN];
  __shared__ double sig[NN];
  __shared__ int ord[NN];
  __shared__ int rotated;
  __shared__ double red4[4];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = a.m, n = a.n;
  const double2 *A = a.A + blockIdx.x * (int64_t)m * n;
  double mx = 0.0;
  for (int e = tid; e < m * n; e += 256) {
    const int x = e / n, y = e - x * n;
    const double2 v = A[e];
    BFC_ASSERT(std::isfinite(v.x) && std::isfinite(v.y));
    Ac[y * MM + x] = v;
    mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
  }
  for (int e = tid; e < n * n; e += 256) {
    const int x = e / n, y = e - x * n;
    Vc[y * NN + x] = make_double2(x == y ? 1.0 : 0.0, 0.0);
  }
  mx = wave_max(mx);
  __syncthreads();
  if (lane == 0) red4[wave] = mx;
  __syncthreads();
  mx = fmax(fmax(red4[0], red4[1]), fmax(red4[2], red4[3]));
  const double scale = mx > 0.0 ? mx : 1.0, inv_scale = 1.0 / scale;
  double f2 = 0.0;
  for (int e = tid; e < m * n; e += 256) {
    const int x = e / n, y = e - x * n;
    const double2 v = cscale(Ac[y * MM + x], inv_scale);
    Ac[y * MM + x] = v;
    f2 += cabs2(v);
  }
  const double tiny = 1e-32 * block_sum(f2, red4);
  const int ne = n + (n & 1);
  for (int sweep = 0; sweep < kJacobiSweeps; ++sweep) {
    __syncthreads();
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int rd = 0; rd < ne - 1; ++rd) {
      for (int pr = wave; pr < ne / 2; pr += 4) {
        int P, Q;
        if (pr == 0) {
          P = ne - 1;
          Q = rd;
        } else {
          P = (rd + pr) % (ne - 1);
          Q = (rd - pr + ne - 1) % (ne - 1);
        }
        if (P >= n || Q >= n) continue;
        double al = 0.0, be = 0.0;
        double2 ga = make_double2(0.0, 0.0);
        for (int x = lane; x < m; x += 64) {
          const double2 u = Ac[P * MM + x], v = Ac[Q * MM + x];
          al += cabs2(u);
          be += cabs2(v);
          ga = cadd(ga, cjmul(u, v));
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga.x = wave_sum(ga.x);
        ga.y = wave_sum(ga.y);
        const double g = sqrt(cabs2(ga));
        if (al <= tiny || be <= tiny || !(g > kJacobiTol * sqrt(al * be))) continue;
        const double2 e = make_double2(ga.x / g, ga.y / g);
        const double zeta = (be - al) / (2.0 * g);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int x = lane; x < m; x += 64) {
          const double2 u = Ac[P * MM + x], v = cjmul(e, Ac[Q * MM + x]);
          Ac[P * MM + x] = csub(cscale(u, c), cscale(v, s));
          Ac[Q * MM + x] = cadd(cscale(u, s), cscale(v, c));
        }
        for (int x = lane; x < n; x += 64) {
          const double2 u = Vc[P * NN + x], v = cjmul(e, Vc[Q * NN + x]);
          Vc[P * NN + x] = csub(cscale(u, c), cscale(v, s));
          Vc[Q * NN + x] = cadd(cscale(u, s), cscale(v, c));
        }
        if (lane == 0) rotated = 1;
      }
      __syncthreads();
    }
    if (!rotated) break;
  }
  __syncthreads();
  for (int j = wave; j < n; j += 4) {
    double s = 0.0;
    for (int x = lane; x < m; x += 64) s += cabs2(Ac[j * MM + x]);
    s = wave_sum(s);
    if (lane == 0) sig[j] = sqrt(s);
  }
  __syncthreads();
  if (tid == 0) {
    for (int j = 0; j < n; ++j) ord[j] = j;
    for (int i = 0; i < n; ++i) {
      int bst = i;
      for (int j = i + 1; j < n; ++j)
        if (sig[ord[j]] > sig[ord[bst]]) bst = j;
      const int tmp = ord[i];
      ord[i] = ord[bst];
      ord[bst] = tmp;
    }
  }
  __syncthreads();
  const int64_t z = blockIdx.x;
  for (int j = tid; j < n; j += 256) a.s[z * n + j] = sig[ord[j]] * scale;
  if (a.U) {
    for (int e = tid; e < m * n; e += 256) {
      const int x = e / n, kk = e - x * n;
      const double sg = sig[ord[kk]];
      a.U[z * (int64_t)m * n + e] = sg > 0.0 ? cscale(Ac[ord[kk] * MM + x], 1.0 / sg) : make_double2(0.0, 0.0);
    }
  }
  for (int e = tid; e < n * n; e += 256) {
    const int x = e / n, kk = e - x * n;
    a.V[z * (int64_t)n * n + e] = Vc[ord[kk] * NN + x];
  }
}

// ---- small batched products ---------------------------------------------------------

// C[z] = op(A[z]) diag(w) op(B[z]) (M x Nn, inner size K).  opa = 1: A^* (A stored
// K x M); opb = 1: B^* (B stored Nn x K).  dmode 1: w = d[z][kk]; dmode 2: w =
// 1/d[z][kk] where d[z][kk] > 1e-14 d[z][0] and 0 elsewhere (the pseudo-inverse of
// a descending singular-value list, relative cutoff 1e-14).  cm > 0 stores block
// z at C block (g % cm) cm + g / cm, g = cg0 + z (the transposed block grid).
struct GemmArgs {
  int64_t nblk, M, Nn, K;
  const double2 *A;
  int64_t lda, bsa;
  int opa;
  const double2 *B;
  int64_t ldb, bsb;
  int opb;
  const double *d;
  int64_t bsd;
  int dmode;
  double2 *C;
  int64_t ldc, bsc, cg0, cm;
};

constexpr double kPinvCut = 1e-14;

__global__ __launch_bounds__(256) void k_zgemm(GemmArgs a) {
  const int64_t per = a.M * a.Nn, total = per * a.nblk;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t z = e / per, rem = e - z * per, x = rem / a.Nn, y = rem - x * a.Nn;
    const double2 *A = a.A + z * a.bsa;
    const double2 *B = a.B + z * a.bsb;
    const double *d = a.d ? a.d + z * a.bsd : nullptr;
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t kk = 0; kk < a.K; ++kk) {
      double2 av = a.opa ? A[kk * a.lda + x] : A[x * a.lda + kk];
      if (a.opa) av.y = -av.y;
      double2 bv = a.opb ? B[y * a.ldb + kk] : B[kk * a.ldb + y];
      if (a.opb) bv.y = -bv.y;
      double w = 1.0;
      if (a.dmode == 1) w = d[kk];
      if (a.dmode == 2) w = d[kk] > kPinvCut * d[0] ? 1.0 / d[kk] : 0.0;
      acc = cadd(acc, cscale(cmul(av, bv), w));
    }
    int64_t cz = z;
    if (a.cm > 0) {
      const int64_t g = a.cg0 + z;
      cz = (g % a.cm) * a.cm + g / a.cm;
    }
    a.C[cz * a.bsc + x * a.ldc + y] = acc;
  }
}

// dst[z][t][y] = src[z][idx[z][t]][y]
struct GatherArgs {
  int64_t nblk;
  const double2 *src;
  int64_t sbs, sld;
  const int64_t *idx;
  int64_t ibs, nrow, ncol;
  double2 *dst;
  int64_t dbs;
};

__global__ __launch_bounds__(256) void k_gather_rows(GatherArgs a) {
  const int64_t per = a.nrow * a.ncol, total = per * a.nblk;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t z = e / per, rem = e - z * per, t = rem / a.ncol, y = rem - t * a.ncol;
    BFC_ASSERT(a.idx[z * a.ibs + t] >= 0 && a.idx[z * a.ibs + t] < a.sbs / a.sld);
    a.dst[z * a.dbs + rem] = a.src[z * a.sbs + a.idx[z * a.ibs + t] * a.sld + y];
  }
}

// Middle level, first form of Sec. 2: from the SVD M = UM diag(sM) VM^* of the
// middle matrix, TU = UM diag(s'), TV = VM diag(s') and S = 1/s' with s' the kept
// singular values (s > 0 and s > drop s_max; the others give zeros).
struct MidFinArgs {
  int64_t nblk, g0;
  int r;
  const double2 *UM, *VM;
  const double *sM;
  double drop;
  double2 *TU, *TV;
  double *S;
};

__global__ __launch_bounds__(256) void k_mid_finish(MidFinArgs a) {
  const int64_t per = (int64_t)a.r * a.r, total = per * a.nblk;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t z = e / per, rem = e - z * per, x = rem / a.r, kk = rem - x * a.r;
    const double sg = a.sM[z * a.r + kk], s0 = a.sM[z * a.r];
    const bool keep = sg > 0.0 && sg > a.drop * s0;
    const double w = keep ? sg : 0.0;
    a.TU[e] = cscale(a.UM[e], w);
    a.TV[e] = cscale(a.VM[e], w);
    if (x == 0) a.S[(a.g0 + z) * a.r + kk] = keep ? 1.0 / sg : 0.0;
  }
}

// Recursion (Sec. 3.2.1): item (R a + c) nbo + jp gathers the rows of child c of
// node a from the R column blocks R jp .. R jp + R - 1 of level array cur
// [nodes][nbk][rows][r]: W[item][row][t r + kk] = cur[a][R jp + t][c crow + row][kk].
struct RecGatherArgs {
  const double2 *cur;
  int64_t item0, nitems;
  int R, r;
  int64_t nbk, rows;
  double2 *W;
};

__global__ __launch_bounds__(256) void k_rec_gather(RecGatherArgs a) {
  const int64_t crow = a.rows / a.R, nbo = a.nbk / a.R, Rr = (int64_t)a.R * a.r;
  const int64_t per = crow * Rr, total = per * a.nitems;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t z = e / per, rem = e - z * per, row = rem / Rr, col = rem - row * Rr;
    const int64_t item = a.item0 + z, node2 = item / nbo, jp = item - node2 * nbo;
    const int64_t an = node2 / a.R, c = node2 - an * a.R;
    const int64_t t = col / a.r, kk = col - t * a.r;
    a.W[e] = a.cur[((an * a.nbk + a.R * jp + t) * a.rows + c * crow + row) * a.r + kk];
  }
}

// From the SVD R = UR diag(sR) VR^* of the R factor of W = Q R: the rank-r
// truncation W ~ (Q UR_r diag(sR_r)) VR_r^*; T = UR_r diag(sR_r) (Rr x r) and the
// transfer block G = VR_r^* (r x Rr), the third form of Sec. 2.
struct RecFinArgs {
  int64_t nitems;
  int Rr, r;
  const double2 *UR, *VR;
  const double *sR;
  double2 *T, *G;
};

__global__ __launch_bounds__(256) void k_rec_finish(RecFinArgs a) {
  const int64_t per = (int64_t)a.Rr * a.r, total = per * a.nitems;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t z = e / per, rem = e - z * per, x = rem / a.r, kk = rem - x * a.r;
    const int64_t sq = (int64_t)a.Rr * a.Rr;
    a.T[e] = cscale(a.UR[z * sq + x * a.Rr + kk], a.sR[z * a.Rr + kk]);
    double2 v = a.VR[z * sq + x * a.Rr + kk];
    v.y = -v.y;
    a.G[z * per + kk * a.Rr + x] = v;
  }
}

// ---- host-side launchers ----------------------------------------------------------

hipError_t launch_entries(const EntArgs &a, hipStream_t s) {
  const int64_t total = a.nblk * a.nx * a.ny;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_entries, dim3(grid_for(total)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sample(const SampArgs &a, int64_t nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_sample, dim3((unsigned)nblk), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_colpiv(const PivArgs &a, int64_t nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_colpiv, dim3((unsigned)nblk), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_qr(const QrArgs &a, int64_t nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_cgs_qr, dim3((unsigned)nblk), dim3(256), 0, s, a);
  return hipGetLastError();
}

bool svd_supported(int m, int n) { return m >= 1 && n >= 1 && ((m <= 128 && n <= 32) || (m <= 64 && n <= 64)); }

hipError_t launch_svd(const SvdArgs &a, int64_t nblk, hipStream_t s) {
  if (a.m <= 128 && a.n <= 32)
    hipLaunchKernelGGL((k_jacobi_svd<128, 32>), dim3((unsigned)nblk), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_jacobi_svd<64, 64>), dim3((unsigned)nblk), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <class K, class A>
hipError_t launch_flat(K kern, const A &a, int64_t total, hipStream_t s) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(kern, dim3(grid_for(total)), dim3(256), 0, s, a);
  return hipGetLastError();
}

GemmArgs gemm(int64_t nblk, int64_t M, int64_t Nn, int64_t K, const double2 *A, int64_t lda, int64_t bsa,
              int opa, const double2 *B, int64_t ldb, int64_t bsb, int opb, double2 *C, int64_t ldc,
              int64_t bsc) {
  GemmArgs g{};
  g.nblk = nblk;
  g.M = M;
  g.Nn = Nn;
  g.K = K;
  g.A = A;
  g.lda = lda;
  g.bsa = bsa;
  g.opa = opa;
  g.B = B;
  g.ldb = ldb;
  g.bsb = bsb;
  g.opb = opb;
  g.C = C;
  g.ldc = ldc;
  g.bsc = bsc;
  return g;
}

hipError_t launch_gemm(const GemmArgs &a, hipStream_t s) {
  return launch_flat(k_zgemm, a, a.nblk * a.M * a.Nn, s);
}

bf_status fail(bf_status st, const std::string &msg) {
  bfly::set_create_error(msg);
  return st;
}

// Device allocations of one call, released on every return path.
struct Arena {
  std::vector<void *> ptrs;
  ~Arena() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  template <class T>
  hipError_t get(T **out, int64_t count) {
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, std::max<int64_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    ptrs.push_back(p);
    *out = (T *)p;
    return hipSuccess;
  }
  void release(void *p) {
    for (auto &q : ptrs)
      if (q == p) {
        (void)hipFree(q);
        q = nullptr;
      }
  }
};

#define BFC_HIP(expr)                                                                        \
  do {                                                                                       \
    const hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                                    \
      return fail(e_ == hipErrorOutOfMemory ? BF_ERR_ALLOC : BF_ERR_HIP,                     \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                        \
  } while (0)

constexpr int64_t kScratchBytes = int64_t(1) << 30;

int64_t ipow(int64_t b, int e) {
  int64_t v = 1;
  for (int i = 0; i < e; ++i) v *= b;
  return v;
}

}  // namespace

extern "C" {

bf_status bf_kernel_entries(int32_t kind, int64_t N, const int64_t *rows, int64_t nrows,
                            const int64_t *cols, int64_t ncols, double *out, int64_t ld,
                            hipStream_t stream) {
  if (kind != BF_KERNEL_FOURIER && kind != BF_KERNEL_FIO) return fail(BF_ERR_INVALID_ARG, "unknown kernel kind");
  if (N < 1 || nrows < 0 || ncols < 0 || ld < ncols) return fail(BF_ERR_INVALID_ARG, "bad sizes");
  if (nrows == 0 || ncols == 0) return BF_OK;
  if (!rows || !cols || !out) return fail(BF_ERR_INVALID_ARG, "NULL pointer");
  EntArgs a{};
  a.kind = kind;
  a.N = N;
  a.nblk = 1;
  a.rl = rows;
  a.cl = cols;
  a.nx = nrows;
  a.ny = ncols;
  a.out = (double2 *)out;
  a.ld = ld;
  BFC_HIP(launch_entries(a, stream));
  return BF_OK;
}

bf_status bf_batched_svd(const double *A, int64_t batch, int32_t m, int32_t n, double *U, double *s,
                         double *V, hipStream_t stream) {
  if (batch < 0 || !A || !s || !V) return fail(BF_ERR_INVALID_ARG, "NULL pointer or negative batch");
  if (!svd_supported(m, n)) return fail(BF_ERR_UNSUPPORTED, "SVD sizes: m <= 128 and n <= 32, or m, n <= 64");
  if (batch == 0) return BF_OK;
  SvdArgs a{(const double2 *)A, m, n, (double2 *)U, s, (double2 *)V};
  BFC_HIP(launch_svd(a, batch, stream));
  return BF_OK;
}

bf_status bf_batched_qr(double *A, int64_t batch, int64_t n, int32_t k, double *R, hipStream_t stream) {
  if (batch < 0 || n < 1 || !A) return fail(BF_ERR_INVALID_ARG, "NULL pointer or bad sizes");
  if (k < 1 || k > kQrMaxK) return fail(BF_ERR_UNSUPPORTED, "QR: 1 <= k <= 64");
  if (batch == 0) return BF_OK;
  QrArgs a{(double2 *)A, n * k, n, k, (double2 *)R};
  BFC_HIP(launch_qr(a, batch, stream));
  return BF_OK;
}

bf_status bf_batched_column_pivots(double *At, int64_t batch, int32_t p, int64_t n, int32_t npiv,
                                   int64_t *piv, hipStream_t stream) {
  if (batch < 0 || !At || !piv) return fail(BF_ERR_INVALID_ARG, "NULL pointer or negative batch");
  if (p < 1 || p > kPivMaxP || n < 1 || n > kMaxDim || npiv < 1 || npiv > n)
    return fail(BF_ERR_UNSUPPORTED, "column pivots: p <= 128, 1 <= npiv <= n <= 8192");
  if (batch == 0) return BF_OK;
  PivArgs a{(double2 *)At, (int64_t)n * p, p, (int)n, npiv, piv};
  BFC_HIP(launch_colpiv(a, batch, stream));
  return BF_OK;
}

bf_status bf_construct_from_kernel(const bf_shape *shape, int32_t kind, int32_t q, int32_t iters,
                                   uint64_t seed, double drop_rel, const bf_factors_out *out,
                                   hipStream_t stream) {
  if (!shape || !out || !out->VL || !out->UL || !out->S) return fail(BF_ERR_INVALID_ARG, "NULL pointer");
  if (kind != BF_KERNEL_FOURIER && kind != BF_KERNEL_FIO) return fail(BF_ERR_INVALID_ARG, "unknown kernel kind");
  const int R = shape->radix, n0 = shape->leaf, L = shape->L, r = shape->r;
  if (R != 2 && R != 4) return fail(BF_ERR_SHAPE, "radix must be 2 or 4");
  if (n0 < 1 || L < 0 || L % 2 || r < 1 || L > 40) return fail(BF_ERR_SHAPE, "leaf >= 1, even L, r >= 1");
  if (shape->N != n0 * ipow(R, L)) return fail(BF_ERR_SHAPE, "N must equal leaf * radix^L");
  if (q < 1 || iters < 1 || !(drop_rel >= 0.0)) return fail(BF_ERR_INVALID_ARG, "q >= 1, iters >= 1, drop_rel >= 0");
  const int h = L / 2, lv = L - h;
  if (lv > 0 && (!out->H || !out->G)) return fail(BF_ERR_INVALID_ARG, "NULL H or G");
  for (int t = 0; t < lv; ++t)
    if (!out->H[t] || !out->G[t]) return fail(BF_ERR_INVALID_ARG, "NULL H[t] or G[t]");
  const int64_t N = shape->N, m = ipow(R, h), b = N / m, nb = m * m;
  const int Rr = R * r;
  const int64_t rq = (int64_t)r * q;
  const int64_t pmax = std::min<int64_t>(b, r + rq);
  if (r > b) return fail(BF_ERR_UNSUPPORTED, "r must not exceed the middle block size N / R^(L/2)");
  if (r > 32 || Rr > 64) return fail(BF_ERR_UNSUPPORTED, "r <= 32 and radix * r <= 64");
  if (pmax > kPivMaxP) return fail(BF_ERR_UNSUPPORTED, "min(b, r (q + 1)) must be at most 128");
  if (b > kMaxDim) return fail(BF_ERR_UNSUPPORTED, "the middle block size must be at most 8192");
  // Switched off: on the GPU this driver gave a less accurate factorization than
  // the same code run on the host (1.5e-3 against 1.1e-4 for the Fourier kernel at
  // N = 1024, r = 24) and, for N = 512 with 128-point leaves, an illegal memory
  // access; the host run under AddressSanitizer is clean and matches the
  // reference accuracy, and the cause on the device is not found yet.  Only a host
  // build of this file made to check the driver (BF_CONSTRUCT_HOST_CHECK) runs it;
  // the library build never defines that macro.
#ifndef BF_CONSTRUCT_HOST_CHECK
  return fail(BF_ERR_UNSUPPORTED,
              "bf_construct_from_kernel is switched off: its device run is under investigation");
#endif

  Arena ar;
  double2 *Uh, *Vh;
  double *Sd;
  BFC_HIP(ar.get(&Uh, nb * b * r));
  BFC_HIP(ar.get(&Vh, nb * b * r));
  BFC_HIP(ar.get(&Sd, nb * r));

  // ---- middle level, Algorithm 2.2 on every block, in chunks of blocks
  const int64_t cd = sizeof(double2);
  const int64_t per_block = cd * (b * pmax + 2 * b * r + 4 * pmax * r + pmax * pmax + 2 * r * pmax + 12 * r * r) +
                            8 * (2 * r + 2 * pmax + 3 * r);
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nb, kScratchBytes / per_block));
  double2 *Ap, *Qc, *Qr, *QcI, *QrJ, *Z, *U1, *V1, *U2, *V2, *X1, *X, *Y1, *M, *UM, *VM, *TU, *TV;
  double *s1, *s2, *sM;
  int64_t *prow, *pcol, *I, *J;
  BFC_HIP(ar.get(&Ap, chunk * b * pmax));
  BFC_HIP(ar.get(&Qc, chunk * b * r));
  BFC_HIP(ar.get(&Qr, chunk * b * r));
  BFC_HIP(ar.get(&QcI, chunk * pmax * r));
  BFC_HIP(ar.get(&QrJ, chunk * pmax * r));
  BFC_HIP(ar.get(&Z, chunk * pmax * pmax));
  BFC_HIP(ar.get(&U1, chunk * pmax * r));
  BFC_HIP(ar.get(&U2, chunk * pmax * r));
  BFC_HIP(ar.get(&X1, chunk * r * pmax));
  BFC_HIP(ar.get(&X, chunk * r * pmax));
  for (double2 **pp : {&V1, &V2, &Y1, &M, &UM, &VM, &TU, &TV}) BFC_HIP(ar.get(pp, chunk * r * r));
  BFC_HIP(ar.get(&s1, chunk * r));
  BFC_HIP(ar.get(&s2, chunk * r));
  BFC_HIP(ar.get(&sM, chunk * r));
  BFC_HIP(ar.get(&prow, chunk * r));
  BFC_HIP(ar.get(&pcol, chunk * r));
  BFC_HIP(ar.get(&I, chunk * pmax));
  BFC_HIP(ar.get(&J, chunk * pmax));

  auto entries = [&](int64_t n, int64_t g0, const int64_t *rl, int64_t rls, const int64_t *cl, int64_t cls,
                     int64_t nx, int64_t ny, int trans, int conj, double2 *o, int64_t ld, int64_t bs) {
    EntArgs a{};
    a.kind = kind;
    a.N = N;
    a.nblk = n;
    a.g0 = g0;
    a.m = m;
    a.b = b;
    a.rl = rl;
    a.rls = rls;
    a.cl = cl;
    a.cls = cls;
    a.nx = nx;
    a.ny = ny;
    a.trans = trans;
    a.conj = conj;
    a.out = o;
    a.ld = ld;
    a.bs = bs;
    return launch_entries(a, stream);
  };
  auto sample = [&](int64_t n, int64_t g0, const int64_t *keep, int64_t nkeep, uint64_t sid, int64_t *o) {
    SampArgs a{g0, b, keep, nkeep, r, rq, seed, sid, o, pmax};
    return launch_sample(a, n, stream);
  };

  for (int64_t g0 = 0; g0 < nb; g0 += chunk) {
    const int64_t n = std::min(chunk, nb - g0);
    int64_t ne = 0;
    for (int it = 0; it < iters; ++it) {
      // step 2: rows I = (important rows) + r q random rows; pivoted QR of Z(I, :)
      const int64_t nI = ne + std::min<int64_t>(rq, b - ne);
      BFC_HIP(sample(n, g0, prow, ne, 4 * (uint64_t)it + 1, I));
      BFC_HIP(entries(n, g0, I, pmax, nullptr, 0, b, nI, 1, 0, Ap, nI, b * pmax));
      BFC_HIP(launch_colpiv(PivArgs{Ap, b * pmax, (int)nI, (int)b, r, pcol}, n, stream));
      // step 3: columns J = (important columns) + r q random columns; pivoted LQ of Z(:, J)
      const int64_t nJ = r + std::min<int64_t>(rq, b - r);
      BFC_HIP(sample(n, g0, pcol, r, 4 * (uint64_t)it + 2, J));
      BFC_HIP(entries(n, g0, nullptr, 0, J, pmax, b, nJ, 0, 1, Ap, nJ, b * pmax));
      BFC_HIP(launch_colpiv(PivArgs{Ap, b * pmax, (int)nJ, (int)b, r, prow}, n, stream));
      ne = r;
    }
    // step 5: orthonormal bases of the important columns and rows
    BFC_HIP(entries(n, g0, nullptr, 0, pcol, r, b, r, 0, 0, Qc, r, b * r));
    BFC_HIP(launch_qr(QrArgs{Qc, b * r, b, r, nullptr}, n, stream));
    BFC_HIP(entries(n, g0, prow, r, nullptr, 0, b, r, 1, 1, Qr, r, b * r));
    BFC_HIP(launch_qr(QrArgs{Qr, b * r, b, r, nullptr}, n, stream));
    // step 6: important plus r q fresh rows and columns; M = Qc(I,:)^+ Z(I,J) (Qr(J,:)^*)^+
    const int64_t nI = r + std::min<int64_t>(rq, b - r), nJ = nI;
    BFC_HIP(sample(n, g0, prow, r, 4 * (uint64_t)iters + 1, I));
    BFC_HIP(sample(n, g0, pcol, r, 4 * (uint64_t)iters + 2, J));
    BFC_HIP(launch_flat(k_gather_rows, GatherArgs{n, Qc, b * r, r, I, pmax, nI, r, QcI, nI * r}, n * nI * r, stream));
    BFC_HIP(launch_flat(k_gather_rows, GatherArgs{n, Qr, b * r, r, J, pmax, nJ, r, QrJ, nJ * r}, n * nJ * r, stream));
    BFC_HIP(entries(n, g0, I, pmax, J, pmax, nI, nJ, 0, 0, Z, nJ, nI * nJ));
    BFC_HIP(launch_svd(SvdArgs{QcI, (int)nI, r, U1, s1, V1}, n, stream));
    BFC_HIP(launch_svd(SvdArgs{QrJ, (int)nJ, r, U2, s2, V2}, n, stream));
    // X1 = U1^* Z (r x nJ); X = V1 diag(s1^+) X1
    BFC_HIP(launch_gemm(gemm(n, r, nJ, nI, U1, r, nI * r, 1, Z, nJ, nI * nJ, 0, X1, nJ, r * nJ), stream));
    GemmArgs gx = gemm(n, r, nJ, r, V1, r, r * r, 0, X1, nJ, r * nJ, 0, X, nJ, r * nJ);
    gx.d = s1;
    gx.bsd = r;
    gx.dmode = 2;
    BFC_HIP(launch_gemm(gx, stream));
    // M = (X U2) diag(s2^+) V2^*
    BFC_HIP(launch_gemm(gemm(n, r, r, nJ, X, nJ, r * nJ, 0, U2, r, nJ * r, 0, Y1, r, r * r), stream));
    GemmArgs gm = gemm(n, r, r, r, Y1, r, r * r, 0, V2, r, r * r, 1, M, r, r * r);
    gm.d = s2;
    gm.bsd = r;
    gm.dmode = 2;
    BFC_HIP(launch_gemm(gm, stream));
    // step 7 and the first form: U^h = Qc UM S0, V^h = Qr VM S0, S^h = S0^{-1}
    BFC_HIP(launch_svd(SvdArgs{M, r, r, UM, sM, VM}, n, stream));
    BFC_HIP(launch_flat(k_mid_finish, MidFinArgs{n, g0, r, UM, VM, sM, drop_rel, TU, TV, Sd}, n * r * r, stream));
    BFC_HIP(launch_gemm(gemm(n, b, r, r, Qc, r, b * r, 0, TU, r, r * r, 0, Uh + g0 * b * r, r, b * r), stream));
    GemmArgs gv = gemm(n, b, r, r, Qr, r, b * r, 0, TV, r, r * r, 0, Vh, r, b * r);
    gv.cg0 = g0;
    gv.cm = m;
    BFC_HIP(launch_gemm(gv, stream));
  }
  BFC_HIP(hipStreamSynchronize(stream));
  for (void *pp : {(void *)Ap, (void *)Qc, (void *)Qr, (void *)QcI, (void *)QrJ, (void *)Z, (void *)U1, (void *)U2,
                   (void *)X1, (void *)X, (void *)V1, (void *)V2, (void *)Y1, (void *)M, (void *)UM, (void *)VM,
                   (void *)TU, (void *)TV, (void *)s1, (void *)s2, (void *)sM, (void *)prow, (void *)pcol,
                   (void *)I, (void *)J})
    ar.release(pp);
  BFC_HIP(hipMemcpy(out->S, Sd, nb * r * sizeof(double), hipMemcpyDeviceToHost));

  // ---- recursion, Sec. 3.2.1 (U -> G, U^L) and 3.2.2 (V -> H, V^L)
  for (int side = 0; side < 2; ++side) {
    double2 *cur = side ? Vh : Uh;
    int64_t nodes = m, nbk = m, rows = b;
    for (int t = 0; t < lv; ++t) {
      const int64_t crow = rows / R, nbo = nbk / R, items = nodes * R * nbo;
      double2 *nxt, *Gd;
      BFC_HIP(ar.get(&nxt, items * crow * r));
      BFC_HIP(ar.get(&Gd, items * r * Rr));
      const int64_t per_item = cd * (crow * Rr + 3 * Rr * Rr + Rr * r) + 8 * Rr;
      const int64_t ich = std::max<int64_t>(1, std::min<int64_t>(items, kScratchBytes / per_item));
      double2 *W, *Rm, *UR, *VR, *T;
      double *sR;
      BFC_HIP(ar.get(&W, ich * crow * Rr));
      BFC_HIP(ar.get(&Rm, ich * Rr * Rr));
      BFC_HIP(ar.get(&UR, ich * Rr * Rr));
      BFC_HIP(ar.get(&VR, ich * Rr * Rr));
      BFC_HIP(ar.get(&T, ich * Rr * r));
      BFC_HIP(ar.get(&sR, ich * Rr));
      for (int64_t i0 = 0; i0 < items; i0 += ich) {
        const int64_t n = std::min(ich, items - i0);
        BFC_HIP(launch_flat(k_rec_gather, RecGatherArgs{cur, i0, n, R, r, nbk, rows, W}, n * crow * Rr, stream));
        BFC_HIP(launch_qr(QrArgs{W, crow * Rr, crow, Rr, Rm}, n, stream));
        BFC_HIP(launch_svd(SvdArgs{Rm, Rr, Rr, UR, sR, VR}, n, stream));
        BFC_HIP(launch_flat(k_rec_finish, RecFinArgs{n, Rr, r, UR, VR, sR, T, Gd + i0 * r * Rr}, n * Rr * r, stream));
        BFC_HIP(launch_gemm(gemm(n, crow, r, Rr, W, Rr, crow * Rr, 0, T, r, Rr * r, 0, nxt + i0 * crow * r, r,
                                 crow * r),
                            stream));
      }
      BFC_HIP(hipStreamSynchronize(stream));
      double *dst = side ? out->H[t] : out->G[t];
      BFC_HIP(hipMemcpy(dst, Gd, items * r * Rr * cd, hipMemcpyDeviceToHost));
      for (void *pp : {(void *)W, (void *)Rm, (void *)UR, (void *)VR, (void *)T, (void *)sR, (void *)Gd, (void *)cur})
        ar.release(pp);
      cur = nxt;
      nodes *= R;
      nbk = nbo;
      rows = crow;
    }
    BFC_HIP(hipStreamSynchronize(stream));
    BFC_HIP(hipMemcpy(side ? out->VL : out->UL, cur, nodes * rows * r * cd, hipMemcpyDeviceToHost));
    ar.release(cur);
  }
  return BF_OK;
}

}  // extern "C"
