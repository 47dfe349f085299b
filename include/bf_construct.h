/*
 * bf_construct.h -- construction of the butterfly factorization on the GPU, FP64.
 *
 * The entry-sampling route of the paper (Sec. 3.1, second case, with the
 * randomized sampling of Algorithm 2.2 on every middle-level block, then the
 * recursive factorization of Sec. 3.2.1 and 3.2.2), run on the current HIP
 * device for the built-in 1D kernels, with the batched FP64 linear algebra it
 * is made of.  The result is the canonical factor set of bf.h, ready for
 * bf_create_from_factors.
 *
 * All calls return a bf_status and never abort; on failure bf_last_error(NULL)
 * holds a message (thread-local).  Every matrix below is complex128 stored as
 * interleaved (re, im) doubles, row-major.  "Device" pointers are HIP device
 * memory owned by the caller; the calls are asynchronous on `stream` unless
 * stated otherwise.
 */
#ifndef BF_CONSTRUCT_H_
#define BF_CONSTRUCT_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#include "bf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Built-in kernels K_{ik} = exp(2 pi i Phi(x_i, xi_k)), x_i = i/N, xi_k = k - N/2
 * (0-based points of Sec. 4, Example 1):
 *   BF_KERNEL_FOURIER: Phi = x xi                                   (Sec. 1.1)
 *   BF_KERNEL_FIO:     Phi = x xi + c(x)|xi|, c(x) = (2 + sin 2 pi x)/8   (Example 1)
 * The product x xi is reduced modulo 1 exactly in integers ((i (k - N/2)) mod N,
 * over N); only c(x)|xi| is reduced in FP64. */
typedef enum { BF_KERNEL_FOURIER = 0, BF_KERNEL_FIO = 1 } bf_kernel_kind;

/* out[a][c] = K[rows[a]][cols[c]] for a < nrows, c < ncols; rows, cols: device
 * int64 indices in [0, N); out: device, row stride ld >= ncols (complex elements).
 * Errors: BF_ERR_INVALID_ARG (NULL, sizes < 0, ld < ncols, unknown kind),
 * BF_ERR_HIP. */
bf_status bf_kernel_entries(int32_t kind, int64_t N, const int64_t *rows, int64_t nrows,
                            const int64_t *cols, int64_t ncols, double *out, int64_t ld,
                            hipStream_t stream);

/* Batched thin SVD A = U diag(s) V^* of `batch` matrices A [batch][m][n] (device),
 * by one-sided Jacobi rotations; m <= 128 and n <= 32, or m <= 64 and n <= 64.
 * U [batch][m][n] (may be NULL; columns of zero singular values are zero),
 * s [batch][n] descending, V [batch][n][n] unitary.  A is not modified.
 * Errors: BF_ERR_INVALID_ARG, BF_ERR_UNSUPPORTED (sizes), BF_ERR_HIP. */
bf_status bf_batched_svd(const double *A, int64_t batch, int32_t m, int32_t n, double *U,
                         double *s, double *V, hipStream_t stream);

/* Batched QR A = Q R of A [batch][n][k] (device, k <= 64, any n >= 1) by classical
 * Gram-Schmidt with one reorthogonalization; Q overwrites A.  A column whose part
 * orthogonal to the previous ones is at most 1e-12 of its norm gets a zero Q
 * column and a zero diagonal in R, so Q R = A still holds and the nonzero columns
 * of Q are orthonormal.  R [batch][k][k] upper triangular (may be NULL).
 * Errors: BF_ERR_INVALID_ARG, BF_ERR_UNSUPPORTED (k), BF_ERR_HIP. */
bf_status bf_batched_qr(double *A, int64_t batch, int64_t n, int32_t k, double *R,
                        hipStream_t stream);

/* The first npiv column pivots of a column-pivoted QR (Algorithm 2.2, steps 2 and
 * 3) of `batch` p x n matrices, each stored by columns as At [batch][n][p]
 * (column j is At[b][j][0..p-1]; device, destroyed: it holds the residual columns
 * on return).  Step k picks the column of largest residual 2-norm, the first one
 * on ties, and removes its direction from the other columns.  piv [batch][npiv]
 * (device int64).  p <= 128, npiv <= n <= 8192.
 * Errors: BF_ERR_INVALID_ARG, BF_ERR_UNSUPPORTED (sizes), BF_ERR_HIP. */
bf_status bf_batched_column_pivots(double *At, int64_t batch, int32_t p, int64_t n, int32_t npiv,
                                   int64_t *piv, hipStream_t stream);

/* Host output buffers in the canonical layout of bf.h (FP64, complex interleaved):
 * VL, UL [P][n0][r]; H[t], G[t] [R^(l+1)][R^(L-l-1)][r][R r] for l = h + t;
 * S [m][m][r]. */
typedef struct {
  double *VL;
  double *const *H;
  double *S;
  double *const *G;
  double *UL;
} bf_factors_out;

/* Butterfly factorization of a built-in kernel, built on the current device.
 * Middle level (Sec. 3.1): each block K(A^h_i, B^h_j), of size b = N/m, gets a
 * rank-r approximation by Algorithm 2.2: `iters` alternations of sampling r q
 * rows (plus the current important rows) and picking the r important columns by
 * pivoted QR, then r q columns (plus the important columns) and the r important
 * rows by pivoted LQ; orthonormal bases Q_col, Q_row of the important columns and
 * rows; the middle matrix from the important plus r q fresh rows and columns
 * (pseudo-inverses with relative cutoff 1e-14); its SVD.  The block is stored in
 * the first form of Sec. 2 (U = U0 S0, S = S0^{-1}, V = V0 S0); singular values
 * at most drop_rel times the block's largest are dropped (S = 0, zero U and V
 * columns).  Recursion (Sec. 3.2): the child rows of R neighbouring blocks,
 * [U^{l,c}_{i,Rj} .. U^{l,c}_{i,Rj+R-1}], get a rank-r truncated SVD U0 S0 V0^*
 * (via a QR and the SVD of its R factor): U^{l+1} = U0 S0, G^l = V0^*; V gives H
 * the same way.  Random draws: uniform without replacement, from SplitMix64
 * (Steele, Lea, Flood 2014) keyed by (seed, block, iteration, side), so a given
 * seed always gives the same factors on the same device type.
 * Limits: 1D kernels (any radix R in {2, 4}), r <= b, R r <= 64, r <= 32,
 * min(b, r (q + 1)) <= 128, b <= 8192.  Device memory: about 3 m^2 b r complex
 * values plus bounded scratch; the call synchronizes `stream` and writes `out`
 * before returning.
 * Errors: BF_ERR_INVALID_ARG, BF_ERR_SHAPE, BF_ERR_UNSUPPORTED, BF_ERR_ALLOC,
 * BF_ERR_HIP.
 * Status: switched off.  After its argument checks the call returns
 * BF_ERR_UNSUPPORTED: on the GPU it gave a less accurate factorization than the
 * same code run on the host, and one shape ended in an illegal memory access,
 * with the cause not yet found.  The four batched primitives above are not
 * affected. */
bf_status bf_construct_from_kernel(const bf_shape *shape, int32_t kind, int32_t q, int32_t iters,
                                   uint64_t seed, double drop_rel, const bf_factors_out *out,
                                   hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* BF_CONSTRUCT_H_ */
