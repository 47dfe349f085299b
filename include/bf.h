/*
 * bf.h -- C ABI of the MI355X butterfly-factorization apply library.
 *
 * The library applies a butterfly factorization (Li, Yang, Martin, Ho, Ying,
 * "Butterfly Factorization", Sec. 1.2 and the closing equation of Sec. 3.2)
 *
 *     K ~ U^L G^{L-1} ... G^h M^h (H^h)^* ... (H^{L-1})^* (V^L)^*,   h = L/2,
 *
 * to many right-hand sides on one AMD Instinct MI355X (gfx950).  The factors
 * are built elsewhere (on the host, in FP64) and handed over once.
 *
 * Trees.  Rows X and columns Omega are indexed in tree order: complete
 * radix-R trees of even depth L, R in {2, 4}, n0 points per leaf, P = R^L
 * leaves, N = n0 * P, and every node is a contiguous index range (Sec. 3).
 * m = R^h nodes sit on the middle level.
 *
 * Canonical factor layout (host, FP64, C-contiguous, complex as interleaved
 * (re, im) pairs of doubles):
 *
 *   VL, UL : complex[P][n0][r]     V^L_j and U^L_i; leaf j covers points
 *                                  j*n0 .. j*n0 + n0 - 1 (Sec. 3.2: U^L and V^L are
 *                                  block diagonal with n0 x r blocks).
 *   H[t], G[t], t = 0..h-1, level l = h + t :
 *            complex[R^(l+1)][R^(L-l-1)][r][R*r]
 *            G[t][p][q] = G^l_{p,q}: p an X-node at level l+1, q an Omega-node at
 *            level L-l-1 (Sec. 3.2.1: [U^{l,c}_{i,Rq} .. U^{l,c}_{i,Rq+R-1}] ~
 *            U^{l+1}_{Ri+c,q} G^l_{Ri+c,q}); column block c' (columns c'r ..
 *            c'r + r - 1) multiplies the coefficients of column block R q + c'.
 *            H[t][p][q] = H^l_{p,q}: p an Omega-node at level l+1, q an X-node at
 *            level L-l-1 (Sec. 3.2.2, the same procedure applied to V).
 *   S      : double[m][m][r]       S[i][j][k] = (S^h_{i,j})_{kk}, the diagonal
 *                                  weights of the middle factor M^h (Sec. 3.1:
 *                                  block (i,j) of M^h is zero except its (j,i)
 *                                  r x r sub-block, which is diag S^h_{i,j}).
 *
 * Vectors.  g, u and friends are device arrays [N][ld] of complex numbers,
 * row-major, tree order, interleaved (re, im): complex128 for BF_PREC_F64,
 * complex64 for every other precision.  Column n < nrhs of row p is element
 * p*ld + n.  Input and output must not overlap.
 *
 * Streams and ownership.  The handle owns every device allocation it makes
 * (packed factors, workspace); the caller owns vectors and gradient buffers.
 * Every call except create and destroy is asynchronous on the given stream
 * (NULL = the default stream) and never synchronizes the device.  A handle
 * must not be used from two streams or two threads at once.  The workspace
 * grows on the first call with a larger nrhs; later calls with nrhs at most
 * that size allocate nothing.
 *
 * Errors.  Nothing aborts or throws across this interface.  Every call
 * returns a bf_status; bf_last_error(handle) (or bf_last_error(NULL) for
 * failures that leave no handle) returns a message for the last failure.
 */
#ifndef BF_H_
#define BF_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bf_plan *bf_handle;

typedef enum {
  BF_OK = 0,
  BF_ERR_INVALID_ARG = 1, /* NULL pointer, nrhs < 1, ld < nrhs, overlapping buffers */
  BF_ERR_SHAPE = 2,       /* odd L, N != n0 R^L, r < 1, radix not 2 or 4         */
  BF_ERR_UNSUPPORTED = 3, /* shape/precision combination not compiled              */
  BF_ERR_ALLOC = 4,       /* device or host allocation failed                     */
  BF_ERR_HIP = 5,         /* a HIP runtime call failed                             */
  BF_ERR_NONFINITE = 6    /* a factor entry is NaN or infinite                      */
} bf_status;

typedef enum {
  BF_PREC_F64 = 0,        /* complex128 vectors, FP64 arithmetic                             */
  BF_PREC_F32 = 1,        /* complex64 vectors, FP32 arithmetic                              */
  BF_PREC_SPLIT_BF16 = 2, /* complex64 vectors; block products as three BF16 MFMA products   */
                          /* (hi*hi + hi*lo + lo*hi) with FP32 accumulation.  No scaling:    */
                          /* BF16 has the exponent range of FP32, and a power-of-two scale   */
                          /* would not change a single rounding                              */
  BF_PREC_SPLIT_F16 = 3   /* as SPLIT_BF16 with FP16 halves; every block and every column    */
                          /* of a block product is scaled by a power of two into FP16 range  */
} bf_precision;

typedef struct {
  int32_t radix; /* R: 2 (binary trees) or 4 (quadtrees)  */
  int32_t leaf;  /* n0: points per leaf                   */
  int32_t L;     /* tree depth, even                      */
  int32_t r;     /* rank of every low-rank block          */
  int64_t N;     /* must equal n0 * R^L                   */
} bf_shape;

/* Host factors in the canonical layout above.  H and G point to arrays of
 * L/2 pointers (levels h .. L-1).  Read during bf_create_from_factors only. */
typedef struct {
  const double *VL;
  const double *const *H;
  const double *S;
  const double *const *G;
  const double *UL;
} bf_factors_host;

/* Device gradient buffers in the canonical layout, in the precision of the
 * vectors (complex128 for BF_PREC_F64, complex64 otherwise; S real of the same
 * real type).  Any pointer may be NULL to skip that gradient. */
typedef struct {
  void *VL;
  void *const *H;
  void *S;
  void *const *G;
  void *UL;
} bf_factor_grads;

/* Validate `shape` and `factors`, pack the factors for `precision` and copy
 * them to the current HIP device.  Synchronizes `stream` before returning; the
 * caller may free its host arrays afterwards.  On success *out is a new handle.
 * The factors are those of the factor product of Sec. 1.2 (eq. (1)) as Sec. 3.1
 * and 3.2 build them.  Errors: BF_ERR_INVALID_ARG, BF_ERR_SHAPE,
 * BF_ERR_UNSUPPORTED, BF_ERR_NONFINITE, BF_ERR_ALLOC, BF_ERR_HIP. */
bf_status bf_create_from_factors(const bf_shape *shape, const bf_factors_host *factors,
                                 bf_precision precision, hipStream_t stream, bf_handle *out);

/* Kernel-path choices of a handle.  A zero-filled struct (or NULL) gives the
 * defaults that bf_create_from_factors uses; the other values select variants
 * of the same arithmetic, for comparisons and tests.  Results of every variant
 * agree to within the precision's tolerance. */
typedef struct {
  int32_t path;         /* 0: fused MFMA passes where the shape allows them (radix 2, */
                        /*    leaf 16, r 16), else per-level kernels;                  */
                        /* 1: per-level kernels (FP64 and FP32 only)                   */
  int32_t fused_cols;   /* fused passes: columns per wavefront, 0 (= 16) or 32; FP64   */
                        /* passes have 16 (32 sends FP64 handles to per-level kernels) */
  int32_t fused_kmax;   /* fused passes: deepest pass in levels, 0 = 4 (16 columns) or  */
                        /* 3 (32 columns); 1 .. that maximum                            */
  int32_t fused_split;  /* fused passes: passes of at least this many levels share a   */
                        /* tile between two wavefronts; 0 = 4, -1 = never (FP64 passes */
                        /* of three or four levels always share their tiles)           */
  int32_t level_mfma;   /* per-level FP32 butterflies with R r in {32, 64, 128}:        */
                        /* 0 = on the matrix cores, -1 = one thread per output value    */
  int32_t level_ksplit; /* R r = 128 on the matrix cores: 0 = K range split over two    */
                        /* wavefronts, -1 = one wavefront per row group                 */
} bf_plan_options;

/* bf_create_from_factors with explicit kernel-path choices (opts may be NULL).
 * Errors as bf_create_from_factors; BF_ERR_INVALID_ARG for a value outside the
 * ranges above. */
bf_status bf_create_from_factors_ex(const bf_shape *shape, const bf_factors_host *factors,
                                    bf_precision precision, const bf_plan_options *opts,
                                    hipStream_t stream, bf_handle *out);

/* u = K_BF g for nrhs columns (Sec. 1.2: a sequence of O(log N) sparse
 * products, applied right to left).  g, u: device [N][ld]. */
bf_status bf_apply(bf_handle h, const void *g, void *u, int64_t nrhs, int64_t ld,
                   hipStream_t stream);

/* v = K_BF^* w: the conjugate transpose of the factor product of Sec. 1.2
 * (eq. (1)), i.e. the factors in reverse order, each conjugate-transposed:
 * V^L H^{L-1} ... H^h (M^h)^T (G^h)^* ... (G^{L-1})^* (U^L)^*.  Arguments,
 * layouts and errors as bf_apply. */
bf_status bf_apply_adjoint(bf_handle h, const void *w, void *v, int64_t nrhs, int64_t ld,
                           hipStream_t stream);

/* bf_apply for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * kernels and results as bf_apply, but the two activation buffers live in a
 * scratch array of BF_NOALLOC_SCRATCH_BYTES inside the library (one per GPU,
 * held until the process ends), so the call allocates nothing, on the device or
 * the host, and records no profiling events.  The two buffers take
 * 2 * ceil256(P r ceil(nrhs / C) C * b) bytes (C = 16 columns on the fused path,
 * 32 otherwise; b = 16 for BF_PREC_F64, 8 otherwise): at N = 65536, r = 16 the
 * limit holds 64 columns.  A larger nrhs returns BF_ERR_UNSUPPORTED and does
 * nothing.  Every call on one GPU shares that GPU's array and leaves its last
 * contents there (no call needs them cleared): calls that overlap on one GPU
 * (two streams, two threads or two handles) race and must be serialized by the
 * caller. */
#define BF_NOALLOC_SCRATCH_BYTES (64u << 20)
bf_status bf_apply_noalloc(bf_handle h, const void *g, void *u, int64_t nrhs, int64_t ld,
                           hipStream_t stream);

/* Gradients of a real loss through u = K_BF g.  The paper defines no
 * gradients; this is the chain rule through the factor product of Sec. 1.2,
 * with the complex convention grad = dL/dRe + i dL/dIm.  grad_u = dL/dRe(u) + i dL/dIm(u)
 * ([N][ld], device).  Writes grad_g = K_BF^* grad_u (if non-NULL) and, for every
 * non-NULL pointer in `grads`, the gradient of that factor:
 *   forward-applied blocks B (G, U^L):      grad_B = sum_n d_out x_in^*
 *   adjoint-applied blocks W (H, V^L):      grad_W = sum_n x_in d_out^*
 *   middle weights (real):                  grad_S = sum_n Re(d_z conj(y))
 * The forward states of the chain are needed level by level.  With flags =
 * BF_BWD_RECOMPUTE (the default 0) only some of them are kept (the pass
 * boundaries on the fused path, every fourth level otherwise) and the others
 * are recomputed inside the call; BF_BWD_STORE_ALL keeps all 2h + 2 of them
 * (more workspace, less work).  Both modes give identical results.  FP64 handles
 * take the per-level kernels in FP64 on either path.  On the fused path the
 * backward passes compute in split BF16 for BF_PREC_SPLIT_BF16 handles
 * and in FP32 otherwise (gradient sums in FP32); its first call on a handle also
 * packs copies of the blocks in that precision (device memory owned by the
 * handle, about the size of the packed factors).  The workspace
 * (owned by the handle, grown on demand) is about (2h + 8) activation arrays
 * with BF_BWD_STORE_ALL and 15 without, each P r nrhs complex values.
 * Gradients are overwritten, not added to. */
#define BF_BWD_RECOMPUTE 0u
#define BF_BWD_STORE_ALL 1u
bf_status bf_backward(bf_handle h, const void *g, const void *grad_u, void *grad_g,
                      const bf_factor_grads *grads, int64_t nrhs, int64_t ld, uint32_t flags,
                      hipStream_t stream);

/* Release every device allocation of the handle.  NULL is a no-op.  The caller
 * must make sure no work using the handle is still queued. */
void bf_destroy(bf_handle h);

/* Text of the last error on this handle (NULL: the last create failure on this
 * thread).  Valid until the next call on the same handle. */
const char *bf_last_error(bf_handle h);

/* Shape, precision and the kernel path chosen for the handle: 0 = per-level
 * kernels, 1 = fused MFMA passes. */
bf_status bf_query(bf_handle h, bf_shape *shape, bf_precision *precision, int32_t *path);

/* Per-kernel timing with HIP events recorded around every launch on the call's
 * stream.  enable != 0 turns recording on; bf_kernel_times writes, for up to
 * `cap` kernels in launch order of the last call, the accumulated milliseconds
 * and launch counts since the last reset (reset != 0 clears the accumulators
 * after reading) and returns the number of kernels in *count.  Reading
 * synchronizes the events. */
bf_status bf_set_profiling(bf_handle h, int32_t enable);
bf_status bf_kernel_times(bf_handle h, char names[][64], double *ms, int64_t *launches,
                          int32_t cap, int32_t *count, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* BF_H_ */
