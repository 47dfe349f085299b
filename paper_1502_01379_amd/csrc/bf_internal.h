// Internal declarations shared by the host side and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "bf.h"

namespace bfly {

// Activation layout used by every kernel between launches: right-hand sides are
// grouped in chunks of C = 2^cs columns (C = 32 or 16: the columns one
// wavefront of the fused kernels owns); a chunk holds, for every slot, its r
// rows in pairs, each pair stored as C columns of two interleaved complex
// values (16 bytes per column in FP32):
//   element (slot, row, n) -> ((n / C * nslots + slot) * ceil(r/2) + row / 2) * 2C
//                             + (n % C) * 2 + row % 2
// nslots = R^L at every level of the tree (R^l nodes of one tree times R^(L-l)
// nodes of the other).
inline int64_t act_elems(int64_t nslots, int r, int64_t nchunks, int cs) {
  return nchunks * nslots * ((r + 1) / 2) * (int64_t(2) << cs);
}

// Slot patterns of one butterfly level.  Butterfly b = hi * blo + lo combines R
// input slots and produces R output slots:
//   strided(b, c)    = hi * R * blo + c * blo + lo
//   contiguous(b, c) = hi * R * blo + R * lo + c
// H-side forward and G-side adjoint levels read strided and write contiguous
// slots; G-side forward and H-side adjoint levels do the opposite.
enum SlotMode : int { kStridedIn = 0, kContigIn = 1 };

// One step of the factor product as the per-level kernels see it.
struct LevelOp {
  enum Kind : int { kLeafIn, kButterfly, kMiddle, kLeafOut } kind;
  SlotMode mode = kStridedIn;
  int64_t nb = 0;    // butterflies (kButterfly)
  int64_t blo = 0;   // see SlotMode
  bool tconj = false; // butterfly: conjugate-transposed blocks; middle: transposed S
  const void *mat = nullptr;  // canonical factor array of this op (device)
  const void *packed = nullptr;  // butterfly, FP32: blocks packed for k_level_mfma (or nullptr)
  int level = -1;             // butterfly: tree level l of the factor
  std::string name;
};

struct FusedPass;  // fused MFMA pass description (bf_fused.hip)

// Device packing of the blocks of one K-level FP32 pass from canonical factors.
struct PackDepth {
  const void *Fb = nullptr;  // canonical blocks of the level at this depth
  int log_blo = 0;           // log2 of the level's blo
  int tconj = 0;             // conjugate-transposed blocks
  int contig = 0;            // the level reads contiguous slots
};
struct PackPassArgs {
  PackDepth dep[4];
  int K = 0, log_slo = 0, mode_si = 0;
  int64_t ntiles = 0;
};

struct ProfRec {
  std::string name;
  hipEvent_t start, stop;
};

}  // namespace bfly

struct bf_plan {
  bf_shape shape{};
  bf_precision prec = BF_PREC_F32;
  bf_plan_options opt{};  // kernel-path choices (all zero: defaults)
  int path = 0;  // 0 = per-level kernels, 1 = fused MFMA passes
  int cs = 5;    // log2 of the activation chunk (columns per wavefront of the fused path)
  int R = 2, n0 = 0, L = 0, r = 0, h = 0;
  int64_t P = 0, m = 0, N = 0;

  // device memory owned by the plan
  std::vector<void *> allocs;
  // per-level path: forward and adjoint op lists
  std::vector<bfly::LevelOp> fwd_ops, adj_ops;
  // fused path
  std::vector<bfly::FusedPass *> fwd_passes, adj_passes;
  // fused passes of the backward pass (same pass split as the apply; the forward
  // list stops before the leaf-out blocks), built on first use: split BF16 for
  // split-BF16 handles, FP32 otherwise
  std::vector<bfly::FusedPass *> bwd_fwd, bwd_adj;
  bool bwd_ready = false;
  bool bwd_bf16 = false;
  // middle weights, FP32 or FP64 by precision: S[i][j][k] and its transpose
  void *S = nullptr, *ST = nullptr;

  // workspace: ping-pong activation buffers plus per-level storage for backward
  void *ws = nullptr;
  size_t ws_bytes = 0;

  std::string err;
  bool profiling = false;
  std::vector<bfly::ProfRec> prof_pending;
  std::vector<hipEvent_t> event_pool;
  std::vector<std::string> prof_names;
  std::vector<double> prof_ms;
  std::vector<int64_t> prof_launches;

  ~bf_plan();
};

namespace bfly {

// Launch helpers (bf_simple.hip)
hipError_t launch_level_op(const bf_plan *p, const LevelOp &op, const void *in, int64_t ld_in,
                           void *out, int64_t ld_out, int64_t nrhs, hipStream_t s);
hipError_t launch_level_grad(const bf_plan *p, const LevelOp &op, const void *X, const void *Y,
                             void *grad, int64_t nrhs, hipStream_t s);
hipError_t launch_leaf_grad(const bf_plan *p, const void *user, int64_t ld, const void *act,
                            void *grad, int64_t nrhs, hipStream_t s);
hipError_t launch_middle_grad(const bf_plan *p, const void *dz, const void *y, void *grad,
                              int64_t nrhs, hipStream_t s);

// Per-level butterflies on the matrix cores (bf_level.hip): FP32, R r in {32, 64, 128}, r even
bool level_mfma_supported(int R, int r);
hipError_t launch_pack_level_mfma(const LevelOp &op, int R, int r, void *out, hipStream_t s);
hipError_t launch_level_mfma(const bf_plan *p, const LevelOp &op, const void *in, void *out,
                             int64_t nrhs, hipStream_t s);

// Backward helpers for fused-path handles (bf_bwd.hip)
// split = true: BF16 hi / lo blocks for the split-BF16 passes, else FP32 blocks
hipError_t launch_pack_pass(const PackPassArgs &a, void *out, bool split, hipStream_t s);
hipError_t launch_pack_leaf16(const void *canon_leaf, void *out, int64_t npairs, int K, bool in,
                              bool split, hipStream_t s);
hipError_t launch_grad_level_mfma(const bf_plan *p, const LevelOp &op, const void *X, const void *Y,
                                  void *grad, int64_t nrhs, hipStream_t s);
// middle weights, 16-column activation chunks, r = 16 (FP32)
hipError_t launch_grad_middle(const bf_plan *p, const void *dz, const void *y, void *grad,
                              int64_t nrhs, hipStream_t s);
hipError_t launch_grad_leaf_mfma(const bf_plan *p, const void *user, int64_t ld, const void *act,
                                 void *grad, int64_t nrhs, hipStream_t s);

// Fused path (bf_fused.hip)
bool fused_supported(const bf_shape &sh, bf_precision prec, const bf_plan_options &opt);
// FP32 passes of the backward pass (blocks packed on the device from the
// canonical factors)
bf_status fused_build_backward(bf_plan *p, hipStream_t s);
// Shape of one pass of a pass list: K levels, leaf blocks in front (li), the
// middle weights in front (mid), leaf blocks behind (lo), and its name.
struct PassShape {
  int K;
  bool li, mid, lo;
  const std::string *name;
};
PassShape fused_pass_shape(const FusedPass *fp);
// One pass with optional per-depth copies of the state: lvl[d] (d = 0 .. K,
// nullptr to skip) receives the state after d levels in the activation layout.
hipError_t fused_run_pass(const bf_plan *p, const FusedPass *fp, const void *in, void *out,
                          void *const *lvl, int64_t nrhs, int64_t ld, hipStream_t s);
bf_status fused_build(bf_plan *p, const bf_factors_host *f);
hipError_t fused_run(bf_plan *p, bool adjoint, const void *g, void *u, int64_t nrhs, int64_t ld,
                     void *buf0, void *buf1, hipStream_t s);
void fused_free(FusedPass *fp);

// Message returned by bf_last_error(NULL) on this thread (bf_api.hip)
void set_create_error(const std::string &msg);

// Profiling hooks (bf_api.hip)
void prof_begin(bf_plan *p, const std::string &name, hipStream_t s);
void prof_end(bf_plan *p, hipStream_t s);

}  // namespace bfly
