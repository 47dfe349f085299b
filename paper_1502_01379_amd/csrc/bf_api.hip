// Host side of the C ABI declared in include/bf.h: argument checking, upload of
// the factors, the order of the factor products, the backward drivers (fused
// passes with per-depth copies, or per-level kernels), workspace and profiling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "bf_internal.h"

using bfly::LevelOp;

namespace {

thread_local std::string g_create_error;

#define BF_TRY_HIP(expr)                                                            \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      set_err(p, std::string(#expr) + ": " + hipGetErrorString(e_));                \
      return e_ == hipErrorOutOfMemory ? BF_ERR_ALLOC : BF_ERR_HIP;                 \
    }                                                                               \
  } while (0)

void set_err(bf_plan *p, const std::string &msg) {
  if (p)
    p->err = msg;
  else
    g_create_error = msg;
}

bf_status fail(bf_plan *p, bf_status st, const std::string &msg) {
  set_err(p, msg);
  return st;
}

int64_t ipow(int64_t b, int e) {
  int64_t v = 1;
  for (int i = 0; i < e; ++i) v *= b;
  return v;
}

bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb) {
  const char *pa = (const char *)a, *pb = (const char *)b;
  return pa < pb + nb && pb < pa + na;
}

size_t cplx_bytes(bf_precision prec) { return prec == BF_PREC_F64 ? 16 : 8; }

bf_status check_shape(const bf_shape *s, bf_plan *p) {
  if (!s) return fail(p, BF_ERR_INVALID_ARG, "shape is NULL");
  if (s->radix != 2 && s->radix != 4) return fail(p, BF_ERR_SHAPE, "radix must be 2 or 4");
  if (s->leaf < 1) return fail(p, BF_ERR_SHAPE, "leaf size must be >= 1");
  if (s->r < 1) return fail(p, BF_ERR_SHAPE, "rank r must be >= 1");
  if (s->L < 2 || (s->L % 2) != 0) return fail(p, BF_ERR_SHAPE, "tree depth L must be even and >= 2");
  if (s->L * (s->radix == 4 ? 2 : 1) > 40) return fail(p, BF_ERR_SHAPE, "tree too deep");
  const int64_t P = ipow(s->radix, s->L);
  if ((int64_t)s->leaf * P != s->N) return fail(p, BF_ERR_SHAPE, "N must equal leaf * radix^L");
  if (P * (int64_t)s->r * s->radix * s->r > (int64_t(1) << 40))
    return fail(p, BF_ERR_SHAPE, "factorization too large");
  return BF_OK;
}

// Convert a canonical FP64 complex array to the compute precision and upload it.
template <class T>
bf_status upload_array(bf_plan *p, const double *src, size_t nreal, void **dst) {
  void *d = nullptr;
  BF_TRY_HIP(hipMalloc(&d, nreal * sizeof(T)));
  p->allocs.push_back(d);
  if (sizeof(T) == sizeof(double)) {
    BF_TRY_HIP(hipMemcpy(d, src, nreal * sizeof(double), hipMemcpyHostToDevice));
  } else {
    const size_t blk = size_t(1) << 24;
    std::vector<T> tmp(std::min(nreal, blk));
    for (size_t o = 0; o < nreal; o += blk) {
      const size_t n = std::min(blk, nreal - o);
      for (size_t i = 0; i < n; ++i) tmp[i] = (T)src[o + i];
      BF_TRY_HIP(hipMemcpy((char *)d + o * sizeof(T), tmp.data(), n * sizeof(T),
                           hipMemcpyHostToDevice));
    }
  }
  *dst = d;
  return BF_OK;
}

bool all_finite(const double *a, size_t n) {
  const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < (size_t(1) << 22) || nt == 1) {
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(a[i])) return false;
    return true;
  }
  std::vector<char> ok(nt, 1);
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      const size_t lo = n * t / nt, hi = n * (t + 1) / nt;
      for (size_t i = lo; i < hi; ++i)
        if (!std::isfinite(a[i])) {
          ok[t] = 0;
          return;
        }
    });
  for (auto &x : th) x.join();
  for (char c : ok)
    if (!c) return false;
  return true;
}

// Device copies of the canonical factors, in compute precision.
struct Canon {
  void *VL = nullptr, *UL = nullptr, *S = nullptr;
  std::vector<void *> H, G;
};

template <class T>
bf_status upload_canonical(bf_plan *p, const bf_factors_host *f, Canon &c) {
  const size_t leaf_n = (size_t)p->P * p->n0 * p->r * 2;
  const size_t lvl_n = (size_t)p->P * p->R * p->r * p->r * 2;
  bf_status st;
  if ((st = upload_array<T>(p, f->VL, leaf_n, &c.VL)) != BF_OK) return st;
  if ((st = upload_array<T>(p, f->UL, leaf_n, &c.UL)) != BF_OK) return st;
  if ((st = upload_array<T>(p, f->S, (size_t)p->m * p->m * p->r, &c.S)) != BF_OK) return st;
  for (int t = 0; t < p->h; ++t) {
    void *dh = nullptr, *dg = nullptr;
    if ((st = upload_array<T>(p, f->H[t], lvl_n, &dh)) != BF_OK) return st;
    if ((st = upload_array<T>(p, f->G[t], lvl_n, &dg)) != BF_OK) return st;
    c.H.push_back(dh);
    c.G.push_back(dg);
  }
  return BF_OK;
}

// The factor product in application order.
//   forward: (V^L)^*, (H^{L-1})^* .. (H^h)^*, M^h, G^h .. G^{L-1}, U^L
//   adjoint: (U^L)^*, (G^{L-1})^* .. (G^h)^*, (M^h)^*, H^h .. H^{L-1}, V^L
void build_ops(bf_plan *p, const Canon &c) {
  const int R = p->R, L = p->L, h = p->h;
  auto lvl = [&](const void *arr, int l, bfly::SlotMode mode, bool tconj, const char *nm) {
    LevelOp op;
    op.kind = LevelOp::kButterfly;
    op.mode = mode;
    op.nb = p->P / R;
    op.blo = ipow(R, L - l - 1);
    op.tconj = tconj;
    op.mat = arr;
    op.level = l;
    op.name = std::string(nm) + std::to_string(l);
    return op;
  };
  auto leaf = [&](LevelOp::Kind k, const void *arr, const char *nm) {
    LevelOp op;
    op.kind = k;
    op.mat = arr;
    op.name = nm;
    return op;
  };
  auto middle = [&](bool transpose) {
    LevelOp op;
    op.kind = LevelOp::kMiddle;
    op.tconj = transpose;
    op.mat = c.S;
    op.name = transpose ? "middle_adj" : "middle";
    return op;
  };
  p->fwd_ops.clear();
  p->adj_ops.clear();
  p->fwd_ops.push_back(leaf(LevelOp::kLeafIn, c.VL, "leaf_in_V"));
  for (int l = L - 1; l >= h; --l) p->fwd_ops.push_back(lvl(c.H[l - h], l, bfly::kStridedIn, true, "H_fwd_"));
  p->fwd_ops.push_back(middle(false));
  for (int l = h; l < L; ++l) p->fwd_ops.push_back(lvl(c.G[l - h], l, bfly::kContigIn, false, "G_fwd_"));
  p->fwd_ops.push_back(leaf(LevelOp::kLeafOut, c.UL, "leaf_out_U"));

  p->adj_ops.push_back(leaf(LevelOp::kLeafIn, c.UL, "leaf_in_U"));
  for (int l = L - 1; l >= h; --l) p->adj_ops.push_back(lvl(c.G[l - h], l, bfly::kStridedIn, true, "G_adj_"));
  p->adj_ops.push_back(middle(true));
  for (int l = h; l < L; ++l) p->adj_ops.push_back(lvl(c.H[l - h], l, bfly::kContigIn, false, "H_adj_"));
  p->adj_ops.push_back(leaf(LevelOp::kLeafOut, c.VL, "leaf_out_V"));
}

bf_status ensure_ws(bf_plan *p, size_t bytes) {
  if (p->ws_bytes >= bytes) return BF_OK;
  if (p->ws) {
    hipError_t e = hipFree(p->ws);
    p->ws = nullptr;
    p->ws_bytes = 0;
    if (e != hipSuccess) return fail(p, BF_ERR_HIP, std::string("hipFree: ") + hipGetErrorString(e));
  }
  void *d = nullptr;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(p, BF_ERR_ALLOC, "workspace allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  p->ws = d;
  p->ws_bytes = bytes;
  return BF_OK;
}

size_t act_bytes(const bf_plan *p, int64_t nrhs) {
  const int64_t nchunks = (nrhs + (int64_t(1) << p->cs) - 1) >> p->cs;
  return (size_t)bfly::act_elems(p->P, p->r, nchunks, p->cs) * cplx_bytes(p->prec);
}

bf_status check_call(bf_plan *p, const void *in, const void *out, int64_t nrhs, int64_t ld) {
  if (!in || !out) return fail(p, BF_ERR_INVALID_ARG, "vector pointer is NULL");
  if (nrhs < 1) return fail(p, BF_ERR_INVALID_ARG, "nrhs must be >= 1");
  if (ld < nrhs) return fail(p, BF_ERR_INVALID_ARG, "ld must be >= nrhs");
  if (nrhs > (int64_t(1) << 24)) return fail(p, BF_ERR_INVALID_ARG, "nrhs too large");
  const size_t span = (size_t)((p->N - 1) * ld + nrhs) * cplx_bytes(p->prec);
  if (ranges_overlap(in, span, out, span)) return fail(p, BF_ERR_INVALID_ARG, "input and output overlap");
  return BF_OK;
}

// The op list through two ping-pong activation buffers of act_bytes(p, nrhs)
// each (buf0 == nullptr: the handle's workspace, grown if needed).
bf_status run_ops(bf_plan *p, const std::vector<LevelOp> &ops, const void *g, void *u,
                  int64_t nrhs, int64_t ld, hipStream_t s, void *buf0 = nullptr, void *buf1 = nullptr) {
  const size_t ab = act_bytes(p, nrhs);
  if (!buf0) {
    bf_status st = ensure_ws(p, 2 * ab);
    if (st != BF_OK) return st;
    buf0 = p->ws;
    buf1 = (char *)p->ws + ab;
  }
  char *buf[2] = {(char *)buf0, (char *)buf1};
  const void *cur = g;
  int which = 0;
  for (size_t t = 0; t < ops.size(); ++t) {
    const bool last = t + 1 == ops.size();
    void *out = last ? u : buf[which];
    bfly::prof_begin(p, ops[t].name, s);
    hipError_t e = bfly::launch_level_op(p, ops[t], cur, ld, out, ld, nrhs, s);
    bfly::prof_end(p, s);
    if (e != hipSuccess) return fail(p, BF_ERR_HIP, ops[t].name + ": " + hipGetErrorString(e));
    cur = out;
    which ^= 1;
  }
  return BF_OK;
}

}  // namespace

bf_plan::~bf_plan() {
  for (auto *fp : fwd_passes) bfly::fused_free(fp);
  for (auto *fp : adj_passes) bfly::fused_free(fp);
  for (auto *fp : bwd_fwd) bfly::fused_free(fp);
  for (auto *fp : bwd_adj) bfly::fused_free(fp);
  for (void *d : allocs) (void)hipFree(d);
  if (ws) (void)hipFree(ws);
  for (auto &r : prof_pending) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  for (auto e : event_pool) (void)hipEventDestroy(e);
}

namespace bfly {

void prof_begin(bf_plan *p, const std::string &name, hipStream_t s) {
  if (!p->profiling) return;
  ProfRec r;
  r.name = name;
  for (hipEvent_t *e : {&r.start, &r.stop}) {
    if (!p->event_pool.empty()) {
      *e = p->event_pool.back();
      p->event_pool.pop_back();
    } else if (hipEventCreate(e) != hipSuccess) {
      (void)hipGetLastError();
      return;
    }
  }
  (void)hipEventRecord(r.start, s);
  p->prof_pending.push_back(r);
}

void prof_end(bf_plan *p, hipStream_t s) {
  if (!p->profiling || p->prof_pending.empty()) return;
  (void)hipEventRecord(p->prof_pending.back().stop, s);
}

}  // namespace bfly

namespace {
void prof_drain(bf_plan *p) {
  for (auto &r : p->prof_pending) {
    float ms = 0.f;
    (void)hipEventSynchronize(r.stop);
    if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) {
      (void)hipGetLastError();
      ms = 0.f;
    }
    size_t k = 0;
    while (k < p->prof_names.size() && p->prof_names[k] != r.name) ++k;
    if (k == p->prof_names.size()) {
      p->prof_names.push_back(r.name);
      p->prof_ms.push_back(0.0);
      p->prof_launches.push_back(0);
    }
    p->prof_ms[k] += ms;
    p->prof_launches[k] += 1;
    p->event_pool.push_back(r.start);
    p->event_pool.push_back(r.stop);
  }
  p->prof_pending.clear();
}
}  // namespace

namespace bfly {
void set_create_error(const std::string &msg) { g_create_error = msg; }
}  // namespace bfly

extern "C" {

bf_status bf_create_from_factors(const bf_shape *shape, const bf_factors_host *f,
                                 bf_precision prec, hipStream_t stream, bf_handle *out) {
  return bf_create_from_factors_ex(shape, f, prec, nullptr, stream, out);
}

bf_status bf_create_from_factors_ex(const bf_shape *shape, const bf_factors_host *f,
                                    bf_precision prec, const bf_plan_options *opts,
                                    hipStream_t stream, bf_handle *out) {
  g_create_error.clear();
  if (!out) return fail(nullptr, BF_ERR_INVALID_ARG, "out is NULL");
  bf_plan_options opt{};
  if (opts) {
    opt = *opts;
    if (opt.path < 0 || opt.path > 1 || (opt.fused_cols != 0 && opt.fused_cols != 16 && opt.fused_cols != 32) ||
        opt.fused_kmax < 0 || opt.fused_kmax > (opt.fused_cols == 32 ? 3 : 4) || opt.fused_split < -1 ||
        opt.level_mfma < -1 || opt.level_mfma > 0 || opt.level_ksplit < -1 || opt.level_ksplit > 0)
      return fail(nullptr, BF_ERR_INVALID_ARG, "plan option out of range");
  }
  *out = nullptr;
  bf_status st = check_shape(shape, nullptr);
  if (st != BF_OK) return st;
  if (!f || !f->VL || !f->UL || !f->S || !f->H || !f->G)
    return fail(nullptr, BF_ERR_INVALID_ARG, "factor pointer is NULL");
  if (prec < BF_PREC_F64 || prec > BF_PREC_SPLIT_F16)
    return fail(nullptr, BF_ERR_INVALID_ARG, "unknown precision");
  const int h = shape->L / 2;
  for (int t = 0; t < h; ++t)
    if (!f->H[t] || !f->G[t]) return fail(nullptr, BF_ERR_INVALID_ARG, "level factor pointer is NULL");

  bf_plan *p = new (std::nothrow) bf_plan();
  if (!p) return fail(nullptr, BF_ERR_ALLOC, "host allocation failed");
  p->shape = *shape;
  p->prec = prec;
  p->opt = opt;
  p->R = shape->radix;
  p->n0 = shape->leaf;
  p->L = shape->L;
  p->r = shape->r;
  p->h = h;
  p->P = ipow(p->R, p->L);
  p->m = ipow(p->R, h);
  p->N = shape->N;

  const bool fused = bfly::fused_supported(*shape, prec, opt);
  if (!fused && (prec == BF_PREC_SPLIT_BF16 || prec == BF_PREC_SPLIT_F16)) {
    delete p;
    return fail(nullptr, BF_ERR_UNSUPPORTED,
                "split precision needs radix 2, leaf 16, r 16 (the fused MFMA passes)");
  }
  const size_t leaf_n = (size_t)p->P * p->n0 * p->r * 2;
  const size_t lvl_n = (size_t)p->P * p->R * p->r * p->r * 2;
  bool finite = all_finite(f->VL, leaf_n) && all_finite(f->UL, leaf_n) &&
                all_finite(f->S, (size_t)p->m * p->m * p->r);
  for (int t = 0; t < h && finite; ++t) finite = all_finite(f->H[t], lvl_n) && all_finite(f->G[t], lvl_n);
  if (!finite) {
    delete p;
    return fail(nullptr, BF_ERR_NONFINITE, "a factor entry is NaN or infinite");
  }

  Canon c;
  st = prec == BF_PREC_F64 ? upload_canonical<double>(p, f, c) : upload_canonical<float>(p, f, c);
  if (st == BF_OK) {
    p->S = c.S;
    build_ops(p, c);
    if (fused) {
      p->path = 1;
      st = bfly::fused_build(p, f);
    } else if (prec == BF_PREC_F32 && bfly::level_mfma_supported(p->R, p->r) && opt.level_mfma == 0) {
      // butterfly levels on the matrix cores: blocks packed on the device
      for (auto *ops : {&p->fwd_ops, &p->adj_ops})
        for (LevelOp &op : *ops) {
          if (op.kind != LevelOp::kButterfly || st != BF_OK) continue;
          void *d = nullptr;
          const size_t bytes = (size_t)op.nb * (size_t)(p->R * p->r) * (size_t)(2 * p->R * p->r) * 4;
          hipError_t e = hipMalloc(&d, bytes);
          if (e != hipSuccess) {
            (void)hipGetLastError();
            st = fail(p, BF_ERR_ALLOC, std::string("level block allocation: ") + hipGetErrorString(e));
            break;
          }
          p->allocs.push_back(d);
          if ((e = bfly::launch_pack_level_mfma(op, p->R, p->r, d, stream)) != hipSuccess)
            st = fail(p, BF_ERR_HIP, std::string("level block packing: ") + hipGetErrorString(e));
          op.packed = d;
        }
    }
  }
  if (st == BF_OK) {
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) st = fail(p, BF_ERR_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  }
  if (st != BF_OK) {
    g_create_error = p->err;
    delete p;
    return st;
  }
  *out = p;
  return BF_OK;
}

bf_status bf_apply(bf_handle p, const void *g, void *u, int64_t nrhs, int64_t ld, hipStream_t s) {
  if (!p) return fail(nullptr, BF_ERR_INVALID_ARG, "handle is NULL");
  bf_status st = check_call(p, g, u, nrhs, ld);
  if (st != BF_OK) return st;
  if (p->path == 1) {
    const size_t ab = act_bytes(p, nrhs);
    if ((st = ensure_ws(p, 2 * ab)) != BF_OK) return st;
    hipError_t e = bfly::fused_run(p, false, g, u, nrhs, ld, p->ws, (char *)p->ws + ab, s);
    if (e != hipSuccess) return fail(p, BF_ERR_HIP, std::string("fused apply: ") + hipGetErrorString(e));
    return BF_OK;
  }
  return run_ops(p, p->fwd_ops, g, u, nrhs, ld, s);
}

bf_status bf_apply_adjoint(bf_handle p, const void *w, void *v, int64_t nrhs, int64_t ld,
                           hipStream_t s) {
  if (!p) return fail(nullptr, BF_ERR_INVALID_ARG, "handle is NULL");
  bf_status st = check_call(p, w, v, nrhs, ld);
  if (st != BF_OK) return st;
  if (p->path == 1) {
    const size_t ab = act_bytes(p, nrhs);
    if ((st = ensure_ws(p, 2 * ab)) != BF_OK) return st;
    hipError_t e = bfly::fused_run(p, true, w, v, nrhs, ld, p->ws, (char *)p->ws + ab, s);
    if (e != hipSuccess) return fail(p, BF_ERR_HIP, std::string("fused adjoint: ") + hipGetErrorString(e));
    return BF_OK;
  }
  return run_ops(p, p->adj_ops, w, v, nrhs, ld, s);
}

// ---- apply without allocations ------------------------------------------------
//
// bf_apply_noalloc runs the same kernels as bf_apply, with its two ping-pong
// activation buffers in this array instead of the handle's workspace.  The array
// is a per-GPU object of the library's code (each GPU the library runs on holds
// its own copy until the process ends); host code reaches its device address only
// through hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) char scratch[BF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
static bf_status noalloc_scratch(bf_plan *p, void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(p, BF_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(p, BF_ERR_UNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(p, BF_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BF_OK;
}

}  // namespace

bf_status bf_apply_noalloc(bf_handle p, const void *g, void *u, int64_t nrhs, int64_t ld,
                                      hipStream_t s) {
  if (!p) return fail(nullptr, BF_ERR_INVALID_ARG, "handle is NULL");
  bf_status st = check_call(p, g, u, nrhs, ld);
  if (st != BF_OK) return st;
  const size_t ab = act_bytes(p, nrhs);
  // two buffers, each starting on a 256-byte boundary
  const size_t ab_al = (ab + 255) & ~size_t(255);
  if (2 * ab_al > BF_NOALLOC_SCRATCH_BYTES)
    return fail(p, BF_ERR_UNSUPPORTED,
                "bf_apply_noalloc: " + std::to_string(nrhs) + " columns need " + std::to_string(2 * ab_al) +
                    " bytes of scratch, more than its " + std::to_string((size_t)BF_NOALLOC_SCRATCH_BYTES) +
                    " bytes; use bf_apply or fewer columns per call");
  void *base = nullptr;
  if ((st = noalloc_scratch(p, &base)) != BF_OK) return st;
  void *buf0 = base, *buf1 = (char *)base + ab_al;
  // no profiling events: recording them may create events
  const bool prof = p->profiling;
  p->profiling = false;
  if (p->path == 1) {
    hipError_t e = bfly::fused_run(p, false, g, u, nrhs, ld, buf0, buf1, s);
    if (e != hipSuccess) st = fail(p, BF_ERR_HIP, std::string("fused apply: ") + hipGetErrorString(e));
  } else {
    st = run_ops(p, p->fwd_ops, g, u, nrhs, ld, s, buf0, buf1);
  }
  p->profiling = prof;
  return st;
}

// Backward pass.  The forward chain is a_0 = (V^L)^* g, a_t = op_t(a_{t-1}) for
// t = 1 .. 2h+1 (H levels, middle, G levels), u = U^L a_{2h+1}.  Going back, the
// gradient of op_t needs its input a_{t-1} and the incoming delta_t (the
// gradient with respect to a_t); delta_{t-1} is the adjoint of op_t applied to
// delta_t.  The adjoint chain b_{-1} = delta_u, b_k = adj_op_k(b_{k-1}) gives
// b_k = delta_{2h+1-k}.

namespace {

#define BWD_LAUNCH(name, call)                                                                      \
  do {                                                                                              \
    bfly::prof_begin(p, name, s);                                                                   \
    hipError_t e_ = (call);                                                                         \
    bfly::prof_end(p, s);                                                                           \
    if (e_ != hipSuccess) return fail(p, BF_ERR_HIP, std::string(name) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Fused-path handles: the forward and the adjoint chains run as the apply's
// multi-level passes (FP32) that also leave a copy of the state after every
// level; the block gradients are MFMA contractions of those copies.  With
// BF_BWD_STORE_ALL every a_t is kept; otherwise only the pass boundaries are
// kept and, before each adjoint pass, the forward pass it mirrors runs again to
// restore the states between them.  The b_k live in a ring of six buffers: an
// adjoint pass reads one and writes at most five, and the gradients of the
// levels it mirrors are taken before the next pass.
static bf_status backward_fused(bf_plan *p, const void *g, const void *grad_u, void *grad_g,
                         const bf_factor_grads *grads, int64_t nrhs, int64_t ld, bool store_all,
                         hipStream_t s) {
  bf_status st;
  if (!p->bwd_ready && (st = bfly::fused_build_backward(p, s)) != BF_OK) return st;
  const int h = p->h, nact = 2 * h + 2;
  const auto &F = p->fwd_ops;
  const auto &FP = p->bwd_fwd, &AP = p->bwd_adj;
  const int np = (int)FP.size();
  // pass j reads a_{tin[j]} (-1: the user vector) and leaves a_{td0[j] + d} after d levels
  auto positions = [&](const std::vector<bfly::FusedPass *> &list, std::vector<int> &tin,
                       std::vector<int> &td0) {
    int t = -1;
    for (const auto *fp : list) {
      const bfly::PassShape sh = bfly::fused_pass_shape(fp);
      tin.push_back(t);
      td0.push_back((sh.li || sh.mid) ? t + 1 : t);
      t = td0.back() + sh.K;
    }
    return t;
  };
  std::vector<int> tin, td0, tinb, td0b;
  if (positions(FP, tin, td0) != nact - 1 || positions(AP, tinb, td0b) != nact - 1)
    return fail(p, BF_ERR_UNSUPPORTED, "backward pass plan does not cover the chain");
  // buffers: kept a_t, the states inside one pass (recompute), the b ring, and the
  // leaf-out result when grad_g is not wanted
  std::vector<int> abuf(nact, -1);
  int nb = 0;
  for (int j = 0; j < np; ++j) {
    const bfly::PassShape sh = bfly::fused_pass_shape(FP[j]);
    for (int d = 0; d <= sh.K; ++d) {
      const int t = td0[j] + d;
      if (t < 0 || abuf[t] >= 0) continue;
      if (store_all || d == sh.K || (d == 0 && (sh.li || sh.mid))) abuf[t] = nb++;
    }
  }
  const int seg0 = nb;
  if (!store_all) nb += 3;  // depths 1 .. K-1 of one pass, K <= 4
  const int ring0 = nb;
  nb += 6;
  const size_t ab = act_bytes(p, nrhs);
  const size_t user_bytes = (size_t)((p->N - 1) * ld + nrhs) * 8;
  if ((st = ensure_ws(p, (size_t)nb * ab + (grad_g ? 0 : user_bytes))) != BF_OK) return st;
  char *const ws = static_cast<char *>(p->ws);
  auto buf = [&](int i) { return static_cast<void *>(ws + (size_t)i * ab); };
  std::vector<void *> aptr(nact, nullptr);
  for (int t = 0; t < nact; ++t)
    if (abuf[t] >= 0) aptr[t] = buf(abuf[t]);
  auto bptr = [&](int k) { return buf(ring0 + k % 6); };
  void *gout = grad_g ? grad_g : static_cast<void *>(ws + (size_t)nb * ab);

  // forward pass j with copies of the states that have a buffer; a second run of a
  // pass (recompute) only restores the states strictly inside it
  auto run_forward = [&](int j, bool again) -> bf_status {
    const bfly::PassShape sh = bfly::fused_pass_shape(FP[j]);
    if (again && sh.K == 1) return BF_OK;  // no state strictly inside a one-level pass
    void *lvl[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    for (int d = (!again && (sh.li || sh.mid)) ? 0 : 1; d < sh.K; ++d) lvl[d] = aptr[td0[j] + d];
    const void *in = tin[j] < 0 ? g : aptr[tin[j]];
    void *out = again ? nullptr : aptr[td0[j] + sh.K];
    BWD_LAUNCH((*sh.name + (again ? "_recompute" : "")).c_str(),
               bfly::fused_run_pass(p, FP[j], in, out, lvl, nrhs, ld, s));
    return BF_OK;
  };
  // recompute mode: the last forward pass leaves the states inside it in the
  // buffers the recomputation would fill, so the first adjoint pass needs no
  // second run of it
  if (!store_all && np > 0) {
    const bfly::PassShape sl = bfly::fused_pass_shape(FP[np - 1]);
    for (int d = 1; d < sl.K; ++d) aptr[td0[np - 1] + d] = buf(seg0 + d - 1);
  }
  for (int j = 0; j < np; ++j)
    if ((st = run_forward(j, false)) != BF_OK) return st;

  // U^L: grad_UL = sum delta_u a_{2h+1}^*
  if (grads && grads->UL)
    BWD_LAUNCH("grad_UL", bfly::launch_grad_leaf_mfma(p, grad_u, ld, aptr[nact - 1], grads->UL, nrhs, s));

  for (int i = 0; i < np; ++i) {
    const int j = np - 1 - i;  // the forward pass over the same levels
    const bfly::PassShape fs = bfly::fused_pass_shape(FP[j]);
    if (!store_all && j != np - 1) {
      for (int d = 1; d < fs.K; ++d) aptr[td0[j] + d] = buf(seg0 + d - 1);
      if ((st = run_forward(j, true)) != BF_OK) return st;
    }
    const bfly::PassShape as = bfly::fused_pass_shape(AP[i]);
    void *lvl[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    for (int d = (as.li || as.mid) ? 0 : 1; d < as.K; ++d) lvl[d] = bptr(td0b[i] + d);
    if (as.lo) lvl[as.K] = bptr(td0b[i] + as.K);
    const void *in = tinb[i] < 0 ? grad_u : bptr(tinb[i]);
    void *out = as.lo ? gout : bptr(td0b[i] + as.K);
    BWD_LAUNCH(as.name->c_str(), bfly::fused_run_pass(p, AP[i], in, out, lvl, nrhs, ld, s));
    // gradients of the ops of forward pass j
    for (int t = td0[j] + ((fs.li || fs.mid) ? 0 : 1); t <= td0[j] + fs.K; ++t) {
      void *dout = bptr(2 * h + 1 - t);
      if (t == 0) {
        if (grads && grads->VL) BWD_LAUNCH("grad_VL", bfly::launch_grad_leaf_mfma(p, g, ld, dout, grads->VL, nrhs, s));
      } else if (t == h + 1) {
        if (grads && grads->S) BWD_LAUNCH("grad_S", bfly::launch_grad_middle(p, dout, aptr[h], grads->S, nrhs, s));
      } else {
        const bfly::LevelOp &op = F[t];
        const bool is_g = t > h + 1;
        void *const *arr = grads ? (is_g ? grads->G : grads->H) : nullptr;
        void *dst = arr ? arr[op.level - h] : nullptr;
        if (!dst) continue;
        const void *xin = aptr[t - 1];
        if (is_g)
          BWD_LAUNCH("grad_G", bfly::launch_grad_level_mfma(p, op, dout, xin, dst, nrhs, s));
        else
          BWD_LAUNCH("grad_H", bfly::launch_grad_level_mfma(p, op, xin, dout, dst, nrhs, s));
      }
    }
  }
  return BF_OK;
}

}  // namespace

bf_status bf_backward(bf_handle p, const void *g, const void *grad_u, void *grad_g,
                      const bf_factor_grads *grads, int64_t nrhs, int64_t ld, uint32_t flags,
                      hipStream_t s) {
  if (!p) return fail(nullptr, BF_ERR_INVALID_ARG, "handle is NULL");
  bf_status st = check_call(p, g, grad_u, nrhs, ld);
  if (st != BF_OK) return st;
  if (grad_g) {
    const size_t span = (size_t)((p->N - 1) * ld + nrhs) * cplx_bytes(p->prec);
    if (ranges_overlap(grad_g, span, grad_u, span) || ranges_overlap(grad_g, span, g, span))
      return fail(p, BF_ERR_INVALID_ARG, "grad_g overlaps an input");
  }
  if (flags & ~BF_BWD_STORE_ALL) return fail(p, BF_ERR_INVALID_ARG, "unknown flags");
  const bool store_all = (flags & BF_BWD_STORE_ALL) != 0;
  // FP64 handles take the per-level backward on either path
  if (p->path == 1 && p->cs == 4 && p->prec != BF_PREC_F64)
    return backward_fused(p, g, grad_u, grad_g, grads, nrhs, ld, store_all, s);

  // per-level kernels: the forward chain level by level, every kc-th activation
  // kept (all of them with BF_BWD_STORE_ALL) and the ones between recomputed when
  // their segment is reached
  const int h = p->h;
  const int nact = 2 * h + 2;          // a_0 .. a_{2h+1}
  const int kc = store_all ? 1 : 4;    // checkpoint spacing
  const int nckpt = (nact + kc - 1) / kc;
  const int nseg = store_all ? 0 : kc - 1;
  const size_t ab = act_bytes(p, nrhs);
  const int nbuf = nckpt + nseg + 2;
  if ((st = ensure_ws(p, (size_t)nbuf * ab)) != BF_OK) return st;
  auto bufp = [&](int i) { return (char *)p->ws + (size_t)i * ab; };
  auto ckpt = [&](int t) { return bufp(t / kc); };         // t % kc == 0
  char *seg0 = bufp(nckpt);                                 // kc - 1 buffers
  char *dbuf[2] = {bufp(nckpt + nseg), bufp(nckpt + nseg + 1)};
  const auto &F = p->fwd_ops;   // F[0] leaf_in, F[1..2h+1], F[2h+2] leaf_out
  const auto &A = p->adj_ops;   // A[0] leaf_in(U^*), A[k] adjoint of F[2h+2-k]
  auto run_op = [&](bool adj, int t, const void *in, void *out) -> hipError_t {
    return bfly::launch_level_op(p, adj ? A[t] : F[t], in, ld, out, ld, nrhs, s);
  };

  // forward sweep keeping checkpoints
  {
    const void *cur = g;
    char *scratch[2] = {seg0, nseg >= 2 ? seg0 + ab : dbuf[0]};
    for (int t = 0; t < nact; ++t) {
      char *dst = (t % kc == 0) ? ckpt(t) : scratch[t & 1];
      BWD_LAUNCH(F[t].name.c_str(), run_op(false, t, cur, dst));
      cur = dst;
    }
  }
  int seg_base = -1;  // segment currently held in seg buffers
  auto act = [&](int t) -> const void * {
    if (t % kc == 0) return ckpt(t);
    return seg0 + (size_t)((t % kc) - 1) * ab;
  };
  auto ensure_seg = [&](int t) -> hipError_t {
    const int base = (t / kc) * kc;
    if (t % kc == 0 || base == seg_base) return hipSuccess;
    const void *cur = ckpt(base);
    for (int q = base + 1; q < std::min(base + kc, nact); ++q) {
      char *dst = seg0 + (size_t)((q % kc) - 1) * ab;
      bfly::prof_begin(p, F[q].name + "_recompute", s);
      hipError_t e2 = run_op(false, q, cur, dst);
      bfly::prof_end(p, s);
      if (e2 != hipSuccess) return e2;
      cur = dst;
    }
    seg_base = base;
    return hipSuccess;
  };

  hipError_t e;
  const int T = nact - 1;  // index of a_{2h+1}
  // U^L: grad_UL = sum delta_u a_T^*, delta_T = (U^L)^* delta_u
  if ((e = ensure_seg(T)) != hipSuccess) return fail(p, BF_ERR_HIP, std::string("recompute: ") + hipGetErrorString(e));
  if (grads && grads->UL) BWD_LAUNCH("grad_UL", bfly::launch_leaf_grad(p, grad_u, ld, act(T), grads->UL, nrhs, s));
  int cur_d = 0;
  BWD_LAUNCH(A[0].name.c_str(), run_op(true, 0, grad_u, dbuf[cur_d]));
  for (int t = T; t >= 1; --t) {
    if ((e = ensure_seg(t - 1)) != hipSuccess) return fail(p, BF_ERR_HIP, std::string("recompute: ") + hipGetErrorString(e));
    const LevelOp &op = F[t];
    const void *xin = act(t - 1);
    const void *dout = dbuf[cur_d];
    if (op.kind == LevelOp::kMiddle) {
      if (grads && grads->S) BWD_LAUNCH("grad_S", bfly::launch_middle_grad(p, dout, xin, grads->S, nrhs, s));
    } else {
      const bool is_g = t > h + 1;
      void *dst = nullptr;
      if (grads) {
        void *const *arr = is_g ? grads->G : grads->H;
        if (arr) dst = arr[op.level - h];
      }
      if (dst) {
        if (is_g)
          BWD_LAUNCH("grad_G", bfly::launch_level_grad(p, op, dout, xin, dst, nrhs, s));
        else
          BWD_LAUNCH("grad_H", bfly::launch_level_grad(p, op, xin, dout, dst, nrhs, s));
      }
    }
    const LevelOp &aop = A[nact - t];
    BWD_LAUNCH(aop.name.c_str(), run_op(true, nact - t, dout, dbuf[cur_d ^ 1]));
    cur_d ^= 1;
  }
  // V^L: grad_VL = sum g delta_0^*, grad_g = V^L delta_0
  if (grads && grads->VL) BWD_LAUNCH("grad_VL", bfly::launch_leaf_grad(p, g, ld, dbuf[cur_d], grads->VL, nrhs, s));
  if (grad_g) BWD_LAUNCH(A[nact].name.c_str(), run_op(true, nact, dbuf[cur_d], grad_g));
  return BF_OK;
}
#undef BWD_LAUNCH

void bf_destroy(bf_handle p) { delete p; }

const char *bf_last_error(bf_handle p) { return p ? p->err.c_str() : g_create_error.c_str(); }

bf_status bf_query(bf_handle p, bf_shape *shape, bf_precision *precision, int32_t *path) {
  if (!p) return fail(nullptr, BF_ERR_INVALID_ARG, "handle is NULL");
  if (shape) *shape = p->shape;
  if (precision) *precision = p->prec;
  if (path) *path = p->path;
  return BF_OK;
}

bf_status bf_set_profiling(bf_handle p, int32_t enable) {
  if (!p) return fail(nullptr, BF_ERR_INVALID_ARG, "handle is NULL");
  p->profiling = enable != 0;
  return BF_OK;
}

bf_status bf_kernel_times(bf_handle p, char names[][64], double *ms, int64_t *launches,
                          int32_t cap, int32_t *count, int32_t reset) {
  if (!p) return fail(nullptr, BF_ERR_INVALID_ARG, "handle is NULL");
  prof_drain(p);
  const int32_t n = (int32_t)p->prof_names.size();
  for (int32_t k = 0; k < n && k < cap; ++k) {
    if (names) {
      std::strncpy(names[k], p->prof_names[k].c_str(), 63);
      names[k][63] = 0;
    }
    if (ms) ms[k] = p->prof_ms[k];
    if (launches) launches[k] = p->prof_launches[k];
  }
  if (count) *count = n;
  if (reset) {
    p->prof_names.clear();
    p->prof_ms.clear();
    p->prof_launches.clear();
  }
  return BF_OK;
}

}  // extern "C"
