// Host side of the fused MFMA passes: the pass plan, the packing of every
// 32 x 32 complex block into per-lane MFMA operand order, and the launches.
// Device code: bf_fused_kernel.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "bf_fused_kernel.h"
#include "bf_internal.h"

namespace bfly {

using namespace fused;

namespace {

using cd = std::complex<double>;

inline int row32(int e, int rho) { return rho < 4 ? 4 * e + rho : 8 + 4 * e + (rho - 4); }

inline uint16_t bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
inline float bf16_to_f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
inline uint16_t f16_rne(float x) {
  _Float16 h = (_Float16)x;  // host conversion, round to nearest even
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}
inline float f16_to_f(uint16_t u) {
  _Float16 h;
  std::memcpy(&h, &u, 2);
  return (float)h;
}

// Lay out one 32 x 32 complex block M[o][k] (o = c r + a, k = c' r + b) as the
// per-lane A operands of the block products in bf_fused_kernel.h.  Returns the
// FP16 block scale (1 otherwise).
float pack_block(const cd *M, int prec, int cols, char *dst) {
  // A value of K index (part, c', row) for output row o: [Re M, -Im M]
  auto aval = [&](int o, int part, int cp, int row) {
    const cd v = M[o * 32 + cp * 16 + row];
    return part == 0 ? v.real() : -v.imag();
  };
  if (prec == kF32) {
    float *out = reinterpret_cast<float *>(dst);
    for (int lane = 0; lane < 64; ++lane) {
      if (cols == 32) {
        const int i = lane & 31, e = lane >> 5;
        for (int s = 0; s < 32; ++s)
          out[((s >> 2) * 64 + lane) * 4 + (s & 3)] =
              (float)aval(i, s >> 4, (s >> 3) & 1, row32(e, s & 7));
      } else {
        // 16-column FP32 products use Gauss's three products: Re M and +Im M
        const int i = lane & 15, e = lane >> 4;
        for (int T = 0; T < 2; ++T)
          for (int s = 0; s < 16; ++s) {
            const int f = 16 * T + s;
            const double v = aval(16 * T + i, s >> 3, (s >> 2) & 1, 4 * e + (s & 3));
            out[((f >> 2) * 64 + lane) * 4 + (f & 3)] = (float)((s >> 3) ? -v : v);
          }
      }
    }
    return 1.f;
  }
  double mx = 0;
  for (int e = 0; e < 1024; ++e) mx = std::max(mx, std::max(std::fabs(M[e].real()), std::fabs(M[e].imag())));
  float bscale = 1.f;
  double pre = 1.0;
  if (prec == kF16 && mx > 0) {
    int ex = 0;
    std::frexp(mx, &ex);
    pre = std::ldexp(1.0, -ex);           // block entries scaled into [0.5, 1)
    bscale = (float)std::ldexp(1.0, ex);  // undone on the accumulator
  }
  uint16_t *out = reinterpret_cast<uint16_t *>(dst);
  auto put = [&](int w, int lane, int j, double x) {
    uint16_t h, l;
    const float xf = (float)(x * pre);
    if (prec == kBF16) {
      h = bf16_rne(xf);
      l = bf16_rne(xf - bf16_to_f(h));
    } else {
      h = f16_rne(xf);
      l = f16_rne(xf - f16_to_f(h));
    }
    out[((w * 64) + lane) * 8 + j] = h;
    out[(((4 + w) * 64) + lane) * 8 + j] = l;
  };
  for (int lane = 0; lane < 64; ++lane) {
    if (cols == 32) {
      const int i = lane & 31, e = lane >> 5;
      for (int t = 0; t < 4; ++t)
        for (int j = 0; j < 8; ++j) put(t, lane, j, aval(i, t >> 1, t & 1, row32(e, j)));
    } else {
      const int i = lane & 15, e = lane >> 4;
      for (int T = 0; T < 2; ++T)
        for (int t = 0; t < 2; ++t)
          for (int j = 0; j < 8; ++j) put(2 * T + t, lane, j, aval(16 * T + i, t, j >> 2, 4 * e + (j & 3)));
    }
  }
  return bscale;
}

// A leaf pair for the 16-column geometry: the diagonal 16 x 16 blocks
// M_c[i][k] = M[c r + i][c r + k] of a block-diagonal 32 x 32 block, each as two
// 16-byte pieces per lane (lane i + 16 e, value j = 4 part + rho:
// [Re M_c, -Im M_c][i][(part, 4 e + rho)]): hi and lo halves for the split
// precisions, part 0 and part 1 as floats for FP32.  Returns the FP16 scale.
float pack_leaf16(const cd *M, int prec, char *dst) {
  auto aval = [&](int c, int i, int j, int e) {
    const cd v = M[(c * 16 + i) * 32 + c * 16 + 4 * e + (j & 3)];
    return (j >> 2) == 0 ? v.real() : -v.imag();
  };
  if (prec == kF32) {
    // Gauss's three products (leaf16_f32): Re M_c and +Im M_c
    float *out = reinterpret_cast<float *>(dst);
    for (int c = 0; c < 2; ++c)
      for (int lane = 0; lane < 64; ++lane)
        for (int j = 0; j < 8; ++j) {
          const double v = aval(c, lane & 15, j, lane >> 4);
          out[((c * 2 + (j >> 2)) * 64 + lane) * 4 + (j & 3)] = (float)((j >> 2) ? -v : v);
        }
    return 1.f;
  }
  double mx = 0;
  for (int e = 0; e < 1024; ++e) mx = std::max(mx, std::max(std::fabs(M[e].real()), std::fabs(M[e].imag())));
  float bscale = 1.f;
  double pre = 1.0;
  if (prec == kF16 && mx > 0) {
    int ex = 0;
    std::frexp(mx, &ex);
    pre = std::ldexp(1.0, -ex);
    bscale = (float)std::ldexp(1.0, ex);
  }
  uint16_t *out = reinterpret_cast<uint16_t *>(dst);
  for (int c = 0; c < 2; ++c)
    for (int lane = 0; lane < 64; ++lane)
      for (int j = 0; j < 8; ++j) {
        const float xf = (float)(aval(c, lane & 15, j, lane >> 4) * pre);
        uint16_t h, l;
        if (prec == kBF16) {
          h = bf16_rne(xf);
          l = bf16_rne(xf - bf16_to_f(h));
        } else {
          h = f16_rne(xf);
          l = f16_rne(xf - f16_to_f(h));
        }
        out[((c * 2 + 0) * 64 + lane) * 8 + j] = h;
        out[((c * 2 + 1) * 64 + lane) * 8 + j] = l;
      }
  return bscale;
}

// FP64 block for k_fused_pass_f64 (Gauss's three products): lane i + 16e holds
// M[16T + i][16c' + 4 rho + e] (K step k = 4c' + rho) at double
// (((2T + part) 4 + k / 2) 64 + lane) 2 + k % 2; part 0: Re M, part 1: Im M.
void pack_block64(const cd *M, char *dst) {
  double *out = reinterpret_cast<double *>(dst);
  for (int T = 0; T < 2; ++T)
    for (int part = 0; part < 2; ++part)
      for (int k = 0; k < 8; ++k)
        for (int lane = 0; lane < 64; ++lane) {
          const int i = lane & 15, e = lane >> 4;
          const cd v = M[(16 * T + i) * 32 + 16 * (k >> 2) + 4 * (k & 3) + e];
          out[(((2 * T + part) * 4 + k / 2) * 64 + lane) * 2 + (k & 1)] = part ? v.imag() : v.real();
        }
}

// FP64 leaf pair: the diagonal 16 x 16 blocks M_c[i][k] = M[16c + i][16c + k];
// lane i + 16e holds M_c[i][4 rho + e] at double (((2c + part) 2 + rho / 2) 64 + lane) 2 + rho % 2.
void pack_leaf64(const cd *M, char *dst) {
  double *out = reinterpret_cast<double *>(dst);
  for (int c = 0; c < 2; ++c)
    for (int part = 0; part < 2; ++part)
      for (int rho = 0; rho < 4; ++rho)
        for (int lane = 0; lane < 64; ++lane) {
          const int i = lane & 15, e = lane >> 4;
          const cd v = M[(16 * c + i) * 32 + 16 * c + 4 * rho + e];
          out[(((2 * c + part) * 2 + rho / 2) * 64 + lane) * 2 + (rho & 1)] = part ? v.imag() : v.real();
        }
}

}  // namespace

struct FusedPass {
  int K = 0, cols = 32, log_slo = 0, mode_si = 1, in_kind = kInAct, out_kind = kOutAct;
  bool split = false;  // tile shared by a pair of wavefronts (k_fused_pass_x2)
  int64_t ntiles = 0;
  void *fac = nullptr, *leaf = nullptr;
  float *fscale = nullptr, *lscale = nullptr;
  const float *Sm = nullptr;
  const double *Sm64 = nullptr;  // FP64 passes
  std::string name;
  std::vector<void *> owned;
};

namespace {

struct HostFactors {
  const bf_factors_host *f;
  int L, h;
  // canonical accessors (complex, FP64)
  cd H(int l, int64_t p, int64_t q, int row, int col) const {
    const int64_t blo = int64_t(1) << (L - l - 1);
    const double *b = f->H[l - h] + (((p * blo + q) * kRank + row) * 2 * kRank + col) * 2;
    return cd(b[0], b[1]);
  }
  cd G(int l, int64_t p, int64_t q, int row, int col) const {
    const int64_t blo = int64_t(1) << (L - l - 1);
    const double *b = f->G[l - h] + (((p * blo + q) * kRank + row) * 2 * kRank + col) * 2;
    return cd(b[0], b[1]);
  }
  cd leafV(int64_t j, int p, int a) const {
    const double *b = f->VL + ((j * kRank + p) * kRank + a) * 2;
    return cd(b[0], b[1]);
  }
  cd leafU(int64_t j, int p, int a) const {
    const double *b = f->UL + ((j * kRank + p) * kRank + a) * 2;
    return cd(b[0], b[1]);
  }
};

// Which factor a pass applies.
enum PassSide : int { kHfwd, kGfwd, kGadj, kHadj };

struct PassPlan {
  PassSide side;
  int K, l_hi, l_lo;
  int in_kind, out_kind;
};

// Block of depth d, local butterfly (ap, b) of tile (hi, lo), as M[o][k].
void butterfly_block(const HostFactors &F, const PassPlan &pp, int d, int64_t hi, int64_t lo,
                     int ap, int b, cd *M) {
  const int K = pp.K;
  const int r = kRank;
  if (pp.side == kHfwd) {  // M[c r + a][c' r + b'] = conj(H_l[2j + c'][i][b'][c r + a])
    const int l = pp.l_hi - d - 1;
    const int64_t j = (hi << (K - d - 1)) + ap, i = (lo << d) + b;
    for (int c = 0; c < 2; ++c)
      for (int a = 0; a < r; ++a)
        for (int cp = 0; cp < 2; ++cp)
          for (int bb = 0; bb < r; ++bb)
            M[(c * r + a) * 32 + cp * r + bb] = std::conj(F.H(l, 2 * j + cp, i, bb, c * r + a));
  } else if (pp.side == kGfwd) {  // M[c r + a][c' r + b'] = G_l[2i + c][j][a][c' r + b']
    const int l = pp.l_lo + d;
    const int64_t i = (hi << d) + b, j = (lo << (K - d - 1)) + ap;
    for (int c = 0; c < 2; ++c)
      for (int a = 0; a < r; ++a)
        for (int k = 0; k < 2 * r; ++k) M[(c * r + a) * 32 + k] = F.G(l, 2 * i + c, j, a, k);
  } else if (pp.side == kGadj) {  // M[co r + b'][ci r + a] = conj(G_l[2i + ci][j][a][co r + b'])
    const int l = pp.l_hi - d - 1;
    const int64_t i = (hi << (K - d - 1)) + ap, j = (lo << d) + b;
    for (int co = 0; co < 2; ++co)
      for (int bb = 0; bb < r; ++bb)
        for (int ci = 0; ci < 2; ++ci)
          for (int a = 0; a < r; ++a)
            M[(co * r + bb) * 32 + ci * r + a] = std::conj(F.G(l, 2 * i + ci, j, a, co * r + bb));
  } else {  // kHadj: M[co r + b'][ci r + a] = H_l[2j + co][i][b'][ci r + a]
    const int l = pp.l_lo + d;
    const int64_t j = (hi << d) + b, i = (lo << (K - d - 1)) + ap;
    for (int co = 0; co < 2; ++co)
      for (int bb = 0; bb < r; ++bb)
        for (int k = 0; k < 2 * r; ++k) M[(co * r + bb) * 32 + k] = F.H(l, 2 * j + co, i, bb, k);
  }
}

// Leaf pair (leaves j0, j0 + 1) as a block-diagonal 32 x 32 block.
//   in  (conj-transposed):  M[c r + a][c r + p] = conj(W[j0 + c][p][a])
//   out:                    M[c r + p][c r + a] = W[j0 + c][p][a]
void leaf_block(const HostFactors &F, bool use_v, bool in, int64_t j0, cd *M) {
  std::fill(M, M + 1024, cd(0, 0));
  for (int c = 0; c < 2; ++c)
    for (int p = 0; p < kRank; ++p)
      for (int a = 0; a < kRank; ++a) {
        const cd w = use_v ? F.leafV(j0 + c, p, a) : F.leafU(j0 + c, p, a);
        if (in)
          M[(c * kRank + a) * 32 + c * kRank + p] = std::conj(w);
        else
          M[(c * kRank + p) * 32 + c * kRank + a] = w;
      }
}

template <class Fn>
void parallel_for(int64_t n, Fn fn) {
  const unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (n < 64 || nt == 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (int64_t i = (int64_t)(n * t / nt); i < (int64_t)(n * (t + 1) / nt); ++i) fn(i);
    });
  for (auto &x : th) x.join();
}

std::vector<int> split_levels(int h, int kmax) {
  const int np = (h + kmax - 1) / kmax;
  std::vector<int> ks;
  for (int i = 0; i < np; ++i) ks.push_back(h / np + (i < h % np ? 1 : 0));
  return ks;
}

bf_status upload(bf_plan *p, FusedPass *fp, const void *src, size_t bytes, void **dst) {
  void *d = nullptr;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p->err = std::string("fused pack allocation: ") + hipGetErrorString(e);
    return BF_ERR_ALLOC;
  }
  fp->owned.push_back(d);
  e = hipMemcpy(d, src, bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    p->err = std::string("fused pack upload: ") + hipGetErrorString(e);
    return BF_ERR_HIP;
  }
  *dst = d;
  return BF_OK;
}

bf_status build_pass(bf_plan *p, const HostFactors &F, const PassPlan &pp, int prec, int cols,
                     const void *Sm, FusedPass **out) {
  FusedPass *fp = new FusedPass();
  *out = fp;
  const int K = pp.K, L = p->L;
  const int NB = 1 << (K - 1);
  fp->K = K;
  fp->cols = cols;
  fp->log_slo = L - pp.l_hi;
  fp->mode_si = (pp.side == kHfwd || pp.side == kGadj) ? 1 : 0;
  fp->in_kind = pp.in_kind;
  fp->out_kind = pp.out_kind;
  fp->ntiles = int64_t(1) << (L - K);
  if (prec == kF64)
    fp->Sm64 = static_cast<const double *>(Sm);
  else
    fp->Sm = static_cast<const float *>(Sm);
  const int64_t bbytes = prec == kF64 ? kBlockBytes64 : kBlockBytes;
  static const char *side_name[] = {"H_fwd", "G_fwd", "G_adj", "H_adj"};
  fp->name = std::string("fused_") + side_name[pp.side] + "_l" + std::to_string(pp.l_hi) + "_" +
             std::to_string(pp.l_lo);
  const int64_t ntiles = fp->ntiles;
  const int64_t nblk = (int64_t)K * ntiles * NB;
  std::vector<char> buf((size_t)(nblk * bbytes));
  std::vector<float> sc((size_t)nblk, 1.f);
  parallel_for(ntiles, [&](int64_t tile) {
    std::vector<cd> M(1024);
    const int64_t hi = tile >> fp->log_slo, lo = tile & ((int64_t(1) << fp->log_slo) - 1);
    for (int d = 0; d < K; ++d)
      for (int ap = 0; ap < (1 << (K - d - 1)); ++ap)
        for (int b = 0; b < (1 << d); ++b) {
          const int beta = ap * (1 << d) + b;
          const int64_t bi = ((int64_t)d * ntiles + tile) * NB + beta;
          butterfly_block(F, pp, d, hi, lo, ap, b, M.data());
          if (prec == kF64)
            pack_block64(M.data(), buf.data() + bi * bbytes);
          else
            sc[bi] = pack_block(M.data(), prec, cols, buf.data() + bi * bbytes);
        }
  });
  bf_status st = upload(p, fp, buf.data(), buf.size(), &fp->fac);
  if (st == BF_OK && prec == kF16)
    st = upload(p, fp, sc.data(), sc.size() * sizeof(float), (void **)&fp->fscale);
  if (st != BF_OK) return st;
  if (pp.in_kind == kInUser || pp.out_kind == kOutUser) {
    // first pass of a direction: leaf in (V^* forward, U^* adjoint);
    // last pass: leaf out (U forward, V adjoint)
    const bool in = pp.in_kind == kInUser;
    const bool use_v = in ? (pp.side == kHfwd) : (pp.side == kHadj);
    const int64_t lbytes = prec == kF64 ? kLeafBytes64 : cols == 16 ? kBlockBytes / 2 : kBlockBytes;
    std::vector<char> lb((size_t)(ntiles * NB * lbytes));
    std::vector<float> ls((size_t)ntiles * NB, 1.f);
    parallel_for(ntiles, [&](int64_t tile) {
      std::vector<cd> M(1024);
      for (int q = 0; q < NB; ++q) {
        const int64_t bi = tile * NB + q;
        leaf_block(F, use_v, in, (tile << K) + 2 * q, M.data());
        if (prec == kF64)
          pack_leaf64(M.data(), lb.data() + bi * lbytes);
        else
          ls[bi] = cols == 16 ? pack_leaf16(M.data(), prec, lb.data() + bi * lbytes)
                              : pack_block(M.data(), prec, cols, lb.data() + bi * lbytes);
      }
    });
    st = upload(p, fp, lb.data(), lb.size(), &fp->leaf);
    if (st == BF_OK && prec == kF16)
      st = upload(p, fp, ls.data(), ls.size() * sizeof(float), (void **)&fp->lscale);
  }
  return st;
}

FusedArgs pass_args(const bf_plan *p, const FusedPass *fp, const void *in, void *out, int64_t nrhs,
                    int64_t ld) {
  FusedArgs a;
  a.in = in;
  a.out = out;
  a.fac = static_cast<const char *>(fp->fac);
  a.leaf = static_cast<const char *>(fp->leaf);
  a.fscale = fp->fscale;
  a.lscale = fp->lscale;
  a.Sm = fp->Sm;
  a.Sm64 = fp->Sm64;
  a.ld = ld;
  a.nrhs = nrhs;
  a.nchunks = (nrhs + fp->cols - 1) / fp->cols;
  a.nslots = p->P;
  a.ntiles = fp->ntiles;
  a.m = p->m;
  a.log_slo = fp->log_slo;
  a.mode_si = fp->mode_si;
  a.in_kind = fp->in_kind;
  a.out_kind = fp->out_kind;
  a.ngroups = 1;
  for (auto &q : a.lvl) q = nullptr;
  a.log_m = 0;
  while ((int64_t(1) << a.log_m) < a.m) ++a.log_m;
  return a;
}

hipError_t launch_pass(const bf_plan *p, const FusedPass *fp, const void *in, void *out,
                       int64_t nrhs, int64_t ld, hipStream_t s) {
  FusedArgs a = pass_args(p, fp, in, out, nrhs, ld);
  const bool li = fp->in_kind == kInUser, lo = fp->out_kind == kOutUser;
  if (p->prec == BF_PREC_F64) return launch_f64(a, fp->K, li, lo, s);
  if (p->prec == BF_PREC_F32) return launch_prec<kF32>(a, fp->cols, fp->K, li, lo, fp->split, s);
  if (p->prec == BF_PREC_SPLIT_BF16)
    return launch_prec<kBF16>(a, fp->cols, fp->K, li, lo, fp->split, s);
  return launch_prec<kF16>(a, fp->cols, fp->K, li, lo, fp->split, s);
}

}  // namespace

bool fused_supported(const bf_shape &sh, bf_precision prec, const bf_plan_options &opt) {
  if (opt.path == 1) return false;
  if (prec == BF_PREC_F64 && opt.fused_cols == 32) return false;  // FP64 passes: 16 columns only
  return sh.radix == 2 && sh.leaf == kRank && sh.r == kRank && sh.L >= 2;
}

bf_status fused_build(bf_plan *p, const bf_factors_host *f) {
  HostFactors F{f, p->L, p->h};
  // wavefront geometry (columns per wavefront) and deepest pass (the handle's
  // options can select other variants, for comparisons)
  const int cols = p->opt.fused_cols == 32 && p->prec != BF_PREC_F64 ? 32 : kDefaultCols;
  const int kcap = cols == 32 ? 3 : 4;
  // four-level passes (four passes per apply at L = 16) for every precision
  const int kmax = p->opt.fused_kmax > 0 ? std::min(kcap, p->opt.fused_kmax) : kcap;
  // passes of at least split_min levels (16-column geometry) share each tile
  // between a pair of wavefronts
  const int split_min = p->opt.fused_split < 0 ? 99 : p->opt.fused_split > 0 ? p->opt.fused_split : 4;
  p->cs = cols == 32 ? 5 : 4;
  const int prec = p->prec == BF_PREC_F64 ? kF64
                   : p->prec == BF_PREC_F32 ? kF32
                   : p->prec == BF_PREC_SPLIT_BF16 ? kBF16 : kF16;

  // middle weights in natural slot order (FP64 for FP64 passes, FP32 otherwise):
  // S for the forward, S^T for the adjoint
  const int64_t m = p->m;
  const size_t wb = prec == kF64 ? 8 : 4;
  std::vector<char> S((size_t)m * m * kRank * wb), ST((size_t)m * m * kRank * wb);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < m; ++j)
      for (int k = 0; k < kRank; ++k) {
        const double v = f->S[(i * m + j) * kRank + k];
        const size_t a = (size_t)((i * m + j) * kRank + k), b = (size_t)((j * m + i) * kRank + k);
        if (prec == kF64) {
          reinterpret_cast<double *>(S.data())[a] = v;
          reinterpret_cast<double *>(ST.data())[b] = v;
        } else {
          reinterpret_cast<float *>(S.data())[a] = (float)v;
          reinterpret_cast<float *>(ST.data())[b] = (float)v;
        }
      }
  FusedPass holder;
  void *dS = nullptr, *dST = nullptr;
  bf_status st = upload(p, &holder, S.data(), S.size(), &dS);
  if (st == BF_OK) st = upload(p, &holder, ST.data(), ST.size(), &dST);
  for (void *d : holder.owned) p->allocs.push_back(d);
  if (st != BF_OK) return st;

  const std::vector<int> ks = split_levels(p->h, kmax);
  for (int dir = 0; dir < 2; ++dir) {
    const bool adj = dir == 1;
    auto &list = adj ? p->adj_passes : p->fwd_passes;
    // first side: from the leaves (level L) down to the middle (level h)
    int l_hi = p->L;
    for (size_t t = 0; t < ks.size(); ++t) {
      PassPlan pp{adj ? kGadj : kHfwd, ks[t], l_hi, l_hi - ks[t], t == 0 ? kInUser : kInAct, kOutAct};
      FusedPass *fp = nullptr;
      st = build_pass(p, F, pp, prec, cols, nullptr, &fp);
      list.push_back(fp);
      if (fp) fp->split = cols == 16 && fp->K >= 3 && fp->K >= split_min;
      if (st != BF_OK) return st;
      l_hi -= ks[t];
    }
    // second side: from the middle (level h) up to the leaves
    int l_lo = p->h;
    for (size_t t = 0; t < ks.size(); ++t) {
      const int K = ks[ks.size() - 1 - t];
      PassPlan pp{adj ? kHadj : kGfwd, K, l_lo + K, l_lo, t == 0 ? kInMiddle : kInAct,
                  t + 1 == ks.size() ? kOutUser : kOutAct};
      FusedPass *fp = nullptr;
      st = build_pass(p, F, pp, prec, cols, t == 0 ? (adj ? dST : dS) : nullptr, &fp);
      list.push_back(fp);
      if (fp) fp->split = cols == 16 && fp->K >= 3 && fp->K >= split_min;
      if (st != BF_OK) return st;
      l_lo += K;
    }
  }
  return BF_OK;
}

hipError_t fused_run(bf_plan *p, bool adjoint, const void *g, void *u, int64_t nrhs, int64_t ld,
                     void *buf0, void *buf1, hipStream_t s) {
  const auto &list = adjoint ? p->adj_passes : p->fwd_passes;
  const void *cur = g;
  void *bufs[2] = {buf0, buf1};
  for (size_t t = 0; t < list.size(); ++t) {
    void *dst = (t + 1 == list.size()) ? u : bufs[t & 1];
    prof_begin(p, list[t]->name, s);
    hipError_t e = launch_pass(p, list[t], cur, dst, nrhs, ld, s);
    prof_end(p, s);
    if (e != hipSuccess) return e;
    cur = dst;
  }
  return hipSuccess;
}

// Passes of the backward pass: the pass split of the apply, 16-column geometry,
// blocks packed on the device from the canonical factors the handle holds (split
// BF16 for split-BF16 handles, FP32 for the others).  The forward list has no leaf-out blocks: the backward pass needs the
// state before U^L, not u.
bf_status fused_build_backward(bf_plan *p, hipStream_t s) {
  const int L = p->L, h = p->h;
  p->bwd_bf16 = p->prec == BF_PREC_SPLIT_BF16;
  const std::vector<int> ks = split_levels(h, 4);
  // middle weights (S, S^T) as the apply passes hold them
  const float *Sm[2] = {nullptr, nullptr};
  for (int dir = 0; dir < 2; ++dir)
    for (const FusedPass *q : dir ? p->adj_passes : p->fwd_passes)
      if (q->in_kind == kInMiddle) Sm[dir] = q->Sm;
  auto alloc = [&](FusedPass *fp, size_t bytes, void **d) -> bf_status {
    hipError_t e = hipMalloc(d, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p->err = std::string("backward pack allocation: ") + hipGetErrorString(e);
      return BF_ERR_ALLOC;
    }
    fp->owned.push_back(*d);
    return BF_OK;
  };
  for (int dir = 0; dir < 2; ++dir) {
    const bool adj = dir == 1;
    const auto &ops = adj ? p->adj_ops : p->fwd_ops;
    auto &list = adj ? p->bwd_adj : p->bwd_fwd;
    int t_first = 1;  // op index of the pass's first butterfly level
    for (int sd = 0; sd < 2; ++sd) {
      int l_edge = sd == 0 ? L : h;
      for (size_t t = 0; t < ks.size(); ++t) {
        const int K = sd == 0 ? ks[t] : ks[ks.size() - 1 - t];
        FusedPass *fp = new FusedPass();
        list.push_back(fp);
        const int l_hi = sd == 0 ? l_edge : l_edge + K;
        const PassSide side = sd == 0 ? (adj ? kGadj : kHfwd) : (adj ? kHadj : kGfwd);
        fp->K = K;
        fp->cols = 16;
        // FP32 backward passes of three levels also share their tiles (2% faster on
        // the N = 2^18, 128-column backward); split BF16 keeps the apply's rule
        const int split_min = p->opt.fused_split < 0  ? 99
                              : p->opt.fused_split > 0 ? p->opt.fused_split
                              : p->bwd_bf16            ? 4
                                                       : 3;
        fp->split = K >= 3 && K >= split_min;
        fp->log_slo = L - l_hi;
        fp->mode_si = (side == kHfwd || side == kGadj) ? 1 : 0;
        fp->in_kind = t == 0 ? (sd == 0 ? kInUser : kInMiddle) : kInAct;
        fp->out_kind = (adj && sd == 1 && t + 1 == ks.size()) ? kOutUser : kOutAct;
        fp->ntiles = int64_t(1) << (L - K);
        fp->Sm = (sd == 1 && t == 0) ? Sm[dir] : nullptr;
        static const char *side_name[] = {"H_fwd", "G_fwd", "G_adj", "H_adj"};
        fp->name = std::string("bwd_") + side_name[side] + "_l" + std::to_string(l_hi) + "_" +
                   std::to_string(l_hi - K);
        if (sd == 1 && t == 0) ++t_first;  // the middle op
        PackPassArgs pa;
        pa.K = K;
        pa.log_slo = fp->log_slo;
        pa.mode_si = fp->mode_si;
        pa.ntiles = fp->ntiles;
        for (int d = 0; d < K; ++d) {
          const LevelOp &op = ops[t_first + d];
          int lb = 0;
          while ((int64_t(1) << lb) < op.blo) ++lb;
          pa.dep[d].Fb = op.mat;
          pa.dep[d].log_blo = lb;
          pa.dep[d].tconj = op.tconj ? 1 : 0;
          pa.dep[d].contig = op.mode == kContigIn ? 1 : 0;
        }
        const int64_t NB = int64_t(1) << (K - 1);
        void *d = nullptr;
        bf_status st = alloc(fp, (size_t)(K * fp->ntiles * NB) * kBlockBytes, &d);
        if (st != BF_OK) return st;
        fp->fac = d;
        hipError_t e = launch_pack_pass(pa, d, p->bwd_bf16, s);
        if (e == hipSuccess && (fp->in_kind == kInUser || fp->out_kind == kOutUser)) {
          const bool in = fp->in_kind == kInUser;
          const LevelOp &lop = in ? ops.front() : ops.back();
          if ((st = alloc(fp, (size_t)(fp->ntiles * NB) * (kBlockBytes / 2), &d)) != BF_OK) return st;
          fp->leaf = d;
          e = launch_pack_leaf16(lop.mat, d, fp->ntiles * NB, K, in, p->bwd_bf16, s);
        }
        if (e != hipSuccess) {
          p->err = std::string("backward pack: ") + hipGetErrorString(e);
          return BF_ERR_HIP;
        }
        t_first += K;
        l_edge = sd == 0 ? l_edge - K : l_edge + K;
      }
    }
  }
  p->bwd_ready = true;
  return BF_OK;
}

PassShape fused_pass_shape(const FusedPass *fp) {
  return PassShape{fp->K, fp->in_kind == kInUser, fp->in_kind == kInMiddle, fp->out_kind == kOutUser,
                   &fp->name};
}

hipError_t fused_run_pass(const bf_plan *p, const FusedPass *fp, const void *in, void *out,
                          void *const *lvl, int64_t nrhs, int64_t ld, hipStream_t s) {
  FusedArgs a = pass_args(p, fp, in, out, nrhs, ld);
  if (lvl)
    for (int d = 0; d <= fp->K; ++d) a.lvl[d] = lvl[d];
  const bool li = fp->in_kind == kInUser, lo = fp->out_kind == kOutUser;
  // a recomputation wants only the states strictly inside the pass
  const bool inner_only = !out && !lo && lvl && !lvl[fp->K];
  if (p->bwd_bf16) return launch_prec<kBF16>(a, fp->cols, fp->K, li, lo, fp->split, s, inner_only);
  return launch_prec<kF32>(a, fp->cols, fp->K, li, lo, fp->split, s, inner_only);
}

void fused_free(FusedPass *fp) {
  if (!fp) return;
  for (void *d : fp->owned) (void)hipFree(d);
  delete fp;
}

}  // namespace bfly
