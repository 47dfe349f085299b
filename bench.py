"""Benchmark of the butterfly-factorization apply on one MI355X.

Workload: the 1D Fourier integral operator shape at N = 2^20 (leaf 16, so
L = 16 binary levels), rank r = 16, 256 right-hand sides of iid complex
Gaussian g.  The factors are seeded synthetic blocks of exactly the shapes a
factorization of that operator has (building one on a CPU takes hours); the
apply's cost does not depend on their values.  Inputs are resident in HBM
before timing starts.

One step = one bf_apply over the whole batch (all passes: leaf projection,
H levels, middle weights, G levels, leaf expansion).  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--precision bf16x3|f32|f16x3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "BF apply RHS·N/s at stated rel. err (FP32 vs split-BF16 vs FP64); % roofline"
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16x3": 2516.6, "f16x3": 2516.6}   # dense MFMA, per dtype
# real MFMA work per algorithmic flop (8 per complex multiply-add): FP64 and FP32
# form each complex block product from three real products (Gauss), split
# precisions from three products per real product
MFMA_WORK = {"f64": 0.75, "f32": 0.75, "bf16x3": 3.0, "f16x3": 3.0}
# bytes of one complex value of the vectors and factors
CPLX_BYTES = {"f64": 16.0, "f32": 8.0, "bf16x3": 8.0, "f16x3": 8.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="bf16x3", choices=["bf16x3", "f32", "f16x3", "f64"])
    ap.add_argument("--variants", default="f32,f64", help="comma list of extra precisions to time")
    ap.add_argument("--log2n", type=int, default=20)
    ap.add_argument("--nrhs", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--options", default="{}",
                    help="JSON dict of bf_plan_options fields for the handles (kernel-path variants)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--shape", choices=sorted(SHAPES), default=None,
                    help="time the apply on another workload shape instead of N=2^20")
    ap.add_argument("--precision-override", default=None, choices=["f64", "f32", "bf16x3", "f16x3"],
                    help="precision for --shape (default: the shape's own)")
    ap.add_argument("--graph", action="store_true",
                    help="with --shape: also time the apply replayed from a HIP graph")
    ap.add_argument("--construct", action="store_true",
                    help="time the construction from products of K F K instead of the apply")
    ap.add_argument("--backward", action="store_true",
                    help="time bf_backward (gradients for every factor block and g) instead")
    return ap.parse_args()


def bench_backward(args):
    """bf_backward (gradients of every factor block and of g) at N = 2^log2n, r = 16,
    nrhs columns, FP32; recomputing the states inside each pass (the default) and
    keeping every state (BF_BWD_STORE_ALL)."""
    import torch
    from bf_inputs import complex_gaussian, synthetic_factors
    from paper_1502_01379_amd import BFHandle, BF_BWD_RECOMPUTE, BF_BWD_STORE_ALL
    dev = torch.device("cuda:0")
    L = args.log2n - 4
    N = 16 * 2 ** L
    f = synthetic_factors(2, 16, L, 16, seed=30)
    g = torch.from_numpy(complex_gaussian((N, args.nrhs), 31, dtype=np.complex64)).to(dev)
    gu = torch.from_numpy(complex_gaussian((N, args.nrhs), 32, dtype=np.complex64)).to(dev)
    h = BFHandle(f, args.precision, options=json.loads(args.options))
    modes = {}
    for mode, flags in (("recompute", BF_BWD_RECOMPUTE), ("store_all", BF_BWD_STORE_ALL)):
        for _ in range(args.warmup):
            h.backward(g, gu, flags=flags)
        torch.cuda.synchronize()
        h.set_profiling(True)
        h.kernel_times(reset=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            h.backward(g, gu, flags=flags)
        e1.record()
        torch.cuda.synchronize()
        h.set_profiling(False)
        kt = h.kernel_times(reset=True)
        top = sorted(kt.items(), key=lambda kv: -kv[1][0])[:10]
        modes[mode] = {"ms": e0.elapsed_time(e1) / args.steps,
                       "top_kernels_ms_per_step": {k: v[0] / args.steps for k, v in top},
                       "launches_per_step": sum(v[1] for v in kt.values()) / args.steps}
        print(f"[bench] backward {mode}: {modes[mode]['ms']:.3f} ms", file=sys.stderr, flush=True)
    # roofline of the gradient contraction of one level (the largest single cost):
    # it reads the level's input and output states (2 P r nrhs complex64) and does
    # (2r)^2 complex multiply-adds per butterfly and column
    P = 2 ** L
    name = "grad_G"
    launches = L // 2  # one per G level
    avg = modes["store_all"]["top_kernels_ms_per_step"].get(name, 0.0) / launches
    bytes_ = 2.0 * P * 16 * args.nrhs * 8
    flops = 8.0 * (P // 2) * 32 * 32 * args.nrhs
    t_mfma, t_hbm = flops / (157.3e12), bytes_ / (HBM_PEAK_GBS * 1e9)
    if avg > 0:
        if t_mfma >= t_hbm:
            roof = {"bound": "mfma", "achieved": flops / (avg * 1e-3) / 1e12, "peak": 157.3,
                    "unit": "TFLOP/s"}
        else:
            roof = {"bound": "hbm", "achieved": bytes_ / (avg * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s"}
        roof.update({"frac": roof["achieved"] / roof["peak"], "traffic": None, "kernel": name,
                     "avg_launch_ms": avg, "launches": launches})
    else:
        roof = None
    out = {"metric": "bf_backward ms (gradients of every factor block and of g)",
           "value": modes["recompute"]["ms"], "unit": "ms", "higher_is_better": False,
           "roofline": roof,
           "precision": args.precision, "data": "synthetic",
           "config": {"workload": f"1D FIO-shaped factorization, N=2^{args.log2n}, leaf 16, r=16, "
                                  f"{args.nrhs} RHS", "N": N, "L": L, "r": 16, "nrhs": args.nrhs},
           "modes": modes}
    print(json.dumps(out), flush=True)


def bench_construct(args):
    """Construction from products with K and K^* (the first case of Sec. 3.1) of the
    composition K~ = K F K (Sec. 4 Example 3) at N = 2^log2n: K is a butterfly
    factorization applied by this library (seeded synthetic FIO-shaped factors,
    FP32), F an FFT.  Reports the time of the black-box products (GPU) and of the
    host FP64 linear algebra."""
    import torch
    from bf_inputs import synthetic_factors
    from paper_1502_01379_amd import BFHandle
    from paper_1502_01379_amd.construct import construct_from_products
    L = args.log2n - 4
    N = 16 * 2 ** L
    r = 16
    hK = BFHandle(synthetic_factors(2, 16, L, r, seed=40), "f32")
    sign = torch.tensor((-1.0) ** np.arange(N), dtype=torch.float32, device="cuda")[:, None]
    t_box = [0.0]

    def timed(fn):
        def run(X):
            torch.cuda.synchronize()
            t = time.time()
            Y = fn(X.to(torch.complex64).contiguous())
            torch.cuda.synchronize()
            t_box[0] += time.time() - t
            return Y
        return run

    # K~ X = K F K X with (F v)_k = sum_j e^{-2 pi i x_j xi_k} v_j = fft((-1)^j v)
    mv = timed(lambda X: hK.apply(torch.fft.fft(hK.apply(X) * sign, dim=0).contiguous()))
    rmv = timed(lambda X: hK.apply_adjoint(
        (torch.fft.ifft(hK.apply_adjoint(X), dim=0) * (N * sign)).contiguous()))
    t0 = time.time()
    f = construct_from_products(N, 2, 16, r, mv, rmv, seed=1)
    total = time.time() - t0
    h2 = BFHandle(f, "bf16x3")
    m = 2 ** (L // 2)
    out = {"metric": "construction seconds from products with K and K^* (K F K)",
           "value": total, "unit": "s", "higher_is_better": False, "data": "synthetic",
           "config": {"workload": f"K F K with K a 1D FIO-shaped factorization, N=2^{args.log2n}, "
                                  f"leaf 16, r={r}, oversampling 5", "N": N, "r": r,
                      "product_columns": 2 * m * (r + 5)},
           "black_box_seconds": t_box[0], "host_fp64_seconds": total - t_box[0],
           "handle_path": h2.path}
    print(json.dumps(out), flush=True)


SHAPES = {
    # name: (radix, leaf, L, r, nrhs, precision, description)
    "fourier1024": (2, 16, 6, 12, 1, "f64", "Fourier-shaped factorization, N=1024, leaf 16, r=12, 1 RHS"),
    "fio65536": (2, 16, 12, 16, 64, "f32", "1D FIO-shaped factorization, N=65536, leaf 16, r=16, 64 RHS"),
    "grt256": (4, 16, 6, 32, 128, "f32",
               "2D GRT-shaped factorization, 256x256 points, quadtrees with 4x4 leaves, r=32, 128 RHS"),
}


def bench_shape(args):
    """Apply timing on one of the other workload shapes (seeded synthetic factors of
    that shape; the apply's cost does not depend on the values), with the roofline of
    the whole apply from its algorithmic work: 2 N r (leaves) + L R r^2 P (butterflies)
    + P r (middle) complex multiply-adds per RHS, and the factor bytes plus g and u."""
    import torch
    from bf_inputs import complex_gaussian, synthetic_factors
    from paper_1502_01379_amd import BFHandle
    R, leaf, L, r, nrhs, prec, desc = SHAPES[args.shape]
    if args.precision_override:
        prec = args.precision_override
    P = R ** L
    N = leaf * P
    f = synthetic_factors(R, leaf, L, r, seed=50)
    cdt = np.complex128 if prec == "f64" else np.complex64
    g = torch.from_numpy(complex_gaussian((N, nrhs), 51, dtype=cdt)).to("cuda")
    u = torch.empty_like(g)
    h = BFHandle(f, prec)
    for _ in range(args.warmup):
        h.apply(g, out=u)
    torch.cuda.synchronize()
    # timed without per-launch events (they cost microseconds on the small shapes),
    # then once more with them for the per-kernel split
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        h.apply(g, out=u)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    graph_ms = None
    if args.graph:
        # the same apply recorded once in a HIP graph and replayed (launch-bound shapes)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            h.apply(g, out=u)
        graph.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        graph_ms = e0.elapsed_time(e1) / args.steps
    h.set_profiling(True)
    h.kernel_times(reset=True)
    for _ in range(args.steps):
        h.apply(g, out=u)
    torch.cuda.synchronize()
    kt = h.kernel_times(reset=True)
    h.set_profiling(False)
    cmac = 2 * N * r + L * R * r * r * P + P * r
    flops = 8.0 * cmac * nrhs
    cb = 16 if prec == "f64" else 8
    bytes_ = (2 * N * r + L * P * R * r * r) * cb + 2 * N * nrhs * cb
    peak = {"f64": 78.6, "f32": 157.3, "bf16x3": 2516.6 / 3, "f16x3": 2516.6 / 3}[prec]
    t_roof = max(flops / (peak * 1e12), bytes_ / (HBM_PEAK_GBS * 1e9)) * 1e3
    out = {"metric": "BF apply RHS·N/s", "value": nrhs * N / (ms * 1e-3), "unit": "RHS·N/s",
           "ms_per_step": ms, "precision": prec, "data": "synthetic",
           "config": {"workload": desc, "N": N, "radix": R, "leaf": leaf, "L": L, "r": r, "nrhs": nrhs},
           "kernel_path": "fused MFMA passes" if h.path == 1 else "per-level kernels",
           "whole_apply_roofline": {"ms": t_roof, "bound": "compute" if flops / (peak * 1e12) >=
                                    bytes_ / (HBM_PEAK_GBS * 1e9) else "hbm",
                                    "frac": t_roof / ms, "flops": flops, "bytes": bytes_},
           "kernels_ms_per_step": {k: v[0] / args.steps for k, v in kt.items()}}
    if graph_ms is not None:
        out["hip_graph_ms_per_step"] = graph_ms
    print(json.dumps(out), flush=True)


def pass_work(L, r, leaf, nrhs, K, reads_g, writes_u, has_middle, cb=8.0):
    """Algorithmic flops and bytes of one fused-pass launch (its share of the apply).

    Unit: one butterfly (a 2r x 2r complex block) applied to one right-hand
    side = (2r)^2 complex multiply-adds = 8 (2r)^2 real flops.  A pass of K
    levels applies K 2^(L-1) of them per column, plus N r multiply-adds per
    column for a leaf block.  Algorithmic bytes count what the whole apply must
    move once: the pass's factor blocks (K 2^(L-1) blocks of (2r)^2 complex64),
    its leaf blocks (N r complex64) and middle weights (P r float32), g if the
    pass reads it and u if it writes it (cb bytes per complex value: 8, or 16 for
    FP64, whose real values take 8).  Activations handed from one pass to the next
    are implementation traffic, not algorithmic.
    """
    P = 2 ** L
    N = P * leaf
    has_leaf = reads_g or writes_u
    cm = K * (P // 2) * (2 * r) ** 2 + (N * r if has_leaf else 0)
    flops = 8.0 * cm * nrhs
    fac = K * (P // 2) * (2 * r) ** 2 * cb + (N * r * cb if has_leaf else 0.0)
    mid = P * r * cb / 2 if has_middle else 0.0
    vec = N * cb * nrhs * ((1 if reads_g else 0) + (1 if writes_u else 0))
    return flops, fac + mid + vec


def apply_work(L, r, leaf, nrhs, R=2, cb=8.0):
    """Algorithmic flops and bytes of a whole apply: 2 N r (leaves) + L R r^2 P
    (butterflies) + P r (middle) complex multiply-adds per column; the factors once
    (cb bytes per complex entry: complex64, or complex128 for FP64; S real of half
    that) plus g and u once."""
    P = R ** L
    N = leaf * P
    flops = 8.0 * (2 * N * r + L * R * r * r * P + P * r) * nrhs
    bytes_ = (2 * N * r + L * P * R * r * r) * cb + P * r * cb / 2 + 2 * N * cb * nrhs
    return flops, bytes_


def roofline_time(flops, bytes_, prec):
    """(seconds, bound) of the roofline for MFMA work flops * MFMA_WORK[prec]."""
    t_mfma = flops * MFMA_WORK[prec] / (PEAK_TFLOPS[prec] * 1e12)
    t_hbm = bytes_ / (HBM_PEAK_GBS * 1e9)
    return (t_mfma, "mfma") if t_mfma >= t_hbm else (t_hbm, "hbm")


def host_record():
    """CPU model, core count and BLAS of the host the oracle runs on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        info = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if info:
            blas = {"library": info[0].get("internal_api"), "version": info[0].get("version"),
                    "threads": info[0].get("num_threads")}
    except Exception:
        pass
    return {"nproc": os.cpu_count(), "sched_cpus": len(os.sched_getaffinity(0)), "cpu_model": model,
            "blas": blas}


def cpu_oracle_baseline(f, g_host, sample, kern_rows, N):
    """The FP64 oracle apply of the same factors on a sample of columns: one warm-up
    run, then the median of three, with BLAS on every core the process may use and
    on one core; plus the dense apply K[rows, :] g of a few sampled rows (the
    analogue of the direct evaluation time of Sec. 4).  Returns (baseline, ref):
    ref is the warm-up result, the FP64 reference of the sampled columns."""
    import oracle
    from oracle import kernels
    from threadpoolctl import threadpool_limits, threadpool_info
    x = g_host[:, sample].astype(np.complex128)
    ncores = len(os.sched_getaffinity(0))
    runs = {}
    ref = None
    for label, limit in (("all", ncores), ("one", 1)):
        with threadpool_limits(limit):
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
            t = time.time()
            out = oracle.bf_apply(f, x)
            warm = time.time() - t
            if ref is None:
                ref = out
            ts = []
            for _ in range(3):
                t = time.time()
                oracle.bf_apply(f, x)
                ts.append(time.time() - t)
        med = float(np.median(ts))
        runs[label] = {"value": len(sample) * N / med, "seconds": med, "warmup_seconds": warm,
                       "threads": threads}
        print(f"[bench] oracle apply, {label} cores ({threads} threads): {med:.2f} s", file=sys.stderr,
              flush=True)
    # dense K[rows, :] g of the 1D FIO of Sec. 4, Example 1, on the sampled columns
    kern = kernels.fio(N)
    t = time.time()
    kernels.dense_apply_rows(kern, kern_rows, x, col_chunk=1 << 16)
    dense_s = time.time() - t
    base = {"value": runs["all"]["value"], "unit": "RHS·N/s", "cores": runs["all"]["threads"],
            "kind": "oracle",
            "sample": f"FP64 oracle apply of the same factors to {len(sample)} of the columns (N={N}); "
                      f"median of 3 after a warm-up, BLAS on {runs['all']['threads']} threads",
            "one_core": runs["one"], "all_cores": runs["all"],
            "dense_rows": {"rows": int(len(kern_rows)), "columns": len(sample), "seconds": dense_s,
                           "note": "dense K[rows,:] g of the 1D FIO (Sec. 4 Example 1), FP64, "
                                   "the analogue of the direct evaluation time"},
            "host": host_record()}
    return base, ref


def profile_traffic(key, source="bf_fused_kernel.h"):
    """HBM bytes per launch of one pass kernel from the committed rocprofv3 counter
    summaries (FETCH_SIZE and WRITE_SIZE, scaled by a copy kernel of known size),
    or None when no summary covers it or the kernel's source file changed since."""
    import glob
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(here, "paper_1502_01379_amd", "csrc", source)
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(here, "profiles", "*.txt"))):
        for line in open(path):
            if line.startswith("traffic: "):
                rec = json.loads(line[len("traffic: "):])
                if rec.get("kernel_source_sha256") == sha and key in rec.get("bytes", {}):
                    return float(rec["bytes"][key])
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.backward:
        bench_backward(args)
        return
    if args.construct:
        bench_construct(args)
        return
    if args.shape:
        bench_shape(args)
        return
    import torch

    from bf_inputs import complex_gaussian, synthetic_factors
    from paper_1502_01379_amd import BFHandle

    dev = torch.device("cuda:0")
    L = args.log2n - 4
    leaf, r, nrhs = 16, 16, args.nrhs
    N = leaf * 2 ** L
    t0 = time.time()
    f = synthetic_factors(2, leaf, L, r, seed=20)
    g_host = complex_gaussian((N, nrhs), 21, dtype=np.complex64)
    g32 = torch.from_numpy(g_host).to(dev)
    print(f"[bench] inputs ready in {time.time() - t0:.1f}s (N={N}, nrhs={nrhs})", file=sys.stderr, flush=True)

    precisions = [args.precision] + [p for p in args.variants.split(",") if p and p != args.precision]
    results = {}
    for prec in precisions:
        # FP64 handles take complex128 vectors (the same values)
        g = g32.to(torch.complex128) if prec == "f64" else g32
        u = torch.empty_like(g)
        t1 = time.time()
        h = BFHandle(f, prec, options=json.loads(args.options))
        print(f"[bench] {prec}: handle created in {time.time() - t1:.1f}s (path {h.path})",
              file=sys.stderr, flush=True)
        stream = torch.cuda.current_stream()
        for _ in range(args.warmup):
            h.apply(g, out=u)
        torch.cuda.synchronize()
        h.set_profiling(True)
        h.kernel_times(reset=True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            h.apply(g, out=u)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        kt = h.kernel_times(reset=True)
        h.set_profiling(False)
        results[prec] = {"ms": ms, "kernels": kt, "handle": h, "u_cols": None}
        print(f"[bench] {prec}: {ms:.3f} ms/step", file=sys.stderr, flush=True)
        cols = [0, nrhs // 2, nrhs - 1]
        results[prec]["u_cols"] = u[:, cols].cpu().numpy()
        h.close()
        del g, u

    # oracle: FP64 apply of the same factors on a bounded sample of columns (the
    # three the GPU results are checked on, plus one); BLAS on all cores and on one
    cpu = None
    cols = [0, nrhs // 2, nrhs - 1]
    ref = None
    if not args.no_cpu_baseline:
        sample = cols + [1]
        rows = np.random.default_rng(22).choice(N, size=32, replace=False)
        cpu, sub = cpu_oracle_baseline(f, g_host, sample, rows, N)
        ref = sub[:, :len(cols)]

    # roofline of the dominant kernel of the headline precision, from its share of
    # the apply's algorithmic work, and of the whole apply
    main_res = results[args.precision]
    kt = main_res["kernels"]
    name, (tot_ms, launches) = max(kt.items(), key=lambda kv: kv[1][0])
    avg_ms = tot_ms / max(1, launches)
    parts = name.split("_")            # fused_<H|G>_<fwd|adj>_l<hi>_<lo>
    l_hi, l_lo = int(parts[3][1:]), int(parts[4])
    K = l_hi - l_lo
    reads_g = l_hi == L and parts[1] == "H"
    writes_u = l_hi == L and parts[1] == "G"
    has_middle = l_lo == L // 2 and parts[1] == "G"
    flops, bytes_ = pass_work(L, r, leaf, nrhs, K, reads_g, writes_u, has_middle, cb=CPLX_BYTES[args.precision])
    t_roof, bound = roofline_time(flops, bytes_, args.precision)
    if bound == "mfma":
        roof = {"bound": "mfma", "achieved": flops * MFMA_WORK[args.precision] / (avg_ms * 1e-3) / 1e12,
                "peak": PEAK_TFLOPS[args.precision], "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": bytes_ / (avg_ms * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    prec_code = {"f32": 0, "bf16x3": 1, "f16x3": 2, "f64": 3}[args.precision]
    roof["traffic"] = profile_traffic(f"{K},{prec_code},{int(reads_g)},{int(writes_u)}",
                                      "bf_fused_f64.hip" if args.precision == "f64" else "bf_fused_kernel.h")
    roof["kernel"] = name
    roof["avg_launch_ms"] = avg_ms
    roof["launches"] = launches
    roof["algorithmic_bytes"] = bytes_
    roof["algorithmic_flops"] = flops
    roof["traffic_over_algorithmic"] = roof["traffic"] / bytes_ if roof["traffic"] else None
    wf, wb = apply_work(L, r, leaf, nrhs, cb=CPLX_BYTES[args.precision])
    wt, wbound = roofline_time(wf, wb, args.precision)
    roof["whole_apply"] = {"bound": wbound, "roofline_ms": wt * 1e3, "ms": main_res["ms"],
                           "frac": wt * 1e3 / main_res["ms"], "algorithmic_bytes": wb,
                           "algorithmic_flops": wf}

    def rel(u_cols):
        if ref is None:
            return None
        d = u_cols.astype(np.complex128) - ref
        return float(np.sqrt(np.sum(np.abs(d) ** 2) / np.sum(np.abs(ref) ** 2)))

    def rel_max_col(u_cols):
        if ref is None:
            return None
        d = u_cols.astype(np.complex128) - ref
        return float(np.max(np.sqrt(np.sum(np.abs(d) ** 2, axis=0) / np.sum(np.abs(ref) ** 2, axis=0))))

    variants = {}
    for prec, res in results.items():
        vf, vb = apply_work(L, r, leaf, nrhs, cb=CPLX_BYTES[prec])
        vt, vbound = roofline_time(vf, vb, prec)
        variants[prec] = {"value": nrhs * N / (res["ms"] * 1e-3), "ms_per_step": res["ms"],
                          "rel_err_vs_fp64": rel(res["u_cols"]),
                          "rel_err_max_column": rel_max_col(res["u_cols"]),
                          "whole_apply_roofline": {"bound": vbound, "roofline_ms": vt * 1e3,
                                                   "frac": vt * 1e3 / res["ms"]},
                          "kernels_ms_per_launch": {k: v[0] / max(1, v[1]) for k, v in res["kernels"].items()}}

    if args.copy_probe:
        x = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()

    ms = main_res["ms"]
    out = {
        "metric": METRIC,
        "value": nrhs * N / (ms * 1e-3),
        "unit": "RHS·N/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16x3": "bf16", "f16x3": "f16", "f32": "f32", "f64": "f64"}[args.precision],
        "precision": {"bf16x3": "split BF16: hi*hi + hi*lo + lo*hi MFMA products, FP32 accumulation",
                      "f16x3": "split FP16: three MFMA products, FP32 accumulation, power-of-two scaling",
                      "f32": "FP32 MFMA", "f64": "FP64 MFMA"}[args.precision],
        "rel_err_vs_fp64": variants[args.precision]["rel_err_vs_fp64"],
        "data": "synthetic",
        "config": {"workload": f"1D FIO-shaped butterfly factorization, N=2^{args.log2n}, leaf 16 "
                               f"(L={L}), r=16, {nrhs} RHS, seeded synthetic factor blocks",
                   "N": N, "leaf": leaf, "L": L, "r": r, "nrhs": nrhs},
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
