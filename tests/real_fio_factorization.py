"""The 1D Fourier integral operator of Sec. 4, Example 1, factorized for real
(N = 65536, leaf 16, r = 16, the library's host FP64 construction from entries in
the O(N log N)-memory order of Sec. 3.3) and applied on the GPU to 64 columns of
iid complex Gaussian g, in FP32 and split BF16.  Prints, as one JSON line:

  * parity: the relative error of each GPU precision against the oracle's FP64
    apply of the same factors, on sampled columns (over them and per column);
  * the approximation error of Sec. 4 (the relative error of the FP64 factor
    apply against the dense kernel on 256 sampled rows, all 64 columns) and of
    each GPU precision against the same dense rows;
  * construction and apply times.

Not collected by pytest (a run takes minutes of CPU for the construction):

    python tests/real_fio_factorization.py [--log2n 16] [--nrhs 64] [--rows 256]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from bf_inputs import complex_gaussian  # noqa: E402
from oracle import kernels  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--log2n", type=int, default=16)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--rows", type=int, default=256)
    ap.add_argument("--rank", type=int, default=16)
    args = ap.parse_args()
    import torch
    from paper_1502_01379_amd import BFHandle
    from paper_1502_01379_amd.construct import construct_from_entries

    N, r = 1 << args.log2n, args.rank
    kern = kernels.fio(N)
    t0 = time.time()
    f = construct_from_entries(N, 2, 16, r, kern.entries, seed=0, streamed=True)
    t_build = time.time() - t0
    print(f"[fio] factorization built in {t_build:.1f} s", file=sys.stderr, flush=True)

    g = complex_gaussian((N, args.nrhs), 1)
    rows = np.sort(np.random.default_rng(2).choice(N, size=args.rows, replace=False))
    cols = [0, args.nrhs // 2, args.nrhs - 1]
    t0 = time.time()
    u_dense = kernels.dense_apply_rows(kern, rows, g)             # K[rows, :] g, FP64
    t_dense = time.time() - t0
    u_bf = oracle.bf_apply(f, g)                                   # FP64 factor apply
    eps_a = oracle.rel_err(u_bf[rows], u_dense)
    out = {"workload": f"1D FIO (Sec. 4 Example 1), N={N}, leaf 16, r={r}, {args.nrhs} RHS",
           "construction_seconds": t_build, "dense_rows_seconds": t_dense,
           "eps_a_fp64_factors_vs_dense": eps_a, "sampled_rows": args.rows, "gpu": {}}
    gd = torch.from_numpy(g.astype(np.complex64)).to("cuda")
    for prec in ("f32", "bf16x3"):
        h = BFHandle(f, prec)
        u = h.apply(gd)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            h.apply(gd, out=u)
        e1.record()
        torch.cuda.synchronize()
        un = u.cpu().numpy().astype(np.complex128)
        per_col = [oracle.rel_err(un[:, c], u_bf[:, c]) for c in cols]
        out["gpu"][prec] = {"path": h.path, "ms_per_apply": e0.elapsed_time(e1) / 20,
                            "rel_err_vs_fp64_factors": oracle.rel_err(un[:, cols], u_bf[:, cols]),
                            "rel_err_vs_fp64_factors_max_column": max(per_col),
                            "eps_a_vs_dense": oracle.rel_err(un[rows], u_dense)}
        h.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
