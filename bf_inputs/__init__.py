"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module draws random numbers and lays them out in the shapes the
butterfly-factorization apply consumes.  It performs none of the method's
arithmetic: no kernel evaluation, no factorization, no apply.  Both the
oracle and the GPU path receive exactly the arrays produced here.

Array conventions (canonical factor layout, tree order, C-contiguous):

    VL, UL : complex[P][n0][r]             leaf blocks V^L_j, U^L_i
    H[t]   : complex[R^(l+1)][R^(L-l-1)][r][R*r]   level l = h + t, t = 0..h-1
    G[t]   : complex[R^(l+1)][R^(L-l-1)][r][R*r]
    S      : real[m][m][r]                 diagonal of the middle weights S^h_{i,j}

with R the tree radix, n0 the points per leaf, P = R^L leaves, N = n0*P,
h = L/2 and m = R^h.  Vectors are complex[N][nrhs].
"""
from __future__ import annotations

import numpy as np


_CHUNK = 1 << 22          # doubles per independently seeded chunk


def _fill_normal(flat, seed, threads=None, scale=1.0):
    """Fill a float64 array with scale * N(0,1) draws, chunk k seeded by (seed, k).

    The values depend only on `seed` and the array length, not on the number
    of threads used to produce them.
    """
    import concurrent.futures as cf
    import os
    n = flat.size
    nchunk = (n + _CHUNK - 1) // _CHUNK
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)

    def work(k):
        child = np.random.SeedSequence(ss.entropy, spawn_key=tuple(ss.spawn_key) + (k,))
        rng = np.random.default_rng(child)
        part = flat[k * _CHUNK:min(n, (k + 1) * _CHUNK)]
        rng.standard_normal(out=part)
        if scale != 1.0:
            part *= scale

    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    if nchunk == 1 or threads == 1:
        for k in range(nchunk):
            work(k)
    else:
        with cf.ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, range(nchunk)))


def complex_gaussian(shape, seed, dtype=np.complex128, scale=1.0):
    """iid complex Gaussian entries (a + i b) * scale / sqrt(2), a, b ~ N(0, 1)."""
    out = np.empty(shape, dtype=np.complex128)
    flat = out.reshape(-1).view(np.float64)
    _fill_normal(flat, seed, scale=scale * np.sqrt(0.5))
    return out.astype(dtype, copy=False)


def sample_rows(N, count, seed):
    """`count` distinct row indices in [0, N), drawn uniformly, returned sorted."""
    rng = np.random.default_rng(seed)
    count = min(int(count), int(N))
    return np.sort(rng.choice(N, size=count, replace=False))


def factor_shapes(radix, leaf, L, r):
    """Shapes of the canonical factor arrays for a tree of depth L (L even)."""
    R, n0 = int(radix), int(leaf)
    P = R ** L
    h = L // 2
    m = R ** h
    shapes = {
        "VL": (P, n0, r),
        "UL": (P, n0, r),
        "S": (m, m, r),
        "H": [(R ** (l + 1), R ** (L - l - 1), r, R * r) for l in range(h, L)],
        "G": [(R ** (l + 1), R ** (L - l - 1), r, R * r) for l in range(h, L)],
    }
    return shapes


def synthetic_factors(radix, leaf, L, r, seed, s_range=(0.25, 4.0)):
    """Random factors of the exact shapes of a depth-L butterfly factorization.

    Entries of every complex block are iid complex Gaussian, scaled by
    1/sqrt(fan-in) so the magnitude of a vector stays O(1) from level to
    level; the middle weights S are log-uniform in `s_range`.  The values
    carry no meaning: they exercise the apply with the real data volume and
    layout when building a factorization of that size on a CPU is too slow.
    """
    R, n0 = int(radix), int(leaf)
    shapes = factor_shapes(R, n0, L, r)
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(4 + 2 * len(shapes["H"]))
    f = {
        "radix": R, "leaf": n0, "L": int(L), "r": int(r),
        "VL": complex_gaussian(shapes["VL"], kids[0], scale=1.0 / np.sqrt(n0)),
        "UL": complex_gaussian(shapes["UL"], kids[1], scale=1.0 / np.sqrt(r)),
    }
    lo, hi = np.log(s_range[0]), np.log(s_range[1])
    f["S"] = np.exp(np.random.default_rng(kids[2]).uniform(lo, hi, shapes["S"]))
    scale = 1.0 / np.sqrt(R * r)
    f["H"] = [complex_gaussian(s, kids[4 + t], scale=scale)
              for t, s in enumerate(shapes["H"])]
    f["G"] = [complex_gaussian(s, kids[4 + len(shapes["H"]) + t], scale=scale)
              for t, s in enumerate(shapes["G"])]
    return f


def loss_target(N, nrhs, seed, base=None, noise=1e-3):
    """Target y for the quadratic loss ||u - y||^2: `base` plus complex noise."""
    eps = complex_gaussian((N, nrhs), seed)
    if base is None:
        return eps
    return base + noise * eps
