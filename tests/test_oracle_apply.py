"""Pins for the oracle's factor apply, adjoint and gradient (CPU only)."""
import os

import numpy as np
import pytest

import oracle
from bf_inputs import complex_gaussian, synthetic_factors
from oracle import sparse
from oracle.apply import bf_apply, bf_apply_adjoint, bf_grad

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig_patterns_L6_r1.txt")


def _load_figure_patterns():
    pats = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, r, c = line.split()
            pats.setdefault(name, set()).add((int(r), int(c)))
    return pats


def _pattern(M):
    M = M.tocoo() if hasattr(M, "tocoo") else None
    return {(int(r), int(c)) for r, c, v in zip(M.row, M.col, M.data) if v != 0}


def _dense_pattern(A):
    r, c = np.nonzero(np.abs(A) > 0)
    return set(zip(r.tolist(), c.tolist()))


def test_factor_patterns_match_paper_figures():
    # Figures 3-5: 64 x 64 matrix, L = 6, h = 3, r = 1, one point per leaf
    pats = _load_figure_patterns()
    f = synthetic_factors(2, 1, 6, 1, seed=3)
    mats = sparse.factor_list(f)
    # order: U^6, G^5, G^4, G^3, M^3, (H^3)^*, (H^4)^*, (H^5)^*, (V^6)^*
    U6, G5, G4, G3, M3, H3h, H4h, H5h, V6h = mats
    assert _pattern(G3) == pats["G3"]
    assert _pattern(G4) == pats["G4"]
    assert _pattern(M3) == pats["M3"]
    assert _pattern(H3h) == pats["H3h"]
    assert _pattern(H4h) == pats["H4h"]
    # partially factorized U^l = U^L G^{L-1} .. G^l and (V^l)^*
    U5 = (U6 @ G5).toarray()
    U4 = U5 @ G4.toarray()
    U3 = U4 @ G3.toarray()
    assert _dense_pattern(U5) == pats["U5"]
    assert _dense_pattern(U4) == pats["U4"]
    assert _dense_pattern(U3) == pats["U3"]
    V5h = (H5h @ V6h).toarray()
    V3h = H3h.toarray() @ (H4h.toarray() @ V5h)
    assert _dense_pattern(V5h) == pats["V5h"]
    assert _dense_pattern(V3h) == pats["V3h"]


@pytest.mark.parametrize("radix,leaf,L,r", [(2, 3, 4, 3), (2, 1, 6, 2), (4, 2, 2, 5), (2, 4, 2, 6)])
def test_structured_apply_equals_sparse_product(radix, leaf, L, r):
    f = synthetic_factors(radix, leaf, L, r, seed=L * 10 + r)
    N = leaf * radix ** L
    g = complex_gaussian((N, 3), 1)
    u = bf_apply(f, g)
    ua = sparse.assembled_apply(f, g)
    assert np.abs(u - ua).max() <= 1e-13 * np.abs(ua).max()
    # one vector at a time, and unit vectors give the columns of the assembled matrix
    assert np.abs(bf_apply(f, g[:, 0]) - u[:, 0]).max() <= 1e-14 * np.abs(u).max()
    Kd = sparse.assembled_dense(f)
    cols = np.stack([bf_apply(f, e) for e in np.eye(N)], 1)
    assert np.abs(cols - Kd).max() <= 1e-13 * np.abs(Kd).max()


@pytest.mark.parametrize("radix,leaf,L,r", [(2, 3, 4, 3), (4, 2, 2, 5), (2, 2, 6, 4)])
def test_adjoint(radix, leaf, L, r):
    f = synthetic_factors(radix, leaf, L, r, seed=99)
    N = leaf * radix ** L
    g = complex_gaussian((N, 2), 3)
    w = complex_gaussian((N, 2), 4)
    lhs = np.vdot(w, bf_apply(f, g))
    rhs = np.vdot(bf_apply_adjoint(f, w), g)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    Kd = sparse.assembled_dense(f)
    assert np.abs(bf_apply_adjoint(f, w) - Kd.conj().T @ w).max() <= 1e-13 * np.abs(Kd).max() * np.abs(w).max() * N


def _loss(f, g, y):
    return float(np.sum(np.abs(bf_apply(f, g) - y) ** 2))


def _entries(f, rng, count):
    """Random (key, level, index) picks over every factor kind."""
    picks = []
    kinds = ["VL", "UL", "S", "H", "G"]
    for t in range(count):
        kind = kinds[t % len(kinds)]
        if kind in ("H", "G"):
            lev = int(rng.integers(len(f[kind])))
            arr = f[kind][lev]
        else:
            lev = None
            arr = f[kind]
        idx = tuple(int(rng.integers(s)) for s in arr.shape)
        picks.append((kind, lev, idx))
    return picks


@pytest.mark.parametrize("radix,leaf,L,r", [(2, 3, 4, 3), (4, 2, 2, 4)])
def test_gradient_matches_central_differences(radix, leaf, L, r):
    # L(theta) = ||K_BF g - y||^2 is quadratic in every single entry, so a central
    # difference is exact up to rounding for any step.
    f = synthetic_factors(radix, leaf, L, r, seed=5)
    N = leaf * radix ** L
    g = complex_gaussian((N, 3), 6)
    y = complex_gaussian((N, 3), 7)
    grad = bf_grad(f, g, 2 * (bf_apply(f, g) - y))
    rng = np.random.default_rng(8)
    delta = 1e-3
    for kind, lev, idx in _entries(f, rng, 40):
        arr = f[kind][lev] if lev is not None else f[kind]
        gval = (grad[kind][lev] if lev is not None else grad[kind])[idx]
        parts = [(1.0, np.real)] if kind == "S" else [(1.0, np.real), (1j, np.imag)]
        for unit, part in parts:
            old = arr[idx]
            arr[idx] = old + delta * unit
            lp = _loss(f, g, y)
            arr[idx] = old - delta * unit
            lm = _loss(f, g, y)
            arr[idx] = old
            fd = (lp - lm) / (2 * delta)
            assert abs(fd - part(gval)) <= 1e-8 * max(1.0, abs(gval)), (kind, lev, idx)
    for n in range(6):
        k = (int(rng.integers(N)), int(rng.integers(3)))
        for unit, part in [(1.0, np.real), (1j, np.imag)]:
            old = g[k]
            g[k] = old + delta * unit
            lp = _loss(f, g, y)
            g[k] = old - delta * unit
            lm = _loss(f, g, y)
            g[k] = old
            assert abs((lp - lm) / (2 * delta) - part(grad["g"][k])) <= 1e-8 * max(1.0, abs(grad["g"][k]))


def test_nonzeros_are_linear_in_N():
    # every factor has O(N) nonzeros (Sec. 1.2); exactly: leaves N r, butterflies N R r^2 / n0, middle N r / n0
    R, leaf, L, r = 2, 2, 6, 3
    f = synthetic_factors(R, leaf, L, r, seed=1)
    N = leaf * R ** L
    P = R ** L
    nnz = sparse.nnz_per_factor(f)
    assert nnz[0] == N * r and nnz[-1] == N * r
    assert nnz[L // 2 + 1] == P * r
    for k in list(range(1, L // 2 + 1)) + list(range(L // 2 + 2, L + 2)):
        assert nnz[k] == P * R * r * r
