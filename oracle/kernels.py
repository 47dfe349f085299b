"""Kernel entries K(x_i, xi_k) of the paper's examples, in FP64.

Rows and columns are indexed in tree order: every node of the row tree T_X
and of the column tree T_Omega is a contiguous index range (Sec. 3: complete
trees of depth L, nodes A^l_i and B^{L-l}_j).  In 1D tree order is the
natural order of the grid; in 2D it is the Morton (quadtree) order.

Phases are reduced exactly where they can be: the bilinear part x.xi has
x = a/n and integer xi, so its fractional part is (a*xi mod n)/n computed in
integers; only the smooth non-bilinear part is reduced in floating point.
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def _frac(v):
    return v - np.floor(v)


class Kernel1D:
    """K_{ik} = exp(2 pi i Phi(x_i, xi_k)), x_i = i/N, xi_k = k - N/2.

    This is the discretisation of Example 1 in Sec. 4 with 0-based indices
    (the paper writes x_i = (i-1)/N and xi_j = j-1-N/2).  Phi = x*xi +
    c(x)|xi|; with c == 0 it is the shifted Fourier matrix of Sec. 1.1.
    """

    radix = 2

    def __init__(self, N, c_fn=None, name="fio"):
        self.N = int(N)
        self.c_fn = c_fn
        self.name = name

    def phase_frac(self, rows, cols):
        """Fractional part of Phi on the grid rows x cols, in [0, 1)."""
        N = self.N
        i = np.asarray(rows, dtype=np.int64)[:, None]
        k = np.asarray(cols, dtype=np.int64)[None, :] - N // 2
        bil = np.mod(i * k, N).astype(np.float64) / N           # x*xi mod 1, exact
        if self.c_fn is None:
            return bil
        x = np.asarray(rows, dtype=np.float64)[:, None] / N
        smooth = _frac(self.c_fn(x) * np.abs(k).astype(np.float64))
        return _frac(bil + smooth)

    def phase_naive(self, rows, cols):
        """Phi evaluated directly in FP64 (no reduction); for checking only."""
        N = self.N
        x = np.asarray(rows, dtype=np.float64)[:, None] / N
        xi = np.asarray(cols, dtype=np.float64)[None, :] - N // 2
        phi = x * xi
        if self.c_fn is not None:
            phi = phi + self.c_fn(x) * np.abs(xi)
        return phi

    def entries(self, rows, cols):
        return np.exp(1j * TWO_PI * self.phase_frac(rows, cols))


def fio_c(x):
    """c(x) = (2 + sin 2 pi x)/8 of Example 1 (Sec. 4)."""
    return (2.0 + np.sin(TWO_PI * x)) / 8.0


def fourier(N):
    return Kernel1D(N, None, name="fourier")


def fio(N):
    return Kernel1D(N, fio_c, name="fio")


def morton_decode(t, bits):
    """Tree-order index -> (a1, a2) grid coordinates.

    Each base-4 digit of t, most significant first, is one quadtree level;
    the digit is c = 2*bit(a1) + bit(a2) at that level.
    """
    t = np.asarray(t, dtype=np.int64)
    a1 = np.zeros_like(t)
    a2 = np.zeros_like(t)
    for lev in range(bits):
        digit = (t >> (2 * (bits - 1 - lev))) & 3
        a1 = (a1 << 1) | (digit >> 1)
        a2 = (a2 << 1) | (digit & 1)
    return a1, a2


class Kernel2D:
    """2D generalised Radon transform on an n x n grid, quadtree (Morton) order.

    x = (a1, a2)/n in [0,1)^2, xi = (b1 - n/2, b2 - n/2) integers in
    [-n/2, n/2)^2, Phi = x.xi + sqrt(c1(x)^2 xi1^2 + c2(x)^2 xi2^2) with
    c1 = (2 + sin 2pi x1 sin 2pi x2)/16, c2 = (2 + cos 2pi x1 cos 2pi x2)/16.
    The paper states that its 1D construction generalises to higher
    dimensions (Sec. 1.2, Sec. 5); this is that generalisation with radix-4
    trees.  With `smooth=False` the phase is x.xi only (a 2D DFT).
    """

    radix = 4

    def __init__(self, n_side, smooth=True):
        self.n = int(n_side)
        self.bits = int(round(np.log2(self.n)))
        assert 1 << self.bits == self.n
        self.N = self.n * self.n
        self.smooth = smooth
        self.name = "grt2d" if smooth else "fourier2d"

    def phase_frac(self, rows, cols):
        n = self.n
        a1, a2 = morton_decode(rows, self.bits)
        b1, b2 = morton_decode(cols, self.bits)
        a1, a2 = a1[:, None], a2[:, None]
        x1, x2 = b1[None, :] - n // 2, b2[None, :] - n // 2
        bil = np.mod(a1 * x1 + a2 * x2, n).astype(np.float64) / n
        if not self.smooth:
            return bil
        y1 = a1.astype(np.float64) / n
        y2 = a2.astype(np.float64) / n
        c1 = (2.0 + np.sin(TWO_PI * y1) * np.sin(TWO_PI * y2)) / 16.0
        c2 = (2.0 + np.cos(TWO_PI * y1) * np.cos(TWO_PI * y2)) / 16.0
        f1 = x1.astype(np.float64)
        f2 = x2.astype(np.float64)
        smooth = np.sqrt(c1 * c1 * f1 * f1 + c2 * c2 * f2 * f2)
        return _frac(bil + _frac(smooth))

    def entries(self, rows, cols):
        return np.exp(1j * TWO_PI * self.phase_frac(rows, cols))


def grt2d(n_side=256, smooth=True):
    return Kernel2D(n_side, smooth)


class LowRankKernel:
    """K = A B^T with A, B given N x T arrays: every submatrix has rank <= T.

    Not one of the paper's examples; used to exercise the construction in a
    regime where the exact answer is known.
    """

    def __init__(self, A, B, radix=2):
        self.A = np.asarray(A)
        self.B = np.asarray(B)
        self.N = self.A.shape[0]
        self.radix = radix
        self.name = "lowrank"

    def entries(self, rows, cols):
        return self.A[np.asarray(rows)] @ self.B[np.asarray(cols)].T


class HankelSum:
    """K_{ij} = H^(1)_{j}(x_i), x_i = N + (2 pi/3) i (Example 2 of Sec. 4, 0-based)."""

    radix = 2

    def __init__(self, N):
        from scipy.special import hankel1
        self._h = hankel1
        self.N = int(N)
        self.name = "hankel"

    def entries(self, rows, cols):
        x = self.N + (2.0 * np.pi / 3.0) * np.asarray(rows, dtype=np.float64)[:, None]
        nu = np.asarray(cols, dtype=np.float64)[None, :]
        return self._h(nu, x)


def dense_matrix(kernel):
    idx = np.arange(kernel.N)
    return kernel.entries(idx, idx)


def dense_apply_rows(kernel, rows, g, col_chunk=4096):
    """u[rows] = K[rows, :] g, the direct O(N) per row evaluation (Sec. 4, T_d)."""
    rows = np.asarray(rows)
    g = np.asarray(g)
    out = np.zeros((rows.size,) + g.shape[1:], dtype=np.complex128)
    for c0 in range(0, kernel.N, col_chunk):
        cols = np.arange(c0, min(kernel.N, c0 + col_chunk))
        out += kernel.entries(rows, cols) @ g[cols]
    return out
