"""Pins for the oracle's kernel entries and dense matvec (CPU only)."""
import numpy as np
import pytest
from scipy.special import hankel1

from bf_inputs import complex_gaussian
from oracle import kernels


def test_fourier_dense_equals_fft():
    # K_jk = exp(2 pi i j (k - N/2)/N) = (-1)^j exp(2 pi i jk/N), so K g = (-1)^j N ifft(g)
    N = 256
    g = complex_gaussian((N, 3), 11)
    K = kernels.dense_matrix(kernels.fourier(N))
    ref = ((-1.0) ** np.arange(N))[:, None] * N * np.fft.ifft(g, axis=0)
    assert np.abs(K @ g - ref).max() <= 1e-12 * np.abs(ref).max()


def test_fio_hand_values():
    # Example 1: Phi = x xi + c(x)|xi|, c = (2 + sin 2 pi x)/8, x_i = i/N, xi_k = k - N/2
    N = 8
    kern = kernels.fio(N)
    # x = 1/4 (i = 2), xi = -4 (k = 0): Phi = -1 + (3/8)*4 = 1/2 -> K = -1
    assert abs(kern.entries([2], [0])[0, 0] - (-1.0)) < 1e-14
    # x = 3/4 (i = 6), xi = 2 (k = 6): Phi = 3/2 + (1/8)*2 = 7/4 -> K = -i
    assert abs(kern.entries([6], [6])[0, 0] - (-1j)) < 1e-14
    # x = 0, xi = 0: K = 1
    assert abs(kern.entries([0], [4])[0, 0] - 1.0) < 1e-15
    assert kernels.fio_c(np.array([0.0, 0.25, 0.75])) == pytest.approx([0.25, 0.375, 0.125])


def test_phase_reduction_matches_naive():
    N = 128
    kern = kernels.fio(N)
    idx = np.arange(N)
    a = kern.phase_frac(idx, idx)
    b = np.mod(kern.phase_naive(idx, idx), 1.0)
    d = np.abs(a - b)
    d = np.minimum(d, 1.0 - d)
    assert d.max() < 1e-12
    assert (a >= 0).all() and (a < 1).all()


def test_phase_reduction_large_N_is_exact_on_bilinear_part():
    # at N = 2^20 the naive phase x*xi loses ~1e-11; the integer path is exact
    N = 1 << 20
    kern = kernels.fourier(N)
    rows = np.array([N - 1, 12345, 777777])
    cols = np.array([0, 1, N - 1])
    frac = kern.phase_frac(rows, cols)
    ref = np.array([[((int(i) * (int(k) - N // 2)) % N) / N for k in cols] for i in rows])
    assert np.array_equal(frac, ref)


def _morton_encode(a1, a2, bits):
    t = 0
    for lev in range(bits):
        b1 = (a1 >> (bits - 1 - lev)) & 1
        b2 = (a2 >> (bits - 1 - lev)) & 1
        t = (t << 2) | (2 * b1 + b2)
    return t


def test_morton_nodes_are_boxes():
    bits = 4
    n = 1 << bits
    t = np.arange(n * n)
    a1, a2 = kernels.morton_decode(t, bits)
    for k in range(bits + 1):
        size = 4 ** k
        for t0 in range(0, n * n, size):
            b1, b2 = a1[t0:t0 + size], a2[t0:t0 + size]
            side = 1 << k
            assert b1.max() - b1.min() == side - 1 and b2.max() - b2.min() == side - 1
            assert len(set(zip(b1.tolist(), b2.tolist()))) == size
    for (x, y) in [(0, 0), (3, 9), (15, 15), (7, 8)]:
        tt = _morton_encode(x, y, bits)
        d1, d2 = kernels.morton_decode(np.array([tt]), bits)
        assert (int(d1[0]), int(d2[0])) == (x, y)


def test_2d_bilinear_is_dft2():
    # without the smooth term the 2D kernel is (-1)^(a1+a2) n^2 ifft2 in grid order
    bits = 4
    n = 1 << bits
    kern = kernels.grt2d(n, smooth=False)
    K = kernels.dense_matrix(kern)
    g_tree = complex_gaussian((n * n,), 5)
    a1, a2 = kernels.morton_decode(np.arange(n * n), bits)
    g_grid = np.zeros((n, n), dtype=complex)
    g_grid[a1, a2] = g_tree
    u_grid = ((-1.0) ** (np.arange(n)[:, None] + np.arange(n)[None, :])) * n * n * np.fft.ifft2(g_grid)
    u_tree = u_grid[a1, a2]
    assert np.abs(K @ g_tree - u_tree).max() <= 1e-12 * np.abs(u_tree).max()


def test_grt_hand_values():
    bits = 4
    n = 1 << bits
    kern = kernels.grt2d(n)
    # x = (0,0): c1 = 1/8, c2 = 3/16; xi = (-8, 0) -> Phi = sqrt((1/8)^2 64) = 1 -> K = 1
    row = _morton_encode(0, 0, bits)
    col = _morton_encode(0, n // 2, bits)
    assert abs(kern.entries([row], [col])[0, 0] - 1.0) < 1e-13
    # x = (1/4, 1/4): c2 = 2/16; xi = (0, 4): Phi = 1 + (1/8)*4 = 3/2 -> K = -1
    row = _morton_encode(n // 4, n // 4, bits)
    col = _morton_encode(n // 2, n // 2 + 4, bits)
    assert abs(kern.entries([row], [col])[0, 0] - (-1.0)) < 1e-13


def test_hankel_entries_satisfy_recurrence():
    # Example 2: K_ij = H^(1)_j(x_i); H_{v+1}(x) + H_{v-1}(x) = (2v/x) H_v(x)
    N = 64
    kern = kernels.HankelSum(N)
    rows = np.array([0, 5, 63])
    K = kern.entries(rows, np.arange(N))
    x = N + (2 * np.pi / 3) * rows
    for v in range(1, N - 1):
        lhs = K[:, v + 1] + K[:, v - 1]
        rhs = (2 * v / x) * K[:, v]
        assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(K[:, v]).max() + 1e-14
    assert abs(K[0, 0] - hankel1(0, N)) < 1e-15


def test_dense_apply_rows():
    N = 512
    kern = kernels.fio(N)
    g = complex_gaussian((N, 2), 3)
    rows = np.array([0, 17, 300, 511])
    u = kernels.dense_apply_rows(kern, rows, g, col_chunk=100)
    ref = kern.entries(rows, np.arange(N)) @ g
    assert np.abs(u - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("N", [64, 1024])
def test_hankel_points_from_the_wronskian(N):
    # Example 2 places row i (0-based) at x_i = N + (2 pi / 3) i.  For Hankel
    # functions of the first kind, J_{v+1} Y_v - J_v Y_{v+1} = 2 / (pi x), so
    # Im(H_{v+1}(x) conj(H_v(x))) = -2 / (pi x): two neighbouring columns of a
    # row give back that row's point, whatever the entries' formula says.
    kern = kernels.HankelSum(N)
    rows = np.array([0, 1, 2, 7, N // 2 + 3, N - 1])
    for v in (0, 5, N // 3, N - 2):
        K = kern.entries(rows, np.array([v, v + 1]))
        w = np.imag(K[:, 1] * np.conj(K[:, 0]))
        x = -2.0 / (np.pi * w)
        expect = N + (2.0 * np.pi / 3.0) * rows
        assert np.abs(x / expect - 1).max() < 1e-10
