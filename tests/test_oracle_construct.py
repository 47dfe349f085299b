"""Pins for the oracle's construction of the factorization (CPU only)."""
import numpy as np
import pytest

import oracle
from bf_inputs import complex_gaussian
from oracle import kernels, lowrank
from oracle.construct import construct_factors, tree_depth


def _err_vs_dense(kern, f, nrhs=4, seed=7):
    g = complex_gaussian((kern.N, nrhs), seed)
    ud = kernels.dense_matrix(kern) @ g
    return oracle.rel_err(oracle.bf_apply(f, g), ud)


@pytest.mark.parametrize("method", ["svd", "sampling"])
def test_full_rank_is_exact_1d(method):
    # r >= every block dimension: every truncation is exact, so K_BF = K
    kern = kernels.fio(64)
    f = construct_factors(kern, leaf=4, r=16, method=method, seed=1)
    assert _err_vs_dense(kern, f) < 1e-13


def test_full_rank_is_exact_2d():
    kern = kernels.grt2d(16)
    f = construct_factors(kern, leaf=1, r=16, method="svd")
    assert f["L"] == 4 and f["radix"] == 4
    assert _err_vs_dense(kern, f) < 1e-13


def test_full_rank_is_exact_radix4_padded_leaves():
    # 2D leaves with fewer points than r: leaf blocks and G/H blocks are zero-padded to r
    kern = kernels.grt2d(16)
    f = construct_factors(kern, leaf=16, r=64, method="svd")
    assert f["UL"].shape == (16, 16, 64)
    assert _err_vs_dense(kern, f) < 1e-13


def test_low_rank_kernel_is_recovered_by_sampling():
    # K = A B^T of rank 5 has rank <= 5 in every block, so rank-8 sampling is exact
    N = 1024
    rng = np.random.default_rng(0)
    x = np.arange(N) / N
    A = np.stack([np.cos(2 * np.pi * t * x) + 1j * np.sin(3 * np.pi * t * x) for t in range(5)], 1)
    B = rng.standard_normal((N, 5)) + 1j * rng.standard_normal((N, 5))
    kern = kernels.LowRankKernel(A, B)
    f = construct_factors(kern, leaf=16, r=8, method="sampling", seed=2)
    assert _err_vs_dense(kern, f) < 1e-11


def test_sampling_tracks_truncated_svd_and_improves_with_rank():
    # one point per leaf, as in the paper's figures; FIO of Example 1
    kern = kernels.fio(256)
    errs_s, errs_v = [], []
    for r in (4, 6, 8):
        errs_s.append(_err_vs_dense(kern, construct_factors(kern, 1, r, "sampling", seed=0)))
        errs_v.append(_err_vs_dense(kern, construct_factors(kern, 1, r, "svd")))
    for es, ev in zip(errs_s, errs_v):
        assert es < 10 * ev
    assert errs_s[0] > errs_s[1] > errs_s[2]
    assert errs_s[2] < 1e-5


def test_error_bounded_below_by_dropped_singular_values():
    # the factorization restricted to a middle block has rank <= r (Sec. 3.1), so by
    # Eckart-Young E||(K - K_BF) g||^2 >= sum over middle blocks of sum_{k>r} sigma_k^2
    N, leaf, r = 1024, 16, 16
    kern = kernels.fourier(N)
    f = construct_factors(kern, leaf, r, "svd")
    K = kernels.dense_matrix(kern)
    L = f["L"]
    m = 2 ** (L // 2)
    b = N // m
    tail = 0.0
    for i in range(m):
        for j in range(m):
            s = np.linalg.svd(K[i * b:(i + 1) * b, j * b:(j + 1) * b], compute_uv=False)
            tail += np.sum(s[r:] ** 2)
    E = K - np.stack([oracle.bf_apply(f, e) for e in np.eye(N)], 1)
    fro2 = np.sum(np.abs(E) ** 2)
    assert fro2 >= tail * (1 - 1e-9)
    assert fro2 < 50 * tail          # the recursion adds error of the same order


def test_fourier_rank32_reaches_1e8():
    kern = kernels.fourier(1024)
    f = construct_factors(kern, 16, 32, "svd")
    assert _err_vs_dense(kern, f, nrhs=2) < 1e-8


def test_streamed_order_gives_identical_factors():
    kern = kernels.fio(256)
    a = construct_factors(kern, 4, 6, "sampling", seed=5, streamed=True)
    b = construct_factors(kern, 4, 6, "sampling", seed=5, streamed=False)
    for key in ("VL", "UL", "S"):
        assert np.array_equal(a[key], b[key])
    for key in ("H", "G"):
        for x, y in zip(a[key], b[key]):
            assert np.array_equal(x, y)


def test_factor_shapes_and_depth_checks():
    kern = kernels.fio(256)
    f = construct_factors(kern, 4, 5, "svd")
    L, h = f["L"], f["L"] // 2
    assert L == 6
    for t, l in enumerate(range(h, L)):
        assert f["G"][t].shape == (2 ** (l + 1), 2 ** (L - l - 1), 5, 10)
        assert f["H"][t].shape == (2 ** (l + 1), 2 ** (L - l - 1), 5, 10)
    assert f["S"].shape == (8, 8, 5)
    with pytest.raises(ValueError):
        tree_depth(256, 8, 2)            # L = 5 is odd
    with pytest.raises(ValueError):
        tree_depth(250, 4, 2)


def test_randomized_sampling_on_exact_low_rank_matrix():
    rng = np.random.default_rng(4)
    Z = (rng.standard_normal((200, 6)) @ rng.standard_normal((6, 150))).astype(complex)
    U0, s, V0h = lowrank.randomized_sampling(lambda I, J: Z[np.ix_(I, J)], 200, 150, 8, rng)
    assert np.abs(U0 @ np.diag(s) @ V0h - Z).max() < 1e-10 * np.abs(Z).max()
    assert np.allclose(U0[:, :6].conj().T @ U0[:, :6], np.eye(6), atol=1e-10)


def test_randomized_svd_on_exact_low_rank_matrix():
    rng = np.random.default_rng(9)
    Z = rng.standard_normal((120, 7)) @ rng.standard_normal((7, 90)) + 0j
    U0, s, V0h = lowrank.randomized_svd(lambda C: Z @ C, lambda R: Z.conj().T @ R,
                                        120, 90, 7, rng)
    assert np.abs(U0 @ np.diag(s) @ V0h - Z).max() < 1e-10 * np.abs(Z).max()
    assert s == pytest.approx(np.linalg.svd(Z, compute_uv=False)[:7], rel=1e-10)


def test_middle_form_drops_null_directions():
    U0 = np.eye(4, 3, dtype=complex)
    V0h = np.eye(3, 5, dtype=complex)
    s = np.array([2.0, 1e-20, 0.0])
    U, S, V = lowrank.form_usv(U0, s, V0h)
    assert np.all(np.isfinite(S)) and S[0] == 0.5 and S[1] == 0 and S[2] == 0
    assert np.abs(U @ np.diag(S) @ V.conj().T - U0[:, :1] @ V0h[:1] * 2).max() < 1e-15


# ---- construction from products with K and K^* (Alg. 2.1, first case of Sec. 3.1)

def _fourier_fft_box(N):
    # K_{jk} = (-1)^j e^{2 pi i j k / N}: K g = (-1)^j N ifft(g), K^* w = fft((-1)^j w)
    sign = (-1.0) ** np.arange(N)
    return (lambda X: sign[:, None] * N * np.fft.ifft(X, axis=0),
            lambda X: np.fft.fft(sign[:, None] * X, axis=0))


def test_matvec_construction_full_rank_is_exact():
    # r >= every block dimension: the sketches span every block, so K_BF = K
    kern = kernels.fio(64)
    K = kernels.dense_matrix(kern)
    f = oracle.construct_factors_matvec(64, 2, 4, 16, lambda X: K @ X, lambda X: K.conj().T @ X,
                                        seed=3)
    assert _err_vs_dense(kern, f) < 1e-12


def test_matvec_construction_recovers_an_exact_butterfly():
    # K is itself a butterfly of rank 3: every middle block and every recursion block
    # has rank <= 3, so rank 5 reproduces K up to rounding
    from bf_inputs import synthetic_factors
    fs = synthetic_factors(2, 4, 6, 3, seed=5)
    N = 256
    K = oracle.bf_apply(fs, np.eye(N, dtype=complex))
    f = oracle.construct_factors_matvec(N, 2, 4, 5, lambda X: K @ X, lambda X: K.conj().T @ X,
                                        seed=6)
    assert oracle.rel_err(oracle.bf_apply(f, np.eye(N)), K) < 1e-11


def test_matvec_construction_with_fft_black_box():
    # the Fourier kernel through the FFT only (K is never formed): the same factors as
    # with the dense black box up to rounding, and the accuracy of the entry-sampling
    # route at the same rank
    N, r = 1024, 24
    kern = kernels.fourier(N)
    K = kernels.dense_matrix(kern)
    mv, rmv = _fourier_fft_box(N)
    g = complex_gaussian((N, 3), 8)
    assert oracle.rel_err(mv(g), K @ g) < 1e-13 and oracle.rel_err(rmv(g), K.conj().T @ g) < 1e-13
    f_fft = oracle.construct_factors_matvec(N, 2, 16, r, mv, rmv, seed=9)
    f_dense = oracle.construct_factors_matvec(N, 2, 16, r, lambda X: K @ X,
                                              lambda X: K.conj().T @ X, seed=9)
    u_fft, u_dense = oracle.bf_apply(f_fft, g), oracle.bf_apply(f_dense, g)
    assert oracle.rel_err(u_fft, u_dense) < 1e-9
    e_mv = oracle.rel_err(u_fft, K @ g)
    e_s = _err_vs_dense(kern, construct_factors(kern, leaf=16, r=r, method="sampling", seed=0), 3, 8)
    assert e_mv < 1e-3 and e_mv < 10 * e_s


def test_middle_from_sketches_is_exact_for_low_rank_blocks():
    rng = np.random.default_rng(4)
    A = (rng.standard_normal((40, 6)) + 1j * rng.standard_normal((40, 6)))
    B = (rng.standard_normal((30, 6)) + 1j * rng.standard_normal((30, 6)))
    Z = A @ B.conj().T                                   # rank 6
    C = rng.standard_normal((30, 13)) + 1j * rng.standard_normal((30, 13))
    Rr = rng.standard_normal((40, 13)) + 1j * rng.standard_normal((40, 13))
    U0, s, V0h = oracle.construct.middle_from_sketches(Z @ C, Z.conj().T @ Rr, C, 8)
    assert np.linalg.norm(U0 * s @ V0h - Z) < 1e-12 * np.linalg.norm(Z)
    assert np.all(np.diff(s) <= 1e-12)                   # decreasing
