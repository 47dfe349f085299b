"""Host linear algebra of the construction from products (CPU; the black box is a
dense matrix or an FFT on CPU tensors), pinned like the oracle's."""
import numpy as np
import pytest

import oracle
from bf_inputs import complex_gaussian, synthetic_factors
from oracle import kernels

torch = pytest.importorskip("torch")


def _dense_box(K):
    Kt = torch.from_numpy(K)
    return (lambda X: Kt @ X, lambda X: Kt.conj().T @ X)


def test_full_rank_is_exact():
    from paper_1502_01379_amd.construct import construct_from_products
    kern = kernels.fio(64)
    K = kernels.dense_matrix(kern)
    f = construct_from_products(64, 2, 4, 16, *_dense_box(K), seed=3, device="cpu")
    g = complex_gaussian((64, 3), 1)
    assert oracle.rel_err(oracle.bf_apply(f, g), K @ g) < 1e-12


@pytest.mark.parametrize("radix,leaf,L,r0", [(2, 4, 6, 3), (4, 2, 4, 2)])
def test_recovers_an_exact_butterfly(radix, leaf, L, r0):
    from paper_1502_01379_amd.construct import construct_from_products
    fs = synthetic_factors(radix, leaf, L, r0, seed=5)
    N = leaf * radix ** L
    K = oracle.bf_apply(fs, np.eye(N, dtype=complex))
    f = construct_from_products(N, radix, leaf, r0 + 2, *_dense_box(K), seed=6, device="cpu")
    assert oracle.rel_err(oracle.bf_apply(f, np.eye(N)), K) < 1e-11


def test_fourier_through_fft_matches_oracle_accuracy():
    from paper_1502_01379_amd.construct import construct_from_products
    N, r = 1024, 24
    K = kernels.dense_matrix(kernels.fourier(N))
    sign = torch.tensor((-1.0) ** np.arange(N))[:, None]
    mv = lambda X: sign * N * torch.fft.ifft(X, dim=0)
    rmv = lambda X: torch.fft.fft(sign * X, dim=0)
    f = construct_from_products(N, 2, 16, r, mv, rmv, seed=9, device="cpu")
    g = complex_gaussian((N, 3), 8)
    e_lib = oracle.rel_err(oracle.bf_apply(f, g), K @ g)
    fo = oracle.construct_factors_matvec(N, 2, 16, r, lambda X: K @ X, lambda X: K.conj().T @ X, seed=9)
    e_ora = oracle.rel_err(oracle.bf_apply(fo, g), K @ g)
    assert e_lib < 3 * e_ora + 1e-12


def test_entries_full_rank_is_exact():
    """Rank r equal to the middle block size: the sampled SVD is exact (Alg. 2.2)."""
    from paper_1502_01379_amd.construct import construct_from_entries
    kern = kernels.fio(64)
    K = kernels.dense_matrix(kern)
    f = construct_from_entries(64, 2, 4, 16, kern.entries, seed=3)
    g = complex_gaussian((64, 3), 1)
    assert oracle.rel_err(oracle.bf_apply(f, g), K @ g) < 1e-12


def test_entries_recovers_a_low_rank_kernel():
    """Every block of A B^T has rank 5: the sampled factorization reproduces it."""
    from paper_1502_01379_amd.construct import construct_from_entries
    N = 256
    rng = np.random.default_rng(4)
    A = rng.standard_normal((N, 5)) + 1j * rng.standard_normal((N, 5))
    B = rng.standard_normal((N, 5)) + 1j * rng.standard_normal((N, 5))
    kern = kernels.LowRankKernel(A, B)
    f = construct_from_entries(N, 2, 4, 7, kern.entries, seed=2)
    assert oracle.rel_err(oracle.bf_apply(f, np.eye(N)), A @ B.T) < 1e-11


@pytest.mark.parametrize("radix,leaf,L,r0", [(2, 4, 6, 3), (4, 2, 4, 2)])
def test_entries_recovers_an_exact_butterfly(radix, leaf, L, r0):
    from paper_1502_01379_amd.construct import construct_from_entries
    fs = synthetic_factors(radix, leaf, L, r0, seed=5)
    N = leaf * radix ** L
    K = oracle.bf_apply(fs, np.eye(N, dtype=complex))
    f = construct_from_entries(N, radix, leaf, r0 + 2, lambda I, J: K[np.ix_(I, J)], seed=6)
    assert oracle.rel_err(oracle.bf_apply(f, np.eye(N)), K) < 1e-11


def test_entries_fourier_matches_oracle_accuracy():
    """Same accuracy as the oracle's sampling construction on the Fourier kernel."""
    from paper_1502_01379_amd.construct import construct_from_entries
    N, r = 1024, 24
    kern = kernels.fourier(N)
    K = kernels.dense_matrix(kern)
    g = complex_gaussian((N, 3), 8)
    f = construct_from_entries(N, 2, 16, r, kern.entries, seed=9)
    e_lib = oracle.rel_err(oracle.bf_apply(f, g), K @ g)
    fo = oracle.construct_factors(kern, leaf=16, r=r, method="sampling", seed=9)
    e_ora = oracle.rel_err(oracle.bf_apply(fo, g), K @ g)
    assert e_lib < 3 * e_ora + 1e-12


def test_entries_seed_fixes_the_result():
    from paper_1502_01379_amd.construct import construct_from_entries
    kern = kernels.fio(256)
    a = construct_from_entries(256, 2, 4, 8, kern.entries, seed=1)
    b = construct_from_entries(256, 2, 4, 8, kern.entries, seed=1)
    for key in ("VL", "UL", "S"):
        assert np.array_equal(a[key], b[key])


@pytest.mark.parametrize("radix,N,leaf,r", [(2, 4096, 16, 16), (4, 1024, 4, 8), (2, 1024, 1, 6)])
def test_streamed_order_gives_the_same_factors(radix, N, leaf, r):
    # Sec. 3.3: one middle node at a time (U side by rows, V side by columns, every
    # block from its own random stream) reproduces the all-at-once factors exactly
    from paper_1502_01379_amd.construct import construct_from_entries
    kern = kernels.fio(N) if radix == 2 else kernels.grt2d(int(round(N ** 0.5)))
    a = construct_from_entries(N, radix, leaf, r, kern.entries, seed=5, streamed=False)
    b = construct_from_entries(N, radix, leaf, r, kern.entries, seed=5, streamed=True)
    for key in ("VL", "UL", "S"):
        assert np.array_equal(a[key], b[key]), key
    for t in range(len(a["G"])):
        assert np.array_equal(a["G"][t], b["G"][t]) and np.array_equal(a["H"][t], b["H"][t]), t
