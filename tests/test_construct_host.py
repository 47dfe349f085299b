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
