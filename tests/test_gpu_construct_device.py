"""Construction on the GPU (include/bf_construct.h): the batched FP64 primitives
against LAPACK/NumPy and the definitions they compute, and the whole
entry-sampling construction (Alg. 2.2 + Sec. 3.2) against the dense kernel and
the oracle's construction of the same kernel.

The device draws its own random samples (SplitMix64), so its factors differ from
the oracle's; what is compared is what the method fixes: exactness at full rank
and the approximation error, which must match the oracle's."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from bf_inputs import complex_gaussian
from oracle import kernels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _c(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.complex128)).to(dev)


@pytest.mark.parametrize("name", ["fourier", "fio"])
def test_kernel_entries_match_oracle(dev, name):
    from paper_1502_01379_amd import kernel_entries
    N = 1 << 16
    kern = kernels.fio(N) if name == "fio" else kernels.fourier(N)
    rng = np.random.default_rng(1)
    rows = np.concatenate([[0, N - 1, N // 2], rng.integers(0, N, 300)])
    cols = np.concatenate([[0, N - 1, N // 2, N // 2 - 1], rng.integers(0, N, 200)])
    got = kernel_entries(name, N, torch.tensor(rows, device=dev), torch.tensor(cols, device=dev)).cpu().numpy()
    ref = kern.entries(rows, cols)
    # |phase error| <= c |xi| eps ~ 1e-12 at N = 2^16
    assert np.max(np.abs(got - ref)) < 1e-10


@pytest.mark.parametrize("m,n,rank", [(64, 16, None), (128, 32, None), (96, 24, None), (64, 64, None),
                                      (48, 48, 5), (5, 3, None), (3, 5, None), (1, 1, None), (64, 32, 7)])
def test_batched_svd(dev, m, n, rank):
    from paper_1502_01379_amd import batched_svd
    bt = 7
    A = complex_gaussian((bt, m, n), m + n)
    if rank is not None:
        A = complex_gaussian((bt, m, rank), 3) @ complex_gaussian((bt, rank, n), 4)
    A[1] *= 1e-3                     # scale invariance
    A[2, :, 0] = 0                   # a zero column
    U, s, V = (t.cpu().numpy() for t in batched_svd(_c(A, dev)))
    for b in range(bt):
        sref = np.linalg.svd(A[b], compute_uv=False)
        sfull = np.zeros(n)
        sfull[:sref.size] = sref
        smax = max(sref[0], 1e-300)
        assert np.allclose(s[b], sfull, rtol=0, atol=1e-13 * smax), b
        assert np.all(np.diff(s[b]) <= 1e-14 * smax)
        assert np.linalg.norm(U[b] * s[b] @ V[b].conj().T - A[b]) <= 1e-13 * np.linalg.norm(A[b])
        assert np.linalg.norm(V[b].conj().T @ V[b] - np.eye(n)) < 1e-13
        nz = s[b] > 1e-10 * smax
        Unz = U[b][:, nz]
        assert np.linalg.norm(Unz.conj().T @ Unz - np.eye(nz.sum())) < 1e-12
        assert np.all(U[b][:, s[b] == 0] == 0)


@pytest.mark.parametrize("n,k,rank", [(1024, 16, None), (200, 64, None), (8, 32, None), (500, 20, 7),
                                      (3000, 32, None), (1, 4, None)])
def test_batched_qr(dev, n, k, rank):
    from paper_1502_01379_amd import batched_qr
    bt = 5
    A = complex_gaussian((bt, n, k), n + k)
    if rank is not None:
        A = complex_gaussian((bt, n, rank), 5) @ complex_gaussian((bt, rank, k), 6)
    A[1] *= 1e5
    Q, R = (t.cpu().numpy() for t in batched_qr(_c(A, dev)))
    for b in range(bt):
        assert np.linalg.norm(Q[b] @ R[b] - A[b]) <= 1e-13 * np.linalg.norm(A[b])
        assert np.all(np.tril(R[b], -1) == 0)
        d = np.diag(R[b])
        assert np.all(d.imag == 0) and np.all(d.real >= 0)
        nz = d.real > 0
        assert nz.sum() == min(n, k, rank or k)
        Qn = Q[b][:, nz]
        assert np.linalg.norm(Qn.conj().T @ Qn - np.eye(nz.sum())) < 1e-12
        assert np.all(Q[b][:, ~nz] == 0)
        if rank is None and n >= k:       # R is unique up to column phases
            Rl = np.linalg.qr(A[b], mode="r")
            assert np.allclose(np.abs(np.diag(Rl)), d.real, rtol=1e-10)


@pytest.mark.parametrize("p,n,npiv", [(64, 1024, 16), (48, 512, 24), (128, 300, 32), (16, 16, 16), (7, 90, 5)])
def test_column_pivots_match_lapack(dev, p, n, npiv):
    from paper_1502_01379_amd import batched_column_pivots
    bt = 6
    A = complex_gaussian((bt, p, n), p * n)
    A[1] *= np.exp(-0.05 * np.arange(n))[None, :]        # graded columns
    A[2] = A[2][:, ::-1].copy()
    piv = batched_column_pivots(_c(A, dev), npiv).cpu().numpy()
    for b in range(bt):
        ref = sla.qr(A[b], mode="r", pivoting=True)[1][:npiv]
        assert np.array_equal(piv[b], ref), (b, piv[b], ref)


def test_column_pivots_take_the_first_on_ties(dev):
    from paper_1502_01379_amd import batched_column_pivots
    A = np.zeros((1, 4, 6), dtype=complex)
    A[0, :, 3] = [1, 0, 0, 0]
    A[0, :, 1] = [0, 1, 0, 0]
    A[0, :, 5] = [0, 0, 1, 0]
    piv = batched_column_pivots(_c(A, dev), 4).cpu().numpy()[0]
    assert list(piv[:3]) == [1, 3, 5] and piv[3] == 0


_DRIVER_OFF = pytest.mark.skip(
    reason="bf_construct_from_kernel is switched off: on the GPU it gave 1.5e-3 instead of the 1.1e-4 "
           "its host run reaches (Fourier, N = 1024, r = 24) and an illegal memory access at N = 512 "
           "with 128-point leaves; the cause is not found")


def _err_vs_dense(f, K, seed=8):
    g = complex_gaussian((K.shape[1], 3), seed)
    return oracle.rel_err(oracle.bf_apply(f, g), K @ g)


@_DRIVER_OFF
@pytest.mark.parametrize("radix,N,leaf,r,name", [(2, 64, 4, 16, "fio"), (4, 64, 4, 16, "fourier"),
                                                 (2, 512, 2, 32, "fio")])
def test_device_construction_full_rank_is_exact(dev, radix, N, leaf, r, name):
    """r equal to the middle block size b: every low-rank step is exact."""
    from paper_1502_01379_amd import construct_on_device
    f = construct_on_device(N, radix, leaf, r, kernel=name, seed=3)
    kern = kernels.fio(N) if name == "fio" else kernels.fourier(N)
    assert _err_vs_dense(f, kernels.dense_matrix(kern)) < 1e-10


@_DRIVER_OFF
@pytest.mark.parametrize("N,leaf,r,name", [(1024, 16, 24, "fourier"), (1024, 1, 8, "fio"), (2048, 2, 10, "fio")])
def test_device_construction_matches_oracle_accuracy(dev, N, leaf, r, name):
    from paper_1502_01379_amd import construct_on_device
    kern = kernels.fio(N) if name == "fio" else kernels.fourier(N)
    K = kernels.dense_matrix(kern)
    e_dev = _err_vs_dense(construct_on_device(N, 2, leaf, r, kernel=name, seed=9), K)
    e_ora = _err_vs_dense(oracle.construct_factors(kern, leaf, r, "sampling", seed=9), K)
    print(f"N={N} leaf={leaf} r={r} {name}: device {e_dev:.3e} oracle {e_ora:.3e}", flush=True)
    assert e_dev < 3 * e_ora + 1e-12


@_DRIVER_OFF
def test_device_construction_is_deterministic_and_feeds_the_apply(dev):
    """Same seed, same factors; the factors go straight into the FP32 fused apply."""
    from paper_1502_01379_amd import BFHandle, construct_on_device
    N = 1 << 14
    f1 = construct_on_device(N, 2, 16, 16, kernel="fio", seed=4)
    f2 = construct_on_device(N, 2, 16, 16, kernel="fio", seed=4)
    for key in ("VL", "UL", "S"):
        assert np.array_equal(f1[key], f2[key])
    for t in range(len(f1["G"])):
        assert np.array_equal(f1["G"][t], f2["G"][t]) and np.array_equal(f1["H"][t], f2["H"][t])
    h = BFHandle(f1, "f32")
    g = complex_gaussian((N, 4), 2)
    u = h.apply(torch.as_tensor(g).to(dev, torch.complex64)).cpu().numpy()
    assert oracle.rel_err(u, oracle.bf_apply(f1, g)) < 1e-5
    h.close()


def test_device_construction_is_switched_off(dev):
    from paper_1502_01379_amd import BFError, construct_on_device
    with pytest.raises(BFError, match="switched off"):
        construct_on_device(64, 2, 4, 16, kernel="fio", seed=3)
