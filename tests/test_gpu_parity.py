"""GPU apply / adjoint / backward vs the FP64 oracle on identical factors.

Tolerances are relative l2 errors over every compared entry: 1e-10 for the
FP64 path, 1e-5 for FP32 and 1e-4 for split BF16 (the stated budgets for
this library); FP16 split is held to 1e-5.
"""
import numpy as np
import pytest

import oracle
from bf_inputs import complex_gaussian, synthetic_factors
from oracle import kernels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5, "bf16x3": 1e-4, "f16x3": 1e-5}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_01379_amd import load_library
    load_library()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def fourier1024():
    # the Fourier matrix of Sec. 1.1 (shifted frequencies), N = 1024, leaf 16, r = 12
    return oracle.construct_factors(kernels.fourier(1024), leaf=16, r=12, method="sampling", seed=0)


@pytest.fixture(scope="module")
def fio4096():
    return oracle.construct_factors(kernels.fio(4096), leaf=16, r=16, method="sampling", seed=0)


def _to(x, dev, prec):
    cd = torch.complex128 if prec == "f64" else torch.complex64
    return torch.as_tensor(x).to(dev, cd)


def _handle(f, prec):
    from paper_1502_01379_amd import BFHandle
    return BFHandle(f, prec)


def test_fourier_f64_one_rhs(dev, fourier1024):
    f = fourier1024
    g = complex_gaussian((1024,), 3)
    h = _handle(f, "f64")
    u = h.apply(_to(g, dev, "f64")).cpu().numpy()
    ref = oracle.bf_apply(f, g)
    assert oracle.rel_err(u, ref) < TOL["f64"]
    # the factorization approximates K: rank 12 is well below the blocks' numerical rank,
    # so the approximation error is O(1) here; the GPU agrees with the oracle regardless
    dense = ((-1.0) ** np.arange(1024)) * 1024 * np.fft.ifft(g)
    e_gpu, e_ora = oracle.rel_err(u, dense), oracle.rel_err(ref, dense)
    assert abs(e_gpu - e_ora) < 1e-8


@pytest.mark.parametrize("radix,leaf,L,r", [(2, 4, 4, 3), (4, 2, 2, 3), (2, 1, 6, 2)])
def test_unit_vectors_reproduce_oracle_columns(dev, radix, leaf, L, r):
    f = synthetic_factors(radix, leaf, L, r, seed=radix + L)
    N = leaf * radix ** L
    eye = np.eye(N, dtype=complex)
    h = _handle(f, "f64")
    cols = h.apply(_to(eye, dev, "f64")).cpu().numpy()
    ref = oracle.bf_apply(f, eye)
    assert np.abs(cols - ref).max() <= 1e-13 * np.abs(ref).max()
    adj = h.apply_adjoint(_to(eye, dev, "f64")).cpu().numpy()
    assert np.abs(adj - ref.conj().T).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nrhs,pad", [(64, 0), (1, 0), (33, 3), (70, 5)])
def test_fio_apply_and_adjoint(dev, fio4096, prec, nrhs, pad):
    f = fio4096
    N = 4096
    g = complex_gaussian((N, nrhs), nrhs)
    gl = np.zeros((N, nrhs + pad), dtype=complex)
    gl[:, :nrhs] = g
    gd = _to(gl, dev, prec)[:, :nrhs]
    h = _handle(f, prec)
    u = h.apply(gd).cpu().numpy()
    assert oracle.rel_err(u, oracle.bf_apply(f, g)) < TOL[prec]
    v = h.apply_adjoint(gd).cpu().numpy()
    assert oracle.rel_err(v, oracle.bf_apply_adjoint(f, g)) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_radix4_grt(dev, prec):
    kern = kernels.grt2d(32)                   # N = 1024, quadtree, leaf 4 (2 x 2), L = 4
    f = oracle.construct_factors(kern, leaf=4, r=8, method="sampling", seed=1)
    g = complex_gaussian((kern.N, 9), 4)
    h = _handle(f, prec)
    u = h.apply(_to(g, dev, prec)).cpu().numpy()
    assert oracle.rel_err(u, oracle.bf_apply(f, g)) < TOL[prec]
    v = h.apply_adjoint(_to(g, dev, prec)).cpu().numpy()
    assert oracle.rel_err(v, oracle.bf_apply_adjoint(f, g)) < TOL[prec]


def _flat_grads(d, h):
    return [d["VL"], d["UL"], d["S"], *d["H"], *d["G"]]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_backward_matches_oracle_gradient(dev, fio4096, prec):
    from paper_1502_01379_amd import BF_BWD_STORE_ALL
    f = fio4096
    N, nrhs = 4096, 40
    g = complex_gaussian((N, nrhs), 7)
    y = complex_gaussian((N, nrhs), 8)
    gu = 2 * (oracle.bf_apply(f, g) - y)
    ref = oracle.bf_grad(f, g, gu)
    h = _handle(f, prec)
    grad_g, grads = h.backward(_to(g, dev, prec), _to(gu, dev, prec))
    assert oracle.rel_err(grad_g.cpu().numpy(), ref["g"]) < TOL[prec]
    errs = [oracle.rel_err(a.cpu().numpy(), b) for a, b in zip(_flat_grads(grads, h), _flat_grads(ref, h))]
    print(f"per-level {prec} factor gradient errors: max {max(errs):.3e}", flush=True)
    assert max(errs) < TOL[prec]
    # keeping every level gives the same numbers as recomputing them
    grad_g2, grads2 = h.backward(_to(g, dev, prec), _to(gu, dev, prec), flags=BF_BWD_STORE_ALL)
    assert torch.equal(grad_g, grad_g2)
    for a, b in zip(_flat_grads(grads, h), _flat_grads(grads2, h)):
        assert torch.equal(a, b)


def test_bad_arguments_on_device(dev, fio4096):
    from paper_1502_01379_amd import binding as B
    h = _handle(fio4096, "f32")
    x = torch.zeros((4096, 8), dtype=torch.complex64, device=dev)
    y = torch.zeros((4096, 8), dtype=torch.complex64, device=dev)
    assert B.bf_apply(h.handle, x.data_ptr(), y.data_ptr(), 0, 8) == B.BF_ERR_INVALID_ARG
    assert B.bf_apply(h.handle, x.data_ptr(), y.data_ptr(), 8, 4) == B.BF_ERR_INVALID_ARG
    assert B.bf_apply(h.handle, x.data_ptr(), x.data_ptr(), 8, 8) == B.BF_ERR_INVALID_ARG
    assert B.bf_apply(h.handle, 0, y.data_ptr(), 8, 8) == B.BF_ERR_INVALID_ARG
    assert "overlap" in B.bf_last_error(h.handle) or "NULL" in B.bf_last_error(h.handle)
    assert B.bf_apply(h.handle, x.data_ptr(), y.data_ptr(), 8, 8) == B.BF_OK


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_repeated_calls_are_bitwise_identical(dev, fio4096, prec):
    g = _to(complex_gaussian((4096, 48), 9), dev, prec)
    h = _handle(fio4096, prec)
    u0 = h.apply(g).clone()
    for _ in range(5):
        assert torch.equal(h.apply(g), u0)


def test_full_size_fio_65536_f32(dev):
    # N = 65536, leaf 16, r = 16 (L = 12), 64 right-hand sides; synthetic factors of the
    # real shapes (values do not matter for parity on identical factors)
    f = synthetic_factors(2, 16, 12, 16, seed=11)
    N = 65536
    g = complex_gaussian((N, 64), 12)
    h = _handle(f, "f32")
    u = h.apply(_to(g, dev, "f32")).cpu().numpy()
    cols = [0, 17, 63]
    ref = oracle.bf_apply(f, g[:, cols])
    assert oracle.rel_err(u[:, cols], ref) < TOL["f32"]


def test_full_size_grt_radix4_65536_f32(dev):
    # the 2D generalized Radon transform shape: 256 x 256 points (N = 65536), quadtrees
    # with 4 x 4 leaves (radix 4, L = 6), r = 32, 128 right-hand sides; synthetic factors
    # of those shapes; apply and adjoint on sampled columns against the oracle
    f = synthetic_factors(4, 16, 6, 32, seed=13)
    N = 65536
    g = complex_gaussian((N, 128), 14)
    h = _handle(f, "f32")
    gd = _to(g, dev, "f32")
    u = h.apply(gd).cpu().numpy()
    v = h.apply_adjoint(gd).cpu().numpy()
    cols = [0, 77, 127]
    assert oracle.rel_err(u[:, cols], oracle.bf_apply(f, g[:, cols])) < TOL["f32"]
    assert oracle.rel_err(v[:, cols], oracle.bf_apply_adjoint(f, g[:, cols])) < TOL["f32"]


@pytest.mark.parametrize("radix,leaf,L,r", [(4, 16, 2, 8), (4, 4, 4, 16), (2, 8, 6, 32),
                                             (4, 16, 4, 32), (2, 16, 4, 64)])
@pytest.mark.parametrize("nrhs", [1, 31, 70])
def test_level_mfma_shapes(dev, radix, leaf, L, r, nrhs):
    # per-level butterflies on the matrix cores (R r = 32, 64, 128 blocks; both slot
    # patterns; ragged 32-column chunks), apply, adjoint and backward, FP32
    f = synthetic_factors(radix, leaf, L, r, seed=7 * radix + L + r)
    N = leaf * radix ** L
    g = complex_gaussian((N, nrhs), r + nrhs)
    gu = complex_gaussian((N, nrhs), r + nrhs + 1)
    h = _handle(f, "f32")
    assert h.path == 0
    u = h.apply(_to(g, dev, "f32")).cpu().numpy()
    assert oracle.rel_err(u, oracle.bf_apply(f, g)) < TOL["f32"]
    v = h.apply_adjoint(_to(g, dev, "f32")).cpu().numpy()
    assert oracle.rel_err(v, oracle.bf_apply_adjoint(f, g)) < TOL["f32"]
    grad_g, grads = h.backward(_to(g, dev, "f32"), _to(gu, dev, "f32"))
    ref = oracle.bf_grad(f, g, gu)
    assert oracle.rel_err(grad_g.cpu().numpy(), ref["g"]) < TOL["f32"]
    errs = [oracle.rel_err(a.cpu().numpy(), b) for a, b in zip(_flat_grads(grads, h), _flat_grads(ref, h))]
    print(f"per-level MFMA factor gradient errors: max {max(errs):.3e}", flush=True)
    assert max(errs) < TOL["f32"]


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_hankel_sum_workload(dev, prec):
    # Example 2 of Sec. 4 (sums of Hankel functions H^(1)_nu(x)) through the same fused
    # apply: parity with the oracle on identical factors, and the approximation error
    # against the dense sum matches the oracle's
    kern = kernels.HankelSum(1024)
    f = oracle.construct_factors(kern, leaf=16, r=16, method="sampling", seed=2)
    g = complex_gaussian((kern.N, 16), 3)
    h = _handle(f, prec)
    assert h.path == 1
    u = h.apply(_to(g, dev, prec)).cpu().numpy()
    ref = oracle.bf_apply(f, g)
    assert oracle.rel_err(u, ref) < TOL[prec]
    rows = np.arange(0, kern.N, 4)
    dense = kernels.dense_apply_rows(kern, rows, g)
    e_gpu, e_ora = oracle.rel_err(u[rows], dense), oracle.rel_err(ref[rows], dense)
    assert abs(e_gpu - e_ora) <= 2 * TOL[prec] + 1e-3 * e_ora


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("radix,leaf,L,r", [(2, 16, 4, 8), (2, 16, 4, 32), (4, 16, 2, 32), (2, 4, 6, 8),
                                            (4, 4, 4, 16), (2, 4, 4, 32), (2, 3, 4, 8)])
@pytest.mark.parametrize("nrhs,pad", [(64, 0), (192, 0), (128, 8)])
def test_leaf_kernels_with_wave_uniform_leaves(dev, prec, radix, leaf, L, r, nrhs, pad):
    """Column counts that are multiples of 64 put every wavefront of the leaf kernels on
    one leaf (leaf blocks read through the scalar path); apply and adjoint against the
    oracle, with and without row padding."""
    f = synthetic_factors(radix, leaf, L, r, seed=31)
    N = leaf * radix ** L
    g = complex_gaussian((N, nrhs), 32)
    h = _handle(f, prec)
    assert h.path == 0
    tol = 1e-10 if prec == "f64" else 1e-5
    gd = _to(np.concatenate([g, np.zeros((N, pad))], 1), dev, prec)[:, :nrhs]
    u = h.apply(gd).cpu().numpy()
    assert oracle.rel_err(u, oracle.bf_apply(f, g)) < tol
    v = h.apply_adjoint(gd).cpu().numpy()
    assert oracle.rel_err(v, oracle.bf_apply_adjoint(f, g)) < tol
    h.close()
