"""FP64 fused passes (binary trees, 16-point leaves, rank 16) vs the FP64 oracle.

Held to 1e-10 relative l2 error over all columns and in every column.  The same
factor product is split into passes of one to four levels; ragged column
counts leave partial workgroups and partial 16-column chunks.
"""
import numpy as np
import pytest

import oracle
from bf_inputs import complex_gaussian, synthetic_factors
from oracle import kernels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_01379_amd import load_library
    load_library()
    return torch.device("cuda:0")


def _handle(f, **opts):
    from paper_1502_01379_amd import BFHandle
    return BFHandle(f, "f64", options=opts)


def _dev(x, dev):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dev, torch.complex128)


def _check(u, ref, what):
    err = oracle.rel_err(u, ref)
    worst = max(oracle.rel_err(u[:, c], ref[:, c]) for c in range(ref.shape[1]))
    assert err < TOL and worst < TOL, f"{what}: {err:.3e} (worst column {worst:.3e})"


@pytest.mark.parametrize("L", [2, 4, 6, 8, 10, 12])
@pytest.mark.parametrize("nrhs", [1, 17, 70])
def test_f64_fused_apply_and_adjoint(dev, L, nrhs):
    # one pass per side up to L = 8 (passes of 1 .. 4 levels, one or two wavefronts
    # per tile), two per side beyond; 70 columns = four full chunks and one of six
    f = synthetic_factors(2, 16, L, 16, seed=500 + L)
    N = 16 * 2 ** L
    g = complex_gaussian((N, nrhs), 501 + nrhs)
    h = _handle(f)
    assert h.path == 1, "expected the fused FP64 passes"
    print(f"f64 fused L={L} nrhs={nrhs}", flush=True)
    _check(h.apply(_dev(g, dev)).cpu().numpy(), oracle.bf_apply(f, g), "apply")
    _check(h.apply_adjoint(_dev(g, dev)).cpu().numpy(), oracle.bf_apply_adjoint(f, g), "adjoint")
    h.close()


@pytest.mark.parametrize("kmax", [1, 2, 3, 4])
def test_f64_fused_pass_depths(dev, kmax):
    # the Sec. 4 FIO factorization at N = 4096 split into passes of at most kmax levels
    f = oracle.construct_factors(kernels.fio(4096), leaf=16, r=16, method="sampling", seed=0)
    g = complex_gaussian((4096, 40), 510)
    h = _handle(f, fused_kmax=kmax)
    assert h.path == 1
    _check(h.apply(_dev(g, dev)).cpu().numpy(), oracle.bf_apply(f, g), f"apply kmax={kmax}")
    _check(h.apply_adjoint(_dev(g, dev)).cpu().numpy(), oracle.bf_apply_adjoint(f, g), f"adjoint kmax={kmax}")
    h.close()


def test_f64_fused_padded_rows_and_per_level_agreement(dev):
    # ld > nrhs (padding columns untouched) and agreement with the per-level kernels
    f = synthetic_factors(2, 16, 8, 16, seed=520)
    N, nrhs, ld = 4096, 33, 40
    g = complex_gaussian((N, nrhs), 521)
    gl = torch.zeros((N, ld), dtype=torch.complex128, device=dev)
    gl[:, :nrhs] = _dev(g, dev)
    out = torch.full((N, ld), 7.0 + 0j, dtype=torch.complex128, device=dev)
    h = _handle(f)
    h.apply(gl[:, :nrhs], out=out[:, :nrhs])
    torch.cuda.synchronize()
    u = out[:, :nrhs].cpu().numpy()
    _check(u, oracle.bf_apply(f, g), "apply")
    assert bool((out[:, nrhs:] == 7.0).all()), "padding columns were written"
    hp = _handle(f, path=1)
    assert hp.path == 0
    up = hp.apply(_dev(g, dev)).cpu().numpy()
    assert oracle.rel_err(u, up) < 1e-12
    h.close()
    hp.close()


def test_f64_backward_on_fused_handle(dev):
    # FP64 handles take the per-level backward: gradients of every factor kind and
    # of g against the oracle's
    f = synthetic_factors(2, 16, 6, 16, seed=530)
    N, nrhs = 1024, 9
    g = complex_gaussian((N, nrhs), 531)
    gu = complex_gaussian((N, nrhs), 532)
    h = _handle(f)
    assert h.path == 1
    grad_g, grads = h.backward(_dev(g, dev), _dev(gu, dev))
    ref = oracle.bf_grad(f, g, gu)
    assert oracle.rel_err(grad_g.cpu().numpy(), ref["g"]) < TOL
    for kind in ("VL", "UL", "S"):
        assert oracle.rel_err(grads[kind].cpu().numpy(), ref[kind]) < TOL, kind
    for kind in ("H", "G"):
        for a, b in zip(grads[kind], ref[kind]):
            assert oracle.rel_err(a.cpu().numpy(), b) < TOL, kind
    h.close()


def test_f64_fused_at_2_18_sampled_columns(dev):
    # N = 2^18 (L = 14: passes of four and three levels), 64 columns; three columns
    # against the oracle's apply of those columns
    L, nrhs = 14, 64
    f = synthetic_factors(2, 16, L, 16, seed=540)
    N = 16 * 2 ** L
    g = complex_gaussian((N, nrhs), 541)
    h = _handle(f)
    u = h.apply(_dev(g, dev))
    cols = [0, 31, 63]
    uc = u[:, cols].cpu().numpy()
    _check(uc, oracle.bf_apply(f, g[:, cols]), "apply")
    h.close()
