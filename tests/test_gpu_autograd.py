"""torch.autograd through the library's backward kernels (BFOperator / bf_apply_autograd):
gradients against the oracle and against central finite differences."""
import numpy as np
import pytest

import oracle
from bf_inputs import complex_gaussian, loss_target, synthetic_factors
from oracle import kernels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_01379_amd import load_library
    load_library()
    return torch.device("cuda:0")


def _loss(op, g, y):
    u = op(g)
    return (u - y).abs().pow(2).sum()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-5), ("bf16x3", 1e-4)])
def test_autograd_matches_oracle_gradient(dev, prec, tol):
    # L = ||K_BF g - y||^2 with y = K g + noise; every parameter gradient and grad g
    from paper_1502_01379_amd import BFOperator
    f = oracle.construct_factors(kernels.fio(1024), leaf=16, r=16, method="sampling", seed=0)
    N, nrhs = 1024, 6
    g = complex_gaussian((N, nrhs), 1)
    y = loss_target(N, nrhs, 2, base=oracle.bf_apply(f, g))
    op = BFOperator(f, prec)
    cd = torch.complex128 if prec == "f64" else torch.complex64
    gt = torch.tensor(g, dtype=cd, device=dev, requires_grad=True)
    yt = torch.tensor(y, dtype=cd, device=dev)
    u = op(gt)
    seen = {}
    u.register_hook(lambda grad: seen.setdefault("grad_u", grad.detach().clone()))
    (u - yt).abs().pow(2).sum().backward()
    # the backward is checked on exactly what it was given: g and the incoming
    # gradient 2 (u - y) in the handle's precision (u - y is a small difference)
    g_in = gt.detach().cpu().numpy().astype(np.complex128)
    gu_in = seen["grad_u"].cpu().numpy().astype(np.complex128)
    ref = oracle.bf_grad(f, g_in, gu_in)
    assert oracle.rel_err(gt.grad.cpu().numpy(), ref["g"]) < tol
    p = op.params
    pairs = [(p["VL"], ref["VL"]), (p["UL"], ref["UL"]), (p["S"], ref["S"])]
    pairs += list(zip(p["H"], ref["H"])) + list(zip(p["G"], ref["G"]))
    for t, r in pairs:
        assert oracle.rel_err(t.grad.cpu().numpy(), r) < (10 * tol if prec != "bf16x3" else tol)


def test_autograd_finite_differences(dev):
    # the loss is quadratic in every single factor entry, so a central difference is
    # exact up to rounding: random block entries (real and imaginary parts) of every
    # factor kind, FP64 on the per-level path
    from paper_1502_01379_amd import BFOperator
    f = synthetic_factors(2, 4, 6, 5, seed=3)
    N, nrhs = 256, 4
    g = complex_gaussian((N, nrhs), 4)
    y = loss_target(N, nrhs, 5, base=oracle.bf_apply(f, g))
    op = BFOperator(f, "f64")
    gt = torch.tensor(g, device=dev)
    yt = torch.tensor(y, device=dev)
    _loss(op, gt, yt).backward()
    rng = np.random.default_rng(6)
    names = ["VL", "UL", "S"] + [("H", t) for t in range(3)] + [("G", t) for t in range(3)]
    checked = 0
    for _ in range(32):
        key = names[rng.integers(len(names))]
        prm = op.params[key] if isinstance(key, str) else op.params[key[0]][key[1]]
        idx = tuple(int(rng.integers(s)) for s in prm.shape)
        parts = [1.0] if not prm.is_complex() else [1.0, 1j]
        for unit in parts:
            delta = 1e-3
            with torch.no_grad():
                base = prm[idx].clone()
                prm[idx] = base + delta * unit
                op.refresh()
                lp = _loss(op, gt, yt).item()
                prm[idx] = base - delta * unit
                op.refresh()
                lm = _loss(op, gt, yt).item()
                prm[idx] = base
            fd = (lp - lm) / (2 * delta)
            gval = prm.grad[idx]
            an = float(gval.real if unit == 1.0 else gval.imag) if prm.is_complex() else float(gval)
            assert abs(fd - an) <= 1e-6 * (1 + abs(an)), (key, idx, unit, fd, an)
            checked += 1
    op.refresh()
    assert checked >= 32
