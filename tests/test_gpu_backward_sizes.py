"""bf_backward on the fused path at the differentiation workload's size and with many
right-hand sides, and central finite differences through a fused FP32 handle.

At N = 2^18 and 2^20 the oracle's gradient over every column would take minutes,
so there the incoming gradient is zero outside a few columns: the GPU still runs
every column through the forward, recompute and adjoint passes and sums the
block gradients over all column chunks, while the exact gradient involves only
the nonzero columns (each block gradient is a sum over columns of
d_out x_in^*, and d_out vanishes where grad_u does).
"""
import numpy as np
import pytest

import oracle
from bf_inputs import complex_gaussian, loss_target, synthetic_factors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16x3": 1e-4}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_01379_amd import load_library
    load_library()
    return torch.device("cuda:0")


def _dev(x, dev):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dev, torch.complex64)


def _flat(d):
    return [d["VL"], d["UL"], d["S"], *d["H"], *d["G"]]


def _names(L):
    h = L // 2
    return ["VL", "UL", "S"] + [f"H{l}" for l in range(h, L)] + [f"G{l}" for l in range(h, L)]


def _check(grad_g, grads, ref, cols, tol, L):
    err = oracle.rel_err(grad_g[:, cols].cpu().numpy(), ref["g"])
    worst = ("g", err)
    assert err < tol, f"grad_g {err:.3e}"
    for name, a, b in zip(_names(L), _flat(grads), _flat(ref)):
        e = oracle.rel_err(a.cpu().numpy(), b)
        worst = max(worst, (name, e), key=lambda t: t[1])
        assert e < tol, f"grad {name} {e:.3e}"
    print(f"largest gradient error {worst[0]} {worst[1]:.3e}", flush=True)


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_backward_128_columns_every_column(dev, prec):
    # N = 4096 (L = 8, one four-level pass per side), 128 columns = eight 16-column
    # chunks in two workgroup column groups, every column nonzero; against the
    # oracle's gradient over all columns; recompute and store-all agree bitwise
    from paper_1502_01379_amd import BFHandle, BF_BWD_STORE_ALL
    L, nrhs = 8, 128
    f = synthetic_factors(2, 16, L, 16, seed=200)
    N = 16 * 2 ** L
    g = complex_gaussian((N, nrhs), 201)
    gu = complex_gaussian((N, nrhs), 202)
    ref = oracle.bf_grad(f, g, gu)
    h = BFHandle(f, prec)
    grad_g, grads = h.backward(_dev(g, dev), _dev(gu, dev))
    _check(grad_g, grads, ref, slice(None), TOL[prec], L)
    grad_g2, grads2 = h.backward(_dev(g, dev), _dev(gu, dev), flags=BF_BWD_STORE_ALL)
    assert torch.equal(grad_g, grad_g2)
    for a, b in zip(_flat(grads), _flat(grads2)):
        assert torch.equal(a, b)
    h.close()


@pytest.mark.parametrize("L,nrhs,prec,cols", [
    (14, 128, "f32", [0, 77, 127]),        # the differentiation workload: N = 2^18, 128 columns
    (16, 32, "f32", [3, 30]),              # N = 2^20: two four-level passes per side
    (16, 32, "bf16x3", [3, 30]),
])
def test_backward_at_workload_size(dev, L, nrhs, prec, cols):
    # loss ||K g - y||^2 restricted to the sampled columns: grad_u = 2 (u - y) there
    # and 0 elsewhere; recompute (the default) against the oracle's gradient of the
    # same columns, and against keeping every state, bit for bit
    from paper_1502_01379_amd import BFHandle, BF_BWD_STORE_ALL
    f = synthetic_factors(2, 16, L, 16, seed=210 + L)
    N = 16 * 2 ** L
    print(f"backward N=2^{L + 4} nrhs={nrhs} prec={prec} columns {cols}", flush=True)
    g = complex_gaussian((N, nrhs), 211, dtype=np.complex64)
    y = loss_target(N, len(cols), 212)
    u_cols = oracle.bf_apply(f, g[:, cols].astype(np.complex128))
    gu_cols = 2 * (u_cols - y)
    gu = np.zeros((N, nrhs), dtype=np.complex64)
    gu[:, cols] = gu_cols
    ref = oracle.bf_grad(f, g[:, cols].astype(np.complex128), gu_cols)
    h = BFHandle(f, prec)
    gd, gud = _dev(g, dev), _dev(gu, dev)
    grad_g, grads = h.backward(gd, gud)
    torch.cuda.synchronize()
    _check(grad_g, grads, ref, cols, TOL[prec], L)
    # columns with a zero incoming gradient get a zero grad_g
    rest = [c for c in range(nrhs) if c not in cols]
    assert float(grad_g[:, rest].abs().max()) == 0.0
    grad_g2, grads2 = h.backward(gd, gud, flags=BF_BWD_STORE_ALL)
    assert torch.equal(grad_g, grad_g2)
    for a, b in zip(_flat(grads), _flat(grads2)):
        assert torch.equal(a, b)
    h.close()


def test_finite_differences_through_fused_f32_handle(dev):
    # L(theta) = ||K g - y||^2 is quadratic in every single real parameter theta (a
    # real or imaginary part of one block entry, or one middle weight), so the central
    # difference (L(theta + d) - L(theta - d)) / 2d equals dL/dtheta exactly for any
    # step d; the losses come from FP32 applies of handles built with the perturbed
    # factors, summed in FP64.  64 random entries across every factor kind.
    from paper_1502_01379_amd import BFHandle
    L, nrhs = 6, 8
    f = synthetic_factors(2, 16, L, 16, seed=220)
    N = 16 * 2 ** L
    g = complex_gaussian((N, nrhs), 221)
    y = loss_target(N, nrhs, 222)
    gd = _dev(g, dev)

    def loss(fac):
        h = BFHandle(fac, "f32")
        assert h.path == 1
        u = h.apply(gd).cpu().numpy().astype(np.complex128)
        h.close()
        return float(np.sum(np.abs(u - y) ** 2))

    h = BFHandle(f, "f32")
    u = h.apply(gd).cpu().numpy().astype(np.complex128)
    _, grads = h.backward(gd, _dev(2 * (u - y), dev))
    h.close()
    rng = np.random.default_rng(223)
    kinds = ["VL", "UL", "S", "H", "G"]
    worst = 0.0
    for k in range(64):
        kind = kinds[k % 5]
        fp = {key: (list(v) if isinstance(v, list) else v) for key, v in f.items()}
        fm = {key: (list(v) if isinstance(v, list) else v) for key, v in f.items()}
        if kind in ("H", "G"):
            t = int(rng.integers(len(f[kind])))
            arr = f[kind][t]
            idx = tuple(int(rng.integers(s)) for s in arr.shape)
            ga = grads[kind][t].cpu().numpy()
        else:
            t = None
            arr = f[kind]
            idx = tuple(int(rng.integers(s)) for s in arr.shape)
            ga = grads[kind].cpu().numpy()
        imag = kind != "S" and bool(rng.integers(2))
        step = 0.5 * (1j if imag else 1.0) if kind != "S" else 0.5
        ap, am = arr.copy(), arr.copy()
        ap[idx] += step
        am[idx] -= step
        if t is None:
            fp[kind], fm[kind] = ap, am
        else:
            fp[kind][t], fm[kind][t] = ap, am
        fd = (loss(fp) - loss(fm)) / (2 * 0.5)
        an = (ga[idx].imag if imag else ga[idx].real) if kind != "S" else ga[idx]
        # relative to the entry, or to the factor's typical gradient when the entry's
        # own is small (the FP32 losses carry an absolute rounding error)
        scale = max(abs(an), float(np.sqrt(np.mean(np.abs(ga) ** 2))))
        err = abs(fd - an) / scale
        worst = max(worst, err)
        assert err < 1e-3, f"{kind}{'' if t is None else t}{idx} {'imag' if imag else 'real'}: fd {fd} grad {an}"
    print(f"largest finite-difference mismatch {worst:.2e}", flush=True)
