"""bf_apply captured in a HIP graph (torch.cuda.CUDAGraph): no allocation, memset or
synchronization on a warmed call, so the launches replay as recorded.  Every replay,
with eager work and new inputs in between, must equal the eager apply bit for bit."""
import numpy as np
import pytest

from bf_inputs import complex_gaussian, synthetic_factors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_01379_amd import load_library
    load_library()
    return torch.device("cuda:0")


@pytest.mark.parametrize("radix,leaf,L,r,prec,nrhs", [
    (2, 16, 6, 12, "f64", 1),        # per-level kernels (FP64, latency-bound shape)
    (4, 16, 4, 32, "f32", 40),       # per-level butterflies on the matrix cores
    (2, 16, 8, 16, "bf16x3", 70),    # fused split-tile passes
    (2, 16, 6, 16, "f32", 33),       # fused one-wavefront passes
    (2, 16, 8, 16, "f64", 40),       # fused FP64 passes (wavefront pairs)
])
def test_apply_replays_in_a_graph(dev, radix, leaf, L, r, prec, nrhs):
    from paper_1502_01379_amd import BFHandle
    f = synthetic_factors(radix, leaf, L, r, seed=L + r)
    N = leaf * radix ** L
    cd = torch.complex128 if prec == "f64" else torch.complex64
    h = BFHandle(f, prec)
    g = torch.from_numpy(complex_gaussian((N, nrhs), 1)).to(dev, cd)
    u = torch.empty_like(g)
    v = torch.empty_like(g)
    h.apply(g, out=u)            # grows the workspace outside the capture
    h.apply_adjoint(g, out=v)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        h.apply(g, out=u)
        h.apply_adjoint(g, out=v)
    for rep in range(4):
        g.copy_(torch.from_numpy(complex_gaussian((N, nrhs), 10 + rep)).to(dev, cd))
        u.zero_()
        v.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        ue = h.apply(g.clone())
        ve = h.apply_adjoint(g.clone())
        torch.cuda.synchronize()
        assert torch.equal(u, ue), rep
        assert torch.equal(v, ve), rep
