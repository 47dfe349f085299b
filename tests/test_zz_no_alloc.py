"""bf_apply_noalloc (the apply whose activation buffers live in the library's
per-GPU scratch array) against bf_apply on the same handle, through the C ABI:
two calls in a row, the second with fewer columns, on the fused MFMA passes and
on the per-level kernels."""
import numpy as np
import pytest

import oracle
from bf_inputs import complex_gaussian, synthetic_factors
from oracle import kernels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5, "bf16x3": 1e-4}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_01379_amd import load_library
    load_library()
    return torch.device("cuda:0")


def _noalloc(h, g, nrhs, ld):
    from paper_1502_01379_amd import binding as B
    u = torch.full((h.N, ld), complex(7.0, -7.0), dtype=g.dtype, device=g.device)
    print(f"bf_apply_noalloc: N={h.N} prec={h.precision} path={h.path} nrhs={nrhs} ld={ld}", flush=True)
    st = B.bf_apply_noalloc(h.handle, g.data_ptr(), u.data_ptr(), nrhs, ld,
                            torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == B.BF_OK, B.bf_last_error(h.handle)
    return u


@pytest.mark.parametrize("prec,path,case", [
    ("f32", 1, "fio4096"), ("bf16x3", 1, "fio4096"), ("f32", 1, "synth_L12"),
    ("f64", 0, "fourier1024"), ("f64", 1, "fio4096"), ("f32", 0, "synth_r8"), ("f32", 0, "grt")])
def test_noalloc_matches_apply_twice(dev, prec, path, case):
    from paper_1502_01379_amd import BFHandle
    if case == "fio4096":
        f = oracle.construct_factors(kernels.fio(4096), leaf=16, r=16, method="sampling", seed=0)
        calls = [(40, 43), (17, 17)]
    elif case == "synth_L12":     # N = 65536, r = 16: 64 columns fill the scratch array
        f = synthetic_factors(2, 16, 12, 16, seed=60)
        calls = [(64, 64), (33, 35)]
    elif case == "fourier1024":
        f = oracle.construct_factors(kernels.fourier(1024), leaf=16, r=12, method="sampling", seed=0)
        calls = [(5, 5), (1, 2)]
    elif case == "synth_r8":
        f = synthetic_factors(2, 16, 8, 8, seed=61)
        calls = [(70, 72), (3, 3)]
    else:
        f = synthetic_factors(4, 16, 4, 32, seed=62)
        calls = [(128, 128), (31, 31)]
    h = BFHandle(f, prec)
    assert h.path == path
    cd = h.complex_dtype
    for k, (nrhs, ld) in enumerate(calls):
        g_host = complex_gaussian((h.N, nrhs), 70 + k)
        gl = torch.zeros((h.N, ld), dtype=cd, device=dev)
        gl[:, :nrhs] = torch.as_tensor(g_host).to(dev, cd)
        u = _noalloc(h, gl, nrhs, ld)
        ref = torch.empty((h.N, ld), dtype=cd, device=dev)
        h.apply(gl[:, :nrhs], out=ref[:, :nrhs])
        torch.cuda.synchronize()
        # same kernels, same order: identical bits; padding columns untouched
        assert torch.equal(u[:, :nrhs], ref[:, :nrhs]), f"call {k}"
        assert bool((u[:, nrhs:] == complex(7.0, -7.0)).all())
        cols = [0, nrhs - 1]
        exp = oracle.bf_apply(f, g_host[:, cols])
        assert oracle.rel_err(u[:, cols].cpu().numpy(), exp) < TOL[prec]
    h.close()


def test_noalloc_rejects_more_columns_than_the_scratch_holds(dev):
    from paper_1502_01379_amd import BFHandle
    from paper_1502_01379_amd import binding as B
    f = synthetic_factors(2, 16, 12, 16, seed=60)   # N = 65536: 64 columns fit, 65 do not
    h = BFHandle(f, "f32")
    g = torch.zeros((h.N, 65), dtype=torch.complex64, device=dev)
    u = torch.full_like(g, 3.0)
    st = B.bf_apply_noalloc(h.handle, g.data_ptr(), u.data_ptr(), 65, 65,
                            torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == B.BF_ERR_UNSUPPORTED
    assert "scratch" in B.bf_last_error(h.handle)
    assert bool((u == 3.0).all())
    h.close()
