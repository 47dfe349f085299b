"""C-ABI checks that need no GPU: the library loads, exports what bf.h declares,
and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1502_01379_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bf_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_1502_01379_amd import build
        build.build()
    return B.load_library()


def test_library_exports_every_declared_symbol(lib):
    syms = _declared_symbols()
    assert {"bf_create_from_factors", "bf_apply", "bf_apply_adjoint", "bf_backward",
            "bf_destroy"} <= set(syms)
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(B.EXPORTED)


def _factors(shape_tuple):
    R, leaf, L, r = shape_tuple
    P = R ** L
    h = L // 2
    keep = {"VL": np.zeros(P * leaf * r * 2), "UL": np.zeros(P * leaf * r * 2),
            "S": np.zeros(R ** h * R ** h * r)}
    lv = [np.zeros(P * R * r * r * 2) for _ in range(2 * h)]
    PD = ctypes.POINTER(ctypes.c_double)
    Harr = (PD * max(h, 1))(*[x.ctypes.data_as(PD) for x in lv[:h]])
    Garr = (PD * max(h, 1))(*[x.ctypes.data_as(PD) for x in lv[h:]])
    fh = B.BFFactorsHost(keep["VL"].ctypes.data_as(PD), Harr, keep["S"].ctypes.data_as(PD), Garr,
                         keep["UL"].ctypes.data_as(PD))
    return fh, (keep, lv, Harr, Garr)


@pytest.mark.parametrize("shape,code", [
    ((2, 16, 5, 16, 16 * 32), B.BF_ERR_SHAPE),        # odd L
    ((3, 4, 2, 4, 36), B.BF_ERR_SHAPE),               # radix 3
    ((2, 16, 4, 16, 1000), B.BF_ERR_SHAPE),           # N != leaf * R^L
    ((2, 16, 4, 0, 256), B.BF_ERR_SHAPE),             # r = 0
    ((2, 0, 4, 4, 0), B.BF_ERR_SHAPE),                # leaf 0
])
def test_create_rejects_bad_shapes(lib, shape, code):
    R, leaf, L, r, N = shape
    fh, keep = _factors((2, 4, 2, 2))
    st, h = B.bf_create_from_factors(B.BFShape(R, leaf, L, r, N), fh, 1)
    assert st == code and not h
    assert B.bf_last_error(None)


def test_create_rejects_null_and_nonfinite_and_bad_precision(lib):
    fh, keep = _factors((2, 4, 2, 2))
    shape = B.BFShape(2, 4, 2, 2, 16)
    st, h = B.bf_create_from_factors(shape, B.BFFactorsHost(), 1)
    assert st == B.BF_ERR_INVALID_ARG and not h
    st, h = B.bf_create_from_factors(shape, fh, 7)
    assert st == B.BF_ERR_INVALID_ARG
    keep[0]["S"][3] = np.nan
    st, h = B.bf_create_from_factors(shape, fh, 1)
    assert st == B.BF_ERR_NONFINITE and "NaN" in B.bf_last_error(None)
    keep[0]["S"][3] = 0
    keep[1][0][5] = np.inf
    st, h = B.bf_create_from_factors(shape, fh, 0)
    assert st == B.BF_ERR_NONFINITE


def test_split_precision_needs_fused_shape(lib):
    # split precision runs only on the fused MFMA passes; radix 4 is not one of them
    fh, keep = _factors((4, 2, 2, 3))
    st, h = B.bf_create_from_factors(B.BFShape(4, 2, 2, 3, 32), fh, 2)
    assert st == B.BF_ERR_UNSUPPORTED and not h


@pytest.mark.parametrize("field,value", [("path", 2), ("path", -1), ("fused_cols", 8), ("fused_kmax", 5),
                                         ("fused_split", -2), ("level_mfma", 1), ("level_ksplit", 3)])
def test_create_ex_rejects_bad_options(lib, field, value):
    fh, keep = _factors((2, 16, 2, 16))
    opts = B.BFPlanOptions()
    setattr(opts, field, value)
    st, h = B.bf_create_from_factors_ex(B.BFShape(2, 16, 2, 16, 64), fh, 1, opts)
    assert st == B.BF_ERR_INVALID_ARG and not h
    assert "option" in B.bf_last_error(None)


def test_split_precision_rejects_the_per_level_path(lib):
    fh, keep = _factors((2, 16, 2, 16))
    opts = B.BFPlanOptions()
    opts.path = 1
    st, h = B.bf_create_from_factors_ex(B.BFShape(2, 16, 2, 16, 64), fh, 2, opts)
    assert st == B.BF_ERR_UNSUPPORTED and not h


def test_null_handle_calls(lib):
    assert B.bf_apply(None, 1, 2, 1, 1) == B.BF_ERR_INVALID_ARG
    assert B.bf_apply_adjoint(None, 1, 2, 1, 1) == B.BF_ERR_INVALID_ARG
    assert B.bf_backward(None, 1, 2, 3, None, 1, 1) == B.BF_ERR_INVALID_ARG
    B.bf_destroy(None)   # no-op
    assert lib.bf_set_profiling(None, 1) == B.BF_ERR_INVALID_ARG


def test_construction_entry_points_reject_bad_arguments(lib):
    """Argument checks of include/bf_construct.h that return before any device work."""
    PD = ctypes.POINTER(ctypes.c_double)
    z = np.zeros(64)
    arr = (PD * 4)(*[z.ctypes.data_as(PD)] * 4)
    out = B.BFFactorsOut(z.ctypes.data_as(PD), arr, z.ctypes.data_as(PD), arr, z.ctypes.data_as(PD))
    cases = [
        (B.BFShape(2, 16, 5, 16, 16 * 32), 1, 3, 3, B.BF_ERR_SHAPE),       # odd L
        (B.BFShape(2, 16, 4, 16, 1000), 1, 3, 3, B.BF_ERR_SHAPE),          # N != leaf R^L
        (B.BFShape(2, 16, 4, 16, 256), 7, 3, 3, B.BF_ERR_INVALID_ARG),     # unknown kernel
        (B.BFShape(2, 16, 4, 16, 256), 1, 0, 3, B.BF_ERR_INVALID_ARG),     # q = 0
        (B.BFShape(2, 1, 4, 8, 16), 1, 3, 3, B.BF_ERR_UNSUPPORTED),        # r > b = 4
        (B.BFShape(2, 64, 4, 40, 1024), 1, 3, 3, B.BF_ERR_UNSUPPORTED),    # r > 32
        (B.BFShape(4, 16, 2, 32, 256), 1, 3, 3, B.BF_ERR_UNSUPPORTED),     # R r > 64
    ]
    for shape, kind, q, iters, code in cases:
        st = B.bf_construct_from_kernel(shape, kind, q, iters, 0, 1e-14, out)
        assert st == code, (shape.N, kind, q, st, B.bf_last_error(None))
        assert B.bf_last_error(None)
    assert B.bf_batched_svd(None, 1, 4, 4, None, None, None) == B.BF_ERR_INVALID_ARG
    assert B.bf_batched_svd(1, 1, 200, 4, None, 1, 1) == B.BF_ERR_UNSUPPORTED
    assert B.bf_batched_svd(1, 1, 64, 65, None, 1, 1) == B.BF_ERR_UNSUPPORTED
    assert B.bf_batched_qr(1, 1, 8, 65, None) == B.BF_ERR_UNSUPPORTED
    assert B.bf_batched_column_pivots(1, 1, 129, 8, 2, 1) == B.BF_ERR_UNSUPPORTED
    assert B.bf_batched_column_pivots(1, 1, 8, 8, 9, 1) == B.BF_ERR_UNSUPPORTED
    assert B.bf_kernel_entries(5, 16, 1, 1, 1, 1, 1, 1) == B.BF_ERR_INVALID_ARG
    assert B.bf_kernel_entries(1, 16, 1, 2, 1, 4, 1, 3) == B.BF_ERR_INVALID_ARG  # ld < ncols


def test_device_construction_driver_is_switched_off(lib):
    PD = ctypes.POINTER(ctypes.c_double)
    z = np.zeros(1 << 14)
    arr = (PD * 4)(*[z.ctypes.data_as(PD)] * 4)
    out = B.BFFactorsOut(z.ctypes.data_as(PD), arr, z.ctypes.data_as(PD), arr, z.ctypes.data_as(PD))
    st = B.bf_construct_from_kernel(B.BFShape(2, 4, 4, 16, 64), 1, 3, 3, 0, 1e-14, out)
    assert st == B.BF_ERR_UNSUPPORTED and "switched off" in B.bf_last_error(None)
