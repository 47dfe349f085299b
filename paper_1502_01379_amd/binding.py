"""ctypes binding of the C ABI in include/bf.h (argument marshalling only).

The functions named like the C entry points take raw pointers (ints) and
return the bf_status; `BFHandle` wraps them for torch tensors on the GPU.
Every computation happens in libbfly.so: if the library is missing this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbfly.so")

BF_OK, BF_ERR_INVALID_ARG, BF_ERR_SHAPE, BF_ERR_UNSUPPORTED, BF_ERR_ALLOC, BF_ERR_HIP, BF_ERR_NONFINITE = range(7)
STATUS_NAMES = ["BF_OK", "BF_ERR_INVALID_ARG", "BF_ERR_SHAPE", "BF_ERR_UNSUPPORTED",
                "BF_ERR_ALLOC", "BF_ERR_HIP", "BF_ERR_NONFINITE"]
PRECISIONS = {"f64": 0, "f32": 1, "bf16x3": 2, "f16x3": 3}
BF_BWD_RECOMPUTE = 0
BF_BWD_STORE_ALL = 1
BF_NOALLOC_SCRATCH_BYTES = 64 << 20

EXPORTED = ["bf_create_from_factors", "bf_create_from_factors_ex", "bf_apply", "bf_apply_noalloc", "bf_apply_adjoint", "bf_backward", "bf_destroy",
            "bf_last_error", "bf_query", "bf_set_profiling", "bf_kernel_times",
            # include/bf_construct.h
            "bf_kernel_entries", "bf_batched_svd", "bf_batched_qr", "bf_batched_column_pivots",
            "bf_construct_from_kernel"]
KERNELS = {"fourier": 0, "fio": 1}


class BFShape(ctypes.Structure):
    _fields_ = [("radix", ctypes.c_int32), ("leaf", ctypes.c_int32), ("L", ctypes.c_int32),
                ("r", ctypes.c_int32), ("N", ctypes.c_int64)]


_PD = ctypes.POINTER(ctypes.c_double)


class BFPlanOptions(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("fused_cols", ctypes.c_int32), ("fused_kmax", ctypes.c_int32),
                ("fused_split", ctypes.c_int32), ("level_mfma", ctypes.c_int32),
                ("level_ksplit", ctypes.c_int32)]


class BFFactorsHost(ctypes.Structure):
    _fields_ = [("VL", _PD), ("H", ctypes.POINTER(_PD)), ("S", _PD),
                ("G", ctypes.POINTER(_PD)), ("UL", _PD)]


class BFFactorGrads(ctypes.Structure):
    _fields_ = [("VL", ctypes.c_void_p), ("H", ctypes.POINTER(ctypes.c_void_p)),
                ("S", ctypes.c_void_p), ("G", ctypes.POINTER(ctypes.c_void_p)),
                ("UL", ctypes.c_void_p)]


class BFFactorsOut(ctypes.Structure):
    _fields_ = [("VL", _PD), ("H", ctypes.POINTER(_PD)), ("S", _PD),
                ("G", ctypes.POINTER(_PD)), ("UL", _PD)]


class BFError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {message}")


_lib = None


def load_library(path=LIB_PATH):
    """Load libbfly.so (built by paper_1502_01379_amd.build); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1502_01379_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
    lib.bf_create_from_factors.argtypes = [ctypes.POINTER(BFShape), ctypes.POINTER(BFFactorsHost),
                                           ctypes.c_int, vp, ctypes.POINTER(vp)]
    lib.bf_create_from_factors.restype = ctypes.c_int
    lib.bf_create_from_factors_ex.argtypes = [ctypes.POINTER(BFShape), ctypes.POINTER(BFFactorsHost),
                                              ctypes.c_int, ctypes.POINTER(BFPlanOptions), vp, ctypes.POINTER(vp)]
    lib.bf_create_from_factors_ex.restype = ctypes.c_int
    for name in ("bf_apply", "bf_apply_adjoint", "bf_apply_noalloc"):
        fn = getattr(lib, name)
        fn.argtypes = [vp, vp, vp, i64, i64, vp]
        fn.restype = ctypes.c_int
    lib.bf_backward.argtypes = [vp, vp, vp, vp, ctypes.POINTER(BFFactorGrads), i64, i64, u32, vp]
    lib.bf_backward.restype = ctypes.c_int
    lib.bf_destroy.argtypes = [vp]
    lib.bf_destroy.restype = None
    lib.bf_last_error.argtypes = [vp]
    lib.bf_last_error.restype = ctypes.c_char_p
    lib.bf_query.argtypes = [vp, ctypes.POINTER(BFShape), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(i32)]
    lib.bf_query.restype = ctypes.c_int
    lib.bf_set_profiling.argtypes = [vp, i32]
    lib.bf_set_profiling.restype = ctypes.c_int
    lib.bf_kernel_times.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                    i32, ctypes.POINTER(i32), i32]
    lib.bf_kernel_times.restype = ctypes.c_int
    lib.bf_kernel_entries.argtypes = [i32, i64, vp, i64, vp, i64, vp, i64, vp]
    lib.bf_kernel_entries.restype = ctypes.c_int
    lib.bf_batched_svd.argtypes = [vp, i64, i32, i32, vp, vp, vp, vp]
    lib.bf_batched_svd.restype = ctypes.c_int
    lib.bf_batched_qr.argtypes = [vp, i64, i64, i32, vp, vp]
    lib.bf_batched_qr.restype = ctypes.c_int
    lib.bf_batched_column_pivots.argtypes = [vp, i64, i32, i64, i32, vp, vp]
    lib.bf_batched_column_pivots.restype = ctypes.c_int
    lib.bf_construct_from_kernel.argtypes = [ctypes.POINTER(BFShape), i32, i32, i32, ctypes.c_uint64,
                                             ctypes.c_double, ctypes.POINTER(BFFactorsOut), vp]
    lib.bf_construct_from_kernel.restype = ctypes.c_int
    _lib = lib
    return lib


# ---- entry points under their C names (raw pointers) ---------------------------

def bf_create_from_factors(shape, factors, precision, stream=0):
    """Returns (status, handle) for a BFShape and BFFactorsHost."""
    lib = load_library()
    h = ctypes.c_void_p()
    st = lib.bf_create_from_factors(ctypes.byref(shape), ctypes.byref(factors), int(precision),
                                    ctypes.c_void_p(stream), ctypes.byref(h))
    return st, h.value


def bf_create_from_factors_ex(shape, factors, precision, options=None, stream=0):
    """Returns (status, handle); options is a BFPlanOptions or None (defaults)."""
    lib = load_library()
    h = ctypes.c_void_p()
    st = lib.bf_create_from_factors_ex(ctypes.byref(shape), ctypes.byref(factors), int(precision),
                                       ctypes.byref(options) if options is not None else None,
                                       ctypes.c_void_p(stream), ctypes.byref(h))
    return st, h.value


def bf_apply(handle, g, u, nrhs, ld, stream=0):
    return load_library().bf_apply(handle, g, u, nrhs, ld, ctypes.c_void_p(stream))


def bf_apply_noalloc(handle, g, u, nrhs, ld, stream=0):
    return load_library().bf_apply_noalloc(handle, g, u, nrhs, ld, ctypes.c_void_p(stream))


def bf_apply_adjoint(handle, w, v, nrhs, ld, stream=0):
    return load_library().bf_apply_adjoint(handle, w, v, nrhs, ld, ctypes.c_void_p(stream))


def bf_backward(handle, g, grad_u, grad_g, grads, nrhs, ld, flags=0, stream=0):
    gp = ctypes.byref(grads) if grads is not None else None
    return load_library().bf_backward(handle, g, grad_u, grad_g, gp, nrhs, ld, flags,
                                      ctypes.c_void_p(stream))


def bf_destroy(handle):
    load_library().bf_destroy(handle)


def bf_last_error(handle=None):
    msg = load_library().bf_last_error(handle)
    return msg.decode() if msg else ""


def bf_kernel_entries(kind, N, rows, nrows, cols, ncols, out, ld, stream=0):
    return load_library().bf_kernel_entries(kind, N, rows, nrows, cols, ncols, out, ld,
                                            ctypes.c_void_p(stream))


def bf_batched_svd(A, batch, m, n, U, s, V, stream=0):
    return load_library().bf_batched_svd(A, batch, m, n, U, s, V, ctypes.c_void_p(stream))


def bf_batched_qr(A, batch, n, k, R, stream=0):
    return load_library().bf_batched_qr(A, batch, n, k, R, ctypes.c_void_p(stream))


def bf_batched_column_pivots(At, batch, p, n, npiv, piv, stream=0):
    return load_library().bf_batched_column_pivots(At, batch, p, n, npiv, piv, ctypes.c_void_p(stream))


def bf_construct_from_kernel(shape, kind, q, iters, seed, drop_rel, out, stream=0):
    return load_library().bf_construct_from_kernel(ctypes.byref(shape), kind, q, iters, seed, drop_rel,
                                                   ctypes.byref(out), ctypes.c_void_p(stream))


# ---- convenience wrappers ------------------------------------------------------

def _raise_on(st):
    if st != BF_OK:
        raise BFError(st, bf_last_error(None))


def _cuda_c128(x, name):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex128):
        raise TypeError(f"{name}: expected a complex128 CUDA tensor")
    return x.contiguous()


def kernel_entries(kernel, N, rows, cols, stream=None):
    """K[rows][:, cols] of a built-in kernel ("fourier" or "fio"), computed on the GPU.

    rows, cols: int64 CUDA tensors.  Returns a complex128 CUDA tensor."""
    import torch
    rows = rows.to(torch.int64).contiguous()
    cols = cols.to(torch.int64).contiguous()
    out = torch.empty((rows.numel(), cols.numel()), dtype=torch.complex128, device=rows.device)
    _raise_on(bf_kernel_entries(KERNELS[kernel], int(N), rows.data_ptr(), rows.numel(), cols.data_ptr(),
                                cols.numel(), out.data_ptr(), cols.numel(), _stream_ptr(stream)))
    return out


def batched_svd(A, stream=None):
    """Thin SVD of every matrix of A [batch][m][n] (complex128, CUDA): (U, s, V), A = U diag(s) V^*."""
    import torch
    A = _cuda_c128(A, "A")
    bt, m, n = A.shape
    U = torch.empty((bt, m, n), dtype=A.dtype, device=A.device)
    s = torch.empty((bt, n), dtype=torch.float64, device=A.device)
    V = torch.empty((bt, n, n), dtype=A.dtype, device=A.device)
    _raise_on(bf_batched_svd(A.data_ptr(), bt, m, n, U.data_ptr(), s.data_ptr(), V.data_ptr(),
                             _stream_ptr(stream)))
    return U, s, V


def batched_qr(A, stream=None):
    """QR of every matrix of A [batch][n][k] (complex128, CUDA): returns (Q, R); A is not modified."""
    import torch
    Q = _cuda_c128(A, "A").clone()
    bt, n, k = Q.shape
    R = torch.empty((bt, k, k), dtype=Q.dtype, device=Q.device)
    _raise_on(bf_batched_qr(Q.data_ptr(), bt, n, k, R.data_ptr(), _stream_ptr(stream)))
    return Q, R


def batched_column_pivots(A, npiv, stream=None):
    """First npiv column pivots of a column-pivoted QR of every p x n matrix of A [batch][p][n]."""
    import torch
    At = _cuda_c128(A, "A").transpose(1, 2).contiguous()
    bt, n, p = At.shape
    piv = torch.empty((bt, npiv), dtype=torch.int64, device=At.device)
    _raise_on(bf_batched_column_pivots(At.data_ptr(), bt, p, n, npiv, piv.data_ptr(), _stream_ptr(stream)))
    return piv


def construct_on_device(N, radix, leaf, r, kernel="fio", q=3, iters=3, seed=0, drop_rel=1e-14,
                        stream=None):
    """Butterfly factorization of a built-in kernel built on the current GPU in FP64.

    Randomized sampling (Alg. 2.2) on every middle-level block and the recursion of
    Sec. 3.2, all in the library's HIP kernels.  Returns the canonical host factor
    dict (numpy, complex128), as BFHandle takes it.  The library currently answers
    BF_ERR_UNSUPPORTED (raised as BFError): the device driver is switched off while
    a device-only error in it is found (include/bf_construct.h)."""
    R, leaf, r = int(radix), int(leaf), int(r)
    P, rem = divmod(int(N), leaf)
    L = 0
    while R ** L < P:
        L += 1
    if rem or R ** L != P:
        raise ValueError("N / leaf must be a power of the radix")
    h = L // 2
    m = R ** h
    f = {"radix": R, "leaf": leaf, "L": L, "r": r,
         "VL": np.zeros((P, leaf, r), dtype=np.complex128),
         "UL": np.zeros((P, leaf, r), dtype=np.complex128),
         "S": np.zeros((m, m, r)),
         "H": [np.zeros((R ** (l + 1), R ** (L - l - 1), r, R * r), dtype=np.complex128) for l in range(h, L)],
         "G": [np.zeros((R ** (l + 1), R ** (L - l - 1), r, R * r), dtype=np.complex128) for l in range(h, L)]}
    Harr = (_PD * max(1, h))(*[_ptr(x.view(np.float64)) for x in f["H"]])
    Garr = (_PD * max(1, h))(*[_ptr(x.view(np.float64)) for x in f["G"]])
    out = BFFactorsOut(_ptr(f["VL"].view(np.float64)), Harr, _ptr(f["S"]), Garr, _ptr(f["UL"].view(np.float64)))
    shape = BFShape(R, leaf, L, r, int(N))
    _raise_on(bf_construct_from_kernel(shape, KERNELS[kernel], int(q), int(iters), int(seed), float(drop_rel),
                                       out, _stream_ptr(stream) if stream is not None else 0))
    return f


# ---- handle wrapper ------------------------------------------------------------

def _as_f64(a):
    a = np.ascontiguousarray(a)
    if np.iscomplexobj(a):
        a = np.ascontiguousarray(a.astype(np.complex128, copy=False))
        return a.view(np.float64)
    return np.ascontiguousarray(a.astype(np.float64, copy=False))


def _ptr(a):
    return a.ctypes.data_as(_PD)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


class BFHandle:
    """A factorization resident on the current GPU (owns a bf_handle)."""

    def __init__(self, factors, precision="f32", stream=None, options=None):
        """options: dict of bf_plan_options fields (kernel-path variants), or None."""
        self.lib = load_library()
        f = factors
        self.radix, self.leaf, self.L, self.r = int(f["radix"]), int(f["leaf"]), int(f["L"]), int(f["r"])
        self.h = self.L // 2
        self.N = self.leaf * self.radix ** self.L
        self.precision = precision
        self.prec_code = PRECISIONS[precision]
        shape = BFShape(self.radix, self.leaf, self.L, self.r, self.N)
        keep = [_as_f64(f["VL"]), _as_f64(f["UL"]), _as_f64(f["S"])]
        Hs = [_as_f64(x) for x in f["H"]]
        Gs = [_as_f64(x) for x in f["G"]]
        Harr = (_PD * max(1, len(Hs)))(*[_ptr(x) for x in Hs])
        Garr = (_PD * max(1, len(Gs)))(*[_ptr(x) for x in Gs])
        fh = BFFactorsHost(_ptr(keep[0]), Harr, _ptr(keep[2]), Garr, _ptr(keep[1]))
        opts = None
        if options:
            opts = BFPlanOptions()
            for k, v in options.items():
                setattr(opts, k, int(v))
        st, h = bf_create_from_factors_ex(shape, fh, self.prec_code, opts,
                                          _stream_ptr(stream) if stream is not None else 0)
        if st != BF_OK:
            raise BFError(st, bf_last_error(None))
        self.handle = h
        path = ctypes.c_int32()
        self.lib.bf_query(h, None, None, ctypes.byref(path))
        self.path = path.value

    @property
    def complex_dtype(self):
        import torch
        return torch.complex128 if self.precision == "f64" else torch.complex64

    def _check(self, st):
        if st != BF_OK:
            raise BFError(st, bf_last_error(self.handle))

    def _prep(self, x):
        import torch
        if x.dim() == 1:
            x = x[:, None]
        if x.dtype != self.complex_dtype or not x.is_cuda:
            raise TypeError(f"expected a {self.complex_dtype} CUDA tensor, got {x.dtype} on {x.device}")
        if x.shape[0] != self.N:
            raise ValueError(f"expected {self.N} rows, got {x.shape[0]}")
        if x.stride(1) != 1:
            x = x.contiguous()
        return x

    def apply(self, g, out=None, stream=None, adjoint=False):
        import torch
        squeeze = g.dim() == 1
        g = self._prep(g)
        nrhs, ld = g.shape[1], g.stride(0)
        if out is None:
            out = torch.empty((self.N, ld), dtype=g.dtype, device=g.device)[:, :nrhs]
        fn = bf_apply_adjoint if adjoint else bf_apply
        self._check(fn(self.handle, g.data_ptr(), out.data_ptr(), nrhs, ld, _stream_ptr(stream)))
        return out[:, 0] if squeeze else out

    def apply_adjoint(self, w, out=None, stream=None):
        return self.apply(w, out=out, stream=stream, adjoint=True)

    def backward(self, g, grad_u, factor_grads=True, need_grad_g=True, flags=BF_BWD_RECOMPUTE,
                 stream=None):
        """Returns (grad_g, grads) with grads a dict in the canonical layout (torch tensors)."""
        import torch
        g = self._prep(g)
        grad_u = self._prep(grad_u)
        if grad_u.stride(0) != g.stride(0):
            grad_u = grad_u.contiguous()
            g = g.contiguous()
        nrhs, ld = g.shape[1], g.stride(0)
        dev = g.device
        cd = self.complex_dtype
        rd = torch.float64 if self.precision == "f64" else torch.float32
        grad_g = torch.empty((self.N, ld), dtype=cd, device=dev)[:, :nrhs] if need_grad_g else None
        grads = None
        out = {}
        if factor_grads:
            R, r, L, h = self.radix, self.r, self.L, self.h
            P = R ** L
            out["VL"] = torch.empty((P, self.leaf, r), dtype=cd, device=dev)
            out["UL"] = torch.empty((P, self.leaf, r), dtype=cd, device=dev)
            out["S"] = torch.empty((R ** h, R ** h, r), dtype=rd, device=dev)
            out["H"] = [torch.empty((R ** (l + 1), R ** (L - l - 1), r, R * r), dtype=cd, device=dev)
                        for l in range(h, L)]
            out["G"] = [torch.empty((R ** (l + 1), R ** (L - l - 1), r, R * r), dtype=cd, device=dev)
                        for l in range(h, L)]
            Harr = (ctypes.c_void_p * h)(*[t.data_ptr() for t in out["H"]])
            Garr = (ctypes.c_void_p * h)(*[t.data_ptr() for t in out["G"]])
            grads = BFFactorGrads(out["VL"].data_ptr(), Harr, out["S"].data_ptr(), Garr,
                                  out["UL"].data_ptr())
            grads._keep = (Harr, Garr)
        st = bf_backward(self.handle, g.data_ptr(), grad_u.data_ptr(),
                         grad_g.data_ptr() if grad_g is not None else None, grads, nrhs, ld,
                         flags, _stream_ptr(stream))
        self._check(st)
        return grad_g, out

    def set_profiling(self, on=True):
        self._check(self.lib.bf_set_profiling(self.handle, 1 if on else 0))

    def kernel_times(self, reset=True):
        cap = 256
        names = (ctypes.c_char * 64 * cap)()
        ms = (ctypes.c_double * cap)()
        launches = (ctypes.c_int64 * cap)()
        count = ctypes.c_int32()
        self._check(self.lib.bf_kernel_times(self.handle, names, ms, launches, cap,
                                             ctypes.byref(count), 1 if reset else 0))
        return {bytes(names[k]).split(b"\0")[0].decode(): (ms[k], launches[k])
                for k in range(min(count.value, cap))}

    def close(self):
        if getattr(self, "handle", None):
            bf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
