"""MI355X butterfly-factorization apply (gfx950 HIP library + thin Python binding).

    from paper_1502_01379_amd import BFHandle, bf_apply_autograd, BFOperator

`BFHandle(factors, precision)` uploads a factorization given in the canonical
layout (see include/bf.h) and applies it to complex torch tensors on the GPU;
`bf_apply_autograd` and `BFOperator` expose the hand-written adjoint and
backward kernels to torch.autograd.  Precisions: "f64", "f32", "bf16x3"
(split BF16, three MFMA products, FP32 accumulation) and "f16x3".
`construct_from_entries` and `construct_from_products` build a factorization on
the host in FP64 from entries of K (Alg. 2.2) or from products with K and K^*
(Alg. 2.1), the two cases of Sec. 3.1.  The batched FP64 GPU primitives of the
construction (`kernel_entries`, `batched_svd`, `batched_qr`,
`batched_column_pivots`) are exposed; `construct_on_device`, their driver for the
whole entry route, is switched off for now (it raises BFError).
"""
from __future__ import annotations

from .binding import (BF_BWD_RECOMPUTE, BF_BWD_STORE_ALL, BFError, BFHandle, PRECISIONS,  # noqa: F401
                      batched_column_pivots, batched_qr, batched_svd, construct_on_device,
                      kernel_entries, load_library)

from .construct import construct_from_entries, construct_from_products  # noqa: F401,E402

__all__ = ["BFHandle", "BFError", "BFOperator", "bf_apply_autograd", "load_library", "PRECISIONS",
           "BF_BWD_RECOMPUTE", "BF_BWD_STORE_ALL", "construct_from_entries", "construct_from_products",
           "construct_on_device", "kernel_entries", "batched_svd", "batched_qr", "batched_column_pivots"]

_FACTOR_KEYS = ("VL", "UL", "S")


def _flat_order(h):
    return list(_FACTOR_KEYS) + [("H", t) for t in range(h)] + [("G", t) for t in range(h)]


def _autograd_function():
    import torch

    class BFApply(torch.autograd.Function):
        """u = K_BF g with gradients for g and for every factor tensor passed in."""

        @staticmethod
        def forward(ctx, g, handle, flags, *factor_tensors):
            ctx.handle = handle
            ctx.flags = flags
            ctx.nfac = len(factor_tensors)
            ctx.save_for_backward(g)
            return handle.apply(g)

        @staticmethod
        def backward(ctx, grad_u):
            (g,) = ctx.saved_tensors
            need_fac = ctx.nfac > 0 and any(ctx.needs_input_grad[3:])
            squeeze = g.dim() == 1
            grad_g, grads = ctx.handle.backward(
                g, grad_u.contiguous(), factor_grads=need_fac,
                need_grad_g=ctx.needs_input_grad[0], flags=ctx.flags)
            if grad_g is not None and squeeze:
                grad_g = grad_g[:, 0]
            flat = [None] * ctx.nfac
            if need_fac:
                for k, key in enumerate(_flat_order(ctx.handle.h)[:ctx.nfac]):
                    flat[k] = grads[key] if isinstance(key, str) else grads[key[0]][key[1]]
            return (grad_g, None, None, *flat)

    return BFApply


_BFApply = None


def bf_apply_autograd(g, handle, *factor_tensors, flags=BF_BWD_RECOMPUTE):
    """Differentiable u = K_BF g.

    `factor_tensors` are optional tensors standing for the factors held by
    `handle`, in the order VL, UL, S, H[0..h-1], G[0..h-1]; their gradients
    come from the library's backward kernels.
    """
    global _BFApply
    if _BFApply is None:
        _BFApply = _autograd_function()
    return _BFApply.apply(g, handle, flags, *factor_tensors)


class BFOperator:
    """A factorization whose factors are torch parameters on the GPU.

    The handle is built from the parameters' values; call `refresh()` after
    changing them (for example after an optimizer step).
    """

    def __init__(self, factors, precision="f32", device="cuda"):
        import torch
        self.precision = precision
        cd = torch.complex128 if precision == "f64" else torch.complex64
        rd = torch.float64 if precision == "f64" else torch.float32
        meta = {k: factors[k] for k in ("radix", "leaf", "L", "r")}
        self.meta = meta
        self.params = {
            "VL": torch.nn.Parameter(torch.as_tensor(factors["VL"]).to(device=device, dtype=cd)),
            "UL": torch.nn.Parameter(torch.as_tensor(factors["UL"]).to(device=device, dtype=cd)),
            "S": torch.nn.Parameter(torch.as_tensor(factors["S"]).to(device=device, dtype=rd)),
            "H": [torch.nn.Parameter(torch.as_tensor(x).to(device=device, dtype=cd)) for x in factors["H"]],
            "G": [torch.nn.Parameter(torch.as_tensor(x).to(device=device, dtype=cd)) for x in factors["G"]],
        }
        self.handle = None
        self.refresh()

    def parameters(self):
        p = self.params
        return [p["VL"], p["UL"], p["S"], *p["H"], *p["G"]]

    def refresh(self):
        p = self.params
        host = dict(self.meta)
        for k in ("VL", "UL", "S"):
            host[k] = p[k].detach().cpu().numpy()
        host["H"] = [x.detach().cpu().numpy() for x in p["H"]]
        host["G"] = [x.detach().cpu().numpy() for x in p["G"]]
        if self.handle is not None:
            self.handle.close()
        self.handle = BFHandle(host, self.precision)

    def __call__(self, g, flags=BF_BWD_RECOMPUTE):
        return bf_apply_autograd(g, self.handle, *self.parameters(), flags=flags)
