"""FP64 CPU oracle for the butterfly factorization (Li, Yang, Martin, Ho, Ying).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this
package: it is used by `tests/`, by `__graft_entry__.smoke()` and by the
CPU-baseline leg of `bench.py`.  It shares no code with the HIP library;
both sides consume the same seeded inputs from `bf_inputs`.

Contents, each written from the paper's text:

    kernels    kernel entries of the paper's examples (Sec. 1.1 Fourier matrix,
               Sec. 4 Example 1 FIO, Example 2 Hankel sum) and the 2D generalised
               Radon transform; dense matvec on selected rows.
    lowrank    truncated SVD and its three forms (Sec. 2), randomized SVD
               (Sec. 2.1, Algorithm 2.1), randomized sampling (Sec. 2.2,
               Algorithm 2.2).
    construct  middle-level factorization (Sec. 3.1) and recursive
               factorization of U^h and V^h (Sec. 3.2), plus the
               O(N log N)-memory streamed order (Sec. 3.3).
    apply      u = K g through the factor product (Sec. 1.2 and the closing
               equation of Sec. 3.2), its adjoint and the gradient of a loss.
    sparse     the factors assembled as explicit sparse matrices following the
               block pictures of Sec. 3.1 and 3.2.
    metrics    the relative error on sampled rows of Sec. 4.
"""
from . import kernels, lowrank, construct, apply, sparse, metrics  # noqa: F401
from .kernels import Kernel1D, Kernel2D, fourier, fio, grt2d  # noqa: F401
from .construct import construct_factors, construct_factors_matvec  # noqa: F401
from .apply import bf_apply, bf_apply_adjoint, bf_grad  # noqa: F401
from .metrics import rel_err  # noqa: F401
