"""Error measure of Sec. 4: relative l2 error over a sampled row set S."""
from __future__ import annotations

import numpy as np


def rel_err(u_a, u_d):
    """sqrt(sum_S |u_a - u_d|^2 / sum_S |u_d|^2), summed over every compared entry.

    With several right-hand sides the sums run over the sampled rows and all
    columns (a Frobenius-norm reading of the one-vector formula of Sec. 4).
    """
    u_a = np.asarray(u_a, dtype=np.complex128)
    u_d = np.asarray(u_d, dtype=np.complex128)
    num = np.sum(np.abs(u_a - u_d) ** 2)
    den = np.sum(np.abs(u_d) ** 2)
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))

