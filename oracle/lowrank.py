"""Low-rank primitives of Sec. 2, in FP64 with LAPACK as the building block.

Readings of points the paper leaves open (each listed with its reason in the
design notes):
  * truncation keeps exactly r triplets; a block with fewer than r singular
    values is zero-padded to r so every factor block has a fixed shape;
  * pivoted QR is LAPACK geqp3 (scipy.linalg.qr with pivoting); a pivoted LQ
    of Z is the pivoted QR of Z^*;
  * sampled rows/columns are drawn uniformly without replacement from the
    indices not already selected; when the sample would cover the whole
    dimension, every index is used;
  * pseudo-inverses use a relative singular-value cutoff of 1e-14.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

PINV_RCOND = 1e-14


def truncated_svd(Z, r):
    """Rank-r truncated SVD Z ~ U0 diag(s) V0h, padded with zeros up to r (Sec. 2).

    Returns U0 (m x r), s (r,), V0h (r x n); singular values in decreasing order.
    """
    Z = np.asarray(Z, dtype=np.complex128)
    m, n = Z.shape
    U, s, Vh = sla.svd(Z, full_matrices=False, lapack_driver="gesdd")
    k = min(r, s.size)
    U0 = np.zeros((m, r), dtype=np.complex128)
    V0h = np.zeros((r, n), dtype=np.complex128)
    s0 = np.zeros(r)
    U0[:, :k] = U[:, :k]
    V0h[:k] = Vh[:k]
    s0[:k] = s[:k]
    return U0, s0, V0h


def form_usv(U0, s, V0h, drop_rel=1e-14):
    """First equivalent form (Sec. 2): U = U0 S0, S = S0^{-1}, V^* = S0 V0^*.

    Triplets with sigma_k <= drop_rel * sigma_1 (including zero padding) get
    zero columns in U and V and a zero weight in S, so S stays finite.
    """
    s = np.asarray(s, dtype=np.float64)
    keep = s > drop_rel * (s[0] if s.size and s[0] > 0 else 0.0)
    keep &= s > 0
    U = U0 * np.where(keep, s, 0.0)[None, :]
    Vs = V0h * np.where(keep, s, 0.0)[:, None]          # S0 V0^*
    S = np.where(keep, 1.0 / np.where(keep, s, 1.0), 0.0)
    return U, S, Vs.conj().T                            # V with V^* = S0 V0^*


def _pivoted_qr(A):
    Q, Rm, piv = sla.qr(A, mode="economic", pivoting=True)
    return Q, Rm, piv


def pivoted_qr_q(A):
    """Q factor of LAPACK's pivoted QR (geqp3) of A (Alg. 2.1, step 2)."""
    return _pivoted_qr(A)[0]


def _qr_pivots(A):
    """Column order chosen by LAPACK's pivoted QR (geqp3) of A."""
    _, piv = sla.qr(A, mode="r", pivoting=True)
    return piv


def _sample_excluding(rng, dim, count, exclude):
    """`count` fresh indices of range(dim) not in `exclude`, or all of them."""
    exclude = np.asarray(sorted(set(int(e) for e in exclude)), dtype=np.int64)
    if count + exclude.size >= dim:
        return np.setdiff1d(np.arange(dim), exclude)
    pool = np.setdiff1d(np.arange(dim), exclude)
    return np.sort(rng.choice(pool, size=count, replace=False))


def randomized_sampling(Z_entries, mdim, ndim, r, rng, q=3, iters=3):
    """Algorithm 2.2 (Sec. 2.2): rank-r approximate SVD from sampled rows/columns.

    `Z_entries(I, J)` returns the dense submatrix Z[I][:, J] of the implicit
    mdim x ndim matrix Z.  q is the multiplicative oversampling and `iters`
    the number of alternations of steps 2 and 3 (the paper uses q = 3 and at
    most three alternations, Sec. 2.2 and Sec. 4).  Returns U0, s, V0h padded
    to rank r.
    """
    rows_all = np.arange(mdim)
    cols_all = np.arange(ndim)
    rq = r * q
    pi_col = np.zeros(0, dtype=np.int64)      # step 1: both important sets empty
    pi_row = np.zeros(0, dtype=np.int64)
    for _ in range(iters):                    # step 4: repeat steps 2 and 3
        # step 2: rq random rows plus the important rows; pivoted QR of Z_{I,:}
        I = np.union1d(_sample_excluding(rng, mdim, rq, pi_row), pi_row)
        piv = _qr_pivots(Z_entries(I, cols_all))
        pi_col = np.sort(piv[:r])
        # step 3: rq random columns plus the important columns; pivoted LQ of Z_{:,J}
        J = np.union1d(_sample_excluding(rng, ndim, rq, pi_col), pi_col)
        piv = _qr_pivots(Z_entries(rows_all, J).conj().T)
        pi_row = np.sort(piv[:r])
    # step 5: orthonormal bases of the important columns and rows
    Qc, _, _ = _pivoted_qr(Z_entries(rows_all, pi_col))
    Qr, _, _ = _pivoted_qr(Z_entries(pi_row, cols_all).conj().T)
    Q_col = Qc[:, :r]
    Q_row = Qr[:, :r]
    Q_row_h = Q_row.conj().T
    # step 6: least-squares middle matrix on the important plus a few extra samples
    J = np.union1d(pi_col, _sample_excluding(rng, ndim, rq, pi_col))
    I = np.union1d(pi_row, _sample_excluding(rng, mdim, rq, pi_row))
    M = (np.linalg.pinv(Q_col[I, :], rcond=PINV_RCOND)
         @ Z_entries(I, J)
         @ np.linalg.pinv(Q_row_h[:, J], rcond=PINV_RCOND))
    # step 7: SVD of the middle matrix
    UM, sM, VMh = sla.svd(M, full_matrices=False, lapack_driver="gesdd")
    k = min(r, sM.size)
    U0 = np.zeros((mdim, r), dtype=np.complex128)
    V0h = np.zeros((r, ndim), dtype=np.complex128)
    s0 = np.zeros(r)
    U0[:, :k] = Q_col @ UM[:, :k]
    V0h[:k] = VMh[:k] @ Q_row_h
    s0[:k] = sM[:k]
    return U0, s0, V0h


def randomized_svd(Z_times, Zh_times, mdim, ndim, r, rng, p=5):
    """Algorithm 2.1 (Sec. 2.1): rank-r approximate SVD from products with Z and Z^*.

    `Z_times(C)` returns Z @ C for an ndim x k matrix C, `Zh_times(R)` returns
    Z^* @ R for an mdim x k matrix R.  p is the additive oversampling (p = 5 in
    the paper's experiments, Sec. 4).
    """
    def gauss(shape):
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * np.sqrt(0.5)

    # step 1: Gaussian test matrices with r + p columns
    R_col = gauss((ndim, r + p))
    R_row = gauss((mdim, r + p))
    # step 2: pivoted QR of Z R_col and Z^* R_row; keep the first r columns of Q
    Q_col = _pivoted_qr(Z_times(R_col))[0][:, :r]
    Q_row = _pivoted_qr(Zh_times(R_row))[0][:, :r]
    # step 3: M = Q_col^* Z Q_row and its truncated SVD
    M = Q_col.conj().T @ Z_times(Q_row)
    UM, sM, VMh = sla.svd(M, full_matrices=False, lapack_driver="gesdd")
    k = min(r, sM.size)
    # step 4
    U0 = np.zeros((mdim, r), dtype=np.complex128)
    V0h = np.zeros((r, ndim), dtype=np.complex128)
    s0 = np.zeros(r)
    U0[:, :k] = Q_col @ UM[:, :k]
    V0h[:k] = VMh[:k] @ Q_row.conj().T
    s0[:k] = sM[:k]
    return U0, s0, V0h
