"""Construction of the butterfly factorization (Sec. 3) on the host in FP64, as the
construction's stability needs; the result is the canonical factor set that
``bf_create_from_factors`` (``BFHandle``) takes.

Two routes, the two cases of Sec. 3.1:

* ``construct_from_entries``: entries of K are available (a callable returning
  submatrices); every middle-level block is factorized by randomized sampling
  (Algorithm 2.2).
* ``construct_from_products``: only products with K and K^* are available (for
  instance this library's ``bf_apply`` composed with an FFT, Sec. 4 Example 3, on
  the GPU); the middle level comes from the randomized SVD (Algorithm 2.1) of two
  products with block-diagonal Gaussian matrices.

Both then factorize the middle level recursively (Sec. 3.2.1, 3.2.2), batched
over all nodes of a level.

    f = construct_from_products(N, radix, leaf, r, apply, apply_adjoint)
    h = BFHandle(f, "bf16x3")

``apply(X)`` and ``apply_adjoint(X)`` take and return device tensors of shape
[N][k] (complex64 or complex128); the result is the canonical host factor set
that ``bf_create_from_factors`` takes.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.linalg as sla


def _depth(N, leaf, radix):
    P, rem = divmod(int(N), int(leaf))
    L = int(round(np.log(P) / np.log(radix))) if P > 1 else 0
    if rem or radix ** L != P:
        raise ValueError("N / leaf must be a power of the radix")
    if L % 2:
        raise ValueError("the tree depth must be even")
    return L


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def _one_blas_thread():
    """BLAS/LAPACK single-threaded while the work is spread over Python threads."""
    try:
        from threadpoolctl import threadpool_limits
        return threadpool_limits(1)
    except Exception:  # threadpoolctl missing: leave the BLAS pool as it is
        import contextlib
        return contextlib.nullcontext()


def _batched_svd(Z):
    """np.linalg.svd over the leading axes, split over threads (LAPACK runs without
    the interpreter lock)."""
    flat = Z.reshape((-1,) + Z.shape[-2:])
    n = flat.shape[0]
    nt = min(_threads(), n)
    if nt <= 1 or n < 8:
        return np.linalg.svd(Z, full_matrices=False)
    cuts = np.linspace(0, n, nt + 1).astype(int)
    with _one_blas_thread(), ThreadPoolExecutor(nt) as ex:
        parts = list(ex.map(lambda q: np.linalg.svd(flat[cuts[q]:cuts[q + 1]], full_matrices=False),
                            range(nt)))
    U = np.concatenate([a[0] for a in parts]).reshape(Z.shape[:-1] + (parts[0][0].shape[-1],))
    s = np.concatenate([a[1] for a in parts]).reshape(Z.shape[:-2] + (parts[0][1].shape[-1],))
    Vh = np.concatenate([a[2] for a in parts]).reshape(Z.shape[:-2] + parts[0][2].shape[-2:])
    return U, s, Vh


def _svd_rank(Z, r):
    """Batched rank-r truncated SVD over the leading axes, zero-padded to r."""
    U, s, Vh = _batched_svd(Z)
    k = min(r, s.shape[-1])
    U0 = np.zeros(Z.shape[:-1] + (r,), dtype=np.complex128)
    s0 = np.zeros(Z.shape[:-2] + (r,))
    V0h = np.zeros(Z.shape[:-2] + (r, Z.shape[-1]), dtype=np.complex128)
    U0[..., :k] = U[..., :k]
    s0[..., :k] = s[..., :k]
    V0h[..., :k, :] = Vh[..., :k, :]
    return U0, s0, V0h


def _middle_block(Y, W, C, r):
    """Rank-r SVD of Z = K^h_ij from Y = Z C and W = Z^* R (Alg. 2.1).

    Q_col and Q_row are the first r columns of the pivoted-QR Q factors of Y and
    W.  The middle matrix Q_col^* Z Q_row is taken from the sketches alone:
    Z ~ Z Q_row Q_row^* gives Q_col^* Y = M (Q_row^* C), solved in the least
    squares sense.
    """
    Qc = sla.qr(Y, mode="economic", pivoting=True)[0][:, :r]
    Qr = sla.qr(W, mode="economic", pivoting=True)[0][:, :r]
    M = np.linalg.lstsq((Qr.conj().T @ C).T, (Qc.conj().T @ Y).T, rcond=1e-14)[0].T
    Um, sm, Vmh = _svd_rank(M, r)
    return Qc @ Um, sm, Vmh @ Qr.conj().T


def _recursive(Wb, R, r, levels):
    """Sec. 3.2.1 for every middle-level node at once.

    Wb[node][j][rows][r] holds the column blocks U^h_{node, j} (or V^h).  At each
    level the rows of child c of every node, over R consecutive column blocks,
    are approximated in the third form U0 S0 . V0^* (batched SVD).  Returns the
    per-level block arrays [node, child-path, j'][r][R r] flattened to the
    canonical order and the leaf blocks.
    """
    cur = Wb                                   # [nodes][nb][rows][r]
    blocks = []
    for _ in range(levels):
        nodes, nb, rows, _ = cur.shape
        crow = rows // R
        # Z[a, c, jp] = [cur[a, R jp + cc, c rows] for cc] -> [nodes][R][nb/R][crow][R r]
        Z = cur.reshape(nodes, nb // R, R, R, crow, r)          # [a][jp][cc][c][crow][r]
        Z = Z.transpose(0, 3, 1, 4, 2, 5).reshape(nodes, R, nb // R, crow, R * r)
        U0, s, V0h = _svd_rank(Z, r)
        blocks.append(V0h.reshape(nodes * R, nb // R, r, R * r))
        cur = (U0 * s[..., None, :]).reshape(nodes * R, nb // R, crow, r)
    return blocks, cur[:, 0]


def _pick(rng, dim, count, taken):
    """`count` random indices of range(dim) outside `taken` (all of them if fewer remain)."""
    free = np.setdiff1d(np.arange(dim), taken, assume_unique=False)
    if free.size <= count:
        return free
    return np.sort(rng.choice(free, size=count, replace=False))


def _sampled_block(entries, b, r, rng, q=3, iters=3):
    """Rank-r SVD of one b x b block Z from O(r) of its rows and columns (Alg. 2.2).

    entries(I, J) returns Z[I][:, J].  Steps 2-3 alternate `iters` times: a
    pivoted QR of the sampled rows (plus the important rows so far) picks the r
    important columns, a pivoted QR of the conjugate transpose of the sampled
    columns (the pivoted LQ) picks the r important rows.  Step 5 fits the middle
    matrix on the important indices plus r q fresh ones in least squares.
    """
    pcol = np.zeros(0, dtype=np.int64)
    prow = np.zeros(0, dtype=np.int64)
    for _ in range(iters):
        I = np.union1d(_pick(rng, b, r * q, prow), prow)
        piv = sla.qr(entries(I, np.arange(b)), mode="r", pivoting=True)[1]
        pcol = np.sort(piv[:r])
        J = np.union1d(_pick(rng, b, r * q, pcol), pcol)
        piv = sla.qr(entries(np.arange(b), J).conj().T, mode="r", pivoting=True)[1]
        prow = np.sort(piv[:r])
    Qc = sla.qr(entries(np.arange(b), pcol), mode="economic", pivoting=True)[0][:, :r]
    Qr = sla.qr(entries(prow, np.arange(b)).conj().T, mode="economic", pivoting=True)[0][:, :r]
    I = np.union1d(prow, _pick(rng, b, r * q, prow))
    J = np.union1d(pcol, _pick(rng, b, r * q, pcol))
    M = (np.linalg.pinv(Qc[I], rcond=1e-14) @ entries(I, J)
         @ np.linalg.pinv(Qr[J].conj().T, rcond=1e-14))
    Um, sm, Vmh = _svd_rank(M, r)
    return Qc @ Um, sm, Vmh @ Qr.conj().T


def _first_form(U0, s, V0h, drop_rel):
    keep = (s > 0) & (s > drop_rel * (s[0] if s.size else 0.0))
    sk = np.where(keep, s, 0.0)
    return U0 * sk, (V0h * sk[:, None]).conj().T, np.where(keep, 1.0 / np.where(keep, s, 1.0), 0.0)


def _from_middle(N, R, leaf, L, r, Uh, Vh, S):
    lv = L - L // 2
    Gb, UL = _recursive(Uh, R, r, lv)
    Hb, VL = _recursive(Vh, R, r, lv)
    return {"radix": R, "leaf": int(leaf), "L": L, "r": int(r),
            "VL": VL, "UL": UL, "S": S, "H": Hb, "G": Gb}


def _factor_shapes(N, R, leaf, L, r):
    h = L // 2
    P = R ** L
    return {"radix": R, "leaf": int(leaf), "L": L, "r": int(r),
            "VL": np.zeros((P, leaf, r), dtype=np.complex128),
            "UL": np.zeros((P, leaf, r), dtype=np.complex128),
            "S": np.zeros((R ** h, R ** h, r)),
            "H": [np.zeros((R ** (l + 1), R ** (L - l - 1), r, R * r), dtype=np.complex128) for l in range(h, L)],
            "G": [np.zeros((R ** (l + 1), R ** (L - l - 1), r, R * r), dtype=np.complex128) for l in range(h, L)]}


def _streamed_from_entries(N, R, leaf, L, r, entries, q, iters, seed, drop_rel):
    """The O(N log N)-memory order of Sec. 3.3: for one middle node at a time, the
    blocks of its row (U side) or column (V side) are factorized by Alg. 2.2 and
    the node's U^h_i (V^h_j) is factorized recursively at once, so only O(N r)
    values of the middle level exist at any time.  Each block draws from its own
    stream, so the U and V sides reproduce the same block factorizations."""
    h = L // 2
    m = R ** h
    b = N // m
    lv = L - h
    f = _factor_shapes(N, R, leaf, L, r)
    per_node = (R ** L) // m                        # leaves below one middle node

    def block(i, j):
        rng = np.random.default_rng([seed, i, j])
        rows, cols = i * b, j * b
        U0, s, V0h = _sampled_block(lambda I, J: entries(rows + I, cols + J), b, r, rng, q, iters)
        return _first_form(U0, s, V0h, drop_rel)

    nt = min(_threads(), m) if b >= 256 else 1
    with _one_blas_thread(), ThreadPoolExecutor(nt) as ex:
        for side in ("U", "V"):
            for a in range(m):
                pairs = [(a, j) for j in range(m)] if side == "U" else [(i, a) for i in range(m)]
                W = np.zeros((1, m, b, r), dtype=np.complex128)
                for k, (U, V, S) in enumerate(ex.map(lambda ij: block(*ij), pairs)):
                    W[0, k] = U if side == "U" else V
                    if side == "U":
                        f["S"][a, k] = S
                blocks, leaves = _recursive(W, R, r, lv)
                dst = f["G"] if side == "U" else f["H"]
                for t in range(lv):
                    n_t = R ** (t + 1)
                    dst[t][a * n_t:(a + 1) * n_t] = blocks[t]
                (f["UL"] if side == "U" else f["VL"])[a * per_node:(a + 1) * per_node] = leaves
    return f


def construct_from_entries(N, radix, leaf, r, entries, q=3, iters=3, seed=0, drop_rel=1e-14,
                           streamed=None):
    """Canonical factors of K from its entries (the second case of Sec. 3.1).

    entries(rows, cols) returns the dense submatrix K[rows][:, cols] (FP64 complex)
    for index arrays in tree order.  Every middle-level block gets its rank-r SVD
    by randomized sampling (Alg. 2.2), with its own random stream, so the result
    does not depend on the order the blocks are processed in; the blocks are
    spread over threads, and the recursion of Sec. 3.2 is batched over every node.

    streamed: True factorizes one middle node at a time (Sec. 3.3: working memory
    O(N r) instead of the 2 N^(3/2) r / leaf^(1/2) values of U^h and V^h, at twice the
    middle-level work); None (default) streams when U^h and V^h would take more than
    4 GB.  Both orders give the same factors.
    """
    R = int(radix)
    L = _depth(N, leaf, R)
    m = R ** (L // 2)
    b = N // m
    if streamed is None:
        streamed = 2 * m * m * b * r * 16 > 4e9
    if streamed:
        return _streamed_from_entries(N, R, leaf, L, r, entries, q, iters, seed, drop_rel)
    Uh = np.zeros((m, m, b, r), dtype=np.complex128)
    Vh = np.zeros((m, m, b, r), dtype=np.complex128)
    S = np.zeros((m, m, r))

    def row(i):
        for j in range(m):
            rng = np.random.default_rng([seed, i, j])
            rows, cols = i * b, j * b
            U0, s, V0h = _sampled_block(lambda I, J: entries(rows + I, cols + J), b, r, rng, q, iters)
            Uh[i, j], Vh[j, i], S[i, j] = _first_form(U0, s, V0h, drop_rel)

    # small blocks spend their time in the interpreter, where threads only contend
    nt = min(_threads(), m) if b >= 256 else 1
    with _one_blas_thread(), ThreadPoolExecutor(nt) as ex:
        list(ex.map(row, range(m)))
    return _from_middle(N, R, leaf, L, r, Uh, Vh, S)


def construct_from_products(N, radix, leaf, r, apply, apply_adjoint, p=5, seed=0, drop_rel=1e-14,
                            device="cuda"):
    """Canonical factors of K (see the module docstring); the test matrices are
    passed to the black box as tensors on `device`."""
    import torch

    R = int(radix)
    L = _depth(N, leaf, R)
    h = L // 2
    m = R ** h
    b = N // m
    k = r + p
    rng = np.random.default_rng(seed)
    Cb = (rng.standard_normal((m, b, k)) + 1j * rng.standard_normal((m, b, k))) / np.sqrt(2)
    Rb = (rng.standard_normal((m, b, k)) + 1j * rng.standard_normal((m, b, k))) / np.sqrt(2)

    probe = apply(torch.zeros((N, 1), dtype=torch.complex128, device=device))
    dt = probe.dtype

    def block_diag(blocks):
        # N x m k with block j (rows j b .., columns j k ..) = blocks[j], built on the device
        X = torch.zeros((m, b, m, k), dtype=dt, device=device)
        idx = torch.arange(m, device=device)
        X[idx, :, idx, :] = torch.from_numpy(blocks).to(device, dt)
        return X.reshape(N, m * k)

    KC = apply(block_diag(Cb)).cpu().numpy().astype(np.complex128)
    KR = apply_adjoint(block_diag(Rb)).cpu().numpy().astype(np.complex128)

    # middle level: K^h_ij ~ U^h_ij S^h_ij (V^h_ji)^*, first form of Sec. 2
    Uh = np.zeros((m, m, b, r), dtype=np.complex128)   # [i][j]
    Vh = np.zeros((m, m, b, r), dtype=np.complex128)   # [j][i]
    S = np.zeros((m, m, r))

    def row(i):
        for j in range(m):
            U0, s, V0h = _middle_block(KC[i * b:(i + 1) * b, j * k:(j + 1) * k],
                                       KR[j * b:(j + 1) * b, i * k:(i + 1) * k], Cb[j], r)
            Uh[i, j], Vh[j, i], S[i, j] = _first_form(U0, s, V0h, drop_rel)

    with _one_blas_thread(), ThreadPoolExecutor(min(_threads(), m)) as ex:
        list(ex.map(row, range(m)))
    # the node of depth t below middle node i with child path c is R^(t+1) i + path:
    # _recursive already orders its outputs that way
    return _from_middle(N, R, leaf, L, r, Uh, Vh, S)
