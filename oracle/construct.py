"""Construction of the butterfly factorization (Sec. 3), FP64.

Stage 1, the middle-level factorization (Sec. 3.1): every block
K^h_{i,j} = K(A^h_i, B^h_j), i, j < m = R^h, gets a rank-r approximation
U^h_{i,j} S^h_{i,j} (V^h_{j,i})^* in the first equivalent form of Sec. 2
(U = U0 S0, S = S0^{-1}, V^* = S0 V0^*), either by randomized sampling of
its entries (Algorithm 2.2, the paper's "second case"), by random
matrix-vector products with K and K^* (Algorithm 2.1, the "first case";
`construct_factors_matvec`) or, as a deterministic reference, by a
truncated SVD of the whole block.

Stage 2, the recursive factorization (Sec. 3.2.1, 3.2.2): for l = h .. L-1,
the rows of U^l_i belonging to child c of X-node i, restricted to the R
column blocks j' R .. j' R + R - 1, are approximated by a truncated SVD in
the third form: [U^{l,c}_{i,Rj'} ... U^{l,c}_{i,Rj'+R-1}] ~ U^{l+1}_{Ri+c,j'} G^l_{Ri+c,j'}.
V is factorized by the same procedure, giving H.

Each X-node i of the middle level (and each Omega-node j) is processed on
its own, which is the O(N log N)-memory order of Sec. 3.3; with
`streamed=False` all middle-level blocks are factorized first and kept.

Output: a dict in the canonical layout documented in `bf_inputs`:
    VL, UL [P][n0][r]; H[t], G[t] [R^(l+1)][R^(L-l-1)][r][R r] for l = h + t;
    S [m][m][r]; plus radix, leaf, L, r.
"""
from __future__ import annotations

import numpy as np

from .lowrank import truncated_svd, randomized_sampling, form_usv, pivoted_qr_q


def tree_depth(N, leaf, radix):
    P, rem = divmod(int(N), int(leaf))
    if rem:
        raise ValueError("N must be a multiple of the leaf size")
    L = 0
    while radix ** L < P:
        L += 1
    if radix ** L != P:
        raise ValueError("N/leaf must be a power of the radix")
    if L % 2:
        raise ValueError("tree depth L must be even (Sec. 1.2)")
    return L


def middle_block(kernel, i, j, b, r, method, seed, q=3, iters=3):
    """Rank-r factorization of K^h_{i,j} in the first form of Sec. 2.

    Returns (U^h_{i,j}, diag S^h_{i,j}, V^h_{j,i}) with shapes (b,r), (r,), (b,r).
    The block's random draws come from a generator seeded by (seed, i, j) so a
    block factorized twice (streamed order) gives the same result.
    """
    rows = np.arange(i * b, (i + 1) * b)
    cols = np.arange(j * b, (j + 1) * b)
    if method == "svd":
        U0, s, V0h = truncated_svd(kernel.entries(rows, cols), r)
    elif method == "sampling":
        rng = np.random.default_rng(np.random.SeedSequence(seed, spawn_key=(i, j)))
        U0, s, V0h = randomized_sampling(
            lambda I, J: kernel.entries(rows[I], cols[J]), b, b, r, rng, q=q, iters=iters)
    else:
        raise ValueError(f"unknown middle-level method {method!r}")
    return form_usv(U0, s, V0h)


def recursive_factorization(W, R, r, levels):
    """Recursive factorization of one middle-level diagonal block (Sec. 3.2.1).

    W: [nb][rows][r] -- the column blocks W_{0..nb-1} of U^h_i (or V^h_j) for
    one tree node at the middle level, nb = R^levels.  Returns (G_list, leaves):
    G_list[t] has shape [R^(t+1)][nb/R^(t+1)][r][R r] indexed by the local
    descendant at depth t+1 and the merged column index j'; leaves has shape
    [R^levels][rows/R^levels][r].
    """
    cur = np.asarray(W)[None]                      # [nodes][nb][rows][r]
    G_list = []
    for _ in range(levels):
        nodes, nb, rows, _ = cur.shape
        crow = rows // R
        nxt = np.zeros((nodes * R, nb // R, crow, r), dtype=np.complex128)
        Gt = np.zeros((nodes * R, nb // R, r, R * r), dtype=np.complex128)
        for a in range(nodes):
            for c in range(R):                     # child c: its rows of every block
                for jp in range(nb // R):          # R consecutive column blocks
                    Z = np.concatenate(
                        [cur[a, R * jp + cc, c * crow:(c + 1) * crow, :] for cc in range(R)],
                        axis=1)
                    U0, s, V0h = truncated_svd(Z, r)
                    nxt[R * a + c, jp] = U0 * s[None, :]     # third form: U0 S0
                    Gt[R * a + c, jp] = V0h                  #             V0^*
        G_list.append(Gt)
        cur = nxt
    return G_list, cur[:, 0]


def _empty_factors(R, leaf, L, r):
    h = L // 2
    P, m = R ** L, R ** h
    return {"radix": R, "leaf": int(leaf), "L": L, "r": int(r),
            "VL": np.zeros((P, leaf, r), dtype=np.complex128),
            "UL": np.zeros((P, leaf, r), dtype=np.complex128),
            "S": np.zeros((m, m, r)),
            "H": [np.zeros((R ** (l + 1), R ** (L - l - 1), r, R * r), dtype=np.complex128)
                  for l in range(h, L)],
            "G": [np.zeros((R ** (l + 1), R ** (L - l - 1), r, R * r), dtype=np.complex128)
                  for l in range(h, L)]}


def _assemble(f, get, b):
    """Stage 2 (Sec. 3.2) on middle-level blocks get(i, j) -> (U^h_ij, S^h_ij, V^h_ji)."""
    R, L, r = f["radix"], f["L"], f["r"]
    h = L // 2
    m = R ** h
    lv = L - h

    def place(dst_list, dst_leaf, node, G_list, leaves):
        for t, Gt in enumerate(G_list):
            span = R ** (t + 1)
            dst_list[t][node * span:(node + 1) * span] = Gt
        span = R ** lv
        dst_leaf[node * span:(node + 1) * span] = leaves

    # U side: X-node i of the middle level, its blocks U^h_{i,j} over j
    for i in range(m):
        W = np.zeros((m, b, r), dtype=np.complex128)
        for j in range(m):
            Uij, Sij, _ = get(i, j)
            W[j] = Uij
            f["S"][i, j] = Sij
        G_list, leaves = recursive_factorization(W, R, r, lv)
        place(f["G"], f["UL"], i, G_list, leaves)

    # V side: Omega-node j of the middle level, its blocks V^h_{j,i} over i
    for j in range(m):
        W = np.zeros((m, b, r), dtype=np.complex128)
        for i in range(m):
            _, _, Vji = get(i, j)
            W[i] = Vji
        H_list, leaves = recursive_factorization(W, R, r, lv)
        place(f["H"], f["VL"], j, H_list, leaves)
    return f


def construct_factors(kernel, leaf, r, method="sampling", seed=0, q=3, iters=3,
                      streamed=True):
    """Butterfly factorization K ~ U^L G^{L-1}..G^h M^h (H^h)^*..(H^{L-1})^* (V^L)^*
    from entries of K (the paper's second case)."""
    R = int(kernel.radix)
    N = int(kernel.N)
    L = tree_depth(N, leaf, R)
    b = N // R ** (L // 2)
    f = _empty_factors(R, leaf, L, r)

    def blk(i, j):
        return middle_block(kernel, i, j, b, r, method, seed, q, iters)

    stored = None
    if not streamed:
        m = R ** (L // 2)
        stored = {(i, j): blk(i, j) for i in range(m) for j in range(m)}
    return _assemble(f, lambda i, j: stored[(i, j)] if stored is not None else blk(i, j), b)


def middle_from_sketches(Y, W, C, r):
    """Rank-r SVD of one middle-level block Z from two sketches (Alg. 2.1, Sec. 2.1).

    Y = Z C and W = Z^* R for Gaussian test matrices C, R with r + p columns.
    Steps 2 and 4 as written; for step 3, M = Q_col^* Z Q_row needs Z Q_row,
    which the first case of Sec. 3.1 does not provide (only Z C and Z^* R are
    formed); since Z ~ Z Q_row Q_row^*, Y ~ (Z Q_row)(Q_row^* C), so
    M = Q_col^* Y (Q_row^* C)^+ (exact when rank Z <= r).
    """
    Q_col = pivoted_qr_q(Y)[:, :r]
    Q_row = pivoted_qr_q(W)[:, :r]
    M = Q_col.conj().T @ Y @ np.linalg.pinv(Q_row.conj().T @ C, rcond=1e-14)
    UM, sM, VMh = truncated_svd(M, r)
    return Q_col @ UM, sM, VMh @ Q_row.conj().T


def construct_factors_matvec(N, radix, leaf, r, matvec, rmatvec, seed=0, p=5):
    """Butterfly factorization from products with K and K^* only (the first case
    of Sec. 3.1).

    matvec(X) = K X and rmatvec(X) = K^* X for N x k complex arrays.  The middle
    level applies K to one block-diagonal Gaussian matrix C (blocks C_jj of size
    (N/m) x (r + p)) and K^* to another, R, so that rows i, column block j of
    K C hold K^h_{i,j} C_jj and rows j, column block i of K^* R hold
    (K^h_{i,j})^* R_ii; each block then gets its rank-r SVD from the two
    sketches (Alg. 2.1), put in the first form of Sec. 2.  Stage 2 is the same
    as for the entry-sampling route.
    """
    R = int(radix)
    L = tree_depth(N, leaf, R)
    m = R ** (L // 2)
    b = N // m
    k = r + p
    rng = np.random.default_rng(np.random.SeedSequence(seed, spawn_key=(7,)))

    def gauss(shape):
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * np.sqrt(0.5)

    Cb = gauss((m, b, k))
    Rb = gauss((m, b, k))
    C = np.zeros((N, m * k), dtype=np.complex128)
    Rm = np.zeros((N, m * k), dtype=np.complex128)
    for j in range(m):
        C[j * b:(j + 1) * b, j * k:(j + 1) * k] = Cb[j]
        Rm[j * b:(j + 1) * b, j * k:(j + 1) * k] = Rb[j]
    KC = np.asarray(matvec(C), dtype=np.complex128)
    KsR = np.asarray(rmatvec(Rm), dtype=np.complex128)
    blocks = {}
    for i in range(m):
        for j in range(m):
            Y = KC[i * b:(i + 1) * b, j * k:(j + 1) * k]          # K^h_ij C_jj
            W = KsR[j * b:(j + 1) * b, i * k:(i + 1) * k]         # (K^h_ij)^* R_ii
            U0, s, V0h = middle_from_sketches(Y, W, Cb[j], r)
            blocks[(i, j)] = form_usv(U0, s, V0h)
    f = _empty_factors(R, leaf, L, r)
    return _assemble(f, lambda i, j: blocks[(i, j)], b)
