"""Construction of the butterfly factorization (Sec. 3), FP64.

Stage 1, the middle-level factorization (Sec. 3.1): every block
K^h_{i,j} = K(A^h_i, B^h_j), i, j < m = R^h, gets a rank-r approximation
U^h_{i,j} S^h_{i,j} (V^h_{j,i})^* in the first equivalent form of Sec. 2
(U = U0 S0, S = S0^{-1}, V^* = S0 V0^*), either by randomized sampling of
its entries (Algorithm 2.2, the paper's "second case") or, as a
deterministic reference, by a truncated SVD of the whole block.

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

from .lowrank import truncated_svd, randomized_sampling, form_usv


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


def construct_factors(kernel, leaf, r, method="sampling", seed=0, q=3, iters=3,
                      streamed=True):
    """Butterfly factorization K ~ U^L G^{L-1}..G^h M^h (H^h)^*..(H^{L-1})^* (V^L)^*."""
    R = int(kernel.radix)
    N = int(kernel.N)
    L = tree_depth(N, leaf, R)
    h = L // 2
    m = R ** h
    b = N // m
    P = R ** L
    lv = L - h

    f = {"radix": R, "leaf": int(leaf), "L": L, "r": int(r),
         "VL": np.zeros((P, leaf, r), dtype=np.complex128),
         "UL": np.zeros((P, leaf, r), dtype=np.complex128),
         "S": np.zeros((m, m, r)),
         "H": [np.zeros((R ** (l + 1), R ** (L - l - 1), r, R * r), dtype=np.complex128)
               for l in range(h, L)],
         "G": [np.zeros((R ** (l + 1), R ** (L - l - 1), r, R * r), dtype=np.complex128)
               for l in range(h, L)]}

    def blk(i, j):
        return middle_block(kernel, i, j, b, r, method, seed, q, iters)

    stored = None
    if not streamed:
        stored = {(i, j): blk(i, j) for i in range(m) for j in range(m)}

    def get(i, j):
        return stored[(i, j)] if stored is not None else blk(i, j)

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
