"""The factors as explicit sparse matrices, assembled from the block pictures.

Each factor is built the way Sec. 3.1 and 3.2 draw it:
  * U^L = diag(U^L_0, ..., U^L_{P-1}) and (V^L)^* likewise (block diagonal);
  * G^l = diag(G^l_0, ..., G^l_{R^l - 1}) where G^l_i stacks, for each child
    c, the row of blocks diag(G^l_{Ri+c,0}, ..., G^l_{Ri+c,R^{L-l-1}-1}); block
    G^l_{Ri+c,j'} (r x Rr) sits in block-row (c, j') and spans the block
    columns R j' .. R j' + R - 1 of U^l_i;
  * H^l has the same structure with the Omega tree, and enters as (H^l)^*;
  * M^h is an m x m grid of m x m grids of r x r blocks whose block (i, j) is
    zero except for its (j, i) sub-block, which is diag S^h_{i,j}.
The columns of U^l (rows of (V^l)^*) are ordered node-major, then the
complementary node, then the rank index -- the order of eq. (9) of Sec. 3.1.

K_BF = U^L G^{L-1} ... G^h M^h (H^h)^* ... (H^{L-1})^* (V^L)^*.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _block_diag_leaves(B):
    """diag(B_0, ..., B_{P-1}) for B of shape [P][n0][r] -> (P n0) x (P r)."""
    P, n0, r = B.shape
    rows, cols, vals = [], [], []
    for i in range(P):
        rr, cc = np.meshgrid(np.arange(n0), np.arange(r), indexing="ij")
        rows.append(i * n0 + rr.ravel())
        cols.append(i * r + cc.ravel())
        vals.append(B[i].ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(P * n0, P * r))


def _butterfly_factor(Bl, R, l, L):
    """G^l (or H^l) as a (P r) x (P r) sparse matrix from blocks [R^(l+1)][R^(L-l-1)][r][R r]."""
    A, Bn, r, _ = Bl.shape
    P = R ** L
    rows, cols, vals = [], [], []
    for i in range(R ** l):                    # diagonal block G^l_i
        for c in range(R):                     # child Ri+c: a block row of G^l_i
            for jp in range(R ** (L - l - 1)):
                blk = Bl[R * i + c, jp]
                r0 = ((R * i + c) * R ** (L - l - 1) + jp) * r
                c0 = i * R ** (L - l) * r + R * jp * r
                rr, cc = np.meshgrid(np.arange(r), np.arange(R * r), indexing="ij")
                rows.append(r0 + rr.ravel())
                cols.append(c0 + cc.ravel())
                vals.append(blk.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(P * r, P * r))


def _middle(S):
    m, _, r = S.shape
    rows, cols, vals = [], [], []
    for i in range(m):
        for j in range(m):
            for k in range(r):
                rows.append((i * m + j) * r + k)     # block (i,j), its (j,i) sub-block ...
                cols.append((j * m + i) * r + k)     # ... hits the Omega-side slot (j,i)
                vals.append(S[i, j, k])
    return sp.csr_matrix((vals, (rows, cols)), shape=(m * m * r, m * m * r))


def factor_list(f):
    """[U^L, G^{L-1}, ..., G^h, M^h, (H^h)^*, ..., (H^{L-1})^*, (V^L)^*] as sparse matrices."""
    R, L = f["radix"], f["L"]
    h = L // 2
    mats = [_block_diag_leaves(f["UL"])]
    for l in range(L - 1, h - 1, -1):
        mats.append(_butterfly_factor(f["G"][l - h], R, l, L))
    mats.append(_middle(f["S"]))
    for l in range(h, L):
        mats.append(_butterfly_factor(f["H"][l - h], R, l, L).conj().T.tocsr())
    mats.append(_block_diag_leaves(f["VL"]).conj().T.tocsr())
    return mats


def assembled_apply(f, g):
    """K_BF g as the product of the explicit sparse factors, rightmost first."""
    x = np.asarray(g, dtype=np.complex128)
    for M in reversed(factor_list(f)):
        x = M @ x
    return x


def assembled_dense(f):
    """K_BF as a dense matrix (small N only)."""
    mats = factor_list(f)
    K = mats[-1].toarray()
    for M in reversed(mats[:-1]):
        K = M @ K
    return np.asarray(K)


def nnz_per_factor(f):
    return [M.nnz for M in factor_list(f)]
