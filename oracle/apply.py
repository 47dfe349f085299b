"""Applying the butterfly factorization, its adjoint and the loss gradient (FP64).

u = U^L G^{L-1} ... G^h M^h (H^h)^* ... (H^{L-1})^* (V^L)^* g   (Sec. 1.2 and
the closing equation of Sec. 3.2), evaluated right to left as O(log N)
sparse products.  The sparse factors are never formed here; each product is
written from the block relations that define the factor:

  leaves, Omega side   y^L_j = (V^L_j)^* g_{B^L_j}
  H side, l = L-1..h   y^l_{j,R i+c} = sum_c' (H^l_{Rj+c',i}[:, c r:(c+1) r])^* y^{l+1}_{Rj+c',i}
                       (Sec. 3.2.2: V^l restricted to Omega-child Rj+c' and
                       X-child Ri+c equals V^{l+1}_{Rj+c',i} H^l_{Rj+c',i}[:, c-block])
  middle               z^h_{i,j} = S^h_{i,j} y^h_{j,i}
                       (Sec. 3.1: block (i,j) of M^h is zero except its (j,i)
                       r x r block, which is diag S^h_{i,j})
  G side, l = h..L-1   z^{l+1}_{Ri+c,j} = G^l_{Ri+c,j} [z^l_{i,Rj}; ...; z^l_{i,Rj+R-1}]
                       (Sec. 3.2.1, the splits of U^l into children)
  leaves, X side       u_{A^L_i} = U^L_i z^L_{i,0}

Vectors are complex[N][nrhs] in tree order.  Activations at a level are
arrays [nodes of the tree being split][nodes of the tree being merged][r][nrhs].
"""
from __future__ import annotations

import numpy as np


def _dims(f):
    R, n0, L, r = f["radix"], f["leaf"], f["L"], f["r"]
    return R, n0, L, r, L // 2, R ** L


def _h_forward(Hl, y, R):
    """y^{l+1} [R^{l+1}][R^{L-l-1}][r][n] -> y^l [R^l][R^{L-l}][r][n]."""
    A, B, r, _ = Hl.shape
    n = y.shape[-1]
    H6 = Hl.reshape(A // R, R, B, r, R, r)           # [j][c'][i][b][c][a]
    y5 = y.reshape(A // R, R, B, r, n)               # [j][c'][i][b][n]
    out = np.einsum("jxibca,jxibn->jican", H6.conj(), y5)
    return out.reshape(A // R, B * R, r, n)


def _h_adjoint(Hl, y, R):
    """Adjoint of _h_forward: y^l [R^l][R^{L-l}] -> y^{l+1} [R^{l+1}][R^{L-l-1}]."""
    A, B, r, _ = Hl.shape
    n = y.shape[-1]
    H6 = Hl.reshape(A // R, R, B, r, R, r)           # [j][c'][i][b][c][a]
    y5 = y.reshape(A // R, B, R, r, n)               # [j][i][c][a][n]
    out = np.einsum("jxibca,jican->jxibn", H6, y5)
    return out.reshape(A, B, r, n)


def _g_forward(Gl, z, R):
    """z^l [R^l][R^{L-l}][r][n] -> z^{l+1} [R^{l+1}][R^{L-l-1}][r][n]."""
    A, B, r, _ = Gl.shape
    n = z.shape[-1]
    G6 = Gl.reshape(A // R, R, B, r, R, r)           # [i][c][j][a][c'][b]
    z5 = z.reshape(A // R, B, R, r, n)               # [i][j][c'][b][n]
    out = np.einsum("icjaxb,ijxbn->icjan", G6, z5)
    return out.reshape(A, B, r, n)


def _g_adjoint(Gl, z, R):
    """Adjoint of _g_forward: z^{l+1} [R^{l+1}][R^{L-l-1}] -> z^l [R^l][R^{L-l}]."""
    A, B, r, _ = Gl.shape
    n = z.shape[-1]
    G6 = Gl.reshape(A // R, R, B, r, R, r)           # [i][c][j][a][c'][b]
    z5 = z.reshape(A // R, R, B, r, n)               # [i][c][j][a][n]
    out = np.einsum("icjaxb,icjan->ijxbn", G6.conj(), z5)
    return out.reshape(A // R, B * R, r, n)


def forward_levels(f, g):
    """All activations of u = K_BF g.

    Returns (ys, zs, u): ys[l] for l = L..h (Omega side, ys[L] the leaf
    projections), zs[l] for l = h..L (X side), and u.
    """
    R, n0, L, r, h, P = _dims(f)
    g = np.asarray(g, dtype=np.complex128)
    squeeze = g.ndim == 1
    if squeeze:
        g = g[:, None]
    n = g.shape[1]
    ys = {}
    ys[L] = np.einsum("jpr,jpn->jrn", f["VL"].conj(), g.reshape(P, n0, n))[:, None]
    for l in range(L - 1, h - 1, -1):
        ys[l] = _h_forward(f["H"][l - h], ys[l + 1], R)
    zs = {h: f["S"][..., None] * ys[h].transpose(1, 0, 2, 3)}
    for l in range(h, L):
        zs[l + 1] = _g_forward(f["G"][l - h], zs[l], R)
    u = np.einsum("ipr,irn->ipn", f["UL"], zs[L][:, 0]).reshape(P * n0, n)
    return ys, zs, (u[:, 0] if squeeze else u)


def bf_apply(f, g):
    """u = K_BF g for g of shape [N] or [N][nrhs]."""
    return forward_levels(f, g)[2]


def adjoint_levels(f, w):
    """All activations of v = K_BF^* w (the factors in reverse order, each adjointed).

    Returns (zs, ys, v): zs[l] for l = L..h (X side, adjoint), ys[l] for
    l = h..L (Omega side), and v.
    """
    R, n0, L, r, h, P = _dims(f)
    w = np.asarray(w, dtype=np.complex128)
    squeeze = w.ndim == 1
    if squeeze:
        w = w[:, None]
    n = w.shape[1]
    zs = {L: np.einsum("ipr,ipn->irn", f["UL"].conj(), w.reshape(P, n0, n))[:, None]}
    for l in range(L - 1, h - 1, -1):
        zs[l] = _g_adjoint(f["G"][l - h], zs[l + 1], R)
    ys = {h: (f["S"][..., None] * zs[h]).transpose(1, 0, 2, 3)}
    for l in range(h, L):
        ys[l + 1] = _h_adjoint(f["H"][l - h], ys[l], R)
    v = np.einsum("jpr,jrn->jpn", f["VL"], ys[L][:, 0]).reshape(P * n0, n)
    return zs, ys, (v[:, 0] if squeeze else v)


def bf_apply_adjoint(f, w):
    """v = K_BF^* w."""
    return adjoint_levels(f, w)[2]


def bf_grad(f, g, grad_u):
    """Gradients of a real loss through u = K_BF g.

    `grad_u` = dL/dRe(u) + i dL/dIm(u) (the convention under which the
    gradient of a complex linear map y = A x is grad_A = grad_y x^*, grad_x =
    A^* grad_y).  Returns a dict with grad_g and gradients for every factor in
    the canonical layout (S real).
    """
    R, n0, L, r, h, P = _dims(f)
    g = np.asarray(g, dtype=np.complex128)
    gu = np.asarray(grad_u, dtype=np.complex128)
    if g.ndim == 1:
        g, gu = g[:, None], gu[:, None]
    n = g.shape[1]
    ys, zs, _ = forward_levels(f, g)
    out = {"H": [None] * (L - h), "G": [None] * (L - h)}

    # X-side leaves: u_i = U^L_i z^L_i
    gub = gu.reshape(P, n0, n)
    out["UL"] = np.einsum("ipn,irn->ipr", gub, zs[L][:, 0].conj())
    dz = np.einsum("ipr,ipn->irn", f["UL"].conj(), gub)[:, None]
    # G side, top down: z^{l+1} = G^l [z^l children]
    for l in range(L - 1, h - 1, -1):
        Gl = f["G"][l - h]
        A, B = Gl.shape[:2]
        zin = zs[l].reshape(A // R, B, R * r, n)                 # [i][j][(c' b)][n]
        dout = dz.reshape(A // R, R, B, r, n)                     # [i][c][j][a][n]
        gG = np.einsum("icjan,ijkn->icjak", dout, zin.conj())     # grad = d_out z_in^*
        out["G"][l - h] = gG.reshape(A, B, r, R * r)
        dz = _g_adjoint(Gl, dz, R)
    # middle: z^h_{i,j} = S_{i,j} y^h_{j,i}, S real
    yT = ys[h].transpose(1, 0, 2, 3)
    out["S"] = np.einsum("ijkn,ijkn->ijk", dz, yT.conj()).real
    dy = (f["S"][..., None] * dz).transpose(1, 0, 2, 3)
    # H side, bottom up: y^l = (H^l)^* y^{l+1}; for out = W^* x, grad_W = x d_out^*
    for l in range(h, L):
        Hl = f["H"][l - h]
        A, B = Hl.shape[:2]
        xin = ys[l + 1]                                           # [R^{l+1}][B][r][n]
        dout = dy.reshape(A // R, B, R * r, n)                    # [j][i][(c a)][n]
        dout = np.repeat(dout, R, axis=0)                         # each child p = R j + c'
        out["H"][l - h] = np.einsum("pibn,pikn->pibk", xin, dout.conj())
        dy = _h_adjoint(Hl, dy, R)
    # Omega-side leaves: y^L_j = (V^L_j)^* g_j
    gb = g.reshape(P, n0, n)
    out["VL"] = np.einsum("jpn,jrn->jpr", gb, dy[:, 0].conj())
    out["g"] = np.einsum("jpr,jrn->jpn", f["VL"], dy[:, 0]).reshape(P * n0, n)
    return out
