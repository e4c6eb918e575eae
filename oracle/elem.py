"""Element-exact near-field integrals by quadrature (paper Eq. hms_d2b, Sec. 3.2.1).

Close to a charge the point-charge superposition of Eq. hms_d2 is
inaccurate; the paper replaces it, for elements near each observer, by
exact integrals over those elements. The charges of a tetrahedron are its
constant volume density and, on its faces that lie on a surface of the
magnetic body, its linear surface density (Eq. hms1), so two integrals are
needed, evaluated here purely by quadrature (no closed forms):

    I_V(r)    = int_e dV' / |r - r'|                 (tetrahedron)
    I_f,l(r)  = int_f lambda_l(r') dS' / |r - r'|    (triangle, linear weight)

* observer at a vertex: Duffy collapse towards that vertex; the 1/R
  singularity cancels against the Jacobian, the radial integral of the
  (linear) weight is done exactly and the rest by Gauss-Legendre;
* otherwise: adaptive subdivision (tetrahedra into 8, triangles into 4)
  until every piece is well separated from r, then collapsed Gauss-Legendre.

A third, independent integral -- the dipole form
    C_j(r) = int_e lambda_j(r') (r - r') / |r - r'|^3 dV'
of the potential of a linearly magnetised tetrahedron -- is kept as a
cross-check: summed over a closed body it must agree with volume plus
surface charges (divergence theorem).
"""
from __future__ import annotations

import numpy as np

_ORDER_VERTEX = 20
_ORDER_PIECE = 8
_SEPARATION = 1.0       # refine while dist(r, piece centroid) < SEP * diameter
_MAX_DEPTH = 9

# children of a tetrahedron (0,1,2,3) in terms of corners + edge midpoints
_MID = {(0, 1): 4, (0, 2): 5, (0, 3): 6, (1, 2): 7, (1, 3): 8, (2, 3): 9}
_CHILDREN = np.array([[0, 4, 5, 6], [4, 1, 7, 8], [5, 7, 2, 9], [6, 8, 9, 3],
                      [4, 5, 6, 8], [4, 5, 7, 8], [5, 6, 8, 9], [5, 7, 8, 9]])


def _gl01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def coeffs_at_vertex(X, a):
    """C[P,4,3] for observers at vertex a[P] of tetrahedra X[P,4,3]."""
    P = X.shape[0]
    perm = np.stack([a, (a + 1) % 4, (a + 2) % 4, (a + 3) % 4], axis=1)
    Y = np.take_along_axis(X, perm[:, :, None], axis=1)          # Y0 = observer
    e1, e2, e3 = (Y[:, k] - Y[:, 0] for k in (1, 2, 3))
    V6 = np.abs(np.einsum("pi,pi->p", e1, np.cross(e2, e3)))       # 6 V
    v, wv = _gl01(_ORDER_VERTEX)
    w, ww = _gl01(_ORDER_VERTEX)
    V_, W_ = np.meshgrid(v, w, indexing="ij")
    WT = np.outer(wv, ww).ravel()
    V_, W_ = V_.ravel(), W_.ravel()
    # d(v,w) = (1-v) e1 + v(1-w) e2 + v w e3  (points of the opposite face - Y0)
    d = ((1 - V_)[None, :, None] * e1[:, None, :] + (V_ * (1 - W_))[None, :, None] * e2[:, None, :]
         + (V_ * W_)[None, :, None] * e3[:, None, :])             # [P,Q,3]
    kern = d / np.linalg.norm(d, axis=2, keepdims=True) ** 3      # d/|d|^3
    # exact u-integrals of lambda_k along the ray: 1/2 * (1, 1-v, v(1-w), v w)
    lam_u = 0.5 * np.stack([np.ones_like(V_), 1 - V_, V_ * (1 - W_), V_ * W_], axis=0)  # [4,Q]
    base = -(V6[:, None] * (V_ * WT)[None, :])                    # [P,Q]
    Cp = np.einsum("pq,kq,pqi->pki", base, lam_u, kern)           # permuted order
    C = np.empty_like(Cp)
    np.put_along_axis(C, perm[:, :, None], Cp, axis=1)
    return C


def _collapsed_rule(n):
    u, wu = _gl01(n)
    U, V, W = np.meshgrid(u, u, u, indexing="ij")
    wt = (wu[:, None, None] * wu[None, :, None] * wu[None, None, :])
    U, V, W, wt = U.ravel(), V.ravel(), W.ravel(), wt.ravel()
    # point = Q0 + U[(1-V) e1 + V(1-W) e2 + V W e3], Jacobian = 6 Vq U^2 V
    return U, V, W, wt * U * U * V


_RULE = _collapsed_rule(_ORDER_PIECE)


def coeffs_regular(r, X, grad):
    """C[P,4,3] for observers r[P,3] that are not vertices of X[P,4,3].

    grad[P,4,3] are the barycentric gradients of the parent tetrahedra.
    """
    P = r.shape[0]
    out = np.zeros((P, 4, 3))
    owner = np.arange(P)
    pieces = X.copy()
    U, V, W, WT = _RULE
    for depth in range(_MAX_DEPTH + 1):
        if pieces.shape[0] == 0:
            break
        cen = pieces.mean(axis=1)
        diam = np.max(np.linalg.norm(pieces[:, :, None, :] - pieces[:, None, :, :], axis=3),
                      axis=(1, 2))
        dist = np.linalg.norm(cen - r[owner], axis=1)
        leaf = (dist >= _SEPARATION * diam) | (depth == _MAX_DEPTH)
        if np.any(leaf):
            Q = pieces[leaf]
            o = owner[leaf]
            e1, e2, e3 = (Q[:, k] - Q[:, 0] for k in (1, 2, 3))
            V6 = np.abs(np.einsum("pi,pi->p", e1, np.cross(e2, e3)))
            pts = (Q[:, None, 0, :] + U[None, :, None] * (
                (1 - V)[None, :, None] * e1[:, None, :]
                + (V * (1 - W))[None, :, None] * e2[:, None, :]
                + (V * W)[None, :, None] * e3[:, None, :]))          # [p,Q,3]
            rr = r[o][:, None, :] - pts
            kern = rr / np.linalg.norm(rr, axis=2, keepdims=True) ** 3
            x0 = X[o][:, 0, :]
            lam = np.einsum("pki,pqi->pkq", grad[o], pts - x0[:, None, :])
            lam[:, 0, :] += 1.0
            c = np.einsum("p,q,pkq,pqi->pki", V6, WT, lam, kern)
            np.add.at(out, o, c)
        keep = ~leaf
        if not np.any(keep):
            break
        Q = pieces[keep]
        o = owner[keep]
        mids = np.stack([0.5 * (Q[:, i] + Q[:, j]) for (i, j) in _MID], axis=1)
        allp = np.concatenate([Q, mids], axis=1)                     # [p,10,3]
        pieces = allp[:, _CHILDREN, :].reshape(-1, 4, 3)
        owner = np.repeat(o, 8)
    return out


def _subdivide_tets(Q):
    mids = np.stack([0.5 * (Q[:, i] + Q[:, j]) for (i, j) in _MID], axis=1)
    allp = np.concatenate([Q, mids], axis=1)
    return allp[:, _CHILDREN, :].reshape(-1, 4, 3)


def tet_inv_r(r, X, vertex):
    """I_V[P] = int over tetrahedron X[P,4,3] of 1/|r - r'|; vertex[P] = local
    index of r in X or -1."""
    P = r.shape[0]
    out = np.zeros(P)
    at = vertex >= 0
    if np.any(at):
        Xa, a = X[at], vertex[at]
        perm = np.stack([a, (a + 1) % 4, (a + 2) % 4, (a + 3) % 4], axis=1)
        Y = np.take_along_axis(Xa, perm[:, :, None], axis=1)
        e1, e2, e3 = (Y[:, k] - Y[:, 0] for k in (1, 2, 3))
        V6 = np.abs(np.einsum("pi,pi->p", e1, np.cross(e2, e3)))
        v, wv = _gl01(_ORDER_VERTEX)
        V_, W_ = np.meshgrid(v, v, indexing="ij")
        WT = np.outer(wv, wv).ravel()
        V_, W_ = V_.ravel(), W_.ravel()
        d = ((1 - V_)[None, :, None] * e1[:, None, :] + (V_ * (1 - W_))[None, :, None] * e2[:, None, :]
             + (V_ * W_)[None, :, None] * e3[:, None, :])
        # r' = Y0 + u d, Jacobian 6V u^2 v, 1/R = 1/(u |d|); int_0^1 u du = 1/2
        out[at] = 0.5 * V6 * np.sum((V_ * WT)[None, :] / np.linalg.norm(d, axis=2), axis=1)
    if np.any(~at):
        rr = r[~at]
        owner = np.arange(rr.shape[0])
        pieces = X[~at].copy()
        acc = np.zeros(rr.shape[0])
        U, V, W, WT = _RULE
        for depth in range(_MAX_DEPTH + 1):
            cen = pieces.mean(axis=1)
            diam = np.max(np.linalg.norm(pieces[:, :, None, :] - pieces[:, None, :, :], axis=3),
                          axis=(1, 2))
            dist = np.linalg.norm(cen - rr[owner], axis=1)
            leaf = (dist >= _SEPARATION * diam) | (depth == _MAX_DEPTH)
            if np.any(leaf):
                Q, o = pieces[leaf], owner[leaf]
                e1, e2, e3 = (Q[:, k] - Q[:, 0] for k in (1, 2, 3))
                V6 = np.abs(np.einsum("pi,pi->p", e1, np.cross(e2, e3)))
                pts = (Q[:, None, 0, :] + U[None, :, None] * (
                    (1 - V)[None, :, None] * e1[:, None, :]
                    + (V * (1 - W))[None, :, None] * e2[:, None, :]
                    + (V * W)[None, :, None] * e3[:, None, :]))
                inv = 1.0 / np.linalg.norm(rr[o][:, None, :] - pts, axis=2)
                np.add.at(acc, o, V6 * (inv @ WT))
            if np.all(leaf):
                break
            pieces = _subdivide_tets(pieces[~leaf])
            owner = np.repeat(owner[~leaf], 8)
        out[~at] = acc
    return out


def _tri_rule(n):
    u, wu = _gl01(n)
    U, V = np.meshgrid(u, u, indexing="ij")
    wt = np.outer(wu, wu).ravel()
    U, V = U.ravel(), V.ravel()
    # point = Q0 + U[(1-V) e1 + V e2], Jacobian = 2 A U
    return U, V, wt * U


_TRI_RULE = _tri_rule(_ORDER_PIECE + 2)


def tri_lambda_inv_r(r, T, vertex):
    """I[P,3] = int over triangle T[P,3,3] of lambda_l(r') / |r - r'|, l = 0..2;
    vertex[P] = local index of r in T or -1."""
    P = r.shape[0]
    out = np.zeros((P, 3))
    at = vertex >= 0
    if np.any(at):
        Ta, a = T[at], vertex[at]
        perm = np.stack([a, (a + 1) % 3, (a + 2) % 3], axis=1)
        Y = np.take_along_axis(Ta, perm[:, :, None], axis=1)
        e1, e2 = Y[:, 1] - Y[:, 0], Y[:, 2] - Y[:, 0]
        A2 = np.linalg.norm(np.cross(e1, e2), axis=1)          # 2 A
        v, wv = _gl01(_ORDER_VERTEX)
        d = (1 - v)[None, :, None] * e1[:, None, :] + v[None, :, None] * e2[:, None, :]
        inv = 1.0 / np.linalg.norm(d, axis=2)                    # [P,Q]
        # r' = Y0 + u d(v), Jacobian 2A u, 1/R = 1/(u|d|); weights along u:
        # lambda_0 = 1-u, lambda_1 = u(1-v), lambda_2 = u v -> int du = 1/2, (1-v)/2, v/2
        lam = 0.5 * np.stack([np.ones_like(v), 1 - v, v], axis=0)   # [3,Q]
        Ip = A2[:, None] * np.einsum("pq,kq,q->pk", inv, lam, wv)
        res = np.empty_like(Ip)
        np.put_along_axis(res, perm, Ip, axis=1)
        out[at] = res
    if np.any(~at):
        rr = r[~at]
        T0 = T[~at]
        owner = np.arange(rr.shape[0])
        pieces = T0.copy()
        # barycentric coordinates of piece corners w.r.t. the parent triangle
        bary = np.broadcast_to(np.eye(3), (rr.shape[0], 3, 3)).copy()
        acc = np.zeros((rr.shape[0], 3))
        U, V, WT = _TRI_RULE
        for depth in range(_MAX_DEPTH + 1):
            cen = pieces.mean(axis=1)
            diam = np.max(np.linalg.norm(pieces[:, :, None, :] - pieces[:, None, :, :], axis=3),
                          axis=(1, 2))
            dist = np.linalg.norm(cen - rr[owner], axis=1)
            leaf = (dist >= _SEPARATION * diam) | (depth == _MAX_DEPTH)
            if np.any(leaf):
                Q, o, B = pieces[leaf], owner[leaf], bary[leaf]
                e1, e2 = Q[:, 1] - Q[:, 0], Q[:, 2] - Q[:, 0]
                A2 = np.linalg.norm(np.cross(e1, e2), axis=1)
                lam_loc = np.stack([1 - U, U * (1 - V), U * V], axis=0)       # [3,Q]
                pts = np.einsum("kq,pki->pqi", lam_loc, Q)
                lam_par = np.einsum("kq,pkl->plq", lam_loc, B)              # [p,3,Q]
                inv = 1.0 / np.linalg.norm(rr[o][:, None, :] - pts, axis=2)
                np.add.at(acc, o, A2[:, None] * np.einsum("plq,pq,q->pl", lam_par, inv, WT))
            if np.all(leaf):
                break
            Q, B = pieces[~leaf], bary[~leaf]
            owner = np.repeat(owner[~leaf], 4)
            mQ = [0.5 * (Q[:, 0] + Q[:, 1]), 0.5 * (Q[:, 1] + Q[:, 2]), 0.5 * (Q[:, 2] + Q[:, 0])]
            mB = [0.5 * (B[:, 0] + B[:, 1]), 0.5 * (B[:, 1] + B[:, 2]), 0.5 * (B[:, 2] + B[:, 0])]
            pieces = np.stack([np.stack([Q[:, 0], mQ[0], mQ[2]], 1), np.stack([mQ[0], Q[:, 1], mQ[1]], 1),
                               np.stack([mQ[2], mQ[1], Q[:, 2]], 1), np.stack([mQ[0], mQ[1], mQ[2]], 1)],
                              axis=1).reshape(-1, 3, 3)
            bary = np.stack([np.stack([B[:, 0], mB[0], mB[2]], 1), np.stack([mB[0], B[:, 1], mB[1]], 1),
                             np.stack([mB[2], mB[1], B[:, 2]], 1), np.stack([mB[0], mB[1], mB[2]], 1)],
                            axis=1).reshape(-1, 3, 3)
        out[~at] = acc
    return out


def element_coeffs(r, X, grad, vertex):
    """C[P,4,3]; vertex[P] is the local index of r in X or -1."""
    out = np.empty((r.shape[0], 4, 3))
    at = vertex >= 0
    if np.any(at):
        out[at] = coeffs_at_vertex(X[at], vertex[at])
    if np.any(~at):
        out[~at] = coeffs_regular(r[~at], X[~at], grad[~at])
    return out
