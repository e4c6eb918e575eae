"""P1 tetrahedral operators on a touching periodic mesh (paper Secs. 2.2, 3.1, 3.2.1).

Magnetisation M = Ms * sum_n m_n phi_n (Eq. M_phi) with linear basis
functions phi = barycentric coordinates lambda. SI units (the paper is in
CGS): M in A/m, A in J/m, mu0 = 4 pi 1e-7.

* Exchange (Eq. hex, Eq. lapl): energy E_ex = sum_t A_t int |grad m|^2 gives
  H_ex,n = -(2 / (mu0 mu_n)) sum_m K_nm m_m with K_nm = sum_t A_t V_t
  grad(lambda_n).grad(lambda_m) and the lumped Ms-volume mu_n = sum_t Ms_t V_t / 4.
* Charges (Eq. hms1, hms_d1): reading of the garbled signs -- volume density
  rho = -div M and surface density sigma = +M.n (outward), so that
  u = (1/4 pi) int G rho + (1/4 pi) oint G sigma and H = -grad u is the
  physical field. The nodal charge is the weak form q_n = int rho lambda_n +
  oint sigma lambda_n, which by the divergence theorem on each tetrahedron is
  q_n = sum_t int_t M . grad(lambda_n) = sum_t Ms_t V_t/4 grad(lambda_n) . sum_j m_j.
  Faces shared by two tetrahedra of equal Ms cancel, so only boundary and
  material-interface faces carry surface charge, as the paper describes.
* Gradient (Eq. hms_d3): H_ms,n = -(1/mu_n) sum_k D_kn u_k, i.e. the
  Ms-volume weighted average of the per-tetrahedron gradient of u; it is the
  transpose of the charge operator, so the pair is energy consistent.

Periodicity (Sec. 3.1, Cases 1-3): every tetrahedron keeps its own (unmapped)
geometry and its vertex indices are replaced by their LCA unknowns before
assembly; summing all tetrahedra around an LCA then forms the union of the
children's neighbourhoods without duplicated edges (Eqs. shift, dedup, lapl_2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

MU0 = 4e-7 * np.pi


def tet_geometry(xyz, tets):
    """Volumes V[T] and barycentric gradients G[T,4,3] of each tetrahedron."""
    X = xyz[tets]                                   # [T,4,3]
    J = X[:, 1:, :] - X[:, :1, :]                   # rows: edge vectors
    V = np.linalg.det(J) / 6.0
    Jinv = np.linalg.inv(J)                          # columns: grad lambda_1..3
    g = np.empty((tets.shape[0], 4, 3))
    g[:, 1:, :] = np.transpose(Jinv, (0, 2, 1))
    g[:, 0, :] = -g[:, 1:, :].sum(axis=1)
    return V, g


class LocalOperators:
    """Assembled FP64 sparse operators on the N' unknowns."""

    def __init__(self, xyz, tets, region, Ms, Aex, uk, n_unknowns):
        self.n = n_unknowns
        V, g = tet_geometry(xyz, tets)
        if np.any(V <= 0):
            raise ValueError("non-positive tetrahedron volume")
        self.V, self.grad = V, g
        ms_t = np.asarray(Ms, dtype=np.float64)[region]
        a_t = np.asarray(Aex, dtype=np.float64)[region]
        U = uk[tets]                                   # [T,4] LCA unknowns
        self.mu = np.bincount(U.ravel(), weights=np.repeat(ms_t * V / 4.0, 4),
                              minlength=n_unknowns)
        rows = np.repeat(U, 4, axis=1).ravel()         # (a,b) -> row U[a]
        cols = np.tile(U, (1, 4)).ravel()              # col U[b]
        kab = np.einsum("tai,tbi->tab", g, g) * (a_t * V)[:, None, None]
        self.K = sp.csr_matrix((kab.ravel(), (rows, cols)), shape=(self.n, self.n))
        dcoef = (ms_t * V / 4.0)[:, None, None] * g      # [T,4,3] for row a
        self.D = [sp.csr_matrix((np.repeat(dcoef[:, :, c], 4, axis=1).ravel(), (rows, cols)),
                                shape=(self.n, self.n)) for c in range(3)]
        self.DT = [d.T.tocsr() for d in self.D]

    def exchange(self, m):
        """H_ex [N',3] in A/m for unit vectors m [N',3]."""
        return -(2.0 / MU0) * (self.K @ m) / self.mu[:, None]

    def charges(self, m):
        """Nodal magnetic charges q [N'] in A m."""
        return sum(self.D[c] @ m[:, c] for c in range(3))

    def gradient_field(self, u, rows=None):
        """H_ms = -(1/mu) D^T u at all unknowns or the given rows.

        With rows given, u only needs to be correct on the neighbours of rows."""
        if rows is None:
            return -np.stack([self.DT[c] @ u for c in range(3)], axis=1) / self.mu[:, None]
        rows = np.asarray(rows)
        return -np.stack([self.DT[c][rows] @ u for c in range(3)], axis=1) / self.mu[rows, None]

    def neighbours(self, rows):
        """Unknowns whose potential enters H_ms at the given rows."""
        sub = abs(self.DT[0][np.asarray(rows)]) + abs(self.DT[1][np.asarray(rows)]) \
            + abs(self.DT[2][np.asarray(rows)])
        return np.union1d(np.unique(sub.indices), np.asarray(rows))

    def exchange_energy(self, m):
        return float(np.sum(m * (self.K @ m)))
