"""Touching periodic unit cells: PBC pairs, LCA merge, unknown numbering.

Paper Sec. 2.2 (after Eq. pm): a node j that is a periodic image of node i
(r_j = r_i + a lattice vector along periodic axes) carries no unknown of its
own. Pairs are merged by union-find into their lowest common ancestor (LCA),
so a corner of a 3D-periodic cube ends up with up to 7 children, and the
problem size drops to N' = N - N_PBC.

Reading: the LCA representative of a class is its smallest original node
index; unknowns are numbered by increasing representative index (the paper's
"first N' points"). Two nodes pair when they coincide modulo the lattice
(any combination of periods, which covers the paper's combined shifts and
the images of a protruding cell).

``remap`` is Eq. shift_hms (Sec. 3.2.2, protruding cells): shift every
unknown by whole periods along each periodic axis so that it lies within half
a period of the centre r0 (mean of the unknown positions); per-axis, ties to
the lower image.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def pbc_pairs(xyz, mask, L, tol_rel=1e-9):
    """All index pairs (i, j), i < j, whose positions differ by a lattice vector.

    Sec. 2.1 defines T-PBC pairs through shifts gamma L_x + zeta L_y + xi L_z
    with gamma + zeta + xi > 0, i.e. along single axes and their
    combinations; a protruding cell can hold images at any lattice offset.
    Reading: i and j pair when they coincide modulo the lattice, which is
    found with a periodic KD-tree on the positions wrapped into the cell.
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    per = [a for a in range(3) if (mask >> a) & 1]
    if not per:
        return np.zeros((0, 2), dtype=np.int64)
    tol = tol_rel * max(float(np.max(np.abs(L))), float(np.ptp(xyz)))
    w = xyz.copy()
    box = np.empty(3)
    for a in range(3):
        if a in per:
            w[:, a] = np.mod(w[:, a], L[a])
            w[w[:, a] >= L[a], a] -= L[a]
            box[a] = L[a]
        else:
            w[:, a] -= w[:, a].min()
            box[a] = 2.0 * np.ptp(xyz[:, a]) + 1.0
    tree = cKDTree(w, boxsize=box)
    return tree.query_pairs(tol, output_type="ndarray").astype(np.int64)


def lca(n_nodes, pairs):
    """Union-find over PBC pairs; returns root[N] (smallest index of each class)."""
    parent = np.arange(n_nodes, dtype=np.int64)

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    for i, j in pairs:
        ri, rj = find(int(i)), find(int(j))
        if ri != rj:
            lo, hi = (ri, rj) if ri < rj else (rj, ri)
            parent[hi] = lo
    return np.array([find(i) for i in range(n_nodes)], dtype=np.int64)


def unknowns(xyz, mask, L, tol_rel=1e-9):
    """Returns (unknown_of_node[N], rep_node_of_unknown[N'], n_pbc_pairs)."""
    pairs = pbc_pairs(xyz, mask, L, tol_rel)
    root = lca(xyz.shape[0], pairs)
    reps = np.unique(root)
    uk = np.searchsorted(reps, root)
    return uk, reps, pairs.shape[0]


def remap(pos, mask, L):
    """Eq. shift_hms: per periodic axis, wrap into [r0 - L/2, r0 + L/2).

    The shifted coordinate is formed as x - k L (k integer), so unshifted
    points keep their coordinates bit for bit."""
    pos = np.array(pos, dtype=np.float64, copy=True)
    r0 = pos.mean(axis=0)
    for a in range(3):
        if (mask >> a) & 1:
            d = pos[:, a] - r0[a]
            pos[:, a] = pos[:, a] - L[a] * np.floor(d / L[a] + 0.5)
    return pos
