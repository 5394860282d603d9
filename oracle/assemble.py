"""Assembled sparse matrices (Sec. 2.2: A_l is the restriction of the bilinear
form to V_l; P is the embedding V_{l-1} -> V_l and R its Euclidean adjoint;
Sec. 2.3: the level blocks A^S, A^{SI}, A^{IS}; Sec. 4.3: cell-wise
coefficient).

On an axis-aligned cell of side h with constant coefficient a, the Q_k
stiffness matrix is a * h^(d-2) * (reference Laplacian) and the mass matrix is
h^d * (reference mass); both are exact with k+1 Gauss points.  Coarser level
cells that are not leaves take the mean coefficient of their children.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .basis import cell_mass, cell_stiffness, embed_1d
from .dofs import FLAG_D, FLAG_I, FLAG_S
from .forest import side


def _assemble(cellmap, scales, ref, n_rows):
    nc, nl = cellmap.shape
    rows = np.repeat(cellmap, nl, axis=1).reshape(-1)
    cols = np.tile(cellmap, (1, nl)).reshape(-1)
    vals = (np.asarray(scales, dtype=np.float64)[:, None] * ref.reshape(1, -1)).reshape(-1)
    return sp.coo_matrix((vals, (rows, cols)), shape=(n_rows, n_rows)).tocsr()


def cell_h(cells, dim):
    return np.array([side(c[0]) / float(1 << 20) for c in cells])


def constraint_matrix(leaf):
    """C: (N + H) x N, identity on DoFs, constraint weights on hanging rows."""
    N, H = leaf.n_dofs, len(leaf.hkeys)
    rows = list(range(N))
    cols = list(range(N))
    vals = [1.0] * N
    for h in range(H):
        for p in range(leaf.c_offsets[h], leaf.c_offsets[h + 1]):
            rows.append(N + h)
            cols.append(int(leaf.c_masters[p]))
            vals.append(float(leaf.c_weights[p]))
    return sp.coo_matrix((vals, (rows, cols)), shape=(N + H, N)).tocsr()


def _extended(cellmap, N):
    cm = cellmap.copy()
    neg = cm < 0
    cm[neg] = N + (-cm[neg] - 1)
    return cm


def leaf_matrices(disc, coeff):
    """(A_L, M_L): constrained stiffness and mass on the leaf DoFs (Dirichlet
    rows/columns still present)."""
    leaf, dim, k = disc.leaf, disc.forest.dim, disc.k
    N, H = leaf.n_dofs, len(leaf.hkeys)
    h = cell_h(leaf.cells, dim)
    cm = _extended(leaf.cellmap, N)
    Ahat = _assemble(cm, np.asarray(coeff) * h ** (dim - 2), cell_stiffness(dim, k), N + H)
    Mhat = _assemble(cm, h ** dim, cell_mass(dim, k), N + H)
    C = constraint_matrix(leaf)
    return (C.T @ Ahat @ C).tocsr(), (C.T @ Mhat @ C).tocsr()


def level_coefficients(disc, coeff):
    """Coefficient of every cell of every level: leaves from the input, other
    cells the mean of their children."""
    f = disc.forest
    val = {c: float(a) for c, a in zip(disc.leaf.cells, coeff)}
    out = []
    for l in range(len(disc.levels) - 1, -1, -1):
        cells = disc.levels[l].cells
        arr = np.zeros(len(cells))
        for i, c in enumerate(cells):
            if c not in val:
                val[c] = float(np.mean([val[ch] for ch in f.children(c)]))
            arr[i] = val[c]
        out.append(arr)
    return out[::-1]


def level_matrix(disc, l, lcoeff):
    lev = disc.levels[l]
    dim, k = disc.forest.dim, disc.k
    h = side(l) / float(1 << 20)
    return _assemble(lev.cellmap, lcoeff * h ** (dim - 2), cell_stiffness(dim, k), lev.n_dofs)


def transfer_matrix(disc, l):
    """P_l: level-(l-1) nodes -> level-l nodes, family-wise E^{x d}.  Entries
    from different families must agree."""
    lev, par = disc.levels[l], disc.levels[l - 1]
    E = embed_1d(disc.k)
    Ed = E
    for _ in range(disc.forest.dim - 1):
        Ed = np.kron(E, Ed)
    fine = lev.family_map
    coarse = par.cellmap[lev.parent_index]
    nf, mf = fine.shape
    nc = coarse.shape[1]
    rows = np.repeat(fine, nc, axis=1).reshape(-1)
    cols = np.tile(coarse, (1, mf)).reshape(-1)
    vals = np.tile(Ed.reshape(-1), nf)
    nz = vals != 0.0
    rows, cols, vals = rows[nz], cols[nz], vals[nz]
    key = rows * par.n_dofs + cols
    order = np.argsort(key, kind="stable")
    key, vals = key[order], vals[order]
    uniq, start = np.unique(key, return_index=True)
    vmax = np.maximum.reduceat(vals, start)
    vmin = np.minimum.reduceat(vals, start)
    assert np.all(vmax - vmin <= 1e-15), "inconsistent prolongation entries"
    r, c = uniq // par.n_dofs, uniq % par.n_dofs
    return sp.coo_matrix((vals[start], (r, c)), shape=(lev.n_dofs, par.n_dofs)).tocsr()


def masks(lev):
    return lev.flags == FLAG_S, lev.flags == FLAG_I, lev.flags == FLAG_D
