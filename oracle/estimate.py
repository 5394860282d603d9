"""Residual-based a posteriori error estimator and marking of the adaptive
loop (Sec. 4.3): for every leaf K

    e(K) = e_cell(K) + e_face(K),
    e_cell(K) = h_K^2 || f + eps Laplace u_h ||_K^2,
    e_face(K) = sum over the faces F of K of h_F || [eps grad u_h . n] ||_F^2,

and the loop refines the 14.2 % of the leaves with the largest e(K).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Written per cell, by
evaluating the cell polynomials at physical quadrature points, with no face
list: plain and slow.

Readings where the paper is silent:
* u_h on a cell is the Q_k polynomial of its constrained nodal values
  (hanging values from the constraints); f is the nodal interpolant f_h of
  the given nodal values, the same function the load vector uses.
* Integrals by Gauss quadrature with k+1 points per direction (exact for
  the squared polynomial integrands when f = f_h).
* h_K and h_F are the side length of K (a face F of K has side h_K).
* Faces on the domain boundary carry no jump term (u = 0 is imposed there).
* Across a refinement face, K's face is the union of the 2^(d-1) faces of
  the finer neighbours; the jump is integrated over each of them.
* The jump is eps_K grad u_K . n_K + eps_N grad u_N . n_N with n_N = -n_K.
* Marking: the round(0.142 n) leaves of largest e(K); equal values in
  canonical leaf order.
"""
from __future__ import annotations

import itertools

import numpy as np

from .assemble import constraint_matrix
from .basis import gauss, lagrange, lagrange_deriv
from .forest import UNIT, side


def lagrange_deriv2(nodes: np.ndarray, xi) -> np.ndarray:
    """S[q, j] = l_j''(xi_q): each Lagrange polynomial built from its roots,
    differentiated twice."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    n = len(nodes)
    S = np.zeros((len(xi), n))
    for j in range(n):
        others = [nodes[m] for m in range(n) if m != j]
        p = np.polynomial.Polynomial.fromroots(others)
        p = p / p(nodes[j])
        S[:, j] = p.deriv(2)(xi)
    return S


class _Cells:
    """Leaves with their constrained nodal values of u and f."""

    def __init__(self, disc, u, f):
        leaf = disc.leaf
        self.dim, self.k = disc.forest.dim, disc.k
        self.nodes = disc.nk.x
        self.cells = leaf.cells
        self.index = {c: i for i, c in enumerate(leaf.cells)}
        C = constraint_matrix(leaf)
        ue, fe = C @ np.asarray(u, np.float64), C @ np.asarray(f, np.float64)
        N = leaf.n_dofs
        ids = np.where(leaf.cellmap >= 0, leaf.cellmap, N + (-leaf.cellmap - 1))
        n = self.k + 1
        shape = (len(leaf.cells),) + (n,) * self.dim          # [cell, (z,) y, x]
        self.u = ue[ids].reshape(shape)
        self.f = fe[ids].reshape(shape)

    def geom(self, i):
        lvl, a = self.cells[i]
        h = side(lvl) / float(UNIT)
        return np.array(a, dtype=np.float64) / UNIT, h

    def _tensor(self, vals, mats):
        """sum_j vals[j] prod_a mats[a][:, j_a] at points (mats[a]: [npts, n])."""
        if self.dim == 2:
            return np.einsum("yx,px,py->p", vals, mats[0], mats[1])
        return np.einsum("zyx,px,py,pz->p", vals, mats[0], mats[1], mats[2])

    def grad(self, i, X):
        """gradient of u_h on cell i at physical points X [npts, dim]"""
        o, h = self.geom(i)
        xi = (X - o) / h
        V = [lagrange(self.nodes, xi[:, a]) for a in range(self.dim)]
        D = [lagrange_deriv(self.nodes, xi[:, a]) for a in range(self.dim)]
        g = np.zeros((len(X), self.dim))
        for a in range(self.dim):
            mats = [D[b] if b == a else V[b] for b in range(self.dim)]
            g[:, a] = self._tensor(self.u[i], mats) / h
        return g


def estimate(disc, u, f_nodal, eps):
    """e(K) for every leaf in canonical order.  u, f_nodal: leaf DoF vectors;
    eps: coefficient per leaf."""
    dim, k = disc.forest.dim, disc.k
    forest = disc.forest
    cs = _Cells(disc, u, f_nodal)
    eps = np.asarray(eps, np.float64)
    q, w = gauss(k + 1)
    n_leaves = len(cs.cells)
    e = np.zeros(n_leaves)
    # cell residuals
    Vq = lagrange(cs.nodes, q)
    Sq = lagrange_deriv2(cs.nodes, q)
    grid = np.array(list(itertools.product(range(len(q)), repeat=dim)))[:, ::-1]  # x fastest
    mats_V = [Vq[grid[:, a]] for a in range(dim)]
    W = np.prod([w[grid[:, a]] for a in range(dim)], axis=0)
    for i in range(n_leaves):
        o, h = cs.geom(i)
        lap = np.zeros(len(grid))
        for a in range(dim):
            mats = [Sq[grid[:, b]] if b == a else mats_V[b] for b in range(dim)]
            lap += cs._tensor(cs.u[i], mats) / h ** 2
        fq = cs._tensor(cs.f[i], mats_V)
        e[i] = h ** 2 * float((W * h ** dim * (fq + eps[i] * lap) ** 2).sum())
    # face jumps, per cell and face
    for i, (lvl, a) in enumerate(cs.cells):
        o, h = cs.geom(i)
        s = side(lvl)
        for ax in range(dim):
            for hi in (0, 1):
                na = list(a)
                na[ax] += s if hi else -s
                na = tuple(na)
                if not forest.inside(na):
                    continue                                     # domain boundary
                nrm = np.zeros(dim)
                nrm[ax] = 1.0 if hi else -1.0
                if (lvl, na) in forest.leaves:
                    parts = [((lvl, na), o, h)]                  # same level: the whole face
                elif (lvl, na) in forest.cells:
                    parts = []                                   # finer neighbours: their faces
                    for ch in forest.children((lvl, na)):
                        touches = (ch[1][ax] == na[ax]) if hi else (ch[1][ax] + side(lvl + 1) == na[ax] + s)
                        if touches:
                            assert ch in forest.leaves, "2:1 balance violated"
                            parts.append((ch, np.array(ch[1], np.float64) / UNIT, h / 2))
                else:
                    parts = [(forest.covering_leaf(lvl, na), o, h)]  # coarser neighbour
                jump2 = 0.0
                for nb, fo, fh in parts:
                    j = cs.index[nb]
                    # Gauss points on the (sub)face box anchored at fo, side fh
                    tang = [b for b in range(dim) if b != ax]
                    pts = np.array(list(itertools.product(range(len(q)), repeat=dim - 1)))
                    X = np.zeros((len(pts), dim))
                    X[:, ax] = o[ax] + (h if hi else 0.0)
                    for t, b in enumerate(tang):
                        X[:, b] = fo[b] + fh * q[pts[:, t]]
                    Wf = np.prod([w[pts[:, t]] for t in range(dim - 1)], axis=0) * fh ** (dim - 1)
                    jmp = eps[i] * cs.grad(i, X) @ nrm - eps[j] * cs.grad(j, X) @ nrm
                    jump2 += float((Wf * jmp ** 2).sum())
                e[i] += h * jump2
    return e


def mark_fraction(eta, fraction=0.142):
    """Flags of the round(fraction n) leaves with the largest eta (ties in
    canonical order)."""
    eta = np.asarray(eta, np.float64)
    n = len(eta)
    m = int(np.floor(fraction * n + 0.5))
    order = np.lexsort((np.arange(n), -eta))
    flags = np.zeros(n, dtype=np.uint8)
    flags[order[:m]] = 1
    return flags
