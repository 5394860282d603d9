"""End-to-end oracle: forest + degree + coefficient + nodal right-hand side ->
CG iterate, iteration count and residual history (Sec. 1: CG preconditioned
by one V-cycle; Sec. 4.1/4.3: stop at 1e-10 in the unpreconditioned residual).

The right-hand side is the Galerkin load vector of the nodal interpolant f_h
(hanging values from the constraints): b = C^T M C f_h with Dirichlet rows
set to zero.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from .assemble import leaf_matrices
from .dofs import discretize
from .forest import Forest
from .mg import LocalSmoothingMG, pcg


@dataclass
class OracleProblem:
    disc: object
    A: object        # constrained leaf stiffness with Dirichlet rows/cols zeroed
    M: object        # constrained leaf mass (rows of Dirichlet DoFs zeroed)
    free: np.ndarray
    mg: LocalSmoothingMG
    coeff: np.ndarray

    @property
    def n_dofs(self):
        return self.disc.leaf.n_dofs

    def rhs(self, f_nodal):
        b = self.M @ np.asarray(f_nodal, dtype=np.float64)
        b[~self.free] = 0.0
        return b

    def solve(self, f_nodal, rtol=1e-10, max_iter=200):
        b = self.rhs(f_nodal)
        x, it, hist, ok = pcg(self.A, b, self.mg.vcycle, rtol, max_iter)
        return x, it, hist, ok

    def exact(self, f_nodal):
        b = self.rhs(f_nodal)
        fr = np.nonzero(self.free)[0]
        u = np.zeros_like(b)
        u[fr] = spla.spsolve(self.A.tocsr()[fr][:, fr].tocsc(), b[fr])
        return u


def mask_dirichlet(A, free):
    import scipy.sparse as sp
    Dm = sp.diags(free.astype(np.float64))
    return (Dm @ A @ Dm).tocsr()


def setup(forest: Forest, k: int, coeff=None, cheb_degree=4, mg_dtype=np.float64,
          eig_iters=10, lo=0.08, hi=1.2, smoother="chebyshev", relax=1.0) -> OracleProblem:
    disc = discretize(forest, k)
    n_leaves = len(disc.leaf.cells)
    coeff = np.ones(n_leaves) if coeff is None else np.asarray(coeff, dtype=np.float64)
    A, M = leaf_matrices(disc, coeff)
    free = disc.leaf.dirichlet == 0
    A = mask_dirichlet(A, free)
    mg = LocalSmoothingMG(disc, coeff, cheb_degree=cheb_degree, lo=lo, hi=hi,
                          eig_iters=eig_iters, dtype=mg_dtype, smoother=smoother, relax=relax)
    return OracleProblem(disc, A, M.tocsr(), free, mg, coeff)


def build_forest(recipe):
    """Run a gmg_inputs recipe through the oracle forest."""
    import gmg_inputs as gi

    def create(dim, origins):
        return Forest(dim, origins)

    def refine(f, flags):
        f.refine(flags)

    def leaves(f):
        return f.leaves_arrays()

    return gi.build_mesh(recipe, create, refine, leaves)
