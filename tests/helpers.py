"""Shared test helpers: build the same seeded workload through the oracle and
through the library."""
import os
import re

import numpy as np

import gmg_inputs as gi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    """Function names declared in include/gmg.h."""
    txt = open(os.path.join(ROOT, "include", "gmg.h")).read()
    return sorted(set(re.findall(r"\b(gmg_[a-z0-9_]+)\s*\(", txt)))


def recipe(coarse, g, cycles, marker):
    return gi.MeshRecipe(coarse, g, cycles, marker)


CASES = {
    # name: (recipe, degree)
    "lshape-q1": (recipe("lshape", 3, 3, "corner"), 1),
    "lshape-q2": (recipe("lshape", 2, 3, "corner"), 2),
    "lshape-q4": (recipe("lshape", 2, 3, "corner"), 4),
    "fichera-q1": (recipe("fichera", 1, 2, "corner+random"), 1),
    "fichera-q2": (recipe("fichera", 1, 2, "corner+random"), 2),
    "fichera-q3": (recipe("fichera", 1, 2, "corner+random"), 3),
    "fichera-q4": (recipe("fichera", 1, 1, "corner+random"), 4),
    "cube-q2": (recipe("cube", 2, 2, "corner"), 2),
    # degenerate meshes: no refinement (one level, coarse solve only), no
    # free DoF at all, one family smaller than a cooperative workgroup
    "cube-q1-g0": (recipe("cube", 0, 0, "corner"), 1),
    "fichera-q2-g0": (recipe("fichera", 0, 0, "corner"), 2),
    "lshape-q2-g0": (recipe("lshape", 0, 0, "corner"), 2),
    "cube-q3-g1": (recipe("cube", 1, 0, "corner"), 3),
}


def oracle_problem(rec, k, coeff_kind="one", **kw):
    from oracle import problem
    f = problem.build_forest(rec)
    coeff = gi.coeff_cells(coeff_kind, *f.leaves_arrays()) if coeff_kind != "one" else None
    return problem.setup(f, k, coeff=coeff, **kw), coeff


def library_problem(rec, k, coeff_kind="one", **opt):
    from paper_1904_03317_amd import gmg
    m = gmg.build_mesh(rec)
    coeff = gi.coeff_cells(coeff_kind, *m.leaves()) if coeff_kind != "one" else None
    P = gmg.Problem(m, gmg.options(degree=k, **opt), coeff=coeff)
    return m, P, coeff


def compare_maps(P, d):
    """Bit-exact comparison of the library's host maps with the oracle's."""
    k = d.k
    npc = (k + 1) ** d.forest.dim
    assert np.array_equal(P.array("LEAF_CELLMAP").reshape(-1, npc), d.leaf.cellmap)
    assert np.array_equal(P.array("LEAF_DIRICHLET"), d.leaf.dirichlet)
    assert np.array_equal(P.array("CON_OFFSETS"), d.leaf.c_offsets)
    assert np.array_equal(P.array("CON_MASTERS"), d.leaf.c_masters)
    if len(d.leaf.c_weights):
        assert np.abs(P.array("CON_WEIGHTS") - d.leaf.c_weights).max() <= 1e-14
    assert np.array_equal(P.array("COPY_LEVEL"), d.copy_level)
    assert np.array_equal(P.array("COPY_INDEX"), d.copy_index)
    info = P.info()
    assert info.n_levels == len(d.levels)
    for l, lev in enumerate(d.levels):
        assert np.array_equal(P.array("LEVEL_CELLMAP", l).reshape(lev.cellmap.shape), lev.cellmap)
        assert np.array_equal(P.array("LEVEL_FLAGS", l), lev.flags)
        if l:
            assert np.array_equal(P.array("LEVEL_PARENT", l), lev.parent_index)


def _abs_ref(dim, k, mass):
    """Cell matrix assembled from the absolute values of the 1D factors: a
    majorant of the size of every product the tensor-product evaluation
    forms, so that (|A|-majorant |x|)_i bounds the rounding of row i."""
    from oracle import basis
    M = np.abs(basis.mass_1d(k))
    K = np.abs(basis.stiff_1d(k))
    if mass:
        return np.kron(np.kron(M, M), M) if dim == 3 else np.kron(M, M)
    if dim == 2:
        return np.kron(M, K) + np.kron(K, M)
    return np.kron(np.kron(M, M), K) + np.kron(np.kron(M, K), M) + np.kron(np.kron(K, M), M)


def leaf_row_scale(op, x, mass=False):
    """Row scales of the constrained leaf operator (or mass matrix) applied
    to x: |C|^T A_abs |C| |x| with the cell majorant above; Dirichlet rows 0."""
    import scipy.sparse as sp
    from oracle.assemble import _assemble, _extended, cell_h, constraint_matrix
    d = op.disc
    leaf, dim, k = d.leaf, d.forest.dim, d.k
    N, H = leaf.n_dofs, len(leaf.hkeys)
    h = cell_h(leaf.cells, dim)
    sc = h ** dim if mass else np.asarray(op.coeff) * h ** (dim - 2)
    Aa = _assemble(_extended(leaf.cellmap, N), sc, _abs_ref(dim, k, mass), N + H)
    C = abs(constraint_matrix(leaf))
    s = C.T @ (Aa @ (C @ np.abs(x)))
    s[~op.free] = 0.0
    return s


def level_row_scale(d, l, lcoeff, x):
    from oracle.assemble import _assemble
    from oracle.forest import side
    lev = d.levels[l]
    dim, k = d.forest.dim, d.k
    h = side(l) / float(1 << 20)
    Aa = _assemble(lev.cellmap, lcoeff * h ** (dim - 2), _abs_ref(dim, k, False), lev.n_dofs)
    return Aa @ np.abs(x)


def row_err(got, want, scale):
    """largest |got_i - want_i| / scale_i over the rows with a nonzero scale;
    rows with a zero scale must match exactly"""
    nz = scale > 0
    assert np.all(got[~nz] == want[~nz])
    return float((np.abs(got - want)[nz] / scale[nz]).max()) if nz.any() else 0.0
