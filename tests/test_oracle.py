"""Pins of the CPU oracle against what the paper and the mathematics fix
(closed forms, invariants, brute force, two independent formulations,
values printed in the paper).  No GPU and no library needed."""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import gmg_inputs as gi
from oracle import basis, problem
from oracle.assemble import (cell_h, constraint_matrix, leaf_matrices, level_coefficients,
                             level_matrix, transfer_matrix)
from oracle.dofs import FLAG_D, FLAG_I, FLAG_S, NodeKeys, discretize
from oracle.forest import Forest, side
from oracle.mg import FullSpaceMG, LocalSmoothingMG, chebyshev, lanczos_lambda_max

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def forest_of(coarse, g=0, cycles=0, marker="corner"):
    return problem.build_forest(gi.MeshRecipe(coarse, g, cycles, marker))


# ------------------------------------------------------------------ 1D basis

def test_1d_matrices_closed_form():
    assert np.allclose(basis.mass_1d(1), np.array([[2, 1], [1, 2]]) / 6.0, atol=1e-15)
    assert np.allclose(basis.stiff_1d(1), np.array([[1, -1], [-1, 1]]), atol=1e-15)
    assert np.allclose(basis.mass_1d(2), np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30.0,
                       atol=1e-15)
    assert np.allclose(basis.stiff_1d(2), np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 3.0,
                       atol=1e-14)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_1d_invariants(k):
    x = basis.gll_points(k)
    assert np.allclose(x + x[::-1], 1.0, atol=0)
    M, K = basis.mass_1d(k), basis.stiff_1d(k)
    assert abs(M.sum() - 1.0) < 1e-14                    # integral of 1 over [0,1]
    assert np.allclose(K @ np.ones(k + 1), 0, atol=1e-12)  # constants in the kernel
    assert abs(x @ K @ x - 1.0) < 1e-12                   # int (x')^2 = 1
    # Gauss-Lobatto nodes are the roots of (1-t^2) P_k'(t)
    t = 2 * x[1:-1] - 1
    assert np.allclose(np.polynomial.legendre.legval(t, np.polynomial.legendre.legder(
        np.eye(k + 1)[k])), 0, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_embedding_reproduces_polynomials(k):
    E = basis.embed_1d(k)
    xp, xf = basis.gll_points(k), basis.family_points(k)
    for p in range(k + 1):
        assert np.allclose(E @ xp ** p, xf ** p, atol=1e-14)


# ------------------------------------------------------------------ forest

def _balanced(f):
    lv = list(f.leaves)
    for a, b in itertools.combinations(lv, 2):
        if abs(a[0] - b[0]) >= 2 and f.touching(a, b):
            return False
    return True


@pytest.mark.parametrize("coarse,g", [("lshape", 3), ("square", 2), ("fichera", 1), ("cube", 2)])
def test_uniform_counts(coarse, g):
    f = forest_of(coarse, g)
    n_c = len(gi.COARSE_MESHES[coarse][1])
    assert len(f.leaves) == n_c * 2 ** (f.dim * g)


@pytest.mark.parametrize("coarse,g,cycles,marker", [("lshape", 2, 3, "corner"),
                                                     ("fichera", 1, 2, "corner+random")])
def test_closure_balanced_bruteforce(coarse, g, cycles, marker):
    f = forest_of(coarse, g, cycles, marker)
    assert _balanced(f)
    n = len(f.leaves)
    assert f.close() == 0 and len(f.leaves) == n        # idempotent


def _bruteforce_balance(f):
    """The definition, directly: while two touching leaves differ by >= 2
    levels, refine the coarser one."""
    while True:
        lv = list(f.leaves)
        bad = {min(a, b) for a, b in itertools.combinations(lv, 2)
               if abs(a[0] - b[0]) >= 2 and f.touching(a, b)}
        if not bad:
            return
        f._refine_cells(bad)


@pytest.mark.parametrize("dim", [2, 3])
def test_closure_equals_definition(dim):
    rng = np.random.default_rng(7)
    origins = [(0,) * dim, (1,) + (0,) * (dim - 1)]
    fa, fb = Forest(dim, origins), Forest(dim, origins)
    for step in range(5 if dim == 2 else 4):
        lv, an = fa.leaves_arrays()
        flags = (rng.random(len(lv)) < (1.0 if step == 0 else 0.15)).astype(np.uint8)
        order_b = fb.leaf_order()
        assert order_b == fa.leaf_order()
        fa.refine(flags)
        fb._refine_cells([c for c, fl in zip(order_b, flags) if fl])
        _bruteforce_balance(fb)
        assert fa.leaves == fb.leaves
    assert max(c[0] for c in fa.leaves) >= 3


def test_canonical_order_is_z_order():
    f = forest_of("square", 2)
    order = f.leaf_order()
    # the first four leaves are the children of the first level-1 cell
    s = side(2)
    assert [c[1] for c in order[:4]] == [(0, 0), (s, 0), (0, s), (s, s)]


# ------------------------------------------------------------------ DoFs

@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("g", [0, 1, 2])
def test_uniform_dof_counts(k, g):
    n = 2 ** g
    d = discretize(forest_of("lshape", g), k)
    assert d.leaf.n_dofs == (2 * k * n + 1) ** 2 - (k * n) ** 2
    assert len(d.leaf.hkeys) == 0
    d = discretize(forest_of("fichera", g), k) if g < 2 else None
    if d is not None:
        assert d.leaf.n_dofs == (2 * k * n + 1) ** 3 - (k * n) ** 3
    d = discretize(forest_of("cube", g), k) if g < 2 else None
    if d is not None:
        assert d.leaf.n_dofs == (k * n + 1) ** 3


def test_paper_fichera_117():
    d = discretize(forest_of("fichera", 0), 2)
    assert d.leaf.n_dofs == GOLD["fichera_coarse_q2_unknowns"]["value"]


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_keys_equal_iff_coordinates_equal(k):
    f = forest_of("lshape", 2, 2, "corner")
    nk = NodeKeys(2, k)
    seen = {}
    for c in f.cells:
        for key in nk.cell_keys(c):
            x = tuple(round(v, 12) for v in nk.coord(key))
            if x in seen:
                assert seen[x] == key
            seen[x] = key
    assert len(set(seen.values())) == len(seen)


def test_constraint_weights_closed_form():
    # Q1: edge midpoints 1/2 (2D); face centres 1/4 (3D)
    f = Forest(2, [(0, 0), (1, 0)])
    f.refine(np.array([1, 0], np.uint8))
    d = discretize(f, 1)
    assert len(d.leaf.hkeys) == 1
    assert np.allclose(d.leaf.c_weights, [0.5, 0.5])
    f = Forest(3, [(0, 0, 0), (1, 0, 0)])
    f.refine(np.array([1, 0], np.uint8))
    d = discretize(f, 1)
    w = sorted(np.diff(d.leaf.c_offsets).tolist())
    assert w == [2, 2, 2, 2, 4]
    for h in range(len(d.leaf.hkeys)):
        ws = d.leaf.c_weights[d.leaf.c_offsets[h]:d.leaf.c_offsets[h + 1]]
        assert np.allclose(ws, 1.0 / len(ws))
    # Q2 at the quarter points: (3/8, 3/4, -1/8) and its mirror
    f = Forest(2, [(0, 0), (1, 0)])
    f.refine(np.array([1, 0], np.uint8))
    d = discretize(f, 2)
    ws = sorted(tuple(np.round(d.leaf.c_weights[d.leaf.c_offsets[h]:d.leaf.c_offsets[h + 1]], 15))
                for h in range(len(d.leaf.hkeys)))
    assert np.allclose(ws[0], [-1 / 8, 3 / 4, 3 / 8]) and np.allclose(ws[1], [3 / 8, 3 / 4, -1 / 8])


@pytest.mark.parametrize("k", [1, 2, 3])
def test_constraints_interpolate_polynomials(k):
    # a hanging value equals the coarse interpolant: exact for degree <= k
    f = forest_of("lshape", 2, 2, "corner")
    d = discretize(f, k)
    assert len(d.leaf.hkeys) > 0
    nk = d.nk
    X = np.array([nk.coord(key) for key in d.leaf.keys])
    H = np.array([nk.coord(key) for key in d.leaf.hkeys])
    for px, py in [(0, 0), (k, 0), (1, k), (k, k)]:
        vals = X[:, 0] ** px * X[:, 1] ** py
        C = constraint_matrix(d.leaf)
        ext = C @ vals
        assert np.allclose(ext[d.leaf.n_dofs:], H[:, 0] ** px * H[:, 1] ** py, atol=1e-13)


def test_level_flags_and_copy_map():
    f = forest_of("fichera", 1, 2, "corner+random")
    d = discretize(f, 2)
    for l, lev in enumerate(d.levels):
        if l == 0:
            assert not (lev.flags == FLAG_I).any()
    # copy targets are S or D nodes with the same key
    for i, key in enumerate(d.leaf.keys):
        lev = d.levels[d.copy_level[i]]
        assert lev.keys[d.copy_index[i]] == key
        assert lev.flags[d.copy_index[i]] != FLAG_I
    # the finest level mesh is all leaves: no I nodes there when it is uniform
    assert d.leaf.dirichlet.sum() > 0


# ------------------------------------------------------------------ operators

def test_q1_stencils():
    f = forest_of("square", 3)
    d = discretize(f, 1)
    A, _ = leaf_matrices(d, np.ones(len(f.leaves)))
    A = A.toarray()
    X = np.array([d.nk.coord(k) for k in d.leaf.keys])
    i = int(np.argmin(((X - 0.5) ** 2).sum(1)))
    row = A[i]
    assert abs(row[i] - 8 / 3) < 1e-13
    nb = np.nonzero(np.abs(row) > 1e-14)[0]
    assert len(nb) == 9 and np.allclose(row[nb[nb != i]], -1 / 3)
    f = forest_of("cube", 2)
    d = discretize(f, 1)
    A, _ = leaf_matrices(d, np.ones(len(f.leaves)))
    A = A.toarray()
    X = np.array([d.nk.coord(k) for k in d.leaf.keys])
    i = int(np.argmin(((X - 0.5) ** 2).sum(1)))
    h = 0.25
    vals = {}
    for j in np.nonzero(np.abs(A[i]) > 1e-15)[0]:
        dist = int(round(np.abs(X[j] - X[i]).sum() / h))
        vals.setdefault(dist, set()).add(round(A[i, j], 13))
    assert vals[0] == {round(8 * h / 3, 13)}
    assert 1 not in vals                        # face neighbours: 0
    assert vals[2] == {round(-h / 6, 13)} and vals[3] == {round(-h / 12, 13)}


@pytest.mark.parametrize("k", [1, 2, 3])
def test_operators_symmetric_and_kernel(k):
    f = forest_of("lshape", 1, 2, "corner")
    d = discretize(f, k)
    coeff = gi.coeff_cells("checker", *f.leaves_arrays())
    A, M = leaf_matrices(d, coeff)
    assert abs(A - A.T).max() < 1e-12
    assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-11        # constants: zero energy
    assert abs(M.sum() - 3.0) < 1e-12                            # area of the L-shape
    lc = level_coefficients(d, coeff)
    for l in range(len(d.levels)):
        Al = level_matrix(d, l, lc[l])
        assert np.abs(Al @ np.ones(Al.shape[0])).max() < 1e-11


@pytest.mark.parametrize("k", [1, 2, 3])
def test_transfer_reproduces_polynomials(k):
    f = forest_of("fichera", 0, 2, "corner")
    d = discretize(f, k)
    for l in range(1, len(d.levels)):
        P = transfer_matrix(d, l)
        Xf = np.array([d.nk.coord(key) for key in d.levels[l].keys])
        Xc = np.array([d.nk.coord(key) for key in d.levels[l - 1].keys])
        rows = np.unique(d.levels[l].family_map)
        for e in [(0, 0, 0), (k, 0, 0), (1, k, 0), (0, 1, k)]:
            qc = np.prod(Xc ** np.array(e), axis=1)
            qf = np.prod(Xf ** np.array(e), axis=1)
            assert np.allclose((P @ qc)[rows], qf[rows], atol=1e-13)


# ------------------------------------------------------------------ smoother pieces

def test_lambda_estimate_bounds():
    for coarse, g in [("square", 4), ("cube", 3)]:
        f = forest_of(coarse, g)
        d = discretize(f, 1)
        lc = level_coefficients(d, np.ones(len(f.leaves)))
        l = len(d.levels) - 1
        A = level_matrix(d, l, lc[l]).tocsr()
        S = np.nonzero(d.levels[l].flags == FLAG_S)[0]
        AS = A[S][:, S]
        dinv = 1.0 / AS.diagonal()
        lam = lanczos_lambda_max(AS, dinv, (S % 12) - 5.5, 10)
        dh = np.sqrt(dinv)
        true = np.linalg.eigvalsh((AS.toarray() * dh[:, None]) * dh[None, :]).max()
        assert lam <= true * (1 + 1e-12) and lam >= 0.9 * true
        # Fourier symbol of Q1: lambda_max(D^-1 A) -> 1.5 as h -> 0 (2D and 3D)
        assert 1.35 < true < 1.5


def test_chebyshev_error_polynomial():
    rng = np.random.default_rng(1)
    n, m = 30, 4
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lamb = np.linspace(0.05, 2.0, n)
    A = Q @ np.diag(lamb) @ Q.T
    A = 0.5 * (A + A.T)
    dinv = 1.0 / np.diag(A)
    dh = np.sqrt(dinv)
    B = (A * dh[:, None]) * dh[None, :]
    mu, V = np.linalg.eigh(B)
    lam = mu.max()
    a, b = 0.08 * lam, 1.2 * lam
    th, de = (a + b) / 2, (b - a) / 2
    T = lambda k, x: np.cosh(k * np.arccosh(x)) if x >= 1 else np.cos(k * np.arccos(np.clip(x, -1, 1)))
    g = rng.standard_normal(n)
    xs = np.linalg.solve(A, g)
    x = chebyshev(A, dinv, g, lam, m)
    # e_m = p_m(D^-1 A) e_0 with p_m(t) = T_m((th - t)/de) / T_m(th/de), e_0 = xs
    e0 = xs / dh                                   # symmetrised coordinates
    pm = np.array([T(m, (th - t) / de) / T(m, th / de) for t in mu])
    em = V @ (pm * (V.T @ e0))
    assert np.allclose((xs - x) / dh, em, atol=1e-12 * np.abs(e0).max())


# ------------------------------------------------------------------ V-cycle and CG

@pytest.mark.parametrize("coarse,g,cycles,marker,k", [
    ("lshape", 3, 3, "corner", 1), ("lshape", 2, 3, "corner", 2),
    ("fichera", 1, 2, "corner+random", 1), ("fichera", 0, 2, "corner+random", 2),
    ("lshape", 1, 2, "corner", 4)])
def test_vcycle_two_formulations(coarse, g, cycles, marker, k):
    f = forest_of(coarse, g, cycles, marker)
    coeff = gi.coeff_cells("checker", *f.leaves_arrays()) if f.dim == 3 else None
    P = problem.setup(f, k, coeff=coeff)
    fs = FullSpaceMG(P.disc, P.coeff, P.mg)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(P.n_dofs)
    r[~P.free] = 0
    z1, z2 = P.mg.vcycle(r), fs.vcycle(r)
    assert np.linalg.norm(z1 - z2) <= 1e-12 * np.linalg.norm(z1)


def test_vcycle_symmetric():
    f = forest_of("lshape", 2, 3, "corner")
    P = problem.setup(f, 2)
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal((2, P.n_dofs))
    u[~P.free] = 0
    v[~P.free] = 0
    Bu, Bv = P.mg.vcycle(u), P.mg.vcycle(v)
    assert abs(Bu @ v - u @ Bv) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(v) * max(
        np.linalg.norm(Bu) / np.linalg.norm(u), 1.0)


def test_uniform_mesh_has_no_interface():
    f = forest_of("fichera", 1)
    d = discretize(f, 2)
    for lev in d.levels:
        assert not (lev.flags == FLAG_I).any()


@pytest.mark.parametrize("name,g,k", [("C1-tiny", None, 1), ("C1", None, 1), ("C2", 1, 2),
                                      ("C2", 2, 2)])
def test_cg_converges_in_paper_band(name, g, k):
    w = gi.workload(name, g=g)
    f = problem.build_forest(w.recipe)
    P = problem.setup(f, k)
    fn = gi.rhs_nodal(w.rhs, P.n_dofs)
    x, it, hist, ok = P.solve(fn)
    lo, hi = GOLD["cg_iterations_band"]["value"]
    assert ok and lo <= it <= hi
    b = P.rhs(fn)
    assert np.linalg.norm(b - P.A @ x) <= 1e-10 * np.linalg.norm(b) * 1.0001
    if P.n_dofs < 20000:
        u = P.exact(fn)
        assert np.linalg.norm(x - u) <= 1e-6 * np.linalg.norm(u)


def test_iteration_counts_flat_under_refinement():
    its = []
    for g in (2, 3, 4, 5):
        f = forest_of("lshape", g, 3, "corner")
        P = problem.setup(f, 1)
        _, it, _, _ = P.solve(np.ones(P.n_dofs))
        its.append(it)
    assert max(its) - min(its) <= 2


@pytest.mark.parametrize("k", [1, 2])
def test_manufactured_solution_rate(k):
    """u = sin(pi x) sin(pi y) on the L-shape, f = 2 pi^2 u (nodal), a = 1:
    L2 error O(h^(k+1))."""
    errs = []
    for g in (1, 2, 3):
        f = forest_of("lshape", g)
        P = problem.setup(f, k)
        d = P.disc
        X = np.array([d.nk.coord(key) for key in d.leaf.keys])
        uex = lambda x, y: np.sin(np.pi * x) * np.sin(np.pi * y)
        fn = 2 * np.pi ** 2 * uex(X[:, 0], X[:, 1])
        x, it, hist, ok = P.solve(fn)
        q, w = basis.gauss(k + 2)
        V = basis.lagrange(d.nk.x, q)
        err = 0.0
        for ci, c in enumerate(d.leaf.cells):
            h = side(c[0]) / float(1 << 20)
            x0, y0 = c[1][0] / float(1 << 20), c[1][1] / float(1 << 20)
            uc = x[d.leaf.cellmap[ci]].reshape(k + 1, k + 1)   # [y, x]
            uh = V @ uc @ V.T                                     # [qy, qx]
            QX, QY = np.meshgrid(x0 + h * q, y0 + h * q)
            err += (h * h * (w[:, None] * w[None, :]) * (uh - uex(QX, QY)) ** 2).sum()
        errs.append(math.sqrt(err))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert abs(rates[-1] - (k + 1)) < 0.15, (errs, rates)


def test_mixed_precision_counts():
    f = forest_of("fichera", 1, 2, "corner+random")
    P64 = problem.setup(f, 2)
    P32 = problem.setup(f, 2, mg_dtype=np.float32)
    fn = gi.rhs_nodal("noise", P64.n_dofs)
    x64, it64, _, ok64 = P64.solve(fn)
    x32, it32, h32, ok32 = P32.solve(fn)
    assert ok64 and ok32 and it32 <= it64 + 1
    assert np.linalg.norm(x32 - x64) <= 1e-8 * np.linalg.norm(x64)
