"""More pins of the CPU oracle, each against something other than the oracle
itself: brute-force geometry for the level splitting S/I/D (Sec. 2.3, Fig. 1),
exact reproduction of global polynomials in the conforming space with hanging
nodes (3D and 2D, degrees 2-4: Galerkin orthogonality gives u_h = u whenever
u lies in V_h and the nodal load interpolates f exactly), L2 convergence rates
k+1 of a smooth manufactured solution on uniform 3D meshes (Sec. 2.1
discretisation), and a volume-weighted brute-force mean for the coefficient
of level cells that are not leaves.  No GPU and no library needed."""
import math

import numpy as np
import pytest

import gmg_inputs as gi
from oracle import basis, problem
from oracle.assemble import constraint_matrix, level_coefficients
from oracle.dofs import FLAG_D, FLAG_I, FLAG_S, discretize
from oracle.forest import UNIT, side


def forest_of(coarse, g=0, cycles=0, marker="corner"):
    return problem.build_forest(gi.MeshRecipe(coarse, g, cycles, marker))


def _coords(nk, keys):
    return np.array([nk.coord(key) for key in keys], dtype=np.float64).reshape(len(keys), -1)


def _on_boundary_float(f, X, delta=1e-7):
    """A point is on the domain boundary iff one of the 2^d points at distance
    delta along the diagonals lies outside every (open) coarse cell."""
    dim = f.dim
    org = np.array(f.origins, dtype=np.float64)
    out = np.zeros(len(X), dtype=bool)
    for s in range(1 << dim):
        sg = np.array([1.0 if (s >> i) & 1 else -1.0 for i in range(dim)])
        P = X + delta * sg
        inside = ((P[:, None, :] > org[None]) & (P[:, None, :] < org[None] + 1.0)).all(axis=2).any(axis=1)
        out |= ~inside
    return out


@pytest.mark.parametrize("coarse,g,cycles,marker,k", [
    ("lshape", 2, 3, "corner", 1), ("lshape", 2, 2, "corner", 3),
    ("fichera", 1, 2, "corner+random", 2), ("fichera", 1, 1, "corner+random", 3),
    ("cube", 2, 2, "corner", 1)])
def test_level_flags_bruteforce(coarse, g, cycles, marker, k):
    """Fig. 1 / Sec. 2.3 on the level mesh T_l (level-l cells plus the coarser
    leaves): a node of a level-l cell is D on the domain boundary, else I when
    it lies in the closed cell of some leaf of level < l, else S.  Checked
    against a brute-force point-in-box test over all leaves, which shares
    nothing with the oracle's neighbour walk."""
    f = forest_of(coarse, g, cycles, marker)
    d = discretize(f, k)
    leaves = f.leaf_order()
    lv = np.array([c[0] for c in leaves])
    lo = np.array([c[1] for c in leaves], dtype=np.float64) / UNIT
    hi = lo + np.array([side(c[0]) for c in leaves], dtype=np.float64)[:, None] / UNIT
    n_i = 0
    for l, lev in enumerate(d.levels):
        X = _coords(d.nk, lev.keys)
        bd = _on_boundary_float(f, X)
        coarser = lv < l
        if coarser.any():
            eps = 1e-12
            inI = ((X[:, None, :] >= lo[coarser][None] - eps) &
                   (X[:, None, :] <= hi[coarser][None] + eps)).all(axis=2).any(axis=1)
        else:
            inI = np.zeros(len(X), dtype=bool)
        want = np.where(bd, FLAG_D, np.where(inI, FLAG_I, FLAG_S)).astype(np.uint8)
        assert np.array_equal(lev.flags, want), l
        n_i += int((want == FLAG_I).sum())
    assert n_i > 0  # the meshes are adaptive: some level has an interface


# ------------------------------------------------------------------ polynomial reproduction

def _poly_case(coarse):
    """A polynomial u = prod p(x_i) vanishing on the whole boundary of the
    domain (faces at x_i in {-1, 0, 1} for the L-shape and the Fichera corner,
    {0, 1} for the unit cube), its Laplacian, and the smallest degree k whose
    Q_k space contains u."""
    if coarse == "cube":
        p = lambda x: x * (1.0 - x)                     # noqa: E731
        pp = lambda x: -2.0 + 0.0 * x                   # noqa: E731
        return p, pp, 2
    p = lambda x: x - x ** 3                            # noqa: E731  (x+1) x (1-x)
    pp = lambda x: -6.0 * x                             # noqa: E731
    return p, pp, 3


@pytest.mark.parametrize("coarse,g,cycles,marker,k", [
    ("cube", 2, 2, "corner", 2), ("cube", 2, 1, "corner", 3),
    ("fichera", 1, 2, "corner+random", 3), ("fichera", 1, 1, "corner+random", 4),
    ("lshape", 2, 3, "corner", 3), ("lshape", 2, 2, "corner", 4)])
def test_polynomial_reproduction_adaptive(coarse, g, cycles, marker, k):
    """u in V_h (a global Q_k polynomial that vanishes on the boundary) and
    f = -Laplace u in Q_k, so f_h = f and Galerkin orthogonality gives
    u_h = u exactly: on adaptive meshes with hanging nodes this pins the
    constrained leaf stiffness, the mass matrix of the load vector, the
    hanging-node weights (their interpolated values must match u too) and the
    Dirichlet detection, in 2D and 3D, at degrees 2-4."""
    p, pp, kmin = _poly_case(coarse)
    assert k >= kmin
    f = forest_of(coarse, g, cycles, marker)
    P = problem.setup(f, k)
    d = P.disc
    X = _coords(d.nk, d.leaf.keys)
    dim = f.dim
    u = np.prod([p(X[:, i]) for i in range(dim)], axis=0)
    lap = np.zeros(len(X))
    for i in range(dim):
        t = pp(X[:, i])
        for j in range(dim):
            if j != i:
                t = t * p(X[:, j])
        lap += t
    fn = -lap
    assert len(d.leaf.hkeys) > 0
    uh = P.exact(fn)
    scale = np.abs(u).max()
    assert np.abs(uh - u).max() <= 1e-10 * scale
    # hanging nodes: constrained values equal u at their coordinates
    H = _coords(d.nk, d.leaf.hkeys)
    uH = np.prod([p(H[:, i]) for i in range(dim)], axis=0)
    ext = constraint_matrix(d.leaf) @ uh
    assert np.abs(ext[d.leaf.n_dofs:] - uH).max() <= 1e-10 * scale
    # the multigrid-preconditioned CG reaches the same iterate
    x, it, hist, ok = P.solve(fn)
    assert ok and np.abs(x - u).max() <= 1e-7 * scale


# ------------------------------------------------------------------ convergence rates

def _l2_error(P, x, uex, k):
    d = P.disc
    dim = d.forest.dim
    q, w = basis.gauss(k + 2)
    V = basis.lagrange(d.nk.x, q)                       # [nq, k+1]
    err = 0.0
    C = constraint_matrix(d.leaf)
    xe = C @ x
    N = d.leaf.n_dofs
    for ci, c in enumerate(d.leaf.cells):
        h = side(c[0]) / float(UNIT)
        o = np.array(c[1], dtype=np.float64) / UNIT
        ids = d.leaf.cellmap[ci]
        ids = np.where(ids >= 0, ids, N + (-ids - 1))
        uc = xe[ids].reshape((k + 1,) * dim)            # [z, y, x] (x fastest)
        if dim == 3:
            uh = np.einsum("ai,bj,ck,kji->abc", V, V, V, uc)   # [qx, qy, qz]
            QX, QY, QZ = np.meshgrid(o[0] + h * q, o[1] + h * q, o[2] + h * q, indexing="ij")
            W = h ** 3 * w[:, None, None] * w[None, :, None] * w[None, None, :]
            err += (W * (uh - uex(QX, QY, QZ)) ** 2).sum()
        else:
            uh = np.einsum("ai,bj,ji->ab", V, V, uc)
            QX, QY = np.meshgrid(o[0] + h * q, o[1] + h * q, indexing="ij")
            W = h ** 2 * w[:, None] * w[None, :]
            err += (W * (uh - uex(QX, QY)) ** 2).sum()
    return math.sqrt(err)


@pytest.mark.parametrize("coarse,k,gs", [
    ("fichera", 1, (1, 2, 3)), ("fichera", 2, (0, 1, 2)), ("fichera", 3, (0, 1, 2)),
    ("fichera", 4, (0, 1, 2)), ("cube", 1, (2, 3, 4)), ("cube", 2, (1, 2, 3)),
    ("cube", 3, (0, 1, 2)), ("cube", 4, (0, 1, 2))])
def test_manufactured_solution_rate_3d(coarse, k, gs):
    """u = sin(pi x) sin(pi y) sin(pi z) vanishes on every face of both domains
    (faces at integer coordinates); f = 3 pi^2 u, a = 1.  On uniform meshes
    the L2 error of the Q_k solution decreases as h^(k+1)."""
    uex = lambda x, y, z: np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)  # noqa: E731
    errs = []
    for g in gs:
        f = forest_of(coarse, g)
        P = problem.setup(f, k)
        X = _coords(P.disc.nk, P.disc.leaf.keys)
        fn = 3 * np.pi ** 2 * uex(X[:, 0], X[:, 1], X[:, 2])
        x, it, hist, ok = P.solve(fn, rtol=1e-12)
        assert ok
        errs.append(_l2_error(P, x, uex, k))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert abs(rates[-1] - (k + 1)) < 0.2, (errs, rates)


# ------------------------------------------------------------------ level coefficient

def test_level_coefficient_volume_mean():
    """A level cell that is not a leaf takes the mean coefficient of its
    children, recursively: for cells of equal volume per level that is the
    volume-weighted mean of the leaves inside it (brute-force containment).
    On levels >= 2 every cell of the checkerboard recipe (blocks of 1/4) lies
    in one block, so its value is the block's."""
    f = forest_of("fichera", 1, 2, "corner+random")
    leaves = f.leaf_order()
    coeff = gi.coeff_cells("checker", *f.leaves_arrays())
    d = discretize(f, 1)
    lc = level_coefficients(d, coeff)
    lv = np.array([c[0] for c in leaves])
    an = np.array([c[1] for c in leaves], dtype=np.int64)
    vol = np.array([float(side(c[0])) ** 3 for c in leaves])
    for l, lev in enumerate(d.levels):
        for i, (cl, a) in enumerate(lev.cells):
            s = side(cl)
            inside = (lv >= cl) & np.all((an >= np.array(a)) & (an < np.array(a) + s), axis=1)
            want = float((vol[inside] * coeff[inside]).sum() / vol[inside].sum())
            assert abs(lc[l][i] - want) <= 1e-13 * want, (l, i)
            if l >= 2:
                blk = gi.coeff_cells("checker", np.array([cl], dtype=np.int8), np.array([a]))[0]
                assert lc[l][i] == blk


# ------------------------------------------------------------------ the "MF" smoother of Sec. 4.3

def test_jacobi_closed_form():
    """m relaxed Jacobi steps from x0 are x* + (I - omega D^-1 A)^m (x0 - x*)
    (the error propagation of a stationary iteration); from a zero start the
    first step is omega D^-1 g."""
    from oracle.mg import jacobi
    rng = np.random.default_rng(2)
    B = rng.standard_normal((9, 9))
    A = B @ B.T + 9 * np.eye(9)
    g = rng.standard_normal(9)
    xs = np.linalg.solve(A, g)
    dinv = 1.0 / np.diag(A)
    for omega, m in ((1.0, 1), (1.0, 3), (0.6, 4)):
        G = np.eye(9) - omega * dinv[:, None] * A
        x0 = rng.standard_normal(9)
        want = xs + np.linalg.matrix_power(G, m) @ (x0 - xs)
        assert np.allclose(jacobi(A, dinv, g, omega, m, x0=x0), want, rtol=0, atol=1e-13)
        want0 = xs + np.linalg.matrix_power(G, m) @ (-xs)
        assert np.allclose(jacobi(A, dinv, g, omega, m), want0, rtol=0, atol=1e-13)


@pytest.mark.parametrize("coarse,g,cycles,k", [("fichera", 1, 2, 2), ("lshape", 2, 3, 1)])
def test_vcycle_jacobi_two_formulations_and_symmetry(coarse, g, cycles, k):
    """With the Sec. 4.3 smoother (one undamped Jacobi step) the local
    smoothing V-cycle equals Alg. 2 on the constrained full spaces, and it is
    symmetric (the post-smoothing step is the adjoint of the pre-smoothing
    step)."""
    from oracle.mg import FullSpaceMG
    f = forest_of(coarse, g, cycles, "corner+random" if coarse == "fichera" else "corner")
    coeff = gi.coeff_cells("eps", *f.leaves_arrays()) if f.dim == 3 else None
    P = problem.setup(f, k, coeff=coeff, cheb_degree=1, smoother="jacobi", relax=1.0)
    fs = FullSpaceMG(P.disc, P.coeff, P.mg)
    rng = np.random.default_rng(12)
    u, v = rng.standard_normal((2, P.n_dofs))
    u[~P.free] = 0
    v[~P.free] = 0
    Bu, Bv = P.mg.vcycle(u), P.mg.vcycle(v)
    assert np.linalg.norm(Bu - fs.vcycle(u)) <= 1e-12 * np.linalg.norm(Bu)
    assert abs(Bu @ v - u @ Bv) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(v) * max(
        np.linalg.norm(Bu) / np.linalg.norm(u), 1.0)


def test_eps_coefficient_pattern():
    """Sec. 4.3: eps = 1 where min(x, y, z) > -1/2, 100 elsewhere (checked at
    cell centres in floating point against the exact-integer generator)."""
    f = forest_of("fichera", 2, 1, "corner+random")
    lv, an = f.leaves_arrays()
    a = gi.coeff_cells("eps", lv, an)
    h = np.array([side(int(l)) for l in lv], dtype=np.float64)[:, None] / UNIT
    cen = an / UNIT + 0.5 * h
    assert np.array_equal(a, np.where(cen.min(axis=1) > -0.5, 1.0, 100.0))
    assert (a == 1.0).any() and (a == 100.0).any()


def test_mf_preconditioned_cg():
    """The Sec. 4.3 problem with the "MF" preconditioner converges to the
    exact discrete solution; iteration counts stay flat under refinement."""
    its = []
    for g in (1, 2):
        f = forest_of("fichera", g, 2, "corner+random")
        coeff = gi.coeff_cells("eps", *f.leaves_arrays())
        P = problem.setup(f, 2, coeff=coeff, cheb_degree=1, smoother="jacobi")
        fn = np.ones(P.n_dofs)
        x, it, hist, ok = P.solve(fn)
        assert ok
        b = P.rhs(fn)
        assert np.linalg.norm(b - P.A @ x) <= 1.0001e-10 * np.linalg.norm(b)
        if P.n_dofs < 20000:
            u = P.exact(fn)
            assert np.linalg.norm(x - u) <= 1e-6 * np.linalg.norm(u)
        its.append(it)
    assert max(its) - min(its) <= 3, its


# ------------------------------------------------------------------ estimator of Sec. 4.3

def _nodal(d, fn):
    X = _coords(d.nk, d.leaf.keys)
    return fn(*[X[:, a] for a in range(d.forest.dim)])


@pytest.mark.parametrize("coarse,g,cycles,marker,k", [
    ("fichera", 1, 2, "corner+random", 2), ("fichera", 1, 1, "corner+random", 3),
    ("lshape", 2, 2, "corner", 2), ("cube", 2, 1, "corner", 4)])
def test_estimator_vanishes_for_solutions_in_vh(coarse, g, cycles, marker, k):
    """For u a global Q_k polynomial (so u_h = u, smooth: no flux jumps, also
    across refinement faces with hanging nodes), constant eps and
    f = -eps Laplace u (in Q_k: f_h = f), every e(K) vanishes."""
    from oracle.estimate import estimate
    f = forest_of(coarse, g, cycles, marker)
    d = discretize(f, k)
    assert len(d.leaf.hkeys) > 0
    dim = f.dim
    p = lambda x: 1.0 + 0.5 * x + 0.25 * x ** 2                  # noqa: E731
    pp = lambda x: 0.5 + 0.0 * x                                 # noqa: E731
    u = _nodal(d, lambda *x: np.prod([p(t) for t in x], axis=0))
    lap = _nodal(d, lambda *x: sum(pp(x[a]) * np.prod([p(x[b]) for b in range(dim) if b != a], axis=0)
                                   for a in range(dim)))
    eps = np.full(len(f.leaves), 3.0)
    e = estimate(d, u, -3.0 * lap, eps)
    e_ref = estimate(d, u + 0.01 * np.sin(7 * np.arange(len(u))), -3.0 * lap, eps)
    assert np.abs(e).max() <= 1e-20 * e_ref.max()


def test_estimator_cell_term_closed_form():
    """u = x^2 (k = 2, so u_h = u), eps = 1, f = c: no flux jumps, and
    e(K) = h^2 ||c + 2||_K^2 = h^(d+2) (c + 2)^2."""
    from oracle.estimate import estimate
    f = forest_of("fichera", 1, 1, "corner+random")
    d = discretize(f, 2)
    u = _nodal(d, lambda x, y, z: x ** 2)
    c = 0.7
    e = estimate(d, u, np.full(d.leaf.n_dofs, c), np.ones(len(f.leaves)))
    h = np.array([side(cl[0]) / float(UNIT) for cl in d.leaf.cells])
    assert np.allclose(e, h ** 5 * (c + 2.0) ** 2, rtol=1e-12, atol=0)


@pytest.mark.parametrize("axis", [0, 1])
def test_estimator_face_term_closed_form(axis):
    """u = x_axis (linear, in every V_h), f = 0, eps from the Sec. 4.3
    pattern on a uniform mesh: no cell residual; across an interior face
    normal to the axis the flux jumps by eps_K - eps_N, across other faces by
    0, so e(K) = h * h^(d-1) * sum over K's interior faces normal to the axis
    of (eps_K - eps_N)^2, with eps_N at the neighbour's centre."""
    from oracle.estimate import estimate
    f = forest_of("fichera", 2)
    d = discretize(f, 2)
    lv, an = f.leaves_arrays()
    eps = gi.coeff_cells("eps", lv, an)
    u = _nodal(d, lambda x, y, z: [x, y, z][axis] + 1.0)
    e = estimate(d, u, np.zeros(d.leaf.n_dofs), eps)
    s = side(2)
    h = s / float(UNIT)
    want = np.zeros(len(lv))
    for i in range(len(lv)):
        for sg in (-1, 1):
            nb = an[i].copy()
            nb[axis] += sg * s
            if (2, tuple(int(v) for v in nb)) in f.leaves:
                en = gi.coeff_cells("eps", np.array([2], np.int8), nb[None, :])[0]
                want[i] += h * h ** 2 * (eps[i] - en) ** 2
    assert (want > 0).any()
    assert np.allclose(e, want, rtol=1e-12, atol=1e-14 * want.max())


def test_marking_fraction():
    from oracle.estimate import mark_fraction
    eta = np.array([0.5, 3.0, 1.0, 3.0, 0.1, 2.0, 2.0, 0.0, 1.5, 0.2])
    fl = mark_fraction(eta, 0.3)                  # round(3.0) = 3 largest, ties by index
    assert np.array_equal(np.nonzero(fl)[0], [1, 3, 5])
    assert mark_fraction(eta, 0.142).sum() == 1 and mark_fraction(np.ones(100)).sum() == 14
