"""GPU parity at sizes that span many workgroups and take the chunked
parallel paths of the host set-up: FP64 solves (FP64 V-cycle in FP64 CG)
through the C ABI against the oracle's CG iterate on the same seeded inputs,
with equal iteration counts and a relative solution difference of at most
1e-10 in the 2-norm and entry by entry against the largest entry.  Meshes:
the 2D L-shape Q1 workload (5 global refinements + 3 corner cycles), the 3D
Fichera Q2 workload with noisy right-hand side at 2 global refinements, the
Q3 checkerboard-coefficient Fichera workload at 2 global refinements, and
four requests of the serving stream (unit cube, Q2, refined toward a seeded
point), capped in size so that the oracle finishes in seconds."""
import numpy as np
import pytest

import gmg_inputs as gi
from oracle import problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _close(a, b, tol):
    d = a - b
    return (np.linalg.norm(d) <= tol * np.linalg.norm(b)) and (np.abs(d).max() <= tol * np.abs(b).max())


def _solve_both(forest_oracle, mesh_lib, k, rhs, coeff_kind, label, cheb_degree=4):
    from paper_1904_03317_amd import gmg
    coeff_o = gi.coeff_cells(coeff_kind, *forest_oracle.leaves_arrays()) if coeff_kind != "one" else None
    op = problem.setup(forest_oracle, k, coeff=coeff_o, cheb_degree=cheb_degree)
    fn = gi.rhs_nodal(rhs, op.n_dofs)
    x, it, hist, ok = op.solve(fn)
    print(f"[gpu] {label}: N={op.n_dofs} leaves={len(forest_oracle.leaves)} oracle its={it}", flush=True)
    coeff_l = gi.coeff_cells(coeff_kind, *mesh_lib.leaves()) if coeff_kind != "one" else None
    P = gmg.Problem(mesh_lib, gmg.options(degree=k, mg_precision=64, cheb_degree=cheb_degree), coeff=coeff_l).bind()
    assert P.n_dofs == op.n_dofs
    u = torch.zeros(op.n_dofs, dtype=torch.float64, device="cuda")
    st, its, h = P.solve(torch.as_tensor(fn, device="cuda"), u)
    torch.cuda.synchronize()
    uh = u.cpu().numpy()
    print(f"[gpu] {label}: gpu its={its} rel={np.linalg.norm(uh - x) / np.linalg.norm(x):.2e}", flush=True)
    assert st == 0 and ok
    assert its == it
    assert _close(uh, x, 1e-10)
    assert np.allclose(h, hist, rtol=1e-6, atol=1e-14)
    P.close()


@pytest.mark.parametrize("name,g", [("C1", None), ("C2", 2), ("C5", 2), ("A41", 1)])
def test_workload_fp64_solve_matches_oracle(name, g):
    from paper_1904_03317_amd import gmg
    w = gi.workload(name, g=g)
    _solve_both(problem.build_forest(w.recipe), gmg.build_mesh(w.recipe), w.degree, w.rhs, w.coeff,
                f"{name} g={w.recipe.globals_}", cheb_degree=w.cheb_degree)


def test_annulus_fp32_mg_solve():
    """The paper's V-cycle workload (annulus, Q2, Chebyshev degree 5, FP32
    V-cycle in FP64 CG): the FP32-MG solve reaches the tolerance with the
    true residual (leaf operator) at most 1.0001e-10 and at most one
    iteration more than the oracle's FP64 solve."""
    from paper_1904_03317_amd import gmg
    w = gi.workload("A41", g=1)
    op = problem.setup(problem.build_forest(w.recipe), w.degree, cheb_degree=w.cheb_degree)
    f = np.ones(op.n_dofs)
    x, it, hist, ok = op.solve(f)
    P = gmg.Problem(gmg.build_mesh(w.recipe), gmg.options(degree=2, mg_precision=32, cheb_degree=5)).bind()
    u = torch.zeros(op.n_dofs, dtype=torch.float64, device="cuda")
    st, its, h = P.solve(torch.as_tensor(f, device="cuda"), u)
    uh = u.cpu().numpy()
    print(f"[gpu] A41 g=1 FP32-MG: N={op.n_dofs} its {its} (oracle FP64 {it})", flush=True)
    assert st == 0 and ok and its <= it + 1
    b = op.rhs(f)
    assert np.linalg.norm(b - op.A @ uh) <= 1.0001e-10 * np.linalg.norm(b)
    assert _close(uh, x, 1e-8)
    P.close()


@pytest.mark.parametrize("r", [0, 1, 2, 3])
def test_request_fp64_solve_matches_oracle(r):
    from oracle.forest import Forest
    from paper_1904_03317_amd import gmg
    spec = gi.request_spec(r)
    spec.target_dofs = min(spec.target_dofs, 3e4)
    fo = gi.build_request_mesh(spec, lambda d, o: Forest(d, o), lambda f, fl: f.refine(fl),
                               lambda f: f.leaves_arrays())
    ml = gi.build_request_mesh(spec, lambda d, o: gmg.Mesh(d, o), lambda m, fl: m.refine(fl),
                               lambda m: m.leaves())
    _solve_both(fo, ml, 2, "one", "one", f"request {r}")


def test_leaf_operator_bitwise_repeatable():
    """The leaf operator adds the cells' results of a tile in LDS; its sums
    must come out bit for bit the same on every application and in every
    problem instance (the serving loop's mixed-equals-alone guarantee
    depends on it).  Fichera Q2 with 3 global refinements and 4 adaptive
    cycles: most leaf cells carry in-cell constraints, whose results several
    sibling cells add into the same parent nodes."""
    from paper_1904_03317_amd import gmg
    w = gi.workload("C2", g=3)
    m = gmg.build_mesh(w.recipe)
    P1 = gmg.Problem(m, gmg.options(degree=2, mg_precision=64)).bind()
    P2 = gmg.Problem(m, gmg.options(degree=2, mg_precision=64)).bind()
    n = P1.n_dofs
    print(f"[gpu] leaf repeatability: N={n}", flush=True)
    x = torch.as_tensor(np.random.default_rng(3).standard_normal(n), device="cuda")
    ref = torch.zeros(n, dtype=torch.float64, device="cuda")
    P1.apply_leaf(x, ref)
    y = torch.zeros_like(ref)
    for k in range(20):
        (P1 if k % 2 == 0 else P2).apply_leaf(x, y)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), k
    P1.close()
    P2.close()
