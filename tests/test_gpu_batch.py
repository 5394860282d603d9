"""Batched V-cycle on the GPU (gmg_vcycle_batch): the level sweeps of several
resident problems of different sizes run as one launch per sweep, and each
problem's z = B r equals its own gmg_vcycle bit for bit (FP32 and FP64
levels; 2D Q1, 3D Q2 and the cooperative 3D Q3 kernels)."""
import numpy as np
import pytest

import gmg_inputs as gi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _problems(name, gs, prec):
    from paper_1904_03317_amd import gmg
    out = []
    for g in gs:
        w = gi.workload(name, g=g)
        m = gmg.build_mesh(w.recipe)
        coeff = gi.coeff_cells(w.coeff, *m.leaves()) if w.coeff != "one" else None
        out.append(gmg.Problem(m, gmg.options(degree=w.degree, mg_precision=prec), coeff=coeff).bind())
    return out


@pytest.mark.parametrize("name,gs", [("C1", [3, 5, 4]), ("C2", [2, 1, 3, 2]), ("C5", [1, 2])])
@pytest.mark.parametrize("prec", [32, 64])
def test_batched_vcycle_equals_individual(name, gs, prec):
    from paper_1904_03317_amd import gmg
    ps = _problems(name, gs, prec)
    rng = np.random.default_rng(11)
    rs, zs, ref = [], [], []
    for P in ps:
        r = rng.standard_normal(P.n_dofs)
        r[P.array("LEAF_DIRICHLET").astype(bool)] = 0
        rd = torch.as_tensor(r, device="cuda")
        z = torch.zeros_like(rd)
        P.vcycle(rd, z)
        rs.append(rd)
        ref.append(z)
        zs.append(torch.full_like(rd, float("nan")))
    torch.cuda.synchronize()
    print(f"[gpu] batch {name} FP{prec}: N={[P.n_dofs for P in ps]}", flush=True)
    table = gmg.vcycle_batch(ps, rs, zs)
    for z, zr in zip(zs, ref):
        assert torch.equal(z, zr)
    # again with the same table, results cleared, a different order
    for z in zs:
        z.fill_(float("nan"))
    order = list(reversed(range(len(ps))))
    gmg.vcycle_batch([ps[i] for i in order], [rs[i] for i in order], [zs[i] for i in order], table=table)
    for z, zr in zip(zs, ref):
        assert torch.equal(z, zr)
    for P in ps:
        P.close()


def test_batch_rejects_mixed_and_repeated_problems():
    from paper_1904_03317_amd import gmg
    a = _problems("C2", [1], 32)[0]
    b = _problems("C2", [1], 64)[0]
    r = torch.zeros(a.n_dofs, dtype=torch.float64, device="cuda")
    z = torch.zeros_like(r)
    with pytest.raises(gmg.GMGError):
        gmg.vcycle_batch([a, b], [r, r], [z, z])
    with pytest.raises(gmg.GMGError):
        gmg.vcycle_batch([a, a], [r, r], [z, z])
    a.close()
    b.close()
