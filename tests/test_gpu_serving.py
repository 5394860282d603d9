"""Serving loop on the GPU: requests on different adaptive meshes resident
together give the same result as alone (bitwise: every kernel is
deterministic), admission respects the memory budget, failures are reported
per request."""
import numpy as np
import pytest

import gmg_inputs as gi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _mesh(r, scale=1.0):
    from paper_1904_03317_amd import gmg
    spec = gi.request_spec(r)
    spec.target_dofs = min(spec.target_dofs, 6e4) * scale
    return gi.build_request_mesh(spec, lambda d, o: gmg.Mesh(d, o), lambda m, f: m.refine(f),
                                 lambda m: m.leaves())


def _alone(r, opts):
    from paper_1904_03317_amd import gmg
    m = _mesh(r)
    P = gmg.Problem(m, opts).bind()
    n = P.n_dofs
    u = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, its, h = P.solve(torch.ones(n, dtype=torch.float64, device="cuda"), u)
    torch.cuda.synchronize()
    return st, its, u.cpu().numpy()


def test_mixed_equals_alone():
    from paper_1904_03317_amd import gmg
    opts = gmg.options(degree=2, mg_precision=32)
    ids = list(range(8))
    S = gmg.Server(arena_bytes=1 << 30, max_slots=3, host_threads=3)
    rids = {S.submit(_mesh(r), opts): r for r in ids}
    for rid in rids:
        S.wait(rid, 300)
    st = S.stats()
    assert st["completed"] == len(ids) and st["failed"] == 0 and st["arena_used"] == 0
    for rid, r in rids.items():
        res = S.result(rid)
        s0, its0, u0 = _alone(r, opts)
        print(f"[gpu] request {r}: N={len(u0)} its {res['iterations']} alone {its0}", flush=True)
        assert res["status"] == 0 and s0 == 0
        assert res["iterations"] == its0
        assert np.array_equal(res["u"], u0)
        t = res["timing"]
        assert t["arrival"] <= t["setup_done"] <= t["admitted"] <= t["bound"] <= t["finished"]
        S.release(rid)
    S.close()


def test_budget_rejection_and_small_arena_serialises():
    from paper_1904_03317_amd import gmg
    opts = gmg.options(degree=2, mg_precision=32)
    S = gmg.Server(arena_bytes=1 << 20, max_slots=2, host_threads=1)
    rid = S.submit(_mesh(3), opts)
    S.wait(rid, 120)
    state, status = S.poll(rid)
    assert state == "FAILED" and status == -4
    with pytest.raises(gmg.GMGError):
        S.result(rid)
    S.close()
    # an arena that holds one request at a time still completes them all
    m = _mesh(1)
    P = gmg.Problem(m, opts)
    need = P.workspace_bytes() + 2 * (P.n_dofs * 8 + 256)
    S = gmg.Server(arena_bytes=int(need * 1.5) + 4096, max_slots=4, host_threads=2)
    rids = [S.submit(_mesh(1), opts) for _ in range(3)]
    for rid in rids:
        S.wait(rid, 300)
    us = [S.result(rid)["u"] for rid in rids]
    assert all(np.array_equal(us[0], u) for u in us[1:])
    assert S.stats()["arena_peak"] <= S.stats()["arena_bytes"]
    S.close()


def test_not_converged_reported_per_request():
    from paper_1904_03317_amd import gmg
    S = gmg.Server(arena_bytes=1 << 30, max_slots=2, host_threads=2)
    a = S.submit(_mesh(2), gmg.options(degree=2, max_iter=2))
    b = S.submit(_mesh(2), gmg.options(degree=2))
    S.wait(a, 120)
    S.wait(b, 120)
    ra, rb = S.result(a), S.result(b)
    assert ra["status"] == gmg.GMG_NOT_CONVERGED and ra["iterations"] == 2
    assert rb["status"] == 0 and rb["history"][-1] <= 1e-10
    S.close()
