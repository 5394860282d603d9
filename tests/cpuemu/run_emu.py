"""Run the library's kernels in the CPU emulation (AddressSanitizer build)
on a small seeded case and compare with the oracle.  Invoked by
tests/test_cpu_emulation.py in a subprocess with libasan preloaded; prints
one JSON line.  Usage: run_emu.py <case> <precision> [checks]"""
import ctypes as C
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import gmg_inputs as gi  # noqa: E402
from helpers import CASES, oracle_problem  # noqa: E402
from paper_1904_03317_amd import gmg  # noqa: E402

L = gmg.configure(C.CDLL(os.path.join(HERE, "_build", "libgmg_emu.so")))


def check(code):
    if code < 0:
        raise RuntimeError(f"error {code}: {L.gmg_last_error().decode()}")
    return code


def ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def array(P, which, level, dtype):
    p, n = C.c_void_p(), C.c_int64()
    check(L.gmg_problem_array(P, which, level, C.byref(p), C.byref(n)))
    if n.value == 0:
        return np.zeros(0, dtype)
    buf = (C.c_char * (n.value * np.dtype(dtype).itemsize)).from_address(p.value)
    return np.frombuffer(buf, dtype=dtype).copy()


def rel(a, b):
    """Relative difference; absolute where the reference is zero (meshes
    without free DoFs)."""
    d = float(np.linalg.norm(np.asarray(a, np.float64) - b))
    nb = float(np.linalg.norm(b))
    return d / nb if nb > 0 else d


def aligned(nbytes):
    raw = np.zeros(nbytes + 512, np.uint8)
    off = (-raw.ctypes.data) % 256
    return raw, raw[off:off + nbytes]


def emu_request_mesh(r):
    """A small serving request mesh (unit cube, 2 global refinements, then
    toward the request's seeded point up to about 900 DoFs)."""
    spec = gi.request_spec(r)
    spec.g0, spec.target_dofs = 2, 900.0

    def create(d, o):
        m = C.c_void_p()
        o = np.ascontiguousarray(o, dtype=np.int32)
        check(L.gmg_mesh_create(d, len(o), ptr(o), C.byref(m)))
        return m

    def leaves(m):
        n = C.c_int64()
        check(L.gmg_mesh_num_leaves(m, C.byref(n)))
        lv = np.zeros(n.value, np.int8)
        an = np.zeros((n.value, 3), np.int64)
        check(L.gmg_mesh_leaves(m, ptr(lv), ptr(an)))
        return lv, an

    def refine(m, f):
        check(L.gmg_mesh_refine(m, ptr(np.ascontiguousarray(f, np.uint8)), None))

    return gi.build_request_mesh(spec, create, refine, leaves)


def serve_check(prec):
    """Serving loop in the emulation: two requests through two slots, held
    until both are set up so that their V-cycles run batched, three CG
    iterations each (the scheduler's batched tick,
    staging and launch tables under the address checks), against the solo
    solves.  The emulated threads of a block add into LDS in no fixed order,
    so the comparison allows rounding differences."""
    opts = gmg.gmg_options()
    L.gmg_options_default(C.byref(opts))
    opts.degree, opts.mg_precision, opts.max_iter = 2, prec, 3
    reqs = [0, 1]
    solo = {}
    for r in reqs:
        m = emu_request_mesh(r)
        P = C.c_void_p()
        check(L.gmg_problem_create(m, C.byref(opts), None, C.byref(P)))
        nb = C.c_size_t()
        check(L.gmg_problem_workspace_bytes(P, C.byref(nb)))
        raw, ws = aligned(nb.value)
        check(L.gmg_problem_bind(P, ptr(ws), nb.value, None))
        info = gmg.gmg_info()
        check(L.gmg_problem_info(P, C.byref(info)))
        f = np.ones(info.n_dofs)
        u = np.zeros(info.n_dofs)
        its = C.c_int32()
        st = check(L.gmg_solve(P, ptr(f), ptr(u), C.byref(its), None, None))
        solo[r] = (st, its.value, u)
        L.gmg_problem_destroy(P)
        L.gmg_mesh_destroy(m)
    araw, arena = aligned(64 << 20)
    h = C.c_void_p()
    check(L.gmg_server_create(ptr(arena), arena.nbytes, 2, 2, C.byref(h)))
    # held until both are set up, so that their iterations run together
    check(L.gmg_server_hold(h, 1))
    ids = {}
    for r in reqs:
        rid = C.c_uint64()
        check(L.gmg_server_submit(h, emu_request_mesh(r), C.byref(opts), None, None, 0, C.byref(rid)))
        ids[r] = rid.value
    st, status = C.c_int32(), C.c_int32()
    t0 = time.time()
    while True:
        states = []
        for rid in ids.values():
            check(L.gmg_server_poll(h, rid, C.byref(st), C.byref(status)))
            states.append(st.value)
        if all(x == 4 for x in states) or time.time() - t0 > 300:  # GMG_REQ_RUNNING
            break
        time.sleep(0.05)
    check(L.gmg_server_hold(h, 0))
    worst, same_its = 0.0, True
    for r, rid in ids.items():
        check(L.gmg_server_wait(h, rid, 600.0))
        n, it = C.c_int64(), C.c_int32()
        u = np.zeros(len(solo[r][2]))
        st = check(L.gmg_server_result(h, rid, ptr(u), C.byref(n), C.byref(it), None, None))
        same_its = same_its and (st, it.value) == solo[r][:2]
        worst = max(worst, float(np.abs(u - solo[r][2]).max() / np.abs(solo[r][2]).max()))
    stats = gmg.gmg_server_stats()
    check(L.gmg_server_stats(h, C.byref(stats)))
    L.gmg_server_destroy(h)
    print(json.dumps({"case": "serve", "prec": prec, "same_its": same_its, "rel": worst,
                      "batched_iterations": stats.batched_iterations, "completed": stats.completed}), flush=True)


def main():
    if sys.argv[1] == "serve":
        serve_check(int(sys.argv[2]))
        return
    case, prec = sys.argv[1], int(sys.argv[2])
    checks = sys.argv[3].split(",") if len(sys.argv) > 3 else ["leaf", "level", "vcycle", "estimate", "solve"]
    rec, k = CASES[case]
    coeff_kind = "checker" if rec.coarse == "fichera" else "one"
    op, coeff = oracle_problem(rec, k, coeff_kind=coeff_kind)
    dim, origins = gi.coarse_mesh(rec.coarse)

    def mesh(steps):
        m = C.c_void_p()
        o = np.ascontiguousarray(origins, dtype=np.int32)
        check(L.gmg_mesh_create(dim, len(o), ptr(o), C.byref(m)))
        for step in range(steps):
            n = C.c_int64()
            check(L.gmg_mesh_num_leaves(m, C.byref(n)))
            lv = np.zeros(n.value, np.int8)
            an = np.zeros((n.value, dim), np.int64)
            check(L.gmg_mesh_leaves(m, ptr(lv), ptr(an)))
            f = np.ascontiguousarray(rec.flags(step, lv, an), dtype=np.uint8)
            check(L.gmg_mesh_refine(m, ptr(f), None))
        return m

    opts = gmg.gmg_options()
    L.gmg_options_default(C.byref(opts))
    opts.degree, opts.mg_precision = k, prec
    keep = []

    def problem(m, c):
        P = C.c_void_p()
        check(L.gmg_problem_create(m, C.byref(opts), None if c is None else ptr(c), C.byref(P)))
        nb = C.c_size_t()
        check(L.gmg_problem_workspace_bytes(P, C.byref(nb)))
        raw, ws = aligned(nb.value)
        keep.append(raw)
        check(L.gmg_problem_bind(P, ptr(ws), nb.value, None))
        return P

    m = mesh(rec.steps)
    c = None if coeff is None else np.ascontiguousarray(coeff, np.float64)
    P = problem(m, c)
    out = {"case": case, "prec": prec, "N": op.n_dofs}
    info = gmg.gmg_info()
    check(L.gmg_problem_info(P, C.byref(info)))
    # levels >= 1 only (a mesh without refinement has none)
    out["lam_rel"] = max((abs(info.lambda_max[l] - op.mg.lam[l]) / op.mg.lam[l] for l in range(1, info.n_levels)),
                         default=0.0)
    rng = np.random.default_rng(5)
    N = op.n_dofs
    if "leaf" in checks:
        x = rng.standard_normal(N)
        x[~op.free] = 0
        y = np.zeros(N)
        check(L.gmg_apply_leaf(P, ptr(x), ptr(y), None))
        ref = op.A @ x
        out["leaf_rel"] = rel(y, ref)
        fn = 1.0 + rng.standard_normal(N)
        b = np.zeros(N)
        check(L.gmg_rhs(P, ptr(fn), ptr(b), None))
        rb = op.rhs(fn)
        out["rhs_rel"] = rel(b, rb)
    if "level" in checks:
        from oracle.assemble import level_coefficients, level_matrix
        lc = level_coefficients(op.disc, op.coeff)
        worst = worst_edge = 0.0
        dt = np.float64 if prec == 64 else np.float32
        for l, lev in enumerate(op.disc.levels):
            A = level_matrix(op.disc, l, lc[l]).tocsr()
            perm = array(P, gmg.ARR["LEVEL_PERM"], l, np.int32)
            assert np.array_equal(np.sort(perm), np.arange(lev.n_dofs))
            x = rng.standard_normal(lev.n_dofs).astype(dt)
            xd = np.zeros_like(x)
            xd[perm] = x
            yd = np.zeros(lev.n_dofs, dt)
            check(L.gmg_apply_level(P, l, 0, ptr(xd), ptr(yd), None))
            ref = A @ x.astype(np.float64)
            worst = max(worst, float(np.linalg.norm(yd[perm] - ref) / max(np.linalg.norm(ref), 1e-300)))
            S, I = lev.flags == 0, lev.flags == 1
            want = np.zeros(lev.n_dofs)
            want[S] = A[S][:, I] @ x.astype(np.float64)[I]
            check(L.gmg_apply_level(P, l, 1, ptr(xd), ptr(yd), None))
            got = yd[perm].astype(np.float64)
            if np.linalg.norm(want) > 0:
                worst_edge = max(worst_edge, float(np.linalg.norm(got - want) / np.linalg.norm(want)))
            else:
                worst_edge = max(worst_edge, float(np.abs(got).max()))
        out["level_rel"] = worst
        out["edge_rel"] = worst_edge
    if "vcycle" in checks:
        r = rng.standard_normal(N)
        r[~op.free] = 0
        z = np.zeros(N)
        check(L.gmg_vcycle(P, ptr(r), ptr(z), None))
        zr = op.mg.vcycle(r)
        out["vcycle_rel"] = rel(z, zr)
        # the same V-cycle with its work memory in the fixed scratch array,
        # twice (the second call finds the first call's contents)
        z2 = np.full(N, np.nan)
        check(L.gmg_vcycle_noalloc(P, ptr(r), ptr(z2), None))
        eq = bool(np.array_equal(z2, z))
        z2[:] = np.nan
        check(L.gmg_vcycle_noalloc(P, ptr(r), ptr(z2), None))
        out["noalloc_equal"] = eq and bool(np.array_equal(z2, z))
        # batched V-cycle of this problem and one on a mesh with fewer
        # refinement steps (constant coefficient): each result bit for bit
        # that of its own V-cycle
        m2 = mesh(max(rec.steps - 1, 0))
        P2 = problem(m2, None)
        info2 = gmg.gmg_info()
        check(L.gmg_problem_info(P2, C.byref(info2)))
        n2 = info2.n_dofs
        r2 = rng.standard_normal(n2)
        r2[array(P2, gmg.ARR["LEAF_DIRICHLET"], 0, np.uint8) != 0] = 0
        zb2 = np.zeros(n2)
        check(L.gmg_vcycle(P2, ptr(r2), ptr(zb2), None))
        ph = (C.c_void_p * 2)(P.value, P2.value)
        rp = (C.c_void_p * 2)(r.ctypes.data, r2.ctypes.data)
        za, zb = np.full(N, np.nan), np.full(n2, np.nan)
        zp = (C.c_void_p * 2)(za.ctypes.data, zb.ctypes.data)
        need = C.c_size_t(0)
        check(L.gmg_vcycle_batch(ph, 2, rp, zp, None, C.byref(need), None))
        traw, tab = aligned(need.value)
        cap = C.c_size_t(need.value)
        check(L.gmg_vcycle_batch(ph, 2, rp, zp, ptr(tab), C.byref(cap), None))
        out["batch_equal"] = bool(np.array_equal(za, z)) and bool(np.array_equal(zb, zb2))
        L.gmg_problem_destroy(P2)
        L.gmg_mesh_destroy(m2)
    if "estimate" in checks:
        # error estimator and marking (Sec. 4.3) against the oracle's, on a
        # random u (hanging values from the constraints) and a nodal f
        from oracle.estimate import estimate, mark_fraction
        u = rng.standard_normal(N)
        u[~op.free] = 0
        fn = 1.0 + rng.standard_normal(N)
        eps = np.asarray(op.coeff, np.float64)
        ref = estimate(op.disc, u, fn, eps)
        nb = C.c_size_t()
        check(L.gmg_estimator_workspace_bytes(P, C.byref(nb)))
        wraw, ws = aligned(nb.value)
        eta = np.full(len(ref), np.nan)
        for _ in range(2):  # the second call reuses the uploaded tables
            check(L.gmg_estimate(P, ptr(u), ptr(fn), ptr(ws), nb.value, ptr(eta), None))
        out["est_rel"] = float(np.abs(eta - ref).max() / max(np.abs(ref).max(), 1e-300))
        flags = np.zeros(len(ref), np.uint8)
        check(L.gmg_mark(P, ptr(eta), 0.142, ptr(flags), ptr(ws), nb.value, None))
        out["mark_equal"] = bool(np.array_equal(flags, mark_fraction(eta, 0.142)))
    if "solve" in checks:
        fn = gi.rhs_nodal("noise", N)
        x, it, hist, ok = op.solve(fn)
        u = np.zeros(N)
        its = C.c_int32()
        h = np.zeros(opts.max_iter + 1)
        st = check(L.gmg_solve(P, ptr(fn), ptr(u), C.byref(its), ptr(h), None))
        out.update(status=st, its=its.value, its_oracle=it,
                   solve_rel=rel(u, x))
    L.gmg_problem_destroy(P)
    L.gmg_mesh_destroy(m)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
