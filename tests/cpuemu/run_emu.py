"""Run the library's kernels in the CPU emulation (AddressSanitizer build)
on a small seeded case and compare with the oracle.  Invoked by
tests/test_cpu_emulation.py in a subprocess with libasan preloaded; prints
one JSON line.  Usage: run_emu.py <case> <precision> [checks]"""
import ctypes as C
import json
import os
import sys

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


def main():
    case, prec = sys.argv[1], int(sys.argv[2])
    checks = sys.argv[3].split(",") if len(sys.argv) > 3 else ["leaf", "level", "vcycle", "solve"]
    rec, k = CASES[case]
    coeff_kind = "checker" if rec.coarse == "fichera" else "one"
    op, coeff = oracle_problem(rec, k, coeff_kind=coeff_kind)
    dim, origins = gi.coarse_mesh(rec.coarse)
    m = C.c_void_p()
    o = np.ascontiguousarray(origins, dtype=np.int32)
    check(L.gmg_mesh_create(dim, len(o), ptr(o), C.byref(m)))
    for step in range(rec.steps):
        n = C.c_int64()
        check(L.gmg_mesh_num_leaves(m, C.byref(n)))
        lv = np.zeros(n.value, np.int8)
        an = np.zeros((n.value, dim), np.int64)
        check(L.gmg_mesh_leaves(m, ptr(lv), ptr(an)))
        f = np.ascontiguousarray(rec.flags(step, lv, an), dtype=np.uint8)
        check(L.gmg_mesh_refine(m, ptr(f), None))
    opts = gmg.gmg_options()
    L.gmg_options_default(C.byref(opts))
    opts.degree, opts.mg_precision = k, prec
    P = C.c_void_p()
    c = None if coeff is None else np.ascontiguousarray(coeff, np.float64)
    check(L.gmg_problem_create(m, C.byref(opts), None if c is None else ptr(c), C.byref(P)))
    nb = C.c_size_t()
    check(L.gmg_problem_workspace_bytes(P, C.byref(nb)))
    raw, ws = aligned(nb.value)
    check(L.gmg_problem_bind(P, ptr(ws), nb.value, None))
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
