"""Thin ctypes binding of the C ABI in include/gmg.h (argument marshalling
only; every step of the solver runs in the HIP library).  Device buffers are
torch tensors on the current HIP device; device work goes to the current
torch stream.  The library must be built (paper_1904_03317_amd.build); there
is no fallback."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libgmg.so")

GMG_OK, GMG_NOT_CONVERGED = 0, 1
ARR = dict(LEAF_CELLMAP=1, LEAF_DIRICHLET=2, CON_OFFSETS=3, CON_MASTERS=4, CON_WEIGHTS=5,
           COPY_LEVEL=6, COPY_INDEX=7, LEVEL_CELLMAP=8, LEVEL_FLAGS=9, LEVEL_PARENT=10,
           LEAF_CELLMAP_PARENT=11, LEAF_MASK=12, LEVEL_PERM=13)
_ARR_DTYPE = {1: np.int32, 2: np.uint8, 3: np.int64, 4: np.int32, 5: np.float64, 6: np.int8,
              7: np.int32, 8: np.int32, 9: np.uint8, 10: np.int32, 11: np.int32, 12: np.uint16,
              13: np.int32}


class gmg_options(C.Structure):
    _fields_ = [("degree", C.c_int32), ("mg_precision", C.c_int32), ("cheb_degree", C.c_int32),
                ("cheb_lo", C.c_double), ("cheb_hi", C.c_double), ("eig_iters", C.c_int32),
                ("rtol", C.c_double), ("max_iter", C.c_int32), ("use_graph", C.c_int32),
                ("op_variant", C.c_int32), ("smoother", C.c_int32), ("relax", C.c_double)]


SMOOTHER_CHEBYSHEV, SMOOTHER_JACOBI = 0, 1


class gmg_info(C.Structure):
    _fields_ = [("dim", C.c_int32), ("degree", C.c_int32), ("n_levels", C.c_int32),
                ("mg_precision", C.c_int32), ("n_dofs", C.c_int64), ("n_hanging", C.c_int64),
                ("n_leaves", C.c_int64), ("n_free", C.c_int64), ("level_dofs", C.c_int64 * 24),
                ("level_cells", C.c_int64 * 24), ("lambda_max", C.c_double * 24),
                ("workspace_bytes", C.c_size_t)]


class gmg_timing(C.Structure):
    _fields_ = [("arrival", C.c_double), ("setup_done", C.c_double), ("admitted", C.c_double),
                ("bound", C.c_double), ("finished", C.c_double)]


class gmg_server_stats(C.Structure):
    _fields_ = [("queued", C.c_int64), ("running", C.c_int64), ("completed", C.c_int64),
                ("failed", C.c_int64), ("arena_used", C.c_size_t), ("arena_peak", C.c_size_t),
                ("arena_bytes", C.c_size_t), ("dofs_done", C.c_double), ("clock", C.c_double),
                ("iterations", C.c_int64), ("batched_iterations", C.c_int64), ("batches", C.c_int64)]


REQ_STATES = ["QUEUED", "SETUP", "READY", "BINDING", "RUNNING", "DONE", "FAILED", "WAIT_RHS"]
RHS_LATER = -1


class GMGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gmg error {code}: {msg}")
        self.code = code


_lib = None


def configure(L):
    """Set the ctypes signatures of every exported function on a loaded library."""
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "gmg_options_default": (None, [C.POINTER(gmg_options)]),
        "gmg_last_error": (C.c_char_p, []),
        "gmg_mesh_create": (C.c_int, [C.c_int, C.c_int, vp, C.POINTER(vp)]),
        "gmg_mesh_refine": (C.c_int, [vp, vp, C.POINTER(i64)]),
        "gmg_mesh_num_leaves": (C.c_int, [vp, C.POINTER(i64)]),
        "gmg_mesh_leaves": (C.c_int, [vp, vp, vp]),
        "gmg_mesh_dim": (C.c_int, [vp, C.POINTER(C.c_int)]),
        "gmg_mesh_destroy": (C.c_int, [vp]),
        "gmg_problem_create": (C.c_int, [vp, C.POINTER(gmg_options), vp, C.POINTER(vp)]),
        "gmg_problem_info": (C.c_int, [vp, C.POINTER(gmg_info)]),
        "gmg_problem_clone": (C.c_int, [vp, C.POINTER(gmg_options), C.POINTER(vp)]),
        "gmg_problem_array": (C.c_int, [vp, C.c_int, C.c_int, C.POINTER(vp), C.POINTER(i64)]),
        "gmg_problem_workspace_bytes": (C.c_int, [vp, C.POINTER(C.c_size_t)]),
        "gmg_problem_bind": (C.c_int, [vp, vp, C.c_size_t, vp]),
        "gmg_problem_destroy": (C.c_int, [vp]),
        "gmg_rhs": (C.c_int, [vp, vp, vp, vp]),
        "gmg_solve": (C.c_int, [vp, vp, vp, C.POINTER(i32), vp, vp]),
        "gmg_solve_rhs": (C.c_int, [vp, vp, vp, C.POINTER(i32), vp, vp]),
        "gmg_apply_leaf": (C.c_int, [vp, vp, vp, vp]),
        "gmg_apply_level": (C.c_int, [vp, C.c_int, C.c_int, vp, vp, vp]),
        "gmg_vcycle": (C.c_int, [vp, vp, vp, vp]),
        "gmg_vcycle_noalloc": (C.c_int, [vp, vp, vp, vp]),
        "gmg_vcycle_batch": (C.c_int, [vp, C.c_int, vp, vp, vp, C.POINTER(C.c_size_t), vp]),
        "gmg_estimator_workspace_bytes": (C.c_int, [vp, C.POINTER(C.c_size_t)]),
        "gmg_estimate": (C.c_int, [vp, vp, vp, vp, C.c_size_t, vp, vp]),
        "gmg_mark": (C.c_int, [vp, vp, C.c_double, vp, vp, C.c_size_t, vp]),
        "gmg_problem_last_timing": (C.c_int, [vp, C.POINTER(dbl)]),
        "gmg_server_create": (C.c_int, [vp, C.c_size_t, i32, i32, C.POINTER(vp)]),
        "gmg_server_submit": (C.c_int, [vp, vp, C.POINTER(gmg_options), vp, vp, i64, C.POINTER(C.c_uint64)]),
        "gmg_server_request_dofs": (C.c_int, [vp, C.c_uint64, C.POINTER(i64)]),
        "gmg_server_set_rhs": (C.c_int, [vp, C.c_uint64, vp, i64]),
        "gmg_server_poll": (C.c_int, [vp, C.c_uint64, C.POINTER(i32), C.POINTER(i32)]),
        "gmg_server_wait": (C.c_int, [vp, C.c_uint64, dbl]),
        "gmg_server_result": (C.c_int, [vp, C.c_uint64, vp, C.POINTER(i64), C.POINTER(i32), vp,
                                        C.POINTER(gmg_timing)]),
        "gmg_server_release": (C.c_int, [vp, C.c_uint64]),
        "gmg_server_stats": (C.c_int, [vp, C.POINTER(gmg_server_stats)]),
        "gmg_server_destroy": (C.c_int, [vp]),
        "gmg_server_set_batching": (C.c_int, [vp, i32]),
        "gmg_server_hold": (C.c_int, [vp, i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run paper_1904_03317_amd.build)")
    try:  # share torch's HIP runtime when torch is present
        import torch  # noqa: F401
    except Exception:
        pass
    L = C.CDLL(LIB_PATH)
    configure(L)
    _lib = L
    return L


def exported_symbols():
    """Names the library must export (every function of include/gmg.h)."""
    return ["gmg_options_default", "gmg_last_error", "gmg_mesh_create", "gmg_mesh_refine",
            "gmg_mesh_num_leaves", "gmg_mesh_leaves", "gmg_mesh_dim", "gmg_mesh_destroy",
            "gmg_problem_create", "gmg_problem_clone", "gmg_problem_info", "gmg_problem_array",
            "gmg_problem_workspace_bytes", "gmg_problem_bind", "gmg_problem_destroy", "gmg_rhs",
            "gmg_solve", "gmg_solve_rhs", "gmg_apply_leaf", "gmg_apply_level", "gmg_vcycle", "gmg_vcycle_noalloc", "gmg_vcycle_batch",
            "gmg_estimator_workspace_bytes", "gmg_estimate", "gmg_mark",
            "gmg_problem_last_timing", "gmg_server_create", "gmg_server_submit", "gmg_server_request_dofs",
            "gmg_server_set_rhs", "gmg_server_poll",
            "gmg_server_wait", "gmg_server_result", "gmg_server_release", "gmg_server_stats",
            "gmg_server_destroy", "gmg_server_set_batching", "gmg_server_hold"]


def _check(code):
    if code < 0:
        raise GMGError(code, lib().gmg_last_error().decode())
    return code


def options(**kw):
    o = gmg_options()
    lib().gmg_options_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def vcycle_batch(problems, rs, zs, table=None, stream=None):
    """gmg_vcycle_batch: one V-cycle per problem, level sweeps batched.  rs,
    zs: device tensors; table: a device uint8 tensor for the launch tables
    (allocated here when None).  Returns the table."""
    import torch
    n = len(problems)
    ph = (C.c_void_p * n)(*[p.h.value for p in problems])
    rp = (C.c_void_p * n)(*[r.data_ptr() for r in rs])
    zp = (C.c_void_p * n)(*[z.data_ptr() for z in zs])
    need = C.c_size_t(0)
    _check(lib().gmg_vcycle_batch(ph, n, rp, zp, None, C.byref(need), _stream(stream)))
    if table is None or table.numel() < need.value:
        table = torch.empty(need.value, dtype=torch.uint8, device=rs[0].device)
    cap = C.c_size_t(table.numel())
    _check(lib().gmg_vcycle_batch(ph, n, rp, zp, _ptr(table), C.byref(cap), _stream(stream)))
    return table


class Mesh:
    """Forest of quad/hex trees (gmg_mesh_*)."""

    def __init__(self, dim, origins):
        o = np.ascontiguousarray(np.asarray(origins, dtype=np.int32).reshape(-1, dim))
        h = C.c_void_p()
        _check(lib().gmg_mesh_create(dim, o.shape[0], _ptr(o), C.byref(h)))
        self.h, self.dim = h, dim

    def refine(self, flags):
        f = np.ascontiguousarray(np.asarray(flags, dtype=np.uint8))
        if len(f) != self.n_leaves:
            raise ValueError("one flag per leaf")
        n = C.c_int64()
        _check(lib().gmg_mesh_refine(self.h, _ptr(f), C.byref(n)))
        return n.value

    @property
    def n_leaves(self):
        n = C.c_int64()
        _check(lib().gmg_mesh_num_leaves(self.h, C.byref(n)))
        return n.value

    def leaves(self):
        n = self.n_leaves
        lv = np.zeros(n, np.int8)
        an = np.zeros((n, self.dim), np.int64)
        _check(lib().gmg_mesh_leaves(self.h, _ptr(lv), _ptr(an)))
        return lv, an

    def close(self):
        if self.h:
            lib().gmg_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """Discretisation + multigrid hierarchy of one mesh (gmg_problem_*)."""

    def __init__(self, mesh: Mesh, opts=None, coeff=None, _handle=None):
        self.opts = opts if opts is not None else options()
        self.ws = None
        if _handle is not None:
            self.h = _handle
            return
        c = None if coeff is None else np.ascontiguousarray(np.asarray(coeff, np.float64))
        h = C.c_void_p()
        _check(lib().gmg_problem_create(mesh.h, C.byref(self.opts), _ptr(c), C.byref(h)))
        self.h = h

    def clone(self, opts):
        """Same host set-up, other options (gmg_problem_clone)."""
        h = C.c_void_p()
        _check(lib().gmg_problem_clone(self.h, C.byref(opts), C.byref(h)))
        return Problem(None, opts, _handle=h)

    def info(self):
        i = gmg_info()
        _check(lib().gmg_problem_info(self.h, C.byref(i)))
        return i

    @property
    def n_dofs(self):
        return self.info().n_dofs

    def array(self, name, level=0):
        which = ARR[name]
        p, n = C.c_void_p(), C.c_int64()
        _check(lib().gmg_problem_array(self.h, which, level, C.byref(p), C.byref(n)))
        dt = np.dtype(_ARR_DTYPE[which])
        if n.value == 0:
            return np.zeros(0, dt)
        buf = (C.c_char * (n.value * dt.itemsize)).from_address(p.value)
        return np.frombuffer(buf, dtype=dt).copy()

    def workspace_bytes(self):
        b = C.c_size_t()
        _check(lib().gmg_problem_workspace_bytes(self.h, C.byref(b)))
        return b.value

    def bind(self, device="cuda", workspace=None, stream=None):
        import torch
        nb = self.workspace_bytes()
        if workspace is None:
            workspace = torch.empty(nb, dtype=torch.uint8, device=device)
        self.ws = workspace
        _check(lib().gmg_problem_bind(self.h, _ptr(workspace), workspace.numel(), _stream(stream)))
        return self

    def rhs(self, f, b, stream=None):
        _check(lib().gmg_rhs(self.h, _ptr(f), _ptr(b), _stream(stream)))

    def solve(self, f, u, stream=None, with_history=True):
        it = C.c_int32()
        hist = np.zeros(self.opts.max_iter + 1) if with_history else None
        st = _check(lib().gmg_solve(self.h, _ptr(f), _ptr(u), C.byref(it), _ptr(hist), _stream(stream)))
        return st, it.value, (hist[: it.value + 1] if hist is not None else None)

    def solve_rhs(self, b, u, stream=None):
        it = C.c_int32()
        hist = np.zeros(self.opts.max_iter + 1)
        st = _check(lib().gmg_solve_rhs(self.h, _ptr(b), _ptr(u), C.byref(it), _ptr(hist), _stream(stream)))
        return st, it.value, hist[: it.value + 1]

    def apply_leaf(self, x, y, stream=None):
        _check(lib().gmg_apply_leaf(self.h, _ptr(x), _ptr(y), _stream(stream)))

    def apply_level(self, level, variant, x, y, stream=None):
        """Level operator on level vectors in the device layout of the level
        (x_dev[perm[i]] = x[i] with perm = array("LEVEL_PERM", level))."""
        _check(lib().gmg_apply_level(self.h, level, variant, _ptr(x), _ptr(y), _stream(stream)))

    def vcycle(self, r, z, stream=None):
        _check(lib().gmg_vcycle(self.h, _ptr(r), _ptr(z), _stream(stream)))

    def estimator_workspace(self, device="cuda"):
        """device workspace of the error estimator and the marking"""
        import torch
        b = C.c_size_t()
        _check(lib().gmg_estimator_workspace_bytes(self.h, C.byref(b)))
        return torch.empty(b.value, dtype=torch.uint8, device=device)

    def estimate(self, u, f, eta, workspace, stream=None):
        """gmg_estimate: eta [n_leaves] from the solution u and the nodal f"""
        _check(lib().gmg_estimate(self.h, _ptr(u), _ptr(f), _ptr(workspace), workspace.numel(), _ptr(eta),
                                  _stream(stream)))

    def mark(self, eta, flags, workspace, fraction=0.142, stream=None):
        """gmg_mark: flags [n_leaves] uint8 of the largest fraction of eta"""
        _check(lib().gmg_mark(self.h, _ptr(eta), float(fraction), _ptr(flags), _ptr(workspace), workspace.numel(),
                              _stream(stream)))

    def vcycle_noalloc(self, r, z, stream=None):
        """gmg_vcycle with the work memory in the library's fixed scratch
        array (allocates nothing)"""
        _check(lib().gmg_vcycle_noalloc(self.h, _ptr(r), _ptr(z), _stream(stream)))

    def last_timing(self):
        out = (C.c_double * 3)()
        _check(lib().gmg_problem_last_timing(self.h, out))
        return tuple(out)

    def close(self):
        if self.h:
            lib().gmg_problem_destroy(self.h)
            self.h = None
            self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop (gmg_server_*): resident solves on one HBM arena."""

    def __init__(self, arena_bytes, max_slots=8, host_threads=4, device="cuda", batching=True):
        import torch
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        h = C.c_void_p()
        _check(lib().gmg_server_create(_ptr(self.arena), self.arena.numel(), max_slots, host_threads,
                                       C.byref(h)))
        self.h = h
        if not batching:
            _check(lib().gmg_server_set_batching(self.h, 0))

    def submit(self, mesh: Mesh, opts=None, coeff=None, f=None, rhs_later=False):
        """Queue a solve; the server takes the mesh.  f: nodal right-hand side
        in canonical leaf DoF order, or None for f = 1; rhs_later: supply it
        with set_rhs once request_dofs reports the DoF count."""
        opts = opts if opts is not None else options()
        c = None if coeff is None else np.ascontiguousarray(np.asarray(coeff, np.float64))
        fa = None if f is None else np.ascontiguousarray(np.asarray(f, np.float64))
        n_f = len(fa) if fa is not None else (RHS_LATER if rhs_later else 0)
        rid = C.c_uint64()
        _check(lib().gmg_server_submit(self.h, mesh.h, C.byref(opts), _ptr(c), _ptr(fa), n_f, C.byref(rid)))
        mesh.h = None
        return rid.value

    def request_dofs(self, rid, timeout=600.0):
        """DoF count of a request, waiting for its host set-up."""
        import time
        n = C.c_int64()
        t0 = time.perf_counter()
        while True:
            code = lib().gmg_server_request_dofs(self.h, rid, C.byref(n))
            if code == 0:
                return n.value
            if code != -8 or time.perf_counter() - t0 > timeout:
                _check(code)
                raise GMGError(-8, "timeout waiting for the host set-up of the request")
            state, status = self.poll(rid)
            if state == "FAILED":
                raise GMGError(status, "request failed")
            time.sleep(0.001)

    def set_rhs(self, rid, f):
        fa = np.ascontiguousarray(np.asarray(f, np.float64))
        _check(lib().gmg_server_set_rhs(self.h, rid, _ptr(fa), len(fa)))

    def poll(self, rid):
        st, status = C.c_int32(), C.c_int32()
        _check(lib().gmg_server_poll(self.h, rid, C.byref(st), C.byref(status)))
        return REQ_STATES[st.value], status.value

    def wait(self, rid, timeout=600.0):
        _check(lib().gmg_server_wait(self.h, rid, float(timeout)))

    def result(self, rid, max_iter=100):
        n = C.c_int64()
        it = C.c_int32()
        t = gmg_timing()
        code = lib().gmg_server_result(self.h, rid, None, C.byref(n), C.byref(it), None, C.byref(t))
        _check(code)
        u = np.zeros(n.value)
        hist = np.zeros(max(max_iter, it.value) + 1)
        code = _check(lib().gmg_server_result(self.h, rid, _ptr(u), C.byref(n), C.byref(it), _ptr(hist),
                                              C.byref(t)))
        return dict(status=code, u=u, iterations=it.value, history=hist[: it.value + 1],
                    timing={f: getattr(t, f) for f, _ in gmg_timing._fields_})

    def release(self, rid):
        _check(lib().gmg_server_release(self.h, rid))

    def hold(self, on=True):
        """Stop (True) or resume (False) advancing the resident solves."""
        _check(lib().gmg_server_hold(self.h, 1 if on else 0))

    def stats(self):
        s = gmg_server_stats()
        _check(lib().gmg_server_stats(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in gmg_server_stats._fields_}

    def close(self):
        if self.h:
            lib().gmg_server_destroy(self.h)
            self.h = None
            self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_mesh(recipe):
    """Run a gmg_inputs recipe through the library forest."""
    import gmg_inputs as gi

    def create(dim, origins):
        return Mesh(dim, origins)

    def refine(m, flags):
        m.refine(flags)

    def leaves(m):
        return m.leaves()

    return gi.build_mesh(recipe, create, refine, leaves)
