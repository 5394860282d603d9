"""Smoother, V-cycle and CG (Alg. 1, Alg. 2, Sec. 2.3 local smoothing,
Sec. 4.1 solver parameters, Sec. 1/4.3 CG with a multigrid preconditioner).

Readings of the paper used here:
* Smoother: Chebyshev iteration over point Jacobi, damping the eigenvalue
  range [0.08, 1.2] * lambda_max of D^{-1} A^S (Sec. 4.1), written as the
  standard Chebyshev semi-iteration (three-term recurrence).  One smoothing
  call does m steps; the first step from a zero start needs no product.
* lambda_max: 10 Jacobi-preconditioned CG steps on A^S from the start vector
  (i mod 12) - 5.5 on the S rows (i = level DoF index), largest eigenvalue of
  the Lanczos tridiagonal matrix built from the CG coefficients.
* The "MF" smoother of Sec. 4.3 (one Jacobi step without damping): m steps
  of x += omega D^{-1} (g - A x) on V^S, omega = 1; from a zero start the
  first step needs no product.
* Coarse solve: exact, by a dense Cholesky factorisation of A_0^S.
* CG: x0 = 0, stop when ||r_k||_2 <= rtol ||b||_2 (unpreconditioned,
  recursively updated residual).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .assemble import level_coefficients, level_matrix, leaf_matrices, transfer_matrix
from .dofs import FLAG_D, FLAG_I, FLAG_S, number_active
from .forest import side
from .basis import lagrange


def lanczos_lambda_max(A, dinv, b, iters):
    """Largest Ritz value of D^{-1}A after `iters` Jacobi-PCG steps from x=0."""
    n = len(b)
    iters = min(iters, n)
    if iters == 0:
        return 1.0
    r = b.astype(np.float64).copy()
    z = dinv * r
    p = z.copy()
    rho = float(r @ z)
    alphas, betas = [], []
    for j in range(iters):
        if rho <= 0.0:
            break
        q = A @ p
        pq = float(p @ q)
        if pq <= 0.0:
            break
        alpha = rho / pq
        alphas.append(alpha)
        if j == iters - 1:
            break
        r -= alpha * q
        z = dinv * r
        rho_new = float(r @ z)
        if rho_new <= 0.0:
            break
        beta = rho_new / rho
        betas.append(beta)
        p = z + beta * p
        rho = rho_new
    m = len(alphas)
    if m == 0:
        return 1.0
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = math.sqrt(betas[j]) / alphas[j]
    return float(np.linalg.eigvalsh(T).max())


def chebyshev(A, dinv, g, lam, m, x0=None, lo=0.08, hi=1.2):
    """m steps of Chebyshev-Jacobi for A x = g on [lo*lam, hi*lam].  With
    x0=None the start is zero and the first step needs no product."""
    a, b = lo * lam, hi * lam
    theta, delta = 0.5 * (b + a), 0.5 * (b - a)
    sigma = theta / delta
    rho_old = 1.0 / sigma
    if x0 is None:
        d = dinv * g / theta
        x = d.copy()
    else:
        x = x0.copy()
        d = dinv * (g - A @ x) / theta
        x = x + d
    for _ in range(2, m + 1):
        t = A @ x
        rho = 1.0 / (2.0 * sigma - rho_old)
        d = (rho * rho_old) * d + (2.0 * rho / delta) * (dinv * (g - t))
        x = x + d
        rho_old = rho
    return x


def jacobi(A, dinv, g, omega, m, x0=None):
    """m steps of point Jacobi with relaxation omega for A x = g (Sec. 4.3
    smoother: omega = 1, one step).  With x0=None the start is zero."""
    if x0 is None:
        x = omega * (dinv * g)
        first = 2
    else:
        x = x0.copy()
        first = 1
    for _ in range(first, m + 1):
        x = x + omega * (dinv * (g - A @ x))
    return x


class LevelOps:
    def __init__(self, lev, Ahat, dtype):
        S = np.nonzero(lev.flags == FLAG_S)[0]
        I = np.nonzero(lev.flags == FLAG_I)[0]
        self.S, self.I, self.n = S, I, lev.n_dofs
        Ahat = Ahat.tocsr()
        self.A_S = Ahat[S][:, S].tocsr().astype(dtype)
        self.A_IS = Ahat[I][:, S].tocsr().astype(dtype)
        self.A_SI = Ahat[S][:, I].tocsr().astype(dtype)
        diag = Ahat.diagonal()[S]
        self.dinv = (1.0 / diag).astype(dtype) if len(S) else np.zeros(0, dtype)
        self.free = lev.flags != FLAG_D


class LocalSmoothingMG:
    """The V-cycle of Alg. 2 with local smoothing, in the storage-efficient
    form of Sec. 2.3: level vectors live on level-l cells only, the smoother
    acts on V^S, the interface part enters the residual through A^{IS} and the
    post-smoothing right-hand side through A^{SI}; leaf residuals enter the
    hierarchy on the coarsest level that holds them as S nodes."""

    def __init__(self, disc, coeff, cheb_degree=4, lo=0.08, hi=1.2, eig_iters=10,
                 dtype=np.float64, smoother="chebyshev", relax=1.0):
        self.disc, self.m, self.lo, self.hi, self.dtype = disc, cheb_degree, lo, hi, dtype
        assert smoother in ("chebyshev", "jacobi")
        self.smoother, self.relax = smoother, relax
        lcoeff = level_coefficients(disc, coeff)
        self.ops, self.lam, self.P = [], [], [None]
        for l, lev in enumerate(disc.levels):
            Ahat = level_matrix(disc, l, lcoeff[l])
            ops = LevelOps(lev, Ahat, dtype)
            A64 = Ahat.tocsr()[ops.S][:, ops.S].tocsr()
            v = (ops.S % 12).astype(np.float64) - 5.5
            d64 = (1.0 / A64.diagonal()) if len(ops.S) else np.zeros(0)
            self.lam.append(lanczos_lambda_max(A64, d64, v, eig_iters) if l > 0 else 1.0)
            self.ops.append(ops)
            if l >= 1:
                self.P.append(transfer_matrix(disc, l).astype(dtype))
        o0 = self.ops[0]
        self.n0 = len(o0.S)
        if self.n0:
            A0 = level_matrix(disc, 0, lcoeff[0]).tocsr()[o0.S][:, o0.S].toarray()
            self.chol = sla.cho_factor(A0)
        self.R = [None] + [P.T.tocsr() for P in self.P[1:]]
        self.copy_level, self.copy_index = disc.copy_level, disc.copy_index
        self.leaf_free = disc.leaf.dirichlet == 0

    def smooth(self, l, A, dinv, g, x0=None):
        """m smoothing steps on level l (V^S rows), from zero or from x0."""
        if self.smoother == "jacobi":
            return jacobi(A, dinv, g, self.dtype(self.relax), self.m, x0=x0)
        return chebyshev(A, dinv, g, self.lam[l], self.m, x0=x0, lo=self.lo, hi=self.hi)

    def vcycle(self, r):
        dt = self.dtype
        L = len(self.ops) - 1
        d = [np.zeros(o.n, dtype=dt) for o in self.ops]
        fr = np.nonzero(self.leaf_free)[0]
        for i in fr:
            d[self.copy_level[i]][self.copy_index[i]] = dt(r[i])
        x = [None] * (L + 1)
        for l in range(L, 0, -1):
            o = self.ops[l]
            xl = np.zeros(o.n, dtype=dt)
            if len(o.S):
                xl[o.S] = self.smooth(l, o.A_S, o.dinv, d[l][o.S])
            t = np.zeros(o.n, dtype=dt)
            t[o.S] = d[l][o.S] - o.A_S @ xl[o.S]
            t[o.I] = d[l][o.I] - o.A_IS @ xl[o.S]
            d[l - 1] += self.R[l] @ t
            d[l - 1][~self.ops[l - 1].free] = 0
            x[l] = xl
        o0 = self.ops[0]
        x0 = np.zeros(o0.n, dtype=dt)
        if self.n0:
            x0[o0.S] = sla.cho_solve(self.chol, d[0][o0.S].astype(np.float64)).astype(dt)
        x[0] = x0
        for l in range(1, L + 1):
            o = self.ops[l]
            x[l] = x[l] + self.P[l] @ x[l - 1]
            x[l][~o.free] = 0
            if len(o.S):
                g = d[l][o.S] - o.A_SI @ x[l][o.I]
                x[l][o.S] = self.smooth(l, o.A_S, o.dinv, g, x0=x[l][o.S])
        z = np.zeros(len(r))
        for i in fr:
            z[i] = float(x[self.copy_level[i]][self.copy_index[i]])
        return z


def pcg(A, b, precond, rtol=1e-10, max_iter=200, free=None):
    """Preconditioned CG, x0 = 0, stop at ||r|| <= rtol ||b||.  Returns
    (x, iterations, history of ||r_j||/||b||, converged)."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = float(np.linalg.norm(b))
    hist = [1.0 if nb > 0 else 0.0]
    if nb == 0.0:
        return x, 0, hist, True
    p = None
    rho_old = None
    for it in range(1, max_iter + 1):
        z = precond(r)
        rho = float(r @ z)
        p = z.copy() if p is None else z + (rho / rho_old) * p
        q = A @ p
        alpha = rho / float(p @ q)
        x += alpha * p
        r -= alpha * q
        res = float(np.linalg.norm(r))
        hist.append(res / nb)
        if res <= rtol * nb:
            return x, it, hist, True
        rho_old = rho
    return x, max_iter, hist, False


# --------------------------------------------------------------- full space

class FullSpaceMG:
    """Alg. 2 applied literally to the nested conforming spaces V_l on the
    level meshes T_l = {cells of level l} + {leaves of level < l} (Sec. 2.3),
    each with its own hanging-node constraints, P_l the interpolation of the
    coarse function at the fine nodes and R_l = P_l^T.  Smoothing is restricted
    to V_l^S with the same Chebyshev parameters.  Used on tiny meshes only, as
    an independent check of the storage-efficient V-cycle (the paper states
    the two are algebraically equivalent)."""

    def __init__(self, disc, coeff, ref: LocalSmoothingMG):
        f, k, nk = disc.forest, disc.k, disc.nk
        self.ref = ref
        lcoeff = level_coefficients(disc, coeff)
        cval = {}
        for l, lev in enumerate(disc.levels):
            for c, a in zip(lev.cells, lcoeff[l]):
                cval[c] = a
        L = len(disc.levels) - 1
        self.sp = []
        for l in range(L + 1):
            cells = set(disc.levels[l].cells) | {c for c in f.leaves if c[0] < l}
            cells = sorted(cells, key=f.sort_key)
            num = number_active(f, cells, nk)
            A, _ = leaf_matrices(type("D", (), {"leaf": num, "forest": f, "k": k})(),
                                 np.array([cval[c] for c in cells]))
            free = np.nonzero(num.dirichlet == 0)[0]
            A = A.tocsr()[free][:, free].tocsr()
            pos = {int(g): i for i, g in enumerate(free)}
            lev = disc.levels[l]
            S_loc, S_lev = [], []
            for g in free:
                key = num.keys[g]
                j = lev.dof_of.get(key)
                if j is not None and lev.flags[j] == FLAG_S:
                    S_loc.append(pos[int(g)])
                    S_lev.append(j)
            self.sp.append(dict(num=num, cells=cells, A=A, free=free, S=np.array(S_loc, dtype=np.int64),
                                S_lev=np.array(S_lev, dtype=np.int64)))
        self.P = [None]
        for l in range(1, L + 1):
            self.P.append(self._interp(disc, l))
        A0 = self.sp[0]["A"].toarray()
        self.A0 = A0

    def _interp(self, disc, l):
        f, nk, k, dim = disc.forest, disc.nk, disc.k, disc.forest.dim
        fine, coarse = self.sp[l], self.sp[l - 1]
        cset = set(coarse["cells"])
        cpos = {int(g): i for i, g in enumerate(coarse["free"])}
        cnum = coarse["num"]
        cidx = {c: i for i, c in enumerate(coarse["cells"])}
        rows, cols, vals = [], [], []
        for ri, g in enumerate(fine["free"]):
            x = nk.coord(fine["num"].keys[g])
            cell = None
            for m in range(l - 1, -1, -1):
                s = side(m)
                for sgn in range(1 << dim):
                    a = []
                    for i in range(dim):
                        u = x[i] * (1 << 20)
                        base = math.floor(u / s) * s
                        if (sgn >> i) & 1 and abs(u - base) < 1e-9:
                            base -= s
                        a.append(int(base))
                    cand = (m, tuple(a))
                    if cand in cset:
                        cell = cand
                        break
                if cell is not None:
                    break
            assert cell is not None
            h = side(cell[0])
            xi = [(x[i] * (1 << 20) - cell[1][i]) / h for i in range(dim)]
            V = [lagrange(nk.x, [xi[i]])[0] for i in range(dim)]
            cm = cnum.cellmap[cidx[cell]]
            acc = {}
            for li, jl in enumerate(nk.local):
                w = 1.0
                for i in range(dim):
                    w *= V[i][jl[i]]
                if w == 0.0:
                    continue
                e = int(cm[li])
                if e >= 0:
                    terms = [(e, 1.0)]
                else:
                    hh = -e - 1
                    terms = [(int(cnum.c_masters[p]), float(cnum.c_weights[p]))
                             for p in range(cnum.c_offsets[hh], cnum.c_offsets[hh + 1])]
                for dof, cw in terms:
                    if dof in cpos:
                        acc[cpos[dof]] = acc.get(cpos[dof], 0.0) + w * cw
            for c, v in acc.items():
                if abs(v) > 1e-15:
                    rows.append(ri)
                    cols.append(c)
                    vals.append(v)
        return sp.coo_matrix((vals, (rows, cols)),
                             shape=(len(fine["free"]), len(coarse["free"]))).tocsr()

    def _smooth(self, l, x, g, zero_start):
        s = self.sp[l]
        o = self.ref.ops[l]
        S = s["S"]
        if len(S) == 0:
            return x
        # Jacobi diagonal and Chebyshev interval from the storage-efficient setup
        pos = {int(j): i for i, j in enumerate(o.S)}
        perm = np.array([pos[int(j)] for j in s["S_lev"]], dtype=np.int64)
        dinv = o.dinv[perm].astype(np.float64)
        A = s["A"]
        notS = np.setdiff1d(np.arange(A.shape[0]), S)
        ASS = A[S][:, S]
        rhs = g[S] - A[S][:, notS] @ x[notS]
        x = x.copy()
        x[S] = self.ref.smooth(l, ASS, dinv, rhs, x0=None if zero_start else x[S])
        return x

    def _vc(self, l, g):
        if l == 0:
            if self.A0.shape[0] == 0:
                return np.zeros(0)
            return sla.solve(self.A0, g, assume_a="pos")
        A = self.sp[l]["A"]
        u1 = self._smooth(l, np.zeros(A.shape[0]), g, True)
        c = self._vc(l - 1, self.P[l].T @ (g - A @ u1))
        u2 = u1 + self.P[l] @ c
        return self._smooth(l, u2, g, False)

    def vcycle(self, r):
        L = len(self.sp) - 1
        free = self.sp[L]["free"]
        z = np.zeros(len(r))
        z[free] = self._vc(L, r[free])
        return z
