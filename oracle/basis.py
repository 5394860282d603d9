"""1D ingredients of the tensor-product Q_k element on the reference interval
[0, 1] (Sec. 2.1: nodal basis from interpolation points on the reference cell).

Reading of the paper (it only says "a set of interpolation points"): the nodes
are the Gauss-Lobatto-Legendre points, which coincide with the equidistant
points for k <= 2.  Quadrature is Gauss-Legendre with k+1 points, exact for
the 1D mass and stiffness integrands.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_points(k: int) -> np.ndarray:
    """k+1 Gauss-Lobatto-Legendre points on [0,1]: the endpoints plus the roots
    of P_k', symmetrised so that x_j + x_{k-j} = 1 and the midpoint is 1/2."""
    if k < 1:
        raise ValueError("degree must be >= 1")
    if k == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(k + 1)
    c[k] = 1.0
    r = np.sort(npleg.legroots(npleg.legder(c)).real)
    t = (np.concatenate([[-1.0], r, [1.0]]) + 1.0) / 2.0
    t = 0.5 * (t + (1.0 - t[::-1]))
    t[0], t[-1] = 0.0, 1.0
    if k % 2 == 0:
        t[k // 2] = 0.5
    return t


def gauss(nq: int):
    x, w = npleg.leggauss(nq)
    return (x + 1.0) / 2.0, w / 2.0


def lagrange(nodes: np.ndarray, xi) -> np.ndarray:
    """V[q, j] = l_j(xi_q) for the Lagrange polynomials on `nodes`."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(xi), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                V[:, j] *= (xi - nodes[m]) / (nodes[j] - nodes[m])
    return V


def lagrange_deriv(nodes: np.ndarray, xi) -> np.ndarray:
    """D[q, j] = l_j'(xi_q) by the product rule."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((len(xi), n))
    for j in range(n):
        for i in range(n):
            if i == j:
                continue
            term = np.full(len(xi), 1.0 / (nodes[j] - nodes[i]))
            for m in range(n):
                if m != j and m != i:
                    term *= (xi - nodes[m]) / (nodes[j] - nodes[m])
            D[:, j] += term
    return D


def mass_1d(k: int) -> np.ndarray:
    """M_ij = int_0^1 l_i l_j."""
    x = gll_points(k)
    q, w = gauss(k + 1)
    V = lagrange(x, q)
    return (V * w[:, None]).T @ V


def stiff_1d(k: int) -> np.ndarray:
    """K_ij = int_0^1 l_i' l_j'."""
    x = gll_points(k)
    q, w = gauss(k + 1)
    D = lagrange_deriv(x, q)
    return (D * w[:, None]).T @ D


def family_points(k: int) -> np.ndarray:
    """The 2k+1 node positions of two children of [0,1], in parent
    coordinates: x_j/2 for j=0..k, then (1+x_j)/2 for j=1..k."""
    x = gll_points(k)
    return np.concatenate([x / 2.0, (1.0 + x[1:]) / 2.0])


def embed_1d(k: int) -> np.ndarray:
    """E[i, J] = l_J^parent(child node i): the (2k+1) x (k+1) 1D embedding of
    the parent space into the two children (Sec. 2.2, nested spaces)."""
    return lagrange(gll_points(k), family_points(k))


def cell_stiffness(dim: int, k: int) -> np.ndarray:
    """Reference Laplacian on a Cartesian cell of unit size, node index
    x fastest: sum over directions of K in that direction and M elsewhere."""
    M, K = mass_1d(k), stiff_1d(k)
    if dim == 2:
        return np.kron(M, K) + np.kron(K, M)
    return np.kron(M, np.kron(M, K)) + np.kron(M, np.kron(K, M)) + np.kron(K, np.kron(M, M))


def cell_mass(dim: int, k: int) -> np.ndarray:
    M = mass_1d(k)
    out = M
    for _ in range(dim - 1):
        out = np.kron(M, out)
    return out
