"""The in-cell form of the hanging-node constraints (parent-arranged DoFs on
refinement faces/edges, interpolated per cell with the 1D embedding) rebuilt
in numpy from the library's host arrays equals the oracle's assembled
C^T A C.  CPU only: checks the host data the leaf kernel consumes."""
import numpy as np
import pytest
import scipy.sparse as sp

from helpers import CASES, library_problem, oracle_problem
from oracle.basis import cell_stiffness, embed_1d


def _local_C(mask, dim, k):
    """n^d x n^d matrix: fine local values from parent-arranged local values."""
    n = k + 1
    E = embed_1d(k)
    b = [(mask >> i) & 1 for i in range(dim)]
    face = [(mask >> (3 + i)) & 1 for i in range(dim)]
    edge = [(mask >> (6 + i)) & 1 for i in range(dim)] if dim == 3 else [0] * dim
    npc = n ** dim
    idx = [tuple((p // n ** a) % n for a in range(dim)) for p in range(npc)]
    pos = {j: p for p, j in enumerate(idx)}
    C = np.eye(npc)
    for p, j in enumerate(idx):
        sets = []
        for a in range(dim):
            if face[a] and j[a] == b[a] * k:
                sets.append([c for c in range(dim) if c != a])
            if edge[a] and all(j[c] == b[c] * k for c in range(dim) if c != a):
                sets.append([a])
        if not sets:
            continue
        axes = sets[0]
        row = np.zeros(npc)
        for q, J in enumerate(idx):
            if any(J[c] != j[c] for c in range(dim) if c not in axes):
                continue
            w = 1.0
            for c in axes:
                w *= E[b[c] * k + j[c], J[c]]
            row[q] = w
        C[p] = row
    return C


@pytest.mark.parametrize("case", ["lshape-q1", "lshape-q2", "lshape-q4", "fichera-q1", "fichera-q2",
                                  "fichera-q3", "fichera-q4", "cube-q2"])
def test_incell_constraints_rebuild_leaf_operator(case):
    rec, k = CASES[case]
    op, _ = oracle_problem(rec, k)
    m, P, _ = library_problem(rec, k)
    dim = m.dim
    npc = (k + 1) ** dim
    cm = P.array("LEAF_CELLMAP_PARENT").reshape(-1, npc)
    mask = P.array("LEAF_MASK")
    assert (cm >= 0).all() and (mask >> 3).any()
    lv, _ = m.leaves()
    h = 2.0 ** (-lv.astype(np.float64))
    Aref = cell_stiffness(dim, k)
    N = P.n_dofs
    rows, cols, vals = [], [], []
    cache = {}
    for c in range(len(lv)):
        mk = int(mask[c])
        if mk not in cache:
            Cl = _local_C(mk, dim, k) if (mk >> 3) else np.eye(npc)
            cache[mk] = Cl.T @ Aref @ Cl
        Ak = cache[mk] * h[c] ** (dim - 2)
        ids = cm[c]
        rows.append(np.repeat(ids, npc))
        cols.append(np.tile(ids, npc))
        vals.append(Ak.reshape(-1))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N)).tocsr()
    free = op.free.astype(np.float64)
    A = sp.diags(free) @ A @ sp.diags(free)
    assert abs(A - op.A).max() <= 1e-12 * abs(op.A).max()
