"""Degrees of freedom on the leaf mesh and on the level meshes (Sec. 2.1
nodal basis and continuity, Sec. 2.3 hanging-node elimination, level meshes
and the splitting V_l = V_l^S + V_l^I + V_l^L of Fig. 1).

Node identity.  Along one axis, local node j of a level-l cell with integer
cell index c is identified by its exact dyadic coordinate when j is 0, k, or
k/2 (k even); otherwise (interior Gauss-Lobatto points, k >= 3) by the tuple
(l, c, j), because such a point never coincides with a node of a cell of
another level or position.  A node key is the tuple of its per-axis keys.

Conventions (readings of the paper where it is silent):
* leaf DoFs: leaves in canonical order, local nodes in lexicographic order
  (x fastest); every non-hanging node gets the next index at first touch.
  Dirichlet nodes are numbered and flagged; hanging nodes are not numbered as
  DoFs, they get their own first-touch index h and appear as -(h+1) in the
  cell map.
* a node of a leaf K is hanging iff it lies in the closure of a coarser leaf N
  and is not a node of N.  Its masters are the nodes of N on the smallest
  entity of N containing it whose weight (N's Lagrange basis at the node) is
  nonzero, ordered lexicographically (z slowest); they are never hanging
  themselves.
* level l: the cells of level l (leaves or not) in canonical order, first-touch
  numbering of all their nodes; flag D = on the domain boundary, I = in the
  closure of a leaf of level < l, S = otherwise.
* copy map: leaf DoF i lives on level m_i = the smallest level of the leaves
  having it as a node, where it is an S (or D) node.
* families: level-l cells (l >= 1) come in complete groups of 2^d siblings,
  consecutive in canonical order.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

from .basis import gll_points, lagrange
from .forest import side

FLAG_S, FLAG_I, FLAG_D = 0, 1, 2


class NodeKeys:
    def __init__(self, dim: int, k: int):
        self.dim, self.k = dim, k
        self.n = k + 1
        self.x = gll_points(k)
        self.local = [tuple((idx // self.n ** a) % self.n for a in range(dim))
                      for idx in range(self.n ** dim)]

    def axis_key(self, lvl, a, j):
        s = side(lvl)
        k = self.k
        if j == 0:
            return (0, 2 * a)
        if j == k:
            return (0, 2 * a + 2 * s)
        if k % 2 == 0 and 2 * j == k:
            return (0, 2 * a + s)
        return (1, lvl, a // s, j)

    def key(self, cell, jloc):
        lvl, a = cell
        return tuple(self.axis_key(lvl, a[i], jloc[i]) for i in range(self.dim))

    def cell_keys(self, cell):
        return [self.key(cell, j) for j in self.local]

    def axis_coord(self, ak):
        if ak[0] == 0:
            return ak[1] / float(1 << 21)
        _, lvl, c, j = ak
        return (c + self.x[j]) / float(1 << lvl)

    def coord(self, key):
        return tuple(self.axis_coord(ak) for ak in key)

    def on_boundary(self, key, forest) -> bool:
        """Exact test: some point of the node's neighbourhood (probes at
        +-2^-22 along dyadic axes) lies outside every coarse cell."""
        probes = []
        for ak in key:
            if ak[0] == 0:
                probes.append((2 * ak[1] - 1, 2 * ak[1] + 1))
            else:
                _, lvl, c, _ = ak
                probes.append(((2 * c + 1) << (21 - lvl),))
        for p in itertools.product(*probes):
            if tuple(v >> 22 for v in p) not in forest.tree_of:
                return True
        return False


def _touch_sets(nk: NodeKeys, K, off):
    """Per-axis lists of K-local node indices lying in the closure of the
    neighbour of K's parent at offset `off` (None if K does not touch it)."""
    lvl, a = K
    pa = (a[i] // side(lvl - 1) * side(lvl - 1) for i in range(nk.dim))
    pa = tuple(pa)
    S, s, k = side(lvl - 1), side(lvl), nk.k
    per = []
    for i in range(nk.dim):
        if off[i] == 1:
            if a[i] + s != pa[i] + S:
                return None
            per.append([k])
        elif off[i] == -1:
            if a[i] != pa[i]:
                return None
            per.append([0])
        else:
            per.append(list(range(k + 1)))
    return per


def hanging_constraints(forest, cells, active, nk: NodeKeys):
    """Hanging nodes of the balanced mesh made of `cells` (all of them leaves
    of that mesh; `active` is the set).  Returns {key: [(master_key, w)]}."""
    k, dim = nk.k, nk.dim
    hanging = {}
    offs = forest.offsets()
    for K in cells:
        lvl, a = K
        if lvl == 0:
            continue
        pl, pa = forest.parent(K)
        S, s = side(pl), side(lvl)
        for off in offs:
            na = tuple(pa[i] + off[i] * S for i in range(dim))
            N = (pl, na)
            if N not in active:
                continue
            per = _touch_sets(nk, K, off)
            if per is None:
                continue
            for jl in itertools.product(*per):
                axes = []
                fixed = True
                for i in range(dim):
                    if off[i] == 1:
                        axes.append([(0, 1.0)])
                        continue
                    if off[i] == -1:
                        axes.append([(k, 1.0)])
                        continue
                    kk = nk.axis_key(lvl, a[i], jl[i])
                    match = [J for J in range(k + 1) if nk.axis_key(pl, na[i], J) == kk]
                    if match:
                        axes.append([(match[0], 1.0)])
                    else:
                        fixed = False
                        b = (a[i] - pa[i]) // s
                        xi = 0.5 * b + 0.5 * nk.x[jl[i]]
                        w = lagrange(nk.x, [xi])[0]
                        axes.append([(J, float(w[J])) for J in range(k + 1)])
                if fixed:
                    continue
                key = nk.key(K, jl)
                masters = []
                for combo in itertools.product(*reversed(axes)):
                    combo = combo[::-1]   # back to (x, y, z)
                    mk = tuple(nk.axis_key(pl, na[i], combo[i][0]) for i in range(dim))
                    w = 1.0
                    for c in combo:
                        w *= c[1]
                    masters.append((mk, w))
                if key in hanging:
                    assert [m for m, _ in hanging[key]] == [m for m, _ in masters]
                else:
                    hanging[key] = masters
    return hanging


@dataclass
class ActiveNumbering:
    """Numbering of a (possibly non-conforming) active mesh."""
    cells: list
    cellmap: np.ndarray          # [n_cells, n^d]; >= 0 DoF, < 0 -(h+1)
    keys: list                   # DoF keys in DoF order
    hkeys: list                  # hanging keys in hanging order
    dof_of: dict
    c_offsets: np.ndarray        # [H+1]
    c_masters: np.ndarray        # DoF ids
    c_weights: np.ndarray
    dirichlet: np.ndarray        # uint8 [N]

    @property
    def n_dofs(self):
        return len(self.keys)


def number_active(forest, cells, nk: NodeKeys) -> ActiveNumbering:
    active = set(cells)
    hanging = hanging_constraints(forest, cells, active, nk)
    dof_of, hang_of = {}, {}
    keys, hkeys = [], []
    cellmap = np.zeros((len(cells), nk.n ** nk.dim), dtype=np.int64)
    for ci, K in enumerate(cells):
        for li, key in enumerate(nk.cell_keys(K)):
            if key in hanging:
                if key not in hang_of:
                    hang_of[key] = len(hkeys)
                    hkeys.append(key)
                cellmap[ci, li] = -(hang_of[key] + 1)
            else:
                if key not in dof_of:
                    dof_of[key] = len(keys)
                    keys.append(key)
                cellmap[ci, li] = dof_of[key]
    offs, mas, wts = [0], [], []
    for key in hkeys:
        ms = hanging[key]
        for mk, w in ms:
            assert mk in dof_of, "a master node is itself hanging"
            mas.append(dof_of[mk])
            wts.append(w)
        offs.append(len(mas))
        assert abs(sum(w for _, w in ms) - 1.0) < 1e-13
    dirichlet = np.array([nk.on_boundary(key, forest) for key in keys], dtype=np.uint8)
    for key in hkeys:
        if nk.on_boundary(key, forest):
            assert all(dirichlet[dof_of[mk]] for mk, _ in hanging[key])
    return ActiveNumbering(cells, cellmap, keys, hkeys, dof_of,
                           np.array(offs, dtype=np.int64), np.array(mas, dtype=np.int64),
                           np.array(wts, dtype=np.float64), dirichlet)


@dataclass
class Level:
    lvl: int
    cells: list
    cellmap: np.ndarray      # [C_l, n^d] level DoF ids
    keys: list
    dof_of: dict
    flags: np.ndarray        # uint8 [N_l]: 0 S, 1 I, 2 D
    parent_index: np.ndarray = None  # [F_l] index of the parent in level l-1 cells
    family_map: np.ndarray = None    # [F_l, (2k+1)^d] level-l DoF ids

    @property
    def n_dofs(self):
        return len(self.keys)


def build_level(forest, lvl, nk: NodeKeys) -> Level:
    cells = forest.level_cells(lvl)
    dof_of, keys = {}, []
    cellmap = np.zeros((len(cells), nk.n ** nk.dim), dtype=np.int64)
    for ci, K in enumerate(cells):
        for li, key in enumerate(nk.cell_keys(K)):
            if key not in dof_of:
                dof_of[key] = len(keys)
                keys.append(key)
            cellmap[ci, li] = dof_of[key]
    iset = set()
    if lvl >= 1:
        for K in cells:
            pl, pa = forest.parent(K)
            S = side(pl)
            for off in forest.offsets():
                N = (pl, tuple(pa[i] + off[i] * S for i in range(nk.dim)))
                if N not in forest.leaves:
                    continue
                per = _touch_sets(nk, K, off)
                if per is None:
                    continue
                for jl in itertools.product(*per):
                    iset.add(nk.key(K, jl))
    flags = np.zeros(len(keys), dtype=np.uint8)
    for i, key in enumerate(keys):
        if nk.on_boundary(key, forest):
            flags[i] = FLAG_D
        elif key in iset:
            flags[i] = FLAG_I
    L = Level(lvl, cells, cellmap, keys, dof_of, flags)
    if lvl >= 1:
        nf = 1 << nk.dim
        assert len(cells) % nf == 0
        pidx = {c: i for i, c in enumerate(forest.level_cells(lvl - 1))}
        m = 2 * nk.k + 1
        fam = np.full((len(cells) // nf, m ** nk.dim), -1, dtype=np.int64)
        par = np.zeros(len(cells) // nf, dtype=np.int64)
        for f in range(len(cells) // nf):
            P = forest.parent(cells[f * nf])
            par[f] = pidx[P]
            assert forest.children(P) == cells[f * nf:(f + 1) * nf]
            for cid in range(nf):
                b = [(cid >> i) & 1 for i in range(nk.dim)]
                for li, jl in enumerate(nk.local):
                    fi = 0
                    for i in range(nk.dim - 1, -1, -1):
                        fi = fi * m + b[i] * nk.k + jl[i]
                    v = cellmap[f * nf + cid, li]
                    assert fam[f, fi] in (-1, v)
                    fam[f, fi] = v
        L.parent_index, L.family_map = par, fam
    return L


@dataclass
class Discretization:
    forest: object
    k: int
    nk: NodeKeys
    leaf: ActiveNumbering
    levels: list
    copy_level: np.ndarray   # [N] int
    copy_index: np.ndarray   # [N] int
    leaf_level: np.ndarray   # [n_leaves] int


def discretize(forest, k: int) -> Discretization:
    nk = NodeKeys(forest.dim, k)
    cells = forest.leaf_order()
    leaf = number_active(forest, cells, nk)
    L = forest.max_level()
    levels = [build_level(forest, l, nk) for l in range(L + 1)]
    N = leaf.n_dofs
    m = np.full(N, 1 << 30, dtype=np.int64)
    lv = np.array([c[0] for c in cells], dtype=np.int64)
    for ci in range(len(cells)):
        ids = leaf.cellmap[ci]
        ids = ids[ids >= 0]
        m[ids] = np.minimum(m[ids], lv[ci])
    idx = np.zeros(N, dtype=np.int64)
    for i, key in enumerate(leaf.keys):
        lev = levels[m[i]]
        j = lev.dof_of[key]
        assert lev.flags[j] != FLAG_I
        idx[i] = j
    # complete-layer rule: every parent node touched by a transfer is S or D
    for l in range(1, L + 1):
        par = levels[l - 1]
        for p in levels[l].parent_index:
            assert (par.flags[par.cellmap[p]] != FLAG_I).all(), "layer rule violated"
    return Discretization(forest, k, nk, leaf, levels, m, idx, lv)
