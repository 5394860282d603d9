"""Forest of quad/hex trees over unit coarse cells (Sec. 2.2 mesh hierarchy,
Sec. 2.3 cell levels and leaf mesh, Sec. 3.3/3.5 z-order and 2:1 closure).

A cell is (level, anchor) with a global integer anchor in units of 2^-20 of a
coarse cell; its side is 2^(20-level).  The coarse cells are unit cubes at
integer origins.

Reading of the 2:1 rule (the paper: leaves sharing a degree of freedom differ
by at most one level): any two leaves whose closures touch differ by at most
one level.  It is enforced as the least fixpoint of: for every leaf F of
level L >= 2, every level-(L-1) cell adjacent to F's parent (across faces,
edges or corners, inside the domain) exists; if one is missing, the coarser
leaf covering it is refined.  This is also the paper's complete-layer rule
(a full layer of level L-1 cells around the level-L cells).

Canonical order: by coarse cell, then by the Morton key of the anchor inside
the coarse cell (child id x + 2y + 4z), i.e. depth-first z-order.
"""
from __future__ import annotations

import itertools

import numpy as np

DEPTH = 20
UNIT = 1 << DEPTH
MAX_LEVEL = 18


def side(level: int) -> int:
    return 1 << (DEPTH - level)


def morton(local, dim: int) -> int:
    key = 0
    for b in range(DEPTH - 1, -1, -1):
        for a in range(dim - 1, -1, -1):
            key = (key << 1) | ((local[a] >> b) & 1)
    return key


class Forest:
    def __init__(self, dim: int, origins):
        self.dim = dim
        self.origins = [tuple(int(v) for v in o) for o in np.asarray(origins).reshape(-1, dim)]
        if len(set(self.origins)) != len(self.origins):
            raise ValueError("coarse cells must be distinct")
        self.tree_of = {o: t for t, o in enumerate(self.origins)}
        self.leaves = set()
        self.cells = set()   # every cell ever created (leaves and refined)
        for o in self.origins:
            c = (0, tuple(v * UNIT for v in o))
            self.leaves.add(c)
            self.cells.add(c)
        self._order = None

    # ------------------------------------------------------------ geometry
    def tree(self, anchor):
        return self.tree_of.get(tuple(v >> DEPTH for v in anchor))

    def inside(self, anchor) -> bool:
        return self.tree(anchor) is not None

    def sort_key(self, cell):
        lvl, a = cell
        t = self.tree(a)
        o = self.origins[t]
        local = tuple(a[i] - o[i] * UNIT for i in range(self.dim))
        return (t, morton(local, self.dim), lvl)

    @staticmethod
    def parent(cell):
        lvl, a = cell
        s = side(lvl - 1)
        return (lvl - 1, tuple((v // s) * s for v in a))

    def children(self, cell):
        lvl, a = cell
        s = side(lvl + 1)
        out = []
        for cid in range(1 << self.dim):
            out.append((lvl + 1, tuple(a[i] + ((cid >> i) & 1) * s for i in range(self.dim))))
        return out

    def offsets(self):
        return [o for o in itertools.product((-1, 0, 1), repeat=self.dim) if any(o)]

    # ------------------------------------------------------------ refinement
    def _refine_cells(self, cells):
        for c in cells:
            if c not in self.leaves:
                continue
            if c[0] >= MAX_LEVEL:
                raise ValueError("maximum level exceeded")
            self.leaves.discard(c)
            for ch in self.children(c):
                self.leaves.add(ch)
                self.cells.add(ch)
        self._order = None

    def covering_leaf(self, lvl, anchor):
        """The leaf containing the level-`lvl` cell position `anchor` when that
        cell does not exist."""
        for m in range(lvl - 1, -1, -1):
            s = side(m)
            c = (m, tuple((v // s) * s for v in anchor))
            if c in self.leaves:
                return c
        raise AssertionError("position not covered")

    def close(self) -> int:
        """Least 2:1 balanced refinement containing the current one.  Returns
        the number of cells refined by the closure."""
        added = 0
        while True:
            marks = set()
            for (lvl, a) in self.leaves:
                if lvl < 2:
                    continue
                pl, pa = self.parent((lvl, a))
                s = side(pl)
                for off in self.offsets():
                    na = tuple(pa[i] + off[i] * s for i in range(self.dim))
                    if not self.inside(na) or (pl, na) in self.cells:
                        continue
                    marks.add(self.covering_leaf(pl, na))
            if not marks:
                return added
            added += len(marks)
            self._refine_cells(marks)

    def refine(self, flags) -> int:
        """Refine the flagged leaves (flags in canonical leaf order), then close.
        Returns the number of leaves afterwards."""
        order = self.leaf_order()
        flags = np.asarray(flags).reshape(-1)
        if len(flags) != len(order):
            raise ValueError("one flag per leaf required")
        self._refine_cells([c for c, f in zip(order, flags) if f])
        self.close()
        return len(self.leaves)

    # ------------------------------------------------------------ queries
    def leaf_order(self):
        if self._order is None:
            self._order = sorted(self.leaves, key=self.sort_key)
        return self._order

    def level_cells(self, lvl):
        return sorted((c for c in self.cells if c[0] == lvl), key=self.sort_key)

    def max_level(self):
        return max(c[0] for c in self.leaves)

    def leaves_arrays(self):
        order = self.leaf_order()
        lv = np.array([c[0] for c in order], dtype=np.int8)
        an = np.array([c[1] for c in order], dtype=np.int64).reshape(-1, self.dim)
        return lv, an

    def touching(self, c1, c2) -> bool:
        """Closures of two cells intersect."""
        (l1, a1), (l2, a2) = c1, c2
        s1, s2 = side(l1), side(l2)
        return all(a1[i] <= a2[i] + s2 and a2[i] <= a1[i] + s1 for i in range(self.dim))
