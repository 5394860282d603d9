"""Seeded synthetic workload generators shared by the oracle and the HIP library.

This module holds no arithmetic of the multigrid method: it only produces the
*inputs* of a solve (coarse meshes, refinement flags from geometric markers or
seeded random draws, nodal right-hand-side values, cell coefficients, request
specifications and arrival times).  Refinement itself (2:1 closure), DoF
numbering, operators and solvers live in the oracle and in the library, which
share no code with each other.

Geometry convention (both consumers use it): a coarse cell is the unit cube
[o, o+1]^d at an integer origin o.  A cell of refinement level l is given by its
level and its *global* integer anchor in units of 2^-20 (so its side is
2^(20-l) units).  Cell centres are exact in units of 2^-21: 2*anchor + side.

Workloads (the paper's own workloads are generated meshes; these recipes stand
in for them, see the paper's Section 4):
  C1  2D L-shape [-1,1]^2 minus [0,1]^2, Q1, g global refinements then 3
      cycles refining cells whose centre is within 0.5^(c+1) of the re-entrant
      corner.
  C2/C3/C5  3D Fichera corner [-1,1]^3 minus [0,1]^3, g global refinements then
      4 cycles: corner marks OR seeded uniform draw < 0.05.
  C4  stream of unit-cube requests refined toward a seeded point.
  A41 the paper's "annulus" mesh of its V-cycle scaling runs (Sec. 3.5, 4.1):
      the cube [-1,1]^3 as 5^3 coarse cells (the 125 level-0 cells of the
      paper's per-level workload table), L-3 global refinements, then three
      steps: cells whose centre lies inside the sphere of radius 0.55, then
      in the shell 0.3 <= r <= 0.43, then in 0.335 <= r <= 0.39; Q2,
      Chebyshev degree 5.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

UNIT = 1 << 20  # anchor units per coarse cell side

COARSE_MESHES = {
    # name: (dim, origins of the unit coarse cells, in this order)
    "square": (2, [(0, 0)]),
    "lshape": (2, [(-1, -1), (0, -1), (-1, 0)]),
    "cube": (3, [(0, 0, 0)]),
    "fichera": (3, [(x, y, z) for z in (-1, 0) for y in (-1, 0) for x in (-1, 0)
                    if (x, y, z) != (0, 0, 0)]),
    # [-1,1]^3 as 5^3 unit cells: physical x = 0.4 (mesh x - 2.5)
    "cube5": (3, [(x, y, z) for z in range(5) for y in range(5) for x in range(5)]),
}

# annulus steps of the "cube5" mesh: (r / 0.4)^2 as exact fractions (num,
# den) of the physical radii 0.55, 0.3, 0.43, 0.335, 0.39
ANNULUS_R2 = {"0.55": (121, 64), "0.3": (9, 16), "0.43": (1849, 1600), "0.335": (4489, 6400), "0.39": (1521, 1600)}

SEED_FICHERA = 1904  # shared by C2, C3, C5 (random marks: PCG64(1904*100 + c))
SEED_NOISE = 1905    # C2/C3 nodal noise


def coarse_mesh(name):
    """Return (dim, origins as an int32 array [n_coarse, dim])."""
    dim, origins = COARSE_MESHES[name]
    return dim, np.asarray(origins, dtype=np.int32).reshape(-1, dim)


def _centres_x2(levels, anchors):
    """Cell centres in units of 2^-21 (exact integers), shape [n, dim]."""
    levels = np.asarray(levels, dtype=np.int64)
    anchors = np.asarray(anchors, dtype=np.int64)
    side = (np.int64(1) << (20 - levels)).reshape(-1, 1)
    return 2 * anchors + side


def flags_all(n_leaves):
    return np.ones(int(n_leaves), dtype=np.uint8)


def flags_corner(levels, anchors, cycle):
    """Mark every leaf whose centre lies strictly within 0.5^(cycle+1) of the
    origin (the re-entrant corner of the L-shape and of the Fichera domain).
    Exact integer test: |2*anchor+side|^2 < (2^21 * 2^-(cycle+1))^2."""
    c2 = _centres_x2(levels, anchors)
    if c2.shape[0] == 0:
        return np.zeros(0, dtype=np.uint8)
    r = np.int64(1) << (20 - cycle)
    d2 = (c2.astype(object) ** 2).sum(axis=1) if r > (1 << 30) else (c2 * c2).sum(axis=1)
    return (d2 < r * r).astype(np.uint8)


def _annulus_r2(levels, anchors):
    """Squared physical distance of the cell centres from the centre of the
    "cube5" mesh, as the integer S with r^2 / 0.4^2 = S / 2^42 (exact)."""
    c2 = _centres_x2(levels, anchors) - 5 * (1 << 20)   # units 2^-21, centred
    return (c2 * c2).sum(axis=1)


def _r2_less(S, key):
    num, den = ANNULUS_R2[key]
    return S * den < num * (np.int64(1) << 42)


def flags_annulus(levels, anchors, cycle):
    """Step `cycle` (1, 2, 3) of the annulus refinement on the "cube5" mesh:
    centre inside radius 0.55; centre in the shell 0.3 <= r <= 0.43; centre
    in 0.335 <= r <= 0.39 (exact integer tests)."""
    if len(levels) == 0:
        return np.zeros(0, dtype=np.uint8)
    S = _annulus_r2(levels, anchors)
    if cycle == 1:
        m = _r2_less(S, "0.55")
    elif cycle == 2:
        m = ~_r2_less(S, "0.3") & ~(~_r2_less(S, "0.43") & (S * 1600 != 1849 * (np.int64(1) << 42)))
    elif cycle == 3:
        m = ~_r2_less(S, "0.335") & ~(~_r2_less(S, "0.39") & (S * 1600 != 1521 * (np.int64(1) << 42)))
    else:
        m = np.zeros(len(levels), dtype=bool)
    return m.astype(np.uint8)


def flags_random(n_leaves, seed_cfg, cycle, frac=0.05):
    """One uniform draw per current leaf, in canonical leaf order, from
    PCG64(seed_cfg*100 + cycle); mark iff u < frac."""
    rng = np.random.Generator(np.random.PCG64(seed_cfg * 100 + cycle))
    return (rng.random(int(n_leaves)) < frac).astype(np.uint8)


@dataclass
class MeshRecipe:
    """A refinement recipe: a coarse mesh, `globals_` global refinements, then
    `cycles` adaptive cycles with the given marker."""
    coarse: str
    globals_: int
    cycles: int
    marker: str  # "corner" | "corner+random" | "none"
    seed: int = SEED_FICHERA

    def flags(self, step, levels, anchors):
        """Flags for refinement step `step` (0-based) given the current leaves
        (canonical order).  Steps < globals_ are global refinements."""
        n = len(levels)
        if step < self.globals_:
            return flags_all(n)
        c = step - self.globals_ + 1
        if self.marker == "corner":
            return flags_corner(levels, anchors, c)
        if self.marker == "corner+random":
            return flags_corner(levels, anchors, c) | flags_random(n, self.seed, c)
        if self.marker == "annulus":
            return flags_annulus(levels, anchors, c)
        return np.zeros(n, dtype=np.uint8)

    @property
    def steps(self):
        return self.globals_ + self.cycles


def build_mesh(recipe: MeshRecipe, create, refine, leaves):
    """Drive a recipe through a forest implementation given as callables:
    create(dim, origins) -> handle; refine(handle, flags); leaves(handle) ->
    (levels [n], anchors [n, dim]) in canonical order.  Returns the handle."""
    dim, origins = coarse_mesh(recipe.coarse)
    h = create(dim, origins)
    for s in range(recipe.steps):
        lv, an = leaves(h)
        refine(h, recipe.flags(s, lv, an))
    return h


# ---------------------------------------------------------------- workloads

@dataclass
class Workload:
    name: str
    recipe: MeshRecipe
    degree: int
    rhs: str = "one"          # "one" | "noise"
    coeff: str = "one"        # "one" | "checker"
    mg_precision: int = 64
    cheb_degree: int = 4
    smoother: str = "chebyshev"   # "chebyshev" | "jacobi" (undamped, Sec. 4.3)
    notes: str = ""


def workload(name, g=None):
    """Named workloads.  `g` overrides the number of global refinements."""
    if name == "C1":
        return Workload("C1", MeshRecipe("lshape", 5 if g is None else g, 3, "corner"), 1)
    if name == "C1-tiny":
        return Workload("C1-tiny", MeshRecipe("lshape", 3 if g is None else g, 3, "corner"), 1)
    if name == "C2":
        return Workload("C2", MeshRecipe("fichera", 5 if g is None else g, 4, "corner+random"), 2,
                        rhs="noise")
    if name == "C3-Q2":
        return Workload("C3-Q2", MeshRecipe("fichera", 6 if g is None else g, 4, "corner+random"), 2,
                        rhs="noise", mg_precision=32)
    if name == "C3-Q4":
        return Workload("C3-Q4", MeshRecipe("fichera", 5 if g is None else g, 4, "corner+random"), 4,
                        rhs="noise", mg_precision=32)
    if name == "C5":
        return Workload("C5", MeshRecipe("fichera", 5 if g is None else g, 4, "corner+random"), 3,
                        coeff="checker", mg_precision=32)
    if name == "A41":
        # the paper's V-cycle scaling mesh (Sec. 4.1): annulus refinement of
        # the cube, L = g + 3 (g = 4: the paper's 3D table with 125 ... 2.98e6
        # cells per level), Q2, f = 1, Chebyshev degree 5, FP32 V-cycle
        return Workload("A41", MeshRecipe("cube5", 4 if g is None else g, 3, "annulus"), 2,
                        mg_precision=32, cheb_degree=5)
    if name == "L43":
        # the paper's Laplace comparison (Sec. 4.3): Fichera corner, eps in
        # {1, 100}, f = 1, Q2, "MF" preconditioner (one undamped FP32 Jacobi
        # step per level); mesh from the C2 recipe unless refined adaptively
        return Workload("L43", MeshRecipe("fichera", 4 if g is None else g, 4, "corner+random"), 2,
                        coeff="eps", mg_precision=32, cheb_degree=1, smoother="jacobi")
    raise KeyError(name)


def rhs_nodal(kind, n_dofs, seed=SEED_NOISE):
    """Nodal right-hand-side values, one per leaf DoF in canonical DoF order
    (Dirichlet nodes included): 1, or 1 + N(0, 0.1^2) from PCG64(seed)."""
    if kind == "one":
        return np.ones(int(n_dofs))
    rng = np.random.Generator(np.random.PCG64(seed))
    return 1.0 + rng.normal(0.0, 0.1, int(n_dofs))


def coeff_cells(kind, levels, anchors):
    """Cell-constant coefficient a_K per leaf.  'checker': blocks of side 1/4
    tiling [-1,1]^d; a = 100 where the sum of block indices of the cell centre
    is odd, else 1 (exact integer evaluation).  'eps': the Fichera-corner
    coefficient of the paper's Laplace comparison (Sec. 4.3), 1 where
    min(x, y, z) > -1/2 and 100 elsewhere, at the cell centre (exact: the
    plane x = -1/2 is a cell face on every level >= 1)."""
    n = len(levels)
    if kind == "one":
        return np.ones(n)
    c2 = _centres_x2(levels, anchors)               # units of 2^-21
    if kind == "eps":
        return np.where((c2 > -(1 << 20)).all(axis=1), 1.0, 100.0)
    blk = (c2 + (1 << 21)) >> 19                   # floor(4 * (x + 1))
    odd = (blk.sum(axis=1) & 1).astype(bool)
    return np.where(odd, 100.0, 1.0)


# ---------------------------------------------------------------- serving stream

@dataclass
class RequestSpec:
    """One serving request: unit cube, Q2, refined toward a seeded point."""
    rid: int
    target_dofs: float
    point: tuple
    g0: int
    max_level: int = 7

    def flags(self, step, levels, anchors):
        """Flags for step `step` or None when the recipe is complete.  Steps
        < g0 refine globally; afterwards mark the q leaves whose centres are
        nearest the point (ties in canonical order), q = ceil((C* - C)/7) with
        C* = target_dofs/8 leaves; stop at C >= C* or when no leaf below
        max_level is left."""
        n = len(levels)
        if step < self.g0:
            return flags_all(n)
        target_cells = self.target_dofs / 8.0
        if n >= target_cells:
            return None
        lv = np.asarray(levels)
        ok = lv < self.max_level
        if not ok.any():
            return None
        c = _centres_x2(levels, anchors).astype(np.float64) / float(1 << 21)
        d2 = ((c - np.asarray(self.point)) ** 2).sum(axis=1)
        d2[~ok] = np.inf
        q = int(math.ceil((target_cells - n) / 7.0))
        q = max(1, min(q, int(ok.sum())))
        order = np.argsort(d2, kind="stable")[:q]
        f = np.zeros(n, dtype=np.uint8)
        f[order] = 1
        return f


def request_spec(r):
    rng = np.random.Generator(np.random.PCG64(4000 + r))
    lo, hi = 4.0, math.log10(2e6)
    target = 10.0 ** rng.uniform(lo, hi)
    p = tuple(float(v) for v in rng.random(3))
    g0 = 3
    for g in (3, 4, 5):
        if (2 ** (g + 1) + 1) ** 3 <= target:
            g0 = g
    return RequestSpec(r, target, p, g0)


def build_request_mesh(spec: RequestSpec, create, refine, leaves, max_steps=64):
    dim, origins = coarse_mesh("cube")
    h = create(dim, origins)
    for s in range(max_steps):
        lv, an = leaves(h)
        f = spec.flags(s, lv, an)
        if f is None:
            break
        refine(h, f)
    return h


def arrivals(n, rate, seed=4999):
    """Poisson arrival times (seconds) for n requests at `rate` per second."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, int(n)))
