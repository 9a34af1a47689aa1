"""Seeded coarse tetrahedral meshes (input generators only).

A mesh is a pair ``(xyz, cells)``: ``xyz`` is a float64 array ``[nv, 3]`` of
macro-vertex coordinates and ``cells`` an int64 array ``[nc, 4]`` of global
macro-vertex ids per macro-cell.  The local vertex order of every cell is part
of the input: regular refinement picks its inner diagonal from that order
(Section 3.1 of the paper), so it is kept as generated and never permuted.

Kuhn boxes split every unit cube into the six tetrahedra
``[p, p+e_a, p+e_a+e_b, p+(1,1,1)]`` over the permutations ``(a, b, c)`` of the
three axes.  With lexicographic vertex ids ``x + (X+1)*(y + (Y+1)*z)`` this
local order is the ascending order of the global ids.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np


def reference_tet():
    """The reference tetrahedron (0,0,0),(1,0,0),(0,1,0),(0,0,1)."""
    xyz = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0],
                    [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    cells = np.array([[0, 1, 2, 3]], dtype=np.int64)
    return xyz, cells


def kuhn_box(a: int, b: int, c: int):
    """``a x b x c`` unit cubes, six Kuhn tetrahedra per cube (6abc cells)."""
    if min(a, b, c) < 1:
        raise ValueError("box dimensions must be positive")
    xs, ys, zs = np.meshgrid(np.arange(a + 1), np.arange(b + 1),
                             np.arange(c + 1), indexing="ij")
    nv = (a + 1) * (b + 1) * (c + 1)
    xyz = np.zeros((nv, 3))
    vid = lambda x, y, z: x + (a + 1) * (y + (b + 1) * z)
    for x, y, z in zip(xs.ravel(), ys.ravel(), zs.ravel()):
        xyz[vid(x, y, z)] = (x, y, z)
    unit = np.eye(3, dtype=np.int64)
    cells = []
    for z in range(c):
        for y in range(b):
            for x in range(a):
                p = np.array([x, y, z])
                for perm in itertools.permutations(range(3)):
                    q1 = p + unit[perm[0]]
                    q2 = q1 + unit[perm[1]]
                    q3 = p + 1
                    cells.append([vid(*p), vid(*q1), vid(*q2), vid(*q3)])
    return xyz, np.array(cells, dtype=np.int64)


def _signed_volumes(xyz, cells):
    p = xyz[cells]
    e = p[:, 1:] - p[:, :1]
    return np.linalg.det(e) / 6.0


def jittered_kuhn_box(a: int, b: int, c: int, amplitude: float = 0.1,
                      seed: int = 3):
    """Kuhn box whose interior macro-vertices move by U[-amp, amp]^3.

    Boundary macro-vertices stay put so the domain remains the box.  Kuhn cells
    come in both orientations (the parity of the axis permutation); every cell
    must keep the sign of its signed volume, which the generator asserts.
    """
    xyz, cells = kuhn_box(a, b, c)
    sign0 = np.sign(_signed_volumes(xyz, cells))
    rng = np.random.default_rng(seed)
    interior = ((xyz[:, 0] > 0) & (xyz[:, 0] < a) & (xyz[:, 1] > 0)
                & (xyz[:, 1] < b) & (xyz[:, 2] > 0) & (xyz[:, 2] < c))
    shift = rng.uniform(-amplitude, amplitude, size=(int(interior.sum()), 3))
    xyz = xyz.copy()
    xyz[interior] += shift
    assert (np.sign(_signed_volumes(xyz, cells)) == sign0).all(), \
        "jitter inverted a cell"
    return xyz, cells


def slab(m: int, t: int, amplitude: float = 0.1, seed=0):
    """First ``t`` cells (generation order) of an ``m x 1 x 1`` Kuhn box,
    unused vertices dropped (ids renumbered in ascending order, so the local
    Kuhn order stays ascending), every vertex jittered by U[-amp, amp]^3."""
    if not (1 <= t <= 6 * m):
        raise ValueError("need 1 <= t <= 6m")
    xyz, cells = kuhn_box(m, 1, 1)
    cells = cells[:t]
    used = np.unique(cells)
    remap = -np.ones(len(xyz), dtype=np.int64)
    remap[used] = np.arange(len(used))
    xyz = xyz[used].copy()
    cells = remap[cells]
    sign0 = np.sign(_signed_volumes(xyz, cells))
    rng = np.random.default_rng(seed)
    xyz += rng.uniform(-amplitude, amplitude, size=xyz.shape)
    assert (np.sign(_signed_volumes(xyz, cells)) == sign0).all(), \
        "jitter inverted a cell"
    return xyz, cells


@dataclass
class BatchProblem:
    """One member of a many-small-meshes batch."""
    index: int
    kind: str            # "box" or "slab"
    shape: tuple         # (a, b, c) for boxes, (m, t) for slabs
    level: int
    xyz: np.ndarray
    cells: np.ndarray
    rhs_seed: tuple      # seed for the nodal source values f ~ U[-1, 1]


def _box_shapes(max_cubes=4):
    return [(a, b, c) for a in range(1, max_cubes + 1)
            for b in range(1, max_cubes + 1) for c in range(1, max_cubes + 1)
            if a * b * c <= max_cubes]


def batch_problems(count: int = 256, seed: int = 6, min_level: int = 3,
                   max_level: int = 6):
    """Seeded batch of independent Poisson problems on 1..24-cell meshes.

    Problem ``p`` draws from ``default_rng([seed, p])``: the mesh kind (Kuhn box
    with at most 4 cubes, or a jittered slab of ``m x 1 x 1`` cubes cut to its
    first ``t`` cells) and a level uniform in ``[min_level, max_level]``.
    """
    shapes = _box_shapes()
    out = []
    for p in range(count):
        rng = np.random.default_rng([seed, p])
        if rng.integers(2) == 0:
            shape = shapes[rng.integers(len(shapes))]
            xyz, cells = kuhn_box(*shape)
            kind = "box"
        else:
            m = int(rng.integers(1, 5))
            t = int(rng.integers(1, 6 * m + 1))
            shape = (m, t)
            xyz, cells = slab(m, t, seed=[seed, p, 2])
            kind = "slab"
        level = int(rng.integers(min_level, max_level + 1))
        out.append(BatchProblem(p, kind, tuple(int(s) for s in shape), level,
                                xyz, cells, (seed, p, 1)))
    return out
