"""One stiffness row at one micro-vertex, without the full mesh (oracle, test-only).

For levels whose assembled matrix does not fit in memory the oracle still
needs individual rows a_i. (sampled parity checks).  The row of micro-vertex p
sums, over every micro-tet T that has p as a vertex, row p of the element
matrix of T (Section 5.2.1).  Those micro-tets are found by descending the
refinement tree of eq. (bey) in every macro-cell whose closure holds p: at each
level only the children whose closed simplex contains p are refined further,
so the work is (number of tets around p) x 8 x level.

With a coefficient k (the div(k grad) form of fem.py), each element matrix
is scaled by the degree-3 rule applied to k's values at the micro-tet's
vertices, as in the assembly.
"""
from __future__ import annotations

import numpy as np

from .fem import element_coefficient_mean, element_stiffness
from .refine import key_coordinates, keys_of, refine_once


def _contains(tets: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Which tets (weights [m, 4, 4]) contain the point with weights w [4] in
    their closed simplex: w = sum_m lambda_m V_m with all lambda_m >= 0."""
    rhs = np.broadcast_to(w.astype(np.float64), (len(tets), 4))[..., None]
    lam = np.linalg.solve(np.transpose(tets, (0, 2, 1)).astype(np.float64),
                          rhs)[..., 0]
    return (lam >= -1e-9).all(axis=1)


def local_tets(cell_ids: np.ndarray, n_level: int, level: int,
               key: np.ndarray):
    """Micro-tets of one macro-cell that have the keyed point as a vertex, as
    local weights [m, 4, 4]; empty if the point is outside the cell."""
    ids = key[0::2]
    wts = key[1::2]
    w = np.zeros(4, dtype=np.int64)
    for gid, wt in zip(ids, wts):
        if gid < 0:
            continue
        hit = np.flatnonzero(cell_ids == gid)
        if len(hit) == 0:
            return np.zeros((0, 4, 4), dtype=np.int64)
        w[hit[0]] = wt
    tets = (n_level * np.eye(4, dtype=np.int64))[None]
    for _ in range(level):
        tets = refine_once(tets)
        tets = tets[_contains(tets, w)]
    is_vertex = (tets == w[None, None, :]).all(axis=2).any(axis=1)
    return tets[is_vertex]


def row_at(macro_xyz: np.ndarray, cells: np.ndarray, level: int,
           key: np.ndarray, kappa=None):
    """Row of the P1 stiffness matrix at the keyed micro-vertex.

    ``kappa``, if given, maps micro-vertex keys [m, 4, 8] to the values of
    the coefficient k there [m, 4]; the row is then that of div(k grad).

    Returns (neighbour keys [r, 8], values [r], is_dirichlet).  The point is a
    Dirichlet vertex when one of the micro-faces through it belongs to a
    single micro-tet (all micro-tets through such a face contain the point,
    so they are all among the ones found here).
    """
    n = 2 ** level
    key = np.asarray(key, dtype=np.int64)
    acc = {}
    face_count = {}
    for c in range(len(cells)):
        tets = local_tets(np.asarray(cells[c]), n, level, key)
        if len(tets) == 0:
            continue
        tkeys = keys_of(np.asarray(cells[c]), tets)          # [m, 4, 8]
        P = key_coordinates(macro_xyz, tkeys, n)             # [m, 4, 3]
        K, _ = element_stiffness(P)
        if kappa is not None:
            K = K * element_coefficient_mean(kappa(tkeys))[:, None, None]
        for t in range(len(tets)):
            vk = [tuple(tkeys[t, q]) for q in range(4)]
            q0 = vk.index(tuple(key))
            for r in range(4):
                acc[vk[r]] = acc.get(vk[r], 0.0) + K[t, q0, r]
            for drop in range(4):
                if drop == q0:
                    continue
                f = tuple(sorted(vk[s] for s in range(4) if s != drop))
                face_count[f] = face_count.get(f, 0) + 1
    nbr = np.array(sorted(acc), dtype=np.int64).reshape(-1, 8)
    vals = np.array([acc[tuple(k)] for k in nbr])
    dirichlet = any(v == 1 for v in face_count.values())
    return nbr, vals, dirichlet
