"""P2 (quadratic Lagrange) stiffness on the explicit micro-mesh (oracle, test-only).

Section "Function spaces" of the paper composes the P2 space of one DoF per
micro-vertex and one per micro-edge (the vertex subgroup and the seven edge
subgroups of the subgroup table).  On a regularly refined cell the micro-edge
midpoints of level l together with its micro-vertices are exactly the
micro-vertices of level l + 1, so every P2 node is identified here by its
level-(l + 1) key (refine.py): a vertex with weights w gets 2 w, the midpoint
of the edge (a, b) gets w_a + w_b.

Basis on a micro-tet T with barycentric functions lambda_0..3:
  vertex q:      phi_q  = lambda_q (2 lambda_q - 1)
  edge (q, r):   phi_qr = 4 lambda_q lambda_r
with the edges in the order 01 02 03 12 13 23.  The element matrix
K_T[a, b] = integral over T of grad(phi_a) . grad(phi_b) (Section 5.2.1) has a
degree-2 polynomial integrand, integrated exactly with the degree-3 rule of
fem.py.

Dirichlet nodes: the vertices and edge midpoints of every micro-face that
belongs to a single micro-tet (the domain boundary).  The apply follows the P1
convention: y = A x on interior nodes (boundary values of x act as data) and
y = 0 at Dirichlet nodes.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import TET_Q3_POINTS, TET_Q3_WEIGHTS, barycentric_gradients
from .refine import (key_codec, key_coordinates, keys_of, reference_refinement,
                     refine_once, unique_rows)
from .rows import _contains

EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def node_weights(tets: np.ndarray) -> np.ndarray:
    """Level-(l+1) local weights of the ten P2 nodes of level-l micro-tets
    ``tets`` [m, 4, 4] (weights summing to n): [m, 10, 4], vertices first."""
    v = 2 * tets
    e = np.stack([tets[:, a] + tets[:, b] for a, b in EDGES], axis=1)
    return np.concatenate([v, e], axis=1)


def basis_values(L: np.ndarray) -> np.ndarray:
    """The ten basis functions at barycentric points ``L`` [p, 4]: [p, 10]."""
    v = L * (2 * L - 1)
    e = np.stack([4 * L[:, a] * L[:, b] for a, b in EDGES], axis=1)
    return np.concatenate([v, e], axis=1)


def basis_gradients(L: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Gradients of the ten basis functions at barycentric points ``L`` [p, 4]
    of tets with barycentric gradients ``G`` [m, 4, 3]: [m, p, 10, 3].
    grad(phi_q) = (4 lambda_q - 1) grad(lambda_q);
    grad(phi_qr) = 4 (lambda_q grad(lambda_r) + lambda_r grad(lambda_q))."""
    gv = (4 * L - 1)[None, :, :, None] * G[:, None, :, :]
    ge = [4 * (L[None, :, a, None] * G[:, None, b, :] +
               L[None, :, b, None] * G[:, None, a, :]) for a, b in EDGES]
    return np.concatenate([gv, np.stack(ge, axis=2)], axis=2)


def element_stiffness_p2(P: np.ndarray):
    """P2 element matrices [m, 10, 10] and volumes of tets with vertex
    coordinates ``P`` [m, 4, 3], by the degree-3 rule."""
    G, vol = barycentric_gradients(P)
    dphi = basis_gradients(TET_Q3_POINTS, G)                 # [m, 5, 10, 3]
    K = np.einsum("p,mpad,mpbd->mab", TET_Q3_WEIGHTS, dphi, dphi)
    return vol[:, None, None] * K, vol


def element_load_p2(vol: np.ndarray) -> np.ndarray:
    """Integral of each basis function over the tets [m, 10], by the same
    rule (the right-hand side of a constant source f = 1)."""
    return vol[:, None] * (TET_Q3_WEIGHTS @ basis_values(TET_Q3_POINTS))[None]


class P2System:
    """Assembled P2 stiffness matrix of the level-``level`` micro-mesh, nodes
    in canonical order of their level-(level + 1) keys."""

    def __init__(self, xyz, cells, level: int):
        self.level = int(level)
        self.n = 2 ** self.level
        self.macro_xyz = np.asarray(xyz, dtype=np.float64)
        self.cells = np.asarray(cells, dtype=np.int64)
        local = reference_refinement(self.level)              # [8^l, 4, 4]
        lw = node_weights(local)                               # [8^l, 10, 4]
        nc = len(self.cells)
        allkeys = np.concatenate([keys_of(self.cells[c], lw)
                                  for c in range(nc)]).reshape(-1, 8)
        codec = key_codec(len(self.macro_xyz), 2 * self.n)
        if codec is not None:
            codes = codec[0](allkeys)
            ucodes, inv = np.unique(codes, return_inverse=True)
            self.keys = codec[1](ucodes)
            self.codes = ucodes
        else:
            self.keys, inv = unique_rows(allkeys)
            self.codes = None
        self._codec = codec
        self.tets = inv.reshape(-1, 10).astype(np.int64)      # [M, 10] nodes
        self.xyz = key_coordinates(self.macro_xyz, self.keys, 2 * self.n)
        N = len(self.keys)
        P = self.xyz[self.tets[:, :4]]
        K, vol = element_stiffness_p2(P)
        rows = np.repeat(self.tets, 10, axis=1).ravel()
        cols = np.tile(self.tets, (1, 10)).ravel()
        self.A = sp.coo_matrix((K.ravel(), (rows, cols)), shape=(N, N)).tocsr()
        self.A.sum_duplicates()
        self.tet_volume = vol
        self.load = np.bincount(self.tets.ravel(),
                                weights=element_load_p2(vol).ravel(),
                                minlength=N)
        # boundary micro-faces: a face (triple of vertices) of one micro-tet
        faces = np.concatenate([np.sort(np.delete(self.tets[:, :4], q, axis=1),
                                        axis=1) for q in range(4)])
        uniq, finv = unique_rows(faces)
        count = np.bincount(finv, minlength=len(uniq))
        on_bnd = (count[finv] == 1).reshape(4, -1)             # [drop q, M]
        self.dirichlet = np.zeros(N, dtype=bool)
        for q in range(4):
            hit = on_bnd[q]
            keep = [r for r in range(4) if r != q]
            face_nodes = keep + [4 + e for e, (a, b) in enumerate(EDGES)
                                 if a != q and b != q]
            self.dirichlet[self.tets[hit][:, face_nodes].ravel()] = True
        self.interior = ~self.dirichlet
        self.diag = self.A.diagonal()

    @property
    def num_nodes(self) -> int:
        return len(self.keys)

    def index_of(self, keys: np.ndarray) -> np.ndarray:
        """Node indices of the given level-(l+1) keys (every key must exist)."""
        keys = np.asarray(keys, dtype=np.int64)
        if self._codec is not None:
            c = np.asarray(self._codec[0](keys))
            shape = c.shape
            c = c.reshape(-1)
            idx = np.searchsorted(self.codes, c)
            ok = idx < len(self.codes)
            ok[ok] = self.codes[idx[ok]] == c[ok]
            idx, ok = idx.reshape(shape), ok.reshape(shape)
        else:
            table = {tuple(r): i for i, r in enumerate(self.keys)}
            flat = keys.reshape(-1, 8)
            idx = np.array([table.get(tuple(r), -1) for r in flat])
            idx = idx.reshape(keys.shape[:-1])
            ok = idx >= 0
        if not np.all(ok):
            raise KeyError("key not present among the P2 nodes")
        return idx

    def apply(self, x: np.ndarray) -> np.ndarray:
        """y = A x on interior nodes, 0 at Dirichlet nodes."""
        y = self.A @ x
        y[self.dirichlet] = 0.0
        return y

    def solve_dirichlet(self, b: np.ndarray, g: np.ndarray) -> np.ndarray:
        """u with u = g at Dirichlet nodes and (A u)_I = b_I (sparse direct)."""
        from scipy.sparse.linalg import spsolve
        I = np.flatnonzero(self.interior)
        B = np.flatnonzero(self.dirichlet)
        u = np.array(g, dtype=np.float64)
        rhs = b[I] - self.A[I][:, B] @ g[B]
        u[I] = spsolve(self.A[I][:, I].tocsc(), rhs)
        return u


def p2_row_at(macro_xyz, cells, level: int, key: np.ndarray):
    """Row of the level-``level`` P2 stiffness matrix at the node with
    level-(level + 1) key ``key``, without the full mesh.

    The micro-tets that have the node as a vertex or edge midpoint are found
    by descending the refinement tree of eq. (bey) in every macro-cell whose
    closure holds the point, keeping at each step the children whose closed
    simplex contains it.  Returns (neighbour keys [r, 8], values [r],
    is_dirichlet); the node is a Dirichlet node when one of the micro-faces
    it lies on belongs to a single micro-tet.
    """
    n2 = 2 ** (level + 1)
    key = np.asarray(key, dtype=np.int64)
    acc, face_count = {}, {}
    for c in range(len(cells)):
        cid = np.asarray(cells[c])
        w = np.zeros(4, dtype=np.int64)
        outside = False
        for gid, wt in zip(key[0::2], key[1::2]):
            if gid < 0:
                continue
            hit = np.flatnonzero(cid == gid)
            if len(hit) == 0:
                outside = True
                break
            w[hit[0]] = wt
        if outside:
            continue
        tets = (n2 * np.eye(4, dtype=np.int64))[None]   # level-l weights x 2
        for _ in range(level):
            tets = refine_once(tets)
            tets = tets[_contains(tets, w)]
        nodes = np.concatenate(
            [tets, np.stack([(tets[:, a] + tets[:, b]) // 2 for a, b in EDGES],
                            axis=1)], axis=1)                    # [m, 10, 4]
        is_node = (nodes == w[None, None, :]).all(axis=2)
        sel = is_node.any(axis=1)
        nodes, is_node = nodes[sel], is_node[sel]
        if len(nodes) == 0:
            continue
        nkeys = keys_of(cid, nodes)                               # [m, 10, 8]
        P = key_coordinates(macro_xyz, nkeys[:, :4], n2)
        K, _ = element_stiffness_p2(P)
        for t in range(len(nodes)):
            a = int(np.flatnonzero(is_node[t])[0])
            nk = [tuple(nkeys[t, q]) for q in range(10)]
            for b in range(10):
                acc[nk[b]] = acc.get(nk[b], 0.0) + K[t, a, b]
            for drop in range(4):
                face = [q for q in range(4) if q != drop]
                fnodes = face + [4 + e for e, (p, r) in enumerate(EDGES)
                                 if p != drop and r != drop]
                if a not in fnodes:
                    continue
                f = tuple(sorted(nk[q] for q in face))
                face_count[f] = face_count.get(f, 0) + 1
    nbr = np.array(sorted(acc), dtype=np.int64).reshape(-1, 8)
    vals = np.array([acc[tuple(k)] for k in nbr])
    dirichlet = any(v == 1 for v in face_count.values())
    return nbr, vals, dirichlet


# ------------------------------------------------- subgroup arrays (AoS/SoA) --
# The micro-primitive subgroups of a P2 function on one cell (subgroup table):
# the micro-vertices (width 2^l + 1) and the seven micro-edge subgroups x, y,
# z, xy, xz, yz (width 2^l) and xyz (width 2^l - 1).  Subgroup g at index
# (i, j, k) is the node at fine coordinates 2 (i, j, k) + SUBGROUP_SHIFT[g]:
# the micro-vertex itself, or the midpoint of the micro-edge of that
# direction based there (x: (i,j,k)-(i+1,j,k); xy: (i+1,j,k)-(i,j+1,k); xyz:
# (i,j+1,k)-(i+1,j,k+1), the refinement's inner diagonal).
SUBGROUPS = ("vertex", "x", "y", "z", "xy", "xz", "yz", "xyz")
SUBGROUP_SHIFT = ((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1),
                  (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1))


def subgroup_width(g: int, level: int) -> int:
    n = 2 ** level
    return n + 1 if g == 0 else (n - 1 if g == 7 else n)


def subgroup_arrays(cells, level: int, value_of_keys, m: int, layout: str):
    """Pack a P2 function with m components into the paper's per-cell arrays.

    ``value_of_keys(keys [p, 8]) -> [p, m]`` gives the components at nodes
    identified by their level-(level + 1) keys.  For every cell, in cell
    order, and every subgroup in SUBGROUPS order, the structures of the
    subgroup's micro-primitives are visited in the loop order k, j, i of the
    index polytope, which is the order of t_w (Section 4); the subgroup array
    holds them either as structures one after the other (AoS: element
    m t_w + d) or component by component (SoA: element d N_tet(w) + t_w).
    Returns one flat array: cells, then subgroups, each of m N_tet(w)."""
    assert layout in ("aos", "soa")
    n2 = 2 ** (level + 1)
    out = []
    for c in range(len(cells)):
        cid = np.asarray(cells[c])
        for g in range(8):
            w = subgroup_width(g, level)
            pts = [(i, j, k) for k in range(w) for j in range(w - k)
                   for i in range(w - k - j)]
            if not pts:
                continue
            sh = np.array(SUBGROUP_SHIFT[g])
            fine = 2 * np.array(pts) + sh                       # [p, 3]
            wts = np.concatenate([n2 - fine.sum(axis=1, keepdims=True), fine], axis=1)
            vals = np.asarray(value_of_keys(keys_of(cid, wts)))  # [p, m]
            out.append(vals.reshape(-1) if layout == "aos" else vals.T.reshape(-1))
    return np.concatenate(out)
