"""Explicit regular refinement of tetrahedral macro-cells (oracle, test-only).

Follows Section 3.1 of the paper: a tetrahedron [v0, v1, v2, v3] is split into
the eight children T1..T8 of eq. (bey), whose vertices are the parent vertices
and the six edge midpoints v_ab, in exactly the printed order; the rule is
applied recursively, level times.

Points are kept as integer barycentric weights on the four macro-cell
vertices, scaled so that they sum to n = 2**level.  A midpoint is the sum of two
weight vectors halved, which is exact in integers.  A micro-vertex of the
conforming global mesh is identified by its *key*: the (global macro-vertex
id, weight) pairs with non-zero weight, in ascending id order, padded with
(-1, 0) to four pairs.  Two macro-cells that share a face, edge or vertex give
the same key to every micro-vertex on it, because refinement is conforming
(end of Section 3.1).
"""
from __future__ import annotations

import numpy as np

# eq. (bey): vertices of T1..T8, (a, a) = v_a and (a, b) = midpoint v_ab.
BEY_CHILDREN = (
    ((0, 0), (0, 1), (0, 2), (0, 3)),  # T1
    ((0, 1), (1, 1), (1, 2), (1, 3)),  # T2
    ((0, 2), (1, 2), (2, 2), (2, 3)),  # T3
    ((0, 3), (1, 3), (2, 3), (3, 3)),  # T4
    ((0, 1), (0, 2), (0, 3), (1, 3)),  # T5
    ((0, 1), (0, 2), (1, 2), (1, 3)),  # T6
    ((0, 2), (0, 3), (1, 3), (2, 3)),  # T7
    ((0, 2), (1, 2), (1, 3), (2, 3)),  # T8
)


def point_of(tets: np.ndarray, a: int, b: int) -> np.ndarray:
    """Vertex a (a == b) or midpoint of edge (a, b) of every tet, as weights."""
    if a == b:
        return tets[:, a]
    s = tets[:, a] + tets[:, b]
    assert not (s % 2).any(), "midpoint weights must stay integral"
    return s // 2


def refine_once(tets: np.ndarray) -> np.ndarray:
    """Apply eq. (bey) to every tet. ``tets``: int64 [m, 4 vertices, 4 weights].

    Returns [8m, 4, 4]; the children of tet t are rows 8t .. 8t+7 (T1..T8).
    """
    children = [np.stack([point_of(tets, a, b) for (a, b) in child], axis=1)
                for child in BEY_CHILDREN]
    return np.stack(children, axis=1).reshape(-1, 4, 4)


def reference_refinement(level: int) -> np.ndarray:
    """Micro-tets of one macro-cell after ``level`` refinements, as local
    barycentric weights summing to 2**level.  Shape [8**level, 4, 4]."""
    n = 2 ** level
    tets = (n * np.eye(4, dtype=np.int64))[None]
    for _ in range(level):
        tets = refine_once(tets)
    return tets


def local_index(weights: np.ndarray) -> np.ndarray:
    """(i, j, k) of a point = its weights on local vertices 1, 2, 3."""
    return weights[..., 1:]


# ---------------------------------------------------------------- keys --
def keys_of(cell_ids: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """Keys of points given by local ``weights`` [..., 4] in a macro-cell whose
    global vertex ids are ``cell_ids`` [4].  Returns int64 [..., 8]."""
    order = np.argsort(cell_ids)
    ids = cell_ids[order]
    w = weights[..., order]
    # non-zero weights first, ascending id kept among them (stable order)
    rank = np.where(w > 0, 0, 4) + np.arange(4)
    perm = np.argsort(rank, axis=-1, kind="stable")
    w_sorted = np.take_along_axis(w, perm, axis=-1)
    id_sorted = np.broadcast_to(ids, w.shape)
    id_sorted = np.take_along_axis(id_sorted, perm, axis=-1)
    id_sorted = np.where(w_sorted > 0, id_sorted, -1)
    out = np.empty(w.shape[:-1] + (8,), dtype=np.int64)
    out[..., 0::2] = id_sorted
    out[..., 1::2] = w_sorted
    return out


def key_codec(num_vertices: int, n: int):
    """Order-preserving packing of key rows into one int64 if it fits.

    Digits are (id + 1) in [0, nv] and weight in [0, n]; lexicographic order of
    key rows equals numeric order of the codes.  Returns (encode, decode) or
    None when the code would overflow int64.
    """
    V, W = num_vertices + 1, n + 1
    if V ** 4 * W ** 4 >= 2 ** 62:
        return None

    def encode(keys):
        code = np.zeros(keys.shape[:-1], dtype=np.int64)
        for p in range(4):
            code = code * V + (keys[..., 2 * p] + 1)
            code = code * W + keys[..., 2 * p + 1]
        return code

    def decode(code):
        code = np.array(code, dtype=np.int64)
        out = np.empty(code.shape + (8,), dtype=np.int64)
        for p in reversed(range(4)):
            out[..., 2 * p + 1] = code % W
            code = code // W
            out[..., 2 * p] = code % V - 1
            code = code // V
        return out

    return encode, decode


def unique_rows(rows: np.ndarray):
    """Lexicographically sorted unique rows and the inverse map."""
    rows = np.ascontiguousarray(rows)
    order = np.lexsort(rows.T[::-1])
    srt = rows[order]
    new = np.ones(len(srt), dtype=bool)
    new[1:] = (srt[1:] != srt[:-1]).any(axis=1)
    uniq = srt[new]
    inv = np.empty(len(rows), dtype=np.int64)
    inv[order] = np.cumsum(new) - 1
    return uniq, inv


def key_coordinates(macro_xyz: np.ndarray, keys: np.ndarray, n: int):
    """Physical position of keyed points: sum over pairs of w * X_id / n."""
    ids = keys[..., 0::2]
    w = keys[..., 1::2].astype(np.float64)
    X = np.asarray(macro_xyz)[np.where(ids >= 0, ids, 0)]
    return (w[..., None] * X).sum(axis=-2) / n


# ---------------------------------------------------------- micro mesh --
class MicroMesh:
    """The globally conforming micro-mesh of a coarse mesh at one level.

    Attributes
    ----------
    level, n          refinement level and n = 2**level
    keys   [N, 8]     keys of the unique micro-vertices, canonical (sorted)
    xyz    [N, 3]     coordinates sum_q w_q X_q / n over the key's pairs
    tets   [M, 4]     micro-tets as vertex indices, local vertex order of
                      eq. (bey); tets of macro-cell c are rows c*8**l ..
    tet_cell [M]      macro-cell of every micro-tet
    local  [8**l,4,4] local weights of the reference refinement
    """

    def __init__(self, xyz: np.ndarray, cells: np.ndarray, level: int):
        self.level = int(level)
        self.n = 2 ** self.level
        self.macro_xyz = np.asarray(xyz, dtype=np.float64)
        self.cells = np.asarray(cells, dtype=np.int64)
        nc = len(self.cells)
        self.local = reference_refinement(self.level)
        codec = key_codec(len(self.macro_xyz), self.n)
        per_cell = [keys_of(self.cells[c], self.local) for c in range(nc)]
        allkeys = np.concatenate(per_cell).reshape(-1, 8)
        del per_cell
        if codec is not None:
            encode, decode = codec
            codes = encode(allkeys)
            del allkeys
            ucodes, inv = np.unique(codes, return_inverse=True)
            self.keys = decode(ucodes)
            self.codes = ucodes
        else:
            self.keys, inv = unique_rows(allkeys)
            self.codes = None
        self._codec = codec
        self.tets = inv.reshape(-1, 4).astype(np.int64)
        self.tet_cell = np.repeat(np.arange(nc), len(self.local))
        self.xyz = self.coordinates(self.keys)

    # -- helpers ---------------------------------------------------------
    @property
    def num_vertices(self) -> int:
        return len(self.keys)

    def coordinates(self, keys: np.ndarray) -> np.ndarray:
        return key_coordinates(self.macro_xyz, keys, self.n)

    def index_of(self, keys: np.ndarray) -> np.ndarray:
        """Vertex indices of the given keys (every key must exist)."""
        keys = np.asarray(keys, dtype=np.int64)
        if self._codec is not None:
            c = np.asarray(self._codec[0](keys))
            shape = c.shape
            c = c.reshape(-1)
            idx = np.searchsorted(self.codes, c)
            ok = (idx < len(self.codes))
            ok[ok] = self.codes[idx[ok]] == c[ok]
            idx, ok = idx.reshape(shape), ok.reshape(shape)
        else:
            flat = keys.reshape(-1, 8)
            table = {tuple(r): i for i, r in enumerate(self.keys)}
            idx = np.array([table.get(tuple(r), -1) for r in flat])
            ok = idx >= 0
            idx = idx.reshape(keys.shape[:-1])
            ok = ok.reshape(keys.shape[:-1])
        if not ok.all():
            raise KeyError("key not present in the micro-mesh")
        return idx

    def cell_keys(self, c: int, weights: np.ndarray) -> np.ndarray:
        """Keys of points with local weights in macro-cell c."""
        return keys_of(self.cells[c], weights)

    def edges(self) -> np.ndarray:
        """Unique micro-edges as sorted vertex pairs."""
        pairs = [(a, b) for a in range(4) for b in range(a + 1, 4)]
        e = np.concatenate([np.sort(self.tets[:, [a, b]], axis=1)
                            for a, b in pairs])
        return unique_rows(e)[0]

    def faces(self, return_counts: bool = False):
        """Unique micro-faces as sorted vertex triples (and incidence counts)."""
        f = np.concatenate([np.sort(np.delete(self.tets, q, axis=1), axis=1)
                            for q in range(4)])
        uniq, inv = unique_rows(f)
        if return_counts:
            return uniq, np.bincount(inv, minlength=len(uniq))
        return uniq
