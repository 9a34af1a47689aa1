"""GPU parity of the P2 operator (ht_apply_p2) against the P2 oracle.

Small meshes: the whole result against the oracle's assembled matrix, FP64
and FP32, including a single cell at P2 level 6 (fine lattice n = 128: two
bulk tiles in i with a ragged tail, and rows of every length).  Full size
(the 288-cell box at P2 level 7, the workload of the P2 bench line): rows at
sampled points against the oracle's single-row assembly, plus properties
that hold at any size: affine fields are annihilated on interior nodes, the
interior operator is symmetric, and a quadratic field gives the oracle's
load vector at its interior nodes.  The subgroup arrays (AoS / SoA) of
ht_p2_pack against the oracle's, bit-exact, and ht_p2_unpack as its inverse.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2308_01792_amd as ht  # noqa: E402
from paper_2308_01792_amd import _lib  # noqa: E402
from oracle.p2 import P2System, p2_row_at  # noqa: E402
from tests.conftest import mesh_by_name  # noqa: E402


class P2Pair:
    """Library mesh (levels up to P2 level + 1) and the P2 oracle."""

    def __init__(self, name, level):
        self.level = level
        self.xyz, self.cells = mesh_by_name(name)
        self.S = P2System(self.xyz, self.cells, level)
        self.m = ht.Mesh(self.xyz, self.cells, level + 1, level + 1)
        keys, self.flags = self.m.keys(level + 1)
        self.idx = np.full(len(keys), -1, dtype=np.int64)
        real = self.flags != _lib.HT_SLOT_PAD
        self.idx[real] = self.S.index_of(keys[real])

    def to_gpu(self, v, dtype):
        out = np.zeros(len(self.idx))
        out[self.idx >= 0] = v[self.idx[self.idx >= 0]]
        return torch.tensor(out, dtype=dtype, device="cuda")

    def from_gpu(self, t):
        v = t.double().cpu().numpy()
        own = (self.flags & _lib.HT_SLOT_OWNER) > 0
        out = np.zeros(self.S.num_nodes)
        out[self.idx[own]] = v[own]
        real = self.idx >= 0
        assert np.array_equal(v[real], out[self.idx[real]]), \
            "ghost copies differ from their owner"
        return out


CASES = [("ref_tet", 0), ("ref_tet", 1), ("ref_tet", 3), ("kuhn_211", 2),
         ("jittered_222", 2), ("jittered_288", 1), ("slab_3_11", 2),
         ("slab_1_1", 2), ("ref_tet", 6)]


@pytest.mark.parametrize("name,level", CASES)
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12),
                                       (torch.float32, 2e-5)])
def test_p2_apply_matches_oracle(name, level, dtype, tol):
    print(f"p2 apply {name} level {level} {dtype}", flush=True)
    p = P2Pair(name, level)
    rng = np.random.default_rng(17 + level)
    x = rng.uniform(-1, 1, p.S.num_nodes)
    want = p.S.apply(x)
    xg = p.to_gpu(x, dtype)
    y = torch.full_like(xg, float("nan"))
    p.m.apply_p2(level, xg, y)
    torch.cuda.synchronize()
    got = p.from_gpu(y)
    scale = np.abs(p.S.A) @ np.abs(x)
    assert np.all(np.abs(got - want) <= tol * scale + 1e-300), \
        np.abs(got - want).max()
    assert np.all(got[p.S.dirichlet] == 0.0)
    p.m.close()


def test_p2_apply_is_deterministic():
    p = P2Pair("jittered_222", 3)
    x = p.to_gpu(np.random.default_rng(2).uniform(-1, 1, p.S.num_nodes),
                 torch.float64)
    y1, y2 = torch.empty_like(x), torch.empty_like(x)
    p.m.apply_p2(3, x, y1)
    p.m.apply_p2(3, x, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    p.m.close()


def test_p2_level_errors():
    xyz, cells = mesh_by_name("ref_tet")
    m = ht.Mesh(xyz, cells, 1, 3)
    x = torch.zeros(m.n_slots(3), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    for lvl in (-1, 3):
        with pytest.raises(ht.HytetError) as e:
            m.apply_p2(lvl, x, y)
        assert e.value.code == _lib.HT_ERR_LEVEL
    with pytest.raises(ht.HytetError):
        m.apply_p2(2, x, x)
    m.close()


# ------------------------------------------------------------ full size --
FULL_LEVEL = 7


@pytest.fixture(scope="module")
def box():
    xyz, cells = mesh_by_name("jittered_288")
    m = ht.Mesh(xyz, cells, FULL_LEVEL + 1, FULL_LEVEL + 1)
    yield xyz, cells, m
    m.close()
    torch.cuda.empty_cache()


def _points(n):
    pts = []
    for c in (0, 97, 287):
        pts += [(c, 1, 1, 1), (c, 2, 2, 2), (c, 3, 4, 5), (c, n // 2, n // 3, n // 7),
                (c, 1, 1, n - 3), (c, n - 3, 1, 1), (c, 125, 126, n - 252),
                (c, 0, 5, n - 9), (c, 5, 0, n - 9), (c, n - 14, 5, 9),
                (c, 0, 0, n // 2), (c, 3, 0, 0), (c, 127, 3, 2)]
    # face points at the borders of the face kernel's tiles (8 planes x 128
    # rows): rows 127 / 128 / 129 and planes 7 / 8 / 9, both faces
    for (j, k) in ((127, 7), (128, 8), (129, 9), (1, 8), (126, 15), (128, 16),
                   (n - 18, 16), (3, n - 5)):
        if j + k <= n - 1:
            pts += [(97, 0, j, k), (97, n - j - k, j, k)]
    rng = np.random.default_rng(43)
    while len(pts) < 76:
        i, j, k = rng.integers(0, n + 1, size=3)
        if i + j + k <= n:
            pts.append((int(rng.integers(0, 288)), int(i), int(j), int(k)))
    return pts


def _slot_of_key(m, cells, level, key):
    """Owner slot of a key: its copy in the lowest-numbered cell."""
    ids, wts = key[0::2], key[1::2]
    nz = ids >= 0
    hit = np.flatnonzero(np.isin(cells, ids[nz]).sum(axis=1) == nz.sum())
    c = int(hit[0])
    loc = np.zeros(4, dtype=np.int64)
    for gid, wt in zip(ids[nz], wts[nz]):
        loc[list(cells[c]).index(gid)] = wt
    return m.slot_index(level, c, int(loc[1]), int(loc[2]), int(loc[3]))


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12),
                                       (torch.float32, 2e-5)])
def test_p2_sampled_rows_full_size(box, dtype, tol):
    xyz, cells, m = box
    fine = FULL_LEVEL + 1
    n = 2 ** fine
    g = torch.Generator(device="cuda").manual_seed(9)
    x = (torch.rand(m.n_slots(fine), dtype=torch.float64, device="cuda",
                    generator=g) * 2 - 1)
    m.sync(fine, x)
    x = x.to(dtype)
    y = torch.full_like(x, float("nan"))
    m.apply_p2(FULL_LEVEL, x, y)
    torch.cuda.synchronize()
    checked = 0
    for (c, i, j, k) in _points(n):
        slot = m.slot_index(fine, c, i, j, k)
        key, _ = m.keys(fine, slot, 1)
        nbr, vals, dirichlet = p2_row_at(xyz, cells, FULL_LEVEL, key[0])
        got = float(y[slot].double())
        if dirichlet:
            assert got == 0.0
            continue
        ns = np.array([_slot_of_key(m, cells, fine, kk) for kk in nbr])
        xv = x[torch.as_tensor(ns, device="cuda")].double().cpu().numpy()
        want = float(vals @ xv)
        assert abs(got - want) <= tol * float(np.abs(vals) @ np.abs(xv)), \
            ((c, i, j, k), got, want)
        checked += 1
    assert checked >= 40
    del x, y


def _interior_owner(m, level):
    f = torch.zeros(m.n_slots(level), dtype=torch.uint8, device="cuda")
    m.flags_device(level, f)
    return ((f & ht.HT_SLOT_OWNER) > 0) & ((f & ht.HT_SLOT_DIRICHLET) == 0)


def test_p2_affine_annihilated_and_symmetric_full_size(box):
    _, _, m = box
    fine = FULL_LEVEL + 1
    X = torch.zeros(3 * m.n_slots(fine), dtype=torch.float64, device="cuda")
    m.coords_device(fine, X)
    X = X.view(-1, 3)
    u = 0.4 + 0.3 * X[:, 0] - 1.2 * X[:, 1] + 0.7 * X[:, 2]
    del X
    y = torch.full_like(u, float("nan"))
    m.apply_p2(FULL_LEVEL, u, y)
    inner = _interior_owner(m, fine)
    W = m.p2_stencils(FULL_LEVEL)
    bound = 1e-12 * 40 * np.abs(W).sum(axis=3).max() * u.abs().max().item()
    assert y[inner].abs().max().item() <= bound
    # symmetry of the interior operator: <A a, b> = <a, A b> over unique
    # interior nodes, with a and b zero at Dirichlet nodes
    g = torch.Generator(device="cuda").manual_seed(4)
    a = torch.rand(m.n_slots(fine), dtype=torch.float64, device="cuda", generator=g)
    b = torch.rand(m.n_slots(fine), dtype=torch.float64, device="cuda", generator=g)
    for v in (a, b):
        m.sync(fine, v)
        m.fill_dirichlet(fine, v, 0.0)
    Aa, Ab = torch.empty_like(a), torch.empty_like(b)
    m.apply_p2(FULL_LEVEL, a, Aa)
    m.apply_p2(FULL_LEVEL, b, Ab)
    lhs = torch.sum(Aa[inner] * b[inner]).item()
    rhs = torch.sum(a[inner] * Ab[inner]).item()
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    del u, y, inner, a, b, Aa, Ab
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name,level", [("jittered_222", 3), ("slab_3_11", 2)])
def test_p2_quadratic_gives_the_load(name, level):
    """For quadratic u, (A u)_i = f times the integral of phi_i at interior
    nodes (f = -Laplace u): the oracle's load vector, on the GPU's result."""
    p = P2Pair(name, level)
    Q = np.array([[1.0, 0.3, -0.2], [0.3, -0.5, 0.4], [-0.2, 0.4, 0.8]])
    b = np.array([0.2, -0.7, 0.5])
    X = p.S.xyz
    u = 0.1 + X @ b + np.einsum("pi,ij,pj->p", X, Q, X)
    f = -2.0 * np.trace(Q)
    y = torch.empty(len(p.idx), dtype=torch.float64, device="cuda")
    p.m.apply_p2(level, p.to_gpu(u, torch.float64), y)
    got = p.from_gpu(y)
    I = p.S.interior
    assert np.abs(got[I] - f * p.S.load[I]).max() <= \
        1e-11 * np.abs(p.S.A).max() * np.abs(u).max()
    p.m.close()


# ------------------------------------------------------ subgroup arrays --
@pytest.mark.parametrize("layout", ["aos", "soa"])
@pytest.mark.parametrize("name,level,m,dtype", [
    ("jittered_222", 2, 3, torch.float64), ("ref_tet", 3, 1, torch.float64),
    ("slab_3_11", 1, 2, torch.float32), ("ref_tet", 0, 2, torch.float64)])
def test_p2_subgroup_arrays_match_oracle(name, level, m, dtype, layout):
    """ht_p2_pack against the oracle's per-cell subgroup arrays (t_w order,
    AoS / SoA), bit-exact; ht_p2_unpack restores every non-padding slot."""
    from oracle.p2 import subgroup_arrays
    p = P2Pair(name, level)
    vals = np.random.default_rng(8).uniform(-1, 1, (p.S.num_nodes, m))
    vals = vals.astype(np.float32).astype(np.float64) if dtype == torch.float32 else vals
    lat = torch.cat([p.to_gpu(vals[:, d], dtype) for d in range(m)])
    arr = p.m.p2_pack(level, lat, m, layout)
    torch.cuda.synchronize()
    want = subgroup_arrays(p.cells, level, lambda keys: vals[p.S.index_of(keys)],
                           m, layout)
    assert np.array_equal(arr.double().cpu().numpy(), want)
    back = torch.full_like(lat, float("nan"))
    p.m.p2_unpack(level, arr, back, m, layout)
    real = torch.as_tensor(np.tile(p.idx >= 0, m), device="cuda")
    assert torch.equal(back[real], lat[real])
    p.m.close()


# ------------------------------------------------------------ max level --
def test_p2_sampled_rows_at_the_largest_level():
    """P2 level 9 (the level-10 lattice, the largest the library accepts):
    three jittered cells sharing faces and an edge, rows at points spread
    over the cell blocks and their far ends against the single-row oracle."""
    from workloads import slab
    level = 9
    fine = level + 1
    n = 2 ** fine
    xyz, cells = slab(1, 3, amplitude=0.1, seed=7)
    m = ht.Mesh(xyz, cells, fine, fine)
    g = torch.Generator(device="cuda").manual_seed(12)
    x = torch.rand(m.n_slots(fine), dtype=torch.float64, device="cuda",
                   generator=g) * 2 - 1
    m.sync(fine, x)
    y = torch.full_like(x, float("nan"))
    m.apply_p2(level, x, y)
    torch.cuda.synchronize()
    pts = []
    for c in range(3):
        pts += [(c, 1, 1, 1), (c, 2, 1, 1), (c, 1, 2, 1), (c, 1, 1, 2),
                (c, n // 2, n // 3, n // 7), (c, 1, 1, n - 3), (c, n - 3, 1, 1),
                (c, 1, n - 3, 1), (c, 125, 126, n - 252), (c, 0, 5, n - 9),
                (c, 5, 0, n - 9), (c, n - 14, 5, 9), (c, 0, 0, n // 2),
                (c, 3, n - 5, 1), (c, n - 4, 2, 1)]
    checked = 0
    for (c, i, j, k) in pts:
        slot = m.slot_index(fine, c, i, j, k)
        key, _ = m.keys(fine, slot, 1)
        nbr, vals, dirichlet = p2_row_at(xyz, cells, level, key[0])
        got = float(y[slot])
        if dirichlet:
            assert got == 0.0
            continue
        ns = np.array([_slot_of_key(m, cells, fine, kk) for kk in nbr])
        xv = x[torch.as_tensor(ns, device="cuda")].cpu().numpy()
        want = float(vals @ xv)
        assert abs(got - want) <= 1e-12 * float(np.abs(vals) @ np.abs(xv)), \
            ((c, i, j, k), got, want)
        checked += 1
    assert checked >= 20
    del x, y
    m.close()
    torch.cuda.empty_cache()
