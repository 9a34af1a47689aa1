"""Full-size checks on the 288-cell jittered box at level 8 (802,687,743
DoFs), with the tile shapes the autotuner picks, i.e. the launch
configuration the benchmark times.

The assembled oracle cannot reach level 8, so results are checked in two
ways:

* sampled outputs: rows of the stiffness matrix at chosen micro-vertices
  are assembled one by one by the oracle (``oracle.rows.row_at``, element
  matrices of the micro-tets around the point, Section 5.2.1), and applied
  to the same input values the GPU read;
* properties that hold at any size: affine fields are annihilated on
  interior rows, quadratic fields give -Laplace(u) times the lumped mass
  at cell-interior points, A is symmetric, restriction is the transpose of
  prolongation, and a V(2,2) solve reaches 1e-10 in both precisions.

The variable-coefficient operator div(k grad) gets the same treatment:
sampled rows (the oracle's row with the coefficient values the GPU read)
and constants annihilated on interior rows.

Inputs are drawn with torch's generator on the device; the oracle reads
them at owner copies, which no library kernel writes.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2308_01792_amd as ht  # noqa: E402
from oracle.rows import row_at  # noqa: E402
from workloads import jittered_kuhn_box  # noqa: E402

LEVEL = 8
N = 2 ** LEVEL
FP64_TOL = 1e-12
FP32_TOL = 1e-5
OMEGA = 2.0 / 3.0


class Big:
    def __init__(self):
        self.xyz, self.cells = jittered_kuhn_box(4, 4, 3, amplitude=0.1, seed=3)
        self.m = ht.Mesh(self.xyz, self.cells, 2, LEVEL)
        self.rows64 = self.m.autotune(LEVEL, ht.HT_F64)
        self.rows32 = self.m.autotune(LEVEL, ht.HT_F32)
        self.nslot = self.m.n_slots(LEVEL)

    def interior_mask(self, level=LEVEL):
        f = torch.zeros(self.m.n_slots(level), dtype=torch.uint8, device="cuda")
        self.m.flags_device(level, f)
        return ((f & ht.HT_SLOT_OWNER) > 0) & ((f & ht.HT_SLOT_DIRICHLET) == 0)

    def rand(self, seed, dtype=torch.float64, level=LEVEL, zero_boundary=False):
        g = torch.Generator(device="cuda").manual_seed(seed)
        v = torch.rand(self.m.n_slots(level), dtype=dtype, device="cuda",
                       generator=g) * 2 - 1
        self.m.sync(level, v)
        if zero_boundary:
            self.m.fill_dirichlet(level, v, 0.0)
        return v

    def slot_of_key(self, key):
        """Owner slot of a micro-vertex: its copy in the lowest-numbered cell
        whose vertices include every macro-vertex of the key."""
        ids, wts = key[0::2], key[1::2]
        nz = ids >= 0
        hit = np.flatnonzero(np.isin(self.cells, ids[nz]).sum(axis=1) == nz.sum())
        c = int(hit[0])
        loc = np.zeros(4, dtype=np.int64)
        for gid, wt in zip(ids[nz], wts[nz]):
            loc[list(self.cells[c]).index(gid)] = wt
        return self.m.slot_index(LEVEL, c, int(loc[1]), int(loc[2]), int(loc[3]))

    @staticmethod
    def gather(v, slots):
        idx = torch.as_tensor(np.asarray(slots, dtype=np.int64), device="cuda")
        return v[idx].double().cpu().numpy()

    @staticmethod
    def dot(a, b, mask):
        return float((a.double()[mask] * b.double()[mask]).sum())


@pytest.fixture(scope="module")
def big():
    B = Big()
    yield B
    B.m.close()
    torch.cuda.empty_cache()


def sample_points(seed=21, random_count=60):
    """(cell, i, j, k) points: tile and wave boundaries of the stencil kernel
    (62 outputs per 64-lane tile, rows stacked per wave), the four faces,
    the six edges and the vertices of a cell, plus random points."""
    n = N
    pts = []
    for c in (0, 143, 287):
        pts += [(c, 1, 1, 1), (c, 61, 1, 1), (c, 62, 1, 1), (c, 63, 1, 1),
                (c, 123, 3, 2), (c, 124, 4, 1), (c, 125, 5, 7), (c, 186, 8, 9),
                (c, 1, 15, 16), (c, 1, 16, 16), (c, 2, 31, 1), (c, 2, 32, 1),
                (c, 3, 63, 64), (c, 7, 64, 3), (c, 200, 20, 30),
                (c, 0, 5, 5), (c, 5, 0, 5), (c, 5, 5, 0), (c, n - 15, 5, 10),
                (c, 0, 0, 5), (c, 0, 5, 0), (c, 5, 0, 0), (c, 0, 9, n - 9),
                (c, 9, 0, n - 9), (c, 9, n - 9, 0),
                (c, 0, 0, 0), (c, n, 0, 0), (c, 0, n, 0), (c, 0, 0, n),
                (c, 1, 1, n - 3), (c, n - 3, 1, 1), (c, 1, n - 3, 1)]
    rng = np.random.default_rng(seed)
    while len(pts) < 96 + random_count:
        i, j, k = rng.integers(0, n + 1, size=3)
        if i + j + k <= n:
            pts.append((int(rng.integers(0, 288)), int(i), int(j), int(k)))
    return pts


class Row:
    def __init__(self, slot, own, nslots, vals, dirichlet):
        self.slot, self.own = slot, own
        self.nslots, self.vals, self.dirichlet = nslots, vals, dirichlet
        self.diag = float(vals[np.flatnonzero(nslots == own)[0]])


@pytest.fixture(scope="module")
def rows(big):
    """Oracle rows at the sample points."""
    out = []
    for (c, i, j, k) in sample_points():
        slot = big.m.slot_index(LEVEL, c, i, j, k)
        key, _ = big.m.keys(LEVEL, slot, 1)
        nbr, vals, dirichlet = row_at(big.xyz, big.cells, LEVEL, key[0])
        nslots = np.array([big.slot_of_key(kk) for kk in nbr])
        out.append(Row(slot, big.slot_of_key(key[0]), nslots, vals, dirichlet))
    return out


def test_sample_rows_cover_every_kind_of_point(rows):
    assert sum(r.dirichlet for r in rows) >= 10
    assert sum(not r.dirichlet for r in rows) >= 100
    assert {15, 27} & {len(r.vals) for r in rows if not r.dirichlet}
    assert all(r.diag > 0 for r in rows)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_apply_sampled_rows(big, rows, dtype):
    tdt = torch.float64 if dtype == "f64" else torch.float32
    tol = FP64_TOL if dtype == "f64" else FP32_TOL
    x = big.rand(4, tdt)
    y = torch.full_like(x, float("nan"))
    big.m.apply(LEVEL, x, y)
    got = big.gather(y, [r.slot for r in rows])
    got_own = big.gather(y, [r.own for r in rows])
    assert np.isfinite(got).all()
    assert np.array_equal(got, got_own)          # consistent copies
    for r, g in zip(rows, got):
        xv = big.gather(x, r.nslots)
        want = 0.0 if r.dirichlet else float(r.vals @ xv)
        assert abs(g - want) <= tol * float(np.abs(r.vals) @ np.abs(xv)), \
            (r.slot, g, want)
    del x, y
    torch.cuda.empty_cache()


def test_residual_norm_and_jacobi_sampled_rows(big, rows):
    u, b = big.rand(7), big.rand(8)
    r = torch.zeros_like(u)
    nrm = big.m.residual(LEVEL, u, b, r, want_norm=True)
    # neighbour values before the sweep, then one Jacobi sweep in place
    before = [(big.gather(u, row.nslots), big.gather(u, [row.own])[0],
               big.gather(b, [row.own])[0]) for row in rows]
    res = big.gather(r, [row.slot for row in rows])
    big.m.smooth_jacobi(LEVEL, u, b, OMEGA, 1)
    after = big.gather(u, [row.slot for row in rows])
    for row, (uv, ui, bi), ri, u1 in zip(rows, before, res, after):
        scale = abs(bi) + float(np.abs(row.vals) @ np.abs(uv))
        if row.dirichlet:
            assert ri == 0.0 and u1 == ui
            continue
        want_r = bi - float(row.vals @ uv)
        assert abs(ri - want_r) <= FP64_TOL * scale
        want_u = ui + OMEGA * want_r / row.diag
        assert abs(u1 - want_u) <= FP64_TOL * (abs(ui) + scale / row.diag)
    # the norm over unique interior DoFs, summed independently by torch
    ref = torch.sqrt((r[big.interior_mask()] ** 2).sum()).item()
    assert abs(nrm - ref) <= 1e-12 * ref
    del u, b, r
    torch.cuda.empty_cache()


def _affine(X, coef, c0):
    """c0 + coef . X, elementwise (a GEMV over ~8e8 rows is avoided: torch's
    matmul returned wrong rows at this size on the test machine)."""
    return X[:, 0] * coef[0] + X[:, 1] * coef[1] + X[:, 2] * coef[2] + c0


def test_affine_fields_are_annihilated(big):
    """P1 reproduces affine functions: (A u)_i = 0 on every interior row."""
    X = torch.zeros(3 * big.nslot, dtype=torch.float64, device="cuda")
    big.m.coords_device(LEVEL, X)
    X = X.view(-1, 3)
    mask = big.interior_mask()
    stencil_sum = np.abs(big.m.cell_stencils(LEVEL)).sum(axis=2).max()
    for coef, c0 in (((0.0, 0.0, 0.0), 1.0), ((0.3, -1.2, 0.7), 0.4)):
        u = _affine(X, coef, c0)
        y = torch.full_like(u, float("nan"))
        big.m.apply(LEVEL, u, y)
        worst = y[mask].abs().max().item()
        # a shared row sums the partial rows of up to ~24 incident cells
        assert worst <= FP64_TOL * 30 * stencil_sum * u.abs().max().item()
        del u, y
    del X
    torch.cuda.empty_cache()


def test_quadratic_field_at_cell_interior(big):
    """At points whose micro-tets all lie in one macro-cell, the row applied
    to a quadratic u gives -Laplace(u) times the lumped mass exactly."""
    X = torch.zeros(3 * big.nslot, dtype=torch.float64, device="cuda")
    big.m.coords_device(LEVEL, X)
    X = X.view(-1, 3)
    H = ((2.0, 0.3, -0.5), (0.3, 1.0, 0.7), (-0.5, 0.7, -1.5))
    u = _affine(X, (0.3, -0.2, 0.1), 0.7)
    for a in range(3):
        for b in range(3):
            u += (0.5 * H[a][b]) * X[:, a] * X[:, b]
    del X
    umax = u.abs().max().item()
    y = torch.zeros_like(u)
    big.m.apply(LEVEL, u, y)
    del u
    m = torch.zeros_like(y)
    big.m.lumped_mass(LEVEL, m)
    # cell-interior points: the main block of every cell, i + j + k < n with
    # i, j, k >= 1; sample whole cells through their slot index range
    lap = H[0][0] + H[1][1] + H[2][2]
    # rounding bound: 15 products of size |w| |u| per row
    row_scale = np.abs(big.m.cell_stencils(LEVEL)[:, 0]).sum(axis=1).max() * umax
    for c in (0, 77, 200, 287):
        idx = torch.tensor([big.m.slot_index(LEVEL, c, i, j, k)
                            for (i, j, k) in _interior_points(c)],
                           device="cuda")
        err = (y[idx] + lap * m[idx]).abs().max().item()
        assert err <= FP64_TOL * row_scale
        assert err <= 1e-3 * y[idx].abs().min().item()
    del y, m
    torch.cuda.empty_cache()


def _interior_points(seed, count=4000):
    rng = np.random.default_rng(seed)
    pts = set()
    while len(pts) < count:
        i, j, k = (int(v) for v in rng.integers(1, N - 2, size=3))
        if i + j + k <= N - 1:
            pts.add((i, j, k))
    return sorted(pts)


def test_operator_is_symmetric(big):
    """x.(A z) = (A x).z over the unique interior DoFs, with zero Dirichlet
    data."""
    mask = big.interior_mask()
    x = big.rand(11, zero_boundary=True)
    z = big.rand(12, zero_boundary=True)
    ax = torch.zeros_like(x)
    big.m.apply(LEVEL, x, ax)
    lhs = big.dot(ax, z, mask)
    az = ax
    big.m.apply(LEVEL, z, az)
    rhs = big.dot(x, az, mask)
    scale = (big.dot(az, az, mask) * big.dot(x, x, mask)) ** 0.5
    assert abs(lhs - rhs) <= 1e-12 * scale
    del x, z, ax
    torch.cuda.empty_cache()


def test_restriction_is_transpose_of_prolongation(big):
    """r_f.(P e_c) = (R r_f).e_c between levels 8 and 7 over interior DoFs."""
    mf, mc = big.interior_mask(LEVEL), big.interior_mask(LEVEL - 1)
    r = big.rand(13, zero_boundary=True)
    e = big.rand(14, level=LEVEL - 1, zero_boundary=True)
    pe = torch.zeros_like(r)
    big.m.prolongate_add(LEVEL - 1, e, pe)
    lhs = big.dot(r, pe, mf)
    del pe
    rc = torch.zeros_like(e)
    big.m.restrict(LEVEL, r, rc)
    rhs = big.dot(rc, e, mc)
    scale = float(r.double()[mf].abs().sum()) * e.abs().max().item()
    assert abs(lhs - rhs) <= 1e-13 * scale
    del r, e, rc
    torch.cuda.empty_cache()


def test_solve_both_precisions_at_full_size(big):
    """V(2,2) to 1e-10 (FP64 and FP32-in-FP64); the two solutions agree."""
    m = torch.zeros(big.nslot, dtype=torch.float64, device="cuda")
    big.m.lumped_mass(LEVEL, m)
    b = big.rand(5) * m
    del m
    big.m.sync(LEVEL, b)
    u64 = torch.zeros_like(b)
    st64 = big.m.solve(LEVEL, u64, b, ht.HT_PREC_F64, 1e-10, 60)
    u32 = torch.zeros_like(b)
    st32 = big.m.solve(LEVEL, u32, b, ht.HT_PREC_MIXED, 1e-10, 60)
    assert st64["converged"] and st32["converged"]
    h = np.array(st64["history"])
    assert (h[1:] < h[:-1]).all() and h[-1] <= 1e-10
    assert (h[1:] / h[:-1]).max() < 0.6              # multigrid rate
    assert abs(st64["cycles"] - st32["cycles"]) <= 1
    mask = big.interior_mask()
    diff = (u64 - u32)[mask].norm().item() / u64[mask].norm().item()
    assert diff <= 1e-8
    del b, u64, u32
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_unit_cube_discrete_solution_closed_form(precision):
    """Unit cube as 6 Kuhn tets at level 7 (2,048,383 unknowns): with the
    lumped right-hand side of f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) the
    P1 system is the 7-point scheme, whose solution is c_h u(x) at every
    node, c_h = (pi h / 2)^2 / sin^2(pi h / 2).  Checks the whole GPU solve
    against this closed form, without the oracle."""
    from workloads import kuhn_box
    L = 7
    m = ht.Mesh(*kuhn_box(1, 1, 1), 2, L)
    ns = m.n_slots(L)
    X = torch.zeros(3 * ns, dtype=torch.float64, device="cuda")
    m.coords_device(L, X)
    X = X.view(-1, 3)
    s = (torch.sin(np.pi * X[:, 0]) * torch.sin(np.pi * X[:, 1]) *
         torch.sin(np.pi * X[:, 2]))
    mass = torch.zeros(ns, dtype=torch.float64, device="cuda")
    m.lumped_mass(L, mass)
    b = mass * (3 * np.pi ** 2) * s
    u = torch.zeros_like(b)
    prec = ht.HT_PREC_F64 if precision == "f64" else ht.HT_PREC_MIXED
    st = m.solve(L, u, b, prec, 1e-11, 100)
    assert st["converged"]
    h = 2.0 ** -L
    ch = (np.pi * h / 2) ** 2 / np.sin(np.pi * h / 2) ** 2
    f = torch.zeros(ns, dtype=torch.uint8, device="cuda")
    m.flags_device(L, f)
    interior = ((f & ht.HT_SLOT_DIRICHLET) == 0) & ((f & ht.HT_SLOT_PAD) == 0)
    err = (u - ch * s)[interior].abs().max().item()
    assert err <= 1e-8, err        # discretisation error: 5e-5
    # and it is not the continuous solution: the discretisation error shows
    assert (u - s)[interior].abs().max().item() > 1e-5
    m.close()


def test_fmg_unit_cube_reaches_discretisation_error():
    """Full multigrid with five V(2,2) per level on the unit cube at level 7:
    the algebraic error against the exact discrete solution c_h u is well
    below the discretisation error (c_h - 1) max |u|, with no iteration to a
    residual tolerance."""
    from workloads import kuhn_box
    L = 7
    m = ht.Mesh(*kuhn_box(1, 1, 1), 2, L)
    ns = m.n_slots(L)
    X = torch.zeros(3 * ns, dtype=torch.float64, device="cuda")
    m.coords_device(L, X)
    X = X.view(-1, 3)
    s = (torch.sin(np.pi * X[:, 0]) * torch.sin(np.pi * X[:, 1]) *
         torch.sin(np.pi * X[:, 2]))
    mass = torch.zeros(ns, dtype=torch.float64, device="cuda")
    m.lumped_mass(L, mass)
    b = mass * (3 * np.pi ** 2) * s
    m.fill_dirichlet(L, b, 0.0)
    u = torch.zeros_like(b)
    m.fmg(L, u, b, cycles=5)
    h = 2.0 ** -L
    ch = (np.pi * h / 2) ** 2 / np.sin(np.pi * h / 2) ** 2
    f = torch.zeros(ns, dtype=torch.uint8, device="cuda")
    m.flags_device(L, f)
    interior = ((f & ht.HT_SLOT_DIRICHLET) == 0) & ((f & ht.HT_SLOT_PAD) == 0)
    disc = (ch - 1.0) * s[interior].abs().max().item()
    err = (u - ch * s)[interior].abs().max().item()
    assert err <= 0.25 * disc, (err, disc)
    m.close()


# ------------------------------------------------ variable coefficient --
@pytest.fixture(scope="module")
def kappa(big):
    """k = 1 + sin(2 pi x) sin(2 pi y) sin(2 pi z) / 2 at the slots' own
    coordinates, made consistent."""
    X = torch.zeros(3 * big.nslot, dtype=torch.float64, device="cuda")
    big.m.coords_device(LEVEL, X)
    X = X.view(-1, 3)
    w = 2.0 * np.pi
    k = 1.0 + 0.5 * (torch.sin(w * X[:, 0]) * torch.sin(w * X[:, 1]) *
                     torch.sin(w * X[:, 2]))
    del X
    big.m.sync(LEVEL, k)
    yield k
    del k
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def krows(big, kappa):
    """Oracle rows of div(k grad) at the structured sample points, with the
    coefficient values the GPU holds at the micro-tets' vertices."""
    cache = {}

    def kvals(tkeys):
        flat = tkeys.reshape(-1, 8)
        slots = []
        for kk in flat:
            t = tuple(kk)
            if t not in cache:
                cache[t] = big.slot_of_key(kk)
            slots.append(cache[t])
        return big.gather(kappa, slots).reshape(tkeys.shape[:-1])

    out = []
    for (c, i, j, k) in sample_points(random_count=0):
        slot = big.m.slot_index(LEVEL, c, i, j, k)
        key, _ = big.m.keys(LEVEL, slot, 1)
        nbr, vals, dirichlet = row_at(big.xyz, big.cells, LEVEL, key[0],
                                      kappa=kvals)
        nslots = np.array([big.slot_of_key(kk) for kk in nbr])
        out.append(Row(slot, big.slot_of_key(key[0]), nslots, vals, dirichlet))
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_divkgrad_sampled_rows(big, kappa, krows, dtype):
    tdt = torch.float64 if dtype == "f64" else torch.float32
    # FP32: the bound of the small-size parity tests (about 100 roundings of
    # O(1) terms per row)
    tol = FP64_TOL if dtype == "f64" else 3e-5
    x = big.rand(14, tdt)
    k = kappa.to(tdt)
    y = torch.full_like(x, float("nan"))
    big.m.apply_divkgrad(LEVEL, k, x, y)
    got = big.gather(y, [r.slot for r in krows])
    assert np.isfinite(got).all()
    assert np.array_equal(got, big.gather(y, [r.own for r in krows]))
    for r, g in zip(krows, got):
        xv = big.gather(x, r.nslots)
        want = 0.0 if r.dirichlet else float(r.vals @ xv)
        assert abs(g - want) <= tol * float(np.abs(r.vals) @ np.abs(xv)), \
            (r.slot, g, want)
    del x, k, y
    torch.cuda.empty_cache()


def test_divkgrad_annihilates_constants(big, kappa):
    """Rows of div(k grad) sum to zero: A_k 1 = 0 on every interior row."""
    u = torch.ones_like(kappa)
    y = torch.full_like(u, float("nan"))
    big.m.apply_divkgrad(LEVEL, kappa, u, y)
    mask = big.interior_mask()
    stencil_sum = np.abs(big.m.cell_stencils(LEVEL)).sum(axis=2).max()
    worst = y[mask].abs().max().item()
    assert worst <= FP64_TOL * 30 * 1.5 * stencil_sum
    del u, y
    torch.cuda.empty_cache()
