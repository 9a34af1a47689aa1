"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: counts and
widths printed in the paper, closed-form stencils, exactness of P1 on
constants/linears/quadratics, Euler's formula, an independent nodal-basis
assembly, the exact discrete solution of the 7-point scheme, and textbook
multigrid identities.  A plausible slip in the oracle (wrong child order in
the refinement, a dropped term, a sign, a transposed operand) breaks at least
one of them.
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.fem import P1System
from oracle.refine import MicroMesh, reference_refinement
from oracle.rows import row_at
from tests.conftest import mesh_by_name, oracle_hierarchy
from workloads import fields

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def N_tet(w):
    return w * (w + 1) * (w + 2) // 6


def N_tri(w):
    return w * (w + 1) // 2


def local_index(mesh: MicroMesh):
    """Integer (i, j, k) of every vertex of a single-cell mesh."""
    assert len(mesh.cells) == 1
    w = np.zeros((mesh.num_vertices, 4), dtype=np.int64)
    ids, wts = mesh.keys[:, 0::2], mesh.keys[:, 1::2]
    for q in range(4):
        w[:, q] = np.where(ids == mesh.cells[0][q], wts, 0).sum(axis=1)
    return w[:, 1:]


# ----------------------------------------------------------------- counts --
@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_counts_single_cell(level):
    """Micro-vertices of a refined tet: N_tet(2^l + 1) (the vertex row of the
    subgroup table and eq. for N_tet); micro-cells: 8^l (eq. bey)."""
    m = MicroMesh(*mesh_by_name("ref_tet"), level)
    n = 2 ** level
    assert m.num_vertices == N_tet(n + 1) == (n + 1) * (n + 2) * (n + 3) // 6
    assert len(m.tets) == 8 ** level
    if level == 4:
        assert m.num_vertices == 969          # reference tet, level 4: 969 micro-vertices


@pytest.mark.parametrize("shape,level", [((1, 1, 1), 3), ((2, 1, 1), 2),
                                         ((4, 4, 3), 2)])
def test_counts_kuhn_box(shape, level):
    """Conforming refinement of a box: the micro-vertices are exactly the
    points of the (a n + 1)(b n + 1)(c n + 1) grid."""
    import workloads
    a, b, c = shape
    n = 2 ** level
    m = MicroMesh(*workloads.kuhn_box(a, b, c), level)
    assert m.num_vertices == (a * n + 1) * (b * n + 1) * (c * n + 1)
    grid = np.rint(m.xyz * n).astype(np.int64)
    assert len(np.unique(grid, axis=0)) == m.num_vertices


def test_interior_dof_counts_288_mesh():
    """Interior unknowns of the 4x4x3 box: (4n-1)(4n-1)(3n-1)."""
    H = oracle_hierarchy("jittered_288", 3, 2)
    for lvl in (2, 3):
        n = 2 ** lvl
        assert H[lvl].interior.sum() == (4 * n - 1) ** 2 * (3 * n - 1)
    assert H[2].interior.sum() == 2475


def _golden_widths():
    rows = []
    with open(os.path.join(GOLDEN, "subgroup_widths.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                rows.append((line[0], line[1], int(line[2])))
    return rows


def _pattern_counts(idx, simplices):
    """Count simplices per translation class (shape relative to min corner)."""
    out = {}
    for s in simplices:
        p = idx[s]
        pat = tuple(sorted(map(tuple, p - p.min(axis=0))))
        out[pat] = out.get(pat, 0) + 1
    return out


@pytest.mark.parametrize("level", [2, 3, 4])
def test_subgroup_counts_against_paper_table(level):
    """Subgroup sizes N_tet(w(l)) from the paper's subgroup table.

    Vertices, the 7 edge subgroups and the 6 cell subgroups match the printed
    widths.  For faces the printed xyz-down width 2^l - 2 cannot hold: the
    counted sizes are eight subgroups of N_tet(2^l - 1) and four of
    N_tet(2^l), and Euler's formula V - E + F - C = 1 of the refined
    (contractible) tetrahedron fixes the total face count independently.
    """
    n = 2 ** level
    m = MicroMesh(*mesh_by_name("ref_tet"), level)
    idx = local_index(m)
    rows = _golden_widths()
    want = {p: sorted(N_tet(n + off) for (q, _, off) in rows if q == p)
            for p in ("vertex", "edge", "face", "cell")}
    assert [m.num_vertices] == want["vertex"]
    edges, faces = m.edges(), m.faces()
    assert sorted(_pattern_counts(idx, edges).values()) == want["edge"]
    assert sorted(_pattern_counts(idx, m.tets).values()) == want["cell"]
    got_faces = sorted(_pattern_counts(idx, faces).values())
    assert len(got_faces) == 12
    derived = sorted(N_tet(n + off) for off in [0] * 4 + [-1] * 8)
    assert got_faces == derived
    assert got_faces != want["face"]          # the table's xyz-down width
    assert m.num_vertices - len(edges) + len(faces) - len(m.tets) == 1


def test_example_widths_in_caption():
    """Level-2 example widths printed in the subgroup illustration caption:
    vertices w=5, xy edges w=4, xy-up faces w=3, II-down cells w=3."""
    rows = {(p, s): off for (p, s, off) in _golden_widths()}
    n = 4
    assert n + rows[("vertex", "-")] == 5
    assert n + rows[("edge", "xy")] == 4
    assert n + rows[("face", "xy-up")] == 3
    assert n + rows[("cell", "II-down")] == 3


# ------------------------------------------------------------ refinement --
def test_refinement_is_conforming_and_fills_the_domain():
    """Every micro-face lies in one or two micro-tets; boundary micro-faces
    tile the boundary; micro-tet volumes sum to the domain volume."""
    for name, vol, area in [("ref_tet", 1 / 6, 1.5 + np.sqrt(3) / 2),
                            ("kuhn_211", 2.0, 10.0)]:
        S = P1System(MicroMesh(*mesh_by_name(name), 3))
        faces, counts = S.mesh.faces(return_counts=True)
        assert set(np.unique(counts)) <= {1, 2}
        P = S.mesh.xyz[faces[counts == 1]]
        a = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0],
                                          P[:, 2] - P[:, 0]), axis=1)
        assert np.isclose(a.sum(), area, rtol=1e-13)
        assert np.isclose(S.tet_volume.sum(), vol, rtol=1e-13)


def test_child_vertices_follow_eq_bey():
    """Level 1 of the reference cell: T1 = [v0, v01, v02, v03] and the inner
    diagonal of T5..T8 is v02-v13 (all four contain both points)."""
    t = reference_refinement(1)
    v = {"0": [2, 0, 0, 0], "01": [1, 1, 0, 0], "02": [1, 0, 1, 0],
         "03": [1, 0, 0, 1], "13": [0, 1, 0, 1]}
    assert (t[0] == np.array([v["0"], v["01"], v["02"], v["03"]])).all()
    for c in range(4, 8):
        pts = [list(r) for r in t[c]]
        assert v["02"] in pts and v["13"] in pts


# --------------------------------------------------------- closed forms --
# Interior stencil of the reference tet (every cell-interior point), in units of
# 1/(3n): offsets (di, dj, dk) -> weight.  Derived by hand from the element
# matrices of the six Bey micro-cell shapes of the reference cell.
REF_TET_STENCIL = {(0, 0, 0): 20, (1, 0, 0): -4, (-1, 0, 0): -4, (0, 0, 1): -4,
              (0, 0, -1): -4, (0, 1, 0): -2, (0, -1, 0): -2, (-1, 1, 0): -1,
              (1, -1, 0): -1, (0, -1, 1): -1, (0, 1, -1): -1, (-1, 0, 1): 1,
              (1, 0, -1): 1, (1, -1, 1): 1, (-1, 1, -1): 1}


@pytest.mark.parametrize("level", [2, 3, 4])
def test_reference_tet_interior_rows_closed_form(level):
    n = 2 ** level
    S = P1System(MicroMesh(*mesh_by_name("ref_tet"), level))
    idx = local_index(S.mesh)
    where = {tuple(p): v for v, p in enumerate(idx)}
    inner = np.flatnonzero((idx.min(axis=1) >= 1) & (idx.sum(axis=1) <= n - 1))
    assert len(inner) == N_tet(n - 3)
    A = S.A.tocsr()
    for v in inner:
        row = {}
        for p in range(A.indptr[v], A.indptr[v + 1]):
            d = tuple(idx[A.indices[p]] - idx[v])
            row[d] = A.data[p] * 3 * n
        row = {d: w for d, w in row.items() if abs(w) > 1e-12}
        assert set(row) == set(REF_TET_STENCIL)
        for d, w in REF_TET_STENCIL.items():
            assert abs(row[d] - w) < 1e-11, (d, row[d], w)
    # the seven direction classes are all present with their neighbours
    assert where[(1, 1, 1)] >= 0


@pytest.mark.parametrize("level", [1, 2, 3])
def test_kuhn_box_is_seven_point_laplacian(level):
    """On Kuhn boxes the assembled P1 matrix is h times the 7-point Laplacian
    (diagonal 6h, -h on the six axis neighbours, nothing else) at every
    interior vertex, including those on shared macro-faces and -edges."""
    n = 2 ** level
    h = 1.0 / n
    S = P1System(MicroMesh(*mesh_by_name("kuhn_211"), level))
    grid = np.rint(S.mesh.xyz * n).astype(np.int64)
    A = S.A.tocsr()
    axis = {(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1),
            (0, 0, -1)}
    for v in np.flatnonzero(S.interior):
        for p in range(A.indptr[v], A.indptr[v + 1]):
            d = tuple(grid[A.indices[p]] - grid[v])
            w = A.data[p]
            if d == (0, 0, 0):
                assert abs(w - 6 * h) < 1e-14
            elif d in axis:
                assert abs(w + h) < 1e-14
            else:
                assert abs(w) < 1e-14


def test_level_scaling_halves_the_stencil():
    """Every stiffness entry on level l+1 is half the matching entry on l."""
    a = P1System(MicroMesh(*mesh_by_name("ref_tet"), 3))
    b = P1System(MicroMesh(*mesh_by_name("ref_tet"), 4))
    ia, ib = local_index(a.mesh), local_index(b.mesh)
    where_b = {tuple(p): v for v, p in enumerate(ib)}
    Aa, Ab = a.A.tocsr(), b.A.tocsr()
    for v in range(a.mesh.num_vertices):
        vb = where_b[tuple(2 * ia[v])]
        for p in range(Aa.indptr[v], Aa.indptr[v + 1]):
            d = ia[Aa.indices[p]] - ia[v]
            ub = where_b[tuple(2 * ia[v] + d)]
            assert Ab[vb, ub] * 2 == pytest.approx(Aa.data[p], abs=1e-15)


# ------------------------------------------------------------- invariants --
@pytest.mark.parametrize("name,level", [("ref_tet", 4), ("jittered_288", 2),
                                        ("jittered_222", 3), ("slab_3_11", 3)])
def test_constant_and_linear_fields_are_annihilated(name, level):
    """P1 reproduces affine functions, so (A u)_i = 0 on interior rows."""
    S = P1System(MicroMesh(*mesh_by_name(name), level))
    X = S.mesh.xyz
    scale = abs(S.A).sum(axis=1).max()
    for u in (np.ones(len(X)), X @ np.array([0.3, -1.2, 0.7]) + 0.4):
        y = S.apply(u)
        assert np.abs(y).max() <= 1e-13 * scale


@pytest.mark.parametrize("name,level", [("ref_tet", 3), ("jittered_222", 3)])
def test_quadratic_exact_at_cell_interior(name, level):
    """At points whose 24 micro-tets lie in one macro-cell the P1 row applied
    to a quadratic u gives exactly -Laplace(u) times the lumped mass."""
    S = P1System(MicroMesh(*mesh_by_name(name), level))
    X = S.mesh.xyz
    H = np.array([[2.0, 0.3, -0.5], [0.3, 1.0, 0.7], [-0.5, 0.7, -1.5]])
    u = 0.5 * np.einsum("ni,ij,nj->n", X, H, X) + X @ [0.3, -0.2, 0.1] + 0.7
    y = S.A @ u
    cell_interior = S.mesh.keys[:, 7] > 0          # four non-zero weights
    err = y[cell_interior] + np.trace(H) * S.lumped_mass[cell_interior]
    assert np.abs(err).max() <= 1e-12 * np.abs(y[cell_interior]).max()


def test_symmetric_positive_definite():
    H = oracle_hierarchy("jittered_288", 2, 2)
    AII, _ = H[2].interior_matrix()
    assert abs(AII - AII.T).max() <= 1e-16 * abs(AII).max()
    np.linalg.cholesky(AII.toarray())


def test_lumped_mass_sums_to_volume():
    S = P1System(MicroMesh(*mesh_by_name("jittered_288"), 2))
    assert np.isclose(S.lumped_mass.sum(), 48.0, rtol=1e-13)
    m = P1System(MicroMesh(*mesh_by_name("kuhn_211"), 3))
    n = 8
    grid = np.rint(m.mesh.xyz * n).astype(int)
    inner = (grid.min(axis=1) > 0) & (grid[:, 0] < 2 * n) & (grid[:, 1] < n) \
        & (grid[:, 2] < n)
    assert np.allclose(m.lumped_mass[inner], 1.0 / n ** 3, rtol=1e-13)


def test_brute_force_nodal_basis_assembly():
    """Independent assembly: the hat function of vertex q on micro-tet T is the
    affine c.x + d with value 1 at q and 0 at the other three vertices (a 4x4
    solve), its gradient is c, and a_ij = sum_T |T| c_i . c_j."""
    for name, level in [("jittered_222", 1), ("ref_tet", 2), ("slab_2_7", 1)]:
        S = P1System(MicroMesh(*mesh_by_name(name), level))
        N = S.mesh.num_vertices
        A = np.zeros((N, N))
        for t in S.mesh.tets:
            P = S.mesh.xyz[t]
            M = np.hstack([P, np.ones((4, 1))])
            coef = np.linalg.solve(M, np.eye(4))     # column q: hat of q
            grads = coef[:3].T
            vol = abs(np.linalg.det(P[1:] - P[0])) / 6
            A[np.ix_(t, t)] += vol * grads @ grads.T
        assert np.abs(A - S.A.toarray()).max() <= 1e-14 * np.abs(A).max()


def test_row_oracle_matches_assembly():
    H = oracle_hierarchy("jittered_288", 3, 2)
    S = H[3]
    rng = np.random.default_rng(11)
    for v in rng.choice(S.mesh.num_vertices, 12, replace=False):
        nbr, vals, dirichlet = row_at(S.mesh.macro_xyz, S.mesh.cells, 3,
                                      S.mesh.keys[v])
        assert dirichlet == bool(S.dirichlet[v])
        cols = S.mesh.index_of(nbr)
        dense = S.A[v].toarray().ravel()
        assert np.abs(dense[cols] - vals).max() <= 1e-15
        assert np.count_nonzero(np.abs(dense) > 0) <= len(cols)


# ------------------------------------------------------------- multigrid --
def test_prolongation_reproduces_affine_fields():
    """Nested P1 interpolation: P maps the coarse interpolant of an affine
    field onto the fine interpolant, and its rows sum to one."""
    H = oracle_hierarchy("jittered_288", 3, 2)
    P = H.P[3]
    assert np.allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0, atol=1e-15)
    g = lambda X: X @ [0.7, -0.1, 1.3] - 2.0
    assert np.abs(P @ g(H[2].mesh.xyz) - g(H[3].mesh.xyz)).max() < 1e-13


def test_galerkin_identity():
    """R A_l P = A_(l-1) on interior unknowns (nested conforming spaces)."""
    for name, hi in [("jittered_288", 3), ("ref_tet", 4), ("slab_2_9", 3)]:
        H = oracle_hierarchy(name, hi, hi - 1)
        If, Ic = H[hi].interior, H[hi - 1].interior
        P = H.P[hi][If][:, Ic]
        G = P.T @ H[hi].A[If][:, If] @ P
        Ac = H[hi - 1].A[Ic][:, Ic]
        assert abs(G - Ac).max() <= 1e-13 * abs(Ac).max()


def test_jacobi_error_propagation():
    """One weighted-Jacobi sweep maps the error e = u - u* to
    (I - omega D^-1 A_II) e, and the exact solution is its fixed point."""
    S = oracle_hierarchy("jittered_288", 2, 2)[2]
    AII, I = S.interior_matrix()
    b = np.zeros(S.mesh.num_vertices)
    b[I] = np.random.default_rng(1).uniform(-1, 1, len(I))
    ustar = np.zeros_like(b)
    ustar[I] = np.linalg.solve(AII.toarray(), b[I])
    assert np.abs(S.jacobi(ustar, b, 2 / 3) - ustar).max() < 1e-12
    u0 = ustar + np.where(S.interior, np.sin(np.arange(len(b))), 0.0)
    e0 = (u0 - ustar)[I]
    M = np.eye(len(I)) - (2 / 3) * AII.toarray() / AII.diagonal()[:, None]
    e1 = (S.jacobi(u0, b, 2 / 3) - ustar)[I]
    assert np.abs(e1 - M @ e0).max() < 1e-12


def test_two_grid_cycle_error_propagation():
    """V(1,1) on two levels with an exact coarse solve has error propagation
    S (I - P Ac^-1 R A) S, S = I - omega D^-1 A (dense textbook form)."""
    H = oracle_hierarchy("jittered_222", 2, 1)
    F, C = H[2], H[1]
    AF, IF = F.interior_matrix()
    AC, IC = C.interior_matrix()
    AF, AC = AF.toarray(), AC.toarray()
    P = H.P[2][F.interior][:, C.interior].toarray()
    Sm = np.eye(len(IF)) - (2 / 3) * AF / np.diag(AF)[:, None]
    M = Sm @ (np.eye(len(IF)) - P @ np.linalg.solve(AC, P.T @ AF)) @ Sm
    b = np.zeros(F.mesh.num_vertices)
    b[IF] = np.random.default_rng(2).uniform(-1, 1, len(IF))
    ustar = np.zeros_like(b)
    ustar[IF] = np.linalg.solve(AF, b[IF])
    u0 = np.zeros_like(b)
    u1 = H.vcycle(2, u0, b, nu1=1, nu2=1, coarse_level=1)
    assert np.abs((u1 - ustar)[IF] - M @ (u0 - ustar)[IF]).max() < 1e-13


def test_vcycle_converges_to_direct_solution():
    H = oracle_hierarchy("jittered_288", 3, 2)
    S = H[3]
    f = fields.uniform_values(S.mesh.num_vertices, 5)
    b = S.lumped_mass * f
    u, hist = H.solve(3, b, rel_tol=1e-10, coarse_level=2)
    assert hist[-1] <= 1e-10 and all(np.diff(hist) < 0)
    AII, I = S.interior_matrix()
    ud = spla.spsolve(AII.tocsc(), b[I])
    assert np.abs(u[I] - ud).max() <= 1e-8 * np.abs(ud).max()


# ---------------------------------- manufactured Poisson, unit cube --
def _cube_errors(levels):
    out = []
    for lvl in levels:
        S = P1System(MicroMesh(*mesh_by_name("kuhn_cube"), lvl))
        b = S.lumped_mass * fields.sine_source(S.mesh.xyz)
        AII, I = S.interior_matrix()
        uh = spla.spsolve(AII.tocsc(), b[I])
        out.append((S, I, uh))
    return out


def test_unit_cube_exact_discrete_solution():
    """Kuhn cube + lumped right-hand side = the 7-point scheme, whose discrete
    solution for f = 3 pi^2 sin sin sin is c_h u(x_i) exactly, with
    c_h = (pi h / 2)^2 / sin^2(pi h / 2)."""
    for S, I, uh in _cube_errors([3, 4, 5]):
        h = 1.0 / S.mesh.n
        ch = (np.pi * h / 2) ** 2 / np.sin(np.pi * h / 2) ** 2
        exact = ch * fields.sine_solution(S.mesh.xyz[I])
        assert np.abs(uh - exact).max() <= 1e-10


def test_unit_cube_second_order_convergence():
    """Max nodal error ratios between consecutive levels approach 4 (O(h^2),
    the rate the paper shows for its own convergence study)."""
    errs = [np.abs(uh - fields.sine_solution(S.mesh.xyz[I])).max()
            for S, I, uh in _cube_errors([2, 3, 4, 5])]
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert ((ratios > 3.8) & (ratios < 4.2)).all(), ratios


# ------------------------------------------------ full multigrid (FMG) --
def _cube_problem(H, lvl):
    """Lumped sine right-hand side on the unit cube and its exact discrete
    solution c_h u(x) (the 7-point scheme's eigenfunction)."""
    S = H[lvl]
    b = np.where(S.dirichlet, 0.0,
                 S.lumped_mass * fields.sine_source(S.mesh.xyz))
    h = 1.0 / S.mesh.n
    ch = (np.pi * h / 2) ** 2 / np.sin(np.pi * h / 2) ** 2
    u = fields.sine_solution(S.mesh.xyz)
    disc = np.abs((ch - 1.0) * u)[S.interior].max()
    return S, b, ch * u, disc


def test_fmg_converges_to_the_discrete_solution():
    """Many cycles per level: nested iteration ends at the exact discrete
    solution, known in closed form."""
    H = oracle_hierarchy("kuhn_cube", 4, 2)
    S, b, uh, disc = _cube_problem(H, 4)
    u = H.fmg(4, b, cycles=30, coarse_level=2)
    assert np.abs(u - uh)[S.interior].max() <= 1e-9 * disc


def test_fmg_reaches_the_discretisation_error():
    """Five V(2,2) per level leave an algebraic error well below the
    discretisation error, on every level (the defining property of nested
    iteration: the error does not accumulate across levels)."""
    H = oracle_hierarchy("kuhn_cube", 5, 2)
    for lvl in (3, 4, 5):
        S, b, uh, disc = _cube_problem(H, lvl)
        u = H.fmg(lvl, b, cycles=5, coarse_level=2)
        assert np.abs(u - uh)[S.interior].max() <= 0.25 * disc


def test_fmg_on_the_coarse_level_is_the_direct_solve():
    H = oracle_hierarchy("jittered_288", 2, 2)
    S = H[2]
    b = np.where(S.dirichlet, 0.0, fields.uniform_values(S.mesh.num_vertices, 8))
    u = H.fmg(2, b, cycles=1, coarse_level=2)
    AII, I = S.interior_matrix()
    assert np.allclose(u[I], spla.spsolve(AII.tocsc(), b[I]), rtol=1e-12, atol=1e-14)


# ------------------------------------------------- Chebyshev smoother --
def _generalised_eigen(S):
    """Eigenpairs of D^-1 A on the interior unknowns (A v = lam D v)."""
    import scipy.linalg as sla
    AII, I = S.interior_matrix()
    A = AII.toarray()
    lam, V = sla.eigh(A, np.diag(np.diag(A)))
    return lam, V, I


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_chebyshev_smoother_is_the_chebyshev_polynomial(degree):
    """With b = 0 the smoother maps an eigenvector of D^-1 A (eigenvalue lam)
    to T_m((beta+alpha-2 lam)/(beta-alpha)) / T_m((beta+alpha)/(beta-alpha))
    times itself."""
    from numpy.polynomial import chebyshev as cheb
    from oracle.mg import chebyshev_smooth
    S = oracle_hierarchy("jittered_222", 2, 2)[2]
    lam, V, I = _generalised_eigen(S)
    alpha, beta = 0.07, 2.0
    Tm = [0] * degree + [1]
    for idx in (0, 40, len(lam) // 2, len(lam) - 1):
        u = np.zeros(S.mesh.num_vertices)
        u[I] = V[:, idx]
        out = chebyshev_smooth(S, u, np.zeros_like(u), degree, alpha, beta)
        p = (cheb.chebval((beta + alpha - 2 * lam[idx]) / (beta - alpha), Tm) /
             cheb.chebval((beta + alpha) / (beta - alpha), Tm))
        assert np.abs(out[I] - p * V[:, idx]).max() <= 1e-13


def test_chebyshev_degree_one_is_jacobi():
    """Degree 1 is a Jacobi sweep with weight 1/theta."""
    from oracle.mg import chebyshev_smooth
    S = oracle_hierarchy("jittered_222", 3, 2)[3]
    u = np.where(S.dirichlet, 0.0, fields.uniform_values(S.mesh.num_vertices, 1))
    b = fields.uniform_values(S.mesh.num_vertices, 2)
    alpha, beta = 0.05, 2.1
    out = chebyshev_smooth(S, u, b, 1, alpha, beta)
    assert np.allclose(out, S.jacobi(u, b, 2.0 / (alpha + beta)), rtol=0, atol=1e-14)


@pytest.mark.parametrize("level", [2, 3])
def test_power_iteration_brackets_the_largest_eigenvalue(level):
    """The estimate is below the largest eigenvalue of D^-1 A and the upper
    end of the smoothing interval (1.1 times it) is above."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    from oracle.mg import CHEB_UPPER, lambda_max_estimate
    S = oracle_hierarchy("jittered_222", 3, 2)[level]
    AII, _ = S.interior_matrix()
    lmax = sla.eigsh(AII, k=1, M=sp.diags(AII.diagonal()), which="LA")[0][0]
    est = lambda_max_estimate(S)
    assert est <= lmax * (1 + 1e-12) and CHEB_UPPER * est >= lmax


def test_vcycle_with_chebyshev_smoother_converges():
    H = oracle_hierarchy("jittered_222", 3, 2)
    S = H[3]
    b = S.lumped_mass * fields.uniform_values(S.mesh.num_vertices, 4)
    u = np.zeros_like(b)
    hist = [np.linalg.norm(S.residual(u, b))]
    for _ in range(12):
        u = H.vcycle(3, u, b, 1, 1, coarse_level=2, smoother="chebyshev",
                     degree=2)
        hist.append(np.linalg.norm(S.residual(u, b)))
    rates = np.array(hist[1:]) / np.array(hist[:-1])
    assert rates.max() < 0.35 and hist[-1] <= 1e-7 * hist[0]


# -------------------------- second, lattice-based oracle, reference tet --
def test_ref_tet_lattice_stencil_reproduces_oracle():
    """A separate lattice code (closed-form stencil on the index grid of the
    reference tet, no assembly) reproduces the oracle's apply and ten Jacobi
    sweeps (omega = 2/3) on the reference tet (level 4, u ~ U[-1,1], zero boundary)."""
    level, n = 4, 16
    S = P1System(MicroMesh(*mesh_by_name("ref_tet"), level))
    idx = local_index(S.mesh)
    u = fields.uniform_values(S.mesh.num_vertices, 0)
    u[S.dirichlet] = 0.0
    grid = np.zeros((n + 3,) * 3)
    inner = (idx.min(axis=1) >= 1) & (idx.sum(axis=1) <= n - 1)
    assert (inner == S.interior).all()

    def lattice_apply(vals):
        grid[:] = 0.0
        grid[idx[:, 0] + 1, idx[:, 1] + 1, idx[:, 2] + 1] = vals
        out = np.zeros_like(vals)
        for d, w in REF_TET_STENCIL.items():
            out += w / (3 * n) * grid[idx[:, 0] + 1 + d[0], idx[:, 1] + 1 + d[1],
                                      idx[:, 2] + 1 + d[2]]
        return np.where(inner, out, 0.0)

    assert np.abs(lattice_apply(u) - S.apply(u)).max() < 1e-14
    ul, uo = u.copy(), u.copy()
    b = np.zeros_like(u)
    diag = 20 / (3 * n)
    for _ in range(10):
        ul = np.where(inner, ul + (2 / 3) * (b - lattice_apply(ul)) / diag, ul)
    uo = S.jacobi(uo, b, 2 / 3, sweeps=10)
    assert np.abs(ul - uo).max() < 1e-14


# ----------------------------------------------- variable coefficient --
def test_q3_rule_integrates_cubics_exactly():
    """The degree-3 rule against the closed form of monomial integrals over
    the unit simplex: a! b! c! / (a + b + c + 3)!, times 3! for the volume
    normalisation.  A wrong weight or point breaks some monomial."""
    from math import factorial
    from oracle.fem import TET_Q3_POINTS, TET_Q3_WEIGHTS
    # reference tet with vertices 0, e1, e2, e3: x = lambda_1 .. lambda_3
    X = TET_Q3_POINTS[:, 1:]
    for a in range(4):
        for b in range(4 - a):
            for c in range(4 - a - b):
                quad = (TET_Q3_WEIGHTS * X[:, 0] ** a * X[:, 1] ** b *
                        X[:, 2] ** c).sum() / 6.0
                exact = factorial(a) * factorial(b) * factorial(c) / \
                    factorial(a + b + c + 3)
                assert abs(quad - exact) <= 1e-15, (a, b, c)
    # and it is not exact beyond degree 3
    quad4 = (TET_Q3_WEIGHTS * X[:, 0] ** 4).sum() / 6.0
    assert abs(quad4 - factorial(4) / factorial(7)) > 1e-6


def test_constant_coefficient_scales_the_laplacian():
    mesh = MicroMesh(*mesh_by_name("jittered_222"), 2)
    A = P1System(mesh).A
    Ak = P1System(mesh, kappa=np.full(mesh.num_vertices, 3.7)).A
    assert abs(Ak - 3.7 * A).max() <= 1e-14 * abs(Ak).max()


@pytest.mark.parametrize("name,level", [("jittered_222", 2), ("ref_tet", 3)])
def test_affine_coefficient_uses_the_centroid_value(name, level):
    """For affine k the element integral is |T| k(centroid) exactly.  The
    reference assembly evaluates k at each micro-tet's centroid from the
    coordinates (no vertex values, no quadrature) and scales the Laplacian's
    element matrices by it, via the independent nodal-basis construction."""
    mesh = MicroMesh(*mesh_by_name(name), level)
    g, c0 = np.array([0.4, -0.3, 0.25]), 1.3
    kv = mesh.xyz @ g + c0
    S = P1System(mesh, kappa=kv)
    N = mesh.num_vertices
    A = np.zeros((N, N))
    for t in mesh.tets:
        P = mesh.xyz[t]
        grads = np.linalg.solve(np.hstack([P, np.ones((4, 1))]), np.eye(4))[:3].T
        vol = abs(np.linalg.det(P[1:] - P[0])) / 6
        kc = P.mean(axis=0) @ g + c0
        A[np.ix_(t, t)] += kc * vol * grads @ grads.T
    assert np.abs(A - S.A.toarray()).max() <= 1e-13 * np.abs(A).max()


def test_coefficient_energy_identity():
    """u^T A_k u = sum over T of (integral of k over T) |grad u_T|^2, with
    grad u_T solved from T's edge vectors; the integral of the linear
    interpolant of k is |T| times the vertex mean.  Also: symmetric, rows sum
    to zero, positive definite on the interior unknowns."""
    mesh = MicroMesh(*mesh_by_name("jittered_288"), 1)
    kv = fields.coefficient_field(mesh.xyz)
    S = P1System(mesh, kappa=kv)
    u = fields.uniform_values(mesh.num_vertices, seed=21)
    energy = 0.0
    for t in mesh.tets:
        P = mesh.xyz[t]
        grad = np.linalg.solve(P[1:] - P[0], u[t[1:]] - u[t[0]])
        vol = abs(np.linalg.det(P[1:] - P[0])) / 6
        energy += vol * kv[t].mean() * grad @ grad
    assert abs(u @ (S.A @ u) - energy) <= 1e-12 * energy
    A = S.A
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()
    assert np.abs(A @ np.ones(A.shape[0])).max() <= 1e-13 * abs(A).max()
    AII, _ = S.interior_matrix()
    np.linalg.cholesky(AII.toarray())


def test_row_oracle_with_coefficient_matches_assembly():
    """Single rows of div(k grad), k looked up by key, against the assembled
    matrix of the same coefficient values."""
    mesh = MicroMesh(*mesh_by_name("jittered_288"), 3)
    kv = fields.coefficient_field(mesh.xyz)
    S = P1System(mesh, kappa=kv)

    def kappa(tkeys):
        return kv[mesh.index_of(tkeys)]

    rng = np.random.default_rng(12)
    for v in rng.choice(mesh.num_vertices, 12, replace=False):
        nbr, vals, dirichlet = row_at(mesh.macro_xyz, mesh.cells, 3,
                                      mesh.keys[v], kappa=kappa)
        assert dirichlet == bool(S.dirichlet[v])
        dense = S.A[v].toarray().ravel()
        assert np.abs(dense[mesh.index_of(nbr)] - vals).max() <= 1e-15


def test_threaded_csr_product_equals_scipy():
    """The CPU baseline's threaded CSR product (oracle/spmv.cpp) against
    SciPy's product of the same assembled matrix, for several thread counts
    (the row split must cover every row exactly once)."""
    from oracle import spmv
    if not os.path.exists(spmv.LIB):
        spmv.build()
    S = oracle_hierarchy("jittered_222", 3, 3)[3]
    M = spmv.CSR(S.A)
    x = np.random.default_rng(3).uniform(-1, 1, S.A.shape[0])
    ref = S.A @ x
    for threads in (1, 3, 8, 64):
        y = np.full(S.A.shape[0], np.nan)
        M.apply(x, y, threads)
        assert np.array_equal(y, ref) or np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max()
