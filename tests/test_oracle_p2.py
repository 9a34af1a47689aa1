"""Pins of the P2 oracle (oracle/p2.py) against facts fixed by the paper and
by mathematics: node counts from the subgroup table, energies of quadratics
in closed form, basis integrals, exact reproduction of a quadratic solution
(Galerkin exactness: the solution lies in the space), and the single-row
oracle against the assembly.  A slip in the basis, its gradients, the edge
order, the node keys or the boundary set breaks at least one of them.
"""
import numpy as np
import pytest

from oracle.fem import P1System
from oracle.p2 import (EDGES, P2System, element_load_p2, element_stiffness_p2,
                       p2_row_at)
from oracle.refine import MicroMesh
from tests.conftest import mesh_by_name


def N_tet(w):
    return w * (w + 1) * (w + 2) // 6 if w > 0 else 0


def p2_nodes(P):
    """Coordinates of the ten nodes of tets P [m, 4, 3], vertices first."""
    return np.concatenate([P, np.stack([(P[:, a] + P[:, b]) / 2
                                        for a, b in EDGES], axis=1)], axis=1)


REF = np.array([[[0., 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]])


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_node_count_is_the_subgroup_table(level):
    """One cell: one node per micro-vertex (width 2^l + 1) and per micro-edge
    (six subgroups of width 2^l, xyz of width 2^l - 1), as in the paper's
    subgroup table; together the level-(l+1) vertices N_tet(2^(l+1) + 1)."""
    S = P2System(*mesh_by_name("ref_tet"), level)
    n = 2 ** level
    want = N_tet(n + 1) + 6 * N_tet(n) + N_tet(n - 1)
    assert S.num_nodes == want == N_tet(2 * n + 1)


@pytest.mark.parametrize("u,energy", [
    (lambda x, y, z: x, 1 / 6),                 # |grad|^2 = 1, volume 1/6
    (lambda x, y, z: x * x, 1 / 15),            # 4 int x^2 = 4 * 2!/5!
    (lambda x, y, z: x * y, 1 / 30),            # int x^2 + y^2 = 2 * 2/5!
    (lambda x, y, z: y * z + z * z, 2 / 15),    # 5 int z^2 + int y^2 + 4 int yz
])
def test_energy_of_quadratics_on_the_reference_tet(u, energy):
    """u_h^T K u_h equals the integral of |grad u|^2 for quadratic u (the
    interpolant is u itself); monomial integrals over the unit simplex are
    a! b! c! / (a + b + c + 3)!."""
    K, vol = element_stiffness_p2(REF)
    X = p2_nodes(REF)[0]
    uh = u(X[:, 0], X[:, 1], X[:, 2])
    assert vol[0] == pytest.approx(1 / 6, abs=1e-15)
    assert uh @ K[0] @ uh == pytest.approx(energy, rel=1e-13)


def test_energy_of_random_quadratics_on_random_tets():
    """u = c + b.x + x^T Q x on a random tet: the integral of
    |b + 2 Q x|^2 follows from the volume, centroid and the second-moment
    matrix (1/20)(sum_q P_q P_q^T + s s^T), s = sum_q P_q, of a tetrahedron."""
    rng = np.random.default_rng(11)
    P = rng.normal(size=(20, 4, 3))
    K, vol = element_stiffness_p2(P)
    X = p2_nodes(P)
    for m in range(len(P)):
        c = rng.normal()
        b = rng.normal(size=3)
        Q = rng.normal(size=(3, 3))
        Q = Q + Q.T
        uh = c + X[m] @ b + np.einsum("pi,ij,pj->p", X[m], Q, X[m])
        s = P[m].sum(axis=0)
        M2 = (P[m].T @ P[m] + np.outer(s, s)) / 20.0    # (1/vol) int x x^T
        xbar = s / 4.0
        exact = vol[m] * (b @ b + 4 * b @ Q @ xbar + 4 * np.trace(Q @ Q @ M2))
        assert uh @ K[m] @ uh == pytest.approx(exact, rel=1e-11)


def test_element_matrix_is_symmetric_and_annihilates_constants():
    rng = np.random.default_rng(12)
    K, _ = element_stiffness_p2(rng.normal(size=(10, 4, 3)))
    assert np.abs(K - np.transpose(K, (0, 2, 1))).max() <= 1e-12 * np.abs(K).max()
    assert np.abs(K.sum(axis=2)).max() <= 1e-12 * np.abs(K).max()


def test_basis_integrals():
    """The integral of a vertex basis function is -|T|/20, of an edge basis
    function |T|/5; together they integrate 1 to |T|."""
    vol = np.array([1 / 6, 0.37])
    L = element_load_p2(vol)
    assert np.allclose(L[:, :4], -vol[:, None] / 20, rtol=1e-14, atol=0)
    assert np.allclose(L[:, 4:], vol[:, None] / 5, rtol=1e-14, atol=0)
    assert np.allclose(L.sum(axis=1), vol, rtol=1e-14, atol=0)


@pytest.mark.parametrize("name,level", [("ref_tet", 1), ("ref_tet", 2),
                                        ("kuhn_211", 1), ("jittered_222", 1),
                                        ("slab_3_11", 1)])
def test_nodes_and_boundary_are_the_next_level_vertices(name, level):
    """The P2 nodes of level l are the micro-vertices of level l + 1 and the
    Dirichlet nodes are the level-(l+1) boundary vertices."""
    S = P2System(*mesh_by_name(name), level)
    M = MicroMesh(*mesh_by_name(name), level + 1)
    assert np.array_equal(S.keys, M.keys)
    assert np.array_equal(S.dirichlet, P1System(M).dirichlet)


@pytest.mark.parametrize("name,level", [("ref_tet", 1), ("ref_tet", 2),
                                        ("kuhn_211", 2), ("jittered_222", 1),
                                        ("jittered_288", 0), ("slab_3_11", 1)])
def test_quadratic_solution_is_reproduced_exactly(name, level):
    """-Laplace u = f with u quadratic: f = -2 tr(Q) is constant, the right-
    hand side is f times the basis integrals, and u lies in the P2 space, so
    the discrete solution equals u at every node (Galerkin exactness)."""
    S = P2System(*mesh_by_name(name), level)
    rng = np.random.default_rng(5)
    b = rng.normal(size=3)
    Q = rng.normal(size=(3, 3))
    Q = Q + Q.T
    X = S.xyz
    u = 0.3 + X @ b + np.einsum("pi,ij,pj->p", X, Q, X)
    f = -2.0 * np.trace(Q)
    uh = S.solve_dirichlet(f * S.load, u)
    assert S.interior.sum() > 0
    assert np.abs(uh - u).max() <= 1e-10 * np.abs(u).max()
    # and the apply of the interpolant gives the load on interior nodes
    y = S.apply(u)
    assert np.abs(y[S.interior] - f * S.load[S.interior]).max() \
        <= 1e-11 * np.abs(S.A).max() * np.abs(u).max()


@pytest.mark.parametrize("name,level", [("jittered_222", 1), ("slab_3_11", 1),
                                        ("ref_tet", 2)])
def test_row_oracle_matches_assembly(name, level):
    xyz, cells = mesh_by_name(name)
    S = P2System(xyz, cells, level)
    rng = np.random.default_rng(3)
    picks = rng.choice(S.num_nodes, size=min(40, S.num_nodes), replace=False)
    for p in picks:
        nbr, vals, dirichlet = p2_row_at(xyz, cells, level, S.keys[p])
        assert dirichlet == bool(S.dirichlet[p])
        row = np.zeros(S.num_nodes)
        row[S.index_of(nbr)] = vals
        want = S.A[p].toarray()[0]
        assert np.abs(row - want).max() <= 1e-13 * np.abs(want).max()


# ------------------------------------------------------ subgroup arrays --
from oracle.p2 import SUBGROUPS, subgroup_arrays, subgroup_width  # noqa: E402


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_subgroup_widths_follow_the_table(level):
    """Vertex width 2^l + 1, six edge subgroups 2^l, xyz 2^l - 1 (subgroup
    table); the shifted index polytopes cover the next level's vertices
    exactly once."""
    n = 2 ** level
    assert [subgroup_width(g, level) for g in range(8)] == [n + 1] + [n] * 6 + [n - 1]
    from oracle.p2 import SUBGROUP_SHIFT
    seen = set()
    for g in range(8):
        w = subgroup_width(g, level)
        for k in range(w):
            for j in range(w - k):
                for i in range(w - k - j):
                    p = tuple(2 * np.array((i, j, k)) + SUBGROUP_SHIFT[g])
                    assert sum(p) <= 2 * n and p not in seen
                    seen.add(p)
    assert len(seen) == N_tet(2 * n + 1)


def test_vertex_subgroup_is_the_tw_order_and_aos_soa_agree():
    """On the reference tet with the identity 'function' (each node's
    level-(l+1) local index), the vertex subgroup lists (2i, 2j, 2k) in t_w
    order (the paper's z-down example order for level 2 reappears at the
    vertices), and AoS / SoA hold the same structures (eq. for AoS and SoA)."""
    xyz, cells = mesh_by_name("ref_tet")
    level, m = 2, 3
    n2 = 2 ** (level + 1)

    def vals(keys):
        w = np.zeros((len(keys), 4), dtype=np.int64)
        ids, wt = keys[:, 0::2], keys[:, 1::2]
        for q in range(4):
            w[:, q] = np.where(ids == cells[0][q], wt, 0).sum(axis=1)
        return np.stack([w[:, 1], w[:, 2], w[:, 3]], axis=1).astype(float)

    aos = subgroup_arrays(cells, level, vals, m, "aos")
    soa = subgroup_arrays(cells, level, vals, m, "soa")
    assert len(aos) == len(soa) == m * N_tet(n2 + 1)
    nv = N_tet(2 ** level + 1)
    v = aos[:m * nv].reshape(nv, m)
    order = [(i, j, k) for k in range(5) for j in range(5 - k) for i in range(5 - k - j)]
    assert np.array_equal(v, 2 * np.array(order, dtype=float))
    off = 0
    for g in range(8):
        w = subgroup_width(g, level)
        N = N_tet(w)
        a = aos[off:off + m * N].reshape(N, m)
        s = soa[off:off + m * N].reshape(m, N)
        assert np.array_equal(a, s.T), SUBGROUPS[g]
        off += m * N
