"""Batched solves of many independent small problems.

A batch lays the problems side by side and runs one V-cycle over absolute
levels for all of them.  Every problem must get what it gets when solved on
its own (same iterates up to rounding, same cycle count), and what the
oracle's multigrid computes for it.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2308_01792_amd as ht  # noqa: E402
from tests.gpu_support import Pair, rel_err  # noqa: E402
from workloads import batch_problems, fields  # noqa: E402

PROBLEMS = batch_problems(count=12, seed=6, min_level=3, max_level=5)


def _rhs(mesh, level, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    f = torch.rand(mesh.n_slots(level), dtype=torch.float64, device="cuda",
                   generator=g) * 2 - 1
    mesh.sync(level, f)
    m = torch.zeros_like(f)
    mesh.lumped_mass(level, m)
    return m * f


@pytest.fixture(scope="module")
def setup():
    meshes = [ht.Mesh(p.xyz, p.cells, 2, p.level) for p in PROBLEMS]
    bs = [_rhs(m, p.level, 100 + p.index) for m, p in zip(meshes, PROBLEMS)]
    batch = ht.Batch(meshes, [p.level for p in PROBLEMS])
    return meshes, bs, batch


def _individual(meshes, bs, precision=ht.HT_PREC_F64, **kw):
    out = []
    for m, b, p in zip(meshes, bs, PROBLEMS):
        u = torch.zeros_like(b)
        st = m.solve(p.level, u, b, precision, **kw)
        out.append((u, st))
    return out


def test_batch_problems_span_levels_and_kinds():
    assert {p.level for p in PROBLEMS} == {3, 4, 5}
    assert {p.kind for p in PROBLEMS} == {"box", "slab"}


def test_batch_query(setup):
    meshes, _, batch = setup
    info = batch.info()
    assert info["problems"] == len(PROBLEMS)
    assert info["dofs"] == sum(m.info(p.level)["n_dofs"]
                               for m, p in zip(meshes, PROBLEMS))
    assert info["cells"] == sum(len(p.cells) for p in PROBLEMS)


@pytest.mark.parametrize("nu", [(2, 2), (1, 1), (0, 2), (3, 1)])
def test_fixed_cycles_give_the_individual_iterates(setup, nu):
    """Three cycles (tolerance never met): each problem's iterate equals the
    one its own solve computes."""
    meshes, bs, batch = setup
    kw = dict(rel_tol=0.0, max_cycles=3, nu1=nu[0], nu2=nu[1],
              raise_on_fail=False)
    ref = _individual(meshes, bs, **kw)
    us = [torch.zeros_like(b) for b in bs]
    st = batch.solve(us, bs, **kw)
    for p, (u, (ur, sr)) in enumerate(zip(us, ref)):
        assert st[p]["cycles"] == 3 and not st[p]["converged"]
        assert np.allclose(st[p]["history"], sr["history"], rtol=1e-12, atol=0)
        a, r = u.cpu().numpy(), ur.cpu().numpy()
        assert rel_err(a, r) <= 1e-12, p


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_solve_matches_individual_solves(setup, use_graph):
    meshes, bs, batch = setup
    ref = _individual(meshes, bs, rel_tol=1e-10, max_cycles=100)
    us = [torch.zeros_like(b) for b in bs]
    st = batch.solve(us, bs, rel_tol=1e-10, max_cycles=100,
                     use_graph=use_graph)
    for p, (u, (ur, sr)) in enumerate(zip(us, ref)):
        assert st[p]["converged"] and st[p]["rel_res"] <= 1e-10
        assert abs(st[p]["cycles"] - sr["cycles"]) <= 1
        assert np.allclose(st[p]["history"][:4], sr["history"][:4],
                           rtol=1e-10, atol=0)
        assert rel_err(u.cpu().numpy(), ur.cpu().numpy()) <= 1e-9, p


def test_graph_replay_is_bitwise_eager(setup):
    _, bs, batch = setup
    res = []
    for g in (False, True, True):
        us = [torch.zeros_like(b) for b in bs]
        st = batch.solve(us, bs, rel_tol=1e-10, max_cycles=100, use_graph=g)
        res.append((us, [s["history"] for s in st]))
    for us, hist in res[1:]:
        assert hist == res[0][1]
        assert all(torch.equal(a, b) for a, b in zip(us, res[0][0]))


# ------------------------------------------ FP32-in-FP64 refinement --
def test_mixed_fixed_cycles_give_the_individual_iterates(setup):
    """Three refinement steps: FP32 correction cycles of all problems in one
    batched V-cycle give each problem the iterate of its own mixed solve."""
    meshes, bs, batch = setup
    kw = dict(rel_tol=0.0, max_cycles=3, raise_on_fail=False)
    ref = _individual(meshes, bs, ht.HT_PREC_MIXED, **kw)
    us = [torch.zeros_like(b) for b in bs]
    st = batch.solve(us, bs, precision=ht.HT_PREC_MIXED, **kw)
    for p, (u, (ur, sr)) in enumerate(zip(us, ref)):
        assert st[p]["cycles"] == 3
        assert np.allclose(st[p]["history"], sr["history"], rtol=1e-12, atol=0)
        assert rel_err(u.cpu().numpy(), ur.cpu().numpy()) <= 1e-12, p


@pytest.mark.parametrize("use_graph", [False, True])
def test_mixed_batch_solve_matches_individual_solves(setup, use_graph):
    meshes, bs, batch = setup
    ref = _individual(meshes, bs, ht.HT_PREC_MIXED, rel_tol=1e-10,
                      max_cycles=100)
    us = [torch.zeros_like(b) for b in bs]
    st = batch.solve(us, bs, rel_tol=1e-10, max_cycles=100,
                     use_graph=use_graph, precision=ht.HT_PREC_MIXED)
    for p, (u, (ur, sr)) in enumerate(zip(us, ref)):
        assert st[p]["converged"] and st[p]["rel_res"] <= 1e-10
        assert abs(st[p]["cycles"] - sr["cycles"]) <= 1
        assert rel_err(u.cpu().numpy(), ur.cpu().numpy()) <= 1e-9, p


def test_mixed_graph_replay_is_bitwise_eager(setup):
    _, bs, batch = setup
    res = []
    for g in (False, True, True):
        us = [torch.zeros_like(b) for b in bs]
        st = batch.solve(us, bs, rel_tol=1e-10, max_cycles=100, use_graph=g,
                         precision=ht.HT_PREC_MIXED)
        res.append((us, [s["history"] for s in st]))
    for us, hist in res[1:]:
        assert hist == res[0][1]
        assert all(torch.equal(a, b) for a, b in zip(us, res[0][0]))


def test_batch_against_oracle():
    """Three level-3 problems of different kinds, solved in one batch, match
    the oracle's V(2,2) multigrid."""
    probs = batch_problems(count=40, seed=6, min_level=3, max_level=3)
    pick = [probs[0], next(p for p in probs if p.kind != probs[0].kind),
            probs[5]]
    pairs = [Pair(f"batch{p.index}", 3, 2, arrays=(p.xyz, p.cells))
             for p in pick]
    bs_or = []
    for P, p in zip(pairs, pick):
        S = P.S(3)
        bs_or.append(S.lumped_mass * fields.uniform_values(
            S.mesh.num_vertices, p.rhs_seed))
    batch = ht.Batch([P.m for P in pairs], [3, 3, 3])
    bs = [P.to_gpu(3, b) for P, b in zip(pairs, bs_or)]
    us = [torch.zeros_like(b) for b in bs]
    st = batch.solve(us, bs, rel_tol=1e-10, max_cycles=100)
    for P, b, u, s in zip(pairs, bs_or, us, st):
        uo, hist = P.H.solve(3, b, rel_tol=1e-10, coarse_level=2)
        assert abs(s["cycles"] - (len(hist) - 1)) <= 1
        assert np.allclose(s["history"][:4], hist[:4], rtol=1e-9, atol=0)
        assert rel_err(P.from_gpu(3, u), uo) <= 1e-9
    batch.close()


def test_coarse_level_above_a_problem_is_rejected(setup):
    _, bs, batch = setup
    us = [torch.zeros_like(b) for b in bs]
    with pytest.raises(ht.HytetError, match="HT_ERR_LEVEL"):
        batch.solve(us, bs, coarse_level=4)


def test_autotuned_batch_matches_individual_solves():
    """The batch's union mesh tuned level by level on the problems present
    there (apply kernel, sweep rows, arrangement and march segment) solves
    to the same iterates and cycle counts as the untuned loop of single
    solves, in FP64 and FP32-in-FP64."""
    meshes = [ht.Mesh(p.xyz, p.cells, 2, p.level) for p in PROBLEMS]
    bs = [_rhs(m, p.level, 100 + p.index) for m, p in zip(meshes, PROBLEMS)]
    batch = ht.Batch(meshes, [p.level for p in PROBLEMS])
    batch.autotune()
    shapes = batch.shapes(range(3, 6))
    for lv, per in shapes.items():
        for name, sh in per.items():
            assert sh["apply_rows"] in (0, 4, 8, 16)
            assert sh["sweep_rows"] in (0, 4, 8, 16)   # 0: the band kernel
            assert sh["segment"] in (32, 64, 128)
    for prec in (ht.HT_PREC_F64, ht.HT_PREC_MIXED):
        us = [torch.zeros_like(b) for b in bs]
        st = batch.solve(us, bs, rel_tol=1e-10, max_cycles=100, precision=prec)
        ref = _individual(meshes, bs, prec, rel_tol=1e-10, max_cycles=100)
        for (ur, sr), u, s in zip(ref, us, st):
            assert s["cycles"] == sr["cycles"]
            assert rel_err(u.cpu().numpy(), ur.cpu().numpy()) <= 1e-12


def test_mixed_update_inside_the_last_sweep_matches_a_separate_update():
    """From level 7 on, a single mixed solve adds each FP32 correction to u
    inside its last post-smoothing sweep (band kernel); the batch path keeps
    the separate update pass.  Three refinement steps of one jittered box at
    level 7 give the same iterate both ways."""
    from workloads import jittered_kuhn_box
    L = 7
    m = ht.Mesh(*jittered_kuhn_box(2, 1, 1, amplitude=0.1, seed=4), 2, L)
    b = _rhs(m, L, 77)
    kw = dict(rel_tol=0.0, max_cycles=3, raise_on_fail=False)
    u1 = torch.zeros_like(b)
    s1 = m.solve(L, u1, b, ht.HT_PREC_MIXED, **kw)
    batch = ht.Batch([m], [L])
    u2 = torch.zeros_like(b)
    s2 = batch.solve([u2], [b], precision=ht.HT_PREC_MIXED, **kw)[0]
    assert s1["cycles"] == s2["cycles"] == 3
    assert np.allclose(s1["history"], s2["history"], rtol=1e-12, atol=0)
    assert rel_err(u1.cpu().numpy(), u2.cpu().numpy()) <= 1e-13


def test_batch_problems_stop_when_their_residual_stagnates(setup):
    """A tolerance below the FP64 rounding floor: every problem stops three
    cycles after its residual's last new minimum (stagnated, not converged),
    well before max_cycles, and keeps the iterate of that cycle."""
    meshes, bs, batch = setup
    us = [torch.zeros_like(b) for b in bs]
    st = batch.solve(us, bs, rel_tol=1e-30, max_cycles=200, raise_on_fail=False)
    for p, s in enumerate(st):
        h = np.array(s["history"])
        kbest = int(np.argmin(h))
        assert s["stagnated"] and not s["converged"], p
        assert s["cycles"] < 200 and s["cycles"] - kbest == 3, p
        assert h[kbest] <= 1e-14 and (h[kbest + 1:] >= h[kbest]).all(), p
    # the frozen iterate is the one whose residual was reported
    for p in (0, len(bs) - 1):
        m, lvl = meshes[p], PROBLEMS[p].level
        r = torch.zeros_like(bs[p])
        nr = m.residual(lvl, us[p], bs[p], r, want_norm=True)
        nb = m.norm(lvl, bs[p])
        assert abs(nr / nb - st[p]["rel_res"]) <= 1e-3 * st[p]["rel_res"], p
