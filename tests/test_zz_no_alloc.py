"""ht_residual_noalloc (the allocation-free variant of ht_residual) against
ht_residual through the C ABI: two calls in a row, the second on a smaller
input, and the argument checks."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2308_01792_amd as ht  # noqa: E402
from paper_2308_01792_amd import _lib  # noqa: E402
from tests.gpu_support import Pair, rel_err  # noqa: E402
from workloads import fields  # noqa: E402

FP64_TOL = 1e-12


def _case(name, level, seed):
    P = Pair(name, level, level)
    S = P.S(level)
    N = S.mesh.num_vertices
    u = np.where(S.dirichlet, 0.0, fields.uniform_values(N, seed))
    b = fields.uniform_values(N, seed + 1)
    return P, S, P.to_gpu(level, u), P.to_gpu(level, b), u, b


def test_noalloc_residual_matches_residual_twice():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    big = _case("jittered_288", 4, 31)
    small = _case("ref_tet", 3, 41)              # the second, smaller input
    for (P, S, ug, bg, u, b), level in ((big, 4), (small, 3)):
        # slots that hold micro-vertices (outputs leave the padding alone)
        idx, _ = P.slot_map(level)
        real = torch.tensor(idx >= 0, device="cuda")
        r_ref = torch.zeros_like(ug)
        nrm_ref = P.m.residual(level, ug, bg, r_ref, want_norm=True)
        r = torch.full_like(ug, np.nan)
        nrm = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
        P.m.residual_noalloc(level, ug, bg, r, nrm)
        torch.cuda.synchronize()
        # same kernels, same summation order: equal to the last bit
        assert torch.equal(r[real], r_ref[real])
        assert float(nrm[0]) == nrm_ref
        # and against the oracle
        ro = S.residual(u, b)
        assert rel_err(P.from_gpu(level, r), ro) <= FP64_TOL
        assert float(nrm[0]) == pytest.approx(np.linalg.norm(ro[S.interior]),
                                              rel=FP64_TOL)
        # without a norm destination
        r2 = torch.full_like(ug, np.nan)
        P.m.residual_noalloc(level, ug, bg, r2)
        assert torch.equal(r2[real], r_ref[real])


def test_noalloc_residual_argument_checks():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from tests.conftest import mesh_by_name
    xyz, cells = mesh_by_name("jittered_288")
    t = torch.zeros(1024, dtype=torch.float64, device="cuda")
    # not on the device yet: the upload would allocate
    m = ht.Mesh(xyz, cells, 2, 9)
    with pytest.raises(ht.HytetError) as e:
        m.residual_noalloc(3, t, t.clone(), t.clone())
    assert e.value.code == _lib.HT_ERR_STATE
    m.lumped_mass(2, torch.zeros(m.n_slots(2), dtype=torch.float64, device="cuda"))
    # level 9 of the 288-cell box needs more partials than the scratch holds
    with pytest.raises(ht.HytetError) as e:
        m.residual_noalloc(9, t, t.clone(), t.clone())
    assert e.value.code == _lib.HT_ERR_ARG
    assert "scratch" in str(e.value)
    with pytest.raises(ht.HytetError) as e:
        m.residual_noalloc(3, t, t, t)
    assert e.value.code == _lib.HT_ERR_ARG
