"""GPU parity of the variable-coefficient operator div(k grad).

The HIP path (ht_apply_divkgrad) against the oracle's assembled matrix
(P1System with the coefficient's point values, degree-3 rule), element by
element on the same seeded inputs, and at the bench's full size through
properties that hold exactly: a constant coefficient c gives c times the
Laplacian, and affine fields are annihilated on interior rows.

Tolerances: FP64 1e-12 relative to the oracle's max-norm, as for the
Laplacian.  FP32: a row sums 24 micro-cell terms, each a coefficient sum of
four values times a three-term product, about 100 roundings of O(1)
quantities at 2^-24; 3e-5 relative leaves a factor of ~5 over that.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2308_01792_amd as ht  # noqa: E402
from oracle.fem import P1System  # noqa: E402
from tests.gpu_support import Pair, rel_err  # noqa: E402
from workloads import fields  # noqa: E402

FP64_TOL = 1e-12
FP32_TOL = 3e-5

CASES = [("ref_tet", 1), ("ref_tet", 4), ("kuhn_cube", 4), ("kuhn_211", 3),
         ("jittered_288", 2), ("jittered_288", 3), ("jittered_222", 4),
         ("slab_3_11", 3), ("slab_1_1", 3), ("slab_2_7", 0),
         ("jittered_222", 6)]

_PAIRS = {}


def pair(name, level):
    if (name, level) not in _PAIRS:
        _PAIRS[(name, level)] = Pair(name, level, level)
    return _PAIRS[(name, level)]


def divkgrad_case(name, level, dtype):
    P = pair(name, level)
    mesh = P.S(level).mesh
    kv = fields.coefficient_field(mesh.xyz)
    S = P1System(mesh, kappa=kv)
    x = fields.uniform_values(mesh.num_vertices, 14)     # boundary data too
    if dtype == torch.float32:
        kv = kv.astype(np.float32).astype(np.float64)
        x = x.astype(np.float32).astype(np.float64)
        S = P1System(mesh, kappa=kv)
    kg = P.to_gpu(level, kv, dtype)
    xg = P.to_gpu(level, x, dtype)
    yg = torch.full_like(xg, np.nan)
    P.m.apply_divkgrad(level, kg, xg, yg)
    torch.cuda.synchronize()
    y = P.from_gpu(level, yg)
    return y, S.apply(x), S


@pytest.mark.parametrize("name,level", CASES)
def test_divkgrad_fp64(name, level):
    y, ref, S = divkgrad_case(name, level, torch.float64)
    assert np.isfinite(y).all()
    assert rel_err(y, ref) <= FP64_TOL
    assert (y[S.dirichlet] == 0).all()


@pytest.mark.parametrize("name,level", [("ref_tet", 4), ("jittered_288", 3),
                                        ("kuhn_cube", 5)])
def test_divkgrad_fp32(name, level):
    y, ref, _ = divkgrad_case(name, level, torch.float32)
    err = rel_err(y, ref)
    print(f"fp32 div(k grad) {name} l{level}: rel err {err:.2e}")
    assert err <= FP32_TOL


def test_divkgrad_constant_coefficient_is_scaled_laplacian():
    P = pair("jittered_288", 4)
    x = P.to_gpu(4, fields.uniform_values(P.S(4).mesh.num_vertices, 15))
    k = torch.full_like(x, 2.5)
    y1, y2 = torch.zeros_like(x), torch.zeros_like(x)
    P.m.apply_divkgrad(4, k, x, y1)
    P.m.apply(4, x, y2)
    assert float((y1 - 2.5 * y2).abs().max()) <= 1e-13 * float(y1.abs().max())


def test_divkgrad_rejects_aliasing_and_mixed_dtypes():
    P = pair("ref_tet", 2)
    x = torch.zeros(P.m.n_slots(2), dtype=torch.float64, device="cuda")
    with pytest.raises(ht.HytetError):
        P.m.apply_divkgrad(2, x, x, x)
    with pytest.raises(ValueError):
        P.m.apply_divkgrad(2, x.float(), x, torch.zeros_like(x))


def test_divkgrad_is_deterministic():
    P = pair("jittered_288", 3)
    mesh = P.S(3).mesh
    k = P.to_gpu(3, fields.coefficient_field(mesh.xyz))
    x = P.to_gpu(3, fields.uniform_values(mesh.num_vertices, 16))
    y1, y2 = torch.zeros_like(x), torch.zeros_like(x)
    P.m.apply_divkgrad(3, k, x, y1)
    P.m.apply_divkgrad(3, k, x, y2)
    assert torch.equal(y1, y2)


# ------------------------------------------------ stored-stencil variant --
@pytest.mark.parametrize("name,level", [("ref_tet", 4), ("jittered_288", 3),
                                        ("kuhn_211", 3), ("slab_3_11", 3)])
def test_stored_rows_apply_matches_oracle(name, level):
    P = pair(name, level)
    mesh = P.S(level).mesh
    kv = fields.coefficient_field(mesh.xyz)
    S = P1System(mesh, kappa=kv)
    x = fields.uniform_values(mesh.num_vertices, 17)
    kg, xg = P.to_gpu(level, kv), P.to_gpu(level, x)
    rows = P.m.assemble_divkgrad(level, kg)
    yg = torch.full_like(xg, np.nan)
    P.m.apply_stored(level, rows, xg, yg)
    torch.cuda.synchronize()
    y = P.from_gpu(level, yg)
    assert rel_err(y, S.apply(x)) <= FP64_TOL


def test_stored_rows_are_the_matrix_rows():
    """At points inside one macro-cell the 15 stored entries are the
    oracle's matrix entries a(v, v + d) (the diagonal at d = 0)."""
    from oracle.refine import keys_of
    level = 3
    P = pair("jittered_288", level)
    mesh = P.S(level).mesh
    kv = fields.coefficient_field(mesh.xyz)
    A = P1System(mesh, kappa=kv).A.tocsr()
    rows = P.m.assemble_divkgrad(level, P.to_gpu(level, kv)).cpu().numpy()
    nslot = P.m.n_slots(level)
    stride = nslot // len(mesh.cells)
    offs = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
            (0, 0, 1), (0, 0, -1), (-1, 1, 0), (1, -1, 0), (-1, 0, 1),
            (1, 0, -1), (0, -1, 1), (0, 1, -1), (1, -1, 1), (-1, 1, -1)]
    n = 2 ** level

    def vertex(c, i, j, k):
        w = np.array([[n - i - j - k, i, j, k]], dtype=np.int64)
        return int(mesh.index_of(keys_of(mesh.cells[c], w))[0])

    checked = 0
    for c in (0, 17, 200):
        for (i, j, k) in [(1, 1, 1), (2, 3, 1), (1, 2, 4), (3, 2, 2)]:
            s = P.m.slot_index(level, c, i, j, k)
            local = s - c * stride
            v = vertex(c, i, j, k)
            for d, (di, dj, dk) in enumerate(offs):
                w = vertex(c, i + di, j + dj, k + dk)
                got = rows[c * 15 * stride + d * stride + local]
                assert abs(got - A[v, w]) <= 1e-13 * abs(A[v, v]), (c, i, j, k, d)
            checked += 1
    assert checked == 12


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-13),
                                       (torch.float32, 3e-5)])
def test_stored_equals_matrix_free(dtype, tol):
    P = pair("jittered_288", 4)
    mesh = P.S(4).mesh
    kg = P.to_gpu(4, fields.coefficient_field(mesh.xyz), dtype)
    xg = P.to_gpu(4, fields.uniform_values(mesh.num_vertices, 18), dtype)
    y1, y2 = torch.zeros_like(xg), torch.zeros_like(xg)
    P.m.apply_divkgrad(4, kg, xg, y1)
    P.m.apply_stored(4, P.m.assemble_divkgrad(4, kg), xg, y2)
    scale = float(y1.abs().max())
    assert float((y1 - y2).abs().max()) <= tol * scale


def test_stored_rejects_wrong_row_count():
    P = pair("ref_tet", 2)
    x = torch.zeros(P.m.n_slots(2), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        P.m.apply_stored(2, x, x, torch.zeros_like(x))
