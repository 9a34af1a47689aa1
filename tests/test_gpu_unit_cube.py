"""The unit cube as six Kuhn tetrahedra at level 7 (128 intervals per edge,
2,048,383 unknowns): apply, ghost exchange and V(2,2) iterates over levels
2..7 against the oracle assembled element by element at that level.

The oracle hierarchy 2..7 takes about 90 s and 12 GB of host memory; it is
built once for the module and released afterwards.  The right-hand side is
the manufactured one of the benchmark configuration: b = m * f with
f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) at the micro-vertices."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2308_01792_amd as ht  # noqa: E402
from tests.conftest import mesh_by_name  # noqa: E402
from tests.gpu_support import Pair, rel_err  # noqa: E402
from workloads import fields  # noqa: E402

FP64_TOL = 1e-12
LEVEL = 7


@pytest.fixture(scope="module")
def cube():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    P = Pair("kuhn_cube", LEVEL, 2, arrays=mesh_by_name("kuhn_cube"))
    yield P
    del P


def test_unit_cube_sizes(cube):
    S = cube.S(LEVEL)
    assert int(S.interior.sum()) == 127 ** 3 == cube.m.info(LEVEL)["n_dofs"]


@pytest.mark.parametrize("rows", [0, 4])
def test_apply_level7_unit_cube(cube, rows):
    """Every interior row (cell interiors, the six interior faces, the inner
    diagonal edge) with the band kernel (rows 0) and the tile kernel."""
    S = cube.S(LEVEL)
    x = fields.uniform_values(S.mesh.num_vertices, 4)
    cube.m.set_tile_rows(LEVEL, ht.HT_F64, rows)
    xg = cube.to_gpu(LEVEL, x)
    yg = torch.zeros_like(xg)
    cube.m.apply(LEVEL, xg, yg)
    err = rel_err(cube.from_gpu(LEVEL, yg), S.apply(x))
    print(f"level {LEVEL} apply (rows {rows}): rel err {err:.2e}")
    assert err <= FP64_TOL


def test_vcycle_iterates_level7_unit_cube(cube):
    """Three V(2,2) cycles over levels 2..7 from u0 = 0: every iterate."""
    S = cube.S(LEVEL)
    X = S.mesh.xyz
    f = 3 * np.pi ** 2 * np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * \
        np.sin(np.pi * X[:, 2])
    b = S.lumped_mass * f
    bg = cube.to_gpu(LEVEL, b)
    ug = torch.zeros_like(bg)
    u = np.zeros_like(b)
    for k in range(3):
        cube.m.vcycle(LEVEL, ug, bg, 2, 2, 2.0 / 3.0, 2)
        u = cube.H.vcycle(LEVEL, u, b, 2, 2, 2.0 / 3.0, 2)
        err = rel_err(cube.from_gpu(LEVEL, ug), u)
        print(f"level {LEVEL} V(2,2) iterate {k + 1}: rel err {err:.2e}")
        assert err <= FP64_TOL, k
