import os
import sys
from functools import lru_cache

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an AMD GPU (MI355X / gfx950) and the built HIP "
        "library")
    config.addinivalue_line(
        "markers", "slow: CPU test that takes more than a few seconds")


@lru_cache(maxsize=None)
def oracle_hierarchy(name: str, max_level: int, min_level: int = 0):
    """Cached oracle hierarchies for the named synthetic meshes."""
    from oracle.mg import Hierarchy
    return Hierarchy(*mesh_by_name(name), max_level=max_level,
                     min_level=min_level)


def mesh_by_name(name: str):
    import workloads as W
    if name == "ref_tet":
        return W.reference_tet()
    if name == "kuhn_cube":
        return W.kuhn_box(1, 1, 1)
    if name == "kuhn_211":
        return W.kuhn_box(2, 1, 1)
    if name == "jittered_288":
        return W.jittered_kuhn_box(4, 4, 3, amplitude=0.1, seed=3)
    if name == "jittered_222":
        return W.jittered_kuhn_box(2, 2, 2, amplitude=0.1, seed=3)
    if name.startswith("slab_"):
        _, m, t = name.split("_")
        return W.slab(int(m), int(t), seed=7)
    raise KeyError(name)


@pytest.fixture(scope="session")
def hierarchy():
    return oracle_hierarchy
