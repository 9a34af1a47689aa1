"""Helpers that put oracle vectors into the library's slot layout and back.

The library's keys (host call) map every slot to an oracle vertex; values
always originate on the oracle side (seeded inputs in canonical key order)
and results are compared at owner slots, with every ghost copy required to
equal its owner.
"""
import numpy as np

import paper_2308_01792_amd as ht
from paper_2308_01792_amd import _lib
from tests.conftest import mesh_by_name, oracle_hierarchy


class Pair:
    """Library mesh + oracle hierarchy built from the same synthetic input."""

    def __init__(self, name: str, max_level: int, min_level: int = 0,
                 arrays=None):
        self.name = name
        if arrays is None:
            self.H = oracle_hierarchy(name, max_level, min_level)
            arrays = mesh_by_name(name)
        else:
            from oracle.mg import Hierarchy
            self.H = Hierarchy(*arrays, max_level=max_level,
                               min_level=min_level)
        self.m = ht.Mesh(*arrays, min_level, max_level)
        self._maps = {}

    def S(self, level):
        return self.H[level]

    def slot_map(self, level):
        """(oracle index per slot, -1 for padding; flags per slot)."""
        if level not in self._maps:
            keys, flags = self.m.keys(level)
            idx = np.full(len(keys), -1, dtype=np.int64)
            real = flags != _lib.HT_SLOT_PAD
            idx[real] = self.H[level].mesh.index_of(keys[real])
            self._maps[level] = (idx, flags)
        return self._maps[level]

    def to_gpu(self, level, vec, dtype=None):
        import torch
        dtype = torch.float64 if dtype is None else dtype
        idx, _ = self.slot_map(level)
        out = np.zeros(len(idx))
        out[idx >= 0] = vec[idx[idx >= 0]]
        return torch.tensor(out, dtype=dtype, device="cuda")

    def from_gpu(self, level, t, check_consistent=True):
        """Oracle-ordered vector from the owner slots of t."""
        idx, flags = self.slot_map(level)
        v = t.detach().double().cpu().numpy()
        own = (flags & _lib.HT_SLOT_OWNER) > 0
        out = np.zeros(self.H[level].mesh.num_vertices)
        out[idx[own]] = v[own]
        if check_consistent:
            real = idx >= 0
            assert np.array_equal(v[real], out[idx[real]]), \
                "ghost copies differ from their owner"
        return out


def rel_err(a, b):
    scale = np.abs(b).max()
    return np.abs(a - b).max() / (scale if scale > 0 else 1.0)
