"""Python binding of libhytet (matrix-free P1 on refined macro-tetrahedra).

Argument marshalling only: every computation runs in the HIP kernels of
``libhytet.so`` (C ABI in ``include/hytet.h``).  PyTorch provides device
memory and streams; vectors are 1-D CUDA tensors of ``n_slots`` elements
(float64 or float32) in the library's closure layout.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (HT_F32, HT_F64, HT_PREC_F64, HT_PREC_MIXED,
                   HT_SMOOTH_CHEBYSHEV, HT_SMOOTH_JACOBI,
                   HT_SLOT_DIRICHLET, HT_SLOT_GHOST, HT_SLOT_OWNER,
                   HT_SLOT_PAD, HytetError, check)

__all__ = ["Mesh", "Batch", "HytetError", "load", "HT_F64", "HT_F32", "HT_PREC_F64",
           "HT_PREC_MIXED", "HT_SMOOTH_JACOBI", "HT_SMOOTH_CHEBYSHEV",
           "HT_SLOT_OWNER", "HT_SLOT_GHOST",
           "HT_SLOT_DIRICHLET", "HT_SLOT_PAD", "index_tw", "p2_offsets",
           "selftest_lane_shift"]


def load():
    return _lib.load()


def _layout_code(layout: str) -> int:
    if layout not in ("aos", "soa"):
        raise ValueError("layout must be 'aos' or 'soa'")
    return 0 if layout == "aos" else 1


def p2_offsets():
    """(len[8], d[8][65][3]) stencil offsets of the P2 operator per node
    parity on the finer lattice."""
    ln = np.empty(8, dtype=np.int32)
    d = np.empty((8, 65, 3), dtype=np.int32)
    check(load().ht_p2_offsets(ln.ctypes.data, d.ctypes.data))
    return ln, d


def index_tw(w: int, i: int, j: int, k: int) -> int:
    return int(load().ht_index_tw(w, i, j, k))


def selftest_lane_shift() -> int:
    bad = C.c_int(-1)
    check(load().ht_selftest_lane_shift(C.byref(bad)))
    return bad.value


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return HT_F64
    if t.dtype == torch.float32:
        return HT_F32
    raise TypeError("vectors must be float64 or float32 tensors")


def _ptr(t):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("vectors must be contiguous device tensors")
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Mesh:
    """A coarse tetrahedral mesh refined to levels ``min_level..max_level``."""

    def __init__(self, xyz, cells, min_level: int, max_level: int):
        lib = load()
        self._xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self._cells = np.ascontiguousarray(cells, dtype=np.int64)
        h = C.c_void_p()
        check(lib.ht_mesh_create(self._xyz.ctypes.data, len(self._xyz),
                                 self._cells.ctypes.data, len(self._cells),
                                 min_level, max_level, C.byref(h)))
        self._h = h
        self.min_level, self.max_level = min_level, max_level

    def close(self):
        if getattr(self, "_h", None):
            load().ht_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- host ----
    def info(self, level: int) -> dict:
        li = _lib.LevelInfo()
        check(load().ht_mesh_query(self._h, level, C.byref(li)))
        return {f: getattr(li, f) for f, _ in li._fields_}

    def n_slots(self, level: int) -> int:
        return self.info(level)["n_slots"]

    def keys(self, level: int, first: int = 0, count: int | None = None):
        if count is None:
            count = self.n_slots(level) - first
        keys = np.empty((count, 8), dtype=np.int64)
        flags = np.empty(count, dtype=np.uint8)
        check(load().ht_vertex_keys(self._h, level, first, count,
                                    keys.ctypes.data, flags.ctypes.data))
        return keys, flags

    def coords(self, level: int, first: int = 0, count: int | None = None):
        if count is None:
            count = self.n_slots(level) - first
        out = np.empty((count, 3), dtype=np.float64)
        check(load().ht_vertex_coords(self._h, level, first, count,
                                      out.ctypes.data))
        return out

    def slot_index(self, level: int, cell: int, i: int, j: int, k: int) -> int:
        s = C.c_int64()
        check(load().ht_slot_index(self._h, level, cell, i, j, k, C.byref(s)))
        return s.value

    def cell_stencils(self, level: int) -> np.ndarray:
        out = np.empty((len(self._cells), 16, 15), dtype=np.float64)
        check(load().ht_cell_stencils(self._h, level, out.ctypes.data))
        return out

    def p2_stencils(self, level: int) -> np.ndarray:
        """Class-partial P2 stencils [nc][8 parities][16 classes][65]."""
        out = np.empty((len(self._cells), 8, 16, 65), dtype=np.float64)
        check(load().ht_p2_stencils(self._h, level, out.ctypes.data))
        return out

    # -------------------------------------------------------- device ----
    def new_vector(self, level: int, dtype=None):
        import torch
        dtype = torch.float64 if dtype is None else dtype
        return torch.zeros(self.n_slots(level), dtype=dtype, device="cuda")

    def coords_device(self, level: int, out):
        check(load().ht_vertex_coords_device(self._h, level, _dtype_code(out),
                                             _ptr(out), _stream()))
        return out

    def flags_device(self, level: int, out):
        check(load().ht_slot_flags_device(self._h, level, _ptr(out),
                                          _stream()))
        return out

    def sync(self, level: int, v):
        check(load().ht_sync(self._h, level, _dtype_code(v), _ptr(v),
                             _stream()))
        return v

    def fill_dirichlet(self, level: int, v, value: float = 0.0):
        check(load().ht_fill_dirichlet(self._h, level, _dtype_code(v), _ptr(v),
                                       float(value), _stream()))
        return v

    def lumped_mass(self, level: int, out):
        check(load().ht_lumped_mass(self._h, level, _dtype_code(out),
                                    _ptr(out), _stream()))
        return out

    def norm(self, level: int, v) -> float:
        r = C.c_double()
        check(load().ht_norm(self._h, level, _dtype_code(v), _ptr(v),
                             C.byref(r), _stream()))
        return r.value

    def dot(self, level: int, a, b) -> float:
        r = C.c_double()
        check(load().ht_dot(self._h, level, _dtype_code(a), _ptr(a), _ptr(b),
                            C.byref(r), _stream()))
        return r.value

    def copy(self, level: int, src, dst):
        check(load().ht_copy(self._h, level, _dtype_code(src), _ptr(src),
                             _ptr(dst), _stream()))
        return dst

    def apply(self, level: int, x, y):
        check(load().ht_apply(self._h, level, _dtype_code(x), _ptr(x), _ptr(y),
                              _stream()))
        return y

    def apply_divkgrad(self, level: int, kappa, x, y):
        """y = A_k x, the div(k grad) operator with k given by its values at
        the slots (consistent copies); y = 0 at Dirichlet slots."""
        if kappa.dtype != x.dtype:
            raise ValueError("kappa and x must have the same dtype")
        check(load().ht_apply_divkgrad(self._h, level, _dtype_code(x),
                                       _ptr(kappa), _ptr(x), _ptr(y),
                                       _stream()))
        return y

    def apply_p2(self, level: int, x, y):
        """y = A x for the P2 Laplacian of P2 level ``level``; x and y are
        vectors of level + 1 (the P2 nodes are that level's micro-vertices).
        y = 0 at Dirichlet nodes."""
        check(load().ht_apply_p2(self._h, level, _dtype_code(x), _ptr(x),
                                 _ptr(y), _stream()))
        return y

    def p2_pack(self, level: int, lattice, m: int = 1, layout: str = "aos",
                out=None):
        """Per-cell subgroup arrays of m P2 functions given as m vectors of
        level + 1 back to back in ``lattice`` (see ht_p2_pack)."""
        import torch
        n = 2 ** (level + 1) + 1
        size = len(self._cells) * m * (n * (n + 1) * (n + 2) // 6)
        if out is None:
            out = torch.empty(size, dtype=lattice.dtype, device=lattice.device)
        check(load().ht_p2_pack(self._h, level, _dtype_code(lattice), m,
                                _layout_code(layout), _ptr(lattice), _ptr(out),
                                _stream()))
        return out

    def p2_unpack(self, level: int, arrays, lattice, m: int = 1,
                  layout: str = "aos"):
        """Inverse of p2_pack: write every copy of every node of ``lattice``
        (m vectors of level + 1) from the subgroup arrays."""
        check(load().ht_p2_unpack(self._h, level, _dtype_code(arrays), m,
                                  _layout_code(layout), _ptr(arrays),
                                  _ptr(lattice), _stream()))
        return lattice

    def assemble_divkgrad(self, level: int, kappa, rows=None):
        """The 15 row entries of A_k per slot, [cell][offset][closure slot]
        (15 * n_slots elements, kappa's dtype)."""
        import torch
        if rows is None:
            rows = torch.empty(15 * self.n_slots(level), dtype=kappa.dtype,
                               device=kappa.device)
        check(load().ht_assemble_divkgrad(self._h, level, _dtype_code(kappa),
                                          _ptr(kappa), _ptr(rows), _stream()))
        return rows

    def apply_stored(self, level: int, rows, x, y):
        """y = A x with the rows of :meth:`assemble_divkgrad`."""
        if rows.dtype != x.dtype or rows.numel() != 15 * self.n_slots(level):
            raise ValueError("rows must hold 15 * n_slots entries of x's dtype")
        check(load().ht_apply_stored(self._h, level, _dtype_code(x), _ptr(rows),
                                     _ptr(x), _ptr(y), _stream()))
        return y

    def residual(self, level: int, u, b, r, want_norm: bool = False):
        nrm = C.c_double()
        check(load().ht_residual(self._h, level, _dtype_code(u), _ptr(u),
                                 _ptr(b), _ptr(r),
                                 C.byref(nrm) if want_norm else None,
                                 _stream()))
        return nrm.value if want_norm else r

    def residual_noalloc(self, level: int, u, b, r, norm_dev=None):
        """ht_residual_noalloc: r = b - A u with the library's fixed scratch;
        norm_dev: a one-element FP64 device tensor that receives ||r||_2,
        or None."""
        check(load().ht_residual_noalloc(
            self._h, level, _dtype_code(u), _ptr(u), _ptr(b), _ptr(r),
            _ptr(norm_dev) if norm_dev is not None else None, _stream()))
        return r

    def smooth_jacobi(self, level: int, u, b, omega: float = 2.0 / 3.0,
                      sweeps: int = 1):
        check(load().ht_smooth_jacobi(self._h, level, _dtype_code(u),
                                      float(omega), int(sweeps), _ptr(u),
                                      _ptr(b), _stream()))
        return u

    def restrict(self, fine_level: int, r_fine, r_coarse):
        check(load().ht_restrict(self._h, fine_level, _dtype_code(r_fine),
                                 _ptr(r_fine), _ptr(r_coarse), _stream()))
        return r_coarse

    def prolongate_add(self, coarse_level: int, e_coarse, u_fine):
        check(load().ht_prolongate_add(self._h, coarse_level,
                                       _dtype_code(e_coarse), _ptr(e_coarse),
                                       _ptr(u_fine), _stream()))
        return u_fine

    def coarse_solve(self, level: int, b, u):
        check(load().ht_coarse_solve(self._h, level, _dtype_code(b), _ptr(b),
                                     _ptr(u), _stream()))
        return u

    @staticmethod
    def cycle_opts(nu1=2, nu2=2, omega=2.0 / 3.0, coarse_level=2,
                   smoother=HT_SMOOTH_JACOBI, degree=2):
        return _lib.CycleOpts(nu1, nu2, omega, coarse_level, smoother, degree)

    def lambda_max(self, level: int) -> float:
        r = C.c_double()
        check(load().ht_lambda_max(self._h, level, C.byref(r), _stream()))
        return r.value

    def set_lambda_max(self, level: int, value: float):
        check(load().ht_set_lambda_max(self._h, level, float(value)))

    def vcycle(self, level: int, u, b, nu1=2, nu2=2, omega=2.0 / 3.0,
               coarse_level=2, smoother=HT_SMOOTH_JACOBI, degree=2):
        o = self.cycle_opts(nu1, nu2, omega, coarse_level, smoother, degree)
        check(load().ht_vcycle(self._h, level, _dtype_code(u), C.byref(o),
                               _ptr(u), _ptr(b), _stream()))
        return u

    def solve(self, level: int, u, b, precision=HT_PREC_F64, rel_tol=1e-10,
              max_cycles=100, nu1=2, nu2=2, omega=2.0 / 3.0, coarse_level=2,
              use_graph=True, raise_on_fail=True, smoother=HT_SMOOTH_JACOBI,
              degree=2):
        o = _lib.SolveOpts(self.cycle_opts(nu1, nu2, omega, coarse_level,
                                           smoother, degree),
                           precision, rel_tol, max_cycles, int(use_graph))
        st = _lib.SolveStats()
        code = load().ht_solve(self._h, level, C.byref(o), _ptr(u), _ptr(b),
                               C.byref(st), _stream())
        if code != _lib.HT_ERR_NOT_CONVERGED or raise_on_fail:
            check(code)
        return _stats_dict(st)

    def fmg(self, level: int, u, b, cycles=5, nu1=2, nu2=2, omega=2.0 / 3.0,
            coarse_level=2, want_residual=True, smoother=HT_SMOOTH_JACOBI,
            degree=2):
        """Full multigrid into u; returns the relative residual (or None)."""
        o = self.cycle_opts(nu1, nu2, omega, coarse_level, smoother, degree)
        r = C.c_double()
        check(load().ht_fmg(self._h, level, C.byref(o), int(cycles), _ptr(u),
                            _ptr(b), C.byref(r) if want_residual else None,
                            _stream()))
        return r.value if want_residual else None

    # -------------------------------------------------------- tuning ----
    def set_tile_rows(self, level: int, dtype_code: int, rows: int):
        check(load().ht_set_tile_rows(self._h, level, dtype_code, rows))

    def tile_rows(self, level: int, dtype_code: int) -> int:
        r = C.c_int()
        check(load().ht_get_tile_rows(self._h, level, dtype_code, C.byref(r)))
        return r.value

    def set_sweep_shape(self, level: int, dtype_code: int, rows: int,
                        waves_in_i: bool):
        check(load().ht_set_sweep_shape(self._h, level, dtype_code, rows,
                                        int(waves_in_i)))

    def sweep_shape(self, level: int, dtype_code: int):
        """(rows per wave, waves side by side in i) of the sweep operations."""
        r, w = C.c_int(), C.c_int()
        check(load().ht_get_sweep_shape(self._h, level, dtype_code,
                                        C.byref(r), C.byref(w)))
        return r.value, bool(w.value)

    def set_march_segment(self, level: int, dtype_code: int, planes: int):
        check(load().ht_set_march_segment(self._h, level, dtype_code, planes))

    def march_segment(self, level: int, dtype_code: int) -> int:
        """Planes per march segment of the sweep operations."""
        r = C.c_int()
        check(load().ht_get_march_segment(self._h, level, dtype_code, C.byref(r)))
        return r.value

    def autotune(self, level: int, dtype_code: int, cache_path=None) -> int:
        r = C.c_int()
        check(load().ht_autotune(self._h, level, dtype_code,
                                 cache_path.encode() if cache_path else None,
                                 C.byref(r), _stream()))
        return r.value

    # ----------------------------------------------------- profiling ----
    def profile(self, enable: bool = True):
        check(load().ht_profile_enable(self._h, int(enable)))

    def profile_reset(self):
        check(load().ht_profile_reset(self._h))

    def profile_query(self, prefix: str):
        ms, n = C.c_double(), C.c_int64()
        check(load().ht_profile_query(self._h, prefix.encode(), C.byref(ms),
                                      C.byref(n)))
        return ms.value, n.value


def _stats_dict(st):
    return {"cycles": st.cycles, "converged": bool(st.converged),
            "stagnated": bool(st.stagnated),
            "rel_res": st.rel_res, "seconds": st.seconds,
            "history": list(st.res_history[:st.cycles + 1])}


class Batch:
    """Independent problems (mesh, finest level) solved together."""

    def __init__(self, meshes, levels):
        lib = load()
        n = len(meshes)
        arr = (C.c_void_p * n)(*[m._h.value for m in meshes])
        lv = (C.c_int * n)(*[int(x) for x in levels])
        h = C.c_void_p()
        check(lib.ht_batch_create(arr, lv, n, C.byref(h)))
        self._h = h
        self.levels = list(levels)
        self.n = n

    def close(self):
        if getattr(self, "_h", None):
            load().ht_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        n, d, c = C.c_int(), C.c_int64(), C.c_int64()
        check(load().ht_batch_query(self._h, C.byref(n), C.byref(d),
                                    C.byref(c)))
        return {"problems": n.value, "dofs": d.value, "cells": c.value}

    def autotune(self, cache_path=None):
        """Tune the tile shapes of every level of the union mesh (FP64 and
        FP32) on the problems present there."""
        check(load().ht_batch_autotune(
            self._h, cache_path.encode() if cache_path else None, _stream()))

    def shapes(self, levels) -> dict:
        """Tile shapes of the union mesh per level: apply rows (0 = band
        kernel), sweep rows, sweep waves side by side in i, sweep march
        segment, for FP64 and FP32."""
        lib = load()
        m = C.c_void_p()
        check(lib.ht_batch_mesh(self._h, C.byref(m)))
        out = {}
        for lv in levels:
            for name, code in (("f64", HT_F64), ("f32", HT_F32)):
                a, r, w, g = C.c_int(), C.c_int(), C.c_int(), C.c_int()
                check(lib.ht_get_tile_rows(m, lv, code, C.byref(a)))
                check(lib.ht_get_sweep_shape(m, lv, code, C.byref(r), C.byref(w)))
                check(lib.ht_get_march_segment(m, lv, code, C.byref(g)))
                out.setdefault(str(lv), {})[name] = {
                    "apply_rows": a.value, "sweep_rows": r.value,
                    "waves_in_i": bool(w.value), "segment": g.value}
        return out

    def solve(self, us, bs, rel_tol=1e-10, max_cycles=100, nu1=2, nu2=2,
              omega=2.0 / 3.0, coarse_level=2, use_graph=True,
              raise_on_fail=True, precision=HT_PREC_F64):
        """Solve every problem; us[p], bs[p] are float64 device vectors of
        problem p's mesh at its finest level.  precision: HT_PREC_F64 or
        HT_PREC_MIXED (FP32-in-FP64 refinement).  Returns per-problem
        stats."""
        if len(us) != self.n or len(bs) != self.n:
            raise ValueError("need one u and one b per problem")
        up = (C.c_void_p * self.n)(*[_ptr(u).value for u in us])
        bp = (C.c_void_p * self.n)(*[_ptr(b).value for b in bs])
        o = _lib.SolveOpts(Mesh.cycle_opts(nu1, nu2, omega, coarse_level),
                           precision, rel_tol, max_cycles, int(use_graph))
        st = (_lib.SolveStats * self.n)()
        code = load().ht_batch_solve(self._h, C.byref(o), up, bp, st,
                                     _stream())
        if code != _lib.HT_ERR_NOT_CONVERGED or raise_on_fail:
            check(code)
        return [_stats_dict(x) for x in st]
