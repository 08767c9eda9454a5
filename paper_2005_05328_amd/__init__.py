"""MI355X (gfx950) DZS gravity step: Python binding over libdzs.so.

The five calls of the C ABI — ``dzs_coarsen``, ``pm_force``, ``tree_force``,
``lightcone_emit`` and ``kdk_step`` — are exposed under the same names on :class:`Context`.
This module only marshals arguments (torch tensors -> device pointers, the current torch
stream -> hipStream_t); every step of the path runs in the library's HIP kernels, and
importing it fails if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _abi
from ._abi import (DZS_CRIT_DYNAMICAL, DZS_CRIT_GEOMETRIC, DZS_PM_CHUNK_DEFAULT,
                   DZS_PM_CHUNK_MAX, DZS_PM_CHUNK_MIN, DZS_FP32, DZS_FP64,
                   DZS_OPEN_GEOMETRIC, DZS_OPEN_RELATIVE, Box,
                   CoarsenParams, CoarsenReport, LCParams, LCRecord, PMParams, StepParams,
                   TreeParams)

_lib = _abi.load()

__all__ = ["Context", "State", "Box", "CoarsenParams", "PMParams", "TreeParams", "LCParams",
           "StepParams", "LCRing", "DZSError", "step_factors", "DZS_FP64", "DZS_FP32",
           "DZS_CRIT_GEOMETRIC", "DZS_CRIT_DYNAMICAL", "DZS_OPEN_GEOMETRIC",
           "DZS_OPEN_RELATIVE", "DZS_PM_CHUNK_MIN", "DZS_PM_CHUNK_MAX",
           "DZS_PM_CHUNK_DEFAULT", "halt_check", "forecast_speedup",
           "pm_force_noalloc", "lib"]


def lib():
    return _lib


class DZSError(RuntimeError):
    def __init__(self, call, code, text):
        super().__init__(f"{call} returned {code}: {text}")
        self.code = code


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class State:
    """Particle state in device memory: structure of arrays, fixed capacity, current count n."""

    F64 = ("x", "y", "z", "px", "py", "pz", "gx", "gy", "gz")

    def __init__(self, capacity: int, device="cuda:0"):
        torch = _torch()
        self.capacity = int(capacity)
        self.device = device
        for k in self.F64:
            setattr(self, k, torch.zeros(self.capacity, dtype=torch.float64, device=device))
        self.mult = torch.zeros(self.capacity, dtype=torch.int32, device=device)
        self.id = torch.zeros(self.capacity, dtype=torch.int32, device=device)
        self.type = torch.zeros(self.capacity, dtype=torch.uint8, device=device)
        self.n = 0

    @classmethod
    def from_host(cls, ps, capacity=None, device="cuda:0", g=None):
        """Upload a host particle set (attributes x..pz, mult, id, type as numpy arrays)."""
        torch = _torch()
        n = int(ps.x.shape[0])
        st = cls(capacity or max(n, 1), device)
        for k in ("x", "y", "z", "px", "py", "pz"):
            getattr(st, k)[:n] = torch.from_numpy(np.ascontiguousarray(getattr(ps, k), np.float64))
        if g is not None:
            for a, k in enumerate(("gx", "gy", "gz")):
                getattr(st, k)[:n] = torch.from_numpy(np.ascontiguousarray(g[a], np.float64))
        st.mult[:n] = torch.from_numpy(np.ascontiguousarray(ps.mult, np.uint32).view(np.int32))
        st.id[:n] = torch.from_numpy(np.ascontiguousarray(ps.id, np.uint32).view(np.int32))
        st.type[:n] = torch.from_numpy(np.ascontiguousarray(ps.type, np.uint8))
        st.n = n
        return st

    def to_host(self) -> dict:
        n = self.n
        out = {k: getattr(self, k)[:n].cpu().numpy().copy() for k in self.F64}
        out["mult"] = self.mult[:n].cpu().numpy().view(np.uint32).copy()
        out["id"] = self.id[:n].cpu().numpy().view(np.uint32).copy()
        out["type"] = self.type[:n].cpu().numpy().copy()
        return out

    def view(self) -> _abi.Particles:
        p = _abi.Particles()
        for k in self.F64 + ("mult", "id", "type"):
            setattr(p, k, getattr(self, k).data_ptr())
        p.n = self.n
        p.capacity = self.capacity
        return p


class LCRing:
    """Device ring of lightcone records (64 bytes each) with a device counter and flag."""

    def __init__(self, capacity: int, device="cuda:0"):
        torch = _torch()
        self.capacity = int(capacity)
        self.buf = torch.zeros(self.capacity * 8, dtype=torch.float64, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=device)

    def reset(self):
        self.count.zero_()
        self.overflow.zero_()

    def view(self) -> _abi.LCRing:
        r = _abi.LCRing()
        r.records = self.buf.data_ptr()
        r.capacity = self.capacity
        r.count = self.count.data_ptr()
        r.overflow = self.overflow.data_ptr()
        return r

    def records(self) -> dict:
        n = min(int(self.count.item()), self.capacity)
        raw = self.buf[: 8 * n].cpu().numpy().view(np.uint8).reshape(n, 64)
        rec = np.frombuffer(raw.tobytes(), dtype=np.dtype([("id", "<u4"), ("mult", "<u4"),
                                                           ("a_cross", "<f8"), ("d", "<f8", 3),
                                                           ("p", "<f8", 3)]))
        return {"id": rec["id"].copy(), "mult": rec["mult"].copy(),
                "a_cross": rec["a_cross"].copy(), "d": rec["d"].copy(), "p": rec["p"].copy(),
                "overflow": int(self.overflow.item()), "count": int(self.count.item())}


def make_box(L, m0, eps0, G=43.0091) -> Box:
    return Box(float(L), float(m0), float(eps0), float(G))


def halt_check(balance, ratio, ratio_prev, t, t_prev, max_balance=0.0, min_ratio=0.0,
               runtime_limit_s=0.0, restart_window_s=0.0) -> int:
    """The DZS_HALT_* reasons to stop a run (0: carry on); see dzs_halt_check."""
    prm = _abi.HaltParams(max_balance, min_ratio, runtime_limit_s, restart_window_s)
    st = _abi.HaltState(balance, ratio, ratio_prev, t, t_prev)
    return int(_lib.dzs_halt_check(C.byref(prm), C.byref(st)))


def forecast_speedup(L: float, n_part: float, omega_m: float = 0.3) -> _abi.Forecast:
    """a_DZS, r and the forecast speed-up T_STD / T_DZS; see dzs_forecast_speedup."""
    out = _abi.Forecast()
    rc = _lib.dzs_forecast_speedup(float(L), float(n_part), float(omega_m), C.byref(out))
    if rc != 0:
        raise DZSError("dzs_forecast_speedup", rc, "no a_DZS in [1e-4, 1] or bad argument")
    return out


def pm_force_noalloc(box: Box, st: "State", prm: PMParams, stream=None):
    """pm_force without a context or any device allocation: the meshes live in the library's
    static per-device array (mesh sides up to DZS_PM_NOALLOC_MAX_SIDE)."""
    v = st.view()
    rc = _lib.pm_force_noalloc(C.byref(box), C.byref(v), C.byref(prm), _stream_handle(stream))
    if rc != 0:
        raise DZSError("pm_force_noalloc", rc, "see include/dzs.h (no context, no error text)")


def step_factors(a0: float, a1: float, omega_m: float = 0.3) -> StepParams:
    sp = StepParams()
    rc = _lib.dzs_step_factors(float(a0), float(a1), float(omega_m), C.byref(sp))
    if rc != 0:
        raise DZSError("dzs_step_factors", rc, "invalid scale factors")
    return sp


class Context:
    """A libdzs context: scratch for up to `max_particles` particles and a `max_mesh_side`
    mesh on one device."""

    def __init__(self, max_particles: int, max_mesh_side: int, device: int = 0,
                 fp32_meshes: bool = False, no_copies: bool = False, max_boxes: int = 0,
                 hier_split: bool = False):
        flags = (_abi.DZS_CAP_FP32_MESHES if fp32_meshes else 0) | \
            (_abi.DZS_CAP_NO_COPIES if no_copies else 0) | \
            (_abi.DZS_CAP_HIER_SPLIT if hier_split else 0)
        cap = _abi.Capacity(int(max_particles), int(max_mesh_side), flags, int(max_boxes), 0)
        h = C.c_void_p()
        rc = _lib.dzs_ctx_create(C.byref(h), int(device), C.byref(cap))
        if rc != 0:
            raise DZSError("dzs_ctx_create", rc, "context creation failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.dzs_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, name, rc):
        if rc != 0:
            raise DZSError(name, rc, _lib.dzs_last_error(self._h).decode())

    # ---- the five calls
    def dzs_coarsen(self, box: Box, st: State, prm: CoarsenParams, group_of=None, stream=None):
        v = st.view()
        rep = CoarsenReport()
        self._check("dzs_coarsen", _lib.dzs_coarsen(self._h, C.byref(box), C.byref(v), C.byref(prm),
                                                    _ptr(group_of), C.byref(rep),
                                                    _stream_handle(stream)))
        st.n = int(v.n)
        return rep

    def pm_force(self, box: Box, st: State, prm: PMParams, stream=None):
        v = st.view()
        self._check("pm_force", _lib.pm_force(self._h, C.byref(box), C.byref(v), C.byref(prm),
                                              _stream_handle(stream)))

    def tree_force(self, box: Box, st: State, prm: TreeParams, targets=None, stream=None):
        """Short-range force of `targets` (an int32/uint32 device tensor of indices; every
        particle when None).  Capacity and order errors surface at the next check()."""
        v = st.view()
        nt = 0 if targets is None else int(targets.numel())
        if targets is not None and nt == 0:
            return   # an empty subset (a null pointer would mean every particle)
        self._check("tree_force", _lib.tree_force(self._h, C.byref(box), C.byref(v), C.byref(prm),
                                                  _ptr(targets), nt, _stream_handle(stream)))

    def lightcone_emit(self, box: Box, st: State, prm: LCParams, ring: LCRing, stream=None):
        v = st.view()
        r = ring.view()
        self._check("lightcone_emit", _lib.lightcone_emit(self._h, C.byref(box), C.byref(v),
                                                          C.byref(prm), C.byref(r),
                                                          _stream_handle(stream)))

    def kdk_step(self, box: Box, st: State, prm: StepParams, ring: LCRing | None = None,
                 stream=None):
        v = st.view()
        rep = CoarsenReport()
        rv = C.byref(ring.view()) if ring is not None else None
        self._check("kdk_step", _lib.kdk_step(self._h, C.byref(box), C.byref(v), C.byref(prm), rv,
                                              C.byref(rep), _stream_handle(stream)))
        st.n = int(v.n)
        return rep

    def kdk_step_hier(self, box: Box, st: State, prm: StepParams, max_bin: int, eta: float,
                      a0: float, a1: float, omega_m: float = 0.3, limiter: bool = False,
                      R_lim: float = 0.0, ring: LCRing | None = None, bins_out=None,
                      pm_global: bool = False, stream=None):
        """One global step a0 -> a1 with individual power-of-two time steps (bins 0..max_bin);
        bins_out (optional uint8 tensor) receives the bins in the entry order.  pm_global: the
        long-range force on the global step only (a context made with hier_split=True)."""
        v = st.view()
        rep = CoarsenReport()
        hp = _abi.HierParams(int(max_bin), int(bool(limiter)), float(eta), float(R_lim),
                             float(a0), float(a1), float(omega_m), int(bool(pm_global)), 0)
        rv = C.byref(ring.view()) if ring is not None else None
        self._check("kdk_step_hier", _lib.kdk_step_hier(self._h, C.byref(box), C.byref(v),
                                                        C.byref(prm), C.byref(hp), rv,
                                                        C.byref(rep), _ptr(bins_out),
                                                        _stream_handle(stream)))
        st.n = int(v.n)
        return rep

    def kdk_step_batch(self, boxes, first, ng, r_s, r_cut, st: State, prm: StepParams,
                       ring: LCRing | None = None, stream=None):
        """One step of every box of a batch; box b owns st's particles first[b]:first[b+1]."""
        nb = len(boxes)
        arr_box = (Box * nb)(*boxes)
        arr_first = (C.c_uint64 * (nb + 1))(*[int(v) for v in first])
        arr_ng = (C.c_int32 * nb)(*[int(v) for v in ng])
        arr_rs = (C.c_double * nb)(*[float(v) for v in r_s])
        arr_rc = (C.c_double * nb)(*[float(v) for v in r_cut])
        b = _abi.Batch(nb, 0, arr_box, arr_first, arr_ng, arr_rs, arr_rc)
        v = st.view()
        rv = C.byref(ring.view()) if ring is not None else None
        self._check("kdk_step_batch", _lib.kdk_step_batch(self._h, C.byref(b), C.byref(v),
                                                          C.byref(prm), rv,
                                                          _stream_handle(stream)))

    def kdk_step_batch_stage(self, prm: StepParams):
        """Stage the factors of the next replay of a captured kdk_step_batch."""
        self._check("kdk_step_batch_stage", _lib.kdk_step_batch_stage(self._h, C.byref(prm)))

    def check(self, stream=None):
        """Report what the device recorded since the last check: a tree-capacity or
        walk-stack overflow, or a rejected tree_force input (synchronises)."""
        self._check("dzs_check", _lib.dzs_check(self._h, _stream_handle(stream)))

    # ---- parts of the path
    def morton_keys(self, box: Box, st: State, keys, stream=None):
        v = st.view()
        self._check("dzs_morton_keys", _lib.dzs_morton_keys(self._h, C.byref(box), C.byref(v),
                                                            _ptr(keys), _stream_handle(stream)))

    def sort_state(self, box: Box, st: State, ties_by_id=False, perm=None, stream=None):
        v = st.view()
        self._check("dzs_sort_state", _lib.dzs_sort_state(self._h, C.byref(box), C.byref(v),
                                                          int(bool(ties_by_id)), _ptr(perm),
                                                          _stream_handle(stream)))

    def pair_interactions(self, reset=False) -> int:
        v = C.c_uint64()
        self._check("dzs_counters", _lib.dzs_counters(self._h, int(bool(reset)), C.byref(v)))
        return int(v.value)

    def timing(self, enable=True, reset=False, classes=None) -> dict:
        """Per-class average kernel times since the last reset; `classes` (names) restricts
        the HIP events of the next calls to those classes (all when None)."""
        cap = 32
        names = (C.c_char_p * cap)()
        ms = (C.c_double * cap)()
        calls = (C.c_uint64 * cap)()
        code = int(bool(enable))
        if enable and classes:
            order = [n.decode() for n in names[:_lib.dzs_timing(self._h, -1, 0, names, None,
                                                                None, cap)]]
            code = 0
            for c in classes:
                code |= 1 << (order.index(c) + 1)
        w = _lib.dzs_timing(self._h, code, int(reset), names, ms, calls, cap)
        return {names[i].decode(): (ms[i], int(calls[i])) for i in range(w)}
