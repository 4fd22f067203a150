"""ctypes binding of ``libdsmc.so`` (the C ABI declared in include/dsmc.h).

Argument marshalling only: every phase of a DSMC step runs in the library's
HIP kernels.  PyTorch, when used, only supplies device memory (an arena
tensor) and the HIP stream.  If the library has not been built the import of
this module fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdsmc.so")

DSMC_OK = 0
DSMC_ERR_INVALID_ARG = -1
DSMC_ERR_OUT_OF_MEMORY = -2
DSMC_ERR_DEVICE = -3
DSMC_ERR_STATE = -4
DSMC_ERR_NUMERIC = -5

DSMC_FP64_DETERMINISTIC = 0
DSMC_FP32_FAST = 1
DSMC_FP64_FAST = 2

DSMC_PHASE_MOVE, DSMC_PHASE_SORT, DSMC_PHASE_COLLIDE, DSMC_PHASE_SAMPLE = 1, 2, 4, 8
DSMC_PHASE_ALL = 15
N_MOMENTS = 13

EXPORTS = (
    "dsmc_params_init", "dsmc_footprint_bytes", "dsmc_create", "dsmc_step", "dsmc_sample",
    "dsmc_sync", "dsmc_destroy", "dsmc_get_state", "dsmc_set_state", "dsmc_get_cells",
    "dsmc_set_cells", "dsmc_info", "dsmc_status_string", "dsmc_last_error",
    "dsmc_group_create", "dsmc_group_add", "dsmc_group_remove", "dsmc_group_step",
    "dsmc_group_sync", "dsmc_group_size", "dsmc_group_lanes", "dsmc_group_destroy", "dsmc_group_set_tuning",
    "dsmc_group_set_resident",
    "dsmc_group_autotune", "dsmc_profile_step", "dsmc_group_sample", "dsmc_set_inflow",
    "dsmc_open_state", "dsmc_set_open_state", "dsmc_group_sample_noalloc",
    "dsmc_group_lane_info",
)


class DsmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class dsmc_params(ct.Structure):
    _fields_ = [("struct_size", ct.c_uint32), ("precision", ct.c_int32), ("kn", ct.c_double),
                ("body_force", ct.c_double), ("wall_temperature", ct.c_double),
                ("dt", ct.c_double), ("n_cells", ct.c_int32),
                ("particles_per_cell", ct.c_int32), ("n_sub", ct.c_int32),
                ("debug_phase_mask", ct.c_uint32), ("n_transient", ct.c_int64),
                ("seed", ct.c_uint64), ("domain_length", ct.c_double)]


_dp = ct.POINTER(ct.c_double)


class dsmc_moments(ct.Structure):
    _fields_ = [("n_cells", ct.c_int32), ("pad_", ct.c_int32), ("n_sampled_steps", ct.c_int64),
                ("n", _dp), ("ux", _dp), ("uy", _dp), ("uz", _dp), ("T", _dp), ("pxy", _dp),
                ("qx", _dp), ("qy", _dp), ("raw_sums", _dp), ("mass_flow", ct.c_double),
                ("n_collisions", ct.c_int64), ("pxy_mid", _dp)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2311_14140_amd.build` (hipcc, gfx950)")
    L = ct.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_uint64
    P = ct.POINTER(dsmc_params)
    sig = {
        "dsmc_params_init": [P],
        "dsmc_footprint_bytes": [P, ct.POINTER(u64)],
        "dsmc_create": [P, vp, vp, u64, ct.POINTER(vp)],
        "dsmc_step": [vp, i64],
        "dsmc_sample": [vp, ct.POINTER(dsmc_moments), ct.c_int],
        "dsmc_sync": [vp],
        "dsmc_destroy": [vp],
        "dsmc_get_state": [vp, vp, vp, vp, vp, vp, ct.POINTER(u64)],
        "dsmc_set_state": [vp, vp, vp, vp, vp, vp, u64],
        "dsmc_get_cells": [vp, vp, vp, vp, vp],
        "dsmc_set_cells": [vp, vp, vp, vp, vp],
        "dsmc_info": [vp, ct.POINTER(i32), ct.POINTER(i32), vp],
        "dsmc_group_create": [vp, ct.POINTER(vp)],
        "dsmc_group_add": [vp, vp],
        "dsmc_group_remove": [vp, vp],
        "dsmc_group_step": [vp, i64],
        "dsmc_group_sync": [vp],
        "dsmc_group_size": [vp, ct.POINTER(i32)],
        "dsmc_group_lanes": [vp, ct.POINTER(i32)],
        "dsmc_group_lane_info": [vp, ct.POINTER(i32), ct.POINTER(i32), ct.POINTER(i64),
                                 ct.POINTER(i64)],
        "dsmc_group_sample": [vp, vp, i32, ct.c_int],
        "dsmc_group_sample_noalloc": [vp, vp, i32, ct.c_int],
        "dsmc_set_inflow": [vp, ct.c_double, ct.c_double, ct.c_double, ct.c_double],
        "dsmc_open_state": [vp, ct.POINTER(i32), ct.POINTER(i64), ct.POINTER(i64),
                            ct.POINTER(ct.c_double)],
        "dsmc_set_open_state": [vp, i32, i64, i64, ct.c_double],
        "dsmc_group_destroy": [vp],
        "dsmc_group_set_tuning": [vp, i32, i32, i32],
        "dsmc_group_set_resident": [vp, i32],
        "dsmc_group_autotune": [vp, ct.POINTER(i32), ct.POINTER(i32), ct.POINTER(i32)],
        "dsmc_profile_step": [vp, i64, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ct.c_int
    L.dsmc_status_string.argtypes = [ct.c_int]
    L.dsmc_status_string.restype = ct.c_char_p
    L.dsmc_last_error.argtypes = [vp]
    L.dsmc_last_error.restype = ct.c_char_p
    return L


lib = _load()


def _check(code: int, handle=None):
    if code != DSMC_OK:
        msg = lib.dsmc_last_error(handle).decode(errors="replace")
        raise DsmcError(code, msg or lib.dsmc_status_string(code).decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def make_params(p) -> dsmc_params:
    """A ``dsmc_params`` from any object with the fields of ``synth.Params``."""
    c = dsmc_params()
    lib.dsmc_params_init(ct.byref(c))
    c.precision = int(p.precision)
    c.kn = float(p.kn)
    c.body_force = float(p.body_force)
    c.wall_temperature = float(p.wall_temperature)
    c.dt = float(p.dt)
    c.n_cells = int(p.n_cells)
    c.particles_per_cell = int(p.particles_per_cell)
    c.n_sub = int(getattr(p, "n_sub", 1))
    c.debug_phase_mask = int(getattr(p, "debug_phase_mask", 0))
    c.n_transient = int(p.n_transient)
    c.seed = int(p.seed)
    c.domain_length = float(getattr(p, "domain_length", 0.0))
    return c


def footprint_bytes(p) -> int:
    c = make_params(p)
    out = ct.c_uint64()
    _check(lib.dsmc_footprint_bytes(ct.byref(c), ct.byref(out)))
    return int(out.value)


def _torch_stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Solver:
    """One DSMC instance on the current GPU.

    ``arena="torch"`` takes the device memory from a ``torch.uint8`` tensor;
    ``arena=None`` lets the library allocate.  ``stream`` is a
    ``torch.cuda.Stream`` (or raw HIP stream handle) or None.
    """

    def __init__(self, params, stream=None, arena=None, debug_phase_mask: int = 0):
        c = make_params(params)
        if debug_phase_mask:
            c.debug_phase_mask = debug_phase_mask
        self.params = params
        self.precision = c.precision
        self._arena = None
        ptr, nbytes = None, 0
        if arena == "torch":
            import torch
            nbytes = footprint_bytes(params)
            self._arena = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            ptr = self._arena.data_ptr()
        self._stream_obj = stream
        h = ct.c_void_p()
        _check(lib.dsmc_create(ct.byref(c), _torch_stream(stream), ptr, nbytes, ct.byref(h)))
        self._h = h
        n, cc = ct.c_int32(), ct.c_int32()
        consts = np.zeros(6)
        _check(lib.dsmc_info(h, ct.byref(n), ct.byref(cc), _ptr(consts)), h)
        self.N, self.Cc, self.C = n.value, cc.value, int(params.n_cells)
        self.open = float(getattr(params, "domain_length", 0.0)) > 0.0
        self.constants = dict(dt=consts[0], g=consts[1], kntc=consts[2], crmax0=consts[3],
                              inv_dy=consts[4], lam=consts[5])
        self.real = np.float32 if self.precision == DSMC_FP32_FAST else np.float64

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.dsmc_destroy(self._h)
            self._h = None
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, n: int = 1):
        _check(lib.dsmc_step(self._h, int(n)), self._h)

    def sync(self):
        _check(lib.dsmc_sync(self._h), self._h)

    def sample(self, reset: bool = False, raw: bool = False) -> dict:
        C = self.C
        arrs = {k: np.zeros(C) for k in ("n", "ux", "uy", "uz", "T", "pxy", "qx", "qy", "pxy_mid")}
        m = dsmc_moments()
        m.n_cells = C
        for k, a in arrs.items():
            setattr(m, k, a.ctypes.data_as(_dp))
        rawa = None
        if raw:
            rawa = np.zeros((self.Cc, N_MOMENTS))
            m.raw_sums = rawa.ctypes.data_as(_dp)
        _check(lib.dsmc_sample(self._h, ct.byref(m), 1 if reset else 0), self._h)
        arrs["mass_flow"] = m.mass_flow
        arrs["n_sampled_steps"] = m.n_sampled_steps
        arrs["n_collisions"] = m.n_collisions
        if raw:
            arrs["raw"] = rawa
        return arrs

    # kernel slots of a step: the key histogram (position-only flight), the
    # three column-scan kernels, the move with the stable scatter, and the
    # collide with fused sampling (under a debug phase mask the first and
    # fifth slots are the in-place move and the plain scatter)
    PHASES = ("count", "colsum", "scan", "colprefix", "move_scatter", "collide")

    def profile(self, n_steps: int) -> dict:
        """Device milliseconds per kernel over n_steps eagerly launched steps."""
        out = np.zeros(9)
        _check(lib.dsmc_profile_step(self._h, int(n_steps), _ptr(out)), self._h)
        d = {k: float(v) for k, v in zip(self.PHASES, out[:6])}
        d["kernels_total"] = float(out[6])
        d["wall"] = float(out[7])
        d["resident"] = float(out[8])
        return d

    def set_inflow(self, u: float = 0.0, dudy: float = 0.0, T: float = 1.0, n: float = 1.0):
        """Chapman-Enskog inflow at the open boundary of an open instance."""
        _check(lib.dsmc_set_inflow(self._h, float(u), float(dudy), float(T), float(n)), self._h)

    def open_state(self) -> dict:
        """Live particles, injected and removed totals and the carried
        injection remainder of an open instance."""
        n, a, b, r = ct.c_int32(), ct.c_int64(), ct.c_int64(), ct.c_double()
        _check(lib.dsmc_open_state(self._h, ct.byref(n), ct.byref(a), ct.byref(b), ct.byref(r)),
               self._h)
        return dict(n_live=n.value, n_injected=a.value, n_deleted=b.value, inj_rem=r.value)

    def set_open_state(self, n_live: int, n_injected: int, n_deleted: int, inj_rem: float):
        """Restore an open instance's boundary state (before set_state)."""
        _check(lib.dsmc_set_open_state(self._h, int(n_live), int(n_injected), int(n_deleted),
                                       float(inj_rem)), self._h)

    def live(self) -> int:
        return self.open_state()["n_live"] if self.open else self.N

    def get_state(self):
        n = self.live()
        y, vx, vy, vz = (np.zeros(n, dtype=self.real) for _ in range(4))
        cell = np.zeros(n, dtype=np.int32)
        step = ct.c_uint64()
        _check(lib.dsmc_get_state(self._h, _ptr(y), _ptr(vx), _ptr(vy), _ptr(vz), _ptr(cell),
                                  ct.byref(step)), self._h)
        return y, vx, vy, vz, cell, int(step.value)

    def set_state(self, y=None, vx=None, vy=None, vz=None, cell=None, step: int = 0):
        keep = []
        n_live = self.live()

        def conv(a, dt):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=dt)
            if a.shape != (n_live,):
                raise ValueError("state arrays must have N elements")
            keep.append(a)
            return _ptr(a)

        _check(lib.dsmc_set_state(self._h, conv(y, self.real), conv(vx, self.real),
                                  conv(vy, self.real), conv(vz, self.real),
                                  conv(cell, np.int32), int(step)), self._h)

    def get_cells(self):
        c = self.Cc
        crmax, rem = np.zeros(c), np.zeros(c)
        count, offset = np.zeros(c, dtype=np.int32), np.zeros(c, dtype=np.int32)
        _check(lib.dsmc_get_cells(self._h, _ptr(crmax), _ptr(rem), _ptr(count), _ptr(offset)),
               self._h)
        return crmax, rem, count, offset

    def set_cells(self, crmax=None, rem=None, count=None, offset=None):
        a = [None if x is None else np.ascontiguousarray(x, dtype=dt)
             for x, dt in ((crmax, np.float64), (rem, np.float64), (count, np.int32),
                           (offset, np.int32))]
        _check(lib.dsmc_set_cells(self._h, *[_ptr(x) for x in a]), self._h)


class Group:
    """Many independent instances of one precision stepped together."""

    def __init__(self, stream=None):
        g = ct.c_void_p()
        _check(lib.dsmc_group_create(_torch_stream(stream), ct.byref(g)))
        self._g = g
        self._stream_obj = stream
        self.members: list[Solver] = []

    def add(self, s: Solver):
        _check(lib.dsmc_group_add(self._g, s.handle))
        self.members.append(s)

    def remove(self, s: Solver):
        _check(lib.dsmc_group_remove(self._g, s.handle))
        self.members.remove(s)

    def step(self, n: int = 1):
        _check(lib.dsmc_group_step(self._g, int(n)))

    def sync(self):
        _check(lib.dsmc_group_sync(self._g))

    def sample(self, reset: bool = False, noalloc: bool = False) -> list:
        """Every member's window estimators (as ``Solver.sample`` without raw
        sums), in member order, with one launch, one copy and one
        synchronisation for the whole group.  ``noalloc`` takes them through
        the library's allocation-free variant (fixed scratch, at most 1024
        members and 32 MiB of estimators)."""
        n = len(self.members)
        ms = (dsmc_moments * max(n, 1))()
        outs = []
        for i, s in enumerate(self.members):
            arrs = {k: np.zeros(s.C) for k in ("n", "ux", "uy", "uz", "T", "pxy", "qx", "qy",
                                                 "pxy_mid")}
            ms[i].n_cells = s.C
            for k, a in arrs.items():
                setattr(ms[i], k, a.ctypes.data_as(_dp))
            outs.append(arrs)
        fn = lib.dsmc_group_sample_noalloc if noalloc else lib.dsmc_group_sample
        _check(fn(self._g, ms, n, 1 if reset else 0))
        for i, arrs in enumerate(outs):
            arrs["mass_flow"] = ms[i].mass_flow
            arrs["n_sampled_steps"] = ms[i].n_sampled_steps
            arrs["n_collisions"] = ms[i].n_collisions
        return outs

    def lanes(self) -> int:
        """Lanes the members ran in at the last step (each kernel of a step is
        launched once per lane)."""
        n = ct.c_int32()
        _check(lib.dsmc_group_lanes(self._g, ct.byref(n)))
        return n.value

    def lane_info(self) -> dict:
        """Lanes of the last step: all, resident, and the particles of the
        members stepped resident."""
        n, r, p, c = ct.c_int32(), ct.c_int32(), ct.c_int64(), ct.c_int64()
        _check(lib.dsmc_group_lane_info(self._g, ct.byref(n), ct.byref(r), ct.byref(p),
                                        ct.byref(c)))
        return {"lanes": n.value, "resident_lanes": r.value, "resident_particles": p.value,
                "resident_cells": c.value}

    def set_tuning(self, tile_mult: int = 0, particles_per_block: int = 0, waves_per_cu: int = 0):
        _check(lib.dsmc_group_set_tuning(self._g, int(tile_mult), int(particles_per_block),
                                         int(waves_per_cu)))

    def set_resident(self, enable: bool = True):
        """Step small members in one workgroup each (the default) or with the
        multi-kernel step; the results are the same."""
        _check(lib.dsmc_group_set_resident(self._g, 1 if enable else 0))

    def autotune(self):
        """Tune the launch shape on the group's own steps; returns
        (tile_mult, particles_per_block, waves_per_cu)."""
        a, b, c = ct.c_int32(), ct.c_int32(), ct.c_int32()
        _check(lib.dsmc_group_autotune(self._g, ct.byref(a), ct.byref(b), ct.byref(c)))
        return a.value, b.value, c.value

    def close(self):
        if getattr(self, "_g", None) is not None and self._g.value:
            lib.dsmc_group_destroy(self._g)
            self._g = None
        self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
