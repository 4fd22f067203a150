"""CPU FP64 DSMC oracle: ctypes wrapper around ``dsmc_oracle.c``.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg use this package to check and to time the GPU path; the
product package never imports it.  The C source is compiled with
``-O2 -ffp-contract=off`` (no fast-math) so that every floating-point
expression is evaluated exactly as written.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "dsmc_oracle.c")
LIB = os.path.join(_HERE, "libdsmc_oracle.so")

PHASE_MOVE, PHASE_SORT, PHASE_COLLIDE, PHASE_SAMPLE = 1, 2, 4, 8
PHASE_ALL = 15
TAG_INIT, TAG_WALL, TAG_COLL = 1, 2, 3
NMOM = 13

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle into ``libdsmc_oracle.so`` next to its source."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _Params(ct.Structure):
    _fields_ = [("kn", ct.c_double), ("body_force", ct.c_double),
                ("wall_temperature", ct.c_double), ("dt", ct.c_double),
                ("n_cells", ct.c_int32), ("particles_per_cell", ct.c_int32),
                ("n_sub", ct.c_int32), ("pad_", ct.c_int32),
                ("n_transient", ct.c_int64), ("seed", ct.c_uint64),
                ("domain_length", ct.c_double)]


def _dp():
    return np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    """The oracle library: ``libdsmc_oracle.so`` (built if missing or stale),
    or the build named by DSMC_ORACLE_LIB, which the mutation tests use to run
    the pins against deliberately broken copies of the oracle."""
    global _lib
    with _lock:
        if _lib is None:
            path = os.environ.get("DSMC_ORACLE_LIB")
            if not path:
                build(force=False)
                path = LIB
            L = ct.CDLL(path)
            vp = ct.c_void_p
            L.or_create.restype = vp
            L.or_create.argtypes = [ct.POINTER(_Params)]
            L.or_destroy.argtypes = [vp]
            L.or_step.argtypes = [vp, ct.c_int64, ct.c_uint32]
            L.or_reset_window.argtypes = [vp]
            L.or_estimators.argtypes = [vp] + [vp] * 10
            L.or_n_particles.restype = ct.c_int32
            L.or_n_particles.argtypes = [vp]
            L.or_capacity.restype = ct.c_int32
            L.or_capacity.argtypes = [vp]
            L.or_set_inflow.argtypes = [vp, ct.c_double, ct.c_double, ct.c_double, ct.c_double]
            L.or_open_diagnostics.argtypes = [vp, vp]
            L.or_inject_one.argtypes = [vp, ct.c_int64, ct.c_int64, vp]
            L.or_n_coll_cells.restype = ct.c_int32
            L.or_n_coll_cells.argtypes = [vp]
            L.or_step_index.restype = ct.c_int64
            L.or_step_index.argtypes = [vp]
            L.or_n_sampled.restype = ct.c_int64
            L.or_n_sampled.argtypes = [vp]
            L.or_get_particles.argtypes = [vp] * 6
            L.or_set_particles.argtypes = [vp] * 6
            L.or_get_cells.argtypes = [vp] * 5
            L.or_get_acc.argtypes = [vp, vp]
            L.or_constants.argtypes = [vp, vp]
            L.or_diagnostics.argtypes = [vp, vp]
            L.or_move_one.argtypes = [vp, ct.c_int64, ct.c_int64, vp]
            L.or_philox.argtypes = [vp, vp, vp]
            L.or_log.restype = ct.c_double
            L.or_log.argtypes = [ct.c_double]
            L.or_uniform2.argtypes = [vp, ct.c_int64, ct.c_int64, ct.c_int64, ct.c_uint32,
                                      ct.c_uint32, vp]
            L.or_normal2.argtypes = [vp, ct.c_int64, ct.c_int64, ct.c_int64, ct.c_uint32,
                                     ct.c_uint32, ct.c_double, vp]
            L.or_sphere.argtypes = [vp, ct.c_int64, ct.c_int64, ct.c_int64, ct.c_uint32,
                                    ct.c_uint32, vp]
            L.or_stable_sort_perm.argtypes = [ct.c_int32, vp, ct.c_int32, vp, vp, vp]
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


# ------------------------------------------------------------ primitives
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def series_log(u: float) -> float:
    return lib().or_log(float(u))


def key_of(seed: int) -> np.ndarray:
    return np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)


def uniform2(seed, step, entity, sub, tag, call=0) -> np.ndarray:
    out = np.zeros(2)
    k = key_of(seed)
    lib().or_uniform2(_ptr(k), step, entity, sub, tag, call, _ptr(out))
    return out


def normal2(seed, step, entity, sub, tag, call=0, sqrt_var=1.0) -> np.ndarray:
    out = np.zeros(2)
    k = key_of(seed)
    lib().or_normal2(_ptr(k), step, entity, sub, tag, call, float(sqrt_var), _ptr(out))
    return out


def sphere(seed, step, entity, sub, tag, call=0) -> np.ndarray:
    out = np.zeros(3)
    k = key_of(seed)
    lib().or_sphere(_ptr(k), step, entity, sub, tag, call, _ptr(out))
    return out


def stable_sort_perm(keys, nkeys):
    k = np.ascontiguousarray(keys, dtype=np.int32)
    n = len(k)
    count = np.zeros(max(nkeys, 1), dtype=np.int32)
    offset = np.zeros(max(nkeys, 1), dtype=np.int32)
    perm = np.zeros(max(n, 1), dtype=np.int32)
    lib().or_stable_sort_perm(n, _ptr(k), nkeys, _ptr(count), _ptr(offset), _ptr(perm))
    return perm[:n], count[:nkeys], offset[:nkeys]


# ---------------------------------------------------------------- solver
class Oracle:
    """One oracle instance.  ``params`` is a ``synth.Params`` (or any object
    with the same fields); precision is ignored: the oracle is always FP64."""

    def __init__(self, params):
        p = _Params(kn=params.kn, body_force=params.body_force,
                    wall_temperature=params.wall_temperature, dt=params.dt,
                    n_cells=params.n_cells, particles_per_cell=params.particles_per_cell,
                    n_sub=params.n_sub, pad_=0, n_transient=params.n_transient,
                    seed=params.seed, domain_length=getattr(params, "domain_length", 0.0))
        self._L = lib()
        h = self._L.or_create(ct.byref(p))
        if not h:
            raise ValueError("invalid oracle parameters")
        self._h = ct.c_void_p(h)
        self.params = params
        self.Cc = self._L.or_n_coll_cells(self._h)
        self.capacity = self._L.or_capacity(self._h)
        self.C = params.n_cells

    def close(self):
        if getattr(self, "_h", None):
            self._L.or_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1, phases: int = PHASE_ALL):
        self._L.or_step(self._h, int(n), int(phases))

    @property
    def step_index(self) -> int:
        return self._L.or_step_index(self._h)

    @property
    def n_sampled(self) -> int:
        return self._L.or_n_sampled(self._h)

    def reset_window(self):
        self._L.or_reset_window(self._h)

    @property
    def N(self) -> int:
        """Particles in the domain (changes with each step of an open domain)."""
        return self._L.or_n_particles(self._h)

    def set_inflow(self, u=0.0, dudy=0.0, T=1.0, n=1.0):
        """Chapman-Enskog inflow state at the open boundary (u, du/dy in the
        units of Eq. 6; T and n relative to the reference state)."""
        self._L.or_set_inflow(self._h, float(u), float(dudy), float(T), float(n))

    def inject_one(self, step: int, k: int) -> np.ndarray:
        """Particle k injected at the start of step ``step``: (y, vx, vy, vz)
        before that step's move, in code units."""
        st = np.zeros(4)
        self._L.or_inject_one(self._h, int(step), int(k), _ptr(st))
        return st

    def open_diagnostics(self) -> dict:
        o = np.zeros(5)
        self._L.or_open_diagnostics(self._h, _ptr(o))
        return dict(n_live=int(o[0]), n_injected=int(o[1]), n_deleted=int(o[2]),
                    status=int(o[3]), inj_rem=float(o[4]))

    def particles(self):
        n = self.N
        y, vx, vy, vz = (np.zeros(n) for _ in range(4))
        cell = np.zeros(n, dtype=np.int32)
        self._L.or_get_particles(self._h, _ptr(y), _ptr(vx), _ptr(vy), _ptr(vz), _ptr(cell))
        return y, vx, vy, vz, cell

    def set_particles(self, y=None, vx=None, vy=None, vz=None, cell=None):
        args = []
        keep = []
        for a, dt in ((y, np.float64), (vx, np.float64), (vy, np.float64), (vz, np.float64),
                      (cell, np.int32)):
            if a is None:
                args.append(None)
            else:
                a = np.ascontiguousarray(a, dtype=dt)
                assert a.shape == (self.N,)
                keep.append(a)
                args.append(_ptr(a))
        self._L.or_set_particles(self._h, *args)

    def cells(self):
        c = self.Cc
        crmax, rem = np.zeros(c), np.zeros(c)
        count, offset = np.zeros(c, dtype=np.int32), np.zeros(c, dtype=np.int32)
        self._L.or_get_cells(self._h, _ptr(crmax), _ptr(rem), _ptr(count), _ptr(offset))
        return crmax, rem, count, offset

    def acc(self) -> np.ndarray:
        a = np.zeros((self.Cc, NMOM))
        self._L.or_get_acc(self._h, _ptr(a))
        return a

    def constants(self) -> dict:
        o = np.zeros(6)
        self._L.or_constants(self._h, _ptr(o))
        return dict(dt=o[0], g=o[1], kntc=o[2], crmax0=o[3], inv_dy=o[4], lam=o[5])

    def diagnostics(self) -> dict:
        o = np.zeros(4)
        self._L.or_diagnostics(self._h, _ptr(o))
        return dict(n_coll=int(o[0]), n_hits=int(o[1]), wall_dpx=o[2], wall_de=o[3])

    def estimators(self) -> dict:
        C = self.C
        arrs = {k: np.zeros(C) for k in ("n", "ux", "uy", "uz", "T", "pxy", "qx", "qy", "pxy_mid")}
        Q = np.zeros(1)
        self._L.or_estimators(self._h, *[_ptr(arrs[k]) for k in
                                         ("n", "ux", "uy", "uz", "T", "pxy", "qx", "qy")],
                              _ptr(Q), _ptr(arrs["pxy_mid"]))
        arrs["mass_flow"] = float(Q[0])
        arrs["n_sampled_steps"] = self.n_sampled
        return arrs

    def move_one(self, step, slot, state):
        st = np.ascontiguousarray(state, dtype=np.float64).copy()
        self._L.or_move_one(self._h, int(step), int(slot), _ptr(st))
        return st
