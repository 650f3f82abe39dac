"""Python access to the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product path never imports this package.

All arrays follow the oracle's own layout: positions, velocities,
accelerations and jerks are float64 (N, 3); times and steps are float64 (N,).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.environ.get("NBODY_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")


class Params(ctypes.Structure):
    _fields_ = [
        ("eps2", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("eta_init", ctypes.c_double),
        ("dt_min", ctypes.c_double),
        ("dt_max", ctypes.c_double),
    ]


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile oracle.c into liboracle.so (gcc -O3 -fopenmp, no fast-math)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-fno-fast-math", "-ffp-contract=off", "-Wall", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        d, i64, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
        pp = ctypes.POINTER(Params)
        L.oracle_force.argtypes = [i64, vp, vp, vp, d, i64, vp, vp, vp, vp]
        L.oracle_predict.argtypes = [i64, d, vp, vp, vp, vp, vp, vp, vp]
        L.oracle_correct_one.argtypes = [d] + [vp] * 10
        L.oracle_aarseth_dt.argtypes = [vp, vp, vp, vp, d]
        L.oracle_aarseth_dt.restype = d
        L.oracle_block_dt.argtypes = [d, d, d, pp, vp]
        L.oracle_block_dt.restype = d
        L.oracle_initial_dt.argtypes = [vp, vp, pp, vp]
        L.oracle_initial_dt.restype = d
        L.oracle_init.argtypes = [i64, pp, vp, vp, vp, d, vp, vp, vp, vp, vp]
        L.oracle_block_step.argtypes = [i64, pp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.oracle_block_step.restype = i64
        L.oracle_run.argtypes = [i64, pp, vp, vp, vp, vp, vp, vp, vp, d, i64, vp, vp]
        L.oracle_run.restype = i64
        L.oracle_energy.argtypes = [i64, vp, vp, vp, d, vp, vp]
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def params(eps: float, eta: float = 0.01, eta_init: float = 0.01,
           dt_min_log2: int = -22, dt_max_log2: int = -3) -> Params:
    return Params(eps * eps, eta, eta_init, 2.0 ** dt_min_log2, 2.0 ** dt_max_log2)


def threads() -> int:
    return int(lib().oracle_threads())


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def force(x, v, m, eps: float, i_list=None):
    """Acceleration, jerk and potential on particles i_list (default: all)."""
    x = _f64(x)
    n_total = x.shape[0]
    v = _f64(v, (n_total, 3))
    m = _f64(m, (n_total,))
    il = np.arange(n_total, dtype=np.int64) if i_list is None else \
        np.ascontiguousarray(i_list, dtype=np.int64)
    acc = np.empty((il.size, 3))
    jk = np.empty((il.size, 3))
    pot = np.empty(il.size)
    lib().oracle_force(n_total, _p(x), _p(v), _p(m), float(eps) ** 2, il.size, _p(il),
                       _p(acc), _p(jk), _p(pot))
    return acc, jk, pot


def predict(t, t_i, x, v, a, jk):
    x = _f64(x)
    n_total = x.shape[0]
    t_i = _f64(t_i, (n_total,))
    v, a, jk = (_f64(q, (n_total, 3)) for q in (v, a, jk))
    xp = np.empty_like(x)
    vp = np.empty_like(x)
    lib().oracle_predict(n_total, float(t), _p(t_i), _p(x), _p(v), _p(a), _p(jk), _p(xp), _p(vp))
    return xp, vp


def correct_one(dt, xp, vp, a0, j0, a1, j1):
    ins = [_f64(q, (3,)) for q in (xp, vp, a0, j0, a1, j1)]
    outs = [np.empty(3) for _ in range(4)]
    lib().oracle_correct_one(float(dt), *[_p(q) for q in ins], *[_p(q) for q in outs])
    return tuple(outs)  # x1, v1, a2 at end of step, a3


def aarseth_dt(a, j, a2, a3, eta):
    ins = [_f64(q, (3,)) for q in (a, j, a2, a3)]
    return float(lib().oracle_aarseth_dt(*[_p(q) for q in ins], float(eta)))


def block_dt(dt_old, t_new, dt_raw, prm: Params):
    c = ctypes.c_int(0)
    dt = lib().oracle_block_dt(float(dt_old), float(t_new), float(dt_raw),
                               ctypes.byref(prm), ctypes.byref(c))
    return float(dt), bool(c.value)


def initial_dt(a, j, prm: Params):
    c = ctypes.c_int(0)
    a = _f64(a, (3,))
    j = _f64(j, (3,))
    dt = lib().oracle_initial_dt(_p(a), _p(j), ctypes.byref(prm), ctypes.byref(c))
    return float(dt), bool(c.value)


class System:
    """Integrator state held by the oracle (all float64, AoS)."""

    def __init__(self, x, v, m, prm: Params, t0: float = 0.0):
        self.x = _f64(x).copy()
        n_total = self.x.shape[0]
        self.v = _f64(v, (n_total, 3)).copy()
        self.m = _f64(m, (n_total,)).copy()
        self.prm = prm
        self.a = np.empty((n_total, 3))
        self.jk = np.empty((n_total, 3))
        self.t_i = np.empty(n_total)
        self.dt_i = np.empty(n_total)
        self.n_clamped = ctypes.c_int64(0)
        lib().oracle_init(n_total, ctypes.byref(prm), _p(self.x), _p(self.v), _p(self.m),
                          float(t0), _p(self.a), _p(self.jk), _p(self.t_i), _p(self.dt_i),
                          ctypes.byref(self.n_clamped))

    @classmethod
    def from_state(cls, x, v, m, a, jk, t_i, dt_i, prm: Params):
        """An oracle system holding the given state as is (no start-up sweep)."""
        self = cls.__new__(cls)
        self.x = _f64(x).copy()
        n_total = self.x.shape[0]
        self.v = _f64(v, (n_total, 3)).copy()
        self.m = _f64(m, (n_total,)).copy()
        self.a = _f64(a, (n_total, 3)).copy()
        self.jk = _f64(jk, (n_total, 3)).copy()
        self.t_i = _f64(t_i, (n_total,)).copy()
        self.dt_i = _f64(dt_i, (n_total,)).copy()
        self.prm = prm
        self.n_clamped = ctypes.c_int64(0)
        return self

    @property
    def n(self):
        return self.x.shape[0]

    def step(self):
        """One block step; returns (t, active index array, potential of the block)."""
        t = ctypes.c_double(0.0)
        act = np.empty(self.n, dtype=np.int64)
        pot = np.full(self.n, np.nan)
        nb = lib().oracle_block_step(self.n, ctypes.byref(self.prm), _p(self.x), _p(self.v),
                                     _p(self.a), _p(self.jk), _p(self.m), _p(self.t_i),
                                     _p(self.dt_i), ctypes.byref(t), _p(act),
                                     ctypes.byref(self.n_clamped), _p(pot))
        return t.value, act[:nb].copy(), pot

    def run(self, t_end: float, max_steps: int = 1 << 62):
        """Block steps while the next block time is <= t_end; returns (steps, updates)."""
        upd = ctypes.c_int64(0)
        steps = lib().oracle_run(self.n, ctypes.byref(self.prm), _p(self.x), _p(self.v),
                                 _p(self.a), _p(self.jk), _p(self.m), _p(self.t_i),
                                 _p(self.dt_i), float(t_end), int(max_steps),
                                 ctypes.byref(upd), ctypes.byref(self.n_clamped))
        return int(steps), int(upd.value)

    def energy(self):
        return energy(self.x, self.v, self.m, np.sqrt(self.prm.eps2))


def energy(x, v, m, eps: float):
    """(kinetic, potential) energy of the softened system."""
    x = _f64(x)
    n_total = x.shape[0]
    v = _f64(v, (n_total, 3))
    m = _f64(m, (n_total,))
    ek = ctypes.c_double(0.0)
    ep = ctypes.c_double(0.0)
    lib().oracle_energy(n_total, _p(x), _p(v), _p(m), float(eps) ** 2, ctypes.byref(ek),
                        ctypes.byref(ep))
    return ek.value, ep.value
