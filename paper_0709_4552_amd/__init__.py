"""MI355X (gfx950) direct N-body hot path: Hermite-4 block steps with the
force/jerk sum in hand-written HIP kernels behind the C ABI of include/nbody.h.

`NBody` keeps the particle state in torch device tensors (structure of
arrays) and forwards every operation to libnbody.so; nothing is computed in
Python.  The library must be built (paper_0709_4552_amd/build.py); without it
every entry point raises.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (NBODY_PREC_FP64, NBODY_PREC_MIXED, NBodyError, check,  # noqa: F401
                   nbody_tuning)

__all__ = ["NBody", "NBodyError", "NBODY_PREC_FP64", "NBODY_PREC_MIXED", "nbody_tuning",
           "force_jerk_static"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the HIP path needs a gfx950 device")
    return torch


class NBody:
    """Particle system on one GPU (one cluster, or an ensemble of clusters).

    x, v: float64 (N, 3) host arrays; m: float64 (N,).  cluster_offset (int64,
    C+1) makes an ensemble of independent clusters.
    """

    def __init__(self, x, v, m, eps: float, eta: float = 0.01, eta_init: float = 0.01,
                 dt_min_log2: int = -22, dt_max_log2: int = -3,
                 precision: int = NBODY_PREC_MIXED, cluster_offset=None, device: int = 0):
        torch = _torch()
        self.torch = torch
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        m = np.ascontiguousarray(m, dtype=np.float64)
        n = x.shape[0]
        self.n = n
        self.dev = torch.device("cuda", device)
        self.dt_min_log2 = dt_min_log2
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.pos = torch.from_numpy(np.ascontiguousarray(x.T)).to(**f64).contiguous()
        self.vel = torch.from_numpy(np.ascontiguousarray(v.T)).to(**f64).contiguous()
        self.acc = torch.zeros((3, n), **f64)
        self.jerk = torch.zeros((3, n), **f64)
        self.mass = torch.from_numpy(m).to(**f64).contiguous()
        self.t_tick = torch.zeros(n, dtype=torch.int64, device=self.dev)
        self.level = torch.zeros(n, dtype=torch.int8, device=self.dev)
        st = _lib.nbody_state()
        for c in range(3):
            st.pos[c] = self.pos[c].data_ptr()
            st.vel[c] = self.vel[c].data_ptr()
            st.acc[c] = self.acc[c].data_ptr()
            st.jerk[c] = self.jerk[c].data_ptr()
        st.mass = self.mass.data_ptr()
        st.t_tick = self.t_tick.data_ptr()
        st.level = self.level.data_ptr()
        prm = _lib.nbody_params()
        prm.n_total = n
        if cluster_offset is None:
            prm.n_clusters = 1
            prm.cluster_offset = None
            self._offs = None
        else:
            offs = np.ascontiguousarray(cluster_offset, dtype=np.int64)
            self._offs = offs
            prm.n_clusters = offs.size - 1
            prm.cluster_offset = offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        prm.eps = eps
        prm.eta = eta
        prm.eta_init = eta_init
        prm.dt_min_log2 = dt_min_log2
        prm.dt_max_log2 = dt_max_log2
        prm.precision = precision
        self.params = prm
        self.stream = torch.cuda.current_stream(self.dev)
        self.ctx = _lib.nbody_create(prm, st, self.stream.cuda_stream)

    # --- lifecycle ------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            _lib.nbody_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- C ABI, one to one ---------------------------------------------------
    def init(self):
        check(_lib.nbody_init(self.ctx), "nbody_init")

    def predict(self, t: float):
        check(_lib.nbody_predict(self.ctx, t), "nbody_predict")

    def force_jerk(self, i_list, t: float, want_pot: bool = True, out=None):
        """Returns (acc (3,n), jerk (3,n), pot (n,) or None) as device tensors.

        out: optional (acc, jerk, pot-or-None) float64 device tensors of those
        shapes to write into (no allocation per call)."""
        torch = self.torch
        il = torch.as_tensor(i_list, dtype=torch.int32, device=self.dev).contiguous()
        n = il.numel()
        if out is not None:
            acc, jerk, pot = out
            if (tuple(acc.shape) != (3, n) or tuple(jerk.shape) != (3, n) or
                    acc.dtype != torch.float64 or jerk.dtype != torch.float64 or
                    not (acc.is_contiguous() and jerk.is_contiguous()) or
                    (want_pot and (pot is None or tuple(pot.shape) != (n,) or
                                   pot.dtype != torch.float64))):
                raise ValueError("out must hold float64 (3, n), (3, n) and (n,) tensors")
            if not want_pot:
                pot = None
        else:
            acc = torch.empty((3, n), dtype=torch.float64, device=self.dev)
            jerk = torch.empty((3, n), dtype=torch.float64, device=self.dev)
            pot = torch.empty(n, dtype=torch.float64, device=self.dev) if want_pot else None
        check(_lib.nbody_force_jerk(self.ctx, il.data_ptr(), n, t, acc.data_ptr(),
                                    jerk.data_ptr(), pot.data_ptr() if want_pot else None),
              "nbody_force_jerk")
        self._keep = il
        return acc, jerk, pot

    def correct(self, i_list, t: float, acc, jerk):
        torch = self.torch
        il = torch.as_tensor(i_list, dtype=torch.int32, device=self.dev).contiguous()
        check(_lib.nbody_correct(self.ctx, il.data_ptr(), il.numel(), t, acc.data_ptr(),
                                 jerk.data_ptr()), "nbody_correct")
        self._keep = il

    def step_block(self, want_outputs: bool = True):
        rc, t, n = _lib.nbody_step_block(self.ctx, want_outputs)
        check(rc, "nbody_step_block")
        return t, n

    def run_until(self, t_end: float) -> int:
        rc, steps = _lib.nbody_run_until(self.ctx, t_end)
        check(rc, "nbody_run_until")
        return steps

    def sync(self):
        check(_lib.nbody_sync(self.ctx), "nbody_sync")

    def stats(self):
        rc, s = _lib.nbody_get_stats(self.ctx)
        check(rc, "nbody_get_stats")
        return {"block_steps": s.block_steps, "updates": s.updates,
                "interactions": s.interactions, "dt_clamped": s.dt_clamped}

    def read_predicted(self):
        torch = self.torch
        pos = torch.empty((3, self.n), dtype=torch.float64, device=self.dev)
        vel = torch.empty((3, self.n), dtype=torch.float64, device=self.dev)
        check(_lib.nbody_read_predicted(self.ctx, pos.data_ptr(), vel.data_ptr()),
              "nbody_read_predicted")
        return pos, vel

    def get_tuning(self, size_class: int = 0):
        rc, t = _lib.nbody_get_tuning(self.ctx, size_class)
        check(rc, "nbody_get_tuning")
        return {"size_class": t.size_class, "i_per_lane": t.i_per_lane, "j_lanes": t.j_lanes,
                "j_tile": t.j_tile, "grid": t.grid}

    def set_tuning(self, i_per_lane: int, j_lanes: int, j_tile: int = 256, grid: int = 0,
                   size_class: int = 0):
        t = _lib.nbody_tuning(size_class, i_per_lane, j_lanes, j_tile, grid)
        check(_lib.nbody_set_tuning(self.ctx, t), "nbody_set_tuning")

    def set_fused_predict(self, class_mask: int):
        """Size classes whose block steps predict inside the force kernel."""
        check(_lib.nbody_set_fused_predict(self.ctx, class_mask), "nbody_set_fused_predict")

    def autotune(self, n_probe: int):
        """Pick the fastest launch shape for blocks of n_probe; returns (tuning, ms)."""
        rc, t, ms = _lib.nbody_autotune(self.ctx, n_probe)
        check(rc, "nbody_autotune")
        return ({"size_class": t.size_class, "i_per_lane": t.i_per_lane, "j_lanes": t.j_lanes,
                 "j_tile": t.j_tile, "grid": t.grid}, ms)

    def save(self, path: str):
        """Checkpoint: configuration, statistics, tuning and particle state."""
        check(_lib.nbody_save(self.ctx, str(path)), "nbody_save")

    def load(self, path: str):
        """Resume from a checkpoint of a context with the same configuration;
        the state tensors are overwritten (nbody_init is not needed)."""
        check(_lib.nbody_load(self.ctx, str(path)), "nbody_load")

    # --- host views (copies) ------------------------------------------------
    def host_state(self):
        """(x, v, a, jerk) as float64 (N, 3) numpy arrays, t (N,) and dt (N,)."""
        self.torch.cuda.synchronize(self.dev)
        x = self.pos.T.cpu().numpy().copy()
        v = self.vel.T.cpu().numpy().copy()
        a = self.acc.T.cpu().numpy().copy()
        j = self.jerk.T.cpu().numpy().copy()
        t = self.t_tick.cpu().numpy().astype(np.float64) * 2.0 ** self.dt_min_log2
        dt = 2.0 ** (-self.level.cpu().numpy().astype(np.float64))
        return x, v, a, j, t, dt


def force_jerk_static(pos, vel, mass, eps: float, i_list, precision: int = NBODY_PREC_MIXED,
                      acc_hint=None, jerk_hint=None, want_pot: bool = True, stream=None):
    """Force, jerk and potential on the particles i_list from all particles
    given, through the allocation-free entry point (nbody_force_jerk_static).

    pos, vel: float64 device tensors (3, n_j), contiguous rows; mass: (n_j,);
    acc_hint, jerk_hint: (3, n_j) or None (mixed form only).  Returns
    (acc (3, n), jerk (3, n), pot (n,) or None) as device tensors, allocated
    here by torch (the library call itself allocates nothing).
    """
    torch = _torch()
    dev = pos.device
    il = torch.as_tensor(i_list, dtype=torch.int32, device=dev).contiguous()
    n = il.numel()
    d = _lib.nbody_direct()
    d.n_j = int(mass.numel())
    for c in range(3):
        d.pos[c] = pos[c].data_ptr()
        d.vel[c] = vel[c].data_ptr()
        d.acc_hint[c] = acc_hint[c].data_ptr() if acc_hint is not None else None
        d.jerk_hint[c] = jerk_hint[c].data_ptr() if jerk_hint is not None else None
    d.mass = mass.data_ptr()
    d.eps = float(eps)
    d.precision = int(precision)
    acc = torch.empty((3, n), dtype=torch.float64, device=dev)
    jerk = torch.empty((3, n), dtype=torch.float64, device=dev)
    pot = torch.empty(n, dtype=torch.float64, device=dev) if want_pot else None
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    check(_lib.nbody_force_jerk_static(d, il.data_ptr(), n, acc.data_ptr(), jerk.data_ptr(),
                                       pot.data_ptr() if want_pot else None, s.cuda_stream),
          "nbody_force_jerk_static")
    s.synchronize()  # il must outlive the asynchronous call
    return acc, jerk, pot
