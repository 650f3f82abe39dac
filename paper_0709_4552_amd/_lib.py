"""ctypes binding of libnbody.so (include/nbody.h).  Argument marshalling only.

Every entry point of the C ABI is exposed under the same name; device
pointers are plain integers (torch.Tensor.data_ptr()).  Loading fails loudly
when the shared library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("NBODY_LIB") or os.path.join(HERE, "libnbody.so")

NBODY_OK = 0
NBODY_EINVAL = -1
NBODY_ESTATE = -2
NBODY_ENOMEM = -3
NBODY_EDEVICE = -4
NBODY_ENONFINITE = -5
NBODY_EUNSUPPORTED = -6
NBODY_ERANGE = -7
NBODY_EIO = -8
NBODY_ESCRATCH = -9
NBODY_EEXTENT = -10
NBODY_STATIC_MAX_PARTICLES = 262144

NBODY_PREC_FP64 = 0
NBODY_PREC_MIXED = 1

# every symbol include/nbody.h declares
EXPORTS = (
    "nbody_strerror", "nbody_create", "nbody_destroy", "nbody_init", "nbody_predict",
    "nbody_force_jerk", "nbody_correct", "nbody_step_block", "nbody_run_until", "nbody_sync",
    "nbody_get_stats", "nbody_read_predicted", "nbody_get_tuning", "nbody_set_tuning",
    "nbody_autotune", "nbody_save", "nbody_load", "nbody_set_fused_predict",
    "nbody_force_jerk_static",
)


class nbody_state(ctypes.Structure):
    _fields_ = [
        ("pos", ctypes.c_void_p * 3),
        ("vel", ctypes.c_void_p * 3),
        ("acc", ctypes.c_void_p * 3),
        ("jerk", ctypes.c_void_p * 3),
        ("mass", ctypes.c_void_p),
        ("t_tick", ctypes.c_void_p),
        ("level", ctypes.c_void_p),
    ]


class nbody_params(ctypes.Structure):
    _fields_ = [
        ("n_total", ctypes.c_int64),
        ("n_clusters", ctypes.c_int32),
        ("cluster_offset", ctypes.POINTER(ctypes.c_int64)),
        ("eps", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("eta_init", ctypes.c_double),
        ("dt_min_log2", ctypes.c_int32),
        ("dt_max_log2", ctypes.c_int32),
        ("precision", ctypes.c_int32),
    ]


NBODY_SIZE_CLASSES = 5


class nbody_tuning(ctypes.Structure):
    _fields_ = [
        ("size_class", ctypes.c_int32),
        ("i_per_lane", ctypes.c_int32),
        ("j_lanes", ctypes.c_int32),
        ("j_tile", ctypes.c_int32),
        ("grid", ctypes.c_int32),
    ]


class nbody_direct(ctypes.Structure):
    _fields_ = [
        ("n_j", ctypes.c_int64),
        ("pos", ctypes.c_void_p * 3),
        ("vel", ctypes.c_void_p * 3),
        ("mass", ctypes.c_void_p),
        ("acc_hint", ctypes.c_void_p * 3),
        ("jerk_hint", ctypes.c_void_p * 3),
        ("eps", ctypes.c_double),
        ("precision", ctypes.c_int32),
    ]


class nbody_stats(ctypes.Structure):
    _fields_ = [
        ("block_steps", ctypes.c_int64),
        ("updates", ctypes.c_int64),
        ("interactions", ctypes.c_double),
        ("dt_clamped", ctypes.c_int64),
    ]


class NBodyError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_lib = None


def load(path: str = LIB_PATH):
    """Load libnbody.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_0709_4552_amd/build.py "
                           "(or __graft_entry__.build())")
    L = ctypes.CDLL(path)
    vp, i64, d, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    L.nbody_strerror.argtypes = [i32]
    L.nbody_strerror.restype = ctypes.c_char_p
    L.nbody_create.argtypes = [ctypes.POINTER(nbody_params), ctypes.POINTER(nbody_state), vp,
                               ctypes.POINTER(vp)]
    L.nbody_destroy.argtypes = [vp]
    L.nbody_init.argtypes = [vp]
    L.nbody_predict.argtypes = [vp, d]
    L.nbody_force_jerk.argtypes = [vp, vp, i64, d, vp, vp, vp]
    L.nbody_correct.argtypes = [vp, vp, i64, d, vp, vp]
    L.nbody_step_block.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(i64)]
    L.nbody_run_until.argtypes = [vp, d, ctypes.POINTER(i64)]
    L.nbody_sync.argtypes = [vp]
    L.nbody_get_stats.argtypes = [vp, ctypes.POINTER(nbody_stats)]
    L.nbody_read_predicted.argtypes = [vp, vp, vp]
    L.nbody_get_tuning.argtypes = [vp, ctypes.POINTER(nbody_tuning)]
    L.nbody_set_tuning.argtypes = [vp, ctypes.POINTER(nbody_tuning)]
    L.nbody_set_fused_predict.argtypes = [vp, ctypes.c_int32]
    L.nbody_autotune.argtypes = [vp, i64, ctypes.POINTER(nbody_tuning), ctypes.POINTER(d)]
    L.nbody_force_jerk_static.argtypes = [ctypes.POINTER(nbody_direct), vp, i64, vp, vp, vp, vp]
    L.nbody_save.argtypes = [vp, ctypes.c_char_p]
    L.nbody_load.argtypes = [vp, ctypes.c_char_p]
    for name in EXPORTS:
        if name != "nbody_strerror":
            getattr(L, name).restype = i32
    _lib = L
    return L


def strerror(code: int) -> str:
    return load().nbody_strerror(int(code)).decode()


def check(code: int, where: str) -> int:
    if code != NBODY_OK:
        raise NBodyError(code, where)
    return code


# ---- thin wrappers, same names as the C ABI ---------------------------------

def nbody_create(params: nbody_params, state: nbody_state, stream: int) -> int:
    out = ctypes.c_void_p()
    rc = load().nbody_create(ctypes.byref(params), ctypes.byref(state), ctypes.c_void_p(stream),
                             ctypes.byref(out))
    check(rc, "nbody_create")
    return out.value


def nbody_destroy(ctx: int) -> int:
    return load().nbody_destroy(ctypes.c_void_p(ctx))


def nbody_init(ctx: int) -> int:
    return load().nbody_init(ctypes.c_void_p(ctx))


def nbody_predict(ctx: int, t: float) -> int:
    return load().nbody_predict(ctypes.c_void_p(ctx), float(t))


def nbody_force_jerk(ctx: int, i_list_ptr: int, n: int, t: float, acc_ptr: int, jerk_ptr: int,
                     pot_ptr: int | None) -> int:
    return load().nbody_force_jerk(ctypes.c_void_p(ctx), ctypes.c_void_p(i_list_ptr), int(n),
                                   float(t), ctypes.c_void_p(acc_ptr), ctypes.c_void_p(jerk_ptr),
                                   ctypes.c_void_p(pot_ptr or 0))


def nbody_correct(ctx: int, i_list_ptr: int, n: int, t: float, acc_ptr: int, jerk_ptr: int) -> int:
    return load().nbody_correct(ctypes.c_void_p(ctx), ctypes.c_void_p(i_list_ptr), int(n),
                                float(t), ctypes.c_void_p(acc_ptr), ctypes.c_void_p(jerk_ptr))


def nbody_step_block(ctx: int, want_outputs: bool = True):
    if not want_outputs:
        return load().nbody_step_block(ctypes.c_void_p(ctx), None, None), None, None
    t = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    rc = load().nbody_step_block(ctypes.c_void_p(ctx), ctypes.byref(t), ctypes.byref(n))
    return rc, t.value, n.value


def nbody_run_until(ctx: int, t_end: float):
    n = ctypes.c_int64(0)
    rc = load().nbody_run_until(ctypes.c_void_p(ctx), float(t_end), ctypes.byref(n))
    return rc, n.value


def nbody_sync(ctx: int) -> int:
    return load().nbody_sync(ctypes.c_void_p(ctx))


def nbody_get_stats(ctx: int):
    s = nbody_stats()
    rc = load().nbody_get_stats(ctypes.c_void_p(ctx), ctypes.byref(s))
    return rc, s


def nbody_read_predicted(ctx: int, pos_ptr: int, vel_ptr: int) -> int:
    return load().nbody_read_predicted(ctypes.c_void_p(ctx), ctypes.c_void_p(pos_ptr),
                                       ctypes.c_void_p(vel_ptr))


def nbody_get_tuning(ctx: int, size_class: int = 0):
    t = nbody_tuning()
    t.size_class = size_class
    rc = load().nbody_get_tuning(ctypes.c_void_p(ctx), ctypes.byref(t))
    return rc, t


def nbody_set_tuning(ctx: int, tuning: nbody_tuning) -> int:
    return load().nbody_set_tuning(ctypes.c_void_p(ctx), ctypes.byref(tuning))


def nbody_set_fused_predict(ctx: int, class_mask: int) -> int:
    return load().nbody_set_fused_predict(ctypes.c_void_p(ctx), int(class_mask))


def nbody_autotune(ctx: int, n_probe: int):
    t = nbody_tuning()
    ms = ctypes.c_double(0.0)
    rc = load().nbody_autotune(ctypes.c_void_p(ctx), int(n_probe), ctypes.byref(t),
                               ctypes.byref(ms))
    return rc, t, ms.value


def nbody_save(ctx: int, path: str) -> int:
    return load().nbody_save(ctypes.c_void_p(ctx), os.fsencode(path))


def nbody_load(ctx: int, path: str) -> int:
    return load().nbody_load(ctypes.c_void_p(ctx), os.fsencode(path))


def nbody_force_jerk_static(direct: nbody_direct, i_list_ptr: int, n: int, acc_ptr: int,
                            jerk_ptr: int, pot_ptr: int | None, stream: int | None) -> int:
    return load().nbody_force_jerk_static(ctypes.byref(direct), ctypes.c_void_p(i_list_ptr),
                                          int(n), ctypes.c_void_p(acc_ptr),
                                          ctypes.c_void_p(jerk_ptr), ctypes.c_void_p(pot_ptr or 0),
                                          ctypes.c_void_p(stream or 0))
