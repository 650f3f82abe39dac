"""The C-ABI library loads and exports every entry point include/nbody.h
declares; host-side argument checks reject bad input before any device work.
No GPU needed: nothing here launches a kernel."""
import ctypes
import os
import re

import pytest

from paper_0709_4552_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nbody_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_struct_layouts_match_header():
    # nbody_state: 15 pointers; nbody_params: int64, int32(+pad), ptr, 3 doubles, 3 int32 (+pad)
    assert ctypes.sizeof(_lib.nbody_state) == 15 * 8
    assert ctypes.sizeof(_lib.nbody_params) == 8 + 8 + 8 + 24 + 16
    assert ctypes.sizeof(_lib.nbody_tuning) == 20
    assert ctypes.sizeof(_lib.nbody_stats) == 32
    # nbody_direct: int64, 13 pointers, double, int32 (+pad)
    assert ctypes.sizeof(_lib.nbody_direct) == 8 + 13 * 8 + 8 + 8


def test_strerror_names_every_code():
    for code in range(0, -11, -1):
        assert _lib.strerror(code) != "unknown status"
    assert _lib.strerror(-99) == "unknown status"


def _params(**kw):
    p = _lib.nbody_params()
    p.n_total = kw.get("n_total", 16)
    p.n_clusters = kw.get("n_clusters", 1)
    p.cluster_offset = kw.get("cluster_offset", None)
    p.eps = kw.get("eps", 0.01)
    p.eta = kw.get("eta", 0.01)
    p.eta_init = kw.get("eta_init", 0.01)
    p.dt_min_log2 = kw.get("dt_min_log2", -20)
    p.dt_max_log2 = kw.get("dt_max_log2", -3)
    p.precision = kw.get("precision", 1)
    return p


def _state(null_field=None):
    s = _lib.nbody_state()
    fake = 0x1000  # never dereferenced: creation fails on the host checks first
    for c in range(3):
        s.pos[c] = s.vel[c] = s.acc[c] = s.jerk[c] = fake
    s.mass = s.t_tick = s.level = fake
    if null_field == "mass":
        s.mass = None
    if null_field == "pos":
        s.pos[1] = None
    return s


@pytest.mark.parametrize("kw", [
    dict(n_total=0), dict(n_total=-5), dict(n_clusters=0), dict(n_clusters=20),
    dict(eps=-1.0), dict(eps=float("nan")), dict(eta=0.0), dict(eta_init=-1.0),
    dict(dt_min_log2=-3, dt_max_log2=-20), dict(dt_max_log2=1), dict(dt_min_log2=-41),
    dict(precision=7), dict(n_clusters=2, cluster_offset=None),
])
def test_create_rejects_bad_params(kw):
    L = _lib.load()
    out = ctypes.c_void_p()
    rc = L.nbody_create(ctypes.byref(_params(**kw)), ctypes.byref(_state()), None, ctypes.byref(out))
    assert rc == _lib.NBODY_EINVAL and not out.value


@pytest.mark.parametrize("offs", [[0, 8, 8, 16], [1, 8, 16], [0, 8, 15], [0, 9, 8, 16]])
def test_create_rejects_bad_cluster_offsets(offs):
    L = _lib.load()
    arr = (ctypes.c_int64 * len(offs))(*offs)
    p = _params(n_clusters=len(offs) - 1,
                cluster_offset=ctypes.cast(arr, ctypes.POINTER(ctypes.c_int64)))
    out = ctypes.c_void_p()
    assert L.nbody_create(ctypes.byref(p), ctypes.byref(_state()), None,
                          ctypes.byref(out)) == _lib.NBODY_EINVAL


@pytest.mark.parametrize("field", ["mass", "pos"])
def test_create_rejects_null_state(field):
    L = _lib.load()
    out = ctypes.c_void_p()
    assert L.nbody_create(ctypes.byref(_params()), ctypes.byref(_state(field)), None,
                          ctypes.byref(out)) == _lib.NBODY_EINVAL


def test_null_context_is_rejected():
    L = _lib.load()
    assert L.nbody_init(None) == _lib.NBODY_EINVAL
    assert L.nbody_predict(None, 0.0) == _lib.NBODY_EINVAL
    assert L.nbody_sync(None) == _lib.NBODY_EINVAL
    assert L.nbody_destroy(None) == _lib.NBODY_EINVAL
    assert L.nbody_save(None, b"/tmp/x") == _lib.NBODY_EINVAL
    assert L.nbody_load(None, b"/tmp/x") == _lib.NBODY_EINVAL
    assert L.nbody_set_fused_predict(None, 0) == _lib.NBODY_EINVAL


def _direct(**kw):
    d = _lib.nbody_direct()
    fake = 0x1000  # never dereferenced: the call fails on the host checks first
    d.n_j = kw.get("n_j", 16)
    for c in range(3):
        d.pos[c] = d.vel[c] = fake
    d.mass = fake
    for c in kw.get("hints", ()):
        d.acc_hint[c] = fake
    d.eps = kw.get("eps", 0.01)
    d.precision = kw.get("precision", 1)
    if kw.get("null_mass"):
        d.mass = None
    return d


@pytest.mark.parametrize("kw,n,code", [
    (dict(n_j=_lib.NBODY_STATIC_MAX_PARTICLES + 1), 1, _lib.NBODY_ESCRATCH),
    (dict(n_j=16), _lib.NBODY_STATIC_MAX_PARTICLES + 1, _lib.NBODY_ESCRATCH),
    (dict(n_j=0), 1, _lib.NBODY_EINVAL),
    (dict(n_j=16), 0, _lib.NBODY_EINVAL),
    (dict(eps=-1.0), 1, _lib.NBODY_EINVAL),
    (dict(precision=3), 1, _lib.NBODY_EINVAL),
    (dict(null_mass=True), 1, _lib.NBODY_EINVAL),
    (dict(hints=(0, 1, 2)), 1, _lib.NBODY_EINVAL),  # acceleration hints without jerk hints
])
def test_static_force_rejects_bad_arguments(kw, n, code):
    # checked on the host before any device call (no GPU is touched here)
    L = _lib.load()
    out = ctypes.c_void_p(0x1000)
    rc = L.nbody_force_jerk_static(ctypes.byref(_direct(**kw)), out, n, out, out, None, None)
    assert rc == code
