"""The allocation-free entry point (nbody_force_jerk_static) against the
context entry point it is a variant of (nbody_force_jerk), through the C ABI,
and both against the oracle.

Several calls in a row on one GPU share the library's static scratch array,
which keeps each call's contents: the calls run from the largest input (the
maximum size) down to smaller ones, so stale records, hints, partial sums or
plans of an earlier call would show up in a later one.
"""
import numpy as np
import pytest

import oracle
from nbody_inputs import plummer, plummer_salpeter
from paper_0709_4552_amd import (NBODY_PREC_FP64, NBODY_PREC_MIXED, NBody, NBodyError,
                                 force_jerk_static)
from paper_0709_4552_amd import _lib

pytestmark = pytest.mark.gpu

TOL = {NBODY_PREC_FP64: dict(a=1e-11, j=1e-9, p=1e-12),
       NBODY_PREC_MIXED: dict(a=1e-6, j=1e-5, p=1e-6)}
PREC = [NBODY_PREC_FP64, NBODY_PREC_MIXED]
PID = ["fp64", "mixed"]


def note(msg):
    print(msg, flush=True)


def relerr(g, r):
    g, r = np.asarray(g), np.asarray(r)
    if g.ndim == 1:
        return np.abs(g - r) / np.abs(r)
    return np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)


# (N, n, seed, masses): the maximum size with a random block, a full sweep, a
# short list with duplicates, and a Salpeter cluster
CALLS = ((_lib.NBODY_STATIC_MAX_PARTICLES, 4096, 1021, "equal"),
         (5000, 5000, 1022, "equal"),
         (1200, 77, 1023, "equal"),
         (3000, 600, 1024, "salpeter"))


@pytest.mark.parametrize("hints", [True, False], ids=["hints", "no-hints"])
@pytest.mark.parametrize("prec", PREC, ids=PID)
def test_static_matches_context_entry_point(prec, hints):
    eps = 1 / 256
    for N, n, seed, masses in CALLS:
        note(f"N={N} n={n} masses={masses} prec={prec} hints={hints}")
        x, v, m = plummer(N, seed) if masses == "equal" else plummer_salpeter(N, seed)
        rng = np.random.Generator(np.random.PCG64(seed))
        il = np.arange(N, dtype=np.int32) if n == N else rng.integers(0, N, n).astype(np.int32)
        g = NBody(x, v, m, eps, dt_min_log2=-20, dt_max_log2=-3, precision=prec)
        g.init()  # t = 0: positions and velocities unchanged, a and jerk stored
        g.predict(0.0)
        a0, j0, p0 = g.force_jerk(il, 0.0)
        ah, jh = (g.acc, g.jerk) if hints else (None, None)
        a1, j1, p1 = force_jerk_static(g.pos, g.vel, g.mass, eps, il, prec, ah, jh)
        a0, j0, p0 = a0.T.cpu().numpy(), j0.T.cpu().numpy(), p0.cpu().numpy()
        a1, j1, p1 = a1.T.cpu().numpy(), j1.T.cpu().numpy(), p1.cpu().numpy()
        g.close()
        da, dj, dp = relerr(a1, a0).max(), relerr(j1, j0).max(), relerr(p1, p0).max()
        # both against the oracle on (up to) 512 of the listed particles
        k = min(n, 512)
        ra, rj, rp = oracle.force(x, v, m, eps, il[:k])
        ea, ej, ep = relerr(a1[:k], ra).max(), relerr(j1[:k], rj).max(), relerr(p1[:k], rp).max()
        note(f"  static vs context: acc {da:.2e} jerk {dj:.2e} pot {dp:.2e}; "
             f"static vs oracle: acc {ea:.2e} jerk {ej:.2e} pot {ep:.2e}")
        t = TOL[prec]
        assert da <= t["a"] and dj <= t["j"] and dp <= t["p"]
        assert ea <= t["a"] and ej <= t["j"] and ep <= t["p"]


def test_static_size_limit_is_refused():
    torch = pytest.importorskip("torch")
    N = _lib.NBODY_STATIC_MAX_PARTICLES + 1
    dev = torch.device("cuda", 0)
    z = torch.zeros((3, N), dtype=torch.float64, device=dev)
    with pytest.raises(NBodyError) as e:
        force_jerk_static(z, z, z[0], 0.01, [0], NBODY_PREC_MIXED)
    assert e.value.code == _lib.NBODY_ESCRATCH
