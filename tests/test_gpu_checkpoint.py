"""Checkpoint and resume through the C ABI (nbody_save / nbody_load).

A run interrupted by a checkpoint and continued in a fresh context ends in
bitwise the same state, with the same statistics, as a run that was not
interrupted.  A checkpoint of another configuration, and damaged, truncated or
foreign files, are refused and leave the state untouched."""
import os

import numpy as np
import pytest

from nbody_inputs import ensemble, plummer, plummer_salpeter
from paper_0709_4552_amd import NBODY_PREC_FP64, NBODY_PREC_MIXED, NBody, NBodyError
from paper_0709_4552_amd import _lib

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)


def _system(kind):
    if kind == "ensemble":
        x, v, m, offs = ensemble(6, 1012, 256, 1024)
        return x, v, m, offs
    if kind == "shifted":
        # clusters far from the coordinate origin: the mixed records' origins
        # come from the checkpoint (the fresh context's positions are zero)
        x, v, m, offs = ensemble(6, 1013, 256, 1024)
        for k in range(6):
            x[offs[k]:offs[k + 1]] += [1000.0 * (k - 2), -700.0 * k, 64.0 * k + 5]
        return x, v, m, offs
    if kind == "salpeter":
        # a mass spectrum: the mixed form's per-pair near test, chosen from
        # the masses at start-up, must be chosen the same way on resume
        x, v, m = plummer_salpeter(2000, 1016)
        return x, v, m, None
    x, v, m = plummer(2000, 1010)
    return x, v, m, None


@pytest.mark.parametrize("kind,prec", [("single", NBODY_PREC_FP64), ("single", NBODY_PREC_MIXED),
                                       ("ensemble", NBODY_PREC_MIXED),
                                       ("shifted", NBODY_PREC_MIXED),
                                       ("salpeter", NBODY_PREC_MIXED)],
                         ids=["single-fp64", "single-mixed", "ensemble-mixed", "shifted-mixed",
                              "salpeter-mixed"])
def test_resume_is_bitwise_identical(tmp_path, kind, prec):
    note(f"checkpoint resume {kind} prec={prec}")
    x, v, m, offs = _system(kind)
    kw = dict(dt_min_log2=-20, dt_max_log2=-4, precision=prec, cluster_offset=offs)
    a = NBody(x, v, m, 1 / 256, **kw)
    a.init()
    a.run_until(1 / 16)
    path = str(tmp_path / "ck.bin")
    a.save(path)
    assert os.path.exists(path) and not os.path.exists(path + ".part")
    mid = a.stats()
    a.run_until(1 / 8)
    ref, ref_stats = a.host_state(), a.stats()
    a.close()
    # a fresh context of the same configuration, never initialised: the
    # checkpoint brings the whole state
    b = NBody(np.zeros_like(x), np.zeros_like(v), m, 1 / 256, **kw)
    b.load(path)
    assert b.stats() == mid
    b.run_until(1 / 8)
    got = b.host_state()
    for r, g in zip(ref, got):
        assert np.array_equal(r, g)
    assert b.stats() == ref_stats
    b.close()


def test_checkpoint_refusals(tmp_path):
    import torch
    note("checkpoint refusals")
    x, v, m = plummer(500, 1011)
    kw = dict(dt_min_log2=-20, dt_max_log2=-4, precision=NBODY_PREC_MIXED)
    a = NBody(x, v, m, 1 / 256, **kw)
    with pytest.raises(NBodyError) as e:
        a.save(str(tmp_path / "early.bin"))
    assert e.value.code == _lib.NBODY_ESTATE
    a.init()
    a.run_until(1 / 32)
    path = str(tmp_path / "ck.bin")
    a.save(path)
    # another configuration (softening differs)
    c = NBody(x, v, m, 1 / 128, **kw)
    with pytest.raises(NBodyError) as e:
        c.load(path)
    assert e.value.code == _lib.NBODY_EINVAL
    c.close()
    # damaged, truncated, overlong, foreign: EIO and nothing changed
    raw = open(path, "rb").read()
    flipped = bytearray(raw)
    flipped[len(raw) // 2] ^= 0x40
    cases = {"flip": bytes(flipped), "short": raw[:-9], "long": raw + b"\0", "junk": b"hello"}
    for name, data in cases.items():
        p = str(tmp_path / name)
        with open(p, "wb") as f:
            f.write(data)
        before = [t.clone() for t in (a.pos, a.vel, a.acc, a.t_tick, a.level)]
        with pytest.raises(NBodyError) as e:
            a.load(p)
        assert e.value.code == _lib.NBODY_EIO, name
        for t, b in zip((a.pos, a.vel, a.acc, a.t_tick, a.level), before):
            assert torch.equal(t, b), name
    with pytest.raises(NBodyError) as e:
        a.load(str(tmp_path / "missing.bin"))
    assert e.value.code == _lib.NBODY_EIO
    with pytest.raises(NBodyError) as e:
        a.save(str(tmp_path / "no_such_dir" / "ck.bin"))
    assert e.value.code == _lib.NBODY_EIO
    # the context still works after the refusals
    assert a.run_until(1 / 16) > 0
    a.close()
