"""Checks of the seeded Plummer generator (section 2: Plummer spheres in
virial equilibrium, N-body units)."""
import math

import numpy as np

import oracle
from nbody_inputs import ensemble, ensemble_sizes, plummer


def test_plummer_deterministic_and_centred():
    x1, v1, m1 = plummer(2048, 1001)
    x2, v2, m2 = plummer(2048, 1001)
    np.testing.assert_array_equal(x1, x2)
    np.testing.assert_array_equal(v1, v2)
    assert np.all(m1 == 1.0 / 2048)
    assert np.abs((m1[:, None] * x1).sum(0)).max() < 1e-14
    assert np.abs((m1[:, None] * v1).sum(0)).max() < 1e-14
    x3, _, _ = plummer(2048, 1002)
    assert not np.array_equal(x1, x3)


def test_plummer_units_statistics():
    # Henon units: E = -1/4, virial ratio 1, half-mass radius b/sqrt(2^{2/3}-1)
    n = 8192
    x, v, m = plummer(n, 1002)
    ek, ep = oracle.energy(x, v, m, 0.0)
    assert abs((ek + ep) + 0.25) < 0.02
    assert abs(2 * ek / abs(ep) - 1.0) < 0.05
    rh = np.median(np.linalg.norm(x, axis=1))
    b = 3 * math.pi / 16
    assert abs(rh - b / math.sqrt(2 ** (2 / 3) - 1)) < 0.04
    # the mass cut at 0.999 bounds the largest radius
    assert np.linalg.norm(x, axis=1).max() < b / math.sqrt(0.999 ** (-2 / 3) - 1) + 1e-9 + 0.1


def test_ensemble_sizes_and_offsets():
    s = ensemble_sizes(256, 1004)
    assert s.shape == (256,) and s.min() >= 256 and s.max() <= 8192
    # log-uniform: median near sqrt(256*8192) = 1448
    assert 1000 < np.median(s) < 2100
    x, v, m, offs = ensemble(8, 1004, 256, 512)
    assert offs[0] == 0 and offs[-1] == x.shape[0]
    for k in range(8):
        nk = offs[k + 1] - offs[k]
        assert np.all(m[offs[k]:offs[k + 1]] == 1.0 / nk)


def test_salpeter_masses_follow_the_power_law():
    # against the analytic distribution dN/dm ~ m^-2.35 on [0.1, 100]
    from nbody_inputs import salpeter_masses
    n, lo, hi, a = 200000, 0.1, 100.0, 2.35
    m = salpeter_masses(n, 77)
    assert m.min() >= lo and m.max() <= hi
    assert np.array_equal(m, salpeter_masses(n, 77))
    e = 1.0 - a
    ms = np.sort(m)
    cdf = (ms ** e - lo ** e) / (hi ** e - lo ** e)
    emp_hi = np.arange(1, n + 1) / n
    d = max(np.max(emp_hi - cdf), np.max(cdf - (emp_hi - 1.0 / n)))
    assert d < 1.63 / np.sqrt(n)  # Kolmogorov-Smirnov, 1% level
    z = (hi ** e - lo ** e) / e  # normalisation of m^-a
    mean = (hi ** (2 - a) - lo ** (2 - a)) / (2 - a) / z
    var = (hi ** (3 - a) - lo ** (3 - a)) / (3 - a) / z - mean ** 2
    assert abs(m.mean() - mean) < 5.0 * np.sqrt(var / n)
    # about 0.35 solar masses on average for this range
    assert 0.3 < mean < 0.4


def test_plummer_salpeter_units_and_centre():
    from nbody_inputs import plummer, plummer_salpeter
    x, v, m = plummer_salpeter(5000, 31)
    x0, v0, _ = plummer(5000, 31)
    assert abs(m.sum() - 1.0) < 1e-12
    assert np.abs((m[:, None] * x).sum(axis=0)).max() < 1e-14
    assert np.abs((m[:, None] * v).sum(axis=0)).max() < 1e-14
    # the same positions and velocities, only shifted as a whole
    dx = x - x0
    assert np.abs(dx - dx[0]).max() < 1e-12
    assert m.max() / m.min() > 100.0
