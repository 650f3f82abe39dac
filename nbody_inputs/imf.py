"""Unequal stellar masses: a Salpeter (1955) power-law mass spectrum.

The paper's outlook (section 6) considers star clusters with a Salpeter mass
spectrum over a wide range of stellar masses.  Masses are drawn from
dN/dm proportional to m^-alpha on [m_lo, m_hi] (alpha = 2.35, masses in solar
units, 0.1 to 100 by default) by inverting the cumulative distribution, then
scaled so the cluster's total mass is 1 (N-body units).  Positions and
velocities come from the equal-mass Plummer realisation: masses are assigned
at random, independent of position, and the centre of mass is moved to rest
again with the new masses.
"""
from __future__ import annotations

import numpy as np

from .plummer import plummer

SALPETER_ALPHA = 2.35


def salpeter_masses(n: int, seed: int, m_lo: float = 0.1, m_hi: float = 100.0,
                    alpha: float = SALPETER_ALPHA):
    """n masses (float64) from the power law, in solar units (not normalised)."""
    if n < 1 or not (0.0 < m_lo < m_hi) or alpha == 1.0:
        raise ValueError("need n >= 1, 0 < m_lo < m_hi and alpha != 1")
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(0.0, 1.0, n)
    e = 1.0 - alpha
    lo, hi = m_lo ** e, m_hi ** e
    return (lo + u * (hi - lo)) ** (1.0 / e)


def plummer_salpeter(n: int, seed: int, m_lo: float = 0.1, m_hi: float = 100.0):
    """(x, v, m): Plummer positions and velocities from `seed`, Salpeter masses
    from seed + 500000, total mass 1, centre of mass at rest."""
    x, v, _ = plummer(n, seed)
    m = salpeter_masses(n, seed + 500000, m_lo, m_hi)
    m = m / m.sum()
    x -= (m[:, None] * x).sum(axis=0)
    v -= (m[:, None] * v).sum(axis=0)
    return np.ascontiguousarray(x), np.ascontiguousarray(v), m
