"""Plummer-sphere initial conditions in Henon (N-body) units.

The paper starts every run from a Plummer sphere in virial equilibrium and
integrates for one N-body time unit (section 2, "Experimental setup"); it
states that the particular realisation does not matter for the timings.  We
use the standard realisation:

* G = M = 1, equal masses m = 1/N;
* Plummer scale length b = 3*pi/16, which gives total energy E = -1/4 and
  virial radius 1 for the untruncated model;
* radius from the inverse of the cumulative mass M(r) = r^3/(r^2+b^2)^{3/2},
  with the mass fraction drawn in (0, 0.999) so no particle sits at huge r;
* speed q * v_esc(r), v_esc = sqrt(2) (r^2+b^2)^{-1/4}, with q drawn by
  rejection from the density q^2 (1-q^2)^{7/2} on [0, 1];
* isotropic position and velocity directions;
* finally the centre of mass is moved to rest at the origin.

No exact rescaling to E = -1/4 is done: that would need the pairwise
potential, which belongs to the method under test and not to its inputs.
The sampled model therefore meets E = -1/4 and 2T/|U| = 1 only up to
sampling noise of order 1/sqrt(N).

Every array is float64.  Positions and velocities are returned as (N, 3).
"""
from __future__ import annotations

import math

import numpy as np

PLUMMER_B = 3.0 * math.pi / 16.0
MASS_CUTOFF = 0.999


def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    cos_t = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    return np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t], axis=1)


def _speed_fractions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Rejection sampling of q from g(q) = q^2 (1-q^2)^{7/2}; max g < 0.1."""
    out = np.empty(n)
    filled = 0
    while filled < n:
        want = n - filled
        batch = max(64, int(want * 6))
        q = rng.uniform(0.0, 1.0, batch)
        y = rng.uniform(0.0, 0.1, batch)
        keep = q[y < q * q * (1.0 - q * q) ** 3.5]
        take = min(want, keep.size)
        out[filled:filled + take] = keep[:take]
        filled += take
    return out


def plummer(n: int, seed: int):
    """Return (x, v, m) for an n-particle Plummer sphere drawn from `seed`.

    x, v: float64 (n, 3); m: float64 (n,) all equal to 1/n.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.Generator(np.random.PCG64(seed))
    frac = rng.uniform(0.0, MASS_CUTOFF, n)
    frac = np.maximum(frac, 1e-300)
    r = PLUMMER_B / np.sqrt(frac ** (-2.0 / 3.0) - 1.0)
    x = r[:, None] * _unit_vectors(rng, n)
    q = _speed_fractions(rng, n)
    vesc = math.sqrt(2.0) * (r * r + PLUMMER_B * PLUMMER_B) ** -0.25
    v = (q * vesc)[:, None] * _unit_vectors(rng, n)
    m = np.full(n, 1.0 / n)
    x -= (m[:, None] * x).sum(axis=0) / m.sum()
    v -= (m[:, None] * v).sum(axis=0) / m.sum()
    return np.ascontiguousarray(x), np.ascontiguousarray(v), m


def ensemble_sizes(n_clusters: int, seed: int, n_lo: int = 256, n_hi: int = 8192):
    """Cluster sizes drawn log-uniform in [n_lo, n_hi] from `seed` (int64 array)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(math.log(n_lo), math.log(n_hi), n_clusters)
    return np.clip(np.rint(np.exp(u)).astype(np.int64), n_lo, n_hi)


def ensemble(n_clusters: int, seed: int, n_lo: int = 256, n_hi: int = 8192):
    """Concatenated independent Plummer clusters.

    Cluster k uses seed 1000*seed + k.  Returns (x, v, m, offsets) where
    offsets is int64 (n_clusters+1,) with cluster k at [offsets[k], offsets[k+1]).
    Masses are 1/N_k inside cluster k.
    """
    sizes = ensemble_sizes(n_clusters, seed, n_lo, n_hi)
    offs = np.zeros(n_clusters + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    xs, vs, ms = [], [], []
    for k, nk in enumerate(sizes):
        x, v, m = plummer(int(nk), 1000 * seed + k)
        xs.append(x)
        vs.append(v)
        ms.append(m)
    return (np.concatenate(xs), np.concatenate(vs), np.concatenate(ms), offs)
