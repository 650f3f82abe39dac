"""Pins for the FP64 oracle against closed forms, invariants and brute force.

The paper prints no worked numerical example (no force, trajectory or energy
value), so every pin here comes from mathematics fixed independently of the
oracle's code: Newton's shell theorem and symmetric configurations, finite
differences (jerk = da/dt, a = -grad(potential)), Taylor/polynomial identities
evaluated with numpy.polynomial, two-body orbits in closed form (softened
circular orbit, Kepler's equation), and conservation laws.  Each test names the
part of the method it pins.
"""
import math

import numpy as np
import pytest

import oracle
from nbody_inputs import plummer


def _rot(t):
    c, s = math.cos(t), math.sin(t)
    return np.array([c, s, 0.0])


# --- force / jerk / potential (section 4.1, step 4) -------------------------

def test_two_body_attraction_direction_and_symmetry():
    x = np.array([[0.1, -0.2, 0.3], [0.7, 0.1, -0.2]])
    v = np.zeros((2, 3))
    m = np.array([0.25, 0.75])
    a, j, p = oracle.force(x, v, m, eps=0.05)
    r = x[1] - x[0]
    # attraction: particle 0 accelerates toward 1, particle 1 toward 0
    assert np.dot(a[0], r) > 0 and np.dot(a[1], r) < 0
    # acceleration parallel to the separation
    assert np.linalg.norm(np.cross(a[0], r)) < 1e-14 * np.linalg.norm(a[0]) * np.linalg.norm(r)
    # third law
    np.testing.assert_allclose(m[0] * a[0], -m[1] * a[1], rtol=1e-15, atol=0)
    # at rest: jerk is zero
    np.testing.assert_array_equal(j, 0.0)
    # Plummer-softened point-mass potential of the other body (textbook form)
    d = np.linalg.norm(r)
    assert p[0] == pytest.approx(-m[1] / math.sqrt(d * d + 0.05 ** 2), rel=1e-15)
    assert p[1] == pytest.approx(-m[0] / math.sqrt(d * d + 0.05 ** 2), rel=1e-15)


def test_symmetric_shells_give_zero_force_at_centre():
    # cube vertices + octahedron vertices around a centre particle: the
    # centre feels exactly no force by symmetry, for any softening.
    cube = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], float)
    octa = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    x = np.vstack([[0.0, 0.0, 0.0], 0.3 * cube, 0.7 * octa])
    v = np.zeros_like(x)
    m = np.full(len(x), 1.0 / len(x))
    for eps in (0.0, 0.01, 0.5):
        a, j, p = oracle.force(x, v, m, eps, i_list=[0])
        assert np.all(np.abs(a[0]) < 1e-16)


def test_shell_theorem_outside_fibonacci_sphere():
    # A thin shell of total mass M acts on an outside point as a point mass M
    # at its centre (Newton).  A Fibonacci lattice of K points approximates the
    # shell; its low multipoles vanish to O(1/K), so the test point at 4 radii
    # sees -M/r^2 to well below 1e-4.
    K = 4000
    k = np.arange(K) + 0.5
    th = np.arccos(1 - 2 * k / K)
    ph = math.pi * (1 + 5 ** 0.5) * k
    shell = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
    x = np.vstack([shell, [[0.0, 0.0, 4.0]]])
    m = np.concatenate([np.full(K, 1.0 / K), [1e-3]])
    a, _, p = oracle.force(x, np.zeros_like(x), m, 0.0, i_list=[K])
    assert a[0, 2] == pytest.approx(-1.0 / 16.0, rel=1e-4)
    assert abs(a[0, 0]) < 1e-6 and abs(a[0, 1]) < 1e-6
    assert p[0] == pytest.approx(-1.0 / 4.0, rel=1e-4)
    # inside the shell the force vanishes (to lattice accuracy)
    x[K] = [0.1, -0.05, 0.2]
    a, _, p = oracle.force(x, np.zeros_like(x), m, 0.0, i_list=[K])
    assert np.linalg.norm(a[0]) < 1e-3
    assert p[0] == pytest.approx(-1.0, rel=1e-3)


def test_equilateral_triangle_points_to_centroid():
    s = 0.8
    x = np.array([[0, 0, 0], [s, 0, 0], [s / 2, s * math.sqrt(3) / 2, 0]], float)
    m = np.full(3, 1.0 / 3)
    a, _, _ = oracle.force(x, np.zeros_like(x), m, 0.0)
    c = x.mean(0)
    for i in range(3):
        u = (c - x[i]) / np.linalg.norm(c - x[i])
        # unsoftened: two pulls of m/s^2 at +-30 degrees from the centroid line
        np.testing.assert_allclose(a[i], 2 * (1 / 3) / s ** 2 * math.cos(math.pi / 6) * u,
                                   rtol=1e-14, atol=1e-15)


def test_momentum_balance_with_unequal_masses():
    # Salpeter masses spanning a factor 1000: the force on i must weigh the
    # sources by m_j, or sum m_i a_i no longer vanishes
    from nbody_inputs import plummer_salpeter
    x, v, m = plummer_salpeter(400, 8)
    a, j, p = oracle.force(x, v, m, 1 / 64)
    assert np.all(np.abs((m[:, None] * a).sum(0)) < 1e-14 * np.abs(m[:, None] * a).sum())
    assert np.all(np.abs((m[:, None] * j).sum(0)) < 1e-14 * np.abs(m[:, None] * j).sum())
    # potential energy counted from both ends agrees: sum_i m_i phi_i = 2 U
    u = 0.0
    for i in range(len(m)):
        r = np.sqrt(((x[i + 1:] - x[i]) ** 2).sum(1) + (1 / 64) ** 2)
        u -= (m[i] * m[i + 1:] / r).sum()
    assert (m * p).sum() == pytest.approx(2 * u, rel=1e-13)


def test_momentum_and_angular_momentum_rates_vanish():
    x, v, m = plummer(512, 7)
    a, j, _ = oracle.force(x, v, m, 1 / 64)
    scale = np.abs(m[:, None] * a).sum()
    assert np.all(np.abs((m[:, None] * a).sum(0)) < 1e-14 * scale)
    assert np.all(np.abs((m[:, None] * j).sum(0)) < 1e-14 * np.abs(m[:, None] * j).sum())
    # internal central forces exert no net torque
    tq = (m[:, None] * np.cross(x, a)).sum(0)
    assert np.all(np.abs(tq) < 1e-14 * np.abs(m[:, None] * np.cross(x, a)).sum())


def test_acceleration_is_minus_gradient_of_potential():
    x, v, m = plummer(64, 11)
    eps = 0.05
    a, _, _ = oracle.force(x, v, m, eps, i_list=[5])
    h = 1e-5
    g = np.empty(3)
    for c in range(3):
        xp = x.copy(); xp[5, c] += h
        xm = x.copy(); xm[5, c] -= h
        _, _, pp = oracle.force(xp, v, m, eps, i_list=[5])
        _, _, pm = oracle.force(xm, v, m, eps, i_list=[5])
        g[c] = (pp[0] - pm[0]) / (2 * h)
    np.testing.assert_allclose(a[0], -g, rtol=1e-7, atol=1e-9)


def test_jerk_is_time_derivative_of_acceleration():
    # along straight-line motion x(t) = x + v t, jerk = da/dt (central difference)
    x, v, m = plummer(64, 12)
    eps = 0.05
    a0, j0, _ = oracle.force(x, v, m, eps)

    def fd(h):
        ap, _, _ = oracle.force(x + h * v, v, m, eps)
        am, _, _ = oracle.force(x - h * v, v, m, eps)
        return (ap - am) / (2 * h)

    f1, f2 = fd(2e-3), fd(1e-3)
    e1 = np.abs(f1 - j0).max() / np.abs(j0).max()
    e2 = np.abs(f2 - j0).max() / np.abs(j0).max()
    assert 3.5 < e1 / e2 < 4.5            # O(h^2) convergence onto the jerk
    rich = (4 * f2 - f1) / 3              # Richardson: O(h^4)
    assert np.abs(rich - j0).max() / np.abs(j0).max() < 1e-5


def test_force_scaling_laws():
    # unsoftened gravity: a(lambda x) = a(x)/lambda^2, pot(lambda x) = pot/lambda;
    # linear in the masses of the sources.
    x, v, m = plummer(50, 13)
    a, j, p = oracle.force(x, v, m, 0.0)
    a2, j2, p2 = oracle.force(3.0 * x, v, m, 0.0)
    np.testing.assert_allclose(a2, a / 9.0, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(p2, p / 3.0, rtol=1e-13)
    a3, j3, p3 = oracle.force(x, v, 2.5 * m, 0.0)
    np.testing.assert_allclose(a3, 2.5 * a, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(j3, 2.5 * j, rtol=1e-14, atol=1e-14)


def test_force_sum_order_independent_to_rounding():
    x, v, m = plummer(300, 14)
    perm = np.random.Generator(np.random.PCG64(3)).permutation(300)
    a, j, p = oracle.force(x, v, m, 0.01)
    ap, jp, pp = oracle.force(x[perm], v[perm], m[perm], 0.01)
    inv = np.argsort(perm)
    np.testing.assert_allclose(ap[inv], a, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(jp[inv], j, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(pp[inv], p, rtol=1e-13)


def test_i_list_subset_and_duplicates():
    x, v, m = plummer(200, 15)
    a, j, p = oracle.force(x, v, m, 0.01)
    il = [17, 3, 17, 199, 0]
    a2, j2, p2 = oracle.force(x, v, m, 0.01, i_list=il)
    np.testing.assert_array_equal(a2, a[il])
    np.testing.assert_array_equal(j2, j[il])
    np.testing.assert_array_equal(p2, p[il])


def test_single_particle_feels_nothing():
    a, j, p = oracle.force([[0.3, 0.2, 0.1]], [[1.0, 0.0, 0.0]], [1.0], 0.01)
    assert np.all(a == 0) and np.all(j == 0) and p[0] == 0.0


# --- predictor (section 4.1, step 3) ----------------------------------------

def test_predictor_exact_for_cubic_motion():
    rng = np.random.Generator(np.random.PCG64(5))
    n = 20
    x, v, a, jk = (rng.standard_normal((n, 3)) for _ in range(4))
    t_i = rng.uniform(0, 1, n)
    t = 1.25
    xp, vp = oracle.predict(t, t_i, x, v, a, jk)
    for i in range(n):
        for c in range(3):
            poly = np.polynomial.Polynomial([x[i, c], v[i, c], a[i, c] / 2, jk[i, c] / 6])
            assert xp[i, c] == pytest.approx(poly(t - t_i[i]), rel=1e-13, abs=1e-13)
            assert vp[i, c] == pytest.approx(poly.deriv()(t - t_i[i]), rel=1e-13, abs=1e-13)


def test_predictor_fourth_order_on_circle():
    om = 1.3
    errs = []
    for d in (0.1, 0.05, 0.025):
        x = np.array([[1.0, 0, 0]])
        v = np.array([[0, om, 0]])
        a = np.array([[-om ** 2, 0, 0]])
        jk = np.array([[0, -om ** 3, 0]])
        xp, _ = oracle.predict(d, [0.0], x, v, a, jk)
        errs.append(np.linalg.norm(xp[0] - _rot(om * d)))
    assert 14 < errs[0] / errs[1] < 18 and 14 < errs[1] / errs[2] < 18


# --- corrector (section 4.1, step 5) -----------------------------------------

def test_corrector_exact_for_quintic_trajectory():
    # For x(t) a quintic, a(t) is cubic; the corrector recovers x, v at the end
    # of the step and the 2nd/3rd derivatives of a exactly (algebraic identity).
    rng = np.random.Generator(np.random.PCG64(6))
    for dt in (0.5, 2.0 ** -7):
        coef = rng.standard_normal((3, 6))  # x(t) = sum c_k t^k
        P = [np.polynomial.Polynomial(coef[c]) for c in range(3)]
        ev = lambda k, t: np.array([P[c].deriv(k)(t) if k else P[c](t) for c in range(3)])
        x0, v0, a0, j0 = ev(0, 0.0), ev(1, 0.0), ev(2, 0.0), ev(3, 0.0)
        a1, j1 = ev(2, dt), ev(3, dt)
        xp = x0 + v0 * dt + a0 * dt ** 2 / 2 + j0 * dt ** 3 / 6
        vp = v0 + a0 * dt + j0 * dt ** 2 / 2
        x1, v1, a2e, a3 = oracle.correct_one(dt, xp, vp, a0, j0, a1, j1)
        tol = 1e-12 * max(1.0, dt ** -3)
        np.testing.assert_allclose(x1, ev(0, dt), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(v1, ev(1, dt), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(a2e, ev(4, dt), rtol=1e-9, atol=tol)
        np.testing.assert_allclose(a3, ev(5, 0.0), rtol=1e-9, atol=tol)


# --- time-step criterion and block quantisation (section 2) ----------------

def test_aarseth_step_on_circular_motion():
    # uniform circular motion: |a|=r w^2, |j|=r w^3, |a2|=r w^4, |a3|=r w^5
    # at mutually orthogonal/antiparallel phases, giving dt = sqrt(eta)/w.
    r, w, eta = 0.7, 2.2, 0.01
    a = -r * w ** 2 * _rot(0.0)
    j = -r * w ** 3 * _rot(math.pi / 2)
    a2 = r * w ** 4 * _rot(0.0)
    a3 = r * w ** 5 * _rot(math.pi / 2)
    assert oracle.aarseth_dt(a, j, a2, a3, eta) == pytest.approx(math.sqrt(eta) / w, rel=1e-14)
    prm = oracle.params(0.0, eta=eta, eta_init=0.02, dt_min_log2=-20, dt_max_log2=-1)
    dt, cl = oracle.initial_dt(a, j, prm)
    want = 0.02 / w
    assert dt <= want < 2 * dt and not cl
    assert math.log2(dt) == int(math.log2(dt))


def test_block_dt_rules():
    prm = oracle.params(0.0, dt_min_log2=-10, dt_max_log2=-3)
    # halve until below the request
    assert oracle.block_dt(2 ** -4, 0.5, 0.01, prm) == (2 ** -7, False)
    # clamp at dt_min and flag it
    assert oracle.block_dt(2 ** -4, 0.5, 1e-9, prm) == (2 ** -10, True)
    # double only when the new time is a multiple of the doubled step
    assert oracle.block_dt(2 ** -6, 3 * 2 ** -6, 1.0, prm) == (2 ** -6, False)
    assert oracle.block_dt(2 ** -6, 4 * 2 ** -6, 1.0, prm) == (2 ** -5, False)
    # at most one doubling per step, never above dt_max
    assert oracle.block_dt(2 ** -3, 1.0, 10.0, prm) == (2 ** -3, False)
    # keep when the request lies in [dt, 2 dt)
    assert oracle.block_dt(2 ** -6, 4 * 2 ** -6, 1.5 * 2 ** -6, prm) == (2 ** -6, False)
    # no constraint (+inf) behaves like a large request
    assert oracle.block_dt(2 ** -6, 4 * 2 ** -6, math.inf, prm) == (2 ** -5, False)


# --- whole integrator (section 4.1, steps 1-6) ------------------------------

def _circular_binary(eps, om_sign=1.0):
    m = np.array([0.5, 0.5])
    om = (1.0 / (1.0 + eps * eps) ** 1.5) ** 0.5
    x = np.array([[-0.5, 0, 0], [0.5, 0, 0]])
    v = om_sign * np.array([[0, -0.5 * om, 0], [0, 0.5 * om, 0]])
    return x, v, m, om


@pytest.mark.parametrize("eps", [0.0, 0.2])
def test_softened_circular_orbit_fourth_order(eps):
    # relative orbit of radius 1 with angular speed w^2 = M/(d^2+eps^2)^{3/2}
    T = 2.0
    errs = []
    for k in (5, 6, 7):
        x, v, m, om = _circular_binary(eps)
        s = oracle.System(x, v, m, oracle.params(eps, dt_min_log2=-k, dt_max_log2=-k))
        steps, upd = s.run(T)
        assert steps == int(T * 2 ** k) and upd == 2 * steps
        assert np.all(s.t_i == T)
        want = 0.5 * _rot(om * T)
        errs.append(np.linalg.norm(s.x[1] - want))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


def _kepler_state(e, t):
    # relative orbit, semi-major axis 1, total mass 1, pericentre at t=0
    M = t
    E = M
    for _ in range(60):
        E = E - (E - e * math.sin(E) - M) / (1 - e * math.cos(E))
    r = np.array([math.cos(E) - e, math.sqrt(1 - e * e) * math.sin(E), 0.0])
    edot = 1.0 / (1 - e * math.cos(E))
    w = np.array([-math.sin(E) * edot, math.sqrt(1 - e * e) * math.cos(E) * edot, 0.0])
    return r, w


def test_kepler_eccentric_orbit_fourth_order():
    e, T = 0.5, 3.0
    r0, w0 = _kepler_state(e, 0.0)
    rT, _ = _kepler_state(e, T)
    errs = []
    for k in (6, 7, 8):
        m = np.array([0.3, 0.7])
        x = np.array([-0.7 * r0, 0.3 * r0])
        v = np.array([-0.7 * w0, 0.3 * w0])
        s = oracle.System(x, v, m, oracle.params(0.0, dt_min_log2=-k, dt_max_log2=-k))
        s.run(T)
        errs.append(np.linalg.norm((s.x[1] - s.x[0]) - rT))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


def test_block_steps_on_kepler_orbit_conserve_energy_and_keep_invariants():
    e = 0.5
    r0, w0 = _kepler_state(e, 0.0)
    m = np.array([0.5, 0.5])
    x = np.array([-0.5 * r0, 0.5 * r0])
    v = np.array([-0.5 * w0, 0.5 * w0])
    prm = oracle.params(0.0, eta=0.01, eta_init=0.01, dt_min_log2=-20, dt_max_log2=-3)
    s = oracle.System(x, v, m, prm)
    E0 = sum(s.energy())
    s.run(2 * math.pi)  # one period (the loop stops at the last block time <= 2 pi)
    assert abs(sum(s.energy()) - E0) / abs(E0) < 1e-6
    rT, _ = _kepler_state(e, s.t_i[0])
    assert np.linalg.norm((s.x[1] - s.x[0]) - rT) < 1e-4


def _check_block_invariants(s, prm):
    lv = np.log2(s.dt_i)
    assert np.all(lv == np.round(lv))
    assert np.all(s.dt_i >= prm.dt_min) and np.all(s.dt_i <= prm.dt_max)
    assert np.all(np.fmod(s.t_i, s.dt_i) == 0.0)


def test_block_steps_plummer_invariants_and_energy():
    x, v, m = plummer(256, 21)
    prm = oracle.params(1 / 64, eta=0.01, eta_init=0.01, dt_min_log2=-20, dt_max_log2=-3)
    s = oracle.System(x, v, m, prm)
    E0 = sum(s.energy())
    _check_block_invariants(s, prm)
    t_prev = 0.0
    for _ in range(200):
        t, act, pot = s.step()
        assert t > t_prev
        t_prev = t
        # the block is exactly the set of particles due at t
        assert np.all(s.t_i[act] == t)
        _check_block_invariants(s, prm)
        nxt = s.t_i + s.dt_i
        assert np.all(nxt > t)
    s.run(0.25)
    assert np.all(s.t_i == 0.25)  # 2^-3 divides 0.25: everyone synchronised
    assert abs(sum(s.energy()) - E0) / abs(E0) < 1e-5


def test_shared_step_plummer_energy_and_momentum_config1():
    # Plummer N=1024, eps=1/256, shared dt=1/256 for 32 steps
    x, v, m = plummer(1024, 1001)
    prm = oracle.params(1 / 256, dt_min_log2=-8, dt_max_log2=-8)
    s = oracle.System(x, v, m, prm)
    E0 = sum(s.energy())
    P0 = (m[:, None] * s.v).sum(0)
    steps, upd = s.run(32 / 256)
    assert steps == 32 and upd == 32 * 1024
    assert abs(sum(s.energy()) - E0) / abs(E0) < 1e-5
    assert np.all(np.abs((m[:, None] * s.v).sum(0) - P0) < 1e-13)


def test_potential_energy_matches_half_sum_of_potentials():
    x, v, m = plummer(400, 22)
    _, _, p = oracle.force(x, v, m, 0.01)
    ek, ep = oracle.energy(x, v, m, 0.01)
    assert ep == pytest.approx(0.5 * (m * p).sum(), rel=1e-13)
    assert ek == pytest.approx(0.5 * (m * (v * v).sum(1)).sum(), rel=1e-14)
