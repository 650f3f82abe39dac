"""The section 4.1 performance model (paper_0709_4552_amd.perfmodel): hand-
computed cases, the paper's own Table 3 constants, and the t0 fit."""
import math

import pytest

from paper_0709_4552_amd import perfmodel as pm


def test_single_step_by_hand():
    # N = 1000, n = 10, tau_pred = 1e-9, tau_force = 2e-12, tau_corr = 5e-8, t0 = 3e-6:
    # 3e-6 + 1e-6 + 2e-8 + 5e-7 = 4.52e-6 s
    t = pm.t_step(1000, 10, 1e-9, 2e-12, 5e-8, 3e-6)
    assert t == pytest.approx(4.52e-6, rel=1e-15)
    parts = pm.t_step_parts(1000, 10, 1e-9, 2e-12, 5e-8)
    assert parts == pytest.approx({"t_pred": 1e-6, "t_force": 2e-8, "t_corr": 5e-7}, rel=1e-15)


def test_sum_over_steps_by_hand():
    # three steps of 1, 2 and 4 particles out of N = 8, t0 = 0:
    # pred 3*8*1e-9, force (1+2+4)*8*1e-10, corr 7*1e-8
    T = pm.T_integrate(8, [1, 2, 4], 1e-9, 1e-10, 1e-8)
    assert T == pytest.approx(24e-9 + 56e-10 + 7e-8, rel=1e-15)
    # with t0 every step costs t0 more
    assert pm.T_integrate(8, [1, 2, 4], 1e-9, 1e-10, 1e-8, 1e-6) == pytest.approx(T + 3e-6,
                                                                                  rel=1e-15)
    # equal sizes: the mean form is the same sum
    assert pm.T_integrate(8, [3, 3, 3], 1e-9, 1e-10, 1e-8, 1e-6) == pytest.approx(
        pm.T_integrate_mean(8, 3, 3, 1e-9, 1e-10, 1e-8, 1e-6), rel=1e-15)


def test_block_size_of_section_3_2():
    assert pm.block_size_paper(1) == pytest.approx(0.20)
    # 0.20 * 32768^0.81 = 0.20 * 2^(15*0.81)
    assert pm.block_size_paper(32768) == pytest.approx(0.20 * 2.0 ** 12.15, rel=1e-12)
    assert pm.block_size_paper(196608) == pytest.approx(0.20 * 196608 ** 0.81, rel=1e-12)


def test_paper_table3_constants_in_the_section_4_1_equation():
    # Table 3, host "yoda": tau_pred 0.131 us, tau_force 0.110 us, tau_corr 1.29 us,
    # measured with N = 32768.  With n = 0.20 N^0.81 (about 910) one step takes
    # 0.131e-6*32768 + 0.110e-6*910*32768 + 1.29e-6*910 = 4.29 ms + 3.28 s + 1.17 ms,
    # the force calculation being almost all of it (section 3: the single-PC time
    # is dominated by the force calculation).
    _, tp, tf, tc = pm.PAPER_TABLE3["yoda"]
    N = 32768
    n = pm.block_size_paper(N)
    parts = pm.t_step_parts(N, n, tp, tf, tc)
    assert parts["t_pred"] == pytest.approx(0.131e-6 * 32768, rel=1e-12)
    assert parts["t_force"] == pytest.approx(0.110e-6 * n * 32768, rel=1e-12)
    assert parts["t_force"] == pytest.approx(3.28, rel=2e-3)
    assert parts["t_force"] / sum(parts.values()) > 0.99
    # every host: force dominates, and the hosts order by tau_force
    for host, (_, tp, tf, tc) in pm.PAPER_TABLE3.items():
        p = pm.t_step_parts(N, n, tp, tf, tc)
        assert p["t_force"] > 100 * (p["t_pred"] + p["t_corr"]), host
    assert pm.paper_host_rate("yoda") == pytest.approx(1 / 0.110e-6)
    # GRAPE-6Af (section 4.4) against the fastest host's CPU force loop
    assert pm.TAU_GFORCE < min(v[2] for v in pm.PAPER_TABLE3.values()) / 200


def test_tau_force_table_interpolates_log_log():
    tau = pm.tau_force_table({1: 1e-9, 100: 1e-11, 10000: 1e-12})
    assert tau(1) == pytest.approx(1e-9, rel=1e-12)
    assert tau(100) == pytest.approx(1e-11, rel=1e-12)
    assert tau(10) == pytest.approx(1e-10, rel=1e-12)  # geometric midpoint
    assert tau(1000) == pytest.approx(math.sqrt(1e-11 * 1e-12), rel=1e-12)
    assert tau(1e6) == pytest.approx(1e-12, rel=1e-12)  # held beyond the range
    assert tau(0.5) == pytest.approx(1e-9, rel=1e-12)
    with pytest.raises(ValueError):
        pm.tau_force_table({0: 1.0})
    # a callable tau_force enters t_step as tau(n)
    assert pm.t_step(1000, 10, 0.0, tau, 0.0) == pytest.approx(1e-10 * 10 * 1000, rel=1e-12)


def test_t0_fit_recovers_the_fixed_cost():
    sizes = [1, 5, 64, 700, 3]
    tau = pm.tau_force_table({1: 5e-11, 1024: 8e-13})
    T = pm.T_integrate(4096, sizes, 2e-12, tau, 3e-10, t0=7.5e-6)
    assert pm.fit_t0(T, 4096, sizes, 2e-12, tau, 3e-10) == pytest.approx(7.5e-6, rel=1e-9)
    with pytest.raises(ValueError):
        pm.fit_t0(1.0, 4096, [], 2e-12, tau, 3e-10)
