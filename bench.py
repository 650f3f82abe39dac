#!/usr/bin/env python3
"""Benchmark of the direct N-body hot path on one MI355X.

Workload (the headline configuration): Plummer sphere, N = 196608 equal
masses, eps = 1/1024, Aarseth eta = 0.01, block steps in [2^-20, 2^-3],
mixed precision (FP32 pairwise terms, FP64 coordinates and accumulation).
One step = one full force sweep (acceleration, jerk and potential of all N
particles from all N at t = 0) followed by block steps (select, predict,
force, correct) up to t = 1/8, starting from the same post-start-up state.
The value is whole-step throughput in pairwise acc+jerk interactions per
second (full sweep n*N plus every block step's n*N), with all state resident
on the GPU.  The FP64 form of the same workload, the full-sweep kernel
against the FP32 vector roofline, the oracle's CPU rate on a bounded sample,
and the per-particle force error against the oracle are reported beside it.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import statistics
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "acc+jerk interactions/s, mixed vs FP64, N=196608, rel force err ≤1e-6"
FLOPS_PER_INTERACTION = 60          # convention for acc+jerk
PEAK_FP32 = 157.3e12                # MI355X FP32 vector, published
PEAK_FP64 = 78.6e12                 # MI355X FP64 vector, published
N_DEFAULT = 196608
EPS = 1.0 / 1024
T_END = 1.0 / 8
SEED = 1003
# HBM traffic of the full-sweep kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs, scaled by the
# same counters on an elementwise kernel of known size; valid only for the kernel source it was
# measured on (checked by hash, else "traffic" is reported as null).
SWEEP_TRAFFIC = {"force_source_sha256_prefix": "953190131d06b8a2", "read_bytes": 215.2e6,
                 "write_bytes": 71.4e6}


# Autotuner probe sizes, one per block-size class (n >= 2048, >= 256, >= 32,
# >= 4, below), each inside the range of block sizes the class serves.
CLASS_PROBES = (16384, 1024, 128, 16, 1)


def sweep_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_0709_4552_amd", "csrc", "kernels_force.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if h != SWEEP_TRAFFIC["force_source_sha256_prefix"]:
        return None
    return SWEEP_TRAFFIC["read_bytes"] + SWEEP_TRAFFIC["write_bytes"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


class Run:
    """One precision's system plus a snapshot of its post-start-up state."""

    def __init__(self, x, v, m, precision, torch):
        from paper_0709_4552_amd import NBody
        self.torch = torch
        self.g = NBody(x, v, m, EPS, eta=0.01, eta_init=0.01, dt_min_log2=-20, dt_max_log2=-3,
                       precision=precision)
        self.g.init()
        g = self.g
        # autotune every block-size class (outside any timed region), each at a
        # block size in the middle of the range it serves in block steps
        self.tuning = []
        for n_probe in sorted({min(g.n, p) for p in CLASS_PROBES}, reverse=True):
            t, ms = g.autotune(n_probe)
            t["n_probe"] = n_probe
            t["ms"] = ms
            self.tuning.append(t)
            log(f"autotune n={n_probe}: class {t['size_class']} i_per_lane={t['i_per_lane']} "
                f"j_lanes={t['j_lanes']} {ms:.3f} ms")
        self.snap = [t.clone() for t in (g.pos, g.vel, g.acc, g.jerk, g.t_tick, g.level)]
        self.all = torch.arange(g.n, dtype=torch.int32, device=g.dev)
        self.stream = g.stream
        self.ev0 = torch.cuda.Event(enable_timing=True)
        self.ev1 = torch.cuda.Event(enable_timing=True)
        self.sweep_ms = []
        self.step_ms = []
        self.inter = []

    def restore(self):
        g = self.g
        for dst, src in zip((g.pos, g.vel, g.acc, g.jerk, g.t_tick, g.level), self.snap):
            dst.copy_(src)

    def step(self, timed: bool):
        """Full sweep + block steps to T_END; returns interactions done."""
        g, torch = self.g, self.torch
        self.restore()
        torch.cuda.synchronize()
        st0 = g.stats()
        s0 = st0["interactions"]
        self._steps0 = st0["block_steps"]
        t0 = time.perf_counter()
        with torch.cuda.stream(self.stream):
            g.predict(0.0)
            self.ev0.record(self.stream)
            acc, jerk, pot = g.force_jerk(self.all, 0.0, want_pot=True)
            self.ev1.record(self.stream)
        g.run_until(T_END)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = g.stats()
        inter = float(g.n) * g.n + (st["interactions"] - s0)
        self.block_steps = st["block_steps"] - self._steps0 if hasattr(self, "_steps0") else None
        if timed:
            self.sweep_ms.append(self.ev0.elapsed_time(self.ev1))
            self.step_ms.append((t1 - t0) * 1e3)
            self.inter.append(inter)
        self.last_sweep = (acc, jerk, pot)
        return inter

    def sweep_without_potential_ms(self, reps: int = 2) -> float:
        """Time of the full sweep returning acceleration and jerk only (the
        kernel instance the block steps use)."""
        g, torch = self.g, self.torch
        self.restore()
        with torch.cuda.stream(self.stream):
            g.predict(0.0)
            g.force_jerk(self.all, 0.0, want_pot=False)
            self.ev0.record(self.stream)
            for _ in range(reps):
                g.force_jerk(self.all, 0.0, want_pot=False)
            self.ev1.record(self.stream)
        torch.cuda.synchronize()
        return self.ev0.elapsed_time(self.ev1) / reps

    def host_xv(self):
        """Positions and velocities (N, 3) of the state on the GPU."""
        g = self.g
        return g.pos.T.cpu().numpy(), g.vel.T.cpu().numpy()


def cpu_baseline(x, v, m, sweep_acc, budget_s: float):
    """Oracle force on every particle against all N (CPU, all threads) when a
    probe of 2048 particles says that fits the budget, else on a bounded
    sample; and the GPU full-sweep error on the particles checked."""
    import numpy as np

    import oracle
    n = x.shape[0]
    rng = np.random.Generator(np.random.PCG64(7))
    probe = rng.integers(0, n, min(n, 2048))
    t0 = time.perf_counter()
    oracle.force(x, v, m, EPS, probe)
    dt = time.perf_counter() - t0
    per_i = dt / probe.size
    k = int(min(n, max(256, budget_s / max(per_i, 1e-9))))
    r = np.linalg.norm(x, axis=1)
    if k >= n:
        sample = np.arange(n)
        what = "all"
    else:
        # the most central particles (hardest cancellation) + random ones
        sample = np.unique(np.concatenate([np.argsort(r)[:min(512, k // 4)],
                                           rng.integers(0, n, k)]))[:k]
        what = f"the {min(512, k // 4)} most central + random"
    t0 = time.perf_counter()
    ra, rj, rp = oracle.force(x, v, m, EPS, sample)
    dt = time.perf_counter() - t0
    rate = sample.size * float(n) / dt
    cores = oracle.threads()
    # the same oracle on one thread, over the first 64 particles of the sample
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.force(x, v, m, EPS, sample[:64])
    rate1 = 64.0 * n / (time.perf_counter() - t0)
    oracle.set_threads(cores)
    out = {"value": rate, "unit": "interactions/s", "cores": cores, "kind": "oracle",
           "sample": f"oracle acc+jerk+pot of {sample.size} particles ({what}) against all "
                     f"N={n}, FP64, {dt:.1f} s",
           "value_1_thread": rate1}
    errs = {}
    for name, (a, j) in sweep_acc.items():
        ea = np.linalg.norm(a[sample] - ra, axis=1) / np.linalg.norm(ra, axis=1)
        ej = np.linalg.norm(j[sample] - rj, axis=1) / np.linalg.norm(rj, axis=1)
        errs[name] = {"max_rel_acc_err": float(ea.max()), "p999_rel_acc_err":
                      float(np.quantile(ea, 0.999)), "median_rel_acc_err": float(np.median(ea)),
                      "max_rel_jerk_err": float(ej.max()),
                      "p999_rel_jerk_err": float(np.quantile(ej, 0.999)),
                      "particles": int(sample.size)}
    return out, errs


def blocksize_sweep(torch, n_big: int, cpu_check: bool):
    """Force-only rates at N = n_big (eps = 1/4096, mixed) for block sizes
    1, 64, 4096, 65536 and N; fixed-seed samples of i (seed 1006)."""
    import numpy as np

    from nbody_inputs import plummer
    from paper_0709_4552_amd import NBODY_PREC_MIXED, NBody
    x, v, m = plummer(n_big, 1005)
    g = NBody(x, v, m, 1.0 / 4096, dt_min_log2=-20, dt_max_log2=-3, precision=NBODY_PREC_MIXED)
    g.init()
    tuning = []
    for n_probe in (65536, 4096, 128, 16, 1):
        t, ms = g.autotune(min(n_probe, n_big))
        t["n_probe"], t["ms"] = min(n_probe, n_big), ms
        tuning.append(t)
    g.predict(0.0)
    rng = np.random.Generator(np.random.PCG64(1006))
    out = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    central = np.argsort(np.linalg.norm(x, axis=1))[:64].astype(np.int32)
    for n in (1, 64, "central64", 4096, 65536, n_big):
        label = n
        if n == "central64":
            il, n = central, 64
        else:
            n = min(n, n_big)
            il = np.arange(n_big, dtype=np.int32) if n == n_big else \
                rng.choice(n_big, n, replace=False).astype(np.int32)
        ilt = torch.as_tensor(il, device=g.dev)
        # outputs allocated once, so the host's side of a call stays short of
        # the GPU's even for one-particle blocks
        res = (torch.empty((3, n), dtype=torch.float64, device=g.dev),
               torch.empty((3, n), dtype=torch.float64, device=g.dev), None)
        reps = 20 if n <= 64 else (3 if n < n_big else 1)
        with torch.cuda.stream(g.stream):
            for _ in range(3 if n < n_big else 1):  # warm-up calls, untimed
                g.force_jerk(ilt, 0.0, want_pot=False, out=res)
            ev0.record(g.stream)
            for _ in range(reps):
                acc, jerk, _ = g.force_jerk(ilt, 0.0, want_pot=False, out=res)
            ev1.record(g.stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        rate = float(n) * n_big / (ms * 1e-3)
        rec = {"n_active": n, "i_list": "the 64 most central" if label == "central64" else
               ("all" if n == n_big else "random (seed 1006)"),
               "ms": ms, "interactions_per_s": rate,
               "frac_fp32_peak": FLOPS_PER_INTERACTION * rate / PEAK_FP32,
               "jbuffer_GBps": 40.0 * n_big / (ms * 1e-3) / 1e9}
        if cpu_check and n <= 4096:
            import oracle
            k = min(n, 512)
            ra, _, _ = oracle.force(x, v, m, 1.0 / 4096, il[:k])
            a = acc.T[:k].cpu().numpy()
            rec["max_rel_acc_err"] = float((np.linalg.norm(a - ra, axis=1) /
                                            np.linalg.norm(ra, axis=1)).max())
            rec["checked_particles"] = k
        out.append(rec)
        log(f"N={n_big} n={label}: {ms:.3f} ms {rate:.3e} int/s")
    g.close()
    return {"workload": f"plummer_N{n_big}_eps1/4096_mixed_force_only", "autotuned_shapes": tuning,
            "points": out}


def ensemble_bench(torch, n_clusters: int, t_short: float, t_full: float, per_cluster: bool):
    """256 independent clusters (sizes log-uniform in [256, 8192], seed 1004),
    eps = 1/256, eta = 0.01: one graph-replayed launch sequence per ensemble
    step, against the same clusters run one after another."""
    import numpy as np

    import oracle
    from nbody_inputs import ensemble
    from paper_0709_4552_amd import NBODY_PREC_MIXED, NBody
    x, v, m, offs = ensemble(n_clusters, 1004)
    eps = 1.0 / 256
    kw = dict(eta=0.01, eta_init=0.01, dt_min_log2=-20, dt_max_log2=-3, precision=NBODY_PREC_MIXED)
    g = NBody(x, v, m, eps, cluster_offset=offs, **kw)
    g.init()
    tuning = [g.autotune(n)[0] for n in (2048, 512, 64, 8, 1)]
    snap = [t.clone() for t in (g.pos, g.vel, g.acc, g.jerk, g.t_tick, g.level)]
    torch.cuda.synchronize()
    s0 = g.stats()
    t0 = time.perf_counter()
    steps = g.run_until(t_short)
    torch.cuda.synchronize()
    t_ens = time.perf_counter() - t0
    s1 = g.stats()
    inter_short = s1["interactions"] - s0["interactions"]
    res = {"workload": f"ensemble_{n_clusters}_clusters_N256-8192_eps1/256_mixed",
           "n_total": int(offs[-1]), "clusters": n_clusters, "autotuned_shapes": tuning,
           "short": {"t_end": t_short, "ensemble_s": t_ens, "ensemble_steps": steps,
                     "interactions": inter_short,
                     "ensemble_interactions_per_s": inter_short / t_ens}}
    log(f"ensemble to t={t_short}: {t_ens:.3f} s, {inter_short / t_ens:.3e} int/s")
    if per_cluster:
        tot = 0.0
        inter_pc = 0.0
        for k in range(n_clusters):
            sl = slice(int(offs[k]), int(offs[k + 1]))
            gk = NBody(x[sl], v[sl], m[sl], eps, **kw)
            gk.init()
            for (n_probe, t) in zip((2048, 512, 64, 8, 1), tuning):
                gk.set_tuning(t["i_per_lane"], t["j_lanes"], size_class=t["size_class"])
            torch.cuda.synchronize()
            a0 = gk.stats()["interactions"]
            t0 = time.perf_counter()
            gk.run_until(t_short)
            torch.cuda.synchronize()
            tot += time.perf_counter() - t0
            inter_pc += gk.stats()["interactions"] - a0
            gk.close()
        res["short"].update({"per_cluster_s": tot, "per_cluster_interactions_per_s": inter_pc / tot,
                             "speedup_vs_per_cluster": tot / t_ens})
        log(f"per-cluster to t={t_short}: {tot:.3f} s ({tot / t_ens:.1f}x slower)")
    if t_full:
        for dst, src in zip((g.pos, g.vel, g.acc, g.jerk, g.t_tick, g.level), snap):
            dst.copy_(src)
        torch.cuda.synchronize()
        s0 = g.stats()
        t0 = time.perf_counter()
        steps = g.run_until(t_full)
        torch.cuda.synchronize()
        t_f = time.perf_counter() - t0
        s1 = g.stats()
        xg, vg, _, _, tg, _ = g.host_state()
        dE = []
        for k in range(n_clusters):
            sl = slice(int(offs[k]), int(offs[k + 1]))
            E0 = sum(oracle.energy(x[sl], v[sl], m[sl], eps))
            E1 = sum(oracle.energy(xg[sl], vg[sl], m[sl], eps))
            dE.append(abs(E1 - E0) / abs(E0))
        # oracle integration of the worst cluster and up to 7 smaller ones
        sizes = np.diff(offs)
        worst = int(np.argmax(dE))
        cand = [k for k in np.argsort(sizes) if sizes[k] <= 2048 and k != worst]
        picks = [worst] + [int(k) for k in cand[::max(1, len(cand) // 7)][:7]]
        orc = []
        prm = oracle.params(eps, eta=0.01, eta_init=0.01, dt_min_log2=-20, dt_max_log2=-3)
        for k in picks:
            sl = slice(int(offs[k]), int(offs[k + 1]))
            if sizes[k] > 4096:
                continue
            ref = oracle.System(x[sl], v[sl], m[sl], prm)
            E0 = sum(ref.energy())
            ref.run(t_full)
            E1 = sum(ref.energy())
            orc.append({"cluster": k, "n": int(sizes[k]), "gpu_dE_over_E": dE[k],
                        "oracle_dE_over_E": abs(E1 - E0) / abs(E0)})
            log(f"cluster {k} (N={sizes[k]}): |dE/E| gpu {dE[k]:.2e} oracle {orc[-1]['oracle_dE_over_E']:.2e}")
        res["oracle_clusters"] = orc
        res["full"] = {"t_end": t_full, "ensemble_s": t_f, "ensemble_steps": steps,
                       "interactions": s1["interactions"] - s0["interactions"],
                       "interactions_per_s": (s1["interactions"] - s0["interactions"]) / t_f,
                       "all_at_t_end": bool(np.all(tg == t_full)),
                       "max_abs_dE_over_E": float(max(dE)), "median_abs_dE_over_E":
                       float(np.median(dE))}
        log(f"ensemble to t={t_full}: {t_f:.3f} s, max |dE/E| {max(dE):.2e}")
    g.close()
    return res


def fused_bench(system, mask: int, reps: int):
    """Block steps to T_END with in-kernel prediction for the classes in
    `mask` against the prediction pass, alternating, from the same state."""
    g, torch = system.g, system.torch
    times = {0: [], mask: []}
    for _ in range(reps):
        for mk in (0, mask):
            g.set_fused_predict(mk)
            system.restore()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.run_until(T_END)
            torch.cuda.synchronize()
            times[mk].append((time.perf_counter() - t0) * 1e3)
    g.set_fused_predict(0)
    out = {"workload": f"plummer_N{g.n}_blocksteps_to_t{T_END}", "fused_class_mask": mask,
           "ms_prediction_pass": times[0], "ms_in_kernel": times[mask],
           "ratio_in_kernel_over_pass": min(times[mask]) / min(times[0])}
    log(f"fused prediction mask {mask}: {out}")
    return out


def salpeter_bench(torch, n: int, t_end: float, cpu_check: bool):
    """Unequal masses: a Plummer sphere with Salpeter masses (0.1-100, seed
    1017), eps = 1/1024, mixed form (its per-pair near-field variant): the full
    sweep rate, its accuracy on a sample (the most massive, the most central and
    random particles), and block steps to t_end."""
    import numpy as np

    from nbody_inputs import plummer_salpeter
    from paper_0709_4552_amd import NBODY_PREC_MIXED, NBody
    x, v, m = plummer_salpeter(n, 1017)
    eps = 1.0 / 1024
    g = NBody(x, v, m, eps, eta=0.01, eta_init=0.01, dt_min_log2=-20, dt_max_log2=-3,
              precision=NBODY_PREC_MIXED)
    g.init()
    for n_probe in CLASS_PROBES:
        g.autotune(min(n_probe, n))
    fields = (g.pos, g.vel, g.acc, g.jerk, g.t_tick, g.level)
    snap = [t.clone() for t in fields]
    g.predict(0.0)
    il = torch.arange(n, dtype=torch.int32, device=g.dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(g.stream):
        g.force_jerk(il, 0.0, want_pot=False)
        ev0.record(g.stream)
        for _ in range(3):
            acc, _, _ = g.force_jerk(il, 0.0, want_pot=False)
        ev1.record(g.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / 3
    out = {"workload": f"plummer_salpeter0.1-100_N{n}_eps1/1024_mixed", "n": n,
           "mass_ratio_max_min": float(m.max() / m.min()),
           "sweep_ms_acc_jerk": ms, "sweep_interactions_per_s": float(n) * n / (ms * 1e-3)}
    if cpu_check:
        import oracle
        rng = np.random.Generator(np.random.PCG64(1018))
        r = np.linalg.norm(x, axis=1)
        sample = np.unique(np.concatenate([np.argsort(-m)[:256], np.argsort(r)[:256],
                                           rng.integers(0, n, 3584)]))
        ra, _, _ = oracle.force(x, v, m, eps, sample)
        a = acc.T.cpu().numpy()[sample]
        e = np.linalg.norm(a - ra, axis=1) / np.linalg.norm(ra, axis=1)
        out.update({"max_rel_acc_err": float(e.max()), "median_rel_acc_err": float(np.median(e)),
                    "checked_particles": int(sample.size),
                    "checked": "the 256 most massive, the 256 most central, random"})
    for d, s_ in zip(fields, snap):
        d.copy_(s_)
    torch.cuda.synchronize()
    s0 = g.stats()
    t0 = time.perf_counter()
    g.run_until(t_end)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s1 = g.stats()
    inter = s1["interactions"] - s0["interactions"]
    out.update({"t_end": t_end, "block_steps": s1["block_steps"] - s0["block_steps"],
                "steps_s": wall, "steps_interactions_per_s": inter / wall})
    log(f"salpeter N={n}: sweep {ms:.2f} ms, to t={t_end}: {wall:.3f} s "
        f"({inter / wall:.3e} int/s), max err {out.get('max_rel_acc_err', float('nan')):.2e}")
    g.close()
    return out


def perfmodel_bench(torch, n_list, t_end: float):
    """The single-PC performance model of section 4.1 recast for one GPU
    (paper_0709_4552_amd.perfmodel): for every N this measures the run to t_end
    (wall time, steps, updates, the sequence of block sizes), tau_pred,
    tau_force(n) for n = 4^k and tau_corr, and predicts the run time summed over
    the recorded block sizes and with the mean block size.  The per-step fixed
    cost t0 is fitted on the smallest N alone; the other rows are held out."""
    import numpy as np

    from nbody_inputs import plummer
    from paper_0709_4552_amd import NBODY_PREC_MIXED, NBody
    from paper_0709_4552_amd import perfmodel as pm
    eps = 1.0 / 256
    kw = dict(eta=0.01, eta_init=0.01, dt_min_log2=-20, dt_max_log2=-3, precision=NBODY_PREC_MIXED)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def timed(g, fn, reps):
        with torch.cuda.stream(g.stream):
            fn()
            ev0.record(g.stream)
            for _ in range(reps):
                fn()
            ev1.record(g.stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) * 1e-3 / reps

    rows = []
    for idx, n_tot in enumerate(n_list):
        x, v, m = plummer(n_tot, 1100 + idx)
        g = NBody(x, v, m, eps, **kw)
        g.init()
        for n_probe in CLASS_PROBES:
            g.autotune(min(n_probe, n_tot))
        fields = (g.pos, g.vel, g.acc, g.jerk, g.t_tick, g.level)
        snap = [t.clone() for t in fields]

        def restore():
            for d, s_ in zip(fields, snap):
                d.copy_(s_)
            torch.cuda.synchronize()

        g.run_until(1.0 / 64)  # builds the step graph outside the timed run
        restore()
        s0 = g.stats()
        t0 = time.perf_counter()
        g.run_until(t_end)
        torch.cuda.synchronize()
        t_app = time.perf_counter() - t0
        s1 = g.stats()
        steps = s1["block_steps"] - s0["block_steps"]
        updates = s1["updates"] - s0["updates"]
        inter = s1["interactions"] - s0["interactions"]
        # the block sizes of the same run, step by step (same steps: same state)
        restore()
        sizes = []
        while True:
            t, n = g.step_block(True)
            sizes.append(n)
            if t >= t_end:
                break
        sizes = np.asarray(sizes, dtype=np.int64)
        # tau_pred: the predictor pass over all N
        restore()
        tau_pred = timed(g, lambda: g.predict(0.0), 20) / n_tot
        # tau_force(n) at n = 4^k and at n = N (one force call: plan, force, reduction)
        rng = np.random.Generator(np.random.PCG64(1006))
        grid_n = sorted(set([4 ** k for k in range(0, 20) if 4 ** k < n_tot] + [n_tot]))
        tau_f = {}
        for n in grid_n:
            il = torch.as_tensor(rng.choice(n_tot, n, replace=False).astype(np.int32), device=g.dev)
            res = (torch.empty((3, n), dtype=torch.float64, device=g.dev),
                   torch.empty((3, n), dtype=torch.float64, device=g.dev), None)
            reps = max(1, min(50, int(2e10 / (n * n_tot))))
            tau_f[n] = timed(g, lambda: g.force_jerk(il, 0.0, want_pot=False, out=res),
                             reps) / (n * n_tot)
        g.close()
        # tau_corr: every particle due at once in a shared-step copy of the system
        gs = NBody(x, v, m, eps, eta=0.01, eta_init=0.01, dt_min_log2=-8, dt_max_log2=-8,
                   precision=NBODY_PREC_MIXED)
        gs.init()
        everyone = torch.arange(n_tot, dtype=torch.int32, device=gs.dev)
        gs.predict(2.0 ** -8)
        acc, jerk, _ = gs.force_jerk(everyone, 2.0 ** -8, want_pot=False)
        sfields = (gs.pos, gs.vel, gs.acc, gs.jerk, gs.t_tick, gs.level)
        ssnap = [t.clone() for t in sfields]
        corr = []
        for _ in range(3):
            for d, s_ in zip(sfields, ssnap):
                d.copy_(s_)
            torch.cuda.synchronize()
            with torch.cuda.stream(gs.stream):
                ev0.record(gs.stream)
                gs.correct(everyone, 2.0 ** -8, acc, jerk)
                ev1.record(gs.stream)
            torch.cuda.synchronize()
            corr.append(ev0.elapsed_time(ev1) * 1e-3)
        gs.sync()
        gs.close()
        tau_corr = min(corr) / n_tot
        n_mean = updates / max(steps, 1)
        rows.append({"N": n_tot, "t_end": t_end, "T_app_s": t_app, "block_steps": int(steps),
                     "updates": int(updates), "interactions": inter, "n_mean": n_mean,
                     "n_paper_0.20N^0.81": pm.block_size_paper(n_tot),
                     "tau_pred_us": tau_pred * 1e6, "tau_corr_us": tau_corr * 1e6,
                     "tau_force_us": {str(n): tau_f[n] * 1e6 for n in grid_n},
                     "_sizes": sizes, "_tau": pm.tau_force_table(tau_f),
                     "_pred": tau_pred, "_corr": tau_corr})
        log(f"perfmodel N={n_tot}: T_app {t_app:.3f} s, {steps} steps, n_mean {n_mean:.1f} "
            f"(0.20 N^0.81 = {pm.block_size_paper(n_tot):.1f}), tau_pred {tau_pred * 1e9:.2f} ns, "
            f"tau_corr {tau_corr * 1e9:.2f} ns")
    # fixed cost per block step, fitted on the smallest N alone
    r0 = rows[0]
    t_fixed = pm.fit_t0(r0["T_app_s"], r0["N"], r0["_sizes"], r0["_pred"], r0["_tau"], r0["_corr"])
    for r in rows:
        sizes, tau = r.pop("_sizes"), r.pop("_tau")
        tp, tc = r.pop("_pred"), r.pop("_corr")
        r["t0_us"] = t_fixed * 1e6
        r["T_model_per_step_sizes_s"] = pm.T_integrate(r["N"], sizes, tp, tau, tc, t_fixed)
        r["T_model_mean_block_s"] = pm.T_integrate_mean(r["N"], r["block_steps"], r["n_mean"],
                                                        tp, tau, tc, t_fixed)
        r["model_over_measured"] = r["T_model_per_step_sizes_s"] / r["T_app_s"]
        r["held_out"] = r is not r0
        log(f"perfmodel N={r['N']}: T_app {r['T_app_s']:.3f} s, model (block sizes) "
            f"{r['T_model_per_step_sizes_s']:.3f} s, model (mean block) "
            f"{r['T_model_mean_block_s']:.3f} s{'' if r['held_out'] else ' (t0 fitted here)'}")
    held = [r["model_over_measured"] for r in rows if r["held_out"]]
    return {"workload": f"plummer_eps1/256_mixed_to_t{t_end}", "t0_fitted_on_N": r0["N"],
            "held_out_model_over_measured": {"min": min(held) if held else None,
                                             "max": max(held) if held else None},
            "rows": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=N_DEFAULT, help="particles (default 196608)")
    ap.add_argument("--fp64-steps", type=int, default=1, help="timed FP64 steps (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=25.0,
                    help="CPU oracle budget; all N particles are checked when it suffices")
    ap.add_argument("--no-energy", action="store_true")
    ap.add_argument("--blocksizes", type=int, default=1 << 20,
                    help="force-only rates per block size at this N (0 = skip)")
    ap.add_argument("--ensemble", type=int, default=256,
                    help="the ensemble workload with this many clusters (0 = skip)")
    ap.add_argument("--ensemble-t", type=float, default=1.0 / 64)
    ap.add_argument("--ensemble-full", type=float, default=1.0)
    ap.add_argument("--no-per-cluster", action="store_true")
    ap.add_argument("--perfmodel", type=str, default="1024,4096,16384,65536,196608",
                    help="fit and check the per-step performance model on these N "
                         "(comma separated; empty = skip)")
    ap.add_argument("--perfmodel-t", type=float, default=1.0)
    ap.add_argument("--fused-mask", type=int, default=0b11100)
    ap.add_argument("--fused", type=int, default=0,
                    help="also time block steps with in-kernel prediction for the size "
                         "classes in this bit mask (e.g. 28 = classes 2-4), against the "
                         "prediction pass, this many times each")
    ap.add_argument("--salpeter", type=int, default=196608,
                    help="a Salpeter-mass Plummer sphere of this N (0 = skip)")
    ap.add_argument("--class-probes", type=str, default="",
                    help="autotuner block sizes, one per size class (comma separated)")
    ap.add_argument("--quick", action="store_true",
                    help="the headline workload only (no block sizes, ensemble, Salpeter, "
                         "performance model)")
    ap.add_argument("--only", type=str, default="",
                    help="run just one of blocksizes, ensemble, salpeter, perfmodel and print "
                         "its record (for profiler runs)")
    ap.add_argument("--sweep-only", type=int, default=0,
                    help="only time this many full sweeps, then one 512 MiB elementwise "
                         "copy of known size (for hardware-counter runs); prints one JSON line")
    args = ap.parse_args()
    if args.class_probes:
        global CLASS_PROBES
        CLASS_PROBES = tuple(int(q) for q in args.class_probes.split(","))
    if args.quick:
        args.blocksizes = args.ensemble = args.salpeter = 0
        args.perfmodel = ""
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path "
              "(a sharded design over RCCL is described with the documentation)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from nbody_inputs import plummer
    from paper_0709_4552_amd import NBODY_PREC_FP64, NBODY_PREC_MIXED

    if args.only:
        part = {"blocksizes": lambda: blocksize_sweep(torch, args.blocksizes or (1 << 20),
                                                      not args.no_cpu_baseline),
                "ensemble": lambda: ensemble_bench(torch, args.ensemble or 256, args.ensemble_t,
                                                   args.ensemble_full, not args.no_per_cluster),
                "salpeter": lambda: salpeter_bench(torch, args.salpeter or 196608, 1.0 / 16,
                                                   not args.no_cpu_baseline),
                "perfmodel": lambda: perfmodel_bench(
                    torch, [int(q) for q in (args.perfmodel or "1024,196608").split(",")],
                    args.perfmodel_t)}[args.only]()
        print(json.dumps({"metric": METRIC, "mode": "only", "section": args.only,
                          args.only: part}), flush=True)
        return

    x, v, m = plummer(args.n, SEED)
    log(f"workload: Plummer N={args.n} seed={SEED} eps=1/1024 to t={T_END}")

    if args.sweep_only:
        from paper_0709_4552_amd import NBody
        g = NBody(x, v, m, EPS, eta=0.01, eta_init=0.01, dt_min_log2=-20, dt_max_log2=-3,
                  precision=NBODY_PREC_MIXED)
        g.init()
        g.predict(0.0)
        il = torch.arange(args.n, dtype=torch.int32, device=g.dev)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ms = []
        with torch.cuda.stream(g.stream):
            for _ in range(args.sweep_only):
                ev0.record(g.stream)
                g.force_jerk(il, 0.0, want_pot=True)
                ev1.record(g.stream)
                torch.cuda.synchronize()
                ms.append(ev0.elapsed_time(ev1))
        # plain elementwise copy of known size: 512 MiB read + 512 MiB written
        src = torch.ones(64 << 20, dtype=torch.float64, device=g.dev)
        dst = torch.empty_like(src)
        torch.add(src, 0.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"metric": METRIC, "mode": "sweep-only", "n": args.n, "sweep_ms": ms,
                          "copy_bytes_each_way": src.numel() * 8,
                          "algorithmic_bytes_per_sweep": {"read": args.n * 40 * 2,
                                                          "write": args.n * 56}}), flush=True)
        g.close()
        return

    mixed = Run(x, v, m, NBODY_PREC_MIXED, torch)
    for w in range(args.warmup):
        mixed.step(False)
        log(f"warmup {w + 1}/{args.warmup} done")
    E0 = None
    for k in range(args.steps):
        mixed.step(True)
        log(f"step {k + 1}/{args.steps}: {mixed.step_ms[-1]:.1f} ms, "
            f"{mixed.inter[-1]:.3e} interactions, sweep {mixed.sweep_ms[-1]:.2f} ms")
    acc_m = mixed.last_sweep[0].T.cpu().numpy()
    jerk_m = mixed.last_sweep[1].T.cpu().numpy()
    energy = None
    if not args.no_energy:
        # the oracle's energy (FP64, all pairs) of the start state and of the
        # GPU's state after the block steps to T_END
        import oracle
        mixed.restore()
        mixed.g.run_until(T_END)
        x1, v1 = mixed.host_xv()
        t0 = time.perf_counter()
        E0 = sum(oracle.energy(x, v, m, EPS))
        E1 = sum(oracle.energy(x1, v1, m, EPS))
        energy = {"dE_over_E_t0.125": (E1 - E0) / abs(E0), "E0": E0, "E1": E1,
                  "source": "oracle energy (FP64, all pairs) of the GPU state",
                  "oracle_s": time.perf_counter() - t0}
        log(f"energy (oracle): dE/E = {(E1 - E0) / abs(E0):.3e}")

    sweep_nopot_ms = mixed.sweep_without_potential_ms()
    total_ms = sum(mixed.step_ms)
    total_inter = sum(mixed.inter)
    value = total_inter / (total_ms * 1e-3)
    sweep_ms = sum(mixed.sweep_ms) / len(mixed.sweep_ms)
    sweep_rate = float(args.n) * args.n / (sweep_ms * 1e-3)
    achieved = FLOPS_PER_INTERACTION * sweep_rate

    fp64 = None
    acc64 = None
    if args.fp64_steps > 0:
        r64 = Run(x, v, m, NBODY_PREC_FP64, torch)
        for k in range(args.fp64_steps):
            r64.step(True)
            log(f"fp64 step {k + 1}/{args.fp64_steps}: {r64.step_ms[-1]:.1f} ms")
        s64 = sum(r64.sweep_ms) / len(r64.sweep_ms)
        rate64 = float(args.n) * args.n / (s64 * 1e-3)
        fp64 = {"value": sum(r64.inter) / (sum(r64.step_ms) * 1e-3), "unit": "interactions/s",
                "ms_per_step": sum(r64.step_ms) / len(r64.step_ms),
                "full_sweep_ms": s64, "full_sweep_interactions_per_s": rate64,
                "full_sweep_frac_of_fp64_peak": FLOPS_PER_INTERACTION * rate64 / PEAK_FP64}
        acc64 = (r64.last_sweep[0].T.cpu().numpy(), r64.last_sweep[1].T.cpu().numpy())
        r64.g.close()

    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        sw = {"mixed": (acc_m, jerk_m)}
        if acc64 is not None:
            sw["fp64"] = acc64
        cpu, accuracy = cpu_baseline(x, v, m, sw, args.cpu_seconds)
        log(f"cpu oracle: {cpu['value']:.3e} interactions/s on {cpu['cores']} threads")

    extra_bs = blocksize_sweep(torch, args.blocksizes, not args.no_cpu_baseline) \
        if args.blocksizes else None
    extra_ens = ensemble_bench(torch, args.ensemble, args.ensemble_t, args.ensemble_full,
                               not args.no_per_cluster) if args.ensemble else None

    extra_sal = salpeter_bench(torch, args.salpeter, 1.0 / 16, not args.no_cpu_baseline) \
        if args.salpeter else None
    extra_pm = perfmodel_bench(torch, [int(q) for q in args.perfmodel.split(",")],
                               args.perfmodel_t) if args.perfmodel else None
    extra_fused = fused_bench(mixed, args.fused_mask, args.fused) if args.fused else None

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "ms_per_step_min": min(mixed.step_ms),
        "ms_per_step_median": float(statistics.median(mixed.step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pairwise, f64 coordinates/accumulation",
        "data": "synthetic",
        "config": {"workload": f"plummer_N{args.n}_eps1/1024_eta0.01_fullsweep+blocksteps_to_t0.125",
                   "n": args.n, "eps": EPS, "eta": 0.01, "dt_range": "[2^-20, 2^-3]",
                   "t_end": T_END, "seed": SEED, "precision": "mixed",
                   "interactions_per_step": total_inter / args.steps,
                   "block_steps_per_step": mixed.block_steps,
                   "autotuned_shapes": mixed.tuning},
        "full_sweep": {"ms": sweep_ms, "ms_min": min(mixed.sweep_ms),
                       "ms_median": float(statistics.median(mixed.sweep_ms)),
                       "interactions_per_s": sweep_rate,
                       "returns": "acc, jerk, potential (FP64, 56 B per particle)",
                       "ms_acc_jerk_only": sweep_nopot_ms,
                       "interactions_per_s_acc_jerk_only":
                           float(args.n) * args.n / (sweep_nopot_ms * 1e-3)},
        "roofline": {"bound": "alu",
                     "traffic_note": "HBM bytes per sweep launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, "
                                     "calibrated); algorithmic 26.7e6",
                     "kernel": "k_force<1,1,256,mixed,potential> (the n=N full sweep)",
                     "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": sweep_traffic(),
                     "flops_per_interaction": FLOPS_PER_INTERACTION},
        "fp64": fp64,
        "fused_prediction": extra_fused,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "energy": energy,
        "block_sizes": extra_bs,
        "ensemble": extra_ens,
        "perfmodel": extra_pm,
        "salpeter": extra_sal,
        "context": {"grape6af_interactions_per_s": 1.0 / 4.3e-10,
                    "grape6af_simultaneous_interactions": 42},
    }
    mixed.g.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
