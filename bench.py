#!/usr/bin/env python3
"""Throughput of the deflated-multigrid Wilson-Dirac solve on one MI355X.

Workload: 256 x 256 lattices, beta = 6.0 synthetic U(1) configurations (von
Mises plaquettes, axial gauge), bare mass m0 = m_c + 0.01, three grids
256^2 -> 64^2 -> 16^2 with 24 dof per blocked site, outer FGMRES(8) to true
relative residual 1e-8, GMRES(2) smoothing, partial intermediate solve to 0.2,
coarse GMRES-DR(30, 10) on the first coarse call of each configuration and
GMRES-Proj(30, 10) afterwards, 5 Gaussian right-hand sides per configuration.

A step is one configuration: its 5 right-hand sides solved one after the other
with a fresh (empty) deflation space, so the first solve pays for GMRES-DR.
The hierarchy of every configuration is built before the timed region (setup is
reported separately, not in the rate).  `value` is FP64-preconditioner
solves/s over the timed steps; the same steps are then timed with the FP32
preconditioner (FP64 outer solve) and reported under "mixed".

    python bench.py [--gpus 1] [--steps 10] [--warmup 1]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
RHS_PER_CONFIG = 5


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lattice", type=int, default=256)
    ap.add_argument("--configs", type=int, default=10, help="distinct gauge configurations cycled over")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle solves for the CPU baseline")
    return ap.parse_args()


def percentile(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else float("nan")


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the solver has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    import paper_1912_02868_amd as dmg

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dmg.lib()
    N = a.lattice
    ctx = dmg.Context(0)
    stream = torch.cuda.current_stream()

    # ------------------------------------------------------------ setup (untimed for the rate)
    step_cfgs = [(a.warmup + i) % a.configs for i in range(a.steps)]
    warm_cfgs = [i % a.configs for i in range(a.warmup)]
    need = sorted(set(step_cfgs + warm_cfgs))
    res = {}
    setup_ms = []
    for c in need:
        th = synth.gauge_angles(N, c)
        m0 = synth.bare_mass(N, c)
        g = dmg.Gauge(ctx, th)
        s0 = torch.from_numpy(synth.near_null_starts(N, c, 0)).cuda()
        s1 = torch.from_numpy(synth.near_null_starts(N, c, 1)).cuda()
        b = torch.from_numpy(np.stack([synth.rhs(N, c, j) for j in range(RHS_PER_CONFIG)])).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = dmg.Hierarchy(ctx, g, m0, s0, s1)
        torch.cuda.synchronize()
        setup_ms.append((time.perf_counter() - t0) * 1e3)
        del s0, s1
        res[c] = (g, h, b)

    def run_step(c, precond, lat, stats_all):
        g, h, b = res[c]
        d = dmg.Deflation(h, 30, 10)
        x = torch.empty_like(b)
        prm = dmg.solve_params(precond=precond)
        for j in range(RHS_PER_CONFIG):
            t0 = time.perf_counter()
            st, stats = dmg.solve(ctx, h, d, b[j], x[j], params=prm)
            lat.append((time.perf_counter() - t0) * 1e3)
            stats_all.append(stats[0])
        d.close()
        return x

    def timed(precond):
        for c in warm_cfgs:
            run_step(c, precond, [], [])
        lat, st_all = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in step_cfgs:
            run_step(c, precond, lat, st_all)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, lat, st_all

    # the dominant kernel (the persistent coarse solve) is timed with HIP events by the
    # library itself, launch by launch, over the timed FP64 region
    ctx.timer(dmg.KT_COARSE_PROJ)
    el64, lat64, st64 = timed(dmg.FP64)
    coarse_ms, coarse_launches, coarse_steps = ctx.timer_read(dmg.KT_COARSE_PROJ)
    ctx.timer()
    n_solves = len(step_cfgs) * RHS_PER_CONFIG
    ok64 = all(s["converged"] and s["true_rel_resid"] <= 1e-8 for s in st64)
    out_mixed = None
    if not a.no_mixed:
        el32, lat32, st32 = timed(dmg.FP32)
        ok32 = all(s["converged"] and s["true_rel_resid"] <= 1e-8 for s in st32)
        out_mixed = {
            "value": n_solves / el32, "unit": "solves/s", "dtype": "f32 preconditioner, f64 outer",
            "p50_ms": percentile(lat32, 50), "p99_ms": percentile(lat32, 99),
            "all_converged_1e-8": ok32, "speedup_vs_fp64": (n_solves / el32) / (n_solves / el64),
            "mean_outer_iters": float(np.mean([s["outer_iters"] for s in st32])),
            "max_true_rel_resid": float(max(s["true_rel_resid"] for s in st32)),
        }

    # ------------------------------------------------------------ roofline of the dominant kernel
    roof = coarse_roofline(N, coarse_ms, coarse_launches, coarse_steps, el64)
    roof_int = measure_stencil_roofline(torch, dmg, ctx, res[step_cfgs[0]][1], N)

    # ------------------------------------------------------------ CPU baseline (oracle)
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(N, a.cpu_budget, np.mean([s["outer_iters"] for s in st64]))

    mean = lambda k: float(np.mean([s[k] for s in st64]))
    line = {
        "metric": "solves/s at rel. residual 1e-8 (256^2, mixed vs FP64); p50/p99 solve latency",
        "value": n_solves / el64,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": el64 / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: von Mises(beta=6) U(1) plaquettes in axial gauge, Gaussian right-hand sides",
        "config": {"workload": f"{N}^2 Wilson-Dirac, m0 = m_c + 0.01, 3-grid deflated MG, "
                               f"{RHS_PER_CONFIG} RHS per configuration",
                   "lattice": N, "configs": sorted(set(step_cfgs)), "rhs_per_config": RHS_PER_CONFIG,
                   "outer": "FGMRES(8) tol 1e-8", "coarse": "GMRES-DR(30,10) then GMRES-Proj(30,10)"},
        "p50_ms": percentile(lat64, 50),
        "p99_ms": percentile(lat64, 99),
        "all_converged_1e-8": ok64,
        "max_true_rel_resid": float(max(s["true_rel_resid"] for s in st64)),
        "setup_ms_mean": float(np.mean(setup_ms)),
        "mean_outer_iters": mean("outer_iters"),
        "mean_mvps": {"fine": mean("fine_mvps"), "intermediate": mean("int_mvps"), "coarse": mean("coarse_mvps"),
                      "fine_equivalent": mean("fine_equiv_mvps")},
        "mixed": out_mixed,
        "roofline": roof,
        "roofline_intermediate_stencil": roof_int,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def coarse_roofline(N, total_ms, launches, steps, timed_s):
    """Roofline of the persistent coarse GMRES-Proj kernel (k_coarse_proj<double, false>),
    the kernel with the largest share of the timed region.  Algorithmic bytes: every
    Arnoldi step applies the coarse operator once, reading its 5 blocks of 24 x 24
    complex doubles per coarse site (46,080 B per site; Krylov and deflation slices stay
    in LDS).  achieved = steps x bytes per step / summed launch time."""
    sites = (N // 16) ** 2
    bytes_per_step = sites * 5 * 24 * 24 * 16
    achieved = steps * bytes_per_step / (total_ms * 1e-3) / 1e9 if total_ms > 0 else 0.0
    return {"kernel": "k_coarse_proj<double, false> (persistent GMRES-Proj, coarse grid "
                      f"{N // 16}x{N // 16} sites x 24 dof)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "avg_launch_us": total_ms / max(launches, 1) * 1e3, "launches": launches,
            "arnoldi_steps": steps, "us_per_step": total_ms * 1e3 / max(steps, 1),
            "algorithmic_bytes_per_step": bytes_per_step,
            "share_of_timed_region": total_ms * 1e-3 / timed_s if timed_s > 0 else None,
            "note": "latency bound: two grid barriers per Arnoldi step"}


def measure_stencil_roofline(torch, dmg, ctx, h, N, reps=200):
    """The intermediate-grid block stencil (64x64 sites at 256^2), the kernel that moves the
    most bytes per solve: 5 blocks of 24 x 24 complex doubles plus one input and one output
    24-vector per blocked site (46,848 B), timed by the library's events over `reps` launches."""
    L = N // 4
    sites = L * L
    x = torch.randn(sites * 24, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        h.apply(1, dmg.OP_APPLY, x, y)
    ctx.timer(dmg.KT_BLOCK_APPLY_INT)
    for _ in range(reps):
        h.apply(1, dmg.OP_APPLY, x, y)
    ms, n, units = ctx.timer_read(dmg.KT_BLOCK_APPLY_INT)
    ctx.timer()
    bytes_per_launch = sites * (5 * 24 * 24 * 16 + 2 * 24 * 16)
    avg_ms = ms / max(n, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    return {"kernel": "k_block_apply<double> (intermediate grid, 64x64 sites x 24 dof)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "avg_launch_us": avg_ms * 1e3,
            "algorithmic_bytes_per_launch": bytes_per_launch}


def cpu_baseline(N, budget_s, gpu_outer_iters):
    """The oracle (numpy/scipy FP64) on the same 256^2 workload, bounded in time: the oracle's
    hierarchy of configuration 0 is built (not charged, as the GPU setup is not), then its
    right-hand sides 0, 1, ... are solved to 1e-8 one after the other (a fresh deflation space,
    so the first pays for GMRES-DR) until `budget_s` seconds have been spent; the rate counts
    completed solves only.  If not even one solve completes, the rate is extrapolated from the
    outer iterations done and the GPU run's mean outer iterations per solve."""
    import synth
    from oracle import multigrid
    threads = 1
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        pass
    th = synth.gauge_angles(N, 0)
    m0 = synth.bare_mass(N, 0)
    t0 = time.perf_counter()
    H = multigrid.Hierarchy(th, m0, synth.near_null_starts(N, 0, 0), synth.near_null_starts(N, 0, 1))
    setup_s = time.perf_counter() - t0
    iters = 0
    orig = H.cycle0

    def counted_cycle(v):
        nonlocal iters
        iters += 1
        return orig(v)
    H.cycle0 = counted_cycle
    solves, lat = 0, []
    t0 = time.perf_counter()
    for j in range(RHS_PER_CONFIG):
        if time.perf_counter() - t0 > budget_s:
            break
        t1 = time.perf_counter()
        _, info = H.solve(synth.rhs(N, 0, j))
        lat.append(time.perf_counter() - t1)
        solves += 1 if info.converged else 0
    el = time.perf_counter() - t0
    value = solves / el if solves else 1.0 / (el / max(iters, 1) * gpu_outer_iters)
    return {"value": value, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{N}^2 configuration 0, right-hand sides 0..{len(lat) - 1} solved to 1e-8 in {el:.1f} s "
                      f"({iters} outer iterations; the first solve includes GMRES-DR); oracle setup "
                      f"{setup_s:.1f} s not charged; scipy sparse products are single-threaded",
            "cpu": platform.processor() or platform.machine(), "host_cpus": os.cpu_count()}


if __name__ == "__main__":
    main()
