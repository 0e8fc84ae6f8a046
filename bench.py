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
INFINITY_CACHE_BYTES = 256 * 10 ** 6
RHS_PER_CONFIG = 5
# HBM bytes per launch of k_coarse_proj<double, false, true, true> from the FETCH_SIZE and WRITE_SIZE counter
# passes (scaled by the reference streaming kernels) recorded in profiles/k_coarse_proj_256_hbm_traffic.md;
# valid while that kernel is unchanged
COARSE_TRAFFIC_BYTES = 65_012_838


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
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-rhs", type=int, default=64, help="right-hand sides per lockstep solve")
    ap.add_argument("--batched-configs", type=int, default=1)
    ap.add_argument("--batched-lattice", type=int, default=512,
                    help="lattice of the lockstep form (512: one 512^2 configuration x 64 right-hand sides)")
    ap.add_argument("--no-oracle-error", action="store_true",
                    help="skip the error of every timed solution against sparse LU of the oracle's D")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-sizes", default="64,128,256,512")
    ap.add_argument("--serve-configs", type=int, default=4, help="resident configurations per lattice size")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per arrival rate")
    ap.add_argument("--serve-capacity", type=int, default=16, help="lanes per resident configuration")
    ap.add_argument("--serve-inflight", type=int, default=3, help="lane-batch steps running at once")
    ap.add_argument("--serve-age", type=float, default=0.1,
                    help="seconds of waiting that double a configuration's scheduling weight")
    ap.add_argument("--scan", action="store_true",
                    help="mass-gap and lattice-size scan of six solvers with power-law fits (prints its own JSON)")
    ap.add_argument("--scan-sizes", default="64,128,256")
    ap.add_argument("--scan-configs", type=int, default=2)
    ap.add_argument("--scan-first-config", type=int, default=0,
                    help="first configuration of the scan (configurations first .. first + count - 1)")
    ap.add_argument("--scan-merge", default="",
                    help="comma-separated files holding earlier --scan outputs: combine their rows, refit and print "
                         "(no GPU)")
    ap.add_argument("--scan-gaps", default="1e-1,1e-2,1e-3,1e-4")
    ap.add_argument("--scan-fit-gap", type=float, default=1e-4)
    ap.add_argument("--scan-rhs", type=int, default=2)
    ap.add_argument("--scan-coarse", default="200,40",
                    help="coarse GMRES-DR / GMRES-Proj (m, k) of the deflated multigrid methods (the paper's 200,40)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the multi-RHS stencils at 512^2 x 64 (FP32 Wilson, FP32 and FP64 matrix-core block "
                         "stencils) and a 256 MiB streaming kernel, for hardware counter passes (prints its own JSON)")
    ap.add_argument("--maps", default="",
                    help="write this process's memory map (/proc/self/maps) to the given file before exiting")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for hardware byte counters)")
    return ap.parse_args()


def progress(msg):
    """A line on stderr per stage, so a long run shows it is alive."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def percentile(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else float("nan")


def main():
    a = parse()
    if a.maps:
        import atexit
        import shutil
        atexit.register(lambda: shutil.copyfile("/proc/self/maps", a.maps))
    if a.scan_merge:
        print(json.dumps(scan_merge(a.scan_merge.split(","), a.scan_fit_gap)), flush=True)
        return
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
    if a.kernels_only:
        print(json.dumps(kernels_only(torch, dmg)), flush=True)
        return
    if a.scan:
        ctx = dmg.Context(0)
        out = scan(torch, dmg, ctx, [int(v) for v in a.scan_sizes.split(",")], a.scan_configs,
                   [float(v) for v in a.scan_gaps.split(",")], a.scan_fit_gap, a.scan_rhs,
                   tuple(int(v) for v in a.scan_coarse.split(",")), a.scan_first_config)
        ctx.close()
        print(json.dumps(out), flush=True)
        return
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

    sols = {}  # (precision, configuration) -> solutions of the last timed step of that configuration

    def timed(precond):
        for c in warm_cfgs:
            run_step(c, precond, [], [])
        lat, st_all = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in step_cfgs:
            sols[(precond, c)] = run_step(c, precond, lat, st_all)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, lat, st_all

    # the dominant kernel (the persistent coarse solve) is timed with HIP events by the
    # library itself, launch by launch, over the timed FP64 region
    progress(f"setup of {len(need)} hierarchies done; plain FP64 form")
    ctx.timer(dmg.KT_COARSE_PROJ)
    el64, lat64, st64 = timed(dmg.FP64)
    coarse_ms, coarse_launches, coarse_steps = ctx.timer_read(dmg.KT_COARSE_PROJ)
    ctx.timer()
    n_solves = len(step_cfgs) * RHS_PER_CONFIG
    ok64 = all(s["converged"] and s["true_rel_resid"] <= 1e-8 for s in st64)
    out_mixed = None
    progress(f"plain FP64: {n_solves / el64:.2f} solves/s")
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
        progress(f"FP32 preconditioner: {n_solves / el32:.2f} solves/s")
        el16, lat16, st16 = timed(dmg.FP32_BF16)
        out_mixed["bf16_blocks"] = {
            "value": n_solves / el16, "unit": "solves/s",
            "dtype": "f32 preconditioner with bf16-stored intermediate blocks, f64 outer",
            "p50_ms": percentile(lat16, 50), "p99_ms": percentile(lat16, 99),
            "all_converged_1e-8": all(s["converged"] and s["true_rel_resid"] <= 1e-8 for s in st16),
            "speedup_vs_fp64": (n_solves / el16) / (n_solves / el64),
            "mean_outer_iters": float(np.mean([s["outer_iters"] for s in st16])),
            "max_true_rel_resid": float(max(s["true_rel_resid"] for s in st16)),
        }
        progress(f"BF16 intermediate blocks: {n_solves / el16:.2f} solves/s")
        el16c, lat16c, st16c = timed(dmg.FP32_BF16C)
        out_mixed["bf16_coarse_blocks"] = {
            "value": n_solves / el16c, "unit": "solves/s",
            "dtype": "f32 preconditioner with the coarse blocks rounded to bf16 (f32 accumulate), f64 outer",
            "p50_ms": percentile(lat16c, 50), "p99_ms": percentile(lat16c, 99),
            "all_converged_1e-8": all(s["converged"] and s["true_rel_resid"] <= 1e-8 for s in st16c),
            "speedup_vs_fp64": (n_solves / el16c) / (n_solves / el64),
            "mean_outer_iters": float(np.mean([s["outer_iters"] for s in st16c])),
            "max_true_rel_resid": float(max(s["true_rel_resid"] for s in st16c)),
        }

    if a.calibrate_copy:
        # plain streaming kernels of known size: uniform_ writes 256 MiB; mul reads 256 MiB
        # and writes 256 MiB per launch
        src = torch.empty(256 * 2 ** 20 // 4, dtype=torch.float32, device="cuda").uniform_()
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    # ------------------------------------------------------------ roofline of the dominant kernel
    roof = coarse_roofline(N, coarse_ms, coarse_launches, coarse_steps, el64)
    roof_int = measure_stencil_roofline(torch, dmg, ctx, res[step_cfgs[0]][1], N)
    roof_int16 = measure_bf16_stencil(torch, dmg, res[step_cfgs[0]][1], N)

    # ------------------------------------------------------------ batched and served forms
    progress("stencil rooflines done")
    out_batched = None
    if not a.no_batched:
        NB = a.batched_lattice or N
        cfgs_b = step_cfgs[:a.batched_configs] if NB == N else list(range(a.batched_configs))
        out_batched = batched_form(torch, dmg, ctx, NB, cfgs_b, a.batched_rhs, n_solves / el64)
    progress("batched form done")
    out_served = None
    if not a.no_serve:
        out_served = served_form(torch, dmg, ctx, [int(v) for v in a.serve_sizes.split(",")], a.serve_configs,
                                 a.serve_requests, a.serve_capacity, a.serve_inflight, a.serve_age)

    # ------------------------------------------------------------ error against the oracle
    progress("served form done")
    oracle_err = None
    if not a.no_oracle_error:
        oracle_err = errors_vs_oracle(synth, N, res, sols)
        for prec, key in ((dmg.FP32, None), (dmg.FP32_BF16, "bf16_blocks"), (dmg.FP32_BF16C, "bf16_coarse_blocks")):
            if out_mixed is not None and prec in oracle_err:
                (out_mixed if key is None else out_mixed[key])["error_vs_oracle"] = oracle_err.pop(prec)

    # ------------------------------------------------------------ CPU baseline (oracle)
    progress("errors against the oracle done")
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
        "error_vs_oracle": oracle_err.get(dmg.FP64) if oracle_err else None,
        "mixed": out_mixed,
        "batched": out_batched,
        "served": out_served,
        "roofline": roof,
        "roofline_intermediate_stencil": roof_int,
        "roofline_intermediate_stencil_bf16": roof_int16,
        "cpu_baseline": cpu,
    }
    # release every handle before the interpreter exits (no library teardown at exit time)
    sols.clear()
    for g, h, b in res.values():
        h.close()
        g.close()
    res.clear()
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps(line), flush=True)


def kernels_only(torch, dmg, N=512, nrhs=64, reps=20):
    """The multi-RHS stencils of the batched form on one 512^2 configuration, each launched
    `reps` times through the apply hook (working sets above the 256 MB Infinity Cache:
    541 MB per FP32 Wilson apply, 780 MB per FP32 and 1.56 GB per FP64 block apply on the
    128^2 intermediate grid), then a plain streaming multiply of 256 MiB (reads 256 MiB,
    writes 256 MiB per launch) as the reference for byte counters.  Each kernel's average
    launch time comes from the library's events."""
    import synth
    ctx = dmg.Context(0)
    g = dmg.Gauge(ctx, synth.gauge_angles(N, 0))
    h = dmg.Hierarchy(ctx, g, synth.bare_mass(N, 0), torch.from_numpy(synth.near_null_starts(N, 0, 0)).cuda(),
                      torch.from_numpy(synth.near_null_starts(N, 0, 1)).cuda())
    out = {"workload": f"{N}^2 configuration 0, {nrhs} right-hand sides", "reps": reps}
    out["wilson_fp32"] = batched_wilson_roofline(torch, dmg, ctx, h, N, nrhs, reps=reps)
    out["block_fp32"] = batched_block_roofline(torch, dmg, ctx, h, N, nrhs, reps=reps)
    out["block_fp64"] = batched_block_roofline(torch, dmg, ctx, h, N, nrhs, reps=reps, prec="fp64")
    src = torch.empty(256 * 2 ** 20 // 4, dtype=torch.float32, device="cuda").uniform_()
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    out["autotune"] = dmg.autotune_report().strip().splitlines()
    out["copy_reference"] = {"kernel": "torch.mul float32 (elementwise multiply)", "bytes_read": 256 * 2 ** 20,
                             "bytes_written": 256 * 2 ** 20, "launches": reps}
    del src, dst
    h.close()
    g.close()
    torch.cuda.synchronize()
    ctx.close()
    return out


def errors_vs_oracle(synth, N, res, sols):
    """Relative error of every timed solution against sparse LU of the oracle's D (FP64),
    per preconditioner precision: max and median over the configurations' right-hand sides,
    with the a-posteriori bound kappa-free form ||x - x_LU|| / ||x_LU||.  Computed after the
    timed regions, on the host."""
    import scipy.sparse.linalg as spla
    from oracle import wilson
    t0 = time.perf_counter()
    errs = {}
    for c in sorted({c for (_, c) in sols}):
        progress(f"sparse LU of configuration {c}")
        D = wilson.dirac_matrix(synth.gauge_angles(N, c), synth.bare_mass(N, c))
        lu = spla.splu(D.tocsc(), permc_spec="MMD_AT_PLUS_A")
        b = res[c][2].cpu().numpy()
        ref = [lu.solve(b[j]) for j in range(b.shape[0])]
        for (prec, cc), x in sols.items():
            if cc != c:
                continue
            xh = x.cpu().numpy()
            for j in range(b.shape[0]):
                errs.setdefault(prec, []).append(float(np.linalg.norm(xh[j] - ref[j]) / np.linalg.norm(ref[j])))
    el = time.perf_counter() - t0
    return {prec: {"max": max(v), "median": float(np.median(v)), "solves": len(v),
                   "reference": "sparse LU of the oracle's FP64 D (scipy splu)", "host_s": el}
            for prec, v in errs.items()}


def coarse_roofline(N, total_ms, launches, steps, timed_s):
    """Roofline of the persistent coarse GMRES-Proj kernel (k_coarse_proj<double, false, true, true>),
    the kernel with the largest share of the timed region.  Algorithmic bytes: every
    Arnoldi step applies the coarse operator once, reading its 5 blocks of 24 x 24
    complex doubles per coarse site (46,080 B per site; Krylov and deflation slices stay
    in LDS).  achieved = steps x bytes per step / summed launch time."""
    sites = (N // 16) ** 2
    bytes_per_step = sites * 5 * 24 * 24 * 16
    achieved = steps * bytes_per_step / (total_ms * 1e-3) / 1e9 if total_ms > 0 else 0.0
    per_launch = steps / max(launches, 1) * bytes_per_step
    return {"kernel": "k_coarse_proj<double, false, true, true> (persistent GMRES-Proj, halo form, blocks in registers, coarse grid "
                      f"{N // 16}x{N // 16} sites x 24 dof)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": COARSE_TRAFFIC_BYTES if N == 256 else None,
            "traffic_unit": "HBM bytes per launch (counters, profiles/k_coarse_proj_256_hbm_traffic.md)",
            "algorithmic_bytes_per_launch": per_launch,
            "avg_launch_us": total_ms / max(launches, 1) * 1e3, "launches": launches,
            "arnoldi_steps": steps, "us_per_step": total_ms * 1e3 / max(steps, 1),
            "algorithmic_bytes_per_step": bytes_per_step,
            "share_of_timed_region": total_ms * 1e-3 / timed_s if timed_s > 0 else None,
            "limited_by": "latency: one grid barrier and exchange per Arnoldi step; the operator stays in "
                          "registers, so HBM carries only the counter traffic",
            "counter_gbs": (COARSE_TRAFFIC_BYTES / (total_ms / max(launches, 1) * 1e-3) / 1e9
                            if N == 256 and total_ms > 0 else None)}


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
    return {"kernel": f"k_block_apply<double> (intermediate grid, {L}x{L} sites x 24 dof)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "avg_launch_us": avg_ms * 1e3,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "cache_resident": bytes_per_launch < INFINITY_CACHE_BYTES,
            "note": "working set below the 256 MB Infinity Cache: the fraction is not an HBM figure"
            if bytes_per_launch < INFINITY_CACHE_BYTES else "working set above the 256 MB Infinity Cache"}


def measure_bf16_stencil(torch, dmg, h, N, reps=200):
    """The same stencil with BF16-stored blocks and FP32 vectors (the BF16 preconditioner
    variant): 5 x 576 x 4 B of blocks plus two FP32 24-vectors (384 B) per blocked site,
    timed with stream events around `reps` launches of the apply hook."""
    L = N // 4
    sites = L * L
    x = torch.randn(sites * 24, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        h.apply(1, dmg.OP_APPLY, x, y, bf16=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        h.apply(1, dmg.OP_APPLY, x, y, bf16=True)
    e1.record()
    torch.cuda.synchronize()
    avg_ms = e0.elapsed_time(e1) / reps
    bytes_per_launch = sites * (5 * 24 * 24 * 4 + 2 * 24 * 8)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    return {"kernel": f"k_block_apply<float, bf16> (intermediate grid, {L}x{L} sites x 24 dof, BF16 blocks)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "avg_launch_us": avg_ms * 1e3,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "cache_resident": bytes_per_launch < INFINITY_CACHE_BYTES}


def build_resident(dmg, ctx, synth, N, c):
    """Hierarchy and a built deflation space (GMRES-DR on the seeded coarse warm-up
    right-hand side) of one configuration: the state a server keeps on the device."""
    import torch
    g = dmg.Gauge(ctx, synth.gauge_angles(N, c))
    h = dmg.Hierarchy(ctx, g, synth.bare_mass(N, c), torch.from_numpy(synth.near_null_starts(N, c, 0)).cuda(),
                      torch.from_numpy(synth.near_null_starts(N, c, 1)).cuda())
    d = dmg.Deflation(h, 30, 10)
    d.build(synth.gaussian_complex(24 * (N // 16) ** 2, N, c, 4, 0), 1e-8)
    return g, h, d


def batched_form(torch, dmg, ctx, N, cfgs, nrhs, plain_rate):
    """Lockstep multi-RHS solves (dmg_solve_batched): per configuration, right-hand sides
    0 .. nrhs-1 solved jointly with the FP32 preconditioner (and again with the FP64 one)
    over the configuration's deflation space built beforehand.  Latency of a right-hand
    side = its call's wall time.  The timed calls run as in production (each coarse
    GMRES-Proj cycle replayed from a captured HIP graph).  One more FP32 call on the first
    configuration, with the library's per-launch events on (kernels launched one by one),
    gives the multi-RHS block and Wilson stencils' share of a call; the intermediate-grid
    block stencil alone gives the matrix-core roofline."""
    import synth
    res = {c: build_resident(dmg, ctx, synth, N, c) for c in cfgs}
    B = {c: torch.from_numpy(np.stack([synth.rhs(N, c, j) for j in range(nrhs)])).cuda() for c in cfgs}
    X = torch.empty_like(B[cfgs[0]])
    out = {"workload": f"{N}^2, {nrhs} right-hand sides per lockstep solve, configurations {list(cfgs)}",
           "rhs_per_call": nrhs}
    # like-for-like comparator: the plain FP64 form (one right-hand side at a time) on the same
    # lattice and configuration with the same deflation space already built (GMRES-Proj only)
    g, h, d = res[cfgs[0]]
    n_plain = 8
    xs = torch.empty_like(B[cfgs[0]][0])
    dmg.solve(ctx, h, d, B[cfgs[0]][0], xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(n_plain):
        dmg.solve(ctx, h, d, B[cfgs[0]][j], xs)
    torch.cuda.synchronize()
    plain_same = n_plain / (time.perf_counter() - t0)
    out["plain_fp64_same_lattice"] = {"value": plain_same, "unit": "solves/s",
                                      "sample": f"right-hand sides 0..{n_plain - 1} one at a time, deflation "
                                                "space built beforehand as in the lockstep form"}
    for prec in ("fp32", "fp64", "fp32_bf16"):
        progress(f"batched {prec}")
        prm = dmg.solve_params(precond=prec)
        g, h, d = res[cfgs[0]]
        dmg.solve_batched(ctx, h, d, B[cfgs[0]], X, nrhs, params=prm)  # workspace
        torch.cuda.synchronize()
        lat, stats = [], []
        t0 = time.perf_counter()
        for c in cfgs:
            g, h, d = res[c]
            t1 = time.perf_counter()
            st, ss = dmg.solve_batched(ctx, h, d, B[c], X, nrhs, params=prm)
            torch.cuda.synchronize()
            lat += [(time.perf_counter() - t1) * 1e3] * nrhs
            stats += ss
        el = time.perf_counter() - t0
        kt = None
        if prec == "fp32":
            g, h, d = res[cfgs[0]]
            ctx.timer(dmg.KT_BLOCK_BATCHED, dmg.KT_WILSON_BATCHED)
            t1 = time.perf_counter()
            dmg.solve_batched(ctx, h, d, B[cfgs[0]], X, nrhs, params=prm)
            torch.cuda.synchronize()
            el1 = time.perf_counter() - t1
            kt = {"instrumented_call_ms": el1 * 1e3}
            for name, k in (("block_batched", dmg.KT_BLOCK_BATCHED), ("wilson_batched", dmg.KT_WILSON_BATCHED)):
                ms, n, u = ctx.timer_read(k)
                kt[name] = {"ms": ms, "launches": n, "site_lanes": u, "share_of_call": ms * 1e-3 / el1}
            ctx.timer()
        out[prec] = {"value": len(cfgs) * nrhs / el, "unit": "solves/s",
                     "dtype": {"fp32": "f32", "fp64": "f64", "fp32_bf16": "f32 (bf16 intermediate blocks)"}[prec]
                     + " preconditioner, f64 outer",
                     "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
                     "all_converged_1e-8": all(s["converged"] and s["true_rel_resid"] <= 1e-8 for s in stats),
                     "max_true_rel_resid": float(max(s["true_rel_resid"] for s in stats)),
                     "mean_outer_iters": float(np.mean([s["outer_iters"] for s in stats])),
                     "speedup_vs_plain_fp64_same_lattice": (len(cfgs) * nrhs / el) / plain_same,
                     "ratio_to_headline_plain_fp64": (len(cfgs) * nrhs / el) / plain_rate}
        if kt:
            out[prec]["kernels"] = kt
    out["roofline_block_batched"] = batched_block_roofline(torch, dmg, ctx, res[cfgs[0]][1], N, nrhs)
    out["roofline_wilson_batched"] = batched_wilson_roofline(torch, dmg, ctx, res[cfgs[0]][1], N, nrhs)
    for g, h, d in res.values():
        d.close()
        h.close()
    return out


FP32_MFMA_PEAK_TFLOPS = 157.3
FP64_MFMA_PEAK_TFLOPS = 78.6


def batched_block_roofline(torch, dmg, ctx, h, N, nrhs, reps=50, prec="fp32"):
    """Multi-RHS intermediate-grid block stencil on the matrix cores (FP32, or FP64 with
    prec="fp64"): per blocked site and right-hand side 5 x 576 complex multiply-adds
    (23,040 flop); bytes per site: the 5 blocks (23,040 B FP32, 46,080 B FP64) plus input and
    output 24-vectors of every right-hand side (384 nrhs B FP32, 768 nrhs B FP64).  Timed by
    the library's events around each launch."""
    L = N // 4
    sites = L * L
    n1 = sites * 24
    f64 = prec == "fp64"
    x = torch.randn(nrhs, n1, dtype=torch.complex128 if f64 else torch.complex64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        h.apply_batched(1, dmg.OP_APPLY, x, y, nrhs)
    ctx.timer(dmg.KT_BLOCK_BATCHED)
    for _ in range(reps):
        h.apply_batched(1, dmg.OP_APPLY, x, y, nrhs)
    ms, n, u = ctx.timer_read(dmg.KT_BLOCK_BATCHED)
    ctx.timer()
    avg = ms / max(n, 1)
    flops = sites * nrhs * 23040
    es = 16 if f64 else 8
    byts = sites * (5 * 576 * es + 2 * 24 * es * nrhs)
    tf = flops / (avg * 1e-3) / 1e12
    peak = FP64_MFMA_PEAK_TFLOPS if f64 else FP32_MFMA_PEAK_TFLOPS
    return {"kernel": f"kb_block_mfma_p ({'FP64' if f64 else 'FP32'}, {L}x{L} sites x 24 dof x {nrhs} right-hand "
                      f"sides, {'16x16x4 FP64' if f64 else '16x16x4 FP32'} MFMA)",
            "bound": "mfma", "achieved": tf, "peak": peak, "unit": "TFLOP/s",
            "frac": tf / peak, "traffic": None, "avg_launch_us": avg * 1e3,
            "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": byts,
            "achieved_gbs": byts / (avg * 1e-3) / 1e9}


def batched_wilson_roofline(torch, dmg, ctx, h, N, nrhs, reps=50):
    """Multi-RHS fine Wilson stencil in FP32: per site 32 nrhs B of fields in and out plus
    16 B of links (the links are read once for all right-hand sides)."""
    sites = N * N
    x = torch.randn(nrhs, 2 * sites, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        h.apply_batched(0, dmg.OP_APPLY, x, y, nrhs)
    ctx.timer(dmg.KT_WILSON_BATCHED)
    for _ in range(reps):
        h.apply_batched(0, dmg.OP_APPLY, x, y, nrhs)
    ms, n, u = ctx.timer_read(dmg.KT_WILSON_BATCHED)
    ctx.timer()
    avg = ms / max(n, 1)
    byts = sites * (32 * nrhs + 16)
    gbs = byts / (avg * 1e-3) / 1e9
    return {"kernel": f"kb_wilson (FP32, {N}x{N} sites x {nrhs} right-hand sides)", "bound": "hbm",
            "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
            "avg_launch_us": avg * 1e3, "algorithmic_bytes_per_launch": byts,
            "cache_resident": byts < INFINITY_CACHE_BYTES}


def served_form(torch, dmg, ctx, sizes, ncfg, n_req, cap, inflight_max=3, age_s=0.1):
    """Serving: single-RHS requests, each naming one of the resident configurations
    (every size in `sizes` x configurations 0..ncfg-1, hierarchy and deflation space kept
    on the device), arrive as a seeded Poisson stream; each configuration has a lane
    batch (dmg_batch_*, FP32 preconditioner, `cap` lanes) that requests join and leave
    between outer cycles (continuous batching).

    Scheduler: at most `inflight_max` batch steps run at once (each batch on its own stream,
    stepped from a worker thread); whenever one ends, its finished lanes are retired and the
    next step goes to the configuration with the most work, lanes running plus waiting
    requests that fit, weighted up by the age of its oldest waiting request
    (score = lanes x (1 + wait / age_s)).  So under load the configurations that are not
    being stepped collect requests and their next step carries more lanes, while a lone
    request still gets a step once it has waited long enough.  Latency = arrival to result
    ready.

    The saturated rate (all requests at t = 0) sets the three arrival rates, 0.5x, 0.9x and
    1.2x of it.  The like-for-like comparator is the plain FP64 form serving the same mix one
    request at a time (dmg_solve, FP64 preconditioner, the same resident deflation spaces):
    its capacity is 1 / (mean solve time over the configurations), measured here."""
    import synth

    def known(N, c):
        try:
            synth.critical_mass(N, c)
            return True
        except KeyError:
            return False
    keys = [(N, c) for N in sizes for c in range(ncfg) if known(N, c)]
    res, batches = {}, {}
    prm = dmg.solve_params(precond="fp32")
    t0 = time.perf_counter()
    for k in keys:
        res[k] = build_resident(dmg, ctx, synth, *k)
        batches[k] = dmg.Batch(res[k][1], res[k][2], cap, prm)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    bytes_resident = ctx.bytes_in_use

    def requests(seed_rate, n):
        rng = synth.rng_for(0, 0, 5, seed_rate)
        picks = rng.integers(0, len(keys), size=n)
        return [(keys[p], torch.from_numpy(synth.rhs(keys[p][0], keys[p][1], 1000 + i)).cuda())
                for i, p in enumerate(picks)], rng

    # plain FP64 comparator on the same mix: mean solve time per configuration (3 requests each)
    xs = {k: torch.empty(2 * k[0] * k[0], dtype=torch.complex128, device="cuda") for k in keys}
    t_plain = {}
    for k in keys:
        g, h, d = res[k]
        bs = [torch.from_numpy(synth.rhs(k[0], k[1], 900 + j)).cuda() for j in range(4)]
        dmg.solve(ctx, h, d, bs[0], xs[k])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for b in bs[1:]:
            dmg.solve(ctx, h, d, b, xs[k])
        torch.cuda.synchronize()
        t_plain[k] = (time.perf_counter() - t1) / 3
    plain_mix = 1.0 / float(np.mean(list(t_plain.values())))
    progress(f"served: {len(keys)} configurations resident, plain FP64 on the same mix {plain_mix:.2f} solves/s")
    by_size = {N: 1.0 / float(np.mean([t_plain[k] for k in keys if k[0] == N])) for N in sizes
               if any(k[0] == N for k in keys)}

    xout = {k: torch.empty(2 * k[0] * k[0], dtype=torch.complex128, device="cuda") for k in keys}
    from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor, wait as futures_wait
    workers = ThreadPoolExecutor(max_workers=max(1, inflight_max))

    def serve(reqs, arrivals):
        queues = {k: [] for k in keys}
        busy = {k: {} for k in keys}
        inflight = {}
        lat, bad, lanes_per_step = [], 0, []
        nxt, done = 0, 0
        t_start = time.perf_counter()
        cur = torch.cuda.current_stream()  # the context's stream

        def finish(i, s):
            nonlocal bad, done
            lat.append((time.perf_counter() - t_start - arrivals[i]) * 1e3)
            bad += 0 if (s["converged"] and s["true_rel_resid"] <= 1e-8) else 1
            done += 1

        def retire_done(k):
            bt = batches[k]
            for sl in list(busy[k]):
                if bt.state(sl) == dmg.SLOT_DONE:
                    i = busy[k].pop(sl)
                    st, s = bt.retire(sl, xout[k])
                    cur.synchronize()  # the solution is in xout
                    finish(i, s)

        while done < len(reqs):
            now = time.perf_counter() - t_start
            while nxt < len(reqs) and arrivals[nxt] <= now:
                queues[reqs[nxt][0]].append(nxt)
                nxt += 1
            for k in [k for k, f in inflight.items() if f.done()]:
                inflight.pop(k).result()
                retire_done(k)
            while len(inflight) < inflight_max:
                best, best_score = None, 0.0
                for k in keys:
                    if k in inflight:
                        continue
                    lanes = len(busy[k]) + min(len(queues[k]), cap - len(busy[k]))
                    if lanes == 0:
                        continue
                    wait = now - arrivals[queues[k][0]] if queues[k] else 0.0
                    score = lanes * (1.0 + wait / age_s)
                    if score > best_score:
                        best, best_score = k, score
                if best is None:
                    break
                bt = batches[best]
                for sl in range(cap):
                    if not queues[best]:
                        break
                    if bt.state(sl) == dmg.SLOT_FREE:
                        i = queues[best].pop(0)
                        bt.admit(sl, reqs[i][1])
                        busy[best][sl] = i
                lanes_per_step.append(len(busy[best]))
                inflight[best] = workers.submit(bt.step, 1)
            if inflight:
                wait_s = arrivals[nxt] - (time.perf_counter() - t_start) if nxt < len(reqs) else None
                futures_wait(list(inflight.values()), timeout=None if wait_s is None else max(wait_s, 0.0),
                             return_when=FIRST_COMPLETED)
            elif nxt < len(reqs):
                time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t_start)))
        return (len(reqs) / (time.perf_counter() - t_start), lat, bad,
                float(np.mean(lanes_per_step)) if lanes_per_step else 0.0)

    reqs, _ = requests(0, min(n_req, 64))
    serve(reqs, [0.0] * len(reqs))  # warm the lanes of every batch in use
    reqs, _ = requests(1, n_req)
    sat, lat_sat, bad, lps = serve(reqs, [0.0] * len(reqs))
    out = {"workload": f"{len(keys)} resident configurations ({', '.join(f'{n}^2 {c}' for n, c in keys)}), "
                       f"single-RHS requests, Poisson arrivals, {cap} lanes per configuration, FP32 preconditioner, "
                       f"at most {inflight_max} batch steps at once",
           "requests_per_rate": n_req, "setup_s": setup_s, "resident_bytes": bytes_resident,
           "plain_fp64_same_mix": {"value": plain_mix, "unit": "solves/s", "by_size": by_size,
                                   "sample": "3 requests per configuration, one at a time, FP64 preconditioner, "
                                             "resident deflation spaces"},
           "saturated": {"value": sat, "unit": "solves/s", "p50_ms": percentile(lat_sat, 50),
                         "p99_ms": percentile(lat_sat, 99), "failures": bad, "mean_lanes_per_step": lps,
                         "speedup_vs_plain_fp64_same_mix": sat / plain_mix},
           "rates": []}
    progress(f"served: saturated {sat:.1f} solves/s")
    for ri, frac in enumerate((0.5, 0.9, 1.2)):
        rate = frac * sat
        reqs, rng = requests(2 + ri, n_req)
        arrivals = list(np.cumsum(rng.exponential(1.0 / rate, size=n_req)))
        thr, lat, bad, lps = serve(reqs, arrivals)
        progress(f"served: {frac} x saturated offered, {thr:.1f} solves/s delivered")
        out["rates"].append({"offered_per_s": rate, "fraction_of_saturated": frac, "value": thr, "unit": "solves/s",
                             "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99), "failures": bad,
                             "mean_lanes_per_step": lps, "speedup_vs_plain_fp64_same_mix": thr / plain_mix})
    workers.shutdown()
    for k in keys:
        batches[k].close()
        g, h, d = res[k]
        d.close()
        h.close()
        g.close()
    return out


def cpu_baseline(N, budget_s, gpu_outer_iters):
    """The oracle (numpy/scipy FP64) on the same 256^2 workload, bounded in time: the oracle's
    hierarchy of configuration 0 is built (not charged, as the GPU setup is not), then its
    right-hand sides 0, 1, ... are solved to 1e-8 one after the other (a fresh deflation space,
    so the first pays for GMRES-DR) until `budget_s` seconds have been spent; the rate counts
    completed solves only.  If not even one solve completes, the rate is extrapolated from the
    outer iterations done and the GPU run's mean outer iterations per solve.

    The reported run is limited to one thread (threadpoolctl): the scipy sparse products that
    dominate the oracle are single-threaded anyway.  A second run with the BLAS thread pools at
    the host's size (only the small dense steps use them) is reported beside it."""
    import synth
    from oracle import krylov, multigrid
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_info = threadpool_limits = None
    th = synth.gauge_angles(N, 0)
    m0 = synth.bare_mass(N, 0)
    t0 = time.perf_counter()
    H = multigrid.Hierarchy(th, m0, synth.near_null_starts(N, 0, 0), synth.near_null_starts(N, 0, 1))
    setup_s = time.perf_counter() - t0
    orig = H.cycle0

    def run(budget):
        iters = 0

        def counted_cycle(v):
            nonlocal iters
            iters += 1
            return orig(v)
        H.cycle0 = counted_cycle
        H.deflation = krylov.Deflation()  # a fresh space: the first solve pays for GMRES-DR
        solves, lat = 0, []
        t0 = time.perf_counter()
        for j in range(RHS_PER_CONFIG):
            if time.perf_counter() - t0 > budget:
                break
            t1 = time.perf_counter()
            _, info = H.solve(synth.rhs(N, 0, j))
            lat.append(time.perf_counter() - t1)
            solves += 1 if info.converged else 0
        el = time.perf_counter() - t0
        H.cycle0 = orig
        value = solves / el if solves else 1.0 / (el / max(iters, 1) * gpu_outer_iters)
        return value, el, iters, len(lat)

    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            v1, el1, it1, n1 = run(budget_s)
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    else:
        v1, el1, it1, n1 = run(budget_s)
        blas_threads = 1
    vm, elm, itm, nm = run(budget_s / 2)
    return {"value": v1, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{N}^2 configuration 0, right-hand sides 0..{n1 - 1} solved to 1e-8 in {el1:.1f} s "
                      f"({it1} outer iterations; the first solve includes GMRES-DR), one thread; oracle setup "
                      f"{setup_s:.1f} s not charged",
            "blas_threads_run": {"value": vm, "blas_threads": blas_threads, "solves": nm, "seconds": elm,
                                 "note": "scipy sparse products stay single-threaded; only small dense steps "
                                         "use the BLAS threads"},
            "cpu": platform.processor() or platform.machine(), "host_cpus": os.cpu_count()}


# ---------------------------------------------------------------- mass-gap / lattice-size scan
SCAN_METHODS = ("deflated MG with partial solves", "deflated MG", "GMRES-DR", "nondeflated MG with partial solve",
                "CGNE", "nondeflated MG")
FINE_DR_M, FINE_DR_K = 200, 40  # the paper's fine-grid GMRES-DR (the long-cycle solver)


def power_fit(sizes, values):
    """Least-squares line through (log size, log value): returns (alpha, standard error)."""
    x = np.log(np.asarray(sizes, dtype=float))
    y = np.log(np.asarray(values, dtype=float))
    A = np.stack([x, np.ones_like(x)], axis=1)
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    n = len(x)
    if n <= 2 or len(set(x.tolist())) < 2:
        return float(coef[0]), None
    resid = y - A @ coef
    s2 = float(resid @ resid) / (n - 2)
    se = np.sqrt(s2 / float(((x - x.mean()) ** 2).sum()))
    return float(coef[0]), float(se)


def scan_fits(rows, gap):
    """alpha in Mvps = size^alpha per method over the converged rows at one mass gap."""
    out = {}
    for meth in SCAN_METHODS:
        pts = [(r["N"] * r["N"], r["fine_equiv_mvps"]) for r in rows
               if r["method"] == meth and r["gap"] == gap and r["converged"]]
        if len({p[0] for p in pts}) >= 2:
            a_, se = power_fit([p[0] for p in pts], [p[1] for p in pts])
            out[meth] = {"alpha": a_, "stderr": se, "points": len(pts)}
    return out


def scan_merge(paths, fit_gap):
    """Rows of several scan runs (each file's last line is a --scan JSON line) combined and refitted."""
    runs = []
    for path in paths:
        with open(path) as f:
            runs.append(json.loads([ln for ln in f.read().splitlines() if ln.strip()][-1]))
    rows = [r for run in runs for r in run["rows"]]
    gaps = sorted({r["gap"] for r in rows}, reverse=True)
    return {"scan": runs[0]["scan"], "merged_from": paths, "sizes": sorted({r["N"] for r in rows}),
            "configs": {str(N): sorted({r["cfg"] for r in rows if r["N"] == N}) for N in sorted({r["N"] for r in rows})},
            "gaps": gaps, "rhs_per_config": runs[0]["rhs_per_config"], "fit_gap": fit_gap,
            "size_measure": "lattice sites", "alpha_fits": scan_fits(rows, fit_gap),
            "alpha_fits_by_gap": {f"{gap:g}": scan_fits(rows, gap) for gap in gaps},
            "fine_gmres_dr": runs[0]["fine_gmres_dr"], "coarse_deflation": runs[0]["coarse_deflation"],
            "configs_without_stored_mass": sorted({c for run in runs for c in run["configs_without_stored_mass"]}),
            "rows": rows, "wall_s": sum(run["wall_s"] for run in runs)}


def scan(torch, dmg, ctx, sizes, ncfg, gaps, fit_gap, nrhs, coarse=(200, 40), first=0):
    """Fine-equivalent Mvps (eq. (1)) of six solvers over mass gaps m0 - m_c and lattice sizes,
    on the synthetic ensembles (not the paper's configurations): deflated multigrid with the
    partial intermediate solve (the default), deflated multigrid with intermediate smoothing
    only and the 1e-15 / 1e-8 coarse schedule, the same two without deflation (coarse CGNE to
    1e-8), fine-grid GMRES-DR and fine-grid CGNE.  Each configuration gets its own hierarchy at
    each mass and a fresh deflation space; right-hand sides 0 .. nrhs-1 are solved in turn.
    The power alpha in Mvps = size^alpha is fitted over sizes at the fit gap, with size the
    number of lattice sites (alpha per lattice extent is twice that)."""
    import synth
    gaps = sorted(set(gaps + [fit_gap]), reverse=True)
    rows = []
    t_start = time.perf_counter()
    skipped = []
    for N in sizes:
        for c in range(first, first + ncfg):
            try:
                mc = synth.critical_mass(N, c)
            except KeyError:
                skipped.append(f"{N}/{c}")
                continue
            g = dmg.Gauge(ctx, synth.gauge_angles(N, c))
            B = [torch.from_numpy(synth.rhs(N, c, j)).cuda() for j in range(nrhs)]
            X = torch.empty_like(B[0])
            for gap in gaps:
                t0 = time.perf_counter()
                h = dmg.Hierarchy(ctx, g, mc + gap, torch.from_numpy(synth.near_null_starts(N, c, 0)).cuda(),
                                  torch.from_numpy(synth.near_null_starts(N, c, 1)).cuda())
                torch.cuda.synchronize()
                setup_s = time.perf_counter() - t0
                for meth in SCAN_METHODS:
                    d = dmg.Deflation(h, *coarse) if meth.startswith("deflated") else None
                    prm = dmg.solve_params()
                    if meth in ("deflated MG", "nondeflated MG"):
                        prm = dmg.solve_params(int_mode=1, coarse_tol_first=1e-15, coarse_tol_later=1e-8)
                    per = []
                    t1 = time.perf_counter()
                    for j in range(nrhs):
                        if meth == "GMRES-DR":
                            st, ss = dmg.solve_fine(ctx, h, dmg.FINE_GMRES_DR, B[j], X, m=FINE_DR_M, k=FINE_DR_K,
                                                    max_iters=20000)
                        elif meth == "CGNE":
                            st, ss = dmg.solve_fine(ctx, h, dmg.FINE_CGNE, B[j], X, max_iters=200000)
                        else:
                            st, ss = dmg.solve(ctx, h, d, B[j], X, params=prm)
                        per.append(ss[0])
                    torch.cuda.synchronize()
                    el = time.perf_counter() - t1
                    if d is not None:
                        d.close()
                    row = {"N": N, "cfg": c, "gap": gap, "method": meth,
                           "fine_equiv_mvps": float(np.mean([s["fine_equiv_mvps"] for s in per])),
                           "fine_mvps": float(np.mean([s["fine_mvps"] for s in per])),
                           "int_mvps": float(np.mean([s["int_mvps"] for s in per])),
                           "coarse_mvps": float(np.mean([s["coarse_mvps"] for s in per])),
                           "outer_iters": float(np.mean([s["outer_iters"] for s in per])),
                           "converged": all(s["converged"] == 1 for s in per),
                           "max_true_rel_resid": float(max(s["true_rel_resid"] for s in per)),
                           "seconds": el, "setup_s": setup_s}
                    rows.append(row)
                    print(f"[scan] {N}^2 cfg {c} gap {gap:g} {meth}: {row['fine_equiv_mvps']:.0f} fine-equivalent "
                          f"Mvps, converged {row['converged']}, {el:.1f} s", file=sys.stderr, flush=True)
                h.close()
            g.close()
    fits = scan_fits(rows, fit_gap)
    fits_by_gap = {f"{gap:g}": scan_fits(rows, gap) for gap in gaps}
    return {"scan": "fine-equivalent Mvps vs mass gap and lattice size (synthetic ensembles)",
            "sizes": sizes, "configs_per_size": ncfg, "first_config": first, "gaps": gaps, "rhs_per_config": nrhs,
            "fit_gap": fit_gap, "size_measure": "lattice sites", "alpha_fits": fits,
            "alpha_fits_by_gap": fits_by_gap,
            "fine_gmres_dr": [FINE_DR_M, FINE_DR_K], "coarse_deflation": list(coarse),
            "configs_without_stored_mass": skipped, "rows": rows,
            "wall_s": time.perf_counter() - t_start}


if __name__ == "__main__":
    main()
