"""Compute the critical masses of the synthetic configurations with the oracle and
store them in ``synth/mcrit.json`` (the bare mass of every workload is m_c + 0.01).

    python -m oracle.make_mcrit --sizes 64:10,128:10,256:10,512:4 --jobs 4 --redo-guard-below 1.0

Each entry is m_c = -min Re lambda(D(0)) of configuration (N, cfg); the covered search
also records the range of imaginary parts it covered (``im_guard``, see ``oracle.mcrit``).
Existing entries are kept unless --force is given.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.mcrit import critical_mass  # noqa: E402


def _one(job):
    N, cfg = job
    t0 = time.time()
    mc, guard = critical_mass(synth.gauge_angles(N, cfg))
    return N, cfg, mc, guard, time.time() - t0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="64:4,128:4,256:10,512:4", help="N:count list")
    ap.add_argument("--jobs", type=int, default=1)
    ap.add_argument("--force", action="store_true")
    ap.add_argument("--out", default=None, help="table to read and update (default: the stored one)")
    ap.add_argument("--redo-guard-below", type=float, default=0.0,
                    help="recompute entries whose covered range of imaginary parts is below this (a search "
                         "that did not cover the strip)")
    a = ap.parse_args(argv)
    path = a.out or synth.MCRIT_FILE
    method = ("oracle.mcrit.critical_mass (dense eig up to 32^2; above, shift-invert ARPACK discs covering "
              "the Bendixson strip of the leftmost eigenvalue, im_guard = the covered range of imaginary parts)")
    table = {"mc": {}, "im_guard": {}, "method": method}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    if a.force:
        table["method"] = method
    jobs = []
    for item in a.sizes.split(","):
        N, count = (int(v) for v in item.split(":"))
        for cfg in range(count):
            key = f"{N}/{cfg}"
            stale = table["im_guard"].get(key, float("inf")) < a.redo_guard_below
            if a.force or key not in table["mc"] or stale:
                jobs.append((N, cfg))
    with Pool(max(1, a.jobs)) as pool:
        for N, cfg, mc, guard, dt in pool.imap_unordered(_one, jobs):
            table["mc"][f"{N}/{cfg}"] = mc
            table["im_guard"][f"{N}/{cfg}"] = guard
            with open(path, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            print(f"{N}^2 cfg {cfg}: m_c = {mc:.12f} (im guard {guard:.3f}, {dt:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
