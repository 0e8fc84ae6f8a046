"""CPU checks of the boundary: the built library loads and exports every entry
point that include/dmg.h declares, and the binding mirrors the header's structs."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmg.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dmg_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["dmg_context_create", "dmg_gauge_create", "dmg_apply_dirac", "dmg_setup", "dmg_solve",
              "dmg_deflation_create", "dmg_deflation_build", "dmg_hierarchy_export", "dmg_hierarchy_apply"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1912_02868_amd as dmg
    if not os.path.exists(dmg.LIB_PATH):
        pytest.skip("libdmg.so not built")
    lib = ctypes.CDLL(dmg.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(dmg.EXPORTED) == _declared()


def test_struct_layouts_match_header(tmp_path):
    """sizeof/offsetof of the header's structs, compiled by the C compiler, equal the binding's."""
    import shutil
    import subprocess
    import paper_1912_02868_amd.dmg as b
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "sz.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "dmg.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(dmg_solve_params), sizeof(dmg_setup_params),'
        ' sizeof(dmg_solve_stats), sizeof(dmg_allocator), offsetof(dmg_solve_params, precond),'
        ' offsetof(dmg_solve_stats, true_rel_resid), offsetof(dmg_solve_stats, elapsed_ms)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(b.SolveParams), ctypes.sizeof(b.SetupParams), ctypes.sizeof(b.SolveStats),
            ctypes.sizeof(b.Allocator), b.SolveParams.precond.offset, b.SolveStats.true_rel_resid.offset,
            b.SolveStats.elapsed_ms.offset]
    assert got == want


def test_defaults_without_gpu():
    import paper_1912_02868_amd as dmg
    if not os.path.exists(dmg.LIB_PATH):
        pytest.skip("libdmg.so not built")
    p = dmg.solve_params()
    assert (p.tol, p.outer_m, p.smooth_steps, p.int_tol, p.int_m, p.int_max_iters) == (1e-8, 8, 2, 0.2, 8, 16)
    assert (p.coarse_tol_first, p.coarse_tol_later, p.precond, p.use_x0) == (1e-8, 1e-2, dmg.FP64, 0)
    s = dmg.setup_params()
    assert (s.nvec, s.null_tol, s.null_max_iters) == (12, 1e-4, 2000)


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_bench_power_fit():
    """The scan's power-law fit: an exact power law gives its exponent with zero error; with
    multiplicative noise the estimate stays within a few standard errors of the truth."""
    import numpy as np
    import bench
    sizes = np.array([64, 128, 256, 64, 128, 256], dtype=float) ** 2
    a, se = bench.power_fit(sizes, 7.0 * sizes ** 0.37)
    assert abs(a - 0.37) < 1e-12 and se < 1e-12
    rng = np.random.default_rng(5)
    vals = 7.0 * sizes ** 0.37 * np.exp(0.05 * rng.standard_normal(len(sizes)))
    a, se = bench.power_fit(sizes, vals)
    assert se > 0 and abs(a - 0.37) < 4 * se
    a, se = bench.power_fit([100.0, 100.0], [3.0, 4.0])
    assert se is None


def test_bench_coarse_traffic_matches_its_profile():
    """The HBM bytes per launch that bench.py reports for the persistent coarse kernel are the
    counter values recorded in profiles/k_coarse_proj_256_hbm_traffic.md (FETCH_SIZE x 2 plus
    WRITE_SIZE, KiB per dispatch, the scale factors the reference kernels of known size give)."""
    import bench
    txt = open(os.path.join(ROOT, "profiles", "k_coarse_proj_256_hbm_traffic.md")).read()
    row = re.search(r"\|\s*`k_coarse_proj<double, false, true, true>`\s*\|\s*(\d+)\s*\|\s*([\d,.]+)\s*\|\s*([\d,.]+)\s*\|",
                    txt)
    assert row, "coarse kernel row missing from the traffic profile"
    fetch, write = (float(row.group(k).replace(",", "")) for k in (2, 3))
    ref = re.search(r"\|\s*`vectorized_elementwise_kernel<\.\.\. mul \.\.\.>`[^|]*\|\s*\d+\s*\|\s*([\d,.]+)\s*\|\s*([\d,.]+)\s*\|",
                    txt)
    assert ref, "reference kernel row missing from the traffic profile"
    # the reference kernel reads and writes 256 MiB per launch: the counters' scale factors
    fscale = 262144.0 / float(ref.group(1).replace(",", ""))
    wscale = 262144.0 / float(ref.group(2).replace(",", ""))
    assert abs(fscale - 2.0) < 0.01 and abs(wscale - 1.0) < 0.01
    expect = (round(fscale) * fetch + round(wscale) * write) * 1024
    assert abs(bench.COARSE_TRAFFIC_BYTES - expect) <= 1024
