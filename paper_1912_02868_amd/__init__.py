"""Deflated adaptive-multigrid Wilson-Dirac solver for AMD MI355X (gfx950).

The solver lives in the HIP library ``libdmg.so`` (sources under ``csrc/``,
C-ABI in ``include/dmg.h``); this package holds its build script and a thin
ctypes binding.  There is no CPU fallback: without the built library every call
raises.
"""
from .dmg import (  # noqa: F401
    Context, Gauge, Hierarchy, Deflation, Batch, Pool, DmgError, apply_dirac, solve, solve_batched, solve_fine, FINE_CGNE, FINE_GMRES_DR, FINE_GMRES_PROJ, solve_params, setup_params, lib,
    FP64, FP32, FP32_BF16, FP32_BF16C, PTR_HOST, PTR_DEVICE, PART_NULLVECS, PART_P, PART_BLOCKS, PART_SETUP_ITERS,
    OP_APPLY, OP_APPLY_DAG, OP_RESTRICT, OP_PROLONG, DMG_OK, DMG_W_NOT_CONVERGED, DMG_E_INVALID,
    DMG_E_NONFINITE, DMG_E_BUDGET, DMG_E_BREAKDOWN, EXPORTED, LIB_PATH, KT_COARSE_PROJ, KT_BLOCK_APPLY_INT, KT_BLOCK_BATCHED, KT_WILSON_BATCHED,
    SLOT_FREE, SLOT_RUNNING, SLOT_DONE, POOL_MAX_SLOTS, BATCH_MAX_LANES,
    autotune, autotune_force, autotune_report, TUNE_BLOCK, TUNE_WILSON,
)
