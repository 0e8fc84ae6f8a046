"""The entry point that allocates nothing (dmg_hierarchy_apply_batched_static), through the C-ABI.

Two calls in a row, the second with a smaller input, each compared with
dmg_hierarchy_apply_batched on the same fields (bitwise: the same kernels) and with
the FP64 oracle's operators (1e-13 FP64, 2e-6 FP32).  The library's device memory
accounting and torch's allocator statistics do not move during the calls, and a
request larger than the static scratch fails with DMG_E_INVALID.
"""
import gc

import numpy as np
import pytest

import synth
from oracle import multigrid

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_02868_amd as dmg
    dmg.lib()
    ctx = dmg.Context(0)
    N, cfg = 64, 0
    th = synth.gauge_angles(N, cfg)
    m0 = synth.bare_mass(N, cfg)
    H = multigrid.Hierarchy(th, m0, synth.near_null_starts(N, cfg, 0), synth.near_null_starts(N, cfg, 1))
    g = dmg.Gauge(ctx, th)
    hg = dmg.Hierarchy(ctx, g, m0, np.ascontiguousarray(H.levels[0].null), np.ascontiguousarray(H.levels[1].null),
                       inject=True)
    return dmg, ctx, H, g, hg


def _fields(n, nrhs, seed, dtype):
    return np.stack([synth.gaussian_complex(n, 64, seed, 11, r) for r in range(nrhs)]).astype(dtype)


def _check(dmg, ctx, H, hg, level, op, nrhs, dtype):
    A = H.levels[level].A
    P = H.levels[min(level, 1)].P if op != dmg.OP_APPLY else None
    n_in = A.shape[0] if op != dmg.OP_PROLONG else P.shape[1]
    n_out = A.shape[0] if op != dmg.OP_RESTRICT else P.shape[1]
    x = torch.from_numpy(_fields(n_in, nrhs, 10 * level + op, dtype)).cuda()
    y_static = torch.full((nrhs, n_out), complex(np.nan, np.nan), dtype=x.dtype, device="cuda")
    y_alloc = torch.empty_like(y_static)
    # objects of earlier tests that wait for the cycle collector release their device memory
    # through torch's allocator whenever it runs: collect them first and keep it off meanwhile
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        used, torch_bytes = ctx.bytes_in_use, torch.cuda.memory_allocated()
        hg.apply_batched_static(level, op, x, y_static, nrhs)
        torch.cuda.synchronize()
        assert ctx.bytes_in_use == used and torch.cuda.memory_allocated() == torch_bytes
    finally:
        gc.enable()
    hg.apply_batched(level, op, x, y_alloc, nrhs)
    torch.cuda.synchronize()
    ys, ya, xh = y_static.cpu().numpy(), y_alloc.cpu().numpy(), x.cpu().numpy().astype(complex)
    assert np.array_equal(ys, ya)
    M = A if op == dmg.OP_APPLY else (P.conj().T if op == dmg.OP_RESTRICT else P)
    tol = 1e-13 if dtype == np.complex128 else 2e-6
    for r in range(nrhs):
        ref = M @ xh[r]
        assert np.linalg.norm(ys[r] - ref) / np.linalg.norm(ref) < tol, (level, op, r)


def test_two_calls_second_smaller(setup):
    dmg, ctx, H, g, hg = setup
    _check(dmg, ctx, H, hg, 1, dmg.OP_APPLY, 40, np.complex64)    # 16^2 x 24 dof x 64 lanes, matrix cores
    _check(dmg, ctx, H, hg, 0, dmg.OP_APPLY, 5, np.complex128)    # 64^2 x 2 dof x 8 lanes, FP64
    _check(dmg, ctx, H, hg, 0, dmg.OP_RESTRICT, 3, np.complex128)
    _check(dmg, ctx, H, hg, 1, dmg.OP_PROLONG, 2, np.complex64)


def test_request_beyond_the_scratch_is_refused(setup):
    """256^2 fine fields in FP64 with 64 lanes need 2 x 128 MiB of lane-interleaved copies,
    more than the 64 MiB array: refused before anything is launched (the output keeps its
    contents); 8 lanes (2 x 16 MiB) fit and agree with the allocating entry point."""
    dmg, ctx, H, g, hg = setup
    N = 256
    g2 = dmg.Gauge(ctx, synth.gauge_angles(N, 0))
    h2 = dmg.Hierarchy(ctx, g2, synth.bare_mass(N, 0), synth.near_null_starts(N, 0, 0),
                       synth.near_null_starts(N, 0, 1))
    n = 2 * N * N
    x = torch.from_numpy(_fields(n, 64, 99, np.complex128)).cuda()
    y = torch.zeros_like(x)
    with pytest.raises(dmg.DmgError) as e:
        h2.apply_batched_static(0, dmg.OP_APPLY, x, y, 64)
    assert e.value.code == dmg.DMG_E_INVALID and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert not torch.any(y != 0).item()
    h2.apply_batched_static(0, dmg.OP_APPLY, x[:8].contiguous(), y[:8], 8)
    ya = torch.empty_like(y[:8])
    h2.apply_batched(0, dmg.OP_APPLY, x[:8].contiguous(), ya, 8)
    torch.cuda.synchronize()
    assert torch.equal(y[:8], ya)
    h2.close()
    g2.close()
