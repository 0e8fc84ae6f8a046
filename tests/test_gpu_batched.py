"""Lockstep multi-right-hand-side solve (dmg_solve_batched) through the C-ABI.

Each right-hand side must reach the true relative residual 1e-8 (checked with the
oracle's operator) and its solution must agree with a sparse-LU solve within the
a-posteriori bound at that residual; padding (nrhs not a power of two), a zero
right-hand side and the argument errors are covered.
"""
import numpy as np
import pytest

import synth
from oracle import wilson

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dmg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_02868_amd as dmg
    dmg.lib()
    return dmg


@pytest.fixture(scope="module")
def ctx(dmg):
    return dmg.Context(0)


@pytest.fixture(scope="module")
def cfg64(dmg, ctx):
    N, cfg = 64, 0
    th = synth.gauge_angles(N, cfg)
    m0 = synth.bare_mass(N, cfg)
    g = dmg.Gauge(ctx, th)
    h = dmg.Hierarchy(ctx, g, m0, synth.near_null_starts(N, cfg, 0), synth.near_null_starts(N, cfg, 1))
    d = dmg.Deflation(h, 30, 10)
    d.build(synth.gaussian_complex(24 * (N // 16) ** 2, N, cfg, 4, 0), 1e-8)
    D = wilson.dirac_matrix(th, m0)
    import scipy.sparse.linalg as spla
    lu = spla.splu(D.tocsc())
    return th, m0, g, h, d, D, lu


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("precond", ["fp64", "fp32", "fp32_bf16"])
def test_batched_64(dmg, ctx, cfg64, precond):
    th, m0, g, h, d, D, lu = cfg64
    nrhs = 6  # padded to 8 lanes
    b = np.stack([synth.rhs(64, 0, j) for j in range(nrhs)])
    b[4] = 0.0  # a zero right-hand side solves to x = 0 at once
    x = np.empty_like(b)
    st, stats = dmg.solve_batched(ctx, h, d, b, x, nrhs, params=dmg.solve_params(precond=precond))
    assert st == dmg.DMG_OK
    for j in range(nrhs):
        s = stats[j]
        assert s["converged"] == 1, (j, s)
        if j == 4:
            assert np.all(x[j] == 0) and s["outer_iters"] == 0
            continue
        res = np.linalg.norm(b[j] - D @ x[j]) / np.linalg.norm(b[j])
        assert res <= 1e-8 * (1 + 1e-6) and abs(res - s["true_rel_resid"]) < 1e-12, (j, res, s)
        assert _rel(x[j], lu.solve(b[j])) < 1e-6
        assert 0 < s["outer_iters"] <= 40 and s["coarse_mvps"] > 0 and s["int_mvps"] > 0


def test_batched_single_and_device(dmg, ctx, cfg64):
    th, m0, g, h, d, D, lu = cfg64
    b = synth.rhs(64, 0, 7)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    st, stats = dmg.solve_batched(ctx, h, d, bd, xd, 1)
    torch.cuda.synchronize()
    x = xd.cpu().numpy()
    assert st == dmg.DMG_OK and stats[0]["converged"] == 1
    assert np.linalg.norm(b - D @ x) / np.linalg.norm(b) <= 1e-8 * (1 + 1e-6)
    # the single-field solver reaches the same solution within the residual bound
    xs = np.empty_like(b)
    dmg.solve(ctx, h, d, b, xs)
    assert _rel(x, xs) < 1e-6


def test_batched_errors(dmg, ctx, cfg64):
    th, m0, g, h, d, D, lu = cfg64
    b = np.stack([synth.rhs(64, 0, j) for j in range(2)])
    x = np.empty_like(b)
    fresh = dmg.Deflation(h, 30, 10)
    for args, kw in [((h, fresh, b, x, 2), {}), ((h, d, b, x, 0), {}),
                     ((h, d, b, x, 2), {"params": dmg.solve_params(outer_m=30)}),
                     ((h, d, b, x, 2), {"params": dmg.solve_params(use_x0=1)}),
                     ((h, d, b, x, 2), {"params": dmg.solve_params(smooth_steps=3)})]:
        with pytest.raises(dmg.DmgError) as e:
            dmg.solve_batched(ctx, *args, **kw)
        assert e.value.code == dmg.DMG_E_INVALID
    fresh.close()


@pytest.mark.parametrize("precond", ["fp64", "fp32"])
def test_batched_graph_replay_matches_eager(dmg, ctx, cfg64, precond):
    """Each coarse GMRES-Proj cycle replayed from a captured HIP graph (hundreds of replays per
    solve, with host reads between them) gives bitwise the solution of launching its kernels
    one by one, on two solves in a row."""
    th, m0, g, h, d, D, lu = cfg64
    nrhs = 8
    b = np.stack([synth.rhs(64, 0, 40 + j) for j in range(nrhs)])
    out = {}
    for graphs in (1, 0, 1):
        xs = []
        for rep in range(2):
            x = np.empty_like(b)
            st, stats = dmg.solve_batched(ctx, h, d, b, x, nrhs,
                                          params=dmg.solve_params(precond=precond, graphs=graphs))
            assert st == dmg.DMG_OK and all(s["converged"] == 1 for s in stats)
            xs.append((x, [s["outer_iters"] for s in stats], [s["coarse_mvps"] for s in stats]))
        assert np.array_equal(xs[0][0], xs[1][0]) and xs[0][1:] == xs[1][1:]
        out.setdefault(graphs, []).append(xs[0])
    eager, graph = out[0][0], out[1]
    for gx in graph:
        assert np.array_equal(gx[0], eager[0]) and gx[1:] == eager[1:]
    for j in range(nrhs):
        assert np.linalg.norm(b[j] - D @ eager[0][j]) / np.linalg.norm(b[j]) <= 1e-8 * (1 + 1e-6)


# ---------------------------------------------------------------- multi-RHS kernels vs the oracle
@pytest.fixture(scope="module")
def inj64(dmg, ctx):
    from oracle import multigrid
    N, cfg = 64, 0
    th = synth.gauge_angles(N, cfg)
    m0 = synth.bare_mass(N, cfg)
    H = multigrid.Hierarchy(th, m0, synth.near_null_starts(N, cfg, 0), synth.near_null_starts(N, cfg, 1))
    g = dmg.Gauge(ctx, th)
    hg = dmg.Hierarchy(ctx, g, m0, np.ascontiguousarray(H.levels[0].null), np.ascontiguousarray(H.levels[1].null),
                       inject=True)
    return H, g, hg


def _fields(n, nrhs, seed):
    return np.stack([synth.gaussian_complex(n, 64, seed, 11, j) for j in range(nrhs)])


@pytest.mark.parametrize("prec,nrhs,mfma", [("fp64", 5, True), ("fp64", 16, True), ("fp64", 40, True),
                                            ("fp64", 16, False), ("fp32", 16, True), ("fp32", 16, False),
                                            ("fp32", 40, True), ("fp32", 3, True)])
def test_batched_operators(dmg, inj64, prec, nrhs, mfma):
    """Multi-RHS fine stencil and 24 x 24 block stencils (matrix-core path, FP32 or FP64, with
    16 or more right-hand sides) against the oracle's operators, one product per field."""
    H, g, hg = inj64
    for lvl in range(3):
        A = H.levels[lvl].A
        n = A.shape[0]
        x = _fields(n, nrhs, lvl)
        if prec == "fp32":
            x = x.astype(np.complex64)
        out = np.empty_like(x)
        hg.apply_batched(lvl, dmg.OP_APPLY, x, out, nrhs, mfma=mfma)
        for r in range(nrhs):
            ref = A @ x[r].astype(complex)
            rel = np.linalg.norm(out[r] - ref) / np.linalg.norm(ref)
            elem = np.max(np.abs(out[r] - ref)) / np.max(np.abs(ref))
            if prec == "fp64":
                assert rel < 1e-13 and elem < 1e-13, (lvl, r, rel, elem)
            else:
                assert rel < 2e-6 and elem < 1e-5, (lvl, r, rel, elem)


@pytest.mark.parametrize("nrhs", [5, 16, 40])
def test_batched_bf16_block_operator(dmg, inj64, nrhs):
    """Multi-RHS level-1 stencil with BF16-stored blocks (vector kernel below 16 right-hand
    sides, matrix cores from 16) against the oracle's blocks rounded to bfloat16."""
    from oracle.precision import bf16_round
    H, g, hg = inj64
    A16 = H.levels[1].A.tocsr(copy=True)
    A16.data = bf16_round(A16.data)
    x = _fields(A16.shape[0], nrhs, 60).astype(np.complex64)
    out = np.empty_like(x)
    hg.apply_batched(1, dmg.OP_APPLY, x, out, nrhs, bf16=True)
    for r in range(nrhs):
        ref = A16 @ x[r].astype(complex)
        rel = np.linalg.norm(out[r] - ref) / np.linalg.norm(ref)
        elem = np.max(np.abs(out[r] - ref)) / np.max(np.abs(ref))
        assert rel < 2e-6 and elem < 1e-5, (r, rel, elem)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_autotuned_forms_bitwise(dmg, inj64, prec):
    """Every launch form the autotuner may pick (block stencil: 64, 32 or 16 lanes per
    workgroup; FP32 Wilson stencil: 256, 128, 512, 64 or 1024 threads) gives bitwise the same
    product, and the tuned choice is reported per shape."""
    H, g, hg = inj64
    nrhs = 64
    try:
        for lvl, kern, nforms in ((0, dmg.TUNE_WILSON, 5), (1, dmg.TUNE_BLOCK, 3), (2, dmg.TUNE_BLOCK, 3)):
            n = H.levels[lvl].A.shape[0]
            x = _fields(n, nrhs, 40 + lvl)
            if prec == "fp32":
                x = x.astype(np.complex64)
            outs = []
            for form in range(nforms):
                dmg.autotune_force(kern, form)
                out = np.empty_like(x)
                hg.apply_batched(lvl, dmg.OP_APPLY, x, out, nrhs)
                outs.append(out)
            for out in outs[1:]:
                assert np.array_equal(out, outs[0]), (lvl, prec)
    finally:
        dmg.autotune_force(dmg.TUNE_BLOCK, -1)
        dmg.autotune_force(dmg.TUNE_WILSON, -1)
    rep = dmg.autotune_report()
    assert "block_mfma" in rep and "nb=64" in rep
    with pytest.raises(dmg.DmgError):
        dmg.autotune(3)


@pytest.mark.parametrize("prec,nrhs", [("fp64", 7), ("fp32", 16)])
def test_batched_transfers(dmg, inj64, prec, nrhs):
    H, g, hg = inj64
    for lvl in range(2):
        P = H.levels[lvl].P
        nf, nc = P.shape
        xf = _fields(nf, nrhs, 20 + lvl)
        xc = _fields(nc, nrhs, 30 + lvl)
        if prec == "fp32":
            xf, xc = xf.astype(np.complex64), xc.astype(np.complex64)
        rc = np.empty((nrhs, nc), dtype=xf.dtype)
        pf = np.empty((nrhs, nf), dtype=xf.dtype)
        hg.apply_batched(lvl, dmg.OP_RESTRICT, xf, rc, nrhs)
        hg.apply_batched(lvl, dmg.OP_PROLONG, xc, pf, nrhs)
        tol = 1e-13 if prec == "fp64" else 2e-6
        for r in range(nrhs):
            ref_r = P.conj().T @ xf[r].astype(complex)
            ref_p = P @ xc[r].astype(complex)
            assert np.linalg.norm(rc[r] - ref_r) / np.linalg.norm(ref_r) < tol
            assert np.linalg.norm(pf[r] - ref_p) / np.linalg.norm(ref_p) < tol


# ---------------------------------------------------------------- continuous batching on lanes (dmg_batch_*)
def _run_lanes(dmg, bt, cap, jobs, min_iters=1):
    queue = list(jobs)
    busy, results = {}, {}
    while queue or busy:
        for i in range(cap):
            if queue and bt.state(i) == dmg.SLOT_FREE:
                key, b = queue.pop(0)
                assert bt.admit(i, b) == dmg.DMG_OK
                busy[i] = (key, b)
        bt.step(min_iters)
        for i in list(busy):
            if bt.state(i) == dmg.SLOT_DONE:
                key, b = busy.pop(i)
                x = np.empty_like(b)
                st, s = bt.retire(i, x)
                results[key] = (x, st, s)
    return results


@pytest.mark.parametrize("precond", ["fp64", "fp32"])
def test_lanes_alone_vs_mix(dmg, ctx, cfg64, precond):
    """Requests joining and leaving lockstep lanes get bitwise the result they get alone
    (one request in a batch of the same capacity); each reaches 1e-8 with the oracle's D."""
    th, m0, g, h, d, D, lu = cfg64
    prm = dmg.solve_params(precond=precond)
    cap = 6  # 8 lanes
    jobs = [(j, synth.rhs(64, 0, 10 + j)) for j in range(11)]
    jobs[3] = (3, np.zeros_like(jobs[3][1]))
    bt = dmg.Batch(h, d, cap, prm)
    mix = _run_lanes(dmg, bt, cap, jobs)
    alone = {}
    for key, b in jobs[:5]:
        alone.update(_run_lanes(dmg, bt, cap, [(key, b)], min_iters=3))
    bt.close()
    assert set(mix) == {j for j, _ in jobs}
    for key, b in jobs:
        x, st, s = mix[key]
        assert st == dmg.DMG_OK and s["converged"] == 1
        if key == 3:
            assert np.all(x == 0) and s["outer_iters"] == 0
            continue
        res = np.linalg.norm(b - D @ x) / np.linalg.norm(b)
        assert res <= 1e-8 * (1 + 1e-6) and abs(res - s["true_rel_resid"]) < 1e-12
        if key in alone:
            assert np.array_equal(x, alone[key][0]), key


def test_lanes_device_and_errors(dmg, ctx, cfg64):
    th, m0, g, h, d, D, lu = cfg64
    for cap in (0, dmg.BATCH_MAX_LANES + 1):
        with pytest.raises(dmg.DmgError) as e:
            dmg.Batch(h, d, cap)
        assert e.value.code == dmg.DMG_E_INVALID
    fresh = dmg.Deflation(h, 30, 10)
    with pytest.raises(dmg.DmgError) as e:
        dmg.Batch(h, fresh, 4)
    assert e.value.code == dmg.DMG_E_INVALID
    fresh.close()
    bt = dmg.Batch(h, d, 4)
    b = synth.rhs(64, 0, 30)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    assert bt.admit(2, bd) == dmg.DMG_OK
    with pytest.raises(dmg.DmgError) as e:
        bt.admit(2, bd)
    assert e.value.code == dmg.DMG_E_INVALID
    with pytest.raises(dmg.DmgError) as e:
        bt.retire(2, xd)
    assert e.value.code == dmg.DMG_E_INVALID
    while bt.state(2) != dmg.SLOT_DONE:
        bt.step(8)
    st, s = bt.retire(2, xd)
    torch.cuda.synchronize()
    x = xd.cpu().numpy()
    assert st == dmg.DMG_OK and np.linalg.norm(b - D @ x) / np.linalg.norm(b) <= 1e-8 * (1 + 1e-6)
    assert bt.state(2) == dmg.SLOT_FREE and bt.state(9) == -1
    bt.close()


def test_lanes_concurrent_batches(dmg, ctx, cfg64):
    """Lane batches run on streams of their own: two batches driven at once from two
    host threads (admit, step and retire interleaved) give bitwise the results they give
    one after the other, with device right-hand sides written on the context's stream just
    before admission and device solutions read there just after retirement."""
    from concurrent.futures import ThreadPoolExecutor
    th, m0, g, h, d, D, lu = cfg64
    prm = dmg.solve_params(precond="fp32")
    cap = 4
    jobs = [[(j, synth.rhs(64, 0, 40 + j)) for j in range(6)], [(j, synth.rhs(64, 0, 50 + j)) for j in range(6)]]

    def drive(bt, js):
        queue, busy, out = list(js), {}, {}
        while queue or busy:
            for i in range(cap):
                if queue and bt.state(i) == dmg.SLOT_FREE:
                    key, b = queue.pop(0)
                    bd = torch.from_numpy(b).cuda() * 1.0  # written by a kernel on the context's stream
                    assert bt.admit(i, bd) == dmg.DMG_OK
                    busy[i] = key
            bt.step(1)
            for i in list(busy):
                if bt.state(i) == dmg.SLOT_DONE:
                    key = busy.pop(i)
                    xd = torch.full((2 * 64 * 64,), float("nan"), dtype=torch.complex128, device="cuda")
                    st, s = bt.retire(i, xd)
                    out[key] = (xd.cpu().numpy(), st, s)  # read on the context's stream
        return out

    bts = [dmg.Batch(h, d, cap, prm) for _ in range(2)]
    with ThreadPoolExecutor(max_workers=2) as ex:  # fresh batches: graphs captured at once
        both = list(ex.map(drive, bts, jobs))
    serial = [drive(bt, js) for bt, js in zip(bts, jobs)]
    for bt in bts:
        bt.close()
    for js, a, b in zip(jobs, serial, both):
        assert set(a) == set(b) == {k for k, _ in js}
        for key, rhs in js:
            x, st, s = b[key]
            assert st == dmg.DMG_OK and s["converged"] == 1
            assert np.linalg.norm(rhs - D @ x) / np.linalg.norm(rhs) <= 1e-8 * (1 + 1e-6)
            assert np.array_equal(x, a[key][0]) and s["outer_iters"] == a[key][2]["outer_iters"], key


def test_error_text_per_thread(dmg, ctx, cfg64):
    """The error text of a context is kept per host thread: a failing call on one thread
    leaves another thread's text (of its own successful calls) empty, and each thread reads
    the message of its own failure."""
    import threading
    th, m0, g, h, d, D, lu = cfg64
    bts = [dmg.Batch(h, d, 4) for _ in range(2)]
    b = synth.rhs(64, 0, 60)
    seen = {}
    ready = threading.Barrier(2)

    def bad():
        ready.wait()
        st = dmg.lib().dmg_batch_retire(bts[0].h, 7, None, dmg.PTR_HOST, None)
        seen["bad"] = (st, dmg.lib().dmg_last_error(ctx.h).decode())

    def good():
        ready.wait()
        assert bts[1].admit(0, b) == dmg.DMG_OK
        bts[1].step(1)
        seen["good"] = dmg.lib().dmg_last_error(ctx.h).decode()

    ts = [threading.Thread(target=f) for f in (bad, good)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    for bt in bts:
        bt.close()
    assert seen["bad"][0] == dmg.DMG_E_INVALID and "batch_retire" in seen["bad"][1]
    assert seen["good"] == ""
    assert dmg.lib().dmg_last_error(ctx.h).decode() == ""  # this thread made no failing call


def test_batch_over_budget(dmg, ctx, cfg64):
    """A lane batch whose workspace does not fit the context's HBM budget is refused with
    DMG_E_BUDGET (its partly built workspace and stream released), and a batch created
    afterwards under the full budget solves as usual."""
    th, m0, g, h, d, D, lu = cfg64
    before = ctx.bytes_in_use
    ctx.set_budget(before + (1 << 20))
    try:
        with pytest.raises(dmg.DmgError) as e:
            dmg.Batch(h, d, 8)
        assert e.value.code == dmg.DMG_E_BUDGET
    finally:
        ctx.set_budget(0)
    torch.cuda.synchronize()
    assert ctx.bytes_in_use == before
    b = synth.rhs(64, 0, 70)
    bt = dmg.Batch(h, d, 8)
    res = _run_lanes(dmg, bt, 8, [(0, b)])
    bt.close()
    x, st, s = res[0]
    assert st == dmg.DMG_OK and np.linalg.norm(b - D @ x) / np.linalg.norm(b) <= 1e-8 * (1 + 1e-6)
