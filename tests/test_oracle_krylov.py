"""Pins for the oracle's Krylov solvers: dense LU, special cases that reduce to
plain GMRES, the Arnoldi relation kept by GMRES-DR, harmonic Ritz values from an
independent generalized eigenproblem, and the GMRES-Proj projection against an
explicit least-squares fit."""
import numpy as np
import scipy.linalg as sla
import pytest

import synth
from oracle import krylov, wilson


def _dirac(N=8, cfg=0, m0=0.1):
    return wilson.dirac_matrix(synth.gauge_angles(N, cfg), m0)


def _op(A):
    return lambda v: A @ v


def test_cg_against_lu():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((40, 40)) + 1j * rng.standard_normal((40, 40))
    A = M @ M.conj().T + 0.5 * np.eye(40)
    b = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    x, it = krylov.cg(_op(A), b, 1e-13)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) / np.linalg.norm(x) < 1e-10


@pytest.mark.parametrize("N", [4, 8])
def test_gmres_against_dense_lu(N):
    A = _dirac(N, 1, 0.2)
    b = synth.rhs(N, 1, 0)
    x, info = krylov.gmres(_op(A), b, 8, 1e-13, max_iters=4000)
    xr = np.linalg.solve(A.toarray(), b)
    assert info.converged
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) < 1e-10


def test_fgmres_identity_preconditioner_is_gmres():
    A = _dirac(8, 2, 0.1)
    b = synth.rhs(8, 2, 0)
    x1, i1 = krylov.gmres(_op(A), b, 8, 1e-10, max_iters=2000)
    x2, i2 = krylov.fgmres(_op(A), b, 8, 1e-10, M=lambda v: v.copy(), max_iters=2000)
    assert i1.iters == i2.iters
    assert np.allclose(i1.history, i2.history, rtol=1e-8, atol=0)
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-10


def test_fgmres_exact_preconditioner_one_step():
    A = _dirac(8, 2, 0.1)
    Ad = A.toarray()
    b = synth.rhs(8, 2, 0)
    x, info = krylov.fgmres(_op(A), b, 8, 1e-10, M=lambda v: np.linalg.solve(Ad, v))
    assert info.iters == 1 and info.converged


def test_gmres_steps_residual_from_arnoldi_relation():
    A = _dirac(8, 0, 0.1)
    v = synth.rhs(8, 0, 3)
    y, r = krylov.gmres_steps(_op(A), v, 2)
    assert np.linalg.norm(r - (v - A @ y)) < 1e-13 * np.linalg.norm(v)
    # two steps of GMRES minimise over span{v, Av}: compare with explicit least squares
    K = np.column_stack([v, A @ v])
    c = np.linalg.lstsq(A @ K, v, rcond=None)[0]
    assert np.linalg.norm(y - K @ c) < 1e-11 * np.linalg.norm(y)


def _independent_harmonic_ritz(A, V):
    """Harmonic Ritz values w.r.t. span(V): (AV)^H (AV) g = theta (AV)^H V g."""
    W = A @ V
    return sla.eigvals(W.conj().T @ W, W.conj().T @ V)


def test_harmonic_ritz_matches_generalized_eigenproblem():
    A = _dirac(8, 3, 0.05).toarray()
    b = synth.rhs(8, 3, 0)
    cr = krylov.fgmres_cycle(_op(A), b, 20, -1.0)
    theta, G = krylov.harmonic_ritz(cr.H, 20)
    ref = _independent_harmonic_ritz(A, cr.V[:, :20])
    for t in theta:
        assert np.min(np.abs(ref - t)) < 1e-9 * max(1, abs(t))
    # the k kept are the smallest in magnitude
    theta5, _ = krylov.harmonic_ritz(cr.H, 5)
    assert np.max(np.abs(np.sort(np.abs(theta5)) - np.sort(np.abs(ref))[:5])) < 1e-9


def test_gmres_dr_relation_and_monotone_residual():
    A = _dirac(8, 0, 0.02)
    b = synth.rhs(8, 0, 1)
    x, info, defl = krylov.gmres_dr(_op(A), b, 20, 6, 1e-10)
    assert info.converged
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) < 2e-10
    k = defl.k
    assert k == 6
    rel = np.linalg.norm(A @ defl.V[:, :k] - defl.V @ defl.H) / np.linalg.norm(defl.H)
    assert rel < 1e-12
    assert np.linalg.norm(defl.V.conj().T @ defl.V - np.eye(k + 1)) < 1e-12
    h = np.array(info.history)
    assert np.all(np.diff(h) <= 1e-12)


def test_gmres_dr_relation_after_every_restart(monkeypatch):
    A = _dirac(8, 1, 0.02)
    b = synth.rhs(8, 1, 1)
    seen = []
    orig = krylov._compress

    def spy(V, H, k, s=None):
        out = orig(V, H, k, s)
        if s is not None:
            Vk1, Hk = out[0], out[1]
            seen.append(np.linalg.norm(A @ Vk1[:, :k] - Vk1 @ Hk) / np.linalg.norm(Hk))
        return out
    monkeypatch.setattr(krylov, "_compress", spy)
    krylov.gmres_dr(_op(A), b, 15, 5, 1e-10)
    assert len(seen) >= 2 and max(seen) < 1e-12


def test_gmres_dr_unreachable_tolerance_stops():
    """Tolerance 1e-15 is below what FP64 reaches on this system: the stagnation exit ends
    the solve near the arithmetic's floor, and the stored space still satisfies
    A V_k = V_{k+1} Hbar_k."""
    A = _dirac(8, 0, 0.02)
    b = synth.rhs(8, 0, 3)
    x, info, defl = krylov.gmres_dr(_op(A), b, 20, 6, 1e-15, max_cycles=200)
    assert info.cycles < 200
    assert info.stagnated or info.converged
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) < 1e-12
    k = defl.k
    rel = np.linalg.norm(A @ defl.V[:, :k] - defl.V @ defl.H) / np.linalg.norm(defl.H)
    assert rel < 1e-10


def test_gmres_dr_slow_stretch_above_floor_continues():
    """A cycle with less than 1 % progress ends GMRES-DR only in the rounding regime: on the
    cyclic shift plus 0.05 I (eigenvalues on the unit circle moved by 0.05) a
    short restarted cycle from e_1 leaves the residual at 0.9987, far above
    the floor, so the solve runs to its cycle cap instead of calling that stagnation; with
    the floor raised to 1 it stops after two cycles."""
    n = 24
    A = np.roll(np.eye(n), 1, axis=0).astype(complex) + 0.05 * np.eye(n)
    b = np.zeros(n, dtype=complex)
    b[0] = 1.0
    x, info, _ = krylov.gmres_dr(_op(A), b, 6, 2, 1e-8, max_cycles=7)
    assert not info.stagnated and not info.converged and info.cycles == 7
    assert all(h > 0.99 for h in info.history)
    x, info, _ = krylov.gmres_dr(_op(A), b, 6, 2, 1e-8, max_cycles=7, stall_floor=1.0)
    assert info.stagnated and info.cycles == 2


def test_gmres_dr_k0_is_gmres():
    A = _dirac(8, 2, 0.05)
    b = synth.rhs(8, 2, 2)
    x1, i1, _ = krylov.gmres_dr(_op(A), b, 12, 0, 1e-9)
    x2, i2 = krylov.gmres(_op(A), b, 12, 1e-9, max_iters=5000)
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x2) < 1e-7
    assert abs(i1.iters - i2.iters) <= 1


def test_gmres_dr_ritz_values_converge_to_smallest_eigenvalues():
    A = _dirac(8, 0, 0.02).toarray()
    b = synth.rhs(8, 0, 2)
    x, info, defl = krylov.gmres_dr(_op(A), b, 40, 8, 1e-14)
    lam = np.linalg.eigvals(A)
    small = lam[np.argsort(np.abs(lam))[:4]]
    for t in small:
        assert np.min(np.abs(defl.theta - t)) < 1e-6


def test_gmres_proj_empty_space_is_gmres():
    A = _dirac(8, 2, 0.05)
    b = synth.rhs(8, 2, 3)
    x1, i1 = krylov.gmres_proj(_op(A), b, krylov.Deflation(), 10, 1e-8)
    x2, i2 = krylov.gmres(_op(A), b, 10, 1e-8, max_iters=5000)
    assert abs(i1.iters - i2.iters) <= 1
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x2) < 1e-6


def test_gmres_proj_projection_is_explicit_least_squares():
    A = _dirac(8, 3, 0.02)
    b = synth.rhs(8, 3, 0)
    _, _, defl = krylov.gmres_dr(_op(A), b, 20, 6, 1e-10)
    r = synth.rhs(8, 3, 1)
    k = defl.k
    # one projection step (what GMRES-Proj does before its first GMRES cycle)
    c = defl.V.conj().T @ r
    d = np.linalg.lstsq(defl.H, c, rcond=None)[0]
    AV = A @ defl.V[:, :k]
    d_ref = np.linalg.lstsq(AV, r, rcond=None)[0]
    assert np.linalg.norm(d - d_ref) / np.linalg.norm(d_ref) < 1e-9
    x, info = krylov.gmres_proj(_op(A), r, defl, 20, 1e-9)
    assert info.converged and np.linalg.norm(r - A @ x) / np.linalg.norm(r) < 1e-8
