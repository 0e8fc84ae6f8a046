"""Pins for the oracle's Wilson-Dirac operator (Methods section): closed-form
free-field spectrum and plane-wave action, gamma_5-hermiticity, gauge
covariance and the exact mass shift."""
import numpy as np
import pytest

import synth
from oracle import wilson


def _free_theta(Nx, Nt):
    return np.zeros((Nt, Nx, 2))


@pytest.mark.parametrize("Nx,Nt,m0", [(6, 6, 0.3), (8, 6, -0.1), (4, 8, 0.0)])
def test_free_field_spectrum_closed_form(Nx, Nt, m0):
    D = wilson.dirac_matrix(_free_theta(Nx, Nt), m0).toarray()
    lam = np.linalg.eigvals(D)
    ref = wilson.free_field_eigenvalues(Nx, Nt, m0)
    # match as multisets: sort by (real, imag) after rounding
    key = lambda z: (np.round(z.real, 9), np.round(z.imag, 9))
    a = np.array(sorted(lam, key=key))
    b = np.array(sorted(ref, key=key))
    assert np.max(np.abs(a - b)) < 1e-12


def test_free_field_plane_wave_action():
    """D e^{i p.s} u = [m0 + sum(1 - cos p) + i sum gamma_mu sin p_mu] u fixes the sign
    convention of the hopping terms, which the spectrum alone does not."""
    Nx, Nt, m0 = 8, 6, 0.17
    D = wilson.dirac_matrix(_free_theta(Nx, Nt), m0)
    rng = np.random.default_rng(5)
    g0 = np.array([[0, 1], [1, 0]], complex)
    g1 = np.array([[0, -1j], [1j, 0]], complex)
    for kx, kt in [(0, 0), (1, 2), (3, 5), (7, 1)]:
        px, pt = 2 * np.pi * kx / Nx, (2 * kt + 1) * np.pi / Nt
        u = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        t, x = np.meshgrid(np.arange(Nt), np.arange(Nx), indexing="ij")
        phase = np.exp(1j * (px * x + pt * t)).ravel()
        psi = (phase[:, None] * u[None, :]).ravel()
        Dp = (m0 + (1 - np.cos(px)) + (1 - np.cos(pt))) * np.eye(2) + 1j * (g0 * np.sin(px) + g1 * np.sin(pt))
        want = (phase[:, None] * (Dp @ u)[None, :]).ravel()
        assert np.max(np.abs(D @ psi - want)) < 1e-13


def test_gamma5_hermiticity():
    th = synth.gauge_angles(8, 3)
    D = wilson.dirac_matrix(th, 0.05)
    g5 = wilson.gamma5_vector(64)
    lhs = (g5[:, None] * D.toarray()) * g5[None, :]
    assert np.max(np.abs(lhs - D.conj().T.toarray())) < 1e-14


def test_gauge_covariance():
    """D[U^g] = G D[U] G^dagger with U^g_mu(s) = g(s) U_mu(s) conj(g(s + mu))."""
    N = 8
    th = synth.gauge_angles(N, 1)
    rng = np.random.default_rng(11)
    alpha = rng.uniform(-np.pi, np.pi, size=(N, N))  # alpha[t, x]
    thg = th.copy()
    thg[..., 0] += alpha - np.roll(alpha, -1, axis=1)
    thg[..., 1] += alpha - np.roll(alpha, -1, axis=0)
    D = wilson.dirac_matrix(th, 0.2).toarray()
    Dg = wilson.dirac_matrix(thg, 0.2).toarray()
    G = np.repeat(np.exp(1j * alpha.ravel()), 2)
    assert np.max(np.abs(Dg - (G[:, None] * D) * np.conj(G)[None, :])) < 1e-13
    ev = np.sort_complex(np.round(np.linalg.eigvals(D), 10))
    evg = np.sort_complex(np.round(np.linalg.eigvals(Dg), 10))
    assert np.max(np.abs(ev - evg)) < 1e-9


def test_mass_shift_exact():
    th = synth.gauge_angles(8, 2)
    D0 = wilson.dirac_matrix(th, 0.0)
    D1 = wilson.dirac_matrix(th, 0.37)
    diff = (D1 - D0).toarray()
    off = diff - np.diag(np.diag(diff))
    assert np.array_equal(off, np.zeros_like(off))        # hopping terms untouched
    assert np.max(np.abs(np.diag(diff) - 0.37)) < 1e-15   # (m0 + 2) - 2 up to rounding


def test_antiperiodic_sign_only_on_last_slice():
    th = np.zeros((4, 4, 2))
    U = wilson.fermion_links(th, True)
    assert np.all(U[1, -1] == -1) and np.all(U[1, :-1] == 1) and np.all(U[0] == 1)
