"""Pins for the synthetic gauge ensembles (stand-in for the paper's QCDLAB configs):
plaquettes rebuilt from the links equal the von Mises draws, the torus constraint
holds with an integer charge, and the mean plaquette matches I1(beta)/I0(beta)."""
import numpy as np
from scipy.special import iv

import synth


def _plaquettes(th):
    t0, t1 = th[..., 0], th[..., 1]
    return t0 + np.roll(t1, -1, axis=1) - np.roll(t0, -1, axis=0) - t1


def _wrap(a):
    return (a + np.pi) % (2 * np.pi) - np.pi


def test_plaquettes_match_draws():
    for N, cfg in [(8, 0), (16, 3), (64, 1)]:
        th = synth.gauge_angles(N, cfg)
        phi, hx, ht, q = synth.plaquette_draws(N, cfg)
        assert np.max(np.abs(_wrap(_plaquettes(th) - phi))) < 1e-11
        assert abs(_wrap(_plaquettes(th)).sum() - 2 * np.pi * round(_wrap(_plaquettes(th)).sum() / (2 * np.pi))) < 1e-9
        # holonomies sit where the axial gauge puts them
        assert abs(th[0, :, 0].sum() - hx) < 1e-12 and abs(th[:, 0, 1].sum() - ht) < 1e-12


def test_mean_plaquette_bessel_ratio():
    beta = 6.0
    mean_ref = iv(1, beta) / iv(0, beta)
    assert abs(mean_ref - 0.9123593044) < 1e-10
    e2 = 0.5 * (1 + iv(2, beta) / iv(0, beta))
    sigma1 = np.sqrt(e2 - mean_ref ** 2)
    vals = []
    for cfg in range(4):
        th = synth.gauge_angles(64, cfg)
        vals.append(np.cos(_plaquettes(th)).ravel())
    vals = np.concatenate(vals)
    sigma_mean = sigma1 / np.sqrt(vals.size)
    assert abs(vals.mean() - mean_ref) < 5 * sigma_mean


def test_seeds_are_distinct_and_reproducible():
    a = synth.gauge_angles(16, 0)
    assert np.array_equal(a, synth.gauge_angles(16, 0))
    assert not np.allclose(a, synth.gauge_angles(16, 1))
    r = synth.rhs(16, 0, 0)
    assert r.shape == (512,) and r.dtype == complex
    assert np.array_equal(r, synth.rhs(16, 0, 0)) and not np.allclose(r, synth.rhs(16, 0, 1))
