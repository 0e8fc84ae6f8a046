"""Pins for the oracle's multigrid setup and cycle (Methods section): block
orthonormality, chirality structure, reproduction of the near-null vectors,
Galerkin blocks against dense brute force, gamma_5-hermiticity of the coarse
operators, two-grid projector identities, and whole solves against sparse LU."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import multigrid, wilson, mcrit


def _hier(N, cfg=0, dm=0.05, null_levels=2, **kw):
    th = synth.gauge_angles(N, cfg)
    m0 = mcrit.critical_mass_dense(th) + dm if N <= 16 else kw.pop("m0")
    s0 = synth.near_null_starts(N, cfg, 0)
    s1 = synth.near_null_starts(N, cfg, 1)
    return multigrid.Hierarchy(th, m0, s0, s1, multigrid.Params(**kw)), th, m0


@pytest.fixture(scope="module")
def h16():
    return _hier(16, 2)


def test_prolongator_block_orthonormal(h16):
    H, _, _ = h16
    for lvl in range(2):
        Q = H.levels[lvl].Q
        G = np.einsum("bcri,bcrj->bcij", Q.conj(), Q)
        assert np.max(np.abs(G - np.eye(12))) < 1e-13
        P = H.levels[lvl].P
        PHP = (P.conj().T @ P).toarray()
        assert np.max(np.abs(PHP - np.eye(PHP.shape[0]))) < 1e-13


def test_prolongator_chirality(h16):
    H, _, _ = h16
    for lvl in range(2):
        L, Lc = H.levels[lvl], H.levels[lvl + 1]
        P = L.P.toarray()
        assert np.max(np.abs(L.g5[:, None] * P - P * Lc.g5[None, :])) < 1e-14


def test_prolongator_reproduces_blocked_chiral_null_vectors(h16):
    H, _, _ = h16
    for lvl in range(2):
        L = H.levels[lvl]
        ortho = multigrid.mgs2_columns(L.null.T)
        P = L.P
        for i in range(12):
            for sgn in (+1, -1):
                v = 0.5 * (1 + sgn * L.g5) * ortho[:, i]
                assert np.linalg.norm(v - P @ (P.conj().T @ v)) < 1e-12 * max(1.0, np.linalg.norm(v))


def test_near_null_tolerance(h16):
    H, _, _ = h16
    for lvl in range(2):
        A = H.levels[lvl].A
        starts = [synth.near_null_starts(16, 2, lvl)][0]
        for x, psi in zip(starts, H.levels[lvl].null):
            r = A @ (A.conj().T @ psi)
            r0 = A @ (A.conj().T @ x)
            assert np.linalg.norm(r) <= 1e-4 * np.linalg.norm(r0) * (1 + 1e-8)


def test_galerkin_blocks_against_dense_products_8():
    th = synth.gauge_angles(8, 4)
    D = wilson.dirac_matrix(th, 0.1)
    s0 = synth.near_null_starts(8, 4, 0)
    null, _ = multigrid.near_null_vectors(D, s0, 1e-4)
    P, Q = multigrid.build_prolongator(null, 8, 8, 2, wilson.gamma5_vector(64))
    Ah = multigrid.galerkin(D, P).toarray()
    Pd = P.toarray()
    dense = Pd.conj().T @ D.toarray() @ Pd
    assert np.max(np.abs(Ah - dense)) < 1e-13
    B = multigrid.stencil_blocks(multigrid.galerkin(D, P), 2, 2)
    # on a 2 x 2 coarse lattice +mu and -mu reach the same site: blocks hold the sum
    assert np.max(np.abs(B[0, 1] - dense[0:24, 24:48])) < 1e-13
    assert np.max(np.abs(B[0, 3] - dense[0:24, 48:72])) < 1e-13


def test_galerkin_three_level_chain_dense_32():
    th = synth.gauge_angles(32, 0)
    m0 = 0.1
    H = multigrid.Hierarchy(th, m0, synth.near_null_starts(32, 0, 0), synth.near_null_starts(32, 0, 1))
    D = H.levels[0].A.toarray()
    P = H.levels[0].P.toarray()
    Ph = H.levels[1].P.toarray()
    Dc_dense = (P @ Ph).conj().T @ D @ (P @ Ph)
    assert np.max(np.abs(H.levels[2].A.toarray() - Dc_dense)) < 1e-13 * np.abs(Dc_dense).max()
    # only self and nearest-neighbour blocks of the 8 x 8 intermediate and 2 x 2 coarse lattice
    Dh = H.levels[1].A.toarray()
    B = multigrid.stencil_blocks(H.levels[1].A, 8, 8)
    rebuilt = np.zeros_like(Dh)
    for T in range(8):
        for X in range(8):
            S = X + 8 * T
            nb = [S, (X + 1) % 8 + 8 * T, (X - 1) % 8 + 8 * T, X + 8 * ((T + 1) % 8), X + 8 * ((T - 1) % 8)]
            for d, S2 in enumerate(nb):
                rebuilt[24 * S:24 * S + 24, 24 * S2:24 * S2 + 24] = B[S, d]
    assert np.max(np.abs(rebuilt - Dh)) < 1e-14


def test_coarse_gamma5_hermiticity(h16):
    H, _, _ = h16
    for lvl in (1, 2):
        A = H.levels[lvl].A.toarray()
        g5 = H.levels[lvl].g5
        assert np.max(np.abs(g5[:, None] * A * g5[None, :] - A.conj().T)) < 1e-13


def test_two_grid_projector_identities(h16):
    H, _, _ = h16
    D = H.levels[0].A.toarray()
    P = H.levels[0].P.toarray()
    Dh = P.conj().T @ D @ P
    C = np.eye(D.shape[0]) - P @ np.linalg.solve(Dh, P.conj().T @ D)
    assert np.max(np.abs(C @ C - C)) < 1e-10
    assert np.max(np.abs(P.conj().T @ D @ C)) < 1e-10


def test_whole_solve_against_splu_16(h16):
    H, th, m0 = h16
    b = synth.rhs(16, 2, 0)
    x, info = H.solve(b)
    D = H.levels[0].A
    assert info.converged
    res = np.linalg.norm(b - D @ x) / np.linalg.norm(b)
    assert res <= 1e-8
    xr = spla.splu(D.tocsc()).solve(b)
    # a-posteriori bound: ||x - x*|| <= ||D^{-1}|| ||b - D x||
    smin = np.linalg.svd(D.toarray(), compute_uv=False).min()
    bound = np.linalg.norm(b - D @ x) / smin
    assert np.linalg.norm(x - xr) <= bound * (1 + 1e-6) + 1e-14
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) < 1e-6


def test_non_deflated_variant_solves(h16):
    H, th, m0 = h16
    Hn = multigrid.Hierarchy(th, m0, synth.near_null_starts(16, 2, 0), synth.near_null_starts(16, 2, 1),
                             multigrid.Params(deflate=False))
    b = synth.rhs(16, 2, 1)
    x, info = Hn.solve(b)
    assert info.converged and np.linalg.norm(b - Hn.levels[0].A @ x) / np.linalg.norm(b) <= 1e-8


def test_smoothing_only_variant_solves(h16):
    """The paper's smoothing-only intermediate treatment (one intermediate cycle instead of
    the partial solve) with the oversolved coarse schedule 1e-15 (first call, ended by the
    GMRES-DR stagnation exit) then 1e-8: the solve still reaches 1e-8 and sparse LU's
    solution."""
    H, th, m0 = h16
    Hs = multigrid.Hierarchy(th, m0, synth.near_null_starts(16, 2, 0), synth.near_null_starts(16, 2, 1),
                             multigrid.Params(intermediate="cycle", coarse_tol_first=1e-15, coarse_tol_later=1e-8))
    b = synth.rhs(16, 2, 2)
    x, info = Hs.solve(b)
    D = Hs.levels[0].A
    assert info.converged and np.linalg.norm(b - D @ x) / np.linalg.norm(b) <= 1e-8
    xr = spla.splu(D.tocsc()).solve(b)
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) < 1e-6


def test_fine_equivalent_weights(h16):
    H, _, _ = h16
    c = multigrid.Counters(fine=10, inter=8, coarse=64, n_fine=512, n_int=384, n_coarse=24)
    assert abs(c.fine_equivalent() - (10 + 0.75 * 8 + 24 / 512 * 64)) < 1e-14
    assert H.counters.n_int / H.counters.n_fine == 0.75
    assert H.counters.n_coarse / H.counters.n_fine == 3 / 64
