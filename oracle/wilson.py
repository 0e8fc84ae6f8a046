"""Wilson-Dirac operator of the 2D lattice Schwinger model (Methods section).

The paper names the operator only.  The form used here is the standard r = 1
Wilson discretisation in the "m0 + 2" normalisation,

    (D psi)(s) = (m0 + 2) psi(s)
                 - 1/2 sum_mu [ (1 - g_mu) U_mu(s) psi(s + mu)
                              + (1 + g_mu) conj(U_mu(s - mu)) psi(s - mu) ],

with g_0 = sigma_1, g_1 = sigma_2 and g_5 = sigma_3.  Gauge links are periodic;
the fermion sees an antiperiodic time direction, folded into the links of the
last time slice.  Site s = x + Nx * t, degree of freedom 2 * s + spin.

Pins (tests/test_oracle_wilson.py): free-field plane-wave spectrum in closed
form, sigma_3 D sigma_3 = D^dagger, gauge covariance, D(m0) - D(0) = m0 * I.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SIGMA = [
    np.array([[0, 1], [1, 0]], dtype=complex),      # gamma_0 = sigma_1
    np.array([[0, -1j], [1j, 0]], dtype=complex),   # gamma_1 = sigma_2
]
GAMMA5 = np.array([[1, 0], [0, -1]], dtype=complex)  # sigma_3
ID2 = np.eye(2, dtype=complex)


def fermion_links(theta: np.ndarray, antiperiodic: bool = True) -> np.ndarray:
    """U[mu, t, x] = exp(i theta[t, x, mu]), with the temporal links on the last
    time slice negated when the fermion is antiperiodic in time."""
    U = np.exp(1j * np.moveaxis(theta, 2, 0))
    if antiperiodic:
        U[1, -1, :] *= -1.0
    return U


def site_index(x, t, Nx):
    return x + Nx * t


def dirac_matrix(theta: np.ndarray, m0: float, antiperiodic: bool = True) -> sp.csr_matrix:
    """Sparse Wilson-Dirac matrix (2V x 2V) assembled term by term from its definition."""
    Nt, Nx, _ = theta.shape
    V = Nx * Nt
    U = fermion_links(theta, antiperiodic)
    t, x = np.meshgrid(np.arange(Nt), np.arange(Nx), indexing="ij")
    s = site_index(x, t, Nx).ravel()
    rows, cols, vals = [], [], []

    def add_block(src_sites, dst_sites, mats):
        # mats[n] is the 2x2 matrix acting from site dst_sites[n] into row site src_sites[n]
        for a in range(2):
            for b in range(2):
                rows.append(2 * src_sites + a)
                cols.append(2 * dst_sites + b)
                vals.append(mats[:, a, b])

    diag = np.broadcast_to((m0 + 2.0) * ID2, (V, 2, 2))
    add_block(s, s, diag)
    for mu in range(2):
        g = SIGMA[mu]
        if mu == 0:
            fwd = site_index((x + 1) % Nx, t, Nx).ravel()
            bwd = site_index((x - 1) % Nx, t, Nx).ravel()
            u_here = U[0].ravel()
            u_back = U[0][t, (x - 1) % Nx].ravel()
        else:
            fwd = site_index(x, (t + 1) % Nt, Nx).ravel()
            bwd = site_index(x, (t - 1) % Nt, Nx).ravel()
            u_here = U[1].ravel()
            u_back = U[1][(t - 1) % Nt, x].ravel()
        add_block(s, fwd, -0.5 * u_here[:, None, None] * (ID2 - g)[None])
        add_block(s, bwd, -0.5 * np.conj(u_back)[:, None, None] * (ID2 + g)[None])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    keep = vals != 0
    M = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(2 * V, 2 * V))
    return M.tocsr()


def gamma5_vector(n_sites: int) -> np.ndarray:
    """Diagonal of sigma_3 on the fine lattice: +1 on spin 0, -1 on spin 1."""
    return np.tile(np.array([1.0, -1.0]), n_sites)


def free_field_eigenvalues(Nx: int, Nt: int, m0: float, antiperiodic: bool = True) -> np.ndarray:
    """Closed-form spectrum of D at U = 1: for every momentum p (p_x = 2 pi k / Nx,
    p_t = (2k + 1) pi / Nt when antiperiodic) the two eigenvalues
    m0 + sum_mu (1 - cos p_mu) +- i sqrt(sum_mu sin^2 p_mu)."""
    px = 2 * np.pi * np.arange(Nx) / Nx
    pt = (2 * np.arange(Nt) + (1 if antiperiodic else 0)) * np.pi / Nt
    PX, PT = np.meshgrid(px, pt, indexing="ij")
    re = m0 + (1 - np.cos(PX)) + (1 - np.cos(PT))
    im = np.sqrt(np.sin(PX) ** 2 + np.sin(PT) ** 2)
    return np.concatenate([(re + 1j * im).ravel(), (re - 1j * im).ravel()])
