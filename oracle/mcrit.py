"""Critical mass m_c of a configuration (Results section: the "mass gap").

D(m0) = D(0) + m0 * I exactly, so every eigenvalue's real part moves by m0 and
the bare mass at which the smallest Re(lambda) crosses zero is
m_c = -min Re lambda(D(0)).

Small lattices use a dense eigendecomposition.  Larger ones use ARPACK in
shift-invert mode about a shift sigma placed at or left of the spectrum's left
edge: the eigenvalues nearest sigma are then the leftmost ones, and the search
returns the radius R of the disc about sigma that it has covered, so any
eigenvalue with a smaller real part that was missed would need an imaginary
part of at least sqrt(R^2 - (Re_min - sigma)^2) (reported as ``im_guard``).

Pins (tests/test_oracle_mcrit.py): the free-field closed form
m_c = -(1 - cos(pi / N)) and agreement of the sparse search with dense eig.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .wilson import dirac_matrix

DENSE_LIMIT = 32 * 32 * 2


def critical_mass_dense(theta, antiperiodic=True):
    D0 = dirac_matrix(theta, 0.0, antiperiodic)
    return -float(np.linalg.eigvals(D0.toarray()).real.min())


def leftmost_eigenvalues(theta, antiperiodic=True, sigma=0.0, k=8, tol=1e-11):
    """The k eigenvalues of D(0) nearest sigma (shift-invert ARPACK) and the covered radius.

    Above 256^2 sites the Krylov space is 96 vectors: there the leftmost eigenvalues of
    some configurations lie within a few per cent of each other and a 32-vector space
    stalls for hours.  The answer (the k nearest eigenvalues) does not depend on it."""
    D0 = dirac_matrix(theta, 0.0, antiperiodic)
    n = D0.shape[0]
    lu = spla.splu((D0 - sigma * sp.identity(n, format="csc")).tocsc())
    op = spla.LinearOperator((n, n), matvec=lu.solve, dtype=complex)
    ncv = 96 if n > 2 * 256 * 256 else max(4 * k, 32)
    mu = spla.eigs(op, k=k, which="LM", ncv=ncv, tol=tol, maxiter=100000,
                   return_eigenvectors=False)
    lam = sigma + 1.0 / mu
    return lam, float(np.abs(lam - sigma).max())


def critical_mass(theta, antiperiodic=True, sigma=0.0, k=8):
    """Returns (m_c, im_guard); im_guard is inf for the dense path."""
    n = 2 * theta.shape[0] * theta.shape[1]
    if n <= DENSE_LIMIT:
        return critical_mass_dense(theta, antiperiodic), float("inf")
    lam, R = leftmost_eigenvalues(theta, antiperiodic, sigma, k)
    re_min = lam.real.min()
    guard = float(np.sqrt(max(R * R - (re_min - sigma) ** 2, 0.0)))
    return -float(re_min), guard
