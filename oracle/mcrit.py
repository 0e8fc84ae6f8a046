"""Critical mass m_c of a configuration (Results section: the "mass gap").

D(m0) = D(0) + m0 * I exactly, so every eigenvalue's real part moves by m0 and
the bare mass at which the smallest Re(lambda) crosses zero is
m_c = -min Re lambda(D(0)).

Small lattices use a dense eigendecomposition.  Larger ones use ARPACK in
shift-invert mode: about a shift sigma it returns the k eigenvalues nearest sigma
and the radius R of the disc about sigma that they fill, so any eigenvalue with a
smaller real part that was missed would lie outside that disc; for a real shift it
would need an imaginary part of at least sqrt(R^2 - (Re_min - sigma)^2).

Two facts bound the search from outside it.  The real part of every eigenvalue
lies in the numerical range of the Hermitian part (D + D^dagger)/2 (Bendixson),
which for the r = 1 Wilson operator is m0 + 1/2 times the gauge-covariant
lattice Laplacian, so min Re lambda(D(0)) >= lambda_min((D(0) + D(0)^dagger)/2)
>= 0 and m_c <= 0.  And plain (non-inverted) Arnoldi asked for the eigenvalues
of smallest real part reaches the same edge by a different route.

The search used for the stored workload masses covers the whole strip in which a
leftmost eigenvalue can lie (``critical_mass``): a single shift-invert search about
sigma = 0 finds only the eigenvalues nearest the origin and misses a leftmost
eigenvalue with a larger imaginary part once the spectrum is dense enough (as at
64^2 and 128^2 for some configurations).

Pins (tests/test_oracle_mcrit.py): the free-field closed form
m_c = -(1 - cos(pi / N)) through the dense path and through the covered search;
the shift-invert eigenvalues against the k nearest of a dense eig; the disc and
guard geometry against a dense eig; the covered search against dense eig where a
single nearest-k search misses the leftmost eigenvalue; the stored critical
masses against plain Arnoldi on D(0) (smallest real part) and the Bendixson
bound; Re lambda = 0 at m0 = m_c.
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
    lu = spla.splu((D0 - sigma * sp.identity(n, format="csc")).tocsc(), permc_spec="MMD_AT_PLUS_A")
    op = spla.LinearOperator((n, n), matvec=lu.solve, dtype=complex)
    ncv = 96 if n > 2 * 256 * 256 else max(4 * k, 32)
    mu = spla.eigs(op, k=k, which="LM", ncv=ncv, tol=tol, maxiter=100000,
                   return_eigenvectors=False)
    lam = sigma + 1.0 / mu
    return lam, float(np.abs(lam - sigma).max())


def hermitian_part_min(theta, antiperiodic=True):
    """Smallest eigenvalue of the Hermitian part (D(0) + D(0)^dagger)/2: a lower bound on
    min Re lambda(D(0)) by Bendixson's theorem (shift-invert Lanczos below the spectrum)."""
    D0 = dirac_matrix(theta, 0.0, antiperiodic)
    H = ((D0 + D0.conj().T) * 0.5).tocsc()
    n = H.shape[0]
    if n <= DENSE_LIMIT:
        return float(np.linalg.eigvalsh(H.toarray()).min())
    lam = spla.eigsh(H, k=1, sigma=-0.5, which="LM", return_eigenvectors=False)
    return float(lam.min())


def smallest_real_part_arnoldi(theta, antiperiodic=True, k=6, ncv=96, tol=1e-10):
    """min Re lambda(D(0)) by plain Arnoldi on D(0) itself (ARPACK, smallest real part):
    an independent route to the left spectral edge, slower than shift-invert."""
    D0 = dirac_matrix(theta, 0.0, antiperiodic)
    lam = spla.eigs(D0, k=k, which="SR", ncv=ncv, tol=tol, maxiter=100000,
                    return_eigenvectors=False)
    return float(lam.real.min())


def imaginary_part_bound(theta, antiperiodic=True):
    """||(D - D^dagger) / 2i||_2, which bounds |Im lambda| of every eigenvalue (Bendixson)."""
    D0 = dirac_matrix(theta, 0.0, antiperiodic)
    S = ((D0 - D0.conj().T) * (-0.5j)).tocsc()
    if S.shape[0] <= DENSE_LIMIT:
        return float(np.abs(np.linalg.eigvalsh(S.toarray())).max())
    lam = spla.eigsh(S, k=1, which="LM", return_eigenvectors=False, tol=1e-8)
    return float(np.abs(lam).max()) * (1.0 + 1e-6)


def critical_mass(theta, antiperiodic=True, k=16, force_sparse=False, verbose=False):
    """Returns (m_c, im_guard).  Small lattices: dense eig (im_guard = inf).  Otherwise a
    covered search of the strip where an eigenvalue with the smallest real part can lie.

    Bendixson's theorem puts every eigenvalue in the rectangle hmin <= Re <= ..., |Im| <= ymax
    (hmin, ymax from the Hermitian and skew-Hermitian parts).  Shift-invert Arnoldi about
    sigma = hmin + i y returns the k eigenvalues nearest sigma and the radius R of the disc
    they fill; with re_min the smallest real part found so far and w = re_min - hmin, that disc
    holds every point of [hmin, re_min] x [y - c, y + c], c = sqrt(R^2 - w^2).  Shifts are
    placed up the imaginary axis until these intervals cover [0, ymax]; the spectrum is
    symmetric under conjugation (sigma_3 D sigma_3 = D^dagger), so Im < 0 needs no shifts.
    Every eigenvalue left of the returned real part would have had to lie in a covered disc,
    so none exists (to ARPACK's convergence of the k nearest eigenvalues).  im_guard is ymax:
    the whole range of imaginary parts is covered."""
    n = 2 * theta.shape[0] * theta.shape[1]
    if n <= DENSE_LIMIT and not force_sparse:
        return critical_mass_dense(theta, antiperiodic), float("inf")
    hmin = hermitian_part_min(theta, antiperiodic)
    ymax = imaginary_part_bound(theta, antiperiodic)
    re_min, lead = np.inf, None
    covered, y, kk = 0.0, 0.0, k
    half_prev = None
    while covered < ymax:
        # the covering discs need their radii, not digits: a looser Arnoldi tolerance
        lam, R = leftmost_eigenvalues(theta, antiperiodic, sigma=hmin + 1j * y, k=kk, tol=1e-8)
        i = int(np.argmin(lam.real))
        if lam[i].real < re_min:
            re_min, lead = float(lam[i].real), complex(lam[i])
        w = re_min - hmin
        half = float(np.sqrt(max(R * R - w * w, 0.0)))
        if verbose:
            print(f"  sigma = {hmin:.5f} + {y:.4f}i: k = {kk}, R = {R:.4f}, re_min = {re_min:.10f}, "
                  f"covers Im in [{y - half:.4f}, {y + half:.4f}]", flush=True)
        if half <= 0.0 or y - half > covered:
            # the disc does not reach back to what is covered: more eigenvalues, or a closer shift
            if half > 0.0 and half_prev is not None:
                y = covered + 0.5 * half
            else:
                kk *= 2
                if kk > 512:
                    raise RuntimeError("critical_mass: the shift-invert discs do not reach the left edge")
            continue
        covered = y + half
        half_prev = half
        kk = k
        y = covered + 0.9 * half
    # the leftmost eigenvalue to full accuracy: shift-invert about the one found.  The value
    # from the covering discs (Arnoldi tolerance 1e-8) can be off by far more than 1e-8 for an
    # ill-conditioned pair, so only the converged eigenvalues give the answer.
    lam, _ = leftmost_eigenvalues(theta, antiperiodic, sigma=lead, k=4, tol=1e-13)
    return -float(lam.real.min()), float(ymax)
