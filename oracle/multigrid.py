"""Adaptive multigrid with a deflated coarse solve (Methods section), plain numpy/scipy.

Setup, for each of the two coarsenings (fine -> intermediate -> coarse):
  1. near-null vectors: for 12 random x solve A A^dagger e = -A A^dagger x by CG
     to relative residual 1e-4 and keep psi = x + e;
  2. orthonormalise the 12 vectors over the whole lattice;
  3. chirally double them with (1 +- gamma_5) / 2 (sigma_3 on the fine lattice,
     Gamma_5 = diag(I_12, -I_12) on the blocked lattice);
  4. restrict each to every 4 x 4 block and orthonormalise locally -> columns of P;
  5. Galerkin operator A_next = P^dagger A P.
Solve:
  outer FGMRES(8) on D preconditioned by a fine cycle M0 (GMRES(2) pre-smoother,
  restriction, partial intermediate solve, prolongation, GMRES(2) post-smoother);
  the partial intermediate solve is FGMRES(8) on D_hat to 0.2 ||b|| preconditioned
  by the intermediate cycle M1, whose coarse correction is GMRES-DR(30, 10) on the
  first coarse call (tolerance 1e-8) and GMRES-Proj(30, 10) afterwards (1e-2).

Layouts.  Fine dof index 2 s + spin, s = x + Nx t.  Blocked lattices: dof index
24 S + 12 c + k, S = X + (Nx/4) T, c = 0 for chirality +, 1 for chirality -.
Inside a 4 x 4 block the local site is x_l + 4 t_l and a block row is
(local site) * (dof/2) + (index within the chirality half).

Pins (tests/test_oracle_multigrid.py): P^dagger P = I per block, sigma_3 P =
P Gamma_5, P P^dagger reproduces the blocked chiral near-null vectors, Galerkin
blocks against dense products at 8^2, Gamma_5 A Gamma_5 = A^dagger at every
level, the two-grid projector identities, and whole solves against sparse LU.
Iteration and Mvp counts: parity unpinned (the paper gives trends only).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import krylov
from .wilson import dirac_matrix, gamma5_vector

NVEC = 12
BLOCK = 4


@dataclass
class Params:
    nvec: int = NVEC
    null_tol: float = 1e-4
    outer_m: int = 8
    outer_tol: float = 1e-8
    outer_max_iters: int = 400
    smooth_steps: int = 2
    int_m: int = 8
    int_tol: float = 0.2
    int_max_iters: int = 16
    coarse_m: int = 30
    coarse_k: int = 10
    coarse_tol_first: float = 1e-8
    coarse_tol_later: float = 1e-2
    deflate: bool = True
    coarse_cgne_tol: float = 1e-8
    # "partial": the intermediate grid is solved by FGMRES to int_tol (the paper's partial
    # solve); "cycle": one intermediate cycle M1 (smoothing-only intermediate treatment)
    intermediate: str = "partial"


@dataclass
class Level:
    A: sp.csr_matrix
    g5: np.ndarray          # diagonal of gamma_5 on this level
    Lx: int
    Lt: int
    dof: int                # degrees of freedom per site
    P: sp.csr_matrix | None = None      # prolongator to the next coarser level
    null: np.ndarray | None = None      # near-null vectors (rows) before orthonormalisation
    Q: np.ndarray | None = None         # local bases [nblocks, 2, rows, nvec]


def coarse_gamma5(n_sites: int) -> np.ndarray:
    return np.tile(np.concatenate([np.ones(NVEC), -np.ones(NVEC)]), n_sites)


def mgs2_columns(W):
    """Orthonormalise the columns of W in order with modified Gram-Schmidt applied twice.

    W has shape [..., rows, ncols]; the leading axes are independent problems."""
    Q = np.array(W, dtype=complex, copy=True)
    nc = Q.shape[-1]
    for k in range(nc):
        for _ in range(2):
            for j in range(k):
                h = np.sum(np.conj(Q[..., :, j]) * Q[..., :, k], axis=-1)
                Q[..., :, k] -= h[..., None] * Q[..., :, j]
        nrm = np.sqrt(np.sum(np.abs(Q[..., :, k]) ** 2, axis=-1))
        Q[..., :, k] /= nrm[..., None]
    return Q


def near_null_vectors(A: sp.csr_matrix, starts: np.ndarray, tol: float):
    """psi_i = x_i + e_i with A A^dagger e_i = -A A^dagger x_i solved by CG to ``tol``."""
    AH = A.conj().T.tocsr()
    out = []
    iters = []
    for x in starts:
        def normal(v):
            return A @ (AH @ v)
        b = -normal(x)
        e, it = krylov.cg(normal, b, tol)
        out.append(x + e)
        iters.append(it)
    return np.array(out), iters


def block_rows(Lx, Lt, dof):
    """For every 4 x 4 block and chirality, the fine dof indices of its rows in order.

    Returns idx[nblocks, 2, 16 * dof / 2]; blocks are numbered X + (Lx/4) T."""
    half = dof // 2
    BX, BT = Lx // BLOCK, Lt // BLOCK
    idx = np.zeros((BX * BT, 2, BLOCK * BLOCK * half), dtype=np.int64)
    for T in range(BT):
        for X in range(BX):
            b = X + BX * T
            for c in range(2):
                row = 0
                for tl in range(BLOCK):
                    for xl in range(BLOCK):
                        s = (BLOCK * X + xl) + Lx * (BLOCK * T + tl)
                        for a in range(half):
                            idx[b, c, row] = dof * s + c * half + a
                            row += 1
    return idx


def build_prolongator(vecs: np.ndarray, Lx, Lt, dof, g5):
    """Columns of P from the near-null vectors (rows of ``vecs``).

    Global MGS2 orthonormalisation, chiral doubling with (1 +- gamma_5)/2, then
    per block and chirality MGS2 of the 16 * dof/2 x 12 restriction.  Returns
    (P sparse n_fine x n_coarse, Q[nblocks, 2, rows, 12])."""
    nvec = vecs.shape[0]
    ortho = mgs2_columns(vecs.T)            # columns are the orthonormalised vectors
    plus = 0.5 * (1 + g5)[:, None] * ortho
    minus = 0.5 * (1 - g5)[:, None] * ortho
    idx = block_rows(Lx, Lt, dof)
    nb, _, nrows = idx.shape
    W = np.empty((nb, 2, nrows, nvec), dtype=complex)
    W[:, 0] = plus[idx[:, 0], :]
    W[:, 1] = minus[idx[:, 1], :]
    Q = mgs2_columns(W)
    n_fine = Lx * Lt * dof
    n_coarse = nb * 2 * nvec
    rows = np.broadcast_to(idx[..., None], Q.shape)
    cols = (np.arange(nb)[:, None, None, None] * 2 * nvec
            + np.arange(2)[None, :, None, None] * nvec
            + np.arange(nvec)[None, None, None, :])
    cols = np.broadcast_to(cols, Q.shape)
    P = sp.coo_matrix((Q.ravel(), (rows.ravel(), cols.ravel())), shape=(n_fine, n_coarse)).tocsr()
    return P, Q


def galerkin(A: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    """A_next = P^dagger A P."""
    return (P.conj().T @ A @ P).tocsr()


def stencil_blocks(Ahat: sp.csr_matrix, Lx, Lt, dof=2 * NVEC):
    """Read the nearest-neighbour blocks of a blocked-lattice operator.

    Returns B[S, d] (dof x dof) with d = 0 self, 1 +x, 2 -x, 3 +t, 4 -t: the
    coupling from site S + d into site S.  Where two directions reach the same
    site (extent 2) both entries hold the summed coupling."""
    A = Ahat.toarray() if Ahat.shape[0] <= 20000 else None
    V = Lx * Lt
    B = np.zeros((V, 5, dof, dof), dtype=complex)
    for T in range(Lt):
        for X in range(Lx):
            S = X + Lx * T
            nbrs = [S, (X + 1) % Lx + Lx * T, (X - 1) % Lx + Lx * T,
                    X + Lx * ((T + 1) % Lt), X + Lx * ((T - 1) % Lt)]
            for d, S2 in enumerate(nbrs):
                if A is not None:
                    B[S, d] = A[dof * S:dof * S + dof, dof * S2:dof * S2 + dof]
                else:
                    B[S, d] = Ahat[dof * S:dof * S + dof, dof * S2:dof * S2 + dof].toarray()
    return B


@dataclass
class Counters:
    fine: int = 0
    inter: int = 0
    coarse: int = 0
    n_fine: int = 1
    n_int: int = 1
    n_coarse: int = 1

    def fine_equivalent(self) -> float:
        """Fine-equivalent Mvps, eq. (1): weights are ratios of operator dimensions."""
        return (self.fine + self.n_int / self.n_fine * self.inter
                + self.n_coarse / self.n_fine * self.coarse)


class Hierarchy:
    """Three-level hierarchy: fine D, intermediate D_hat = P^H D P, coarse D_c = Phat^H D_hat Phat."""

    def __init__(self, theta, m0, starts0, starts1, params: Params | None = None,
                 antiperiodic=True, null0=None, null1=None):
        self.params = params or Params()
        p = self.params
        Nt, Nx, _ = theta.shape
        D = dirac_matrix(theta, m0, antiperiodic)
        self.levels = [Level(D, gamma5_vector(Nx * Nt), Nx, Nt, 2)]
        self.setup_iters = []
        for lvl, (starts, inject) in enumerate([(starts0, null0), (starts1, null1)]):
            L = self.levels[-1]
            if inject is None:
                null, its = near_null_vectors(L.A, starts, p.null_tol)
            else:
                null, its = np.array(inject), []
            self.setup_iters.append(its)
            P, Q = build_prolongator(null, L.Lx, L.Lt, L.dof, L.g5)
            L.P, L.Q, L.null = P, Q, null
            Lx, Lt = L.Lx // BLOCK, L.Lt // BLOCK
            self.levels.append(Level(galerkin(L.A, P), coarse_gamma5(Lx * Lt), Lx, Lt, 2 * p.nvec))
        self.deflation = krylov.Deflation()
        self.counters = Counters(n_fine=D.shape[0], n_int=self.levels[1].A.shape[0],
                                 n_coarse=self.levels[2].A.shape[0])
        self.coarse_calls = []

    # -- operators with Mvp counting ------------------------------------------------
    def _op(self, lvl):
        A = self.levels[lvl].A
        attr = ["fine", "inter", "coarse"][lvl]

        def mv(v):
            setattr(self.counters, attr, getattr(self.counters, attr) + 1)
            return A @ v
        return mv

    def coarse_solve(self, bc):
        """C(b_c): GMRES-DR on the first call, GMRES-Proj on every later call."""
        p = self.params
        A = self._op(2)
        if not p.deflate:
            Ac = self.levels[2].A
            AcH = Ac.conj().T.tocsr()

            def normal(v):
                self.counters.coarse += 2
                return Ac @ (AcH @ v)
            y, it = krylov.cg(normal, bc, p.coarse_cgne_tol)
            self.counters.coarse += 1
            self.coarse_calls.append(("cgne", it))
            return AcH @ y
        if not self.deflation.ready:
            x, info, defl = krylov.gmres_dr(A, bc, p.coarse_m, p.coarse_k, p.coarse_tol_first)
            self.deflation = defl
            self.coarse_calls.append(("dr", info.iters))
            return x
        x, info = krylov.gmres_proj(A, bc, self.deflation, p.coarse_m, p.coarse_tol_later)
        self.coarse_calls.append(("proj", info.iters))
        return x

    def cycle1(self, v):
        """Intermediate cycle M1: smooth, coarse correction, smooth."""
        p = self.params
        A = self._op(1)
        P = self.levels[1].P
        y1, r = krylov.gmres_steps(A, v, p.smooth_steps)
        y2 = y1 + P @ self.coarse_solve(P.conj().T @ r)
        r2 = v - A(y2)
        y3 = y2 + krylov.gmres_steps(A, r2, p.smooth_steps)[0]
        return y3

    def partial_solve(self, bh):
        """E1: FGMRES(8) on D_hat preconditioned by M1, to 0.2 ||b|| (at most 16 steps)."""
        p = self.params
        x, _ = krylov.fgmres(self._op(1), bh, p.int_m, p.int_tol, self.cycle1,
                             p.int_max_iters, require_true=False)
        return x

    def cycle0(self, v):
        """Fine cycle M0: smooth, intermediate partial solve (or one intermediate cycle), smooth."""
        p = self.params
        A = self._op(0)
        P = self.levels[0].P
        y1, r = krylov.gmres_steps(A, v, p.smooth_steps)
        rh = P.conj().T @ r
        e = self.partial_solve(rh) if p.intermediate == "partial" else self.cycle1(rh)
        y2 = y1 + P @ e
        r2 = v - A(y2)
        y3 = y2 + krylov.gmres_steps(A, r2, p.smooth_steps)[0]
        return y3

    def solve(self, b):
        """Outer FGMRES(8) to true relative residual outer_tol; returns (x, info)."""
        p = self.params
        return krylov.fgmres(self._op(0), b, p.outer_m, p.outer_tol, self.cycle0,
                             p.outer_max_iters, require_true=True)
