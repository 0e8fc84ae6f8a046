"""Krylov solvers of the Methods section, written plainly in numpy complex128.

* CG (Hestenes-Stiefel) for the Hermitian positive definite normal equations of
  the near-null setup, D D^dagger e = -D D^dagger x.
* GMRES / flexible GMRES (Saad; Saad-Schultz) for the smoother ("two iterations
  of GMRES"), the partial intermediate solve and the outer FGMRES(8).
* GMRES-DR(m, k) (Morgan, deflated restarting) for the first coarse solve, which
  solves the system and computes k harmonic Ritz vectors at the same time.
* GMRES-Proj(m, k) (Morgan-Wilcox) for every later coarse solve: a minimum
  residual projection over the stored GMRES-DR space followed by GMRES(m - k).

Arnoldi orthogonalises with modified Gram-Schmidt applied twice.  The small
least-squares problems min || c - Hbar d || are solved with numpy.linalg.lstsq
and the harmonic Ritz eigenproblem with numpy.linalg.eig (library steps).

Pins (tests/test_oracle_krylov.py): GMRES and FGMRES against dense LU; FGMRES
with M = I reproduces GMRES; M = A^{-1} converges in one step; GMRES-DR keeps
A V_k = V_{k+1} Hbar_k; GMRES-DR(m, 0) equals GMRES(m); harmonic Ritz values
against a dense eigendecomposition; GMRES-Proj with k = 0 equals GMRES(m).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


class CountedOp:
    """A matrix-vector product that counts its applications (one Mvp each)."""

    def __init__(self, matvec, n: int, name: str = ""):
        self._mv = matvec
        self.n = n
        self.name = name
        self.mvps = 0

    def __call__(self, v: np.ndarray) -> np.ndarray:
        self.mvps += 1
        return self._mv(v)


def _mgs2(V, j, w):
    """Orthogonalise w against columns 0..j of V twice (MGS); return (h, w)."""
    h = np.zeros(j + 1, dtype=complex)
    for _ in range(2):
        for i in range(j + 1):
            c = np.vdot(V[:, i], w)
            h[i] += c
            w = w - c * V[:, i]
    return h, w


BREAKDOWN_REL = 1e-12


def _breakdown_filter(hn, wn0):
    """Treat h_{j+1,j} as an exact zero (invariant Krylov space) when orthogonalisation
    removed all but a rounding-level fraction of A v_j."""
    return 0.0 if hn <= BREAKDOWN_REL * wn0 else hn


def cg(apply, b, tol, maxiter=100000):
    """Conjugate gradients from x0 = 0 for Hermitian positive definite ``apply``.

    Stops when ||b - A x|| <= tol * ||b|| (recurrence residual).  Returns (x, iterations)."""
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0
    p = r.copy()
    rr = np.vdot(r, r).real
    for it in range(1, maxiter + 1):
        q = apply(p)
        alpha = rr / np.vdot(p, q).real
        x = x + alpha * p
        r = r - alpha * q
        rr_new = np.vdot(r, r).real
        if np.sqrt(rr_new) <= tol * bn:
            return x, it
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, maxiter


@dataclass
class CycleResult:
    dx: np.ndarray           # correction to the iterate
    steps: int               # Arnoldi steps taken
    est: float               # least-squares residual norm estimate
    V: np.ndarray            # Arnoldi basis, n x (steps + 1)
    H: np.ndarray            # Hessenberg, (steps + 1) x steps
    coef: np.ndarray         # least-squares solution y
    beta: float              # norm of the starting residual


def fgmres_cycle(A, r, m, stop_abs, M=None):
    """One cycle of (flexible) GMRES from residual r, at most m steps.

    With a preconditioner M the search directions z_j = M(v_j) are kept and the
    correction is Z y (flexible GMRES, Saad 1993); without, it is V y.  The cycle
    ends early once the least-squares residual min || beta e1 - Hbar y || drops to
    ``stop_abs``, or on an exact breakdown h_{j+1,j} = 0.
    """
    n = r.shape[0]
    beta = np.linalg.norm(r)
    V = np.zeros((n, m + 1), dtype=complex)
    Z = np.zeros((n, m), dtype=complex) if M is not None else None
    H = np.zeros((m + 1, m), dtype=complex)
    g = np.zeros(m + 1, dtype=complex)
    g[0] = beta
    if beta == 0.0:
        return CycleResult(np.zeros(n, complex), 0, 0.0, V[:, :1], H[:1, :0], np.zeros(0, complex), 0.0)
    V[:, 0] = r / beta
    steps = 0
    y = np.zeros(0, complex)
    est = beta
    for j in range(m):
        if M is not None:
            Z[:, j] = M(V[:, j])
            w = A(Z[:, j])
        else:
            w = A(V[:, j])
        wn0 = np.linalg.norm(w)
        h, w = _mgs2(V, j, w)
        H[: j + 1, j] = h
        hn = _breakdown_filter(np.linalg.norm(w), wn0)
        H[j + 1, j] = hn
        steps = j + 1
        y = np.linalg.lstsq(H[: j + 2, : j + 1], g[: j + 2], rcond=None)[0]
        est = np.linalg.norm(g[: j + 2] - H[: j + 2, : j + 1] @ y)
        if hn == 0.0:
            est = 0.0
            break
        V[:, j + 1] = w / hn
        if est <= stop_abs:
            break
    basis = Z if M is not None else V
    dx = basis[:, :steps] @ y
    return CycleResult(dx, steps, est, V[:, : steps + 1], H[: steps + 1, :steps], y, beta)


def cycle_residual(cr: CycleResult) -> np.ndarray:
    """Residual after a cycle from the Arnoldi relation: V_{j+1} (beta e1 - Hbar y)."""
    s = -(cr.H @ cr.coef)
    s[0] += cr.beta
    return cr.V @ s


def gmres_steps(A, v, steps):
    """The smoother: GMRES with ``steps`` Arnoldi steps from x0 = 0, no early exit.

    Returns (y, r) with r = v - A y taken from the Arnoldi relation (no extra Mvp)."""
    cr = fgmres_cycle(A, v, steps, stop_abs=-1.0)
    return cr.dx, cycle_residual(cr)


@dataclass
class SolveInfo:
    iters: int = 0
    cycles: int = 0
    rel_resid: float = np.nan
    converged: bool = False
    stagnated: bool = False
    history: list = field(default_factory=list)


def fgmres(A, b, m, tol, M=None, max_iters=400, require_true=True):
    """Restarted (flexible) GMRES(m) from x0 = 0.

    ``require_true``: convergence is decided on the explicitly recomputed residual
    b - A x at the end of a cycle (outer solve); otherwise the least-squares
    estimate decides and a residual is recomputed only to restart (partial
    intermediate solve).  At most ``max_iters`` Arnoldi steps in total.
    """
    x = np.zeros_like(b)
    bn = np.linalg.norm(b)
    info = SolveInfo()
    if bn == 0.0:
        info.rel_resid = 0.0
        info.converged = True
        return x, info
    r = b.copy()
    while info.iters < max_iters:
        cr = fgmres_cycle(A, r, min(m, max_iters - info.iters), tol * bn, M)
        x = x + cr.dx
        info.iters += cr.steps
        info.cycles += 1
        info.history.append(cr.est / bn)
        est_ok = cr.est <= tol * bn
        if not require_true and (est_ok or info.iters >= max_iters):
            info.rel_resid = cr.est / bn
            info.converged = est_ok
            return x, info
        r = b - A(x)
        info.rel_resid = np.linalg.norm(r) / bn
        if info.rel_resid <= tol:
            info.converged = True
            return x, info
    return x, info


def gmres(A, b, m, tol, max_iters=400):
    """Restarted GMRES(m), true-residual convergence test at each restart."""
    return fgmres(A, b, m, tol, None, max_iters, True)


def harmonic_ritz(H_bar, k):
    """k harmonic Ritz pairs of smallest magnitude from an (m+1) x m Arnoldi matrix.

    With H the leading m x m block and h = Hbar[m, m-1], f = H^{-H} e_m, the
    harmonic Ritz values are the eigenvalues of H + |h|^2 f e_m^T.  Ties in
    magnitude (conjugate pairs of a gamma_5-hermitian operator) are ordered by
    the imaginary part, then by position.  Returns (theta[k], G[m, k]).
    """
    m = H_bar.shape[1]
    H = H_bar[:m, :m]
    h = H_bar[m, m - 1]
    em = np.zeros(m, dtype=complex)
    em[-1] = 1.0
    f = np.linalg.solve(H.conj().T, em)
    G = H + (abs(h) ** 2) * np.outer(f, em)
    theta, vecs = np.linalg.eig(G)
    mag = np.abs(theta)
    scale = max(mag.max(), 1e-300)
    keyed = sorted(range(m), key=lambda i: (np.round(mag[i] / scale, 12), theta[i].imag, i))
    idx = keyed[:k]
    return theta[idx], vecs[:, idx]


@dataclass
class Deflation:
    """Deflation space A V_k = V_{k+1} Hbar_k produced by GMRES-DR, used by GMRES-Proj."""
    V: np.ndarray | None = None     # n x (k+1), orthonormal columns
    H: np.ndarray | None = None     # (k+1) x k
    theta: np.ndarray | None = None  # harmonic Ritz values of the stored space

    @property
    def ready(self) -> bool:
        return self.V is not None

    @property
    def k(self) -> int:
        return 0 if self.H is None else self.H.shape[1]


def _compress(V, H_bar, k, s=None):
    """Deflated restart / final compression of GMRES-DR.

    From A V_m = V_{m+1} Hbar_m keep the k smallest harmonic Ritz vectors g_i,
    padded with a zero row, plus one more direction (the residual s during
    restarts, or the common harmonic residual direction [-|h|^2 f; h] at the
    end).  Returns (V_{k+1}, Hbar_k, P_{k+1}, theta).
    """
    m = H_bar.shape[1]
    theta, Gk = harmonic_ritz(H_bar, k)
    Gpad = np.vstack([Gk, np.zeros((1, k), dtype=complex)])
    if s is None:
        Hm = H_bar[:m, :m]
        h = H_bar[m, m - 1]
        em = np.zeros(m, dtype=complex)
        em[-1] = 1.0
        f = np.linalg.solve(Hm.conj().T, em)
        s = np.concatenate([-(abs(h) ** 2) * f, [h]])
    P, _ = np.linalg.qr(np.column_stack([Gpad, s]))
    Pk = P[:m, :k]          # its last row vanishes: the g_i are padded with zero
    Hk = P.conj().T @ H_bar @ Pk
    Vk1 = V @ P
    # re-orthogonalise the last column against the first k
    h, w = _mgs2(Vk1, k - 1, Vk1[:, k].copy())
    Vk1[:, k] = w / np.linalg.norm(w)
    return Vk1, Hk, P, theta


def gmres_dr(A, b, m, k, tol, max_cycles=1000, stall=0.99, stall_floor=1e-10):
    """GMRES-DR(m, k) from x0 = 0 (Morgan, deflated restarting).

    Returns (x, info, Deflation).  Each cycle extends the Arnoldi relation to m
    columns, solves min || c - Hbar d ||, and restarts with the k smallest
    harmonic Ritz vectors plus the residual direction, so that the kept space
    satisfies A V_k = V_{k+1} Hbar_k.  On termination the space is compressed
    once more to k vectors for later projections.  Once the relative residual
    is at or below `stall_floor` (the rounding regime of these FP64 systems), a
    cycle that lowers it by less than the factor `stall` ends the solve: a
    tolerance below what the arithmetic reaches, such as 1e-15, otherwise never
    stops, while a slow stretch above the floor is ordinary convergence.
    """
    n = b.shape[0]
    x = np.zeros_like(b)
    bn = np.linalg.norm(b)
    info = SolveInfo()
    if bn == 0.0:
        info.rel_resid, info.converged = 0.0, True
        return x, info, Deflation()
    V = np.zeros((n, m + 1), dtype=complex)
    H = np.zeros((m + 1, m), dtype=complex)
    c = np.zeros(m + 1, dtype=complex)
    V[:, 0] = b / bn
    c[0] = bn
    j0 = 0
    for cycle in range(max_cycles):
        steps = j0
        d = None
        converged = False
        for j in range(j0, m):
            w = A(V[:, j])
            wn0 = np.linalg.norm(w)
            h, w = _mgs2(V, j, w)
            H[: j + 1, j] = h
            hn = _breakdown_filter(np.linalg.norm(w), wn0)
            H[j + 1, j] = hn
            steps = j + 1
            info.iters += 1
            d = np.linalg.lstsq(H[: j + 2, : j + 1], c[: j + 2], rcond=None)[0]
            est = np.linalg.norm(c[: j + 2] - H[: j + 2, : j + 1] @ d)
            if hn == 0.0:
                est = 0.0
            else:
                V[:, j + 1] = w / hn
            if est <= tol * bn:
                converged = True
                break
        info.cycles += 1
        x = x + V[:, :steps] @ d
        info.history.append(est / bn)
        if converged or hn == 0.0:
            info.converged = True
            info.rel_resid = est / bn
            break
        if (stall and len(info.history) > 1 and info.history[-1] > stall * info.history[-2]
                and info.history[-1] <= stall_floor):
            info.stagnated = True
            info.rel_resid = est / bn
            break
        s = c - H @ d
        Vk1, Hk, P, _ = _compress(V, H, k, s)
        c_new = P.conj().T @ s
        V[:] = 0.0
        H[:] = 0.0
        c[:] = 0.0
        V[:, : k + 1] = Vk1
        H[: k + 1, :k] = Hk
        c[: k + 1] = c_new
        j0 = k
    else:
        info.rel_resid = est / bn
    # stored deflation space
    Hs = H[: steps + 1, :steps]
    Vs = V[:, : steps + 1]
    if steps > k and Hs[steps, steps - 1] != 0.0:
        Vk1, Hk, _, theta = _compress(Vs, Hs, k)
        defl = Deflation(Vk1, Hk, theta)
    else:
        defl = Deflation(Vs.copy(), Hs.copy(), None)
    return x, info, defl


def gmres_proj(A, b, defl: Deflation, m, tol, max_cycles=1000):
    """GMRES-Proj(m, k) from x0 = 0 (Morgan-Wilcox).

    Each cycle first projects over the deflation space, minimising || r - A V_k d ||
    through A V_k = V_{k+1} Hbar_k (c = V_{k+1}^H r, no Mvp), then runs one
    GMRES(m - k) cycle; residuals follow the Arnoldi recurrence.  Stops when the
    residual norm reaches tol * ||b||.
    """
    x = np.zeros_like(b)
    bn = np.linalg.norm(b)
    info = SolveInfo()
    if bn == 0.0:
        info.rel_resid, info.converged = 0.0, True
        return x, info
    r = b.copy()
    k = defl.k
    for cycle in range(max_cycles):
        if k > 0:
            cvec = defl.V.conj().T @ r
            d = np.linalg.lstsq(defl.H, cvec, rcond=None)[0]
            x = x + defl.V[:, :k] @ d
            r = r - defl.V @ (defl.H @ d)
        rn = np.linalg.norm(r)
        if rn <= tol * bn:
            info.converged = True
            break
        cr = fgmres_cycle(A, r, m - k, tol * bn)
        x = x + cr.dx
        r = cycle_residual(cr)
        info.iters += cr.steps
        info.cycles += 1
        rn = np.linalg.norm(r)
        info.history.append(rn / bn)
        if rn <= tol * bn:
            info.converged = True
            break
    info.rel_resid = rn / bn
    return x, info
