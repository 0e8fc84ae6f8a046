"""Seeded synthetic inputs shared by the GPU solver, its tests and the CPU oracle.

This module draws random numbers and arranges them into arrays; it holds none of
the solver's arithmetic (no Dirac operator, no fermion boundary sign, no Krylov
or multigrid step).  Both the HIP path and the oracle consume exactly these
arrays, so no random-number parity between the two is needed.

Stand-in for the paper's ensembles (Methods section): the paper made ten U(1)
configurations per lattice size with QCDLAB 1.0 at beta = 6.0.  Those files are
not available, so plaquette angles are drawn from the von Mises distribution,
which is the exact single-plaquette law of the 2D U(1) Wilson gauge action
exp(beta * cos theta_P), and assembled into link angles in axial gauge.

Every draw comes from ``numpy.random.Generator(PCG64(SeedSequence(words)))``
with ``words = [N, cfg_idx, purpose, j]``:

    purpose 0  gauge plaquettes and holonomies
    purpose 1  level-0 near-null start vectors (j = vector index)
    purpose 2  level-1 near-null start vectors (j = vector index)
    purpose 3  right-hand sides (j = RHS index)
    purpose 4  coarse deflation warm-up right-hand side
    purpose 5  serving arrivals and configuration choice
"""
from __future__ import annotations

import json
import os

import numpy as np

__all__ = [
    "rng_for",
    "gauge_angles",
    "plaquette_draws",
    "gaussian_complex",
    "rhs",
    "near_null_starts",
    "critical_mass",
    "bare_mass",
    "MASS_OFFSET",
    "BETA",
]

BETA = 6.0
# m0 = m_c + 0.01: the distance to the critical mass used by every workload.
MASS_OFFSET = 0.01

_HERE = os.path.dirname(os.path.abspath(__file__))
MCRIT_FILE = os.path.join(_HERE, "mcrit.json")


def rng_for(*words: int) -> np.random.Generator:
    """Generator seeded from the entropy words ``[N, cfg_idx, purpose, j]``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(w) for w in words])))


def plaquette_draws(N: int, cfg: int, beta: float = BETA):
    """Raw draws for one configuration: von Mises plaquettes ``phi[t, x]`` and two
    Haar-uniform holonomy angles ``(h_x, h_t)``.

    The plaquettes are then shifted uniformly so their sum is an integer multiple
    of 2*pi (the torus constraint: every link enters two plaquettes with opposite
    signs, so the plaquette angles of a periodic lattice sum to 2*pi*Q).
    """
    rng = rng_for(N, cfg, 0, 0)
    phi = rng.vonmises(0.0, beta, size=(N, N))
    total = phi.sum()
    q = np.round(total / (2.0 * np.pi))
    phi = phi - (total - 2.0 * np.pi * q) / (N * N)
    hx, ht = rng.uniform(-np.pi, np.pi, size=2)
    return phi, float(hx), float(ht), int(q)


def gauge_angles(N: int, cfg: int, beta: float = BETA) -> np.ndarray:
    """Link angles ``theta[t, x, mu]`` (float64, radians) of an N x N periodic lattice.

    mu = 0 is the x direction, mu = 1 the t direction.  Axial gauge: temporal links
    vanish except on the last time slice, spatial links on t = 0 vanish except the
    last, which carries the x holonomy; the temporal link at (x=0, t=N-1) carries
    the t holonomy.  Spatial links on later slices are fixed by the plaquettes of
    the slice below, and the last time slice's temporal links by its plaquettes.
    The plaquette at (x, t) is
        theta_x(x,t) + theta_t(x+1,t) - theta_x(x,t+1) - theta_t(x,t)
    and equals ``phi[t, x]`` modulo 2*pi for every site.
    """
    phi, hx, ht, _ = plaquette_draws(N, cfg, beta)
    th = np.zeros((N, N, 2))
    th[0, N - 1, 0] = hx
    for t in range(N - 1):
        th[t + 1, :, 0] = th[t, :, 0] - phi[t, :]
    th[N - 1, 0, 1] = ht
    for x in range(N - 1):
        th[N - 1, x + 1, 1] = th[N - 1, x, 1] + phi[N - 1, x] - th[N - 1, x, 0] + th[0, x, 0]
    return th


def gaussian_complex(n: int, *words: int) -> np.ndarray:
    """Complex vector of length n with independent N(0,1) real and imaginary parts."""
    rng = rng_for(*words)
    z = rng.standard_normal((n, 2))
    return z[:, 0] + 1j * z[:, 1]


def rhs(N: int, cfg: int, j: int) -> np.ndarray:
    """Gaussian right-hand side j of configuration cfg, fine layout [t][x][spin]."""
    return gaussian_complex(2 * N * N, N, cfg, 3, j)


def near_null_starts(N: int, cfg: int, level: int, nvec: int = 12, dof: int | None = None) -> np.ndarray:
    """Random start vectors x_i (rows) for the near-null solves at ``level``.

    Level 0 vectors live on the fine lattice (2 dof per site); level 1 vectors on
    the lattice blocked by 4 in each direction with 24 dof per site.
    """
    if dof is None:
        dof = 2 * N * N if level == 0 else 24 * (N // 4) * (N // 4)
    return np.stack([gaussian_complex(dof, N, cfg, 1 + level, i) for i in range(nvec)])


def critical_mass(N: int, cfg: int) -> float:
    """m_c of configuration (N, cfg), as stored by the oracle's eigenvalue scan."""
    with open(MCRIT_FILE) as f:
        table = json.load(f)
    key = f"{N}/{cfg}"
    if key not in table["mc"]:
        raise KeyError(f"no critical mass stored for lattice {N}^2 configuration {cfg}")
    return float(table["mc"][key])


def bare_mass(N: int, cfg: int) -> float:
    """Bare mass m0 = m_c + 0.01 of configuration (N, cfg)."""
    return critical_mass(N, cfg) + MASS_OFFSET
