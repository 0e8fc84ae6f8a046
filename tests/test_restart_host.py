"""The long-cycle GMRES-DR dense steps (harmonic-Ritz restart, Arnoldi column update with its
Givens rotations, least-squares solve) compiled for the host and run on one thread, against
the oracle's harmonic-Ritz restart (oracle.krylov) and numpy least squares.

The Arnoldi matrices come from the oracle's Arnoldi process on the Wilson-Dirac operator of
a near-critical 32^2 configuration, at the paper's sizes (m = 200, k = 40) and at smaller ones.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle import krylov, wilson

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cxx = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(cxx):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("rh")
    exe = d / "restart_host"
    r = subprocess.run([cxx, "-O2", "-std=c++17", "--offload-arch=gfx950", os.path.join(ROOT, "tests", "restart_host.cpp"),
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe, d


def _arnoldi(m, N=32, cfg=0, m0=-0.0747, seed=3):
    """Arnoldi relation A V_m = V_{m+1} Hbar_m of the oracle's D (modified Gram-Schmidt twice).
    The 32^2 configuration 0 at 0.01 above its critical mass (-0.08467): 200 steps leave a
    relative residual near 1e-2, as a restart meets it."""
    D = wilson.dirac_matrix(synth.gauge_angles(N, cfg), m0)
    n = D.shape[0]
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    V = np.zeros((n, m + 1), complex)
    H = np.zeros((m + 1, m), complex)
    V[:, 0] = v / np.linalg.norm(v)
    for j in range(m):
        w = D @ V[:, j]
        h, w = krylov._mgs2(V, j, w)
        H[: j + 1, j] = h
        H[j + 1, j] = np.linalg.norm(w)
        V[:, j + 1] = w / H[j + 1, j]
    return D, V, H, np.linalg.norm(v)


def _run(harness, mode, payload):
    exe, d = harness
    fi, fo = d / "in.bin", d / "out.bin"
    fi.write_bytes(payload)
    r = subprocess.run([str(exe), mode, str(fi), str(fo)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return np.frombuffer(fo.read_bytes(), dtype=np.uint8)


class _Reader:
    def __init__(self, buf):
        self.b, self.o = buf.tobytes(), 0

    def ints(self, n):
        v = np.frombuffer(self.b, dtype=np.int32, count=n, offset=self.o)
        self.o += 4 * n
        return v

    def dbl(self, n):
        v = np.frombuffer(self.b, dtype=np.float64, count=n, offset=self.o)
        self.o += 8 * n
        return v

    def cx(self, n):
        v = np.frombuffer(self.b, dtype=np.complex128, count=n, offset=self.o)
        self.o += 16 * n
        return v.copy()


def _principal_sines(A, B):
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    sv = np.linalg.svd(qa.conj().T @ qb, compute_uv=False)
    return np.sqrt(np.maximum(0.0, 1.0 - sv ** 2)).max()


@pytest.mark.parametrize("m,k,final", [(200, 40, 0), (200, 40, 1), (60, 20, 0), (30, 10, 1)])
def test_restart_against_oracle(harness, m, k, final):
    D, V, H, beta = _arnoldi(m)
    c = np.zeros(m + 1, complex)
    c[0] = beta
    y = np.linalg.lstsq(H, c, rcond=None)[0]
    u = c - H @ y
    assert np.linalg.norm(u) > 1e-6 * beta  # a cycle that has not converged
    payload = np.array([m, k, final], np.int32).tobytes() + H.T.astype(np.complex128).tobytes() + \
        c.tobytes() + u.tobytes()
    rd = _Reader(_run(harness, "restart", payload))
    status, nrot = rd.ints(2)
    est = rd.dbl(1)[0]
    theta = rd.cx(k)
    P = rd.cx((m + 1) * (k + 1)).reshape(k + 1, m + 1).T
    Hk = rd.cx((k + 1) * k).reshape(k, k + 1).T
    cn = rd.cx(k + 1)
    gn = rd.cx(k + 1)
    assert status == 0
    # the oracle's restart of the same relation
    theta_o, _ = krylov.harmonic_ritz(H, k)
    s = u if not final else None
    _, Hk_o, P_o, _ = krylov._compress(V, H, k, s)
    # kept harmonic Ritz values: the same set
    dist = np.abs(theta[:, None] - theta_o[None, :])
    assert np.max(dist.min(axis=1) / np.abs(theta)) < 1e-8
    # P orthonormal, the same span as the oracle's (to the sensitivity of the kept invariant
    # subspace: rounding over the gap between kept and dropped harmonic Ritz values), last row of
    # P_k zero
    assert np.linalg.norm(P.conj().T @ P - np.eye(k + 1)) < 1e-12
    assert _principal_sines(P, P_o) < 1e-6
    assert np.max(np.abs(P[m, :k])) < 1e-14
    # the kept relation: Hbar P_k = P Hbar_k
    assert np.linalg.norm(H @ P[:m, :k] - P @ Hk) < 1e-11 * np.linalg.norm(H)
    # the same small matrix up to the basis change: equal eigenvalues of its top k x k block
    ev = np.sort_complex(np.linalg.eigvals(Hk[:k, :k]))
    ev_o = np.sort_complex(np.linalg.eigvals(Hk_o[:k, :k]))
    assert np.max(np.abs(ev - ev_o)) < 1e-8 * np.abs(ev_o).max()
    if not final:
        sv = u
        assert np.linalg.norm(cn - P.conj().T @ sv) < 1e-12 * np.linalg.norm(sv)
        # Givens QR of the kept block: k (k+1) / 2 rotations, |g_k| is the least-squares residual
        assert nrot == k * (k + 1) // 2
        d = np.linalg.lstsq(Hk, cn, rcond=None)[0]
        assert abs(est - np.linalg.norm(cn - Hk @ d)) < 1e-10 * np.linalg.norm(cn)


@pytest.mark.parametrize("m,k,m2", [(200, 40, 200), (200, 40, 120), (48, 16, 40)])
def test_columns_and_least_squares(harness, m, k, m2):
    """Columns appended one by one (held rotations, a new one each) solve the least-squares
    problem of the Arnoldi matrix; after a restart, new columns appended to the kept block solve
    the problem of the combined matrix."""
    D, V, H, beta = _arnoldi(m)
    rng = np.random.default_rng(7)
    H2 = np.triu(rng.standard_normal((m2 + 1, m2)) + 1j * rng.standard_normal((m2 + 1, m2)), -1)
    idx = np.arange(m2)
    H2[idx + 1, idx] = np.abs(H2[idx + 1, idx])  # Arnoldi subdiagonals are norms
    payload = np.array([m, k], np.int32).tobytes() + H.T.astype(np.complex128).tobytes() + \
        np.array([beta]).tobytes() + np.array([m2], np.int32).tobytes() + H2.T.astype(np.complex128).tobytes()
    rd = _Reader(_run(harness, "columns", payload))
    steps = rd.ints(1)[0]
    est = rd.dbl(1)[0]
    y = rd.cx(steps)
    c = np.zeros(m + 1, complex)
    c[0] = beta
    y_o = np.linalg.lstsq(H, c, rcond=None)[0]
    assert steps == m
    assert np.linalg.norm(y - y_o) < 1e-9 * np.linalg.norm(y_o)
    assert abs(est - np.linalg.norm(c - H @ y_o)) < 1e-10 * beta
    status = rd.ints(1)[0]
    P = rd.cx((m + 1) * (k + 1))
    Hk = rd.cx((k + 1) * k).reshape(k, k + 1).T
    cn = rd.cx(k + 1)
    steps2 = rd.ints(1)[0]
    est2 = rd.dbl(1)[0]
    y2 = rd.cx(steps2)
    assert status == 0 and steps2 == m2
    C = H2.copy()
    C[:, :k] = 0.0
    C[: k + 1, :k] = Hk
    rhs = np.zeros(m2 + 1, complex)
    rhs[: k + 1] = cn
    y2_o = np.linalg.lstsq(C, rhs, rcond=None)[0]
    # the appended random columns may leave the combined matrix nearly rank deficient, so the
    # minimiser is compared through the residual it reaches (and the estimate through it)
    res2 = np.linalg.norm(rhs - C @ y2)
    assert res2 <= np.linalg.norm(rhs - C @ y2_o) + 1e-10 * np.linalg.norm(rhs)
    assert abs(est2 - res2) < 1e-10 * np.linalg.norm(rhs)
