"""Observables (oracle; test infrastructure only).

Energy <H>/<psi|psi> (sections II.A and II.B measure it), <S^z_i>, fidelity,
and the one-axis-twisting moments of eqs. (13)-(15).
"""
from __future__ import annotations

import numpy as np

from . import ed
from . import mps as M
from .tdvp import left_env_update


def energy(psi, Ws) -> float:
    """<psi|H|psi>/<psi|psi> by a left-to-right contraction through the MPO."""
    L = np.ones((1, 1, 1), dtype=np.complex128)
    for t, W in zip(psi, Ws):
        L = left_env_update(L, t, W)
    return float(L[0, 0, 0].real / M.inner(psi, psi).real)


def sz(psi) -> np.ndarray:
    return M.local_expectations(psi, ed.SZ).real


def sx_total(psi) -> float:
    return float(M.local_expectations(psi, ed.SX).real.sum())


def oat_sx_exact(N: int, t: float) -> float:
    """Closed form of eq. (13): <S^x(t)> = (N/2) cos^(N-1)(t)."""
    return 0.5 * N * np.cos(t) ** (N - 1)


def oat_t_opt(N: int) -> float:
    """Optimal squeezing time quoted in section II.B: 12^(1/6) (N/2)^(-2/3) / 2."""
    return 12.0 ** (1.0 / 6.0) * (N / 2.0) ** (-2.0 / 3.0) / 2.0


def xi2_from_moments(N, sx, syy, szz, syz, szy):
    """Eq. (15): xi^2/N = (s_yy + s_zz - sqrt((s_yy - s_zz)^2 + (s_yz + s_zy)^2)) / (2 <S^x>^2),
    with s_ab = <S^a S^b> (the paper writes sigma_ab^2 for this second moment)."""
    return N * (syy + szz - np.sqrt((syy - szz) ** 2 + (syz + szy) ** 2)) / (2.0 * sx ** 2)


def dicke_spin_matrices(N: int):
    """Total-spin operators J_x, J_y, J_z on the symmetric subspace, j = N/2,
    basis m = j, j-1, ..., -j, with J_+|j,m> = sqrt(j(j+1) - m(m+1))|j,m+1>."""
    j = 0.5 * N
    m = j - np.arange(N + 1)
    Jp = np.zeros((N + 1, N + 1))
    for k in range(1, N + 1):
        Jp[k - 1, k] = np.sqrt(j * (j + 1) - m[k] * (m[k] + 1))
    Jm = Jp.T
    return 0.5 * (Jp + Jm), -0.5j * (Jp - Jm), np.diag(m)


def oat_moments_dicke(N: int, t: float) -> dict:
    """Exact one-axis-twisting dynamics (eq. (12) with chi = 1) from the +x
    product state, which lies in the symmetric subspace (the top eigenvector
    of J_x): psi(t) = exp(-i t J_z^2) psi(0).  Returns <S^a> and the second
    moments s_ab = <S^a S^b> that eq. (15) takes, plus the anticommutator
    s_yz + s_zy."""
    Jx, Jy, Jz = dicke_spin_matrices(N)
    _, V = np.linalg.eigh(Jx)
    psi = np.exp(-1j * t * np.diag(Jz) ** 2) * V[:, -1]
    ev = lambda A: complex(np.vdot(psi, A @ psi))
    out = {"sx": ev(Jx).real, "sy": ev(Jy).real, "sz": ev(Jz).real, "syy": ev(Jy @ Jy).real,
           "szz": ev(Jz @ Jz).real, "syz": ev(Jy @ Jz), "szy": ev(Jz @ Jy)}
    out["syz_szy"] = (out["syz"] + out["szy"]).real
    return out


def oat_xi2_dicke(N: int, t: float) -> float:
    m = oat_moments_dicke(N, t)
    return float(xi2_from_moments(N, m["sx"], m["syy"], m["szz"], m["syz_szy"], 0.0))


def xi2_dense(psi_vec: np.ndarray, N: int) -> float:
    """Eq. (14) evaluated directly: N min over n_perp of the variance along
    n_perp divided by <S>^2, by scanning the angle in the y-z plane."""
    Sy = sum(ed.site_op(ed.SY, i, N) for i in range(N))
    Sz = sum(ed.site_op(ed.SZ, i, N) for i in range(N))
    Sx = sum(ed.site_op(ed.SX, i, N) for i in range(N))
    sx = ed.expect(Sx, psi_vec).real
    best = np.inf
    for th in np.linspace(0.0, np.pi, 20001):
        S = np.cos(th) * Sy + np.sin(th) * Sz
        var = ed.expect(S @ S, psi_vec).real - ed.expect(S, psi_vec).real ** 2
        best = min(best, var)
    return float(N * best / sx ** 2)
