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
