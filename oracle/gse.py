"""One GSE-TDVP1 time step (oracle; test infrastructure only).

Section I.C: (1) build the MPO of 1 - i tau H and apply it k-1 times to psi
(cutoff eps_K, eq. (10)), by the density-matrix or the variational route;
(2) extend the basis of psi by those states, ending with the center at the
first site (cutoff eps_M, section I.A); (3) one-site TDVP sweep left to right
then right to left (cutoff eps).

Reading: the expansion is skipped when every bond of psi is already at its
largest useful size min(chi_max, 2^(i+1), 2^(N-i-1)) (the introduction notes
the enlargement is easy to turn off); psi is still brought to the gauge the
sweep needs.
"""
from __future__ import annotations

from . import extension as X
from . import krylov as K
from . import mps as M
from . import tdvp as T


def gse_step(psi, Ws_H, Ws_op, dt, k, eps_K, eps_M, eps, chi_max,
             tol=1e-12, maxiter=30, normalize=False, apply="denmat", fit_passes=3):
    stats = {}
    N = len(psi)
    full = all(m >= c for m, c in zip(M.bond_dims(psi), M.max_bond_dims(N, chi_max)))
    if k >= 2 and not full:
        psi_l = M.left_canonicalize(psi)
        kv = K.krylov_vectors(psi_l, Ws_op, k, eps_K, chi_max, apply, fit_passes)
        psi_e, xs = X.basis_extension(psi_l, kv, eps_M, chi_max)
        stats["krylov_bonds"] = [M.bond_dims(v) for v in kv]
        stats["added"] = xs["added"]
    else:
        psi_e = M.right_canonicalize(psi)
        stats["added"] = [0] * (N - 1)
    stats["bonds_extended"] = M.bond_dims(psi_e)
    psi_t, st = T.tdvp1_sweep(psi_e, Ws_H, dt, eps, chi_max, tol, maxiter, normalize)
    stats.update(st)
    return psi_t, stats
