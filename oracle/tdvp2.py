"""Two-site TDVP (oracle; test infrastructure only).

The conventional two-site TDVP step with which sections I.C and II compare
GSE-TDVP1 (the cost ratio at equal bond dimension in section I.C, the
benchmarks of Figs. 3 and 4).  It is the projector-splitting integrator of
the introduction with two-site local updates; the readings match the one-site
sweep of ``oracle.tdvp``:

* symmetric second-order sweep: left to right over the bond pairs (i, i+1)
  with dt/2 each, then right to left with dt/2; the two evolutions of the
  last pair are merged into one evolution by dt;
* forward pair evolution exp(-i dt/2 H2_eff) of Theta = C_i B_{i+1}, a split
  by a truncated SVD (discarded weight <= eps ||Theta||^2, at most chi_max
  kept, the numerical-zero floor and multiplet rule of ``keep_count``; with
  eps = 0 only zero weights and the cap cut), and a backward evolution
  exp(+i dt/2 H1_eff) of the new one-site center, except after the last pair
  of each half sweep;
* with ``normalize`` every local result is renormalised (imaginary time).

Two-site effective Hamiltonian (definition):
    Y[a',t,u,b'] = sum L[a',al,a] W1[al,be,t,s] W2[be,ga,u,v] Th[a,s,v,b] R[b',ga,b]
    (einsum 'xAa,ABts,BGuv,asvb,yGb->xtuy').
"""
from __future__ import annotations

import numpy as np

from . import mps as M
from .tdvp import (boundary_env, expm_krylov, heff_apply, keep_count, left_env_update, right_env_update,
                   right_envs)


def heff2_apply(L, W1, W2, R, Th):
    """Two-site H_eff on Th[a,s,v,b], evaluated as pairwise tensordot stages."""
    T1 = np.tensordot(L, Th, axes=(2, 0))                  # [a',al,s,v,b]
    T2 = np.tensordot(T1, W1, axes=([1, 2], [0, 3]))       # [a',v,b,be,t]
    T3 = np.tensordot(T2, W2, axes=([3, 1], [0, 3]))       # [a',b,t,ga,u]
    return np.tensordot(T3, R, axes=([3, 1], [1, 2]))      # [a',t,u,b']


def _svd_cut(Thm, eps, chi_max):
    U, S, Vh = np.linalg.svd(Thm, full_matrices=False)
    w = S ** 2
    n = keep_count(w, eps, w.sum(), chi_max)
    return U[:, :n], S[:n], Vh[:n], float(w[n:].sum())


def split2_left(Th, eps, chi_max):
    """Th[a,s,v,b] -> A[a,s,k] (left-orthonormal) and C[k,v,b] = S V^dagger."""
    ml, d1, d2, mr = Th.shape
    U, S, Vh, disc = _svd_cut(Th.reshape(ml * d1, d2 * mr), eps, chi_max)
    n = len(S)
    return U.reshape(ml, d1, n), (S[:, None] * Vh).reshape(n, d2, mr), disc


def split2_right(Th, eps, chi_max):
    """Th[a,s,v,b] -> C[a,s,k] = U S and B[k,v,b] (right-orthonormal)."""
    ml, d1, d2, mr = Th.shape
    U, S, Vh, disc = _svd_cut(Th.reshape(ml * d1, d2 * mr), eps, chi_max)
    n = len(S)
    return (U * S[None, :]).reshape(ml, d1, n), Vh.reshape(n, d2, mr), disc


def tdvp2_sweep(mps, Ws, dt, eps=0.0, chi_max=10 ** 9, tol=1e-12, maxiter=30, normalize=False):
    """One symmetric two-site TDVP sweep (left->right then right->left).

    Precondition: center at site 0, sites 1..N-1 right-canonical (N >= 2).
    Postcondition: the same.  Returns (mps, stats)."""
    psi = M.copy(mps)
    N = len(psi)
    if N < 2:
        raise ValueError("two-site TDVP needs at least two sites")
    half = dt / 2.0
    R = right_envs(psi, Ws)
    L = [None] * (N + 1)
    L[0] = boundary_env()
    stats = {"n_matvec": 0, "n_back": 0, "discarded": 0.0}

    def evolve(f, x, step, key):
        y, n = expm_krylov(lambda v: f(v.reshape(x.shape)).ravel(), x.ravel(), step, tol, maxiter)
        stats[key] += n
        y = y.reshape(x.shape)
        return y / np.linalg.norm(y) if normalize else y

    def evolve_pair(i, Th, step):
        return evolve(lambda x: heff2_apply(L[i], Ws[i], Ws[i + 1], R[i + 2], x), Th, step, "n_matvec")

    def evolve_site(i, C, step):
        return evolve(lambda x: heff_apply(L[i], Ws[i], R[i + 1], x), C, step, "n_back")

    # left -> right
    for i in range(N - 1):
        Th = np.tensordot(psi[i], psi[i + 1], axes=(2, 0))
        if i < N - 2:
            Th = evolve_pair(i, Th, half)
            A, C, disc = split2_left(Th, eps, chi_max)
            stats["discarded"] += disc
            psi[i] = A
            L[i + 1] = left_env_update(L[i], A, Ws[i])
            psi[i + 1] = evolve_site(i + 1, C, -half)
        else:
            # last pair: both half steps merged; the center moves left
            Th = evolve_pair(i, Th, dt)
            C, B, disc = split2_right(Th, eps, chi_max)
            stats["discarded"] += disc
            psi[i], psi[i + 1] = C, B
            R[i + 1] = right_env_update(R[i + 2], B, Ws[i + 1])
    # right -> left
    for i in range(N - 3, -1, -1):
        psi[i + 1] = evolve_site(i + 1, psi[i + 1], -half)
        Th = np.tensordot(psi[i], psi[i + 1], axes=(2, 0))
        Th = evolve_pair(i, Th, half)
        C, B, disc = split2_right(Th, eps, chi_max)
        stats["discarded"] += disc
        psi[i], psi[i + 1] = C, B
        R[i + 1] = right_env_update(R[i + 2], B, Ws[i + 1])
    return psi, stats
