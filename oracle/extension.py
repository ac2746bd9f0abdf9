"""State-averaged basis extension (oracle; test infrastructure only).

Section I.A, the reformed algorithm (eqs. (5)-(7)) with the center moves of
eq. (3).  Inputs: psi and the k-1 Krylov vectors psi~_l, all left-canonical
with their centers on the last site (eq. (1)).  Sweeping from the right end
to site 1, at site i:

1. SVD the center of psi without truncation, C = U S B (reading: only
   directions whose weight s^2 is at round-off level, s^2 <= 1e-14 s_1^2 --
   the numerical-zero floor shared by every cut -- are left out; they carry
   no weight and would otherwise put arbitrary rows into B);
2. project every Krylov center on the null space of B, X_l = C~_l P with
   P = 1 - B^dagger B, and mix rho_bar = sum_l X_l^dagger X_l = P rho~ P
   (eqs. (5)-(6));
3. diagonalise rho_bar = B_bar^dagger S_bar^2 B_bar and keep the leading rows
   by the cutoff eps_M (reading: the discarded eigenvalue sum stays
   <= eps_M * Tr rho~ with Tr rho~ = sum_l |C~_l|^2; at most chi_max - r rows
   and at most d m' - r; zero rows allowed; nothing when P = 0);
4. re-orthogonalise B_bar against B and orthonormalise it (QR), then
   B' = [B; B_bar] (eq. (7)) is the new right-orthonormal tensor at site i;
5. move the centers one site left, separately per state (eq. (3)):
   C_{i-1} = A_{i-1} C_i B'^dagger and C~_{i-1} = A~_{i-1} C~_i B'^dagger.

The Krylov centers are discarded at the end; psi is returned right-canonical
with its center at site 0 and is unchanged as a state.
"""
from __future__ import annotations

import numpy as np

from . import mps as M
from .tdvp import keep_count

RANK_WEIGHT_REL = 1e-14


def _rank(S):
    if len(S) == 0 or S[0] <= 0.0:
        return 0
    return int(np.count_nonzero(S ** 2 > RANK_WEIGHT_REL * S[0] ** 2))


def extension_step(C, Ct_list, eps_M, chi_max, use_gram_of_stack=False):
    """Rows B' (eq. (7)) for one site; C: (m, d m') matrix, Ct_list: (m~_l, d m')."""
    U, S, Vh = np.linalg.svd(C, full_matrices=False)
    r = _rank(S)
    B = Vh[:r]
    D = C.shape[1]
    Xs = [Ct - (Ct @ B.conj().T) @ B for Ct in Ct_list]
    tr_ref = float(sum(np.vdot(Ct, Ct).real for Ct in Ct_list))
    cap = min(chi_max - r, D - r)
    if cap <= 0 or not Xs:
        return B, r, 0
    if use_gram_of_stack:
        # equivalent route (eq. (6) remark): SVD of the stacked projected centers
        Xst = np.vstack(Xs)
        _, s2, vh2 = np.linalg.svd(Xst, full_matrices=False)
        lam, Bbar_all = s2 ** 2, vh2
    else:
        rho_bar = sum(X.conj().T @ X for X in Xs)
        rho_bar = 0.5 * (rho_bar + rho_bar.conj().T)
        lam, V = np.linalg.eigh(rho_bar)
        lam, V = lam[::-1], V[:, ::-1]
        Bbar_all = V.conj().T
    n = keep_count(lam, eps_M, tr_ref, cap, min_keep=0)
    # only directions that carry weight are meaningful
    n = min(n, int(np.count_nonzero(lam > 1e-14 * max(tr_ref, 1e-300))))
    if n == 0:
        return B, r, 0
    Bbar = Bbar_all[:n]
    Bbar = Bbar - (Bbar @ B.conj().T) @ B
    q, _ = np.linalg.qr(Bbar.conj().T, mode="reduced")
    Bbar = q.conj().T
    return np.vstack([B, Bbar]), r, n


def basis_extension(psi, krylovs, eps_M, chi_max, use_gram_of_stack=False):
    """Extend the bond bases of psi by the Krylov vectors; returns (psi', stats)."""
    psi = M.copy(psi)
    kv = [M.copy(k) for k in krylovs]
    N = len(psi)
    added = []
    for i in range(N - 1, 0, -1):
        ml, d, mr = psi[i].shape
        C = psi[i].reshape(ml, d * mr)
        Cts = [k[i].reshape(k[i].shape[0], d * mr) for k in kv]
        Bp, r, n = extension_step(C, Cts, eps_M, chi_max, use_gram_of_stack)
        added.append(n)
        psi[i] = Bp.reshape(Bp.shape[0], d, mr)
        psi[i - 1] = np.tensordot(psi[i - 1], C @ Bp.conj().T, axes=(2, 0))
        for k, Ct in zip(kv, Cts):
            k[i - 1] = np.tensordot(k[i - 1], Ct @ Bp.conj().T, axes=(2, 0))
    return psi, {"added": added[::-1]}


def direct_sum_extension(psi, krylovs):
    """First formulation of section I.A (eqs. (2)-(4)): stack the states,
    sweep right to left with untruncated SVDs of the stacked center, move the
    centers separately (eq. (3)) and keep only psi's center.  Used only to
    cross-check that the reformed algorithm spans the same bond spaces."""
    states = [M.copy(psi)] + [M.copy(k) for k in krylovs]
    N = len(psi)
    out = M.copy(psi)
    for i in range(N - 1, 0, -1):
        d, mr = states[0][i].shape[1], states[0][i].shape[2]
        Cs = [s[i].reshape(s[i].shape[0], d * mr) for s in states]
        stack = np.vstack(Cs)
        _, S, Vh = np.linalg.svd(stack, full_matrices=False)
        Bp = Vh[:_rank(S)]
        out[i] = Bp.reshape(Bp.shape[0], d, mr)
        for s, Cm in zip(states, Cs):
            s[i - 1] = np.tensordot(s[i - 1], Cm @ Bp.conj().T, axes=(2, 0))
        out[i - 1] = states[0][i - 1]
    return out
