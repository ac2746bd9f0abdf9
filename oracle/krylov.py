"""Global Krylov vectors by MPO application (oracle; test infrastructure only).

Section I.B: the basis of psi is enlarged with the states
(1 - i tau H)^l |psi>, l = 1..k-1 (eq. (10)), each produced by applying the
MPO of 1 - i tau H to the previous one with the density-matrix approach
(exact for small MPO bond dimension), truncated with the cutoff eps_K.

Density-matrix application of an MPO O to |phi>, written out:

* right double-layer environments, built right to left from E_N = 1:
  E_i[a,al,al',a'] = sum M_i[a,s,b] W_i[al,be,t,s] E_{i+1}[b,be,be',b']
                     conj(W_i[al',be',t,s']) conj(M_i[a',s',b'])
  (E_i is the partial trace over sites i..N-1 of O|phi><phi|O^dagger);
* a left-to-right sweep carrying X[k,al,a] = the exact left part of O|phi>
  projected on the kept left basis k, starting from X = 1.  At site i:
  Y[k,t,be,b] = sum X[k,al,a] M_i[a,s,b] W_i[al,be,t,s];
  the reduced density matrix of the left block is
  rho[(k,t),(k',t')] = sum Y[k,t,be,b] E_{i+1}[b,be,be',b'] conj(Y[k',t',be',b']);
  its leading eigenvectors (descending eigenvalues) form A_i, and
  X <- A_i^dagger Y;
* the last site takes C = Y with the trivial right boundary.

Readings: the eps_K cut discards eigenvalues while their sum stays
<= eps_K * Tr(rho) (at most chi_max kept, at least one); each Krylov vector
is normalised to unit norm (section I.B offers both normalisation and the
(1 - i tau H)^l form; both are used).  The result is left-canonical with its
center on the last site.
"""
from __future__ import annotations

import numpy as np

from . import mps as M
from .tdvp import keep_count


def double_layer_envs(mps, Ws):
    """E[i] for i = 1..N (E[N] is the trivial boundary)."""
    N = len(mps)
    E = [None] * (N + 1)
    E[N] = np.ones((1, 1, 1, 1), dtype=np.complex128)
    for i in range(N - 1, 0, -1):
        E[i] = _env_step(mps[i], Ws[i], E[i + 1])
    return E


def _env_step(Mi, Wi, E):
    # E_new[a,x,X,A] = sum M[a,s,b] W[x,y,t,s] E[b,y,Y,B] conj(W[X,Y,t,S]) conj(M[A,S,B])
    F1 = np.tensordot(Mi, E, axes=([2], [0]))             # [a,s,y,Y,B]
    F2 = np.tensordot(F1, Wi, axes=([1, 2], [3, 1]))      # [a,Y,B,x,t]
    F3 = np.tensordot(F2, np.conj(Wi), axes=([1, 4], [1, 2]))   # [a,B,x,X,S]
    return np.tensordot(F3, np.conj(Mi), axes=([1, 4], [2, 1]))  # [a,x,X,A]


def _left_block(X, Mi, Wi):
    # Y[k,t,y,b] = sum X[k,x,a] M[a,s,b] W[x,y,t,s]
    T1 = np.tensordot(X, Mi, axes=([2], [0]))             # [k,x,s,b]
    T2 = np.tensordot(T1, Wi, axes=([1, 2], [0, 3]))      # [k,b,y,t]
    return np.ascontiguousarray(T2.transpose(0, 3, 2, 1))


def apply_mpo_denmat(mps, Ws, eps_K, chi_max, normalize=True):
    """O|phi> truncated by the density-matrix algorithm; returns (mps, discarded)."""
    N = len(mps)
    E = double_layer_envs(mps, Ws)
    X = np.ones((1, 1, 1), dtype=np.complex128)            # [k, al, a]
    out = []
    disc_total = 0.0
    for i in range(N - 1):
        Y = _left_block(X, mps[i], Ws[i])
        kd, d = Y.shape[0], Y.shape[1]
        # rho[k,t,K,T] = sum Y[k,t,y,b] E[b,y,Y,B] conj(Y[K,T,Y,B])
        G = np.tensordot(Y, E[i + 1], axes=([2, 3], [1, 0]))  # [k,t,Y,B]
        rho = np.tensordot(G, np.conj(Y), axes=([2, 3], [2, 3]))
        rho = rho.reshape(kd * d, kd * d)
        rho = 0.5 * (rho + rho.conj().T)
        lam, U = np.linalg.eigh(rho)
        lam, U = lam[::-1], U[:, ::-1]
        n = keep_count(lam, eps_K, float(np.trace(rho).real), chi_max)
        disc_total += float(np.clip(lam[n:], 0, None).sum())
        A = U[:, :n]
        out.append(A.reshape(kd, d, n))
        X = np.tensordot(np.conj(A), Y.reshape(kd * d, *Y.shape[2:]), axes=([0], [0]))
    Y = _left_block(X, mps[N - 1], Ws[N - 1])
    C = Y[:, :, 0, 0][:, :, None]
    if normalize:
        C = C / np.linalg.norm(C)
    out.append(C)
    return out, disc_total


def apply_mpo_exact(mps, Ws):
    """O|phi> with bond dimension m*w (no truncation): direct product of tensors."""
    out = []
    for Mi, Wi in zip(mps, Ws):
        T = np.tensordot(Wi, Mi, axes=([3], [1])).transpose(0, 3, 2, 1, 4)   # [x,a,t,y,b]
        out.append(T.reshape(Wi.shape[0] * Mi.shape[0], 2, Wi.shape[1] * Mi.shape[2]))
    return out


def svd_compress(mps, eps, chi_max):
    """Right-canonicalise, then truncated SVDs left to right (same cut rule).

    For a right-canonical input the reduced density matrix of the left block
    at each bond is C C^dagger, so this is the same truncation as the density
    matrix route; used only to cross-check it.
    """
    psi = M.right_canonicalize(mps)
    N = len(psi)
    disc = 0.0
    for i in range(N - 1):
        ml, d, mr = psi[i].shape
        U, S, Vh = np.linalg.svd(psi[i].reshape(ml * d, mr), full_matrices=False)
        w = S ** 2
        n = keep_count(w, eps, w.sum(), chi_max)
        disc += float(w[n:].sum())
        psi[i] = U[:, :n].reshape(ml, d, n)
        psi[i + 1] = np.tensordot(S[:n, None] * Vh[:n], psi[i + 1], axes=(1, 0))
    return psi, disc


def krylov_vectors(psi, Ws_op, k, eps_K, chi_max, apply="denmat", fit_passes=3):
    """[(1 - i tau H)^l psi, l = 1..k-1], each normalised and truncated, by
    the density-matrix route or (apply="fit") by variational fitting."""
    from .fit import apply_mpo_variational
    out = []
    cur = psi
    for _ in range(k - 1):
        if apply == "fit":
            cur, _ = apply_mpo_variational(cur, Ws_op, eps_K, chi_max, fit_passes)
        else:
            cur, _ = apply_mpo_denmat(cur, Ws_op, eps_K, chi_max)
        out.append(cur)
    return out
