"""One-site TDVP (oracle; test infrastructure only).

Section I.C, step 3: a conventional one-site TDVP sweep left to right and then
right to left, in the projector-splitting (Lie-Trotter) integration scheme the
introduction refers to.  The paper does not spell out the integrator; the
readings used here are:

* symmetric second-order sweep: the left-to-right half-sweep evolves every
  site by dt/2 and the right-to-left half-sweep by another dt/2; the two
  evolutions of the last site are merged into one evolution by dt;
* forward site evolution exp(-i dt/2 H_eff), backward bond evolution
  exp(+i dt/2 K_eff) (imaginary time uses dt = -i dtau, which turns these into
  exp(-dtau/2 H_eff) and exp(+dtau/2 K_eff));
* the cutoff eps of section I.B (used only when unitarity is not required)
  acts at the gauge moves: eps = 0 uses QR/LQ, eps > 0 uses an SVD that drops
  the smallest singular values while the discarded weight stays
  <= eps * ||C||^2, with at most chi_max kept;
* with ``normalize`` the site and bond tensors are renormalised after every
  local evolution (imaginary time).

Tensor conventions: L[a', alpha, a], R[b', beta, b] (primed index on the bra
side), W[alpha, beta, s', s], C[a, s, b].
"""
from __future__ import annotations

import numpy as np

from . import mps as M

# Weights (squared singular values or density-matrix eigenvalues) below this
# fraction of the largest one are treated as numerical zeros.
WEIGHT_FLOOR = 1e-14
# Two neighbouring weights closer than this fraction of the largest weight
# belong to one multiplet and are never split by a cut.
TIE_REL = 1e-12


# --------------------------------------------------------------------------
# Environments and effective Hamiltonians
# --------------------------------------------------------------------------

def left_env_update(L, A, W):
    """L_new[b', beta, b] = sum conj(A[a',s',b']) L[a',alpha,a] W[alpha,beta,s',s] A[a,s,b]."""
    T1 = np.tensordot(L, A, axes=([2], [0]))              # [a',al,s,b]
    T2 = np.tensordot(T1, W, axes=([1, 2], [0, 3]))       # [a',b,be,s']
    out = np.tensordot(np.conj(A), T2, axes=([0, 1], [0, 3]))  # [b',b,be]
    return np.ascontiguousarray(out.transpose(0, 2, 1))


def right_env_update(R, B, W):
    """R_new[a', alpha, a] = sum conj(B[a',s',b']) W[alpha,beta,s',s] R[b',beta,b] B[a,s,b]."""
    T1 = np.tensordot(B, R, axes=([2], [2]))              # [a,s,b',be]
    T2 = np.tensordot(T1, W, axes=([1, 3], [3, 1]))       # [a,b',al,s']
    out = np.tensordot(np.conj(B), T2, axes=([1, 2], [3, 1]))  # [a',a,al]
    return np.ascontiguousarray(out.transpose(0, 2, 1))


def heff_apply(L, W, R, C):
    """One-site effective Hamiltonian: y[a',s',b'] = sum L[a',al,a] W[al,be,s',s] C[a,s,b] R[b',be,b]."""
    T1 = np.tensordot(L, C, axes=([2], [0]))              # [a',al,s,b]
    T2 = np.tensordot(T1, W, axes=([1, 2], [0, 3]))       # [a',b,be,s']
    return np.tensordot(T2, R, axes=([1, 2], [2, 1]))     # [a',s',b']


def keff_apply(L, R, X):
    """Zero-site effective Hamiltonian: y[a',b'] = sum L[a',al,a] X[a,b] R[b',al,b]."""
    T1 = np.tensordot(L, X, axes=([2], [0]))              # [a',al,b]
    return np.tensordot(T1, R, axes=([1, 2], [1, 2]))     # [a',b']


def boundary_env():
    return np.ones((1, 1, 1), dtype=np.complex128)


def right_envs(mps, Ws):
    """R[i] for i = 1..N (R[i] covers sites i..N-1; R[N] is the trivial boundary)."""
    N = len(mps)
    R = [None] * (N + 1)
    R[N] = boundary_env()
    for i in range(N - 1, 0, -1):
        R[i] = right_env_update(R[i + 1], mps[i], Ws[i])
    return R


# --------------------------------------------------------------------------
# Lanczos exponential
# --------------------------------------------------------------------------

def expm_krylov(apply, v, dt, tol=1e-12, maxiter=30):
    """exp(-i dt H) v by a Lanczos process with full reorthogonalisation.

    v_1 = v/|v|; for each j: w = H v_j, alpha_j = Re<v_j|w>,
    w -= alpha_j v_j + beta_{j-1} v_{j-1}, then w is reorthogonalised against
    all previous vectors (twice) and beta_j = |w|.  With T_j the tridiagonal
    Lanczos matrix, c = exp(-i dt T_j) e_1 (through its eigendecomposition).
    Stop when beta_j |c_j| <= tol |c| (the next Krylov coefficient is
    negligible), on breakdown (beta_j <= 1e-14 max|T|), or after maxiter
    steps.  Returns (|v| V c, number of H applications).
    """
    nrm = np.linalg.norm(v)
    if nrm == 0.0:
        return np.array(v, copy=True), 0
    V = [v / nrm]
    alpha, beta = [], []
    c = np.ones(1, dtype=np.complex128)
    n_app = 0
    for j in range(maxiter):
        w = apply(V[j])
        n_app += 1
        a = float(np.vdot(V[j], w).real)
        w = w - a * V[j]
        if j > 0:
            w = w - beta[j - 1] * V[j - 1]
        for _ in range(2):
            for u in V:
                w = w - np.vdot(u, w) * u
        b = float(np.linalg.norm(w))
        alpha.append(a)
        T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
        lam, Q = np.linalg.eigh(T)
        c = Q @ (np.exp(-1j * dt * lam) * Q[0, :])
        scale = max(np.max(np.abs(alpha)), max(beta) if beta else 0.0)
        if b * abs(c[-1]) <= tol * np.linalg.norm(c) or b <= 1e-14 * scale or j == maxiter - 1:
            break
        beta.append(b)
        V.append(w / b)
    y = np.zeros_like(V[0])
    for cj, u in zip(c, V):
        y = y + cj * u
    return nrm * y, n_app


# --------------------------------------------------------------------------
# Truncation rule shared by every cut in the oracle
# --------------------------------------------------------------------------

def keep_count(weights, eps, trace_ref, cap, min_keep=1):
    """Number of leading weights (sorted descending) to keep.

    Smallest n with sum(weights[n:]) <= eps * trace_ref, never keeping weights
    below WEIGHT_FLOOR * weights[0]; a multiplet straddling that cut is kept
    whole; then at most `cap` (a multiplet straddling the cap is dropped
    whole), and at least `min_keep`.
    """
    w = np.clip(np.asarray(weights, dtype=np.float64), 0.0, None)
    n_all = len(w)
    if n_all == 0:
        return 0
    w0 = w[0]
    if w0 <= 0.0:
        return min(min_keep, n_all, cap) if cap > 0 else 0
    tail = np.concatenate([np.cumsum(w[::-1])[::-1], [0.0]])   # tail[n] = sum w[n:]
    n = 0
    while n < n_all and (tail[n] > eps * trace_ref) and w[n] > WEIGHT_FLOOR * w0:
        n += 1
    while 0 < n < n_all and w[n] > WEIGHT_FLOOR * w0 and (w[n - 1] - w[n]) <= TIE_REL * w0:
        n += 1
    if n > cap:
        n = cap
        nc = n
        while 0 < nc < n_all and (w[nc - 1] - w[nc]) <= TIE_REL * w0:
            nc -= 1
        n = nc if nc > 0 else cap
    return max(n, min(min_keep, n_all, max(cap, 0)))


def split_left(C, eps, chi_max):
    """C[a,s,b] -> A[a,s,k] R[k,b]: QR when eps == 0, truncated SVD otherwise."""
    ml, d, mr = C.shape
    Cm = C.reshape(ml * d, mr)
    if eps == 0.0:
        q, r = np.linalg.qr(Cm, mode="reduced")
        return q.reshape(ml, d, q.shape[1]), r, 0.0
    U, S, Vh = np.linalg.svd(Cm, full_matrices=False)
    w = S ** 2
    n = keep_count(w, eps, w.sum(), chi_max)
    disc = float(w[n:].sum())
    return U[:, :n].reshape(ml, d, n), S[:n, None] * Vh[:n], disc


def split_right(C, eps, chi_max):
    """C[a,s,b] -> L[a,k] B[k,s,b]: LQ when eps == 0, truncated SVD otherwise."""
    ml, d, mr = C.shape
    Cm = C.reshape(ml, d * mr)
    if eps == 0.0:
        q, r = np.linalg.qr(Cm.T, mode="reduced")
        return r.T, q.T.reshape(q.shape[1], d, mr), 0.0
    U, S, Vh = np.linalg.svd(Cm, full_matrices=False)
    w = S ** 2
    n = keep_count(w, eps, w.sum(), chi_max)
    disc = float(w[n:].sum())
    return U[:, :n] * S[None, :n], Vh[:n].reshape(n, d, mr), disc


# --------------------------------------------------------------------------
# One-site TDVP sweep
# --------------------------------------------------------------------------

def tdvp1_sweep(mps, Ws, dt, eps=0.0, chi_max=10 ** 9, tol=1e-12, maxiter=30, normalize=False):
    """One symmetric one-site TDVP sweep (left->right then right->left).

    Precondition: center at site 0, sites 1..N-1 right-canonical.
    Postcondition: center at site 0, sites 1..N-1 right-canonical.
    Returns (mps, stats).
    """
    psi = M.copy(mps)
    N = len(psi)
    half = dt / 2.0
    R = right_envs(psi, Ws)
    L = [None] * (N + 1)
    L[0] = boundary_env()
    stats = {"n_matvec": 0, "n_keff": 0, "discarded": 0.0}

    def evolve_site(i, C, step):
        f = lambda x: heff_apply(L[i], Ws[i], R[i + 1], x.reshape(C.shape)).ravel()
        y, n = expm_krylov(f, C.ravel(), step, tol, maxiter)
        stats["n_matvec"] += n
        y = y.reshape(C.shape)
        if normalize:
            y = y / np.linalg.norm(y)
        return y

    def evolve_bond(Lenv, Renv, X, step):
        f = lambda x: keff_apply(Lenv, Renv, x.reshape(X.shape)).ravel()
        y, n = expm_krylov(f, X.ravel(), step, tol, maxiter)
        stats["n_keff"] += n
        y = y.reshape(X.shape)
        if normalize:
            y = y / np.linalg.norm(y)
        return y

    # left -> right
    for i in range(N - 1):
        psi[i] = evolve_site(i, psi[i], half)
        A, Rm, disc = split_left(psi[i], eps, chi_max)
        stats["discarded"] += disc
        psi[i] = A
        L[i + 1] = left_env_update(L[i], A, Ws[i])
        Rm = evolve_bond(L[i + 1], R[i + 1], Rm, -half)
        psi[i + 1] = np.tensordot(Rm, psi[i + 1], axes=(1, 0))
    # last site: both half steps merged
    psi[N - 1] = evolve_site(N - 1, psi[N - 1], dt)
    # right -> left
    for i in range(N - 1, 0, -1):
        if i < N - 1:
            psi[i] = evolve_site(i, psi[i], half)
        Lm, B, disc = split_right(psi[i], eps, chi_max)
        stats["discarded"] += disc
        psi[i] = B
        R[i] = right_env_update(R[i + 1], B, Ws[i])
        Lm = evolve_bond(L[i], R[i], Lm, -half)
        psi[i - 1] = np.tensordot(psi[i - 1], Lm, axes=(2, 0))
    if N > 1:
        psi[0] = evolve_site(0, psi[0], half)
    return psi, stats


def center_energy(mps, Ws):
    """<C|H_eff C>/<C|C> at site 0 for an MPS with center 0 (right-canonical rest)."""
    R = right_envs(mps, Ws)
    C = mps[0]
    y = heff_apply(boundary_env(), Ws[0], R[1], C)
    return float(np.vdot(C, y).real / np.vdot(C, C).real)
