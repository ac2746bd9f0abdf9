"""Variational (fitting) MPO application (oracle; test infrastructure only).

Section I.C names two ways to apply the MPO of 1 - i tau H to an MPS: the
density-matrix approach (exact for a small MPO bond dimension, in
``krylov.py``) and the variational approach of Paeckel et al. (2019), whose
cost per Krylov vector is O(m^3 w d) instead of O(m^3 w^2 d).  This module
writes out the variational one in its two-site form:

* the target is |t> = O|psi>; the approximation |phi> starts from a guess
  (|psi> itself unless given) brought to right-canonical form (odd pass
  counts) or left-canonical form (even counts);
* mixed environments L_i = <phi|O|psi> over sites < i and R_i over sites
  >= i (bra index first, as in ``tdvp.py``);
* a pass from left to right visits the pairs (i, i+1), i = 0..N-2: the
  two-site tensor that maximises the overlap with |t> in the current bases
  of the other sites is the exact local projection
  Phi[a',t,u,b'] = sum L_i[a',al,a] W_i[al,be,t,s] W_{i+1}[be,ga,u,v]
                   Psi[a,s,v,b] R_{i+2}[b',ga,b],
  Psi = psi_i psi_{i+1}; a truncated SVD (the relative eps / chi_max cut
  of ``tdvp.keep_count``, numerical zeros dropped) splits it into a left-canonical phi_i and the centre
  phi_{i+1}, and L_{i+1} is updated with the new phi_i;
* a pass from right to left does the mirror image, leaving phi_{i+1}
  right-canonical;
* passes alternate and the last one runs from left to right, so the result
  is left-canonical with its centre on the last site (the gauge of the
  density-matrix route): an odd count starts from the left, an even count
  from the right; the result is normalised.

Readings (the paper cites the method without details): the number of passes
is a parameter (the paper fixes none); the direction of the first pass is
chosen so that the last pass ends in the left-canonical gauge (no gauge
sweep after the fit; a left-canonical input then needs none before it
either); the cut is the same relative discarded-weight rule as eps_K; the
discarded weight reported is that of the last pass.
"""
from __future__ import annotations

import numpy as np

from . import mps as M
from .tdvp2 import heff2_apply, split2_left, split2_right


def left_env_mixed(L, bra, W, ket):
    """L_new[b',be,b] = sum conj(bra[a',s',b']) L[a',al,a] W[al,be,s',s] ket[a,s,b]."""
    T1 = np.tensordot(L, ket, axes=([2], [0]))            # [a',al,s,b]
    T2 = np.tensordot(T1, W, axes=([1, 2], [0, 3]))       # [a',b,be,s']
    out = np.tensordot(np.conj(bra), T2, axes=([0, 1], [0, 3]))  # [b',b,be]
    return np.ascontiguousarray(out.transpose(0, 2, 1))


def right_env_mixed(R, bra, W, ket):
    """R_new[a',al,a] = sum conj(bra[a',s',b']) W[al,be,s',s] R[b',be,b] ket[a,s,b]."""
    T1 = np.tensordot(ket, R, axes=([2], [2]))            # [a,s,b',be]
    T2 = np.tensordot(T1, W, axes=([1, 3], [3, 1]))       # [a,b',al,s']
    out = np.tensordot(np.conj(bra), T2, axes=([1, 2], [3, 1]))  # [a',a,al]
    return np.ascontiguousarray(out.transpose(0, 2, 1))


def _pair(a, b):
    """Psi[a,s,v,b] = sum_c a[a,s,c] b[c,v,b]."""
    return np.tensordot(a, b, axes=([2], [0]))


def apply_mpo_variational(mps, Ws, eps, chi_max, passes=1, guess=None):
    """O|psi> by two-site variational fitting; returns (mps, discarded).

    ``passes`` >= 1 alternating passes, the last from left to right (odd
    counts start from the left, even counts from the right); ``guess``
    replaces |psi> as the starting approximation.
    """
    if passes < 1:
        raise ValueError("passes must be >= 1")
    N = len(mps)
    from_right = passes % 2 == 0
    start = M.copy(guess if guess is not None else mps)
    phi = M.left_canonicalize(start) if from_right else M.right_canonicalize(start)
    one = np.ones((1, 1, 1), dtype=np.complex128)
    Ls = [None] * (N + 1)
    Rs = [None] * (N + 1)
    Ls[0] = one
    Rs[N] = one
    if from_right:
        for i in range(N - 2):
            Ls[i + 1] = left_env_mixed(Ls[i], phi[i], Ws[i], mps[i])
    else:
        for i in range(N - 1, 1, -1):
            Rs[i] = right_env_mixed(Rs[i + 1], phi[i], Ws[i], mps[i])
    disc = 0.0
    for p in range(passes):
        disc = 0.0
        if N == 1:                                           # phi[a,t,b] = sum W[0,0,t,s] psi[a,s,b]
            phi[0] = np.tensordot(Ws[0][0, 0], mps[0], axes=([1], [1])).transpose(1, 0, 2)
            break
        if (p % 2 == 0) != from_right:                       # left to right
            for i in range(N - 1):
                Th = heff2_apply(Ls[i], Ws[i], Ws[i + 1], Rs[i + 2], _pair(mps[i], mps[i + 1]))
                phi[i], phi[i + 1], dd = split2_left(Th, eps, chi_max)
                disc += dd
                Ls[i + 1] = left_env_mixed(Ls[i], phi[i], Ws[i], mps[i])
        else:                                                # right to left
            for i in range(N - 2, -1, -1):
                Th = heff2_apply(Ls[i], Ws[i], Ws[i + 1], Rs[i + 2], _pair(mps[i], mps[i + 1]))
                phi[i], phi[i + 1], dd = split2_right(Th, eps, chi_max)
                disc += dd
                Rs[i + 1] = right_env_mixed(Rs[i + 2], phi[i + 1], Ws[i + 1], mps[i + 1])
    nrm = np.linalg.norm(phi[N - 1])
    phi[N - 1] = phi[N - 1] / nrm
    return phi, disc
