"""Finite MPS utilities (oracle; test infrastructure only).

An MPS is a Python list of complex128 arrays M_i[a, s, b] (eq. (1)): a is the
left bond (size m_{i-1}), s the physical index (d = 2), b the right bond
(size m_i); m_{-1} = m_{N-1} = 1.  Left-canonical tensors A satisfy
sum_{a,s} conj(A[a,s,b']) A[a,s,b] = delta_{b'b}; right-canonical tensors B
satisfy sum_{s,b} B[a,s,b] conj(B[a',s,b]) = delta_{aa'}.
"""
from __future__ import annotations

from typing import List

import numpy as np


def copy(mps) -> List[np.ndarray]:
    return [np.array(t, dtype=np.complex128, copy=True) for t in mps]


def bond_dims(mps) -> List[int]:
    return [t.shape[2] for t in mps[:-1]]


def to_dense(mps) -> np.ndarray:
    """Contract into the 2^N amplitude vector; site 0 is most significant."""
    v = mps[0].reshape(-1, mps[0].shape[2])           # (s0, b)
    for t in mps[1:]:
        v = np.tensordot(v, t, axes=(1, 0))            # (S, s, b)
        v = v.reshape(-1, t.shape[2])
    return v[:, 0]


def left_canonicalize(mps) -> List[np.ndarray]:
    """QR sweep left to right; sites 0..N-2 become A, the last site holds C."""
    out = copy(mps)
    N = len(out)
    for i in range(N - 1):
        ml, d, mr = out[i].shape
        q, r = np.linalg.qr(out[i].reshape(ml * d, mr), mode="reduced")
        out[i] = q.reshape(ml, d, q.shape[1])
        out[i + 1] = np.tensordot(r, out[i + 1], axes=(1, 0))
    return out


def right_canonicalize(mps) -> List[np.ndarray]:
    """LQ sweep right to left; sites 1..N-1 become B, site 0 holds C."""
    out = copy(mps)
    N = len(out)
    for i in range(N - 1, 0, -1):
        ml, d, mr = out[i].shape
        # LQ of M = (ml, d*mr) from QR of M^T
        q, r = np.linalg.qr(out[i].reshape(ml, d * mr).T, mode="reduced")
        out[i] = q.T.reshape(q.shape[1], d, mr)
        out[i - 1] = np.tensordot(out[i - 1], r.T, axes=(2, 0))
    return out


def inner(a, b) -> complex:
    """<a|b> by a left-to-right transfer contraction."""
    T = np.ones((1, 1), dtype=np.complex128)           # [a', a]
    for ta, tb in zip(a, b):
        T = np.tensordot(T, np.conj(ta), axes=([0], [0]))   # [a, s, p]
        T = np.tensordot(T, tb, axes=([0, 1], [0, 1]))      # [p, q]
    return complex(T[0, 0])


def norm(mps) -> float:
    return float(np.sqrt(abs(inner(mps, mps))))


def fidelity(a, b) -> float:
    """|<a|b>|^2 / (<a|a><b|b>)."""
    return float(abs(inner(a, b)) ** 2 / (inner(a, a).real * inner(b, b).real))


def local_expectations(mps, op: np.ndarray) -> np.ndarray:
    """<psi|op_i|psi>/<psi|psi> for every site i (any gauge)."""
    N = len(mps)
    left = [np.ones((1, 1), dtype=np.complex128)]
    for t in mps:
        T = np.tensordot(left[-1], np.conj(t), axes=([0], [0]))     # [y,s,p]
        left.append(np.tensordot(T, t, axes=([0, 1], [0, 1])))       # [p,q]
    right = [None] * (N + 1)
    right[N] = np.ones((1, 1), dtype=np.complex128)
    for i in range(N - 1, -1, -1):
        T = np.tensordot(np.conj(mps[i]), right[i + 1], axes=([2], [0]))  # [x,s,q]
        right[i] = np.tensordot(T, mps[i], axes=([1, 2], [1, 2]))         # [x,y]
    nrm = left[N][0, 0].real
    out = np.empty(N, dtype=np.complex128)
    for i in range(N):
        # sum left[x,y] conj(M[x,t,p]) op[t,s] M[y,s,q] right[p,q]
        T1 = np.tensordot(left[i], np.conj(mps[i]), axes=([0], [0]))   # [y,t,p]
        T2 = np.tensordot(mps[i], right[i + 1], axes=([2], [1]))       # [y,s,p]
        T3 = np.tensordot(op, T2, axes=([1], [1]))                      # [t,y,p]
        out[i] = np.tensordot(T1, T3, axes=([0, 1, 2], [1, 0, 2]))
    return out / nrm


def is_left_canonical(mps, tol=1e-12) -> bool:
    for t in mps[:-1]:
        ml, d, mr = t.shape
        a = t.reshape(ml * d, mr)
        if np.abs(a.conj().T @ a - np.eye(mr)).max() > tol:
            return False
    return True


def is_right_canonical(mps, tol=1e-12) -> bool:
    for t in mps[1:]:
        ml, d, mr = t.shape
        b = t.reshape(ml, d * mr)
        if np.abs(b @ b.conj().T - np.eye(ml)).max() > tol:
            return False
    return True


def max_bond_dims(N: int, chi_max: int) -> List[int]:
    """Largest meaningful bond dims min(chi_max, 2^(i+1), 2^(N-i-1))."""
    return [int(min(chi_max, 2 ** min(i + 1, 60), 2 ** min(N - i - 1, 60))) for i in range(N - 1)]
