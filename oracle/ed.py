"""Exact diagonalisation from a term list (oracle; test infrastructure only).

Builds the many-body operator directly as a sum of Kronecker products of
single-site matrices, a route that shares nothing with the MPO construction,
so it can pin the MPO and everything built on it.  Site 0 is the leftmost
(most significant) tensor factor, matching the MPS contraction order of
eq. (1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

SZ = np.array([[0.5, 0.0], [0.0, -0.5]], dtype=np.complex128)
SP = np.array([[0.0, 1.0], [0.0, 0.0]], dtype=np.complex128)   # |up><down|
SM = np.array([[0.0, 0.0], [1.0, 0.0]], dtype=np.complex128)   # |down><up|
SX = 0.5 * (SP + SM)
SY = -0.5j * (SP - SM)
ID = np.eye(2, dtype=np.complex128)
OPS = {0: ID, 1: SP, 2: SM, 3: SZ}


def site_op(op: np.ndarray, i: int, N: int) -> sp.csr_matrix:
    left = sp.identity(2 ** i, dtype=np.complex128, format="csr")
    right = sp.identity(2 ** (N - i - 1), dtype=np.complex128, format="csr")
    return sp.kron(sp.kron(left, sp.csr_matrix(op)), right, format="csr")


def hamiltonian(N: int, terms, c0: complex = 0.0, c1: complex = 1.0) -> sp.csr_matrix:
    """c0 * 1 + c1 * sum_terms coef * op_i(i) op_j(j) as a sparse 2^N x 2^N matrix."""
    H = sp.csr_matrix((2 ** N, 2 ** N), dtype=np.complex128)
    for (i, j, oi, oj, cf) in terms:
        if j < 0:
            H = H + cf * site_op(OPS[oi], i, N)
        else:
            H = H + cf * (site_op(OPS[oi], i, N) @ site_op(OPS[oj], j, N))
    H = c1 * H
    if c0 != 0.0:
        H = H + c0 * sp.identity(2 ** N, dtype=np.complex128, format="csr")
    return H.tocsr()


def product_vector(states) -> np.ndarray:
    """|s_0 s_1 ... s_{N-1}> as a dense vector."""
    v = np.ones(1, dtype=np.complex128)
    for s in states:
        e = np.zeros(2, dtype=np.complex128)
        e[s] = 1.0
        v = np.kron(v, e)
    return v


def local_vector_product(vecs) -> np.ndarray:
    v = np.ones(1, dtype=np.complex128)
    for e in vecs:
        v = np.kron(v, np.asarray(e, dtype=np.complex128))
    return v


def evolve(H: sp.csr_matrix, psi: np.ndarray, dt: complex) -> np.ndarray:
    """exp(-i H dt) psi for complex dt (imaginary time: dt = -i dtau)."""
    return spla.expm_multiply(-1j * dt * H, psi)


def ground_energy(H: sp.csr_matrix) -> float:
    n = H.shape[0]
    if n <= 4096:
        return float(np.linalg.eigvalsh(H.toarray())[0])
    vals = spla.eigsh(H, k=1, which="SA", tol=1e-13)[0]
    return float(vals[0])


def sz_sector(N: int, sz2: int) -> np.ndarray:
    """Indices of basis states with 2*S^z_tot = sz2."""
    idx = np.arange(2 ** N)
    n_down = np.zeros(2 ** N, dtype=np.int64)
    for b in range(N):
        n_down += (idx >> b) & 1
    return np.nonzero((N - 2 * n_down) == sz2)[0]


def expect(op: sp.spmatrix, psi: np.ndarray) -> complex:
    return complex(np.vdot(psi, op @ psi) / np.vdot(psi, psi))


def sz_profile(psi: np.ndarray, N: int) -> np.ndarray:
    return np.array([expect(site_op(SZ, i, N), psi).real for i in range(N)])
