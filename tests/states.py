"""Test inputs with a prescribed Schmidt spectrum (used by CPU and GPU tests
alike; seeded NumPy construction, none of the method's steps)."""
import numpy as np


def mps_with_schmidt(N, b, s, seed):
    """Random MPS on N sites whose Schmidt values across bond b (between
    sites b-1 and b) are s / |s|: a left-orthonormal part A_0..A_{b-1} and a
    right-orthonormal part B_b..B_{N-1} of seeded random isometries, joined
    by diag(s) at bond b.  Bond dims grow as min(2^i, 2^(N-i), len(s)) and
    must allow the isometries (each left and right dim at most doubles)."""
    rng = np.random.default_rng(seed)
    s = np.asarray(s, dtype=np.float64)
    m = len(s)
    dims = [1] + [min(2 ** i, 2 ** (N - i), m) for i in range(1, N)] + [1]
    dims[b] = m
    tens = []
    for i in range(N):
        ml, mr = dims[i], dims[i + 1]
        n = 2 * max(ml, mr)
        X = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        if i < b:   # left-orthonormal: (ml*2) x mr isometry
            assert 2 * ml >= mr
            tens.append(np.linalg.qr(X[:2 * ml, :mr])[0].reshape(ml, 2, mr))
        else:       # right-orthonormal: ml x (2*mr) with orthonormal rows
            assert 2 * mr >= ml
            Bq = np.linalg.qr(X[:2 * mr, :ml])[0]
            tens.append(Bq.conj().T.reshape(ml, 2, mr))
    tens[b] = np.tensordot(np.diag(s / np.linalg.norm(s)).astype(np.complex128), tens[b], axes=(1, 0))
    return tens
