"""Pins for the oracle's variational (fitting) MPO application (CPU only).

Each check is fixed by something other than the oracle itself: exact
diagonalisation of the same operator, the fixed-point property of the local
projections, the identity operator, the optimality of fitting against a
sequential SVD truncation of the exact product, and dense overlaps for the
mixed environments."""
import numpy as np
import pytest

from paper_2005_06104_amd import inputs as I
from oracle import ed, fit as F, krylov as K, mpo, mps as M


def _sys(L=4, path="snake"):
    lat = I.ladder(L, 1.0, 1.0, path)
    return lat.n_sites, I.heisenberg_terms(lat.couplings)


def _dense_target(N, terms, tau, psi):
    v = ed.hamiltonian(N, terms, 1.0, -1j * tau) @ M.to_dense(psi)
    return v / np.linalg.norm(v)


def _infid(ref, mps):
    v = M.to_dense(mps)
    return 1.0 - abs(np.vdot(ref, v)) ** 2 / np.vdot(v, v).real


@pytest.mark.parametrize("tau", [0.1, -0.25j])
def test_mixed_environments_give_the_dense_overlap(tau):
    """Contracting the whole chain from either side is <phi|O|psi>."""
    N, terms = _sys()
    Wop = mpo.build_mpo(N, terms, 1.0, -1j * tau)
    psi, phi = I.random_mps(N, 4, 31), I.random_mps(N, 3, 32)
    dense = np.vdot(M.to_dense(phi), ed.hamiltonian(N, terms, 1.0, -1j * tau) @ M.to_dense(psi))
    L = np.ones((1, 1, 1), dtype=np.complex128)
    R = np.ones((1, 1, 1), dtype=np.complex128)
    for i in range(N):
        L = F.left_env_mixed(L, phi[i], Wop[i], psi[i])
    for i in range(N - 1, -1, -1):
        R = F.right_env_mixed(R, phi[i], Wop[i], psi[i])
    assert abs(L.ravel()[0] - dense) <= 1e-12 * abs(dense)
    assert abs(R.ravel()[0] - dense) <= 1e-12 * abs(dense)


@pytest.mark.parametrize("tau", [0.1, -0.25j])
@pytest.mark.parametrize("passes", [2, 3])
def test_fit_exact_without_truncation(tau, passes):
    """With no cut the bases reach the exact product after two passes."""
    N, terms = _sys()
    Wop = mpo.build_mpo(N, terms, 1.0, -1j * tau)
    psi = I.random_mps(N, 4, 21)
    out, _ = F.apply_mpo_variational(psi, Wop, 0.0, 10 ** 6, passes)
    assert _infid(_dense_target(N, terms, tau, psi), out) < 1e-12
    assert abs(M.norm(out) - 1.0) < 1e-12
    assert M.is_left_canonical(out, 1e-12)


def test_fit_fixed_point_at_the_exact_guess():
    """Started from the exact product, one pass returns it unchanged."""
    N, terms = _sys()
    Wop = mpo.build_mpo(N, terms, 1.0, -0.1j)
    psi = I.random_mps(N, 3, 23)
    out, disc = F.apply_mpo_variational(psi, Wop, 0.0, 10 ** 6, 1, guess=K.apply_mpo_exact(psi, Wop))
    assert _infid(_dense_target(N, terms, 0.1, psi), out) < 1e-13
    assert disc < 1e-20


def test_fit_identity_returns_the_state():
    N, terms = _sys()
    Wid = mpo.build_mpo(N, terms, 1.0, 0.0)
    psi = I.random_mps(N, 4, 24)
    out, _ = F.apply_mpo_variational(psi, Wid, 1e-14, 10 ** 6, 1)
    assert M.fidelity(out, psi) > 1 - 1e-13


@pytest.mark.parametrize("cap", [4, 8])
def test_fit_under_a_cap_improves_with_passes_and_beats_svd_truncation(cap):
    """Each pass maximises the overlap in the current bases, so the error
    does not grow with passes, and the converged fit is at least as close to
    the exact product as the sequential SVD truncation at the same cap."""
    N, terms = _sys(5)
    Wop = mpo.build_mpo(N, terms, 1.0, -0.1j)
    psi = I.random_mps(N, 6, 22)
    ref = _dense_target(N, terms, 0.1, psi)
    errs = []
    for passes in (1, 3, 5):
        out, _ = F.apply_mpo_variational(psi, Wop, 1e-14, cap, passes)
        assert max(M.bond_dims(out)) <= cap
        errs.append(_infid(ref, out))
    assert errs[1] <= errs[0] + 1e-13 and errs[2] <= errs[1] + 1e-13
    svd, _ = K.svd_compress(K.apply_mpo_exact(psi, Wop), 1e-14, cap)
    assert errs[2] <= _infid(ref, svd) + 1e-13


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_fit_with_relative_cut_matches_the_density_matrix_route(eps):
    """Same relative cut: after three passes the same bond dimensions as the
    density-matrix route (itself pinned to the SVD of the exact product) and
    the same state to within the discarded weight."""
    N, terms = _sys(5)
    Wop = mpo.build_mpo(N, terms, 1.0, -0.1j)
    psi = M.left_canonicalize(I.random_mps(N, 6, 22))
    a, _ = F.apply_mpo_variational(psi, Wop, eps, 10 ** 6, 3)
    b, _ = K.apply_mpo_denmat(psi, Wop, eps, 10 ** 6)
    assert M.bond_dims(a) == M.bond_dims(b)
    assert 1 - M.fidelity(a, b) <= 10 * eps


def test_krylov_vectors_by_fitting_span_the_same_states():
    N, terms = _sys()
    Wop = mpo.build_mpo(N, terms, 1.0, -0.1j)
    psi = M.left_canonicalize(I.random_mps(N, 4, 25))
    kd = K.krylov_vectors(psi, Wop, 3, 1e-12, 10 ** 6)
    kf = K.krylov_vectors(psi, Wop, 3, 1e-12, 10 ** 6, apply="fit", fit_passes=3)
    for a, b in zip(kd, kf):
        assert 1 - M.fidelity(a, b) < 1e-10
