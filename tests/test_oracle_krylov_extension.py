"""Pins for the oracle's global Krylov vectors (density-matrix MPO
application) and the state-averaged basis extension (CPU only)."""
import numpy as np
import pytest

from paper_2005_06104_amd import inputs as I
from oracle import ed, extension as X, krylov as K, mpo, mps as M


def _sys(L=4, path="snake", Jr=1.0):
    lat = I.ladder(L, 1.0, Jr, path)
    N = lat.n_sites
    terms = I.heisenberg_terms(lat.couplings)
    return lat, N, terms


@pytest.mark.parametrize("tau", [0.1, -1j / 4.0])
def test_denmat_apply_exact_without_truncation(tau):
    lat, N, terms = _sys()
    Wop = mpo.build_mpo(N, terms, 1.0, -1j * tau)
    psi = I.random_mps(N, 4, 21)
    out, disc = K.apply_mpo_denmat(psi, Wop, 0.0, 10 ** 6)
    ref = ed.hamiltonian(N, terms, 1.0, -1j * tau) @ M.to_dense(psi)
    ref = ref / np.linalg.norm(ref)
    v = M.to_dense(out)
    assert abs(np.linalg.norm(v) - 1.0) < 1e-12
    assert 1 - abs(np.vdot(ref, v)) ** 2 < 1e-12
    assert M.is_left_canonical(out, 1e-12)


def test_denmat_apply_matches_svd_compression():
    lat, N, terms = _sys(5)
    Wop = mpo.build_mpo(N, terms, 1.0, -0.1j)
    psi = I.random_mps(N, 6, 22)
    for eps in (1e-3, 1e-6):
        a, da = K.apply_mpo_denmat(psi, Wop, eps, 10 ** 6)
        b, db = K.svd_compress(K.apply_mpo_exact(psi, Wop), eps, 10 ** 6)
        assert M.bond_dims(a) == M.bond_dims(b)
        assert M.fidelity(a, b) > 1 - 1e-12
        assert M.bond_dims(a) != M.bond_dims(K.apply_mpo_denmat(psi, Wop, 0.0, 10 ** 6)[0])
    # a cap binds the same way on both routes
    a, _ = K.apply_mpo_denmat(psi, Wop, 0.0, 5)
    b, _ = K.svd_compress(K.apply_mpo_exact(psi, Wop), 0.0, 5)
    assert max(M.bond_dims(a)) <= 5 and M.fidelity(a, b) > 1 - 1e-10


def test_denmat_apply_identity_returns_state():
    lat, N, terms = _sys()
    Wid = mpo.build_mpo(N, terms, 1.0, 0.0)
    psi = I.random_mps(N, 4, 23)
    out, _ = K.apply_mpo_denmat(psi, Wid, 1e-14, 10 ** 6)
    assert M.fidelity(out, psi) > 1 - 1e-13
    assert M.bond_dims(out) == M.bond_dims(M.left_canonicalize(psi))


def _right_basis(Bs, i, N):
    """Dense vectors of the right block basis at the bond left of site i."""
    T = Bs[N - 1][:, :, 0]
    for j in range(N - 2, i - 1, -1):
        T = np.tensordot(Bs[j], T, axes=(2, 0)).reshape(Bs[j].shape[0], -1)
    return T


def _projector_rows(B):
    q, _ = np.linalg.qr(B.conj().T)
    return q @ q.conj().T


def _setup_extension(N_leg=4, chi=3, seed=30, k=3):
    lat, N, terms = _sys(N_leg)
    Wop = mpo.build_mpo(N, terms, 1.0, -1j * 0.1)
    psi = M.left_canonicalize(I.random_mps(N, chi, seed))
    psi[-1] = psi[-1] / np.linalg.norm(psi[-1])
    kv = K.krylov_vectors(psi, Wop, k, 1e-12, 10 ** 6)
    return N, psi, kv


def test_extension_keeps_state_and_orthonormality():
    N, psi, kv = _setup_extension()
    out, st = X.basis_extension(psi, kv, 1e-8, 10 ** 6)
    v0, v1 = M.to_dense(psi), M.to_dense(out)
    assert np.abs(v0 - v1).max() < 1e-13          # psi is kept exactly
    assert M.is_right_canonical(out, 1e-12)        # B' B'^dagger = 1
    assert sum(st["added"]) > 0
    assert all(b1 >= b0 for b1, b0 in zip(M.bond_dims(out), M.bond_dims(psi)))


def test_extension_new_rows_orthogonal_to_old():
    # B_bar B^dagger = 0 (eq. (6) remark); a product state leaves room at the last site
    N, psi, kv = _setup_extension(chi=1)
    C = psi[-1].reshape(psi[-1].shape[0], -1)
    Cts = [k[-1].reshape(k[-1].shape[0], -1) for k in kv]
    Bp, r, n = X.extension_step(C, Cts, 0.0, 10 ** 6)
    assert n > 0
    assert np.abs(Bp[r:] @ Bp[:r].conj().T).max() < 1e-13
    assert np.abs(Bp @ Bp.conj().T - np.eye(r + n)).max() < 1e-13
    # the old rows are the row space of the center
    assert np.abs(C - (C @ Bp[:r].conj().T) @ Bp[:r]).max() < 1e-13


def test_extension_without_cut_holds_krylov_vectors():
    # eps_M = 0 and no cap: every Krylov vector lies in the extended right bases
    N, psi, kv = _setup_extension()
    out, _ = X.basis_extension(psi, kv, 0.0, 10 ** 6)
    Rb = _right_basis(out, 1, N)           # basis states of sites 1..N-1
    for k in kv:
        v = M.to_dense(k).reshape(2, -1)   # (s0, rest)
        proj = (v @ Rb.conj().T) @ Rb
        assert np.abs(proj - v).max() < 1e-12


def test_extension_eigh_route_equals_stacked_svd_route():
    N, psi, kv = _setup_extension()
    a, _ = X.basis_extension(psi, kv, 1e-6, 10 ** 6, use_gram_of_stack=False)
    b, _ = X.basis_extension(psi, kv, 1e-6, 10 ** 6, use_gram_of_stack=True)
    assert M.bond_dims(a) == M.bond_dims(b)
    for i in range(1, N):
        Pa = _projector_rows(_right_basis(a, i, N))
        Pb = _projector_rows(_right_basis(b, i, N))
        assert np.abs(Pa - Pb).max() < 1e-10


def test_extension_matches_direct_sum_route():
    # at zero cutoffs the reformed algorithm spans the same bond spaces as the
    # direct-sum formulation of eqs. (2)-(4)
    N, psi, kv = _setup_extension(k=2)
    a, _ = X.basis_extension(psi, kv, 0.0, 10 ** 6)
    b = X.direct_sum_extension(psi, kv)
    assert M.bond_dims(a) == M.bond_dims(b)
    for i in range(1, N):
        Pa = _projector_rows(_right_basis(a, i, N))
        Pb = _projector_rows(_right_basis(b, i, N))
        assert np.abs(Pa - Pb).max() < 1e-10
    assert np.abs(M.to_dense(a) - M.to_dense(b)).max() < 1e-12


def test_extension_full_bond_adds_nothing():
    # when B already spans the whole row space (P = 0) no state can be added
    C = np.linalg.qr(np.random.default_rng(0).standard_normal((4, 4)) + 0j)[0]
    Ct = np.random.default_rng(1).standard_normal((3, 4)) + 0j
    Bp, r, n = X.extension_step(C, [Ct], 0.0, 100)
    assert r == 4 and n == 0


def test_extension_respects_cap():
    N, psi, kv = _setup_extension()
    out, _ = X.basis_extension(psi, kv, 0.0, 5)
    assert max(M.bond_dims(out)) <= 5
    assert np.abs(M.to_dense(out) - M.to_dense(psi)).max() < 1e-13


# The reading of "SVD without truncation" (section I.A): directions of the
# centre whose weight s^2 is at most 1e-14 s_1^2 are not part of B.  Pinned
# here on a state with prescribed Schmidt values across one bond, two of them
# inside (1e-13, 1e-7) s_1 (weights 4e-16 and 2.5e-17 of s_1^2) and one just
# above the floor (weight 4e-14): (a) when no Krylov vector carries the two
# directions, the extension changes psi by exactly their weight (the bound
# of the reading is attained, and nothing else moves); (b) when a Krylov
# vector carries them, they return through rho_bar and psi is kept exactly.
SCHMIDT = [1.0, 0.6, 0.3, 2e-7, 2e-8, 5e-9]


def _schmidt_state(seed=3):
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from states import mps_with_schmidt
    return M.left_canonicalize(mps_with_schmidt(7, 3, SCHMIDT, seed))


def test_extension_floor_drops_exactly_the_subfloor_weight():
    pl = _schmidt_state()
    s = np.array(SCHMIDT) / np.linalg.norm(SCHMIDT)
    dropped = float(np.sum(s[s ** 2 <= 1e-14 * s[0] ** 2] ** 2))
    assert 1e-16 < dropped < 1e-15
    out, _ = X.basis_extension(pl, [pl], 1e-8, 10 ** 6)
    d = np.linalg.norm(M.to_dense(out) - M.to_dense(pl)) ** 2
    assert abs(d - dropped) < 1e-3 * dropped, (d, dropped)
    assert M.bond_dims(out)[2] == 4          # bond 3 keeps 4 of 6 directions (1e-7 s_1 is kept)
    assert M.is_right_canonical(out, 1e-12)


def test_extension_floor_directions_return_through_krylov_vectors():
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from states import mps_with_schmidt
    pl = _schmidt_state()
    # same isometries, flat Schmidt values: this Krylov vector carries the
    # sub-floor directions with weight 1/3 of its norm
    phi = M.left_canonicalize(mps_with_schmidt(7, 3, [1.0] * 6, 3))
    out, st = X.basis_extension(pl, [phi], 1e-8, 10 ** 6)
    d = np.linalg.norm(M.to_dense(out) - M.to_dense(pl)) ** 2
    assert d < 1e-26, d
    assert M.bond_dims(out)[2] == 6
    # and the Krylov vector itself now lies in the extended bases
    v = M.to_dense(phi)
    T = out[6][:, :, 0]
    for j in range(5, 2, -1):
        T = np.tensordot(out[j], T, axes=(2, 0)).reshape(out[j].shape[0], -1)
    q, _ = np.linalg.qr(T.conj().T)
    V = v.reshape(-1, q.shape[0])
    assert np.linalg.norm(V - (V @ q) @ q.conj().T) < 1e-12
