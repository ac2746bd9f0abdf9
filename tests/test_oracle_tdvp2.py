"""Two-site TDVP oracle (the comparison method of sections I.C and II):
pinned against exact diagonalisation and against the projected Hamiltonian
built from explicit isometries."""
import numpy as np
import pytest

from oracle import ed, mps as M, tdvp as T, tdvp2 as T2
from paper_2005_06104_amd import inputs as I

from test_oracle_tdvp import _normalised_right_canonical, _system, _system_terms, complex_hermitian_terms


@pytest.mark.parametrize("site", [0, 2, 4])
@pytest.mark.parametrize("ham", ["ladder", "complex"])
def test_heff2_is_projected_hamiltonian(site, ham):
    if ham == "ladder":
        N, terms, Ws, H = _system(I.ladder(3, 1.0, 1.0, "snake"))
    else:
        N, terms, Ws, H = _system_terms(6, complex_hermitian_terms(6, 4))
    psi = I.random_mps(N, 4, 7)
    left = M.left_canonicalize(psi)
    right = M.right_canonicalize(psi)
    Lenv = T.boundary_env()
    for i in range(site):
        Lenv = T.left_env_update(Lenv, left[i], Ws[i])
    Renv = T.boundary_env()
    for i in range(N - 1, site + 1, -1):
        Renv = T.right_env_update(Renv, right[i], Ws[i])
    ml = left[site - 1].shape[2] if site > 0 else 1
    mr = right[site + 2].shape[0] if site + 2 < N else 1
    shape = (ml, 2, 2, mr)
    dim = int(np.prod(shape))
    P = np.zeros((2 ** N, dim), dtype=complex)
    Heff = np.zeros((dim, dim), dtype=complex)
    for k in range(dim):
        e = np.zeros(dim, dtype=complex)
        e[k] = 1.0
        th = e.reshape(shape)
        # the two-site center as two tensors (identity split on the pair bond)
        a = th.reshape(ml, 2, 2 * mr)
        b = np.eye(2 * mr, dtype=complex).reshape(2 * mr, 2, mr)
        t = left[:site] + [a, b] + right[site + 2:]
        P[:, k] = M.to_dense(t)
        Heff[:, k] = T2.heff2_apply(Lenv, Ws[site], Ws[site + 1], Renv, th).ravel()
    assert np.abs(P.conj().T @ P - np.eye(dim)).max() < 1e-12
    assert np.abs(Heff - P.conj().T @ (H @ P)).max() < 1e-12
    assert np.abs(Heff - Heff.conj().T).max() < 1e-12


@pytest.mark.parametrize("dt,normalize", [(0.1, False), (0.3 + 0.0j, False), (-0.2j, True)])
def test_tdvp2_exact_at_full_bond_dimension(dt, normalize):
    # with complete bond spaces every local step is the exact evolution in a
    # rotated basis, so one sweep equals exp(-i H dt) (imaginary: normalised)
    N, terms, Ws, H = _system(I.ladder(3, 1.0, 0.7, "zigzag"))
    psi = _normalised_right_canonical(N, 64, 3)
    assert M.bond_dims(psi) == M.max_bond_dims(N, 64)
    out, st = T2.tdvp2_sweep(psi, Ws, dt, eps=0.0, normalize=normalize)
    ref = ed.evolve(H, M.to_dense(psi), dt)
    ref = ref / np.linalg.norm(ref)
    v = M.to_dense(out)
    fid = abs(np.vdot(ref, v)) ** 2 / np.vdot(v, v).real
    assert 1 - fid < 1e-12
    assert st["discarded"] < 1e-20


def test_tdvp2_grows_a_product_state():
    # the two-site update enlarges the bonds (one-site TDVP keeps a product
    # state); with eps = 0 nothing is truncated and the norm is conserved
    N, terms, Ws, H = _system(I.ladder(4, 1.0, 1.0, "snake"))
    lat = I.ladder(4, 1.0, 1.0, "snake")
    psi = I.product_mps(lat.neel())
    out, st = T2.tdvp2_sweep(psi, Ws, 0.1, eps=0.0)
    assert max(M.bond_dims(out)) > 1
    assert abs(M.norm(out) - 1.0) < 1e-12
    one, _ = T.tdvp1_sweep(psi, Ws, 0.1)
    assert max(M.bond_dims(one)) == 1


def test_tdvp2_truncation_caps_and_conserves_more_with_smaller_eps():
    N, terms, Ws, H = _system(I.ladder(4, 1.0, 1.0, "snake"))
    lat = I.ladder(4, 1.0, 1.0, "snake")
    psi = I.product_mps(lat.neel())
    v0 = M.to_dense(psi)
    errs = []
    for chi in (2, 4, 16):
        p = psi
        for _ in range(4):
            p, _ = T2.tdvp2_sweep(p, Ws, 0.05, eps=0.0, chi_max=chi)
        assert max(M.bond_dims(p)) <= chi
        ref = ed.evolve(H, v0, 0.2)
        v = M.to_dense(p)
        errs.append(1 - abs(np.vdot(ref, v)) ** 2 / np.vdot(v, v).real)
    assert errs[2] < errs[1] < errs[0]
