"""Parity of the MPO application on the GPU (tdvp_apply_mpo, both routes of
section I.C) and of GSE-TDVP1 steps whose Krylov vectors come from the
variational route, against the CPU oracle on the same seeded inputs.  Only
gauge-invariant quantities are compared: bond dimensions, fidelity, norm,
discarded weight, energy."""
import numpy as np
import pytest

from paper_2005_06104_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    from paper_2005_06104_amd import tdvp as T
    ctx = T.Context(0)
    yield T, ctx
    ctx.close()


def _case(L=5, chi=6, seed=22):
    lat = I.ladder(L, 1.0, 1.0, "snake")
    return lat.n_sites, I.heisenberg_terms(lat.couplings), I.random_mps(lat.n_sites, chi, seed)


def _close(a, b, rel, floor=0.0):
    return abs(a - b) <= rel * max(abs(a), abs(b)) + floor


def _target_norm2(N, terms, tau, psi):
    from oracle import ed, mps as M
    return float(np.linalg.norm(ed.hamiltonian(N, terms, 1.0, -1j * tau) @ M.to_dense(psi)) ** 2)


@pytest.mark.parametrize("passes", [1, 2, 3])
@pytest.mark.parametrize("eps", [1e-3, 1e-8])
def test_fit_matches_oracle(env, eps, passes):
    T, ctx = env
    from oracle import fit as F, mpo, mps as M
    N, terms, psi = _case()
    Wop = mpo.build_mpo(N, terms, 1.0, -0.1j)
    ref, dref = F.apply_mpo_variational(psi, Wop, eps, 24, passes)
    op = T.tdvp_create_mpo(ctx, N, terms, 1.0, -0.1j)
    g = T.tdvp_mps_from_host(ctx, psi)
    h, disc = T.tdvp_apply_mpo(ctx, g, op, "fit", eps, 24, passes)
    out = T.tdvp_mps_to_host(h)
    assert M.bond_dims(out) == M.bond_dims(ref)
    assert 1 - M.fidelity(out, ref) < 1e-11
    assert abs(M.norm(out) - 1.0) < 1e-12
    assert M.is_left_canonical(out, 1e-11)
    # the GPU cut works on Gram eigenvalues, whose null directions carry
    # rounding-level weight (~1e-15 of the total) that the SVD has not
    assert _close(disc, dref, 1e-6, 1e-12 * _target_norm2(N, terms, 0.1, psi))
    # the input is left as it was
    assert all(np.array_equal(a, b) for a, b in zip(T.tdvp_mps_to_host(g), psi))


@pytest.mark.parametrize("tau", [0.1, -0.25j])
def test_fit_exact_without_truncation(env, tau):
    T, ctx = env
    from oracle import ed, mps as M
    N, terms, psi = _case(4, 4, 21)
    ref = ed.hamiltonian(N, terms, 1.0, -1j * tau) @ M.to_dense(psi)
    ref = ref / np.linalg.norm(ref)
    op = T.tdvp_create_mpo(ctx, N, terms, 1.0, -1j * tau)
    h, _ = T.tdvp_apply_mpo(ctx, T.tdvp_mps_from_host(ctx, psi), op, "fit", 0.0, 1 << 20, 2)
    v = M.to_dense(T.tdvp_mps_to_host(h))
    assert 1 - abs(np.vdot(ref, v)) ** 2 < 1e-12


@pytest.mark.parametrize("eps,cap", [(1e-3, 24), (1e-10, 24), (0.0, 7)])
def test_denmat_entry_matches_oracle(env, eps, cap):
    T, ctx = env
    from oracle import krylov as K, mpo, mps as M
    N, terms, psi = _case()
    Wop = mpo.build_mpo(N, terms, 1.0, -0.1j)
    ref, dref = K.apply_mpo_denmat(M.left_canonicalize(psi), Wop, eps, cap)
    op = T.tdvp_create_mpo(ctx, N, terms, 1.0, -0.1j)
    h, disc = T.tdvp_apply_mpo(ctx, T.tdvp_mps_from_host(ctx, psi), op, "denmat", eps, cap)
    out = T.tdvp_mps_to_host(h)
    assert M.bond_dims(out) == M.bond_dims(ref)
    assert 1 - M.fidelity(out, ref) < 1e-11
    assert M.is_left_canonical(out, 1e-11)
    assert _close(disc, dref, 1e-6, 1e-12 * _target_norm2(N, terms, 0.1, psi))


def test_both_routes_match_oracle_at_32_sites(env):
    """32 sites, bonds up to 80: each route against its oracle, and the two
    routes against each other (same cut, no binding cap)."""
    T, ctx = env
    from oracle import fit as F, krylov as K, mpo, mps as M
    lat = I.ladder(16, 1.0, 1.0, "snake")
    N, terms = lat.n_sites, I.heisenberg_terms(lat.couplings)
    Wop = mpo.build_mpo(N, terms, 1.0, -0.05j)
    psi = M.left_canonicalize(I.random_mps(N, 16, 7))
    ra, _ = K.apply_mpo_denmat(psi, Wop, 1e-10, 512)
    rb, _ = F.apply_mpo_variational(psi, Wop, 1e-10, 512, 3)
    op = T.tdvp_create_mpo(ctx, N, terms, 1.0, -0.05j)
    g = T.tdvp_mps_from_host(ctx, psi)
    a, _ = T.tdvp_apply_mpo(ctx, g, op, "denmat", 1e-10, 512)
    b, _ = T.tdvp_apply_mpo(ctx, g, op, "fit", 1e-10, 512, 3)
    A, B = T.tdvp_mps_to_host(a), T.tdvp_mps_to_host(b)
    assert M.bond_dims(A) == M.bond_dims(ra) and M.bond_dims(B) == M.bond_dims(rb)
    assert 1 - M.fidelity(A, ra) < 1e-10 and 1 - M.fidelity(B, rb) < 1e-10
    assert 1 - M.fidelity(A, B) < 1e-10


def test_apply_rejects_bad_arguments(env):
    T, ctx = env
    N, terms, psi = _case(2, 2, 3)
    op = T.tdvp_create_mpo(ctx, N, terms, 1.0, -0.1j)
    g = T.tdvp_mps_from_host(ctx, psi)
    lib = ctx.lib
    import ctypes as C
    h, d = C.c_void_p(), C.c_double()
    assert lib.tdvp_apply_mpo(ctx.h, g.h, op.h, 1, 1e-8, 8, 0, C.byref(h), C.byref(d)) == T.TDVP_ERR_ARG
    assert lib.tdvp_apply_mpo(ctx.h, g.h, op.h, 7, 1e-8, 8, 1, C.byref(h), C.byref(d)) == T.TDVP_ERR_ARG
    assert lib.tdvp_apply_mpo(ctx.h, g.h, op.h, 1, -1.0, 8, 1, C.byref(h), C.byref(d)) == T.TDVP_ERR_ARG
    assert lib.tdvp_apply_mpo(ctx.h, g.h, op.h, 1, 1e-8, 0, 1, C.byref(h), C.byref(d)) == T.TDVP_ERR_ARG
    assert lib.tdvp_apply_mpo(ctx.h, g.h, None, 1, 1e-8, 8, 1, C.byref(h), C.byref(d)) == T.TDVP_ERR_ARG
    other = T.tdvp_create_mpo(ctx, N - 1, [t for t in terms if max(t[0], t[1]) < N - 1], 1.0, -0.1j)
    assert lib.tdvp_apply_mpo(ctx.h, g.h, other.h, 1, 1e-8, 8, 1, C.byref(h), C.byref(d)) == T.TDVP_ERR_ARG


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_gse_with_fitted_krylov_vectors_matches_oracle(env, prec):
    """2x6 ladder, Neel quench, k = 3 with the Krylov vectors fitted (three
    passes) on both sides: fidelity, energy and bonds follow the oracle.  The
    mixed paths run the fit's contractions (and the sweep's) in FP32 or with
    BF16 inputs; their splits stay FP64."""
    T, ctx = env
    tol_f, tol_e, bond_frac = {"fp64": (1e-8, 1e-9, 10), "fp32": (1e-5, 1e-5, 5), "bf16x3": (2e-5, 2e-4, 5)}[prec]
    from oracle import gse, mpo, mps as M, observables as O
    w = I.workload(0)
    N = w.lattice.n_sites
    Ws = mpo.build_mpo(N, w.terms)
    Wop = mpo.build_mpo(N, w.terms, 1.0, -1j * w.tau)
    H = T.tdvp_create_mpo(ctx, N, w.terms)
    op = T.tdvp_create_mpo(ctx, N, w.terms, 1.0, -1j * w.tau)
    psi = w.initial_mps()
    g = T.tdvp_mps_from_host(ctx, psi)
    t = 0.0
    for step in range(6):
        psi, _ = gse.gse_step(psi, Ws, Wop, w.dt, 3, w.eps_K, w.eps_M, w.eps, w.chi_max, 1e-12, 30, w.normalize,
                              apply="fit", fit_passes=3)
        T.tdvp_expand_basis(ctx, [g], [op], 3, w.eps_K, w.eps_M, w.chi_max, prec, apply="fit", fit_passes=3)
        T.tdvp_sweep(ctx, [g], [H], w.dt, w.eps, w.chi_max, 1e-12, 30, prec, w.normalize)
        out = T.tdvp_mps_to_host(g)
        t += abs(w.dt)
        e_ref = O.energy(psi, Ws)
        assert 1 - M.fidelity(out, psi) < tol_f * t + 1e-12, prec
        assert abs(O.energy(out, Ws) - e_ref) < tol_e * max(1.0, abs(e_ref)), prec
        bg, bo = M.bond_dims(out), M.bond_dims(psi)
        assert all(abs(a - b) <= max(2, b // bond_frac) for a, b in zip(bg, bo)), (prec, bg, bo)
