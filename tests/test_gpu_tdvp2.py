"""Two-site TDVP on the device (tdvp_sweep2) against the two-site oracle and
exact diagonalisation."""
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


def _fid(a, b):
    from oracle import mps as M
    va, vb = M.to_dense(a), M.to_dense(b)
    return abs(np.vdot(va, vb)) ** 2 / (np.vdot(va, va).real * np.vdot(vb, vb).real)


def _rc(N, chi, seed):
    from oracle import mps as M
    psi = M.right_canonicalize(I.random_mps(N, chi, seed))
    psi[0] = psi[0] / np.linalg.norm(psi[0])
    return psi


def _run(T, ctx, N, terms, psi, steps, dt, eps, chi, normalize=False, prec="fp64"):
    from oracle import mpo, mps as M, tdvp2 as T2
    Ws = mpo.build_mpo(N, terms)
    H = T.tdvp_create_mpo(ctx, N, terms)
    g = T.tdvp_mps_from_host(ctx, psi)
    ref = psi
    rows = []
    for _ in range(steps):
        ref, _ = T2.tdvp2_sweep(ref, Ws, dt, eps, chi, 1e-12, 30, normalize)
        st = T.tdvp_sweep2(ctx, [g], [H], dt, eps, chi, 1e-12, 30, prec, normalize)[0]
        out = T.tdvp_mps_to_host(g)
        rows.append((1 - _fid(out, ref), M.bond_dims(out), M.bond_dims(ref), st, out, ref))
    return rows


def test_sweep2_exact_at_full_bond_dimension(env):
    T, ctx = env
    from oracle import ed, mps as M
    lat = I.ladder(3, 1.0, 0.7, "zigzag")
    terms = I.heisenberg_terms(lat.couplings)
    psi = _rc(6, 64, 3)
    rows = _run(T, ctx, 6, terms, psi, 1, 0.1, 0.0, 64)
    loss, bg, bo, st, out, _ = rows[0]
    assert loss < 1e-12 and bg == bo
    ref = ed.evolve(ed.hamiltonian(6, terms), M.to_dense(psi), 0.1)
    v = M.to_dense(out)
    assert 1 - abs(np.vdot(ref, v)) ** 2 / np.vdot(v, v).real < 1e-12


def test_sweep2_neel_quench_with_cap_matches_oracle(env):
    # real time from the Neel state with the chi cap active (bonds grow to it)
    T, ctx = env
    lat = I.ladder(4, 1.0, 1.0, "snake")
    terms = I.heisenberg_terms(lat.couplings)
    rows = _run(T, ctx, 8, terms, I.product_mps(lat.neel()), 6, 0.05, 1e-10, 6)
    for loss, bg, bo, st, out, ref in rows:
        assert loss < 1e-10
        assert all(abs(a - b) <= max(1, b // 10) for a, b in zip(bg, bo)), (bg, bo)
        assert max(bg) <= 6
    assert max(rows[-1][1]) == 6


def test_sweep2_imaginary_time_matches_oracle(env):
    T, ctx = env
    from oracle import mpo, observables as O
    lat = I.ladder(4, 1.0, 0.5, "zigzag")
    terms = I.heisenberg_terms(lat.couplings)
    rows = _run(T, ctx, 8, terms, _rc(8, 4, 11), 5, -0.2j, 1e-10, 16, normalize=True)
    Ws = mpo.build_mpo(8, terms)
    for loss, bg, bo, st, out, ref in rows:
        assert loss < 1e-10
        assert abs(st["energy"] - O.energy(ref, Ws)) < 1e-9


def test_sweep2_complex_hamiltonian_matches_oracle(env):
    T, ctx = env
    from test_oracle_tdvp import complex_hermitian_terms
    terms = complex_hermitian_terms(6, 4)
    rows = _run(T, ctx, 6, terms, _rc(6, 3, 5), 3, 0.07, 1e-12, 8)
    for loss, bg, bo, *_ in rows:
        assert loss < 1e-10 and bg == bo


def test_sweep2_fp32_within_mixed_bound(env):
    T, ctx = env
    lat = I.ladder(4, 1.0, 1.0, "snake")
    terms = I.heisenberg_terms(lat.couplings)
    rows = _run(T, ctx, 8, terms, I.product_mps(lat.neel()), 4, 0.05, 1e-10, 16, prec="fp32")
    t = 0.0
    for loss, *_ in rows:
        t += 0.05
        assert loss < 1e-5 * t


def test_sweep2_rejects_single_site(env):
    T, ctx = env
    H = T.tdvp_create_mpo(ctx, 1, [(0, -1, I.OP_SZ, I.OP_I, 1.0)])
    g = T.tdvp_mps_from_host(ctx, I.product_mps([0]))
    with pytest.raises(T.TdvpError):
        T.tdvp_sweep2(ctx, [g], [H], 0.1)
