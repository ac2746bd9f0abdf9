"""Error contract of the C-ABI on the GPU: strict mode completes the sweep
and keeps the state valid, a state given twice in one batched call is
rejected before anything changes, and the one-site sweep with eps = 0 never
truncates (exact, unitary gauge moves) whatever chi_max says."""
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


def _rc(N, chi, seed):
    from oracle import mps as M
    psi = M.right_canonicalize(I.random_mps(N, chi, seed))
    psi[0] = psi[0] / np.linalg.norm(psi[0])
    return psi


def test_strict_noconv_completes_sweep_and_keeps_state(env):
    T, ctx = env
    from oracle import mpo, mps as M, tdvp as OT
    lat = I.ladder(4, 1.0, 1.0, "snake")
    N = lat.n_sites
    terms = I.heisenberg_terms(lat.couplings)
    Ws = mpo.build_mpo(N, terms)
    psi = _rc(N, 8, 70)
    H = T.tdvp_create_mpo(ctx, N, terms)
    g = T.tdvp_mps_from_host(ctx, psi)
    # two Lanczos vectors cannot reach 1e-12 for a step of 0.4
    with pytest.raises(T.TdvpError) as ei:
        T.tdvp_sweep(ctx, [g], [H], 0.4, 0.0, 1 << 30, 1e-12, 2, "fp64", False, strict=True)
    assert ei.value.status == T.TDVP_ERR_NOCONV
    st = ei.value.stats[0]
    assert st["n_unconverged"] > 0 and st["max_lanczos"] == 2
    # the handle stays valid and holds the completed sweep with the
    # unconverged local steps: the oracle's sweep with the same limit
    ref, _ = OT.tdvp1_sweep(psi, Ws, 0.4, 0.0, 1 << 30, 1e-12, 2, False)
    out = T.tdvp_mps_to_host(g)
    assert 1 - M.fidelity(out, ref) < 1e-11
    m = T.tdvp_measure(ctx, [g], [H])[0]
    assert abs(m["norm"] - 1.0) < 1e-12            # Lanczos keeps the norm exactly
    T.tdvp_sweep(ctx, [g], [H], 0.05, 0.0, 1 << 30, 1e-12, 30, "fp64", False, strict=True)


def test_duplicate_state_in_batch_is_rejected(env):
    T, ctx = env
    lat = I.ladder(3, 1.0, 1.0, "snake")
    N = lat.n_sites
    terms = I.heisenberg_terms(lat.couplings)
    H = T.tdvp_create_mpo(ctx, N, terms)
    op = T.tdvp_create_mpo(ctx, N, terms, 1.0, -0.1j)
    psi = _rc(N, 4, 71)
    g = T.tdvp_mps_from_host(ctx, psi)
    before = T.tdvp_mps_to_host(g)
    for call in (lambda: T.tdvp_sweep(ctx, [g, g], [H, H], 0.1),
                 lambda: T.tdvp_sweep2(ctx, [g, g], [H, H], 0.1),
                 lambda: T.tdvp_expand_basis(ctx, [g, g], [op, op], 3, 1e-10, 1e-8, 16)):
        with pytest.raises(T.TdvpError) as ei:
            call()
        assert ei.value.status == T.TDVP_ERR_ARG
    after = T.tdvp_mps_to_host(g)
    assert all(np.array_equal(a, b) for a, b in zip(before, after))


def test_eps_zero_sweep_never_truncates(env):
    T, ctx = env
    from oracle import mpo, mps as M, tdvp as OT
    lat = I.ladder(4, 1.0, 1.0, "snake")
    N = lat.n_sites
    terms = I.heisenberg_terms(lat.couplings)
    Ws = mpo.build_mpo(N, terms)
    psi = _rc(N, 12, 72)
    H = T.tdvp_create_mpo(ctx, N, terms)
    g = T.tdvp_mps_from_host(ctx, psi)
    dims = M.bond_dims(psi)
    assert max(dims) > 6
    T.tdvp_sweep(ctx, [g], [H], 0.1, 0.0, 6, 1e-12, 30, "fp64", False)   # chi_max below the bonds
    out = T.tdvp_mps_to_host(g)
    assert M.bond_dims(out) == dims
    ref, _ = OT.tdvp1_sweep(psi, Ws, 0.1, 0.0, 1 << 30, 1e-12, 30, False)
    assert 1 - M.fidelity(out, ref) < 1e-12
    assert abs(T.tdvp_measure(ctx, [g], [H])[0]["norm"] - 1.0) < 1e-12
