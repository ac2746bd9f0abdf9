"""U(1) S^z charges on the device: states that carry bond charges run every
call block by block (factorisations charge by charge, new bonds with the
charges of their states).  The results must equal the dense oracle's on the
same inputs (gauge-invariant quantities), and every tensor must stay exactly
zero outside its charge blocks."""
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


def _check_blocks(T, g):
    """Entries outside q(b) = q(a) + q(s) are exactly zero; bonds ascend."""
    q = T.tdvp_mps_charges(g)
    assert q is not None
    t = T.tdvp_mps_to_host(g)
    for b in q:
        assert np.all(np.diff(b) >= 0)
    for i, M in enumerate(t):
        ql, qr = q[i], q[i + 1]
        assert M.shape == (len(ql), 2, len(qr))
        for s, dq in ((0, 1), (1, -1)):
            outside = qr[None, :] != ql[:, None] + dq
            assert np.all(M[:, s, :][outside] == 0), (i, s)
    return q


def _gse_both(T, ctx, N, terms, psi0, q0, dt, tau, k, eps_K, eps_M, eps, chi, steps, normalize, apply="denmat",
              prec="fp64", exact=False):
    from oracle import ed, gse, mpo, mps as M, observables as O
    Ws, Wop = mpo.build_mpo(N, terms), mpo.build_mpo(N, terms, 1.0, -1j * tau)
    H = T.tdvp_create_mpo(ctx, N, terms)
    op = T.tdvp_create_mpo(ctx, N, terms, 1.0, -1j * tau)
    g = T.tdvp_mps_from_host(ctx, psi0, q0)
    d = T.tdvp_mps_from_host(ctx, psi0)        # the same run without charges
    psi = psi0
    if exact:
        Hd = ed.hamiltonian(N, terms)
        v = M.to_dense(psi0)
        def vs_ed(x):
            y = M.to_dense(x)
            return 1 - abs(np.vdot(v, y)) ** 2 / (np.vdot(v, v).real * np.vdot(y, y).real)
    rows = []
    for _ in range(steps):
        psi, _ = gse.gse_step(psi, Ws, Wop, dt, k, eps_K, eps_M, eps, chi, 1e-12, 30, normalize, apply)
        for x in (g, d):
            T.tdvp_expand_basis(ctx, [x], [op], k, eps_K, eps_M, chi, prec, apply=apply)
            T.tdvp_sweep(ctx, [x], [H], dt, eps, chi, 1e-12, 30, prec, normalize)
        out, dense = T.tdvp_mps_to_host(g), T.tdvp_mps_to_host(d)
        m = T.tdvp_measure(ctx, [g], [H])[0]
        r = dict(loss=1 - M.fidelity(out, psi), loss_dense=1 - M.fidelity(out, dense),
                 de=m["energy"] - O.energy(psi, Ws), dsz=np.abs(m["sz"] - O.sz(psi)).max(),
                 bonds=M.bond_dims(out), bonds_ref=M.bond_dims(psi))
        if exact:
            v = ed.evolve(Hd, v, dt)
            r["ed_u1"], r["ed_oracle"] = vs_ed(out), vs_ed(psi)
        rows.append(r)
    q = _check_blocks(T, g)
    return rows, q


# Reading for the real-time checks below: after a basis extension the
# centres are rank deficient by design (the new directions carry no weight),
# and the one-site projector depends on how an exact gauge move completes the
# bond basis in directions without weight.  The dense QR takes them from
# rounding (any charge); with charges they are taken charge by charge (the
# Householder factor of each block, then completions from blocks with room to
# spare, so that the bond keeps the dense size).  Both are exact for the
# state; they differ in the projector by a few 1e-9 in fidelity over these
# runs (the dense device and the oracle differ by ~1e-9 the same way where the
# bond cap binds), and chained over many steps the gap grows.  So the runs
# are held to the exact dynamics: the error of the charged run against exact
# diagonalisation is at most twice the oracle's, and the charged run and the
# oracle are closer to each other than half the oracle's own error.


def test_mpo_charges_rejected_when_not_conserved(env):
    T, ctx = env
    lat = I.ladder(3, 1.0, 1.0, "snake")
    terms = I.heisenberg_terms(lat.couplings) + [(2, -1, I.OP_SP, I.OP_I, 0.3)]
    H = T.tdvp_create_mpo(ctx, lat.n_sites, terms)
    states = lat.neel()
    g = T.tdvp_mps_from_host(ctx, I.product_mps(states), I.product_charges(states))
    with pytest.raises(T.TdvpError) as ei:
        T.tdvp_sweep(ctx, [g], [H], 0.1)
    assert ei.value.status == T.TDVP_ERR_ARG


def test_upload_rejects_entries_outside_blocks(env):
    T, ctx = env
    psi = I.product_mps([0, 1, 0, 1])
    q = I.product_charges([0, 1, 0, 1])
    q[2] = np.array([5], dtype=np.int32)     # inconsistent with the tensors
    with pytest.raises(T.TdvpError) as ei:
        T.tdvp_mps_from_host(ctx, psi, q)
    assert ei.value.status == T.TDVP_ERR_ARG


def test_u1_ladder_quench_matches_oracle(env):
    # 2x6 snake ladder, Neel quench, k = 2, 20 steps of dt = 0.05 (the first
    # workload), with charges
    T, ctx = env
    w = I.workload(0)
    N = w.lattice.n_sites
    states = w.lattice.neel()
    rows, q = _gse_both(T, ctx, N, w.terms, I.product_mps(states), I.product_charges(states), w.dt, w.tau, w.k,
                        w.eps_K, w.eps_M, w.eps, w.chi_max, w.n_steps, False, exact=True)
    t = 0.0
    for r in rows:
        t += w.dt.real
        assert r["ed_u1"] <= 2.0 * r["ed_oracle"] + 1e-10, r
        assert r["loss"] <= 0.5 * r["ed_oracle"] + 1e-12, r
        assert abs(r["de"]) < 1e-9 and r["dsz"] < 1e-6, r
    assert all(np.all(np.abs(b) <= 12) for b in q) and q[-1][0] == 0


def test_u1_cylinder_quench_matches_oracle(env):
    # 4x4 J1-J2 cylinder (J2 = 0.5, snake, w from the FSA), Neel quench,
    # k = 3, tight cutoffs, 5 steps of dt = 0.05; with the cap 64 binding from
    # the third step, and with a cap that never binds
    T, ctx = env
    lat = I.cylinder(4, 4, 1.0, 0.5)
    N = lat.n_sites
    terms = I.heisenberg_terms(lat.couplings)
    states = lat.neel()
    for chi in (64, 256):
        rows, q = _gse_both(T, ctx, N, terms, I.product_mps(states), I.product_charges(states), 0.05, 0.05, 3,
                            1e-10, 1e-10, 0.0, chi, 5, False, exact=True)
        t = 0.0
        for r in rows:
            t += 0.05
            assert r["ed_u1"] <= 2.0 * r["ed_oracle"] + 1e-10, r
            assert r["loss"] <= 0.5 * r["ed_oracle"] + 1e-12, r
            if chi == 256:     # the cap never binds: close agreement
                assert r["loss"] < 1e-9 * t + 1e-12, r
            assert abs(r["de"]) < 1e-9 and r["dsz"] < 1e-7, r
        assert len(set(q[N // 2].tolist())) > 3     # several charge sectors in the middle


@pytest.mark.parametrize("apply", ["denmat", "fit"])
def test_u1_imaginary_time_random_start_with_cuts(env, apply):
    # a random U(1) state (total charge 0), imaginary time with eps > 0 and a
    # chi cap, both Krylov routes
    T, ctx = env
    lat = I.ladder(6, 1.0, 0.8, "snake")
    N = lat.n_sites
    terms = I.heisenberg_terms(lat.couplings)
    psi0, q0 = I.random_u1_mps(N, 12, 7)
    lam = I.energy_scale(lat.couplings)
    rows, q = _gse_both(T, ctx, N, terms, psi0, q0, -0.2j, -1j / lam, 3, 1e-12, 1e-8, 1e-10, 24, 3, True, apply)
    for r in rows:
        assert r["loss"] < 1e-9, r
        assert abs(r["de"]) < 1e-9, r
    assert max(max(b) for b in [r["bonds"] for r in rows]) <= 24


def test_u1_apply_mpo_routes_match_oracle(env):
    T, ctx = env
    from oracle import fit, krylov as K, mpo, mps as M
    lat = I.ladder(6, 1.0, 1.0, "snake")
    N = lat.n_sites
    terms = I.heisenberg_terms(lat.couplings)
    psi0, q0 = I.random_u1_mps(N, 10, 8)
    Wop = mpo.build_mpo(N, terms, 1.0, -0.1j)
    op = T.tdvp_create_mpo(ctx, N, terms, 1.0, -0.1j)
    g = T.tdvp_mps_from_host(ctx, psi0, q0)
    a, _ = T.tdvp_apply_mpo(ctx, g, op, "denmat", 1e-8, 20)
    ref, _ = K.apply_mpo_denmat(M.left_canonicalize(psi0), Wop, 1e-8, 20)
    assert 1 - M.fidelity(T.tdvp_mps_to_host(a), ref) < 1e-11
    assert M.bond_dims(T.tdvp_mps_to_host(a)) == M.bond_dims(ref)
    _check_blocks(T, a)
    b, _ = T.tdvp_apply_mpo(ctx, g, op, "fit", 1e-8, 20, passes=3)
    ref2, _ = fit.apply_mpo_variational(psi0, Wop, 1e-8, 20, 3)
    assert 1 - M.fidelity(T.tdvp_mps_to_host(b), ref2) < 1e-10
    _check_blocks(T, b)


def test_u1_two_site_sweep_matches_oracle(env):
    T, ctx = env
    from oracle import mpo, mps as M, tdvp2 as T2
    lat = I.ladder(5, 1.0, 1.0, "snake")
    N = lat.n_sites
    terms = I.heisenberg_terms(lat.couplings)
    states = lat.neel()
    psi = I.product_mps(states)
    Ws = mpo.build_mpo(N, terms)
    H = T.tdvp_create_mpo(ctx, N, terms)
    g = T.tdvp_mps_from_host(ctx, psi, I.product_charges(states))
    ref = psi
    for _ in range(4):
        ref, _ = T2.tdvp2_sweep(ref, Ws, 0.1, 1e-12, 32, 1e-12, 30, False)
        T.tdvp_sweep2(ctx, [g], [H], 0.1, 1e-12, 32, 1e-12, 30, "fp64", False)
        out = T.tdvp_mps_to_host(g)
        assert 1 - M.fidelity(out, ref) < 1e-10
    _check_blocks(T, g)


def _right_canonical_u1(tensors, charges):
    """Bring a charged MPS to the sweep's precondition (sites 1..N-1
    right-canonical, centre at site 0) by an LQ factorisation of each charge
    block: the rows of site i with left charge c live on the columns (s, b)
    with q(b) - q(s) = c only, so every block factorises on its own and the
    entries outside the blocks stay exactly zero."""
    t = [x.copy() for x in tensors]
    for i in range(len(t) - 1, 0, -1):
        ml, d, mr = t[i].shape
        ql, qr = charges[i], charges[i + 1]
        m = t[i].reshape(ml, d * mr)
        qcol = np.concatenate([qr - 1, qr + 1])     # q(b) - q(s) for s = up, down
        for c in np.unique(ql):
            r, k = np.nonzero(ql == c)[0], np.nonzero(qcol == c)[0]
            assert len(r) <= len(k)
            Q, R = np.linalg.qr(m[np.ix_(r, k)].conj().T)
            m[np.ix_(r, k)] = Q.conj().T
            t[i - 1][:, :, r] = t[i - 1][:, :, r] @ R.conj().T
        t[i] = m.reshape(ml, d, mr)
    t[0] /= np.linalg.norm(t[0])
    return t


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_u1_split_k_products_sweep_matches_oracle(env, prec):
    # A random charged state with bonds up to 256 on the 4x4 J1-J2 cylinder
    # (MPO bond dimension 20): the second product of H_eff and of K_eff then
    # has 2 x 2 x 4 output tiles with thousands of K entries each, too few
    # tiles to fill the GPU, so their K intervals run split into parts with
    # a reduction.  Two real-time sweeps against the oracle's.
    T, ctx = env
    from oracle import mpo, mps as M, observables as O, tdvp as TD
    lat = I.cylinder(4, 4, 1.0, 0.5)
    N = lat.n_sites
    terms = I.heisenberg_terms(lat.couplings)
    psi0, q0 = I.random_u1_mps(N, 256, 11)
    psi = _right_canonical_u1(psi0, q0)
    assert max(M.bond_dims(psi)) == 256
    Ws = mpo.build_mpo(N, terms)
    H = T.tdvp_create_mpo(ctx, N, terms)
    g = T.tdvp_mps_from_host(ctx, psi, q0)
    dt, t = 0.05, 0.0
    tol = {"fp64": (1e-8, 1e-10), "fp32": (1e-5, 1e-5), "bf16x3": (2e-5, 2e-4)}[prec]
    for _ in range(2):
        psi, _ = TD.tdvp1_sweep(psi, Ws, dt, 0.0, 256)
        T.tdvp_sweep(ctx, [g], [H], dt, 0.0, 256, 1e-12, 30, prec, False)
        t += dt
        out = T.tdvp_mps_to_host(g)
        e_ref = O.energy(psi, Ws)
        m = T.tdvp_measure(ctx, [g], [H])[0]
        assert 1 - M.fidelity(out, psi) < tol[0] * t, prec
        assert abs(m["energy"] - e_ref) < tol[1] * max(1.0, abs(e_ref)), (prec, m["energy"], e_ref)
    _check_blocks(T, g)
