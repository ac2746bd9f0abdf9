"""Call-level parity on the GPU: tdvp_sweep, tdvp_expand_basis,
tdvp_measure and whole GSE-TDVP1 runs against the CPU oracle on the same
seeded inputs.  MPS tensors differ by gauge and phase, so only
gauge-invariant quantities are compared: fidelity, energy, norm, <S^z_i>,
bond dimensions."""
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
    return M.fidelity(a, b)


def _system(lat):
    from oracle import mpo
    terms = I.heisenberg_terms(lat.couplings)
    return terms, mpo.build_mpo(lat.n_sites, terms)


def _rc(N, chi, seed):
    from oracle import mps as M
    psi = M.right_canonicalize(I.random_mps(N, chi, seed))
    psi[0] = psi[0] / np.linalg.norm(psi[0])
    return psi


def test_measure_matches_oracle(env):
    T, ctx = env
    from oracle import mps as M, observables as O
    lat = I.ladder(5, 1.0, 0.7, "snake")
    terms, Ws = _system(lat)
    psi = I.random_mps(lat.n_sites, 6, 40)
    phi = I.random_mps(lat.n_sites, 3, 41)
    H = T.tdvp_create_mpo(ctx, lat.n_sites, terms)
    gp, gf = T.tdvp_mps_from_host(ctx, psi), T.tdvp_mps_from_host(ctx, phi)
    r = T.tdvp_measure(ctx, [gp], [H], [gf])[0]
    assert abs(r["energy"] - O.energy(psi, Ws)) < 1e-11
    assert abs(r["norm"] - M.norm(psi)) < 1e-10 * M.norm(psi)
    assert np.abs(r["sz"] - O.sz(psi)).max() < 1e-12
    assert abs(r["overlap"] - M.inner(phi, psi)) < 1e-10 * M.norm(psi) * M.norm(phi)
    assert r["bond_dims"] == [1] + M.bond_dims(psi) + [1]
    back = T.tdvp_mps_to_host(gp)
    assert all(np.array_equal(a, b) for a, b in zip(back, psi))


@pytest.mark.parametrize("case", ["real", "imag_trunc", "complex_ham"])
def test_sweep_matches_oracle(env, case):
    T, ctx = env
    from oracle import mpo, mps as M, observables as O, tdvp as OT
    if case == "complex_ham":
        N = 9
        rng = np.random.default_rng(4)
        terms = []
        for _ in range(14):
            i, j = (int(x) for x in rng.choice(N, size=2, replace=False))
            c = complex(rng.standard_normal(), rng.standard_normal())
            terms += [(i, j, 1, 2, c), (i, j, 2, 1, c.conjugate()), (i, j, 3, 3, complex(rng.standard_normal()))]
        Ws = mpo.build_mpo(N, terms)
    else:
        lat = I.ladder(5, 1.0, 1.0, "snake")
        N = lat.n_sites
        terms, Ws = _system(lat)
    psi = _rc(N, 12, 50)
    kw = dict(dt=0.1, eps=0.0, chi_max=1 << 30, normalize=False)
    if case == "imag_trunc":
        kw = dict(dt=-0.3j, eps=1e-6, chi_max=10, normalize=True)
    ref, rst = OT.tdvp1_sweep(psi, Ws, kw["dt"], kw["eps"], kw["chi_max"], 1e-12, 30, kw["normalize"])
    H = T.tdvp_create_mpo(ctx, N, terms)
    g = T.tdvp_mps_from_host(ctx, psi)
    st = T.tdvp_sweep(ctx, [g], [H], kw["dt"], kw["eps"], kw["chi_max"], 1e-12, 30, "fp64", kw["normalize"])[0]
    out = T.tdvp_mps_to_host(g)
    assert M.bond_dims(out) == M.bond_dims(ref)
    assert 1 - _fid(out, ref) < 1e-12
    assert abs(M.norm(out) - M.norm(ref)) < 1e-12
    assert abs(O.energy(out, Ws) - O.energy(ref, Ws)) < 1e-10
    assert abs(st["energy"] - O.energy(ref, Ws)) < 1e-10
    assert M.is_right_canonical(out, 1e-11)
    assert st["n_matvec"] > 0 and st["n_unconverged"] == 0
    assert abs(st["n_matvec"] - rst["n_matvec"]) <= 2


def test_expand_matches_oracle(env):
    T, ctx = env
    from oracle import extension as X, krylov as K, mpo, mps as M
    lat = I.ladder(5, 1.0, 1.0, "snake")
    N = lat.n_sites
    terms, Ws = _system(lat)
    dt = 0.1
    Wop = mpo.build_mpo(N, terms, 1.0, -1j * dt)
    psi = _rc(N, 3, 60)
    pl = M.left_canonicalize(psi)
    kv = K.krylov_vectors(pl, Wop, 3, 1e-10, 24)
    ref, _ = X.basis_extension(pl, kv, 1e-8, 24)
    op = T.tdvp_create_mpo(ctx, N, terms, 1.0, -1j * dt)
    g = T.tdvp_mps_from_host(ctx, psi)
    st = T.tdvp_expand_basis(ctx, [g], [op], 3, 1e-10, 1e-8, 24, "fp64")[0]
    out = T.tdvp_mps_to_host(g)
    assert M.bond_dims(out) == M.bond_dims(ref)
    assert 1 - _fid(out, psi) < 1e-13                 # the state is kept exactly
    assert M.is_right_canonical(out, 1e-11)
    assert st["n_added"] == sum(M.bond_dims(ref)) - sum(M.bond_dims(pl))
    # same extended bond spaces: the right-block projectors agree
    for i in (1, N // 2, N - 1):
        def proj(B):
            T_ = B[N - 1][:, :, 0]
            for j in range(N - 2, i - 1, -1):
                T_ = np.tensordot(B[j], T_, axes=(2, 0)).reshape(B[j].shape[0], -1)
            q, _ = np.linalg.qr(T_.conj().T)
            return q @ q.conj().T
        assert np.abs(proj(out) - proj(ref)).max() < 1e-9


def _run_both(T, ctx, w, steps, prec="fp64"):
    from oracle import gse, mpo, mps as M, observables as O
    N = w.lattice.n_sites
    Ws = mpo.build_mpo(N, w.terms)
    Wop = mpo.build_mpo(N, w.terms, 1.0, -1j * w.tau)
    H = T.tdvp_create_mpo(ctx, N, w.terms)
    op = T.tdvp_create_mpo(ctx, N, w.terms, 1.0, -1j * w.tau)
    psi = w.initial_mps()
    g = T.tdvp_mps_from_host(ctx, psi)
    rows = []
    for step in range(steps):
        psi, _ = gse.gse_step(psi, Ws, Wop, w.dt, w.k, w.eps_K, w.eps_M, w.eps, w.chi_max, 1e-12, 30, w.normalize)
        T.tdvp_expand_basis(ctx, [g], [op], w.k, w.eps_K, w.eps_M, w.chi_max, prec)
        T.tdvp_sweep(ctx, [g], [H], w.dt, w.eps, w.chi_max, 1e-12, 30, prec, w.normalize)
        out = T.tdvp_mps_to_host(g)
        m = T.tdvp_measure(ctx, [g], [H])[0]
        rows.append((1 - _fid(out, psi), m["energy"] - O.energy(psi, Ws),
                     np.abs(m["sz"] - O.sz(psi)).max(), M.bond_dims(out), M.bond_dims(psi)))
    return rows


def test_gse_config1_fp64_matches_oracle(env):
    # 2x6 snake ladder, Neel quench, k = 2, 20 steps of dt = 0.05
    T, ctx = env
    w = I.workload(0)
    rows = _run_both(T, ctx, w, w.n_steps)
    t = 0.0
    for (loss, de, dsz, bg, bo) in rows:
        t += w.dt.real
        assert loss < 1e-8 * t + 1e-12          # fidelity loss < 1e-8 per unit time
        assert abs(de) < 1e-9 and dsz < 1e-7
        # a cut can land on an eigenvalue within rounding of the threshold; such a
        # state carries weight ~eps_M, so bonds may differ by a state or two
        assert all(abs(a - b) <= max(2, b // 10) for a, b in zip(bg, bo)), (bg, bo)


def test_gse_config1_fp32_within_mixed_bound(env):
    T, ctx = env
    w = I.workload(0)
    rows = _run_both(T, ctx, w, 10, prec="fp32")
    t = 0.0
    for (loss, de, dsz, bg, bo) in rows:
        t += w.dt.real
        assert loss < 1e-5 * t                  # mixed path: < 1e-5 per unit time
        assert abs(de) < 1e-4


def test_gse_config1_bf16x3_within_mixed_bound(env):
    # three-term BF16 split (~16-bit operands, FP32 accumulation) in every
    # contraction; FP64 Lanczos, factorisations and stored tensors
    T, ctx = env
    w = I.workload(0)
    rows = _run_both(T, ctx, w, 10, prec="bf16x3")
    t = 0.0
    for (loss, de, dsz, bg, bo) in rows:
        t += w.dt.real
        assert loss < 1e-5 * t                  # mixed path: < 1e-5 per unit time
        assert abs(de) < 1e-4


def test_gse_config1_bf16_single_term(env):
    # plain BF16 operands (8 significant bits) do not reach the 1e-5 per unit
    # time mixed-path target on this quench (about 1.6e-5 at t = 0.5); the
    # test pins the level it does reach, a tenth of a percent in energy
    T, ctx = env
    w = I.workload(0)
    rows = _run_both(T, ctx, w, 10, prec="bf16")
    t = 0.0
    for (loss, de, dsz, bg, bo) in rows:
        t += w.dt.real
        assert loss < 1e-4 * t
        assert abs(de) < 1e-2 and dsz < 1e-2


def test_gse_imaginary_time_random_start(env):
    # small version of the rung-decoupled zigzag workload from a random MPS
    T, ctx = env
    w = I.workload(1)
    lat = I.ladder(6, 1.0, 0.0, "zigzag")
    w = I.Workload("small_imag", lat, "random", 8, 2, w.dt, 6, 3, 1e-12, 1e-8, 1e-10, 32, "fp64",
                   complex(0, -1.0 / I.energy_scale(lat.couplings)), True)
    rows = _run_both(T, ctx, w, w.n_steps)
    for (loss, de, dsz, bg, bo) in rows:
        assert loss < 1e-9 and abs(de) < 1e-9


def test_gse_oat_closed_form_on_device(env):
    # eq. (13): <S^x(t)> = (N/2) cos^(N-1) t for the one-axis-twisting model
    # (w = 3 long-range MPO), section II.B settings dt = 0.025, tau = dt, k = 3,
    # eps = 0; real-time energy error below 1e-10 (Fig. 4(c)).  At N = 16 the
    # method itself is 1.1e-8 off the closed form at t = 0.25 (the oracle shows
    # the same), so the device must agree with the oracle far more tightly.
    T, ctx = env
    from oracle import gse, mpo, observables as O
    N = 16
    terms = I.oat_terms(N)
    dt = 0.025
    H = T.tdvp_create_mpo(ctx, N, terms)
    op = T.tdvp_create_mpo(ctx, N, terms, 1.0, -1j * dt)
    assert max(H.dims) == 3
    g = T.tdvp_mps_from_host(ctx, I.x_polarized_mps(N))
    Ws, Wop = mpo.build_mpo(N, terms), mpo.build_mpo(N, terms, 1.0, -1j * dt)
    psi = I.x_polarized_mps(N)
    e0 = T.tdvp_measure(ctx, [g], [H])[0]["energy"]
    t = 0.0
    for _ in range(10):
        T.tdvp_expand_basis(ctx, [g], [op], 3, 1e-10, 1e-10, 64, "fp64")
        T.tdvp_sweep(ctx, [g], [H], dt, 0.0, 64, 1e-12, 30, "fp64", False)
        psi, _ = gse.gse_step(psi, Ws, Wop, dt, 3, 1e-10, 1e-10, 0.0, 64)
        t += dt
        m = T.tdvp_measure(ctx, [g], [H])[0]
        assert abs(m["energy"] - e0) < 1e-10 * abs(e0)
        assert np.abs(m["sz"]).max() < 1e-10            # <S^z> = 0
        sx = O.sx_total(T.tdvp_mps_to_host(g))
        assert abs(sx - O.sx_total(psi)) < 1e-10
        assert abs(sx - O.oat_sx_exact(N, t)) < 5e-8


def test_oat_squeezing_moments_on_device(env):
    # eqs. (14)-(15): the total-spin moments measured on the device as MPO
    # expectation values agree with the oracle's state to rounding and with
    # the exact symmetric-subspace dynamics to the method's error (1e-5 on xi^2)
    T, ctx = env
    from oracle import gse, mpo, observables as O
    N, dt = 16, 0.025
    terms = I.oat_terms(N)
    H = T.tdvp_create_mpo(ctx, N, terms)
    op = T.tdvp_create_mpo(ctx, N, terms, 1.0, -1j * dt)
    names = ("x", "yy", "zz", "yz")
    dev_ops = {k: T.tdvp_create_mpo(ctx, N, I.spin_moment_terms(N, k)) for k in names}
    cpu_ops = {k: mpo.build_mpo(N, I.spin_moment_terms(N, k)) for k in names}
    Ws, Wop = mpo.build_mpo(N, terms), mpo.build_mpo(N, terms, 1.0, -1j * dt)
    g = T.tdvp_mps_from_host(ctx, I.x_polarized_mps(N))
    psi = I.x_polarized_mps(N)
    t = 0.0
    for _ in range(10):
        T.tdvp_expand_basis(ctx, [g], [op], 3, 1e-10, 1e-10, 64, "fp64")
        T.tdvp_sweep(ctx, [g], [H], dt, 0.0, 64, 1e-12, 30, "fp64", False)
        psi, _ = gse.gse_step(psi, Ws, Wop, dt, 3, 1e-10, 1e-10, 0.0, 64)
        t += dt
        dev = {k: T.tdvp_measure(ctx, [g], [dev_ops[k]])[0]["energy"] for k in names}
        ref = {k: O.energy(psi, cpu_ops[k]) for k in names}
        for k in names:
            assert abs(dev[k] - ref[k]) < 1e-9 * max(1.0, abs(ref[k])), (k, dev[k], ref[k])
        xi2 = O.xi2_from_moments(N, dev["x"], dev["yy"], dev["zz"], dev["yz"], 0.0)
        assert abs(xi2 - O.oat_xi2_dicke(N, t)) < 1e-5 * O.oat_xi2_dicke(N, t)


def test_batched_instances_match_single_runs(env):
    # several independent ladders of different sizes and couplings in one call
    # (worker streams): each instance agrees with the oracle's run of that
    # ladder, and with the same ladder stepped alone on the device
    T, ctx = env
    from oracle import gse, mpo, mps as M, observables as O
    lats = [I.ladder(L, jl, jr, "snake") for (L, jl, jr) in ((4, 1.0, 0.6), (6, 0.8, 1.2), (5, 1.1, 0.9),
                                                             (3, 1.0, 1.0), (7, 0.7, 1.3))]
    Hs, ops, batch, single, refs, cpu = [], [], [], [], [], []
    for j, lat in enumerate(lats):
        terms = I.heisenberg_terms(lat.couplings)
        lam = I.energy_scale(lat.couplings)
        tau = -1j / lam
        Hs.append(T.tdvp_create_mpo(ctx, lat.n_sites, terms))
        ops.append(T.tdvp_create_mpo(ctx, lat.n_sites, terms, 1.0, -1j * tau))
        psi0 = I.product_mps(lat.neel())
        batch.append(T.tdvp_mps_from_host(ctx, psi0))
        single.append(T.tdvp_mps_from_host(ctx, psi0))
        refs.append(psi0)
        cpu.append((mpo.build_mpo(lat.n_sites, terms), mpo.build_mpo(lat.n_sites, terms, 1.0, -1j * tau)))
    for _ in range(3):
        T.tdvp_expand_basis(ctx, batch, ops, 3, 1e-12, 1e-8, 32, "fp64")
        T.tdvp_sweep(ctx, batch, Hs, -0.2j, 1e-10, 32, 1e-12, 30, "fp64", True)
        for j in range(len(lats)):
            T.tdvp_expand_basis(ctx, [single[j]], [ops[j]], 3, 1e-12, 1e-8, 32, "fp64")
            T.tdvp_sweep(ctx, [single[j]], [Hs[j]], -0.2j, 1e-10, 32, 1e-12, 30, "fp64", True)
            refs[j], _ = gse.gse_step(refs[j], cpu[j][0], cpu[j][1], -0.2j, 3, 1e-12, 1e-8, 1e-10, 32, 1e-12, 30,
                                      True)
    mb = T.tdvp_measure(ctx, batch, Hs)
    ms = T.tdvp_measure(ctx, single, Hs)
    for j in range(len(lats)):
        a, b = T.tdvp_mps_to_host(batch[j]), T.tdvp_mps_to_host(single[j])
        assert M.bond_dims(a) == M.bond_dims(b)
        assert 1 - M.fidelity(a, b) < 1e-12
        assert abs(mb[j]["energy"] - ms[j]["energy"]) < 1e-11
        # against the oracle (imaginary time, 3 steps: fidelity loss < 1e-8 per unit time)
        assert 1 - M.fidelity(a, refs[j]) < 1e-8 * 0.6 + 1e-12, j
        assert abs(mb[j]["energy"] - O.energy(refs[j], cpu[j][0])) < 1e-9, j
        assert np.abs(mb[j]["sz"] - O.sz(refs[j])).max() < 1e-7, j


def test_expand_floor_reading_on_device(env):
    # "SVD without truncation" (section I.A) reads as: directions with weight
    # s^2 <= 1e-14 s_1^2 are not part of B.  On a state with two Schmidt
    # values inside (1e-13, 1e-7) s_1 across one bond and a Krylov vector that
    # does not carry them (the identity MPO: its density-matrix cut drops the
    # same directions), psi changes by exactly their weight, as in the oracle.
    import os, sys
    sys.path.insert(0, os.path.dirname(__file__))
    from states import mps_with_schmidt
    T, ctx = env
    from oracle import extension as X, krylov as K, mpo, mps as M
    sch = [1.0, 0.6, 0.3, 2e-7, 2e-8, 5e-9]
    pl = M.left_canonicalize(mps_with_schmidt(7, 3, sch, 3))
    s = np.array(sch) / np.linalg.norm(sch)
    dropped = float(np.sum(s[s ** 2 <= 1e-14 * s[0] ** 2] ** 2))
    terms = I.heisenberg_terms(I.chain(7).couplings)
    op = T.tdvp_create_mpo(ctx, 7, terms, 1.0, 0.0)
    g = T.tdvp_mps_from_host(ctx, pl)
    T.tdvp_expand_basis(ctx, [g], [op], 2, 0.0, 1e-8, 1 << 20, "fp64", skip_if_full=False)
    out = T.tdvp_mps_to_host(g)
    d = np.linalg.norm(M.to_dense(out) - M.to_dense(pl)) ** 2
    assert abs(d - dropped) < 1e-2 * dropped, (d, dropped)
    kv = K.krylov_vectors(pl, mpo.build_mpo(7, terms, 1.0, 0.0), 2, 0.0, 1 << 20)
    ref, _ = X.basis_extension(pl, kv, 1e-8, 1 << 20)
    assert M.bond_dims(out) == M.bond_dims(ref)
    assert M.bond_dims(out)[2] == 4
