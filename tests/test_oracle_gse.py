"""Pins for whole GSE-TDVP1 steps of the oracle against exact
diagonalisation and the closed forms of the paper (CPU only)."""
import json
import os

import numpy as np
import pytest

from paper_2005_06104_amd import inputs as I
from oracle import ed, gse, mpo, mps as M, observables as O, tdvp as T

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _run(w, psi, Ws, Wop, steps):
    for _ in range(steps):
        psi, st = gse.gse_step(psi, Ws, Wop, w.dt, w.k, w.eps_K, w.eps_M, w.eps, w.chi_max,
                               normalize=w.normalize)
    return psi


def test_config1_real_time_against_ed():
    # 2x6 snake ladder, Neel quench, k = 2: per-step fidelity vs ED and exact
    # conservation of norm and energy (eps = 0 keeps the step unitary)
    w = I.workload(0)
    N = w.lattice.n_sites
    Ws = mpo.build_mpo(N, w.terms)
    Wop = mpo.build_mpo(N, w.terms, 1.0, -1j * w.tau)
    H = ed.hamiltonian(N, w.terms)
    psi = w.initial_mps()
    v = M.to_dense(psi)
    e0 = O.energy(psi, Ws)
    for step in range(6):
        psi = _run(w, psi, Ws, Wop, 1)
        v = ed.evolve(H, v, w.dt)
        f = abs(np.vdot(M.to_dense(psi), v)) ** 2
        assert 1 - f < 1e-5
        assert abs(M.norm(psi) - 1) < 1e-12
        assert abs(O.energy(psi, Ws) - e0) < 1e-10
    assert np.abs(O.sz(psi) - ed.sz_profile(v, N)).max() < 1e-3
    assert max(M.bond_dims(psi)) <= w.chi_max


def test_time_step_convergence():
    # error falls at least quadratically in dt (the expansion removes the
    # projection error that would otherwise freeze it)
    w = I.workload(0)
    N = w.lattice.n_sites
    Ws = mpo.build_mpo(N, w.terms)
    H = ed.hamiltonian(N, w.terms)
    errs = []
    for dt in (0.1, 0.05):
        Wop = mpo.build_mpo(N, w.terms, 1.0, -1j * dt)
        psi = w.initial_mps()
        for _ in range(int(round(0.2 / dt))):
            psi, _ = gse.gse_step(psi, Ws, Wop, dt, 3, 1e-12, 1e-12, 0.0, 64)
        v = ed.evolve(H, M.to_dense(w.initial_mps()), 0.2)
        errs.append(1 - abs(np.vdot(M.to_dense(psi), v)) ** 2)
    assert errs[0] / errs[1] > 16.0


def test_rung_decoupled_failure_mechanism():
    # Fig. 1(c) mechanism: from a Neel product state on the rung-decoupled
    # zigzag ladder, one-site TDVP cannot move, GSE-TDVP1 reaches the ground state
    lat = I.ladder(4, 1.0, 0.0, "zigzag")
    N = lat.n_sites
    terms = I.heisenberg_terms(lat.couplings)
    Ws = mpo.build_mpo(N, terms)
    lam = I.energy_scale(lat.couplings)
    Wop = mpo.build_mpo(N, terms, 1.0, -1j * (-1j / lam))
    e_neel = O.energy(I.product_mps(lat.neel()), Ws)
    p1 = M.right_canonicalize(I.product_mps(lat.neel()))
    for _ in range(4):
        p1, _ = T.tdvp1_sweep(p1, Ws, -0.5j, 1e-10, 64, normalize=True)
    assert abs(O.energy(p1, Ws) - e_neel) < 1e-12
    p2 = I.product_mps(lat.neel())
    for _ in range(30):
        p2, _ = gse.gse_step(p2, Ws, Wop, -0.5j, 3, 1e-12, 1e-8, 1e-10, 64, normalize=True)
    e0 = ed.ground_energy(ed.hamiltonian(N, terms))
    assert O.energy(p2, Ws) - e0 < 1e-7


def test_imaginary_time_reaches_ed_ground_energy():
    lat = I.ladder(4, 1.0, 1.0, "snake")
    N = lat.n_sites
    terms = I.heisenberg_terms(lat.couplings)
    Ws = mpo.build_mpo(N, terms)
    lam = I.energy_scale(lat.couplings)
    Wop = mpo.build_mpo(N, terms, 1.0, -1j * (-1j / lam))
    psi = I.product_mps(lat.neel())
    for _ in range(30):
        psi, _ = gse.gse_step(psi, Ws, Wop, -0.5j, 3, 1e-12, 1e-8, 1e-12, 64, normalize=True)
    assert abs(O.energy(psi, Ws) - ed.ground_energy(ed.hamiltonian(N, terms))) < 1e-8


def test_oat_closed_form():
    # eq. (13) and the energy-conservation bound of Fig. 4(c), section II.B settings
    # (dt = 0.025, tau = dt, k = 3, eps = 0) on a small chain of spins
    N = 8
    terms = I.oat_terms(N)
    Ws = mpo.build_mpo(N, terms)
    assert max(mpo.bond_dims(Ws)) == GOLDEN["oat_mpo_bond_dim"]["value"]
    dt = 0.025
    Wop = mpo.build_mpo(N, terms, 1.0, -1j * dt)
    psi = I.x_polarized_mps(N)
    e0 = O.energy(psi, Ws)
    t = 0.0
    for _ in range(10):
        psi, _ = gse.gse_step(psi, Ws, Wop, dt, 3, 1e-10, 1e-10, 0.0, 64)
        t += dt
        assert abs(O.sx_total(psi) - O.oat_sx_exact(N, t)) < 1e-10
        assert abs(O.energy(psi, Ws) - e0) < GOLDEN["real_energy_error_bound"]["value"] * abs(e0)
    assert abs(t - GOLDEN["oat_final_time"]["value"]) < 1e-12
