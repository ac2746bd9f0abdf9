"""One-axis twisting (section II.B, eqs. (12)-(15)): the exact symmetric-
subspace reference and the total-spin moment term lists, pinned against
dense exact diagonalisation and the closed form of eq. (13)."""
import numpy as np
import pytest

from oracle import ed, observables as O
from paper_2005_06104_amd import inputs as I


def _dense_totals(N):
    S = {a: sum(ed.site_op(op, i, N) for i in range(N)) for a, op in (("x", ed.SX), ("y", ed.SY), ("z", ed.SZ))}
    return S


def _dense_state(N, t):
    plus = np.array([1.0, 1.0], dtype=complex) / np.sqrt(2.0)
    psi = ed.local_vector_product([plus] * N)
    Sz = _dense_totals(N)["z"]
    return ed.evolve((Sz @ Sz).tocsr(), psi, t)


@pytest.mark.parametrize("t", [0.0, 0.13, 0.4])
def test_dicke_moments_match_dense_dynamics(t):
    N = 6
    S = _dense_totals(N)
    psi = _dense_state(N, t)
    m = O.oat_moments_dicke(N, t)
    assert abs(m["sx"] - ed.expect(S["x"], psi).real) < 1e-12
    assert abs(m["sy"] - ed.expect(S["y"], psi).real) < 1e-12
    assert abs(m["sz"] - ed.expect(S["z"], psi).real) < 1e-12
    assert abs(m["syy"] - ed.expect(S["y"] @ S["y"], psi).real) < 1e-12
    assert abs(m["szz"] - ed.expect(S["z"] @ S["z"], psi).real) < 1e-12
    anti = ed.expect(S["y"] @ S["z"] + S["z"] @ S["y"], psi).real
    assert abs(m["syz_szy"] - anti) < 1e-12


def test_dicke_sx_is_the_closed_form():
    # eq. (13) at the paper's N = 100
    for t in (0.01, 0.0557, 0.1, 0.25):
        assert abs(O.oat_moments_dicke(100, t)["sx"] - O.oat_sx_exact(100, t)) < 1e-11 * 50


def test_dicke_xi2_matches_the_minimisation():
    # eq. (15) from the Dicke moments equals eq. (14) minimised over the y-z plane
    N = 6
    for t in (0.1, 0.3):
        assert abs(O.oat_xi2_dicke(N, t) - O.xi2_dense(_dense_state(N, t), N)) < 1e-6


@pytest.mark.parametrize("which", ["x", "y", "z", "yy", "zz", "yz"])
def test_spin_moment_terms_are_the_operators(which):
    N = 6
    S = _dense_totals(N)
    ref = {"x": S["x"], "y": S["y"], "z": S["z"], "yy": S["y"] @ S["y"], "zz": S["z"] @ S["z"],
           "yz": S["y"] @ S["z"] + S["z"] @ S["y"]}[which]
    H = ed.hamiltonian(N, I.spin_moment_terms(N, which))
    assert abs(H - ref).max() < 1e-13


def test_squeezing_is_strong_near_t_opt():
    # section II.B: at N = 100 the optimal squeezing time is t_opt ~ 0.056;
    # xi^2 there is far below the coherent-state value 1
    N = 100
    t = O.oat_t_opt(N)
    assert O.oat_xi2_dicke(N, 0.0) == pytest.approx(1.0, abs=1e-12)
    assert O.oat_xi2_dicke(N, t) < 0.1
    ts = np.linspace(0.02, 0.12, 101)
    best = ts[int(np.argmin([O.oat_xi2_dicke(N, x) for x in ts]))]
    assert abs(best - t) < 0.01
