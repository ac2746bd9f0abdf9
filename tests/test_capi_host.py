"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/tdvp.h declares, its host MPO builder agrees with the oracle's, and
bad arguments are rejected with TDVP_ERR_ARG."""
import ctypes as C
import os

import numpy as np
import pytest

from paper_2005_06104_amd import inputs as I
from paper_2005_06104_amd import tdvp as T

pytestmark = pytest.mark.skipif(not os.path.exists(T.LIB_PATH), reason="HIP library not built")


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(T.LIB_PATH)
    declared = T.header_functions()
    assert "tdvp_sweep" in declared and "tdvp_expand_basis" in declared and len(declared) >= 20
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    assert T.tdvp_version().startswith("tdvp-mi355x")


@pytest.mark.parametrize("case", ["snake", "zigzag", "cyl", "oat", "complex"])
def test_host_mpo_matches_oracle(case):
    from oracle import ed, mpo
    if case == "snake":
        lat = I.ladder(3, 1.0, 1.0, "snake"); N = lat.n_sites; terms = I.heisenberg_terms(lat.couplings)
    elif case == "zigzag":
        lat = I.ladder(3, 1.0, 0.0, "zigzag"); N = lat.n_sites; terms = I.heisenberg_terms(lat.couplings)
    elif case == "cyl":
        lat = I.cylinder(4, 2, 1.0, 0.5); N = lat.n_sites; terms = I.heisenberg_terms(lat.couplings)
    elif case == "oat":
        N = 7; terms = I.oat_terms(N)
    else:
        rng = np.random.default_rng(5); N = 6; terms = []
        for _ in range(20):
            i, j = rng.choice(N, size=2, replace=False)
            terms.append((int(i), int(j), int(rng.integers(0, 4)), int(rng.integers(0, 4)),
                          complex(rng.standard_normal(), rng.standard_normal())))
        terms += [(i, -1, 3, 0, 0.3 + 0.1j * i) for i in range(N)]
    c0, c1 = 1.0, -0.2j
    Ws = T.tdvp_build_mpo_host(N, terms, c0, c1)
    ref = mpo.build_mpo(N, terms, c0, c1)
    assert [W.shape[0] for W in Ws] == [W.shape[0] for W in ref]
    assert np.abs(mpo.mpo_to_dense(Ws) - ed.hamiltonian(N, terms, c0, c1).toarray()).max() < 1e-12
    if case == "oat":
        assert max(W.shape[0] for W in Ws) == 3


def test_host_mpo_rejects_bad_terms():
    lib = T.load()
    dims = np.zeros(5, dtype=np.int32)
    for bad in ([(0, 9, 3, 3, 1.0)], [(0, 0, 3, 3, 1.0)], [(0, 1, 7, 3, 1.0)], [(-1, 1, 3, 3, 1.0)]):
        arr = T.terms_array(bad)
        st = lib.tdvp_build_mpo_host(4, arr, 1, 0.0, 0.0, 1.0, 0.0, T._iptr(dims), None, 0)
        assert st == T.TDVP_ERR_ARG
    arr = T.terms_array([(0, 1, 3, 3, 1.0)])
    assert lib.tdvp_build_mpo_host(0, arr, 1, 0.0, 0.0, 1.0, 0.0, T._iptr(dims), None, 0) == T.TDVP_ERR_ARG
    assert lib.tdvp_build_mpo_host(4, arr, 1, 0.0, 0.0, 1.0, 0.0, None, None, 0) == T.TDVP_ERR_ARG
    # output capacity too small
    buf = np.zeros(4)
    assert lib.tdvp_build_mpo_host(4, arr, 1, 0.0, 0.0, 1.0, 0.0, T._iptr(dims), T._dptr(buf), 4) == T.TDVP_ERR_ARG


def test_null_handles_are_rejected():
    lib = T.load()
    assert lib.tdvp_sweep(None, 1, None, None, None, None) == T.TDVP_ERR_ARG
    assert lib.tdvp_expand_basis(None, 1, None, None, None, None) == T.TDVP_ERR_ARG
    assert lib.tdvp_measure(None, 1, None, None, None, None) == T.TDVP_ERR_ARG
    out, disc = C.c_void_p(), C.c_double()
    assert lib.tdvp_apply_mpo(None, None, None, 1, 1e-8, 8, 1, C.byref(out), C.byref(disc)) == T.TDVP_ERR_ARG
    assert lib.tdvp_synchronize(None) == T.TDVP_ERR_ARG
    h = C.c_void_p()
    assert lib.tdvp_ctx_create(0, None, T.ALLOC_FN(), T.FREE_FN(), None, None) == T.TDVP_ERR_ARG
    lib.tdvp_ctx_destroy(None)
    lib.tdvp_mps_destroy(None)
    lib.tdvp_mpo_destroy(None)


def test_squeezing_xi2_matches_eq14_scan():
    """tdvp_squeezing_xi2 (eq. (15)) against eq. (14) evaluated directly (the
    variance minimised over directions in the y-z plane by an angle scan) on
    one-axis-twisted states and on random states whose mean spin also has y
    and z components."""
    from oracle import ed
    from oracle.observables import xi2_dense

    def moments(v, N):
        S = {a: sum(ed.site_op(op, i, N) for i in range(N)) for a, op in (("x", ed.SX), ("y", ed.SY), ("z", ed.SZ))}
        e = lambda A: ed.expect(A, v)
        return (e(S["x"]).real, e(S["y"]).real, e(S["z"]).real, e(S["y"] @ S["y"]).real, e(S["z"] @ S["z"]).real,
                e(S["y"] @ S["z"] + S["z"] @ S["y"]).real)

    N = 6
    Sz = sum(ed.site_op(ed.SZ, i, N) for i in range(N))
    plus = np.ones(2 ** N, dtype=np.complex128) / np.sqrt(2 ** N)
    szd = Sz.diagonal().real
    states = [np.exp(-1j * t * szd ** 2) * plus for t in (0.05, 0.2, 0.45)]
    rng = np.random.default_rng(11)
    for _ in range(2):   # a random perturbation of the +x state: nonzero <S^y>, <S^z>
        v = plus + 0.15 * (rng.normal(size=2 ** N) + 1j * rng.normal(size=2 ** N)) / np.sqrt(2 ** N)
        states.append(v / np.linalg.norm(v))
    for v in states:
        sx, sy, sz, syy, szz, syz = moments(v, N)
        got = T.tdvp_squeezing_xi2(N, sx, syy, szz, syz, sy=sy, sz=sz)
        ref = xi2_dense(v, N)
        assert abs(got - ref) <= 1e-6 * abs(ref) + 1e-12, (got, ref)


def test_squeezing_xi2_rejects_bad_moments():
    with pytest.raises(T.TdvpError):
        T.tdvp_squeezing_xi2(10, 0.0, 1.0, 1.0, 0.0)
    with pytest.raises(T.TdvpError):
        T.tdvp_squeezing_xi2(0, 1.0, 1.0, 1.0, 0.0)
    with pytest.raises(T.TdvpError):
        T.tdvp_squeezing_xi2(4, 1.0, float("nan"), 1.0, 0.0)


@pytest.mark.parametrize("case", ["ladder", "cyl", "oat", "broken"])
def test_mpo_channel_charges(case):
    """Channel charges of the host MPO: every nonzero W[al,be,s',s] satisfies
    qw(be) = qw(al) + q(s') - q(s) with q(up) = 1, q(down) = -1, and both
    ends carry charge 0; a one-site S^+ term breaks the conservation."""
    if case == "ladder":
        lat = I.ladder(4, 1.0, 0.5, "zigzag"); N = lat.n_sites; terms = I.heisenberg_terms(lat.couplings)
    elif case == "cyl":
        lat = I.cylinder(4, 3, 1.0, 0.5); N = lat.n_sites; terms = I.heisenberg_terms(lat.couplings)
    elif case == "oat":
        N = 8; terms = I.oat_terms(N)
    else:
        lat = I.ladder(3, 1.0, 1.0, "snake"); N = lat.n_sites
        terms = I.heisenberg_terms(lat.couplings) + [(1, -1, I.OP_SP, I.OP_I, 0.5)]
    for c0, c1 in ((0.0, 1.0), (1.0, -0.1j)):
        q = T.tdvp_mpo_charges_host(N, terms, c0, c1)
        if case == "broken":
            assert q is None
            continue
        Ws = T.tdvp_build_mpo_host(N, terms, c0, c1)
        assert q[0].tolist() == [0] and q[-1].tolist() == [0]
        qs = np.array([1, -1])
        for i, W in enumerate(Ws):
            allowed = (q[i + 1][None, :, None, None] == q[i][:, None, None, None] + qs[None, None, :, None]
                       - qs[None, None, None, :])
            assert np.all(W[~allowed] == 0), i
