"""Cholesky factorisation with the inverse of the factor on the device
(tdvp_cholesky, the factorisation behind the gauge moves' Cholesky-QR steps
and no-cut certificates) against numpy's LAPACK Cholesky: the backward
residual L L^H - G, the inverse L^-1 L - I, the factor itself (unique for a
positive diagonal), exact zeros above the diagonal of L^-1, the in-place
form, failure on indefinite input, and sizes across the 16 x 16 blocking
(one block, ragged last block row, up to the 512 limit).

Tolerances from the arithmetic (u = 2^-53): Cholesky is backward stable,
|L L^H - G| <= c n u |G| (c = 16 here); the inverse of a triangular factor
satisfies |Linv L - I| <= c n u cond(L); the factor's forward error is at
most c n u cond(G) relative to |L|."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2005_06104_amd import tdvp as T
    ctx = T.Context(0)
    yield T, torch, ctx
    ctx.close()


def _hpd(n, seed, extra=3):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n + extra, n)) + 1j * rng.standard_normal((n + extra, n))
    return X.conj().T @ X


def _run(env, G, inplace=False):
    T, torch, ctx = env
    n = G.shape[0]
    Gd = torch.from_numpy(np.ascontiguousarray(G)).cuda()
    L = Gd if inplace else torch.zeros_like(Gd)
    Li = torch.full_like(Gd, complex(np.nan, np.nan))
    info = T.tdvp_cholesky(ctx, Gd, L, Li)
    return info, np.tril(L.cpu().numpy()), Li.cpu().numpy()


@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 31, 33, 64, 100, 255, 256, 300, 511, 512])
def test_cholesky_matches_lapack(env, n):
    G = _hpd(n, 4000 + n)
    info, L, Li = _run(env, G)
    assert info == 0
    c = 16.0
    gn = np.linalg.norm(G)
    assert np.linalg.norm(L @ L.conj().T - G) <= c * n * U * gn
    condL = np.linalg.cond(L)
    assert np.linalg.norm(Li @ L - np.eye(n)) <= c * n * U * condL * np.sqrt(n)
    assert np.all(np.triu(Li, 1) == 0)
    assert np.all(np.diag(L).real > 0) and np.all(np.diag(L).imag == 0)
    Lref = np.linalg.cholesky(G)
    assert np.linalg.norm(L - Lref) <= c * n * U * np.linalg.cond(G) * np.linalg.norm(Lref)


@pytest.mark.parametrize("n", [16, 40, 256])
def test_cholesky_in_place_equals_out_of_place(env, n):
    G = _hpd(n, 4100 + n)
    info_a, La, Lia = _run(env, G)
    info_b, Lb, Lib = _run(env, G, inplace=True)
    assert info_a == info_b == 0
    assert np.array_equal(La, Lb) and np.array_equal(Lia, Lib)


@pytest.mark.parametrize("n,where", [(1, 0), (16, 15), (17, 16), (100, 3), (300, 290)])
def test_cholesky_reports_indefinite(env, n, where):
    # a Hermitian matrix whose leading (where+1) x (where+1) block is indefinite
    G = _hpd(n, 4200 + n)
    G[where, where] = -abs(G[where, where])
    info, _, _ = _run(env, G)
    assert info == 1


def test_cholesky_reports_zero_pivot(env):
    info, _, _ = _run(env, np.zeros((20, 20), dtype=np.complex128))
    assert info == 1


def test_cholesky_rejects_bad_arguments(env):
    import ctypes as C
    T, torch, ctx = env
    for n in (0, 513):
        m = max(n, 1)
        G = torch.zeros((m, m), dtype=torch.complex128, device="cuda")
        Li = torch.zeros_like(G)
        info = C.c_int(-1)
        assert ctx.lib.tdvp_cholesky(ctx.h, n, T._tp(G), T._tp(G), T._tp(Li), C.byref(info)) == T.TDVP_ERR_ARG
    G = torch.eye(8, dtype=torch.complex128, device="cuda")
    info = C.c_int(-1)
    assert ctx.lib.tdvp_cholesky(ctx.h, 8, T._tp(G), T._tp(G), T._tp(G), C.byref(info)) == T.TDVP_ERR_ARG
