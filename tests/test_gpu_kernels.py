"""Kernel-level parity on the GPU: complex GEMM, one-site and zero-site
effective Hamiltonians and environment updates against the CPU oracle, on
the same seeded inputs, through the C-ABI."""
import numpy as np
import pytest

from paper_2005_06104_amd import inputs as I

pytestmark = pytest.mark.gpu

# tolerances relative to max|result|: FP64 ~ u sqrt(K) with margin, FP32 the same for u = 2^-24
TOL = {"fp64": 1e-12, "fp32": 2e-5}


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2005_06104_amd import tdvp as T
    ctx = T.Context(0)
    yield T, torch, ctx
    ctx.close()


def _dev(torch, a, prec):
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()


def _host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def _op(a, op):
    return {0: a, 1: a.T, 2: a.conj().T, 3: a.conj()}[op]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("opa", [0, 1, 2, 3])
@pytest.mark.parametrize("opb", [0, 1, 2, 3])
def test_gemm_all_ops_ragged_batched(env, prec, opa, opb):
    T, torch, ctx = env
    M, N, K, batch = 77, 45, 131, 3
    rng = np.random.default_rng(100 + 4 * opa + opb)
    ashape = (M, K) if opa in (0, 3) else (K, M)
    bshape = (K, N) if opb in (0, 3) else (N, K)
    A = rng.standard_normal((batch,) + ashape) + 1j * rng.standard_normal((batch,) + ashape)
    B = rng.standard_normal((batch,) + bshape) + 1j * rng.standard_normal((batch,) + bshape)
    C0 = rng.standard_normal((batch, M, N)) + 1j * rng.standard_normal((batch, M, N))
    alpha, beta = 0.7 - 0.3j, -0.4 + 0.2j
    dA, dB, dC = _dev(torch, A, prec), _dev(torch, B, prec), _dev(torch, C0, prec)
    T.tdvp_gemm(ctx, opa, opb, M, N, K, alpha, dA, ashape[1], ashape[0] * ashape[1], dB, bshape[1],
                bshape[0] * bshape[1], beta, dC, N, M * N, batch)
    torch.cuda.synchronize()
    ref = np.stack([alpha * _op(A[b], opa) @ _op(B[b], opb) + beta * C0[b] for b in range(batch)])
    err = np.abs(_host(dC) - ref).max() / np.abs(ref).max()
    assert err < TOL[prec], err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (1, 300, 7), (256, 256, 256), (513, 130, 65), (64, 64, 4096)])
def test_gemm_shapes(env, prec, M, N, K):
    T, torch, ctx = env
    rng = np.random.default_rng(M + N + K)
    A = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    B = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    dA, dB = _dev(torch, A, prec), _dev(torch, B, prec)
    dC = _dev(torch, np.zeros((M, N)), prec)
    T.tdvp_gemm(ctx, 0, 0, M, N, K, 1.0, dA, K, 0, dB, N, 0, 0.0, dC, N, 0, 1)
    torch.cuda.synchronize()
    ref = A @ B
    assert np.abs(_host(dC) - ref).max() / np.abs(ref).max() < TOL[prec] * max(1.0, np.sqrt(K / 256))


def _heff_inputs(ml, wl, wr, mr, seed):
    L = I.random_hermitian_env(ml, wl, seed)
    R = I.random_hermitian_env(mr, wr, seed + 1)
    W = I.random_mpo_site(wl, wr, seed + 2)
    C = I.random_complex((ml, 2, mr), seed + 3)
    return L, W, R, C


SIZES = [(1, 1, 5, 16), (37, 5, 8, 29), (64, 8, 8, 64), (130, 8, 8, 70), (16, 8, 1, 1)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ml,wl,wr,mr", SIZES)
def test_heff_matches_oracle(env, prec, ml, wl, wr, mr):
    from oracle import tdvp as O
    T, torch, ctx = env
    L, W, R, C = _heff_inputs(ml, wl, wr, mr, 7 * ml + mr)
    Rt = np.ascontiguousarray(R.transpose(1, 2, 0))      # Rt[be, b, b'] = R[b', be, b]
    dL, dRt, dC = _dev(torch, L, prec), _dev(torch, Rt, prec), _dev(torch, C, prec)
    dY = _dev(torch, np.zeros_like(C), prec)
    T.tdvp_heff_apply(ctx, W, dL, dRt, dC, dY)
    torch.cuda.synchronize()
    ref = O.heff_apply(L, W, R, C)
    err = np.abs(_host(dY) - ref).max() / np.abs(ref).max()
    assert err < TOL[prec], err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ml,w,mr", [(1, 5, 3), (33, 8, 47), (128, 8, 128)])
def test_keff_matches_oracle(env, prec, ml, w, mr):
    from oracle import tdvp as O
    T, torch, ctx = env
    L = I.random_hermitian_env(ml, w, 3 * ml)
    R = I.random_hermitian_env(mr, w, 5 * mr)
    X = I.random_complex((ml, mr), ml + mr)
    dL, dRt, dX = _dev(torch, L, prec), _dev(torch, np.ascontiguousarray(R.transpose(1, 2, 0)), prec), _dev(torch, X, prec)
    dY = _dev(torch, np.zeros_like(X), prec)
    T.tdvp_keff_apply(ctx, dL, dRt, dX, dY)
    torch.cuda.synchronize()
    ref = O.keff_apply(L, R, X)
    assert np.abs(_host(dY) - ref).max() / np.abs(ref).max() < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ml,wl,wr,mr", SIZES)
def test_env_updates_match_oracle(env, prec, ml, wl, wr, mr):
    from oracle import tdvp as O
    T, torch, ctx = env
    L, W, R, A = _heff_inputs(ml, wl, wr, mr, 11 * ml + mr)
    dL, dA = _dev(torch, L, prec), _dev(torch, A, prec)
    dLo = _dev(torch, np.zeros((mr, wr, mr)), prec)
    T.tdvp_env_left(ctx, W, dL, dA, dLo)
    dRt = _dev(torch, np.ascontiguousarray(R.transpose(1, 2, 0)), prec)
    dRo = _dev(torch, np.zeros((wl, ml, ml)), prec)
    T.tdvp_env_right(ctx, W, dRt, dA, dRo)
    torch.cuda.synchronize()
    refL = O.left_env_update(L, A, W)
    refR = O.right_env_update(R, A, W).transpose(1, 2, 0)
    assert np.abs(_host(dLo) - refL).max() / np.abs(refL).max() < TOL[prec]
    assert np.abs(_host(dRo) - refR).max() / np.abs(refR).max() < TOL[prec]
