"""Hermitian eigendecomposition on the device (tdvp_eigh): the cooperative
Householder tridiagonalisation with the own tridiagonal divide and conquer
(method 1; rocSOLVER's above n = 512) or rocSOLVER's (method 3), and the rocSOLVER route (2), against the
eigenvalues of numpy's LAPACK eigensolver, orthonormality and reconstruction,
on Gram matrices with decaying spectra, exact multiplets, rank deficiency,
graded spectra, tight clusters, the zero matrix and already-reduced (diagonal /
tridiagonal) inputs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2005_06104_amd import tdvp as T
    ctx = T.Context(0)
    yield T, torch, ctx
    ctx.close()


def _gram(n, seed, decay=12.0):
    rng = np.random.default_rng(seed)
    X = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * np.exp(-decay * np.arange(n) / n)
    return X @ X.conj().T


def _multiplets(n, seed):
    # eigenvalues repeated in multiplets of 1..4 (as the SU(2) multiplets of
    # the Heisenberg models), some exactly zero
    rng = np.random.default_rng(seed)
    lam = []
    v = 1.0
    while len(lam) < n:
        lam += [v] * int(rng.integers(1, 5))
        v *= 0.7
    lam = np.array(lam[:n])
    lam[-max(1, n // 8):] = 0.0
    U, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return (U * lam) @ U.conj().T


def _tridiagonal(n, seed):
    rng = np.random.default_rng(seed)
    H = np.diag(rng.standard_normal(n)).astype(complex)
    off = rng.standard_normal(n - 1) + 1j * rng.standard_normal(n - 1)
    return H + np.diag(off, 1) + np.diag(off.conj(), -1)


def _spectrum(lam, seed):
    n = len(lam)
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return (U * lam) @ U.conj().T


def _graded(n, seed):
    # eigenvalues spread over fifteen decades (the tail of a density matrix)
    return _spectrum(np.logspace(0, -15, n), seed)


def _clusters(n, seed):
    # two tight clusters (relative splittings 1e-10) and their mirror images:
    # deflation by rotation in the tridiagonal divide and conquer
    rng = np.random.default_rng(seed)
    lam = np.concatenate([1.0 + 1e-10 * rng.standard_normal(n // 2), -0.5 + 1e-10 * rng.standard_normal(n - n // 2)])
    return _spectrum(lam, seed + 1)


CASES = {"gram": _gram, "multiplets": _multiplets, "tridiagonal": _tridiagonal,
         "diagonal": lambda n, s: np.diag(np.random.default_rng(s).standard_normal(n)).astype(complex),
         "zero": lambda n, s: np.zeros((n, n), complex), "graded": _graded, "clusters": _clusters}


def _check(T, torch, ctx, H, method):
    n = H.shape[0]
    dH = torch.from_numpy(H).cuda()
    rows = torch.zeros_like(dH)
    lam = T.tdvp_eigh(ctx, dH, rows, method)
    V = rows.cpu().numpy()
    ref = np.linalg.eigvalsh(H)[::-1]
    scale = max(np.abs(ref).max(), 1e-300)
    tol = (1e-14 * n + 1e-13) * scale
    assert np.all(np.diff(lam) <= 0)
    assert np.abs(lam - ref).max() <= tol
    assert np.abs(V @ V.conj().T - np.eye(n)).max() <= 1e-14 * n + 1e-13
    assert np.abs((V.conj().T * lam) @ V - H).max() <= tol


@pytest.mark.parametrize("kind", sorted(CASES))
@pytest.mark.parametrize("n", [2, 3, 17, 32, 33, 64, 100, 255, 256, 301, 512])
@pytest.mark.parametrize("method", [1, 2, 3])
def test_eigh_routes(env, kind, n, method):
    T, torch, ctx = env
    _check(T, torch, ctx, CASES[kind](n, 7 * n + len(kind)), method)


@pytest.mark.parametrize("kind", sorted(CASES))
@pytest.mark.parametrize("n", [513, 700, 1024])
@pytest.mark.parametrize("method", [1, 3])
def test_eigh_routes_large(env, kind, n, method):
    # above 512 the reduction keeps its Q rows in the output (four rows per
    # workgroup, up to 256 workgroups) and the tridiagonal problem goes to
    # rocSOLVER's divide and conquer
    T, torch, ctx = env
    _check(T, torch, ctx, CASES[kind](n, 7 * n + len(kind)), method)


@pytest.mark.parametrize("n", [1, 513, 700, 1025])
def test_eigh_auto_outside_cooperative_range(env, n):
    T, torch, ctx = env
    _check(T, torch, ctx, _gram(n, n), 0)


def test_eigh_cooperative_route_refuses_large(env):
    T, torch, ctx = env
    H = _gram(1025, 1)
    dH = torch.from_numpy(H).cuda()
    with pytest.raises(T.TdvpError):
        T.tdvp_eigh(ctx, dH, torch.zeros_like(dH), 1)


def test_eigh_routes_agree_on_subspaces(env):
    # the two routes give the same eigenvalues and the same spectral
    # projectors onto well-separated groups
    T, torch, ctx = env
    H = _gram(300, 5)
    dH = torch.from_numpy(H).cuda()
    out = []
    for m in (1, 2):
        rows = torch.zeros_like(dH)
        lam = T.tdvp_eigh(ctx, dH, rows, m)
        out.append((lam, rows.cpu().numpy()))
    assert np.abs(out[0][0] - out[1][0]).max() <= 1e-12 * out[0][0][0]
    for k in (10, 50):
        P = [r[:k].conj().T @ r[:k] for _, r in out]
        assert np.abs(P[0] - P[1]).max() < 1e-9


def test_eigh_sectors_many_uneven_blocks(env):
    # block diagonal under scattered index charges: 1 x 1 blocks (three with
    # equal values, whose order follows the charges), more than 16 blocks for
    # the side-by-side divide and conquer (several launches), and one block
    # above 512 (rocSOLVER's tridiagonal route); every spectrum kind above
    T, torch, ctx = env
    sizes = [1, 1, 1, 2, 3, 5, 15, 16, 17, 31, 32, 33, 47, 64, 65, 100, 128, 129, 200, 257, 512, 600]
    kinds = sorted(CASES)
    rng = np.random.default_rng(77)
    n = sum(sizes)
    charge_of_block = 2 * np.arange(len(sizes)) - len(sizes)
    q = np.repeat(charge_of_block, sizes)[rng.permutation(n)]
    H = np.zeros((n, n), complex)
    ref = []
    for b, (c, m) in enumerate(zip(charge_of_block, sizes)):
        idx = np.flatnonzero(q == c)
        B = CASES[kinds[b % len(kinds)]](m, 500 + b) if m > 1 else np.array([[0.25 + 0j]])
        H[np.ix_(idx, idx)] = B
        ref.append(np.linalg.eigvalsh(B))
    ref = np.sort(np.concatenate(ref))[::-1]
    dH = torch.from_numpy(H).cuda()
    rows = torch.zeros_like(dH)
    lam, qo = T.tdvp_eigh_sectors(ctx, dH, q, rows)
    V = rows.cpu().numpy()
    scale = np.abs(ref).max()
    tol = (1e-14 * max(sizes) + 1e-13) * scale
    assert np.all(np.diff(lam) <= 0)
    assert np.abs(lam - ref).max() <= tol
    # each eigenvector lies in the block of its charge, exactly
    for c, m in zip(charge_of_block, sizes):
        assert int((qo == c).sum()) == m
    assert np.all(V[q[None, :] != qo[:, None]] == 0)
    # equal eigenvalues of different charges: lower charge first
    tie = np.flatnonzero(lam == 0.25)
    assert len(tie) >= 3 and np.all(np.diff(qo[tie]) > 0)
    assert np.abs(V @ V.conj().T - np.eye(n)).max() <= 1e-14 * max(sizes) + 1e-13
    assert np.abs((V.conj().T * lam) @ V - H).max() <= tol
