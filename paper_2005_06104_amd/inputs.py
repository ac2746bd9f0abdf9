"""Seeded synthetic workloads for GSE-TDVP1: lattices, coupling lists, initial states.

This module only *describes* inputs.  It contains none of the method's
arithmetic (no MPO construction, no contraction, no factorisation), so both
the CPU oracle and the HIP library consume exactly the same arrays.

Conventions
-----------
* Spin-1/2, local dimension d = 2, basis order {up, down}: index 0 has
  S^z = +1/2 and index 1 has S^z = -1/2.
* Operator codes used in term lists: 0 = identity, 1 = S^+, 2 = S^-, 3 = S^z.
* A term is ``(i, j, op_i, op_j, coef)`` meaning ``coef * op_i(i) op_j(j)``
  for ``i != j``, or ``(i, -1, op_i, 0, coef)`` for the one-site term
  ``coef * op_i(i)``.  Coefficients are complex.
* Site tensors are ``M[a, s, b]`` (left bond, physical, right bond),
  row-major, complex128.

Workloads follow the benchmark systems of the paper: the spin-1/2 Heisenberg
ladder of eq. (11) (rung-decoupled, section II.A and Fig. 1(a)), its
rung-coupled variant (Fig. 1(b)), and the one-axis-twisting model of eq. (12)
(section II.B).  The J1-J2 cylinder and the many-ladder batch are synthetic
workloads of the same kind (Heisenberg couplings mapped to a 1D path).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

OP_I, OP_SP, OP_SM, OP_SZ = 0, 1, 2, 3

Term = Tuple[int, int, int, int, complex]
Coupling = Tuple[int, int, float]


# --------------------------------------------------------------------------
# Lattices mapped to a one-dimensional path (Fig. 1(a) caption: zigzag or
# snake path through a two-leg ladder).
# --------------------------------------------------------------------------

def ladder_index(x: int, r: int, path: str) -> int:
    """Path position of ladder site (column x = 1..L, leg r = 1..2).

    zigzag: every column is visited leg 1 then leg 2, so rungs join path
    neighbours and leg bonds span distance 2.  snake: odd columns are visited
    leg 1 -> 2, even columns leg 2 -> 1, so every odd path bond is a rung and
    leg bonds alternate between distance 3 and 1.
    """
    if path == "zigzag":
        return 2 * (x - 1) + (r - 1)
    if path == "snake":
        return 2 * (x - 1) + ((r - 1) if x % 2 == 1 else (2 - r))
    raise ValueError(f"unknown path {path!r}")


@dataclasses.dataclass
class Lattice:
    n_sites: int
    couplings: List[Coupling]          # (i, j, J) for J S_i . S_j, i < j
    coords: List[Tuple[int, int]]      # lattice coordinates per path position
    name: str = ""

    def neel(self) -> List[int]:
        """Checkerboard Neel state on the lattice: up iff x + y is even."""
        return [0 if (x + y) % 2 == 0 else 1 for (x, y) in self.coords]


def ladder(L: int, J_leg: float = 1.0, J_rung: float = 1.0, path: str = "snake") -> Lattice:
    """Two-leg Heisenberg ladder of leg length L (eq. (11) when J_rung = 0)."""
    n = 2 * L
    coords = [None] * n
    for x in range(1, L + 1):
        for r in (1, 2):
            coords[ladder_index(x, r, path)] = (x, r)
    bonds = []
    for r in (1, 2):
        for x in range(1, L):
            bonds.append((ladder_index(x, r, path), ladder_index(x + 1, r, path), J_leg))
    if J_rung != 0.0:
        for x in range(1, L + 1):
            bonds.append((ladder_index(x, 1, path), ladder_index(x, 2, path), J_rung))
    bonds = [(min(i, j), max(i, j), J) for (i, j, J) in bonds]
    bonds.sort()
    return Lattice(n, bonds, coords, f"ladder{L}_{path}_Jl{J_leg:g}_Jr{J_rung:g}")


def chain(N: int, J: float = 1.0) -> Lattice:
    """Open nearest-neighbour Heisenberg chain."""
    return Lattice(N, [(i, i + 1, J) for i in range(N - 1)], [(i, 0) for i in range(N)], f"chain{N}")


def cylinder(W: int, Lx: int, J1: float = 1.0, J2: float = 0.5) -> Lattice:
    """J1-J2 Heisenberg cylinder, periodic in y (width W), open in x, snake path.

    Column x is ordered y = 1..W when x is odd and y = W..1 when x is even.
    J1 bonds: (x,y)-(x+1,y) and (x,y)-(x,y+1); J2 bonds: (x,y)-(x+1,y+-1).
    """
    def idx(x, y):
        y = (y - 1) % W + 1
        return W * (x - 1) + ((y - 1) if x % 2 == 1 else (W - y))

    n = W * Lx
    coords = [None] * n
    for x in range(1, Lx + 1):
        for y in range(1, W + 1):
            coords[idx(x, y)] = (x, y)
    bonds = {}

    def add(i, j, J):
        if i == j or J == 0.0:
            return
        key = (min(i, j), max(i, j))
        bonds[key] = bonds.get(key, 0.0) + J

    for x in range(1, Lx + 1):
        for y in range(1, W + 1):
            if W > 2 or y < W:
                add(idx(x, y), idx(x, y + 1), J1)
            if x < Lx:
                add(idx(x, y), idx(x + 1, y), J1)
                add(idx(x, y), idx(x + 1, y + 1), J2)
                if W > 2:
                    add(idx(x, y), idx(x + 1, y - 1), J2)
    cpl = sorted((i, j, J) for (i, j), J in bonds.items())
    return Lattice(n, cpl, coords, f"cyl{W}x{Lx}_J2{J2:g}")


# --------------------------------------------------------------------------
# Hamiltonians as term lists
# --------------------------------------------------------------------------

def heisenberg_terms(couplings: Sequence[Coupling]) -> List[Term]:
    """J S_i . S_j = J S^z_i S^z_j + J/2 (S^+_i S^-_j + S^-_i S^+_j)  (eq. (11))."""
    terms: List[Term] = []
    for (i, j, J) in couplings:
        terms.append((i, j, OP_SZ, OP_SZ, complex(J)))
        terms.append((i, j, OP_SP, OP_SM, complex(0.5 * J)))
        terms.append((i, j, OP_SM, OP_SP, complex(0.5 * J)))
    return terms


def oat_terms(N: int, chi: float = 1.0) -> List[Term]:
    """One-axis twisting H = chi (S^z_tot)^2 (eq. (12)) as a term list.

    (sum_i S^z_i)^2 = sum_i (S^z_i)^2 + 2 sum_{i<j} S^z_i S^z_j and
    (S^z_i)^2 = 1/4 for spin 1/2.
    """
    terms: List[Term] = [(i, -1, OP_I, OP_I, complex(0.25 * chi)) for i in range(N)]
    for i in range(N):
        for j in range(i + 1, N):
            terms.append((i, j, OP_SZ, OP_SZ, complex(2.0 * chi)))
    return terms


def spin_moment_terms(N: int, which: str) -> List[Term]:
    """Term lists of the total-spin moments that eqs. (13)-(15) use, for
    measuring them as MPO expectation values: "x", "y", "z" (S^a_tot),
    "yy", "zz" ((S^a_tot)^2) and "yz" (S^y_tot S^z_tot + S^z_tot S^y_tot).
    S^y = (S^+ - S^-) / 2i; (S^a_i)^2 = 1/4 and {S^y_i, S^z_i} = 0 for spin 1/2."""
    one = {"x": [(OP_SP, 0.5), (OP_SM, 0.5)], "y": [(OP_SP, -0.5j), (OP_SM, 0.5j)], "z": [(OP_SZ, 1.0)]}
    if which in one:
        return [(i, -1, op, OP_I, complex(c)) for i in range(N) for op, c in one[which]]
    if which == "zz":
        return oat_terms(N)
    if which == "yy":
        terms: List[Term] = [(i, -1, OP_I, OP_I, complex(0.25)) for i in range(N)]
        pairs = [(OP_SP, OP_SP, -0.25), (OP_SP, OP_SM, 0.25), (OP_SM, OP_SP, 0.25), (OP_SM, OP_SM, -0.25)]
        for i in range(N):
            for j in range(i + 1, N):
                terms += [(i, j, a, b, complex(2.0 * c)) for a, b, c in pairs]
        return terms
    if which == "yz":
        sy = [(OP_SP, -0.5j), (OP_SM, 0.5j)]
        terms = []
        for i in range(N):
            for j in range(i + 1, N):
                for op, c in sy:
                    terms.append((i, j, op, OP_SZ, complex(2.0 * c)))
                    terms.append((i, j, OP_SZ, op, complex(2.0 * c)))
        return terms
    raise ValueError(f"unknown moment {which}")


def terms_as_arrays(terms: Sequence[Term]):
    """Split a term list into the plain arrays the C-ABI takes."""
    ii = np.array([t[0] for t in terms], dtype=np.int32)
    jj = np.array([t[1] for t in terms], dtype=np.int32)
    oi = np.array([t[2] for t in terms], dtype=np.int32)
    oj = np.array([t[3] for t in terms], dtype=np.int32)
    cf = np.array([complex(t[4]) for t in terms], dtype=np.complex128)
    return ii, jj, oi, oj, cf


def energy_scale(couplings: Sequence[Coupling]) -> float:
    """lambda = sum_ij J_ij / 4: the fully polarised energy, exact top of the
    spectrum for antiferromagnetic couplings; used as i*tau = 1/lambda."""
    return float(sum(J for (_, _, J) in couplings)) / 4.0


# --------------------------------------------------------------------------
# Initial states
# --------------------------------------------------------------------------

def product_mps(states: Sequence[int]) -> List[np.ndarray]:
    """Product state with the given local basis indices; bond dimension 1."""
    out = []
    for s in states:
        t = np.zeros((1, 2, 1), dtype=np.complex128)
        t[0, s, 0] = 1.0
        out.append(t)
    return out


def product_charges(states: Sequence[int]) -> List[np.ndarray]:
    """U(1) bond charges of a product state: bond b carries twice the S^z of
    sites 0..b-1 (up = +1, down = -1)."""
    q = [0]
    for s in states:
        q.append(q[-1] + (1 if s == 0 else -1))
    return [np.array([v], dtype=np.int32) for v in q]


def u1_sector_dims(N: int, b: int, chi: int, total: int = 0) -> dict:
    """States per charge at bond b (b sites on the left) of a random U(1) MPS
    with total charge `total`: charge q is possible when both sides can
    carry it; at most min(left count, right count) states, the chi states
    spread in proportion to sqrt(left count * right count) (the weight of a
    typical state), every possible charge getting at least one while chi
    lasts, central charges first."""
    def count(n, q):
        if (n + q) % 2 or abs(q) > n:
            return 0
        return math.comb(n, (n + q) // 2)
    qs = [q for q in range(-b, b + 1, 2) if count(b, q) and count(N - b, total - q)]
    cap = {q: min(count(b, q), count(N - b, total - q)) for q in qs}
    wts = {q: math.sqrt(count(b, q)) * math.sqrt(count(N - b, total - q)) for q in qs}
    if sum(cap.values()) <= chi:
        return dict(sorted(cap.items()))
    order = sorted(qs, key=lambda q: -wts[q])
    dims = {q: 0 for q in qs}
    left = chi
    for q in order:           # one state per charge, most probable first
        if left == 0:
            break
        dims[q] = 1
        left -= 1
    tot_w = sum(wts[q] for q in qs)
    while left > 0:
        grew = False
        for q in order:
            want = max(1, int(round(chi * wts[q] / tot_w)))
            if left > 0 and dims[q] < min(cap[q], want):
                dims[q] += 1
                left -= 1
                grew = True
        if not grew:
            for q in order:
                if left > 0 and dims[q] < cap[q]:
                    dims[q] += 1
                    left -= 1
                    grew = True
            if not grew:
                break
    return {q: d for q, d in sorted(dims.items()) if d > 0}


def random_u1_mps(N: int, chi: int, seed: int, total: int = 0):
    """Random MPS with U(1) charges (total charge `total`): bond sectors from
    u1_sector_dims, entries N(0,1) + i N(0,1) inside the blocks q(b) = q(a) +
    q(s) and zero outside.  Returns (tensors, charges)."""
    rng = np.random.default_rng(seed)
    charges = []
    for b in range(N + 1):
        sec = u1_sector_dims(N, b, chi, total)
        charges.append(np.concatenate([np.full(d, q, dtype=np.int32) for q, d in sec.items()]))
    out = []
    for i in range(N):
        ql, qr = charges[i], charges[i + 1]
        t = rng.standard_normal((len(ql), 2, len(qr))) + 1j * rng.standard_normal((len(ql), 2, len(qr)))
        for s, dq in ((0, 1), (1, -1)):
            t[:, s, :] *= (qr[None, :] == ql[:, None] + dq)
        out.append(t)
    return out, charges


def x_polarized_mps(N: int) -> List[np.ndarray]:
    """All spins along +x: each site (|up> + |down>)/sqrt(2)."""
    t = np.full((1, 2, 1), 1.0 / math.sqrt(2.0), dtype=np.complex128)
    return [t.copy() for _ in range(N)]


def random_bond_dims(N: int, chi: int) -> List[int]:
    """Bond dims min(chi, 2^(i+1), 2^(N-i-1)) for bonds i = 0..N-2."""
    return [int(min(chi, 2 ** min(i + 1, 60), 2 ** min(N - i - 1, 60))) for i in range(N - 1)]


def random_mps(N: int, chi: int, seed: int) -> List[np.ndarray]:
    """Random MPS with i.i.d. N(0,1) + i N(0,1) entries (not normalised)."""
    rng = np.random.default_rng(seed)
    dims = [1] + random_bond_dims(N, chi) + [1]
    out = []
    for i in range(N):
        shape = (dims[i], 2, dims[i + 1])
        out.append(rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
    return out


def random_complex(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def random_hermitian_env(m: int, w: int, seed: int, bra_first: bool = True) -> np.ndarray:
    """Random environment tensor E[x', alpha, x] that is Hermitian in (x', x)
    for every alpha, like a true left/right environment of a Hermitian MPO
    with Hermitian channel operators."""
    e = random_complex((m, w, m), seed)
    return 0.5 * (e + np.conj(np.transpose(e, (2, 1, 0))))


def charged_bond(sectors) -> np.ndarray:
    """Bond charges in ascending order from {charge: number of states}."""
    return np.repeat(np.array(sorted(sectors), dtype=np.int32), [sectors[c] for c in sorted(sectors)])


def random_charged_heff_operands(ql, qr, qwl, qwr, seed: int):
    """Seeded operands of a one-site effective Hamiltonian on charged bonds
    (bond charges ql of a, a'; qr of b, b'; MPO channel charges qwl, qwr;
    physical charge +1 for s = 0, -1 for s = 1): L[a', al, a], R[b', be, b]
    and C[a, s, b] with complex Gaussian entries where the charges allow them
    (L: q(a) = q(a') - qw(al); R: q(b) = q(b') - qw(be); C: q(b) = q(a) + q(s))
    and exact zeros elsewhere."""
    ql, qr, qwl, qwr = (np.asarray(x) for x in (ql, qr, qwl, qwr))
    ps = np.array([1, -1])
    rng = np.random.default_rng(seed)

    def gauss(shape):
        return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)

    L = gauss((len(ql), len(qwl), len(ql)))
    L[ql[None, None, :] != ql[:, None, None] - qwl[None, :, None]] = 0.0
    R = gauss((len(qr), len(qwr), len(qr)))
    R[qr[None, None, :] != qr[:, None, None] - qwr[None, :, None]] = 0.0
    C = gauss((len(ql), 2, len(qr)))
    C[qr[None, None, :] != ql[:, None, None] + ps[None, :, None]] = 0.0
    return L, R, C


def random_mpo_site(wl: int, wr: int, seed: int, density: float = 0.3) -> np.ndarray:
    """Random sparse MPO tensor W[alpha, beta, s', s] (about `density` nonzeros)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((wl, wr, 2, 2)) + 1j * rng.standard_normal((wl, wr, 2, 2))
    mask = rng.random((wl, wr, 2, 2)) < density
    w = w * mask
    if not np.any(w):
        w[0, 0, 0, 0] = 1.0
    return w


# --------------------------------------------------------------------------
# The five workloads (parameters the paper leaves open are readings; each
# is listed with its rationale in the design notes).
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    lattice: Lattice
    init: str                 # "neel", "random", "xpol"
    init_chi: int
    init_seed: int
    dt: complex               # evolves exp(-i H dt); imaginary time uses dt = -i dtau
    n_steps: int
    k: int                    # Krylov order (k-1 global Krylov vectors)
    eps_K: float
    eps_M: float
    eps: float
    chi_max: int
    prec: str                 # "fp64", "fp32", "bf16"
    tau: complex              # MPO is 1 - i tau H
    normalize: bool

    @property
    def terms(self) -> List[Term]:
        if self.name.startswith("oat"):
            return oat_terms(self.lattice.n_sites)
        return heisenberg_terms(self.lattice.couplings)

    def initial_mps(self) -> List[np.ndarray]:
        if self.init == "neel":
            return product_mps(self.lattice.neel())
        if self.init == "xpol":
            return x_polarized_mps(self.lattice.n_sites)
        if self.init == "random":
            return random_mps(self.lattice.n_sites, self.init_chi, self.init_seed)
        raise ValueError(self.init)


def _real_time(name, lat, dt, steps, k, eps_K, eps_M, chi_max, prec, init="neel"):
    return Workload(name, lat, init, 1, 0, complex(dt), steps, k, eps_K, eps_M, 0.0,
                    chi_max, prec, complex(dt), False)


def _imag_time(name, lat, dtau, steps, k, eps_K, eps_M, eps, chi_max, prec, init, chi0=1, seed=0):
    lam = energy_scale(lat.couplings)
    # i*tau = 1/lambda  ->  tau = -i/lambda
    return Workload(name, lat, init, chi0, seed, complex(0.0, -dtau), steps, k, eps_K, eps_M, eps,
                    chi_max, prec, complex(0.0, -1.0 / lam), True)


def workload(idx: int) -> Workload:
    """The benchmark workloads, by index 0..3 (the batch of ladders is `ladder_batch`)."""
    if idx == 0:
        return _real_time("ladder2x6_snake_real", ladder(6, 1.0, 1.0, "snake"), 0.05, 20,
                          2, 1e-10, 1e-10, 32, "fp64")
    if idx == 1:
        return _imag_time("ladder2x32_zigzag_decoupled_imag", ladder(32, 1.0, 0.0, "zigzag"),
                          0.5, 40, 3, 1e-12, 1e-8, 1e-10, 256, "fp64", "random", 16, 2)
    if idx == 2:
        return _real_time("ladder2x64_snake_real", ladder(64, 1.0, 1.0, "snake"), 0.1, 50,
                          3, 1e-4, 1e-8, 512, "fp32")
    if idx == 3:
        return _real_time("cyl4x16_j1j2_real", cylinder(4, 16, 1.0, 0.5), 0.1, 50,
                          3, 1e-4, 1e-8, 1024, "bf16")
    raise IndexError(idx)


def oat_workload(N: int = 100, dt: float = 0.025, k: int = 3, eps_K: float = 1e-4,
                 eps_M: float = 1e-4, t_final: float = 0.25, chi_max: int = 256) -> Workload:
    """One-axis twisting quench from the +x state (section II.B settings)."""
    lat = Lattice(N, [], [(i, 0) for i in range(N)], f"oat{N}")
    steps = int(round(t_final / dt))
    w = Workload(f"oat{N}", lat, "xpol", 1, 0, complex(dt), steps, k, eps_K, eps_M, 0.0,
                 chi_max, "fp64", complex(dt), False)
    return w


def ladder_batch(n: int = 64, seed: int = 5) -> List[Workload]:
    """Independent ladders with leg length U{8..32} and J_leg, J_rung ~ U[0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        L = int(rng.integers(8, 33))
        jl, jr = (float(v) for v in rng.uniform(0.5, 1.5, size=2))
        lat = ladder(L, jl, jr, "snake")
        out.append(_imag_time(f"batch{b}_{lat.name}", lat, 0.2, 30, 3, 1e-12, 1e-8, 1e-10,
                              128, "fp32", "neel"))
    return out
