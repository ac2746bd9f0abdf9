"""MPO of c0*1 + c1*H from a term list (oracle; test infrastructure only).

Section I.C, step 1 asks for the MPO of 1 - i tau H; its bond dimension is the
same w as that of H.  The MPO is written as a finite-state automaton read
left to right, with tensors W_i[alpha, beta, s', s] (s' is the output index):

* channel "start" (index 0): nothing placed yet, carries the identity;
* channel "done" (last index): the term is complete, carries the identity;
* open channels: an operator op_i has been placed at a source site i and a
  partner j > current bond is still pending; it carries the identity until a
  partner site, where it emits coef * op_j into "done".

Exact compression: at every bond, open (source, op) items whose whole pending
future (partner sites, partner operators, coefficients) is identical are
merged into one channel, which then carries the sum of their source
operators.  For the one-axis-twisting Hamiltonian this merges all pending
S^z into a single channel and gives w = 3, the value the paper quotes for
eq. (12).  c0 * 1 is placed in the start->done element of site 0 and c1
multiplies every term.
"""
from __future__ import annotations

from collections import OrderedDict

import numpy as np

from .ed import OPS


def _normalise_terms(terms):
    one, two = [], []
    for (i, j, oi, oj, cf) in terms:
        cf = complex(cf)
        if j < 0:
            one.append((i, oi, cf))
        elif i == j:
            raise ValueError("two-site term on one site")
        elif i < j:
            two.append((i, j, oi, oj, cf))
        else:
            two.append((j, i, oj, oi, cf))
    return one, two


def build_mpo(N: int, terms, c0: complex = 0.0, c1: complex = 1.0):
    """Return the list of W_i with shapes (w_{i}, w_{i+1}, 2, 2); w_0 = w_N = 1."""
    one, two = _normalise_terms(terms)
    # item = (source i, op_i); its future = {(j, op_j): coef}
    futures = OrderedDict()
    for (i, j, oi, oj, cf) in two:
        fut = futures.setdefault((i, oi), {})
        fut[(j, oj)] = fut.get((j, oj), 0.0) + cf

    def groups_at_bond(b):
        """Open channels at bond b (between site b and b+1)."""
        groups = OrderedDict()
        for (i, oi), fut in futures.items():
            if i > b:
                continue
            pend = tuple(sorted((j, oj, c) for (j, oj), c in fut.items() if j > b and c != 0))
            if not pend:
                continue
            key = (oi, pend)
            groups.setdefault(key, []).append(i)
        return list(groups.items())

    bond_groups = [groups_at_bond(b) for b in range(N - 1)]
    dims = [1] + [2 + len(g) for g in bond_groups] + [1]

    Ws = []
    for p in range(N):
        wl, wr = dims[p], dims[p + 1]
        W = np.zeros((wl, wr, 2, 2), dtype=np.complex128)
        left_first = p == 0
        right_last = p == N - 1
        l_start = 0
        l_done = wl - 1
        r_start = 0
        r_done = wr - 1
        lg = bond_groups[p - 1] if p > 0 else []
        rg = bond_groups[p] if p < N - 1 else []
        # identity passes
        if not right_last and not left_first:
            W[l_start, r_start] += OPS[0]
        if left_first and not right_last:
            W[0, r_start] += OPS[0]
        if not left_first:
            W[l_done, r_done] += OPS[0]
        # start -> done: one-site terms at p (times c1), c0 on site 0
        onsite = np.zeros((2, 2), dtype=np.complex128)
        for (i, oi, cf) in one:
            if i == p:
                onsite += cf * OPS[oi]
        onsite = c1 * onsite
        if p == 0:
            onsite = onsite + c0 * OPS[0]
        W[l_start, r_done] += onsite
        # start -> open channel at bond p: items whose source is p
        for gi, ((oi, pend), sources) in enumerate(rg):
            if p in sources:
                W[l_start, 1 + gi] += OPS[oi]
        # open channel at bond p-1 -> open channel at bond p (pass identity)
        for gl, ((oi_l, pend_l), src_l) in enumerate(lg):
            still = tuple(t for t in pend_l if t[0] > p)
            if not still:
                continue
            for gr, ((oi_r, pend_r), src_r) in enumerate(rg):
                if oi_r == oi_l and pend_r == still and set(src_l) <= set(src_r):
                    W[1 + gl, 1 + gr] += OPS[0]
                    break
            else:
                raise RuntimeError("channel continuation not found")
        # open channel at bond p-1 -> done at p: emit partner operators
        for gl, ((oi_l, pend_l), src_l) in enumerate(lg):
            for (j, oj, c) in pend_l:
                if j == p:
                    W[1 + gl, r_done] += c1 * c * OPS[oj]
        Ws.append(W)
    return Ws


def bond_dims(Ws):
    return [W.shape[0] for W in Ws] + [Ws[-1].shape[1]]


def mpo_to_dense(Ws) -> np.ndarray:
    """Contract the MPO into a dense 2^N x 2^N matrix (small N only)."""
    acc = Ws[0][0]                    # (beta, out, in)
    for W in Ws[1:]:
        # acc[alpha, O, I], W[alpha, beta, t, s] -> new[beta, O t, I s]
        new = np.einsum("aOI,abts->bOtIs", acc, W)
        b = new.shape[0]
        o = new.shape[1] * new.shape[2]
        acc = new.reshape(b, o, o)
    return acc[0]
