"""Matrix-product operators built one channel per open operator string.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The textbook construction: at the bond between chain sites k and k+1 the
channels are
    'I'  nothing placed yet (identity so far),
    one channel per operator string whose first site is <= k and whose last
         site is > k (the string is 'open' across the bond),
    'F'  a complete string has been placed (identity from here on).
W_k[cl, cr] is the d x d operator that moves channel cl to channel cr at
site k.  This is deliberately the plainest correct form; its bond dimension is
larger than a compressed automaton's, which does not change the operator.

W arrays are complex [w_left, w_right, d_out, d_in]; the operator acts on the
physical (P) leg of the purified state only.
"""
from __future__ import annotations

import numpy as np

from . import model as M


def build_mpo(model, terms):
    """MPO (list of W arrays) of sum_t coef_t prod_s op_{t,s}."""
    dims = M.site_dims(model)
    L = len(dims)
    starts = [min(s for s, _ in ops) for _, ops in terms]
    ends = [max(s for s, _ in ops) for _, ops in terms]

    def channels(k):
        """Channel labels of the bond to the right of site k."""
        if k < 0:
            return ["I"]
        if k >= L - 1:
            return ["F"]
        open_ = [t for t in range(len(terms)) if starts[t] <= k < ends[t]]
        return ["I"] + open_ + ["F"]

    Ws = []
    for k in range(L):
        d = dims[k]
        cl, cr = channels(k - 1), channels(k)
        W = np.zeros((len(cl), len(cr), d, d), dtype=complex)
        il = {c: i for i, c in enumerate(cl)}
        ir = {c: i for i, c in enumerate(cr)}
        eye = np.eye(d)
        if "I" in il and "I" in ir:
            W[il["I"], ir["I"]] += eye
        if "F" in il and "F" in ir:
            W[il["F"], ir["F"]] += eye
        for t, (coef, ops) in enumerate(terms):
            here = dict(ops)
            op = M.local_op(model, k, here[k]) if k in here else eye
            s0, s1 = starts[t], ends[t]
            if s0 == k == s1:                       # single-site string
                W[il["I"], ir["F"]] += coef * op
            elif s0 == k:                           # string opens here
                W[il["I"], ir[t]] += coef * op
            elif s0 < k < s1:                       # passes through
                W[il[t], ir[t]] += op
            elif k == s1 and s0 < k:                # string closes here
                W[il[t], ir["F"]] += op
        Ws.append(W)
    return Ws


def hamiltonian_mpo(model):
    return build_mpo(model, M.hamiltonian_terms(model))


def current_mpo(model):
    return build_mpo(model, M.current_terms(model))


def hop_mpo(model, i, j):
    """MPO of c+_j c_i (moves the carrier from molecule i to molecule j; the
    number operator n_i when i == j).  With one carrier the hard-core string
    between the two sites is +1."""
    idx = M.index_of(model)
    ei, ej = idx[("e", i, -1)], idx[("e", j, -1)]
    if i == j:
        return build_mpo(model, [(1.0, [(ei, "n")])])
    return build_mpo(model, [(1.0, [(ej, "sp"), (ei, "sm")])])


def densify(Ws):
    """Dense matrix of an MPO on the full product space (tiny chains only)."""
    T = Ws[0][0]                      # [wr, d, d]
    for W in Ws[1:]:
        # T[c, P, p] (x) W[c, c', P2, p2] -> [c', (P P2), (p p2)]
        wr = W.shape[1]
        T = np.einsum("cPp,cCQq->CPQpq", T, W)
        n = T.shape[1] * T.shape[2]
        T = T.reshape(wr, n, n)
    return T[0]
