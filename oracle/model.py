"""Chain layout and operator strings of the (Holstein-)Peierls model.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Hamiltonian, Eq. (1) of the paper:
  H_e    = V sum_n (c+_{n+1} c_n + c+_n c_{n+1})
  H_ph   = sum_{n,m} omega_m b+_{n,m} b_{n,m}
  H_e-ph = sum_{n,m} g_m omega_m (b+_{n,m} + b_{n,m}) c+_n c_n
plus, for the Holstein-Peierls model of the closing section, one set of
bond modes per bond (n, n+1) with
  sum_{n,m} g2_m omega_m (b+ + b)_{n,m} (c+_n c_{n+1} + c+_{n+1} c_n).
Current (the operator written under the Kubo formula):
  j = (e0 R / i) sum_n (V + sum_m g2_m omega_m x_{n,m}) (c+_{n+1} c_n - c+_n c_{n+1})
which reduces to the printed Holstein current when g2 = 0 and equals
i[H, e0 R sum_n n c+_n c_n] for the open chain.

Readings where the paper is silent:
  * one carrier; hard-core electron site with basis |0> (empty), |1>
    (occupied).  With a single carrier the Jordan-Wigner string is +1, also on
    the periodic wrap bond, so c+_{n'} c_n = sigma+_{n'} sigma-_n exactly.
  * chain order: e_0, its local modes, the bond modes of bond (0,1), e_1, ...;
    the bond modes of the wrap bond (N-1, 0) come after molecule N-1.
  * each mode keeps `levels` number states, b|v> = sqrt(v)|v-1>.
"""
from __future__ import annotations

import numpy as np


def site_list(model):
    """[(kind, molecule, mode)] in chain order; kind in {'e','loc','nl'}."""
    out = []
    N = model.n_mol
    for n in range(N):
        out.append(("e", n, -1))
        for m in range(model.n_loc):
            out.append(("loc", n, m))
        if model.periodic or n < N - 1:
            for m in range(model.n_nl):
                out.append(("nl", n, m))
    return out


def site_dims(model):
    dims = []
    for kind, _, _ in site_list(model):
        if kind == "e":
            dims.append(2)
        elif kind == "loc":
            dims.append(model.levels_loc)
        else:
            dims.append(model.levels_nl)
    return dims


def index_of(model):
    """Map (kind, molecule, mode) -> chain position."""
    return {s: i for i, s in enumerate(site_list(model))}


def boson_ops(levels):
    b = np.zeros((levels, levels))
    for v in range(1, levels):
        b[v - 1, v] = np.sqrt(v)
    bd = b.T.copy()
    return {"1": np.eye(levels), "b": b, "bd": bd, "nb": bd @ b, "x": b + bd}


def electron_ops():
    # basis |0> empty, |1> occupied
    sp = np.array([[0.0, 0.0], [1.0, 0.0]])   # |1><0|
    sm = sp.T.copy()                          # |0><1|
    return {"1": np.eye(2), "sp": sp, "sm": sm, "n": np.diag([0.0, 1.0])}


def local_op(model, site, name):
    kind = site_list(model)[site][0]
    if kind == "e":
        return electron_ops()[name]
    lv = model.levels_loc if kind == "loc" else model.levels_nl
    return boson_ops(lv)[name]


def _bonds(model):
    N = model.n_mol
    out = [(n, n + 1) for n in range(N - 1)]
    if model.periodic:
        out.append((N - 1, 0))
    return out


def _hop_terms(model, fwd, bwd):
    """Hopping-type strings with site factors (V + sum_m g2_m w_m x_m).

    fwd multiplies c+_{n'} c_n (carrier moves n -> n'), bwd multiplies
    c+_n c_{n'}.  Returns [(coef, [(site, op), ...])] sorted by site."""
    idx = index_of(model)
    terms = []
    for n, n2 in _bonds(model):
        en, en2 = idx[("e", n, -1)], idx[("e", n2, -1)]
        factors = [(model.V, None)]
        for m in range(model.n_nl):
            factors.append((model.g_nl[m] * model.omega_nl[m], idx[("nl", n, m)]))
        for amp, xs in factors:
            for c, opn, opn2 in ((fwd, "sm", "sp"), (bwd, "sp", "sm")):
                ops = [(en, opn), (en2, opn2)]
                if xs is not None:
                    ops.append((xs, "x"))
                terms.append((c * amp, sorted(ops)))
    return terms


def hamiltonian_terms(model):
    """H of Eq. (1) (+ Peierls) as [(coef, [(site, opname), ...])]."""
    idx = index_of(model)
    terms = []
    for (kind, n, m), s in idx.items():
        if kind == "loc":
            terms.append((model.omega_loc[m], [(s, "nb")]))
        elif kind == "nl":
            terms.append((model.omega_nl[m], [(s, "nb")]))
    for n in range(model.n_mol):
        for m in range(model.n_loc):
            c = model.g_loc[m] * model.omega_loc[m]
            terms.append((c, [(idx[("e", n, -1)], "n"), (idx[("loc", n, m)], "x")]))
    terms += _hop_terms(model, 1.0, 1.0)
    return terms


def current_terms(model):
    """j = (e0 R / i) sum (V + Peierls) (c+_{n+1} c_n - c+_n c_{n+1})."""
    a = model.e0 * model.R / 1j
    return _hop_terms(model, a, -a)


def dense_term(model, coef, ops):
    """Dense matrix of one operator string on the full (unrestricted) space.
    Only for tiny chains (tests)."""
    dims = site_dims(model)
    by_site = dict(ops)
    mat = np.array([[1.0 + 0j]])
    for s, d in enumerate(dims):
        o = local_op(model, s, by_site[s]) if s in by_site else np.eye(d)
        mat = np.kron(mat, o)
    return coef * mat


def one_carrier_basis(model):
    """Indices (into the full product space, site order, last site fastest)
    of the states with exactly one occupied electronic site, ordered by carrier
    position n, then phonon occupations in chain order (last fastest)."""
    dims = site_dims(model)
    sl = site_list(model)
    e_sites = [i for i, s in enumerate(sl) if s[0] == "e"]
    ph_sites = [i for i, s in enumerate(sl) if s[0] != "e"]
    strides = np.ones(len(dims), dtype=np.int64)
    for i in range(len(dims) - 2, -1, -1):
        strides[i] = strides[i + 1] * dims[i + 1]
    ph_dims = [dims[i] for i in ph_sites]
    out = []
    for n, es in enumerate(e_sites):
        for occ in np.ndindex(*ph_dims) if ph_dims else [()]:
            k = strides[es]
            for s, v in zip(ph_sites, occ):
                k += strides[s] * v
            out.append(int(k))
    return np.array(out, dtype=np.int64)
