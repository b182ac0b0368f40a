"""Exact diagonalisation of the truncated one-carrier problem.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Basis |n> (x) |v_1 ... v_M>: carrier on molecule n, every mode of the chain in
number state v (chain order, last mode fastest), each truncated to `levels`
states.  H and j are written directly from Eq. (1), the Peierls term and the
current operator; they do not reuse the operator strings of model.py, so the
MPO builders can be checked against them.

Observables (purification section of the paper):
  rho_beta = exp(-beta H) / Z,  Z = Tr exp(-beta H) over the one-carrier space
  C(t) = Tr[rho_beta exp(iHt) j exp(-iHt) j]
       = sum_ab w_a exp(i(E_a - E_b) t) |j_ab|^2,  w_a = exp(-beta E_a)/Z
in the eigenbasis of H.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import model as M


def _mode_list(model):
    """Modes in chain order: (kind, molecule, mode, omega, levels)."""
    out = []
    for kind, n, m in M.site_list(model):
        if kind == "loc":
            out.append((kind, n, m, model.omega_loc[m], model.levels_loc))
        elif kind == "nl":
            out.append((kind, n, m, model.omega_nl[m], model.levels_nl))
    return out


def _embed(op, k, dims):
    """Operator `op` on mode k of the phonon product space (sparse)."""
    mats = [sp.identity(d, format="csr") for d in dims]
    mats[k] = sp.csr_matrix(op)
    out = sp.identity(1, format="csr")
    for m in mats:
        out = sp.kron(out, m, format="csr")
    return out


def build(model):
    """Return (H, K, dim) with H real symmetric and j = (e0 R / i) K,
    K real antisymmetric, both dense, in the one-carrier basis."""
    modes = _mode_list(model)
    dims = [lv for *_, lv in modes]
    nph = int(np.prod(dims)) if dims else 1
    N = model.n_mol

    def ladder(lv):
        b = np.diag(np.sqrt(np.arange(1, lv, dtype=float)), 1)
        return b

    X, NB = [], []
    for k, (_, _, _, w, lv) in enumerate(modes):
        b = ladder(lv)
        X.append(_embed(b + b.T, k, dims))
        NB.append(_embed(b.T @ b, k, dims))

    Hph = sp.csr_matrix((nph, nph))
    for k, (_, _, _, w, _) in enumerate(modes):
        Hph = Hph + w * NB[k]

    # local (Holstein) phonon displacement felt by a carrier on molecule n
    onsite = []
    for n in range(N):
        A = sp.csr_matrix((nph, nph))
        for k, (kind, mol, m, w, _) in enumerate(modes):
            if kind == "loc" and mol == n:
                A = A + model.g_loc[m] * w * X[k]
        onsite.append(A)

    # transfer factor of bond (n, n+1): V + sum_m g2_m w_m x_{n,m}
    bonds = [(n, n + 1) for n in range(N - 1)]
    if model.periodic:
        bonds.append((N - 1, 0))
    factor = {}
    for n, n2 in bonds:
        F = model.V * sp.identity(nph, format="csr")
        for k, (kind, mol, m, w, _) in enumerate(modes):
            if kind == "nl" and mol == n:
                F = F + model.g_nl[m] * w * X[k]
        factor[(n, n2)] = F

    dim = N * nph
    Hd = np.zeros((dim, dim))
    Kd = np.zeros((dim, dim))
    for n in range(N):
        blk = (Hph + onsite[n]).toarray()
        Hd[n * nph:(n + 1) * nph, n * nph:(n + 1) * nph] += blk
    for (n, n2), F in factor.items():
        Fd = F.toarray()
        # c+_{n2} c_n : carrier n -> n2 ; matrix element <n2|..|n>
        Hd[n2 * nph:(n2 + 1) * nph, n * nph:(n + 1) * nph] += Fd
        Hd[n * nph:(n + 1) * nph, n2 * nph:(n2 + 1) * nph] += Fd
        Kd[n2 * nph:(n2 + 1) * nph, n * nph:(n + 1) * nph] += Fd
        Kd[n * nph:(n + 1) * nph, n2 * nph:(n2 + 1) * nph] -= Fd
    return Hd, Kd, dim


class EDResult:
    def __init__(self, model, beta):
        self.model = model
        self.beta = beta
        H, K, dim = build(model)
        self.H = H
        self.j = (model.e0 * model.R / 1j) * K
        E, U = np.linalg.eigh(H)
        self.E = E
        self.U = U
        Kt = U.T @ K @ U
        self.J2 = (model.e0 * model.R) ** 2 * Kt * Kt   # |j_ab|^2
        x = -beta * (E - E[0])
        self.w = np.exp(x) / np.exp(x).sum()
        self.logZ = -beta * E[0] + np.log(np.exp(x).sum())
        self.dim = dim

    def corr(self, times):
        """C(t) at the given times (complex array)."""
        times = np.asarray(times, dtype=float)
        ph_b = np.exp(-1j * np.outer(self.E, times))          # [b, t]
        inner = self.J2 @ ph_b                                # [a, t]
        ph_a = np.exp(1j * np.outer(self.E, times))          # [a, t]
        return np.einsum("a,at,at->t", self.w, ph_a, inner)

    def energy(self):
        return float(self.w @ self.E)

    def reduced_density(self):
        """sigma = Tr_ph rho_beta (N x N): sigma_ij = sum_v rho[(i v), (j v)]
        = Tr[rho c+_j c_i] (the coherent-length passage)."""
        N = self.model.n_mol
        nph = self.dim // N
        rho = (self.U * self.w) @ self.U.T
        return np.einsum("ivjv->ij", rho.reshape(N, nph, N, nph))

    def density_expectation(self):
        """<c+_n c_n> in the thermal state, per molecule."""
        N = self.model.n_mol
        nph = self.dim // N
        diag = np.einsum("ia,a,ia->i", self.U, self.w, self.U)
        return diag.reshape(N, nph).sum(axis=1)


def thermal_state_vector(ed, beta):
    """exp(-beta H / 2) applied to the purified identity, as the dense matrix
    M = exp(-beta H/2) (P index rows, Q index columns).  Tests only."""
    return (ed.U * np.exp(-0.5 * beta * ed.E)) @ ed.U.T


# ------------------------------------------------------ exact mobility gradient
# Derivative of the Kubo mobility of the truncated model with respect to the
# shared mode parameters, exactly (no finite differences, no TDVP): mu is
# (beta / e0) times the trapezoid sum of Re C(t_k) on the run grid (the
# mobility passage, Eq. (kubo)), C(t) = Tr[e^{-beta H} e^{iHt} j e^{-iHt} j] /
# Z.  H and K (j = (e0 R / i) K) are affine in each omega and each g at fixed
# other parameters, so dH/dx and dK/dx are exact differences of two builds.
# The derivative of a function f(H) along A is, in the eigenbasis of H,
# Gamma_f o (U^T A U) with Gamma_f[a, b] the divided difference
# (f(E_a) - f(E_b)) / (E_a - E_b) (f'(E_a) where E_a = E_b): the
# Daleckii-Krein formula, here for f = exp(s E), s = -beta and -+ i t.


def _divided_exp(E, s):
    """Gamma[a, b] = (exp(s E_a) - exp(s E_b)) / (E_a - E_b), s exp(s E_a)
    where E_a == E_b; expm1 keeps nearly equal energies accurate."""
    d = E[:, None] - E[None, :]
    eb = np.exp(s * E)[None, :]
    safe = np.where(d == 0.0, 1.0, d)
    G = eb * np.expm1(s * d) / safe
    return np.where(d == 0.0, s * np.exp(s * E)[:, None] * np.ones_like(d), G)


def _parameter_directions(model):
    """[(name, index, dH, dK)] for every shared mode parameter: the exact
    change of the dense H and K per unit change of that parameter."""
    import dataclasses
    H0, K0, _ = build(model)
    out = []
    for name in ("omega_loc", "g_loc", "omega_nl", "g_nl"):
        vals = list(getattr(model, name))
        for i in range(len(vals)):
            up = dataclasses.replace(model, **{name: vals[:i] + [vals[i] + 1.0] + vals[i + 1:]})
            H1, K1, _ = build(up)
            out.append((name, i, H1 - H0, K1 - K0))
    return out


def mobility_gradient(model, beta, dt, n_steps):
    """Exact mu (a.u.) on the grid t_k = k dt, k = 0..n_steps (trapezoid), and
    {"omega_loc", "g_loc", "omega_nl", "g_nl"} -> arrays of d mu / d x."""
    H, K, _ = build(model)
    E, U = np.linalg.eigh(H)
    E = E - E[0]                       # a shift of H changes no C(t)
    c = model.e0 * model.R / 1j        # j = c K
    Kt = U.T @ K @ U
    p = np.exp(-beta * E)
    Z = p.sum()
    times = np.arange(n_steps + 1) * dt
    wq = np.full(n_steps + 1, dt)
    wq[0] = wq[-1] = 0.5 * dt
    Gb = _divided_exp(E, -beta)
    # per time: V = exp(-iHt), its divided differences, C(t)
    per_t = []
    C = np.zeros(n_steps + 1, dtype=complex)
    for k, t in enumerate(times):
        v = np.exp(-1j * E * t)
        jt = c * Kt
        # G(t) = Tr[P V^H j V j] in the eigenbasis (P, V diagonal)
        M = (np.conj(v)[:, None] * jt) * v[None, :]           # V^H j V
        G = np.sum(p[:, None] * M * jt.T)                      # Tr[P M j]
        C[k] = G / Z
        per_t.append((v, jt, M, _divided_exp(E, -1j * t), _divided_exp(E, 1j * t)))
    mu = beta / model.e0 * float(np.sum(wq * C.real))
    grads = {"omega_loc": [], "g_loc": [], "omega_nl": [], "g_nl": []}
    for name, i, dH, dK in _parameter_directions(model):
        At = U.T @ dH @ U
        dj = c * (U.T @ dK @ U)
        dP = Gb * At                                           # d exp(-beta H)
        dZ = float(np.trace(dP).real)
        dmu = 0.0
        for k, (v, jt, M, Gm, Gp) in enumerate(per_t):
            dV = Gm * At                                       # d exp(-iHt)
            dVh = Gp * At                                      # d exp(+iHt)
            Pm = p[:, None]
            Vh = np.conj(v)
            # the five terms of d Tr[P V^H j V j]
            dG = np.trace(dP @ (M @ jt))
            dG += np.trace(Pm * ((dVh @ jt) * v[None, :]) @ jt)
            dG += np.trace(Pm * (Vh[:, None] * (jt @ dV)) @ jt)
            dG += np.trace(Pm * ((Vh[:, None] * dj) * v[None, :]) @ jt)
            dG += np.trace(Pm * M @ dj)
            dC = (dG - C[k] * dZ) / Z
            dmu += wq[k] * dC.real
        grads[name].append(beta / model.e0 * dmu)
    return mu, {k: np.array(v) for k, v in grads.items()}
