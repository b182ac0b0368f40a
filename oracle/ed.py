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
