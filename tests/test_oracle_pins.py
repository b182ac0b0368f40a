"""Pins of the CPU oracle against things other than itself: closed forms,
exact diagonalisation, exactness properties of the integrator, conservation
laws and library routines.  CPU only."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

from helpers import small_model
from oracle import analysis as An
from oracle import ed as ED
from oracle import model as Mdl
from oracle import mpo as OM
from oracle import tdvp as T
from paper_2003_13245_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


# ---------------------------------------------------------------- operators
@pytest.mark.parametrize("n_mol,n_loc,n_nl,periodic", [(3, 1, 0, 1), (4, 1, 0, 1), (3, 1, 1, 1),
                                                       (3, 0, 2, 1), (3, 1, 1, 0), (4, 0, 1, 0)])
def test_mpo_densifies_to_ed_matrices(n_mol, n_loc, n_nl, periodic):
    """The MPOs of H and j, densified and restricted to the one-carrier space,
    equal the matrices written directly from Eq. (1), the Peierls term and the
    current operator."""
    m = small_model(n_mol=n_mol, n_loc=n_loc, n_nl=n_nl, levels=2, periodic=periodic)
    idx = Mdl.one_carrier_basis(m)
    H, K, _ = ED.build(m)
    Hd = OM.densify(OM.hamiltonian_mpo(m))
    Jd = OM.densify(OM.current_mpo(m))
    assert np.abs(Hd[np.ix_(idx, idx)] - H).max() < 1e-14
    assert np.abs(Jd[np.ix_(idx, idx)] - (m.e0 * m.R / 1j) * K).max() < 1e-14
    # H conserves the carrier number: no matrix elements leave the sector
    mask = np.ones(Hd.shape[0], bool)
    mask[idx] = False
    assert np.abs(Hd[np.ix_(mask, idx)]).max() < 1e-14


def test_current_is_commutator_with_position_open_chain():
    """For the open chain j = i [H, e0 R sum_n n c+_n c_n] (the Peierls factor
    included), which fixes the sign and the factor of the current."""
    m = small_model(n_mol=4, n_loc=1, n_nl=1, levels=2, periodic=0)
    H, K, dim = ED.build(m)
    nph = dim // m.n_mol
    X = np.kron(np.diag(np.arange(m.n_mol, dtype=float)), np.eye(nph)) * m.e0 * m.R
    j = (m.e0 * m.R / 1j) * K
    assert np.abs(1j * (H @ X - X @ H) - j).max() < 1e-13


def test_identity_state_is_purified_identity():
    m = small_model(n_mol=3, n_loc=1, n_nl=0, levels=2)
    psi = T.identity_mps(m)
    v = T.to_dense(psi)
    dims = Mdl.site_dims(m)
    L = len(dims)
    # interleaved (p1 q1 p2 q2 ...) -> (P, Q) matrix
    t = v.reshape([d for d in dims for _ in range(2)])
    t = np.transpose(t, list(range(0, 2 * L, 2)) + list(range(1, 2 * L, 2)))
    n = int(np.prod(dims))
    M = t.reshape(n, n)
    idx = Mdl.one_carrier_basis(m)
    ref = np.zeros((n, n))
    ref[idx, idx] = 1.0
    assert np.abs(M - ref).max() < 1e-13
    assert abs(2 * psi.log_norm - math.log(len(idx))) < 1e-13


# ---------------------------------------------------------------- ED pins
def test_tight_binding_closed_form():
    """g = 0: j commutes with H, C(t) = <j^2> = 4/(1 + cosh 2) for N = 4,
    V = beta = 1, at every t, real."""
    m = W.Model(n_mol=4, periodic=1, omega_loc=[1.0], g_loc=[0.0], omega_nl=[], g_nl=[],
                levels_loc=3, levels_nl=1, V=1.0)
    r = ED.EDResult(m, 1.0)
    C = r.corr(np.linspace(0, 20, 41))
    ref = GOLD["tight_binding_N4_V1_beta1"]["value"]
    assert abs(ref - 4 / (1 + math.cosh(2))) < 1e-15
    assert np.abs(C - ref).max() < 1e-12
    assert abs(An.tight_binding_corr(4, 1.0, 1.0) - ref) < 1e-14
    # Z factorises: electrons x truncated oscillators
    k = 2 * np.pi * np.arange(4) / 4
    z_e = np.exp(-2 * np.cos(k)).sum()
    z_ph = sum(math.exp(-v) for v in range(3)) ** 4
    assert abs(r.logZ - math.log(z_e * z_ph)) < 1e-12


def test_ed_c0_and_time_reversal():
    m = small_model(n_mol=3, n_loc=1, n_nl=1, levels=3)
    r = ED.EDResult(m, 0.8)
    t = np.linspace(0, 7, 15)
    C = r.corr(t)
    Cm = r.corr(-t)
    assert np.abs(Cm - C.conj()).max() < 1e-12
    rho = (r.U * r.w) @ r.U.T
    assert abs(C[0] - np.trace(rho @ r.j @ r.j)) < 1e-12
    assert abs(C[0].imag) < 1e-13 and C[0].real > 0
    # beta = 0: C(0) = 2 (e0 V R)^2 + Peierls fluctuation (Holstein only here)
    mh = small_model(n_mol=4, n_loc=1, n_nl=0, levels=3)
    r0 = ED.EDResult(mh, 0.0)
    assert abs(r0.corr([0.0])[0] - 2 * (mh.e0 * mh.V * mh.R) ** 2) < 1e-12


def test_ed_thermal_density_is_uniform():
    m = small_model(n_mol=4, n_loc=1, n_nl=0, levels=3)
    r = ED.EDResult(m, 1.3)
    assert np.abs(r.density_expectation() - 0.25).max() < 1e-12


def test_fermi_golden_rule_limit():
    """V -> 0: C(t)/V^2 approaches the hopping-limit closed form (derived
    reading of the printed formula, see oracle.analysis.fgr_corr).  The first
    correction is linear in V; a wrong sign of Im C, a missing factor 2 or a
    missing g^2 doubling gives an O(1) mismatch."""
    w, g, beta = 1.0, 0.5, 1.0
    t = np.linspace(0, 12, 25)
    errs, conj_errs = [], []
    for V in (1e-2, 1e-3):
        m = W.Model(n_mol=3, periodic=1, omega_loc=[w], g_loc=[g], omega_nl=[], g_nl=[],
                    levels_loc=12, levels_nl=1, V=V)
        C = ED.EDResult(m, beta).corr(t) / V ** 2
        F = An.fgr_corr(t, V, [w], [g], beta) / V ** 2
        errs.append(np.abs(C - F).max() / np.abs(F).max())
        conj_errs.append(np.abs(C - F.conj()).max() / np.abs(F).max())
    assert errs[1] < 2e-3
    assert errs[1] < errs[0] / 5
    assert min(conj_errs) > 0.3          # the printed (conjugate) time dependence


# ------------------------------------------------------------- oracle algebra
def test_qr_and_lq_conventions():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((9, 4)) + 1j * rng.standard_normal((9, 4))
    Q, R = T.qr_pos(M)
    assert np.allclose(Q @ R, M, atol=1e-14)
    assert np.allclose(Q.conj().T @ Q, np.eye(4), atol=1e-14)
    assert np.all(np.abs(np.diag(R).imag) < 1e-15) and np.all(np.diag(R).real >= 0)
    assert np.allclose(np.tril(R, -1), 0)
    L, Qr = T.lq_pos(M.T)
    assert np.allclose(L @ Qr, M.T, atol=1e-14)
    assert np.allclose(Qr @ Qr.conj().T, np.eye(4), atol=1e-14)
    assert np.all(np.diag(L).real >= 0) and np.allclose(np.triu(L, 1), 0)


@pytest.mark.parametrize("z", [-0.3j, -0.7, 0.25 + 0.1j])
def test_krylov_expm_matches_dense_expm(z):
    rng = np.random.default_rng(1)
    A = rng.standard_normal((60, 60)) + 1j * rng.standard_normal((60, 60))
    H = (A + A.conj().T) / 4
    v = rng.standard_normal(60) + 1j * rng.standard_normal(60)
    y, m = T.expm_krylov(lambda x: H @ x, v, z, tol=1e-14, mmax=60)
    ref = sla.expm(z * H) @ v
    assert np.abs(y - ref).max() / np.abs(ref).max() < 1e-12
    assert m < 60


def test_krylov_exhausted_space_is_exact():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((5, 5))
    H = A + A.T
    v = rng.standard_normal(5).astype(complex)
    y, m = T.expm_krylov(lambda x: H @ x, v, -2.0j, tol=1e-30, mmax=40)
    assert m == 5
    assert np.abs(y - sla.expm(-2.0j * H) @ v).max() < 1e-12


def test_truncation_rule_keeps_multiplets_whole():
    s = np.array([1.0, 0.5, 0.5 * (1 - 1e-12), 0.2, 1e-12])
    assert T.truncation_rank(s, 2, 1e-10) == 1
    assert T.truncation_rank(s, 3, 1e-10) == 3
    assert T.truncation_rank(s, 10, 1e-10) == 4
    assert T.truncation_rank(np.array([0.0, 0.0]), 4, 1e-10) == 1


def test_compress_without_truncation_is_exact():
    m = small_model(n_mol=3, n_loc=1, n_nl=0, levels=2)
    Jw = OM.current_mpo(m)
    psi = T.identity_mps(m)
    X = T.apply_mpo(Jw, psi)
    Y = T.compress(X, 10 ** 6, 0.0)
    assert np.abs(T.to_dense(Y) - T.to_dense(X)).max() < 1e-13


def _schmidt_state(rng, s, dims, cut):
    """Dense purified vector sum_i s_i |L_i>|R_i> with orthonormal L_i on
    sites < cut and R_i on sites >= cut (random unitaries), as an exact MPS
    whose every bond is then put in a random non-canonical gauge (A_i G,
    G^-1 A_{i+1}), so nothing about the tensors is orthonormal."""
    nl = int(np.prod([d * d for d in dims[:cut]]))
    nr = int(np.prod([d * d for d in dims[cut:]]))

    def unitary(n):
        q, r = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]

    U, V = unitary(nl), unitary(nr)
    k = len(s)
    vec = (U[:, :k] * s[None, :]) @ V[:, :k].T
    psi = T.full_rank_mps(vec.reshape(-1), dims)
    for i in range(len(dims) - 1):
        b = psi.A[i].shape[3]
        G = np.eye(b) + 0.5 * (rng.standard_normal((b, b)) + 1j * rng.standard_normal((b, b)))
        psi.A[i] = np.tensordot(psi.A[i], G, axes=([3], [0]))
        psi.A[i + 1] = np.tensordot(np.linalg.inv(G), psi.A[i + 1], axes=([1], [0]))
    return vec.reshape(-1), psi


@pytest.mark.parametrize("k", [4, 6, 11])
def test_truncated_compression_is_eckart_young_optimal(k):
    """Truncating one Schmidt cut of a state with known Schmidt values s_i to
    k values is, by the Eckart-Young theorem, the best rank-k approximation:
    the residual is ||psi - psi_k||^2 = sum_{i>k} s_i^2 and the overlap
    <psi|psi_k> = |psi_k|^2 = sum_{i<=k} s_i^2, whatever gauge the input
    tensors are in.  Four sites of d = 2 (bonds 4, 16, 4); the middle cut
    carries 16 distinct Schmidt values and is the only bond truncated (the
    outer bonds have rank 4 <= k)."""
    rng = np.random.default_rng(17)
    dims = [2, 2, 2, 2]
    s = np.sort(np.exp(-0.45 * np.arange(16)) * (1 + 0.05 * rng.uniform(size=16)))[::-1]
    s = s / np.linalg.norm(s)
    v, psi = _schmidt_state(rng, s, dims, 2)
    assert np.abs(T.to_dense(psi) - v).max() < 1e-12
    out = T.compress(psi, k, 1e-10)
    assert out.bond_dims() == [4, k, 4]
    w = T.to_dense(out)
    tail, head = float(np.sum(s[k:] ** 2)), float(np.sum(s[:k] ** 2))
    assert abs(np.linalg.norm(v - w) ** 2 - tail) < 1e-13
    assert abs(np.vdot(v, w) - head) < 1e-13
    assert abs(np.linalg.norm(w) ** 2 - head) < 1e-13


def test_mps_add_and_taylor_growth_against_dense():
    """One growth step equals the fourth-order Taylor polynomial of
    exp(-dtau H) applied to |I> when nothing is truncated."""
    m = small_model(n_mol=3, n_loc=1, n_nl=0, levels=2)
    Hw = OM.hamiltonian_mpo(m)
    psi = T.compress(T.identity_mps(m), 10 ** 6, 0.0)
    dtau = 0.07
    out = T.taylor_growth_step(psi, Hw, dtau, 10 ** 6, 0.0)
    Hfull = OM.densify(Hw)
    dims = Mdl.site_dims(m)
    L = len(dims)
    n = int(np.prod(dims))
    # H acts on the P legs of the interleaved dense vector
    v = T.to_dense(psi).reshape([d for d in dims for _ in range(2)])
    v = np.transpose(v, list(range(0, 2 * L, 2)) + list(range(1, 2 * L, 2))).reshape(n, n)
    P = np.eye(n)
    term = np.eye(n)
    for k in range(1, 5):
        term = term @ (-dtau * Hfull) / k
        P = P + term
    ref = (P @ v).reshape([d for d in dims] * 2)
    ref = np.transpose(ref, [x for i in range(L) for x in (i, L + i)]).reshape(-1)
    assert np.abs(T.to_dense(out) - ref).max() < 1e-13


# ---------------------------------------------------------- integrator pins
def _full_rank_setup():
    m = small_model(n_mol=3, n_loc=1, n_nl=0, levels=2, V=0.6)
    dims = Mdl.site_dims(m)
    return m, dims, OM.hamiltonian_mpo(m), OM.current_mpo(m)


def test_full_rank_tdvp_equals_exact_thermal_prep():
    """At maximal bond dimension every projector is the identity and the
    projector-splitting integrator is exact: imaginary-time TDVP from |I>
    reproduces ln Z of exact diagonalisation."""
    m, dims, Hw, _ = _full_rank_setup()
    beta, n = 1.2, 6
    psi0 = T.identity_mps(m)
    psi = T.full_rank_mps(T.to_dense(psi0), dims)
    psi.log_norm = 0.0
    # full_rank_mps leaves the norm on the last site; sweep it to site 0
    psi = T.MPS(psi.A)
    A = psi.A
    for i in range(len(A) - 1, 0, -1):
        a, d, _, b = A[i].shape
        Lm, Q = T.lq_pos(A[i].reshape(a, d * d * b))
        A[i] = Q.reshape(a, d, d, b)
        A[i - 1] = np.tensordot(A[i - 1], Lm, axes=([3], [0]))
    T.normalize(psi)
    for _ in range(n):
        T.tdvp_step(psi, Hw, -beta / (2 * n))
        T.normalize(psi)
    logz = 2 * psi.log_norm
    r = ED.EDResult(m, beta)
    assert abs(logz - r.logZ) < 1e-10


def test_full_rank_tdvp_real_time_equals_ed():
    m, dims, Hw, Jw = _full_rank_setup()
    beta = 0.9
    r = ED.EDResult(m, beta)
    # exact purified thermal state, then j|psi>, both at full rank
    psi0 = T.identity_mps(m)
    v0 = T.to_dense(psi0)
    L = len(dims)
    n = int(np.prod(dims))
    Hfull = OM.densify(Hw)
    Jfull = OM.densify(Jw)
    Mb = sla.expm(-0.5 * beta * Hfull)

    def act(Op, v):
        t = v.reshape([d for d in dims for _ in range(2)])
        t = np.transpose(t, list(range(0, 2 * L, 2)) + list(range(1, 2 * L, 2))).reshape(n, n)
        t = (Op @ t).reshape(dims + dims)
        return np.transpose(t, [x for i in range(L) for x in (i, L + i)]).reshape(-1)

    vb = act(Mb, v0)
    vb = vb / np.linalg.norm(vb)
    vj = act(Jfull, vb)

    def canon(v):
        p = T.full_rank_mps(v, dims)
        A = p.A
        for i in range(len(A) - 1, 0, -1):
            a, d, _, b = A[i].shape
            Lm, Q = T.lq_pos(A[i].reshape(a, d * d * b))
            A[i] = Q.reshape(a, d, d, b)
            A[i - 1] = np.tensordot(A[i - 1], Lm, axes=([3], [0]))
        return p

    psi, phi = canon(vb), canon(vj)
    dt, ns = 0.2, 10
    C = [T.overlap(psi, Jw, phi)]
    for _ in range(ns):
        T.tdvp_step(psi, Hw, -1j * dt)
        T.tdvp_step(phi, Hw, -1j * dt)
        C.append(T.overlap(psi, Jw, phi))
    ref = r.corr(np.arange(ns + 1) * dt)
    assert np.abs(np.array(C) - ref).max() < 1e-10


def test_norm_and_energy_conserved_in_real_time():
    m = small_model(n_mol=3, n_loc=1, n_nl=1, levels=2)
    Hw = OM.hamiltonian_mpo(m)
    psi, _ = T.thermal_prep(m, Hw, 1.0, 4, 4, 6)
    e0 = T.overlap(psi, Hw, psi).real
    n0 = T.norm(psi)
    for _ in range(10):
        T.tdvp_step(psi, Hw, -0.15j)
    assert abs(T.norm(psi) - n0) < 1e-12
    assert abs(T.overlap(psi, Hw, psi).real - e0) < 1e-10


def _low_bond_state(seed=3, D=3):
    from helpers import random_mps
    m = small_model(n_mol=3, n_loc=1, n_nl=1, levels=3)
    dims = Mdl.site_dims(m)
    return m, dims, OM.hamiltonian_mpo(m), random_mps(dims, D, np.random.default_rng(seed), 0)


def test_expansion_at_zero_time_keeps_the_state():
    """A step of length zero with bond expansion only changes the basis: every
    exponential is the identity and the new directions enter with zero
    coefficients, so the represented state is the same to rounding while the
    bonds grow to min(D, what the neighbouring sites carry); the result is
    right-canonical (orthonormal rows on every site but the first)."""
    m, dims, Hw, psi = _low_bond_state()
    v0 = T.to_dense(psi)
    before = psi.bond_dims()
    T.tdvp_step(psi, Hw, 0.0, expand=(12, 1e-10))
    after = psi.bond_dims()
    assert all(a >= b for a, b in zip(after, before)) and sum(after) > sum(before)
    assert max(after) == 12
    assert np.abs(T.to_dense(psi) - v0).max() < 1e-13 * np.abs(v0).max()
    for A in psi.A[1:]:
        a = A.shape[0]
        M = A.reshape(a, -1)
        assert np.abs(M @ M.conj().T - np.eye(a)).max() < 1e-12


def test_expansion_captures_the_local_residual():
    """With room for all of it, the widened basis contains the whole part of
    H_eff A outside the old basis: what is left outside the new span is at
    rounding level, and the new columns are orthonormal and orthogonal to
    the old ones."""
    rng = np.random.default_rng(8)
    m, n = 60, 5
    Q, _ = np.linalg.qr(rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n)))
    Y = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    U = T.expansion_columns(Q, Y, 40, 1e-12)
    assert U.shape == (m, n)
    Qn = np.concatenate([Q, U], axis=1)
    assert np.abs(Qn.conj().T @ Qn - np.eye(2 * n)).max() < 1e-13
    assert np.linalg.norm(Y - Qn @ (Qn.conj().T @ Y)) < 1e-13 * np.linalg.norm(Y)
    # a cap keeps the leading part only; nothing is added for Y inside span(Q)
    assert T.expansion_columns(Q, Y, 2, 1e-12).shape == (m, 2)
    assert T.expansion_columns(Q, Q @ Y[:n], 40, 1e-10).shape == (m, 0)


def test_expansion_conserves_norm_and_energy_in_real_time():
    """One-site TDVP conserves <psi|psi> and <psi|H|psi> exactly on any
    manifold (each sub-step is the exponential of a Hermitian operator
    projected with orthonormal environments); an expansion changes the
    manifold but not the state, so both stay conserved while the bonds grow.
    A misplaced zero block, a wrong rectangular bond environment or a
    non-orthonormal new basis breaks this."""
    m, dims, Hw, psi = _low_bond_state(seed=5)
    e0 = T.overlap(psi, Hw, psi).real
    n0 = T.norm(psi)
    b0 = sum(psi.bond_dims())
    for _ in range(6):
        T.tdvp_step(psi, Hw, -0.15j, expand=(10, 1e-10))
    assert sum(psi.bond_dims()) > b0
    assert abs(T.norm(psi) - n0) < 1e-12
    assert abs(T.overlap(psi, Hw, psi).real - e0) < 1e-10 * max(1.0, abs(e0))


def test_g0_correlation_constant_under_tdvp():
    """g = 0: j commutes with H, so C(t) = C(0) = 4/(1 + cosh 2) exactly.  The
    truncated TDVP trajectory drifts only by integrator error, which shrinks
    as the step is refined."""
    m = W.Model(n_mol=4, periodic=1, omega_loc=[1.0], g_loc=[0.0], omega_nl=[], g_nl=[],
                levels_loc=2, levels_nl=1, V=1.0)
    Hw, Jw = OM.hamiltonian_mpo(m), OM.current_mpo(m)
    psi, logz = T.thermal_prep(m, Hw, 1.0, 10, 10, 12)
    ref = GOLD["tight_binding_N4_V1_beta1"]["value"]
    drift = []
    for dt, n in ((0.2, 8), (0.05, 32)):
        C = T.corr_current(Hw, Jw, psi, 12, dt, n)
        assert abs(C[0] - ref) < 1e-5
        drift.append(np.abs(C - C[0]).max())
    assert drift[1] < drift[0] / 3
    assert drift[1] < 2e-6


def test_thermal_prep_converges_to_ed_with_bond_dimension():
    wl = W.tiny_fp64()
    m = wl.model
    Hw = OM.hamiltonian_mpo(m)
    r = ED.EDResult(m, 1.0)
    errs = []
    for D in (4, 8, 16):
        psi, logz = T.thermal_prep(m, Hw, 1.0, 8, 8, D)
        errs.append(abs(logz - r.logZ))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-3


def test_translation_invariance_of_thermal_density():
    m = small_model(n_mol=3, n_loc=1, n_nl=0, levels=2)
    Hw = OM.hamiltonian_mpo(m)
    psi, _ = T.thermal_prep(m, Hw, 1.0, 6, 6, 64)      # untruncated (max bond 35)
    idx = Mdl.index_of(m)
    for n in range(3):
        Nw = OM.build_mpo(m, [(1.0, [(idx[("e", n, -1)], "n")])])
        assert abs(T.overlap(psi, Nw, psi) - 1 / 3) < 1e-12


# --------------------------------------------------------------- mobility
def test_mobility_quadrature_and_units():
    tau, dt, n, beta = 3.0, 0.01, 3001, 2.0
    t = np.arange(n) * dt
    C = np.exp(-t / tau) * (1 + 0.3j)
    mu, mu_cm = An.mobility(C, dt, beta)
    exact = beta * tau * (1 - math.exp(-t[-1] / tau))
    assert abs(mu - exact) / exact < 1e-5
    assert abs(An.MOBILITY_AU_CM2VS - GOLD["mobility_au_in_cm2_per_Vs"]["value"]) < 1e-11
    assert abs(mu_cm / mu - An.MOBILITY_AU_CM2VS) < 1e-15
    lmfp, v, tau_e = An.mean_free_path(C, dt)
    assert abs(v - 1.0) < 1e-15 and abs(tau_e - exact / beta) / tau < 1e-5


# --------------------------------------------------------------- workloads
def test_workloads_are_seeded_and_in_range():
    a, b = W.headline(), W.headline()
    assert a.model.to_json() == b.model.to_json()
    lam = sum(g * g * w for g, w in zip(a.model.g_loc, a.model.omega_loc))
    assert abs(lam - W.mev(150.0)) < 1e-15
    for w in a.model.omega_loc + a.model.omega_nl:
        assert W.cm1(50.0) <= w <= W.cm1(1600.0)
    assert abs(a.run.beta - 1052.58) < 0.01
    assert abs(W.fs(0.5) - 20.67) < 0.01
    c2 = W.fp64_chain()
    assert all(0.2 <= g * g <= 1.0 for g in c2.model.g_loc)


def test_adaptive_growth_rule():
    """Stop rule of adaptive growth: no bond raised, < 2 % summed growth, or
    every bond full."""
    from oracle import tdvp as T
    full = [4, 16, 16, 4]
    assert T.growth_done([2, 2, 2, 2], [4, 16, 16, 4], 32, full)          # all full
    assert not T.growth_done([2, 2, 2, 2], [4, 8, 8, 4], 32, full)        # grew a lot
    assert T.growth_done([4, 8, 8, 4], [4, 8, 8, 4], 32, full)            # no bond raised
    assert T.growth_done([4, 100, 100, 4], [4, 100, 100, 5], 128, [4, 900, 900, 36])
    assert not T.growth_done([4, 60, 60, 4], [4, 64, 64, 4], 128, [4, 900, 900, 36])
    assert T.full_bonds([2, 3, 2]) == [4, 4]


def test_adaptive_growth_matches_fixed_count():
    """The adaptive preparation equals the fixed-count one with the number of
    growth steps it chose (same state, same ln Z)."""
    from oracle import tdvp as T
    from paper_2003_13245_amd import workloads as W
    wl = W.tiny_fp64()
    m, r = wl.model, wl.run
    Hw = OM.hamiltonian_mpo(m)
    st = T.Stats()
    psi_a, lz_a = T.thermal_prep(m, Hw, r.beta, 6, -1, 8, stats=st)
    assert 1 <= st.growth_steps < 6
    psi_f, lz_f = T.thermal_prep(m, Hw, r.beta, 6, st.growth_steps, 8)
    assert psi_a.bond_dims() == psi_f.bond_dims()
    assert abs(lz_a - lz_f) < 1e-13


# --------------------------------------------------------- coherent length
@pytest.mark.parametrize("kind", ["holstein", "peierls"])
def test_reduced_density_sum_rule_and_symmetries(kind):
    """sigma = Tr_ph rho: unit trace (one carrier), Hermitian, and invariant
    under translation along the periodic ring."""
    m = small_model(n_mol=4, n_loc=1, n_nl=1 if kind == "peierls" else 0,
                    levels=2 if kind == "peierls" else 3)
    s = ED.EDResult(m, 0.8).reduced_density()
    N = m.n_mol
    assert abs(np.trace(s) - 1) < 1e-13
    assert np.abs(s - s.conj().T).max() < 1e-13
    for i in range(N):
        for j in range(N):
            assert abs(s[i, j] - s[(i + 1) % N, (j + 1) % N]) < 1e-12


def test_coherent_length_limits():
    """The paper's two limits: sigma = I/N gives L = 1 (infinite temperature,
    where the one-carrier thermal state is uniform), and a completely
    delocalised state (g = 0 ring at low temperature: the band-edge Bloch
    state) gives L = N."""
    N = 5
    assert abs(An.coherent_length(np.eye(N) / N) - 1) < 1e-14
    assert abs(An.coherent_length(np.full((N, N), 1 / N)) - N) < 1e-13
    m = small_model(n_mol=4, n_loc=1, levels=3)
    assert abs(An.coherent_length(ED.EDResult(m, 0.0).reduced_density()) - 1) < 1e-12
    m0 = W.Model(n_mol=4, periodic=1, omega_loc=[1.0], g_loc=[0.0], omega_nl=[], g_nl=[],
                 levels_loc=2, levels_nl=1, V=1.0)
    L = An.coherent_length(ED.EDResult(m0, 30.0).reduced_density())
    assert abs(L - 4) < 1e-10


def test_reduced_density_from_full_rank_mps_equals_ed():
    """sigma from the MPS expectation values of c+_j c_i (the two-point MPO)
    on the exact purified thermal state equals the partial trace of the
    dense thermal density matrix."""
    m, dims, Hw, _ = _full_rank_setup()
    beta = 0.9
    r = ED.EDResult(m, beta)
    v0 = T.to_dense(T.identity_mps(m))
    Mb = sla.expm(-0.5 * beta * OM.densify(Hw))
    L = len(dims)
    n = int(np.prod(dims))
    # to_dense interleaves the legs (p1 q1 ... pL qL): apply Mb on the P legs
    t = v0.reshape([d for d in dims for _ in (0, 1)])
    perm = list(range(0, 2 * L, 2)) + list(range(1, 2 * L, 2))
    t = np.transpose(t, perm).reshape(n, n)
    t = (Mb @ t).reshape([d for d in dims] * 2)
    vb = np.transpose(t, np.argsort(perm)).reshape(-1)
    psi = T.full_rank_mps(vb, dims)
    s = T.reduced_density(m, psi)
    assert np.abs(s - r.reduced_density()).max() < 1e-12
