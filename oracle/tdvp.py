"""Purified-MPS finite-temperature TD-DMRG, float64 / complex128 reference.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

What is computed (purification / thermal-field-dynamics section, Eqs. for
rho_beta, |Psi_beta> and C(t)):
  |I>       = sum_i |i>_P |i>_Q over the one-carrier space (P = physical,
              Q = auxiliary copy)
  |Psi_b>   = exp(-beta H / 2) |I>,  Z = <Psi_b|Psi_b>
  C(t)      = <Psi_b| exp(iHt) j exp(-iHt) j |Psi_b> / Z
with H acting on P only and inner products over P and Q.  Time evolution is
the time-dependent variational principle with projector splitting (the
integrator the paper cites), one-site variant, second-order symmetric sweep.

Site tensors are A[a, p, q, b] (left bond, P leg, Q leg, right bond).

Readings where the paper is silent (they bind the HIP path too):
  * bond growth: the first n_grow imaginary steps are taken by
    propagation-and-compression with a fourth-order Taylor polynomial of
    exp(-dtau H) in Horner form, each stage psi + c H phi formed exactly and
    SVD-compressed (exact right-canonical form, then a left-to-right sweep
    keeping at most D singular values with s/s_max > cutoff, never splitting
    a multiplet whose relative gap is below 1e-8);
  * the remaining imaginary steps and all real-time steps are one-site TDVP
    sweeps: left-to-right with half step, then right-to-left with half step,
    the last site evolved twice, the bond matrix evolved backwards;
  * QR gauge with a real non-negative diagonal of R;
  * Krylov exponential: Lanczos with full (twice-applied classical
    Gram-Schmidt) reorthogonalisation; stop when beta_k |e_k^T exp(zT_k) e_1|
    <= tol |exp(zT_k) e_1|, or when the Krylov space is exhausted;
  * j|Psi_b> is compressed to the same D by the same SVD compression and
    keeps the norm the truncation leaves;
  * bond expansion (optional, tdvp_step's `expand`): after each site's
    forward step and gauge factorisation the orthonormal factor is widened,
    up to D, by the leading directions of H_eff A outside its span, with
    zero coefficients in the bond matrix, so the state is unchanged and the
    following backward bond step and site step evolve into them.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
from scipy.linalg import eigh_tridiagonal

from . import model as Mdl

# LAPACK driver of the compression SVD.  "gesdd" and "gesvd" compute the same
# decomposition up to rounding; the tests run the oracle with both to measure
# how far rounding alone moves C(t) on a given workload.
SVD_DRIVER = "gesdd"


def svd(M):
    """Thin SVD M = U diag(s) Vh with s descending."""
    return sla.svd(M, full_matrices=False, lapack_driver=SVD_DRIVER)


# --------------------------------------------------------------------------
# MPS containers
# --------------------------------------------------------------------------


class MPS:
    """List of site tensors A[a, p, q, b]; `log_norm` carries a scalar
    normalisation factor exp(log_norm) kept outside the tensors."""

    def __init__(self, tensors, log_norm=0.0):
        self.A = [np.asarray(t, dtype=complex) for t in tensors]
        self.log_norm = log_norm

    def copy(self):
        return MPS([a.copy() for a in self.A], self.log_norm)

    def __len__(self):
        return len(self.A)

    def bond_dims(self):
        return [a.shape[3] for a in self.A[:-1]]


def identity_mps(model):
    """The purified identity |I> of the one-carrier space (normalised) and
    0.5 ln <I|I>.  Bond states: 0 = carrier not yet placed, 1 = placed; after
    the last electronic site only 'placed' survives."""
    sl = Mdl.site_list(model)
    dims = Mdl.site_dims(model)
    e_sites = [i for i, s in enumerate(sl) if s[0] == "e"]
    first_e, last_e = e_sites[0], e_sites[-1]
    tensors = []
    # bond-state labels on the left of each site
    for i, (kind, n, m) in enumerate(sl):
        d = dims[i]
        left = ["none"] if i <= first_e else (["placed"] if i > last_e else ["none", "placed"])
        right = ["none"] if i < first_e else (["placed"] if i >= last_e else ["none", "placed"])
        A = np.zeros((len(left), d, d, len(right)), dtype=complex)
        for ia, a in enumerate(left):
            for ib, b in enumerate(right):
                if kind == "e":
                    if a == "none" and b == "none":
                        A[ia, 0, 0, ib] = 1.0
                    elif a == "none" and b == "placed":
                        A[ia, 1, 1, ib] = 1.0
                    elif a == "placed" and b == "placed":
                        A[ia, 0, 0, ib] = 1.0
                else:
                    if a == b:
                        for v in range(d):
                            A[ia, v, v, ib] = 1.0
        tensors.append(A)
    ph = [dims[i] for i, s in enumerate(sl) if s[0] != "e"]
    dim = model.n_mol * int(np.prod(ph)) if ph else model.n_mol
    psi = MPS(tensors)
    # normalise: every component of |I> is 1, so <I|I> = dim
    psi.A[0] = psi.A[0] / math.sqrt(dim)
    psi.log_norm = 0.5 * math.log(dim)
    return psi


def full_rank_mps(vec, dims):
    """Exact MPS of a dense purified vector (site order, P then Q leg per
    site) with every bond at its largest possible dimension, built by reduced
    QR sweeps without truncation; the last tensor carries the norm.  At these
    bond dimensions every tangent-space projector is the identity, so the
    projector-splitting integrator is exact (tests only)."""
    L = len(dims)
    rest = np.asarray(vec, dtype=complex).reshape(1, -1)
    A = []
    Dl = 1
    for i in range(L - 1):
        d = dims[i]
        M = rest.reshape(Dl * d * d, -1)
        Q, R = qr_pos(M)
        A.append(Q.reshape(Dl, d, d, Q.shape[1]))
        Dl = Q.shape[1]
        rest = R
    d = dims[-1]
    A.append(rest.reshape(Dl, d, d, 1))
    return MPS(A)


def to_dense(psi):
    """Dense coefficient array over (p_1 q_1 ... p_L q_L), tiny chains only."""
    T = psi.A[0]
    for A in psi.A[1:]:
        T = np.tensordot(T, A, axes=([T.ndim - 1], [0]))
    return T.reshape(-1) * math.exp(psi.log_norm)


# --------------------------------------------------------------------------
# Dense linear algebra conventions
# --------------------------------------------------------------------------


# Relative size of a random perturbation applied to every QR / LQ factor Q
# (0: none).  Off in every computation; the tests set it to measure how far
# rounding-level differences in the gauge moves alone move C(t).
QR_NOISE = 0.0
_qr_noise_rng = np.random.default_rng(7)


def qr_pos(M):
    """Reduced QR with a real non-negative diagonal of R."""
    Q, R = np.linalg.qr(M, mode="reduced")
    d = np.diag(R)
    ph = np.ones_like(d)
    nz = np.abs(d) > 0
    ph[nz] = d[nz] / np.abs(d[nz])
    Q = Q * ph[None, :]
    R = np.conj(ph)[:, None] * R
    if QR_NOISE:
        Q = Q * (1 + QR_NOISE * (_qr_noise_rng.standard_normal(Q.shape)
                                 + 1j * _qr_noise_rng.standard_normal(Q.shape)))
    return Q, R


def lq_pos(M):
    """M = L Q with Q having orthonormal rows and L's diagonal real >= 0."""
    Q, R = qr_pos(M.conj().T)
    return R.conj().T, Q.conj().T


def truncation_rank(s, D, cutoff):
    """How many singular values (sorted descending) to keep."""
    if s.size == 0 or s[0] == 0.0:
        return 1
    k = int(np.sum(s > cutoff * s[0]))
    k = max(1, min(k, D))
    # never cut inside a (near-)degenerate multiplet
    while 1 < k < s.size and (s[k - 1] - s[k]) <= 1e-8 * s[k - 1]:
        k -= 1
    return k


# --------------------------------------------------------------------------
# MPO x MPS, sums and compression
# --------------------------------------------------------------------------


def apply_mpo(Ws, psi):
    """Exact product: bond dimension multiplies by the MPO bond dimension."""
    out = []
    for W, A in zip(Ws, psi.A):
        a, d, _, b = A.shape
        wl, wr = W.shape[0], W.shape[1]
        B = np.tensordot(W, A, axes=([3], [1])).transpose(3, 0, 2, 4, 5, 1)
        out.append(B.reshape(a * wl, d, d, b * wr))
    return MPS(out, psi.log_norm)


def add(psi, phi, c):
    """psi + c * phi as an exact MPS (block-diagonal bonds).  Both must carry
    the same log_norm."""
    assert abs(psi.log_norm - phi.log_norm) < 1e-300 + 1e-15 * max(1, abs(psi.log_norm))
    L = len(psi)
    out = []
    for i, (A, B) in enumerate(zip(psi.A, phi.A)):
        if i == 0:
            B = c * B
        a1, d, _, b1 = A.shape
        a2, _, _, b2 = B.shape
        if L == 1:
            out.append(A + B)
            continue
        if i == 0:
            C = np.zeros((1, d, d, b1 + b2), dtype=complex)
            C[:, :, :, :b1] = A
            C[:, :, :, b1:] = B
        elif i == L - 1:
            C = np.zeros((a1 + a2, d, d, 1), dtype=complex)
            C[:a1] = A
            C[a1:] = B
        else:
            C = np.zeros((a1 + a2, d, d, b1 + b2), dtype=complex)
            C[:a1, :, :, :b1] = A
            C[a1:, :, :, b1:] = B
        out.append(C)
    return MPS(out, psi.log_norm)


def right_canonicalize(A):
    """LQ sweep from the right without truncation (in place on a list)."""
    for i in range(len(A) - 1, 0, -1):
        a, d, _, b = A[i].shape
        Lm, Q = lq_pos(A[i].reshape(a, d * d * b))
        A[i] = Q.reshape(Q.shape[0], d, d, b)
        A[i - 1] = np.tensordot(A[i - 1], Lm, axes=([3], [0]))
    return A


def svd_compress(X, D, cutoff):
    """SVD compression of an MPS: bring it to right-canonical form exactly,
    then sweep left to right truncating each bond to at most D singular
    values with s/s_max > cutoff (whole multiplets), then return it to
    right-canonical form.  The result depends only on the state, not on how
    the input tensors are gauged or which MPO produced them."""
    A = right_canonicalize([t.copy() for t in X.A])
    L = len(A)
    for i in range(L - 1):
        a, d, _, b = A[i].shape
        U, s, Vh = svd(A[i].reshape(a * d * d, b))
        k = truncation_rank(s, D, cutoff)
        A[i] = U[:, :k].reshape(a, d, d, k)
        A[i + 1] = np.tensordot(s[:k, None] * Vh[:k], A[i + 1], axes=([1], [0]))
    return MPS(right_canonicalize(A), X.log_norm)


def compress_terms(terms, D, cutoff):
    """Compressed sum_t c_t O_t |psi_t> (O_t an MPO or None for the
    identity): the exact sum is formed and SVD-compressed."""
    X = None
    for c, Ws, p in terms:
        Y = apply_mpo(Ws, p) if Ws is not None else p.copy()
        if X is None:
            Y.A[0] = c * Y.A[0]
            X = Y
        else:
            X = add(X, Y, c)
    return svd_compress(X, D, cutoff)


def compress(psi, D, cutoff):
    """SVD compression of a single MPS."""
    return svd_compress(psi, D, cutoff)


def normalize(psi):
    """For a right-canonical MPS: move the norm of the first tensor into
    log_norm.  Returns the norm that was removed."""
    n = np.linalg.norm(psi.A[0])
    psi.A[0] = psi.A[0] / n
    psi.log_norm += math.log(n)
    return n


def taylor_growth_step(psi, Hw, dtau, D, cutoff, order=4):
    """exp(-dtau H) psi by propagation and compression, Taylor order 4 in
    Horner form: phi <- psi + (-dtau/k) H phi, k = order..1."""
    phi = psi
    for k in range(order, 0, -1):
        phi = compress_terms([(1.0, None, psi), (-dtau / k, Hw, phi)], D, cutoff)
    return phi


# --------------------------------------------------------------------------
# Environments and effective Hamiltonians
# --------------------------------------------------------------------------


def left_env(Lenv, bra, W, ket):
    """L'[c', b', b] = sum conj(bra[a',p',q,b']) L[c,a',a] W[c,c',p',p] ket[a,p,q,b]."""
    T = np.tensordot(Lenv, ket, axes=([2], [0]))            # [c, a', p, q, b]
    U = np.tensordot(W, T, axes=([0, 3], [0, 2]))           # [c', p', a', q, b]
    out = np.tensordot(U, bra.conj(), axes=([2, 1, 3], [0, 1, 2]))  # [c', b, b']
    return out.transpose(0, 2, 1)


def right_env(Renv, bra, W, ket):
    """R'[c, a', a] = sum ket[a,p,q,b] R[c',b',b] W[c,c',p',p] conj(bra[a',p',q,b'])."""
    T = np.tensordot(ket, Renv, axes=([3], [2]))            # [a, p, q, c', b']
    U = np.tensordot(W, T, axes=([1, 3], [3, 1]))           # [c, p', a, q, b']
    out = np.tensordot(U, bra.conj(), axes=([1, 3, 4], [1, 2, 3]))  # [c, a, a']
    return out.transpose(0, 2, 1)


def heff_apply(Lenv, W, Renv, A):
    """y[a',p',q,b'] = sum L[c,a',a] W[c,c',p',p] A[a,p,q,b] R[c',b',b]."""
    T = np.tensordot(Lenv, A, axes=([2], [0]))              # [c, a', p, q, b]
    U = np.tensordot(W, T, axes=([0, 3], [0, 2]))           # [c', p', a', q, b]
    y = np.tensordot(U, Renv, axes=([0, 4], [0, 2]))        # [p', a', q, b']
    return y.transpose(1, 0, 2, 3)


def keff_apply(Lenv, Renv, C):
    """y[a',b'] = sum_c L[c,a',a] C[a,b] R[c,b',b]."""
    T = np.tensordot(Lenv, C, axes=([2], [0]))              # [c, a', b]
    return np.tensordot(T, Renv, axes=([0, 2], [0, 2]))


# --------------------------------------------------------------------------
# Krylov exponential
# --------------------------------------------------------------------------


class KrylovNotConverged(RuntimeError):
    pass


def expm_krylov(apply, v, z, tol=1e-14, mmax=40):
    """exp(z H) v for Hermitian H given as `apply`, by Lanczos with full
    reorthogonalisation.  Returns (result, number of Krylov vectors)."""
    shape = v.shape
    v = v.reshape(-1)
    n = v.size
    beta0 = np.linalg.norm(v)
    if beta0 == 0.0:
        return v.reshape(shape).copy(), 0
    Q = np.zeros((min(mmax, n) + 1, n), dtype=complex)
    Q[0] = v / beta0
    alpha, beta = [], []
    for k in range(min(mmax, n)):
        w = apply(Q[k].reshape(shape)).reshape(-1)
        alpha.append(np.vdot(Q[k], w).real)
        Qk = Q[:k + 1]
        for _ in range(2):
            w = w - Qk.T @ (Qk.conj() @ w)
        bk = np.linalg.norm(w)
        a = np.array(alpha)
        if k == 0:
            lam, S = a.copy(), np.ones((1, 1))
        else:
            lam, S = eigh_tridiagonal(a, np.array(beta))
        u = S @ (np.exp(z * lam) * S[0, :])
        exhausted = (k + 1 == n)
        if exhausted or bk * abs(u[-1]) <= tol * np.linalg.norm(u) or bk == 0.0:
            return (beta0 * (Q[:k + 1].T @ u)).reshape(shape), k + 1
        beta.append(bk)
        Q[k + 1] = w / bk
    raise KrylovNotConverged(f"Lanczos did not converge in {mmax} steps")


# --------------------------------------------------------------------------
# One-site TDVP, projector splitting, second order
# --------------------------------------------------------------------------


def _boundary(shape_w):
    e = np.zeros((shape_w, 1, 1), dtype=complex)
    e[0, 0, 0] = 1.0
    return e


def right_envs(psi, Ws):
    """R[i] = contraction of sites i..L-1 (R[L] is the boundary)."""
    L = len(psi)
    R = [None] * (L + 1)
    R[L] = _boundary(1)
    for i in range(L - 1, 0, -1):
        R[i] = right_env(R[i + 1], psi.A[i], Ws[i], psi.A[i])
    return R


class Stats:
    def __init__(self):
        self.krylov = []


# --------------------------------------------------------------------------
# Bond expansion (adaptive bond dimension; the paper needs larger D at low T
# and large V but is silent on how a one-site integrator grows it)
# --------------------------------------------------------------------------


def expansion_rank(s, ref, cap, tol):
    """How many new bond directions to add: the singular values s (descending)
    of the projected residual that exceed tol * ref, at most cap, never
    splitting a near-degenerate multiplet (relative gap 1e-8)."""
    if cap <= 0 or s.size == 0:
        return 0
    k = min(int(np.sum(s > tol * ref)), cap)
    while 0 < k < s.size and (s[k - 1] - s[k]) <= 1e-8 * s[k - 1]:
        k -= 1
    return k


def expansion_columns(Q, Y, cap, tol):
    """Orthonormal columns spanning the leading part of Y outside span(Q):
    Y minus its projection on the orthonormal columns of Q (taken twice),
    then the left singular vectors whose singular values pass
    expansion_rank with ref = |Y|_F."""
    P = Y - Q @ (Q.conj().T @ Y)
    P = P - Q @ (Q.conj().T @ P)
    U, s, _ = svd(P)
    k = expansion_rank(s, np.linalg.norm(Y), cap, tol)
    return U[:, :k]


def tdvp_step(psi, Ws, z, tol=1e-14, mmax=40, stats=None, expand=None):
    """One symmetric sweep pair evolving psi by exp(z H): z = -i dt for real
    time, z = -dtau for imaginary time.  psi must be right-canonical with the
    centre on site 0; it is returned in the same form.

    expand = (D, etol): bond expansion.  After each site's forward step and
    its gauge factorisation, while the bond it opens is below
    min(D, what the two neighbouring sites can carry), the orthonormal
    factor is widened by the leading directions of H_eff A outside its span
    (expansion_columns with etol); the bond matrix gets zero rows (columns,
    right to left) for them, so the state is unchanged, and the backward
    bond step and the next site's step then evolve into the enlarged
    basis."""
    L = len(psi)
    A = psi.A
    R = right_envs(psi, Ws)
    Lenv = [None] * (L + 1)
    Lenv[0] = _boundary(1)
    h = 0.5 * z

    def site_evolve(i):
        f = lambda x: heff_apply(Lenv[i], Ws[i], R[i + 1], x)
        A[i], m = expm_krylov(f, A[i], h, tol, mmax)
        if stats is not None:
            stats.krylov.append(m)

    # left to right
    for i in range(L - 1):
        site_evolve(i)
        a, d, _, b = A[i].shape
        Q, C = qr_pos(A[i].reshape(a * d * d, b))
        if expand is not None:
            _, dn, _, bn = A[i + 1].shape
            cap = min(expand[0], a * d * d, dn * dn * bn) - b
            if cap > 0:
                Y = heff_apply(Lenv[i], Ws[i], R[i + 1], A[i]).reshape(a * d * d, b)
                U = expansion_columns(Q, Y, cap, expand[1])
                Q = np.concatenate([Q, U], axis=1)
                C = np.concatenate([C, np.zeros((U.shape[1], b), dtype=complex)], axis=0)
        A[i] = Q.reshape(a, d, d, Q.shape[1])
        Lenv[i + 1] = left_env(Lenv[i], A[i], Ws[i], A[i])
        f = lambda x: keff_apply(Lenv[i + 1], R[i + 1], x)
        C, m = expm_krylov(f, C, -h, tol, mmax)
        if stats is not None:
            stats.krylov.append(m)
        A[i + 1] = np.tensordot(C, A[i + 1], axes=([1], [0]))
    site_evolve(L - 1)
    # right to left
    site_evolve(L - 1)
    for i in range(L - 1, 0, -1):
        a, d, _, b = A[i].shape
        C, Q = lq_pos(A[i].reshape(a, d * d * b))
        if expand is not None:
            ap, dp = A[i - 1].shape[0], A[i - 1].shape[1]
            cap = min(expand[0], d * d * b, ap * dp * dp) - a
            if cap > 0:
                Y = heff_apply(Lenv[i], Ws[i], R[i + 1], A[i]).reshape(a, d * d * b)
                Wr = expansion_columns(Q.conj().T, Y.conj().T, cap, expand[1]).conj().T
                Q = np.concatenate([Q, Wr], axis=0)
                C = np.concatenate([C, np.zeros((a, Wr.shape[0]), dtype=complex)], axis=1)
        A[i] = Q.reshape(Q.shape[0], d, d, b)
        R[i] = right_env(R[i + 1], A[i], Ws[i], A[i])
        f = lambda x: keff_apply(Lenv[i], R[i], x)
        C, m = expm_krylov(f, C, -h, tol, mmax)
        if stats is not None:
            stats.krylov.append(m)
        A[i - 1] = np.tensordot(A[i - 1], C, axes=([3], [0]))
        site_evolve(i - 1)
    return psi


# --------------------------------------------------------------------------
# Observables
# --------------------------------------------------------------------------


def overlap(bra, Ws, ket):
    """<bra| O |ket> for an MPO O (ignores log_norm factors)."""
    E = _boundary(1)
    for A, W, B in zip(bra.A, Ws, ket.A):
        E = left_env(E, A, W, B)
    return E[0, 0, 0]


def norm(psi):
    E = np.ones((1, 1), dtype=complex)
    for A in psi.A:
        E = np.einsum("xy,xpqa,ypqb->ab", E, A.conj(), A)
    return math.sqrt(E[0, 0].real)


# --------------------------------------------------------------------------
# The pipeline
# --------------------------------------------------------------------------


def growth_done(before, after, D, full):
    """Stop rule of adaptive growth (n_grow < 0): stop after a growth step
    that raised no bond, or raised the summed bond dimension by less than
    2 %, or left every bond at min(D, its largest possible value)."""
    if all(b >= min(D, f) for b, f in zip(after, full)):
        return True
    if not any(a > b for a, b in zip(after, before)):
        return True
    return sum(after) < 1.02 * sum(before)


def full_bonds(dims):
    """Largest possible bond dimension at each bond of a purified MPS."""
    L = len(dims)
    left = np.cumprod([float(d) ** 2 for d in dims])
    right = np.cumprod([float(d) ** 2 for d in dims[::-1]])[::-1]
    return [min(left[i], right[i + 1]) for i in range(L - 1)]


def thermal_prep(model, Hw, beta, n_imag, n_grow, D, cutoff=1e-10, tol=1e-14,
                 mmax=40, stats=None, expand_tol=0.0):
    """|Psi_beta> = exp(-beta H/2)|I> in n_imag steps of beta/(2 n_imag):
    the first n_grow steps by propagation and compression (n_grow < 0:
    adaptive, see growth_done), the rest by one-site TDVP, with bond
    expansion up to D (tdvp_step's expand) when expand_tol > 0, each such
    step followed by an SVD compression at `cutoff` (no bond keeps Schmidt
    values below cutoff * s_max, which imaginary time can produce).
    Returns the normalised right-canonical state and ln Z."""
    dtau = beta / (2.0 * n_imag)
    psi = identity_mps(model)
    psi = compress(psi, D, cutoff)
    normalize(psi)
    full = full_bonds([t.shape[1] for t in psi.A])
    steps = 0
    for _ in range(n_imag if n_grow < 0 else n_grow):
        before = psi.bond_dims()
        psi = taylor_growth_step(psi, Hw, dtau, D, cutoff)
        normalize(psi)
        steps += 1
        if n_grow < 0 and growth_done(before, psi.bond_dims(), D, full):
            break
    ex = (D, expand_tol) if expand_tol > 0 else None
    for _ in range(n_imag - steps):
        tdvp_step(psi, Hw, -dtau, tol, mmax, stats, expand=ex)
        if ex is not None:
            # imaginary time damps some of the added directions towards zero
            # weight: drop Schmidt values below the compression cutoff so that
            # no bond carries a numerically null direction
            psi = svd_compress(psi, D, cutoff)
        normalize(psi)
    if stats is not None:
        stats.growth_steps = steps
    return psi, 2.0 * psi.log_norm


def reduced_density(model, psi):
    """sigma_ij = <psi| c+_j c_i |psi> / <psi|psi> (operators on the P leg;
    the inner product traces P and Q)."""
    from . import mpo as OM
    N = model.n_mol
    nrm2 = norm(psi) ** 2
    sig = np.zeros((N, N), dtype=complex)
    for i in range(N):
        for j in range(N):
            sig[i, j] = overlap(psi, OM.hop_mpo(model, i, j), psi) / nrm2
    return sig


def apply_current(Jw, psi, D, cutoff=1e-10):
    """j|psi> compressed to bond dimension D (norm kept, log_norm reset)."""
    phi = compress_terms([(1.0, Jw, psi)], D, cutoff)
    phi.log_norm = 0.0
    return phi


def corr_current(Hw, Jw, psi_beta, D, dt, n_steps, cutoff=1e-10, tol=1e-14,
                 mmax=40, stats=None, callback=None):
    """C(t_k), k = 0..n_steps, t_k = k dt, for a normalised psi_beta."""
    psi = psi_beta.copy()
    psi.log_norm = 0.0
    phi = apply_current(Jw, psi, D, cutoff)
    C = np.zeros(n_steps + 1, dtype=complex)
    C[0] = overlap(psi, Jw, phi)
    for k in range(1, n_steps + 1):
        tdvp_step(psi, Hw, -1j * dt, tol, mmax, stats)
        tdvp_step(phi, Hw, -1j * dt, tol, mmax, stats)
        C[k] = overlap(psi, Jw, phi)
        if callback is not None:
            callback(k, psi, phi)
    return C
