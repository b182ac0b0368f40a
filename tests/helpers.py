"""Shared test helpers: seeded models and canonical random MPS built with the
oracle's conventions (tests only)."""
import numpy as np

from paper_2003_13245_amd import workloads as W


def small_model(n_mol=3, n_loc=1, n_nl=0, levels=3, V=0.7, seed=5, periodic=1):
    rng = np.random.default_rng(seed)
    om = list(np.sort(rng.uniform(0.4, 1.5, n_loc)))
    g = list(rng.uniform(0.3, 1.0, n_loc))
    on = list(rng.uniform(0.2, 0.9, n_nl))
    gn = list(rng.uniform(0.1, 0.4, n_nl))
    return W.Model(n_mol=n_mol, periodic=periodic, omega_loc=om, g_loc=g, omega_nl=on,
                   g_nl=gn, levels_loc=levels, levels_nl=levels, V=V, R=1.3, e0=1.0)


def random_mps(dims, D, rng, center):
    """Random MPS with bond dims min(D, max rank), left-orthonormal left of
    `center`, right-orthonormal right of it."""
    from oracle import tdvp as T
    L = len(dims)
    lp, rp = [1.0] * L, [1.0] * L
    acc = 1.0
    for i in range(L):
        acc = min(acc * dims[i] ** 2, 1e18)
        lp[i] = acc
    acc = 1.0
    for i in range(L - 1, -1, -1):
        acc = min(acc * dims[i] ** 2, 1e18)
        rp[i] = acc
    bonds = [int(min(D, lp[i], rp[i + 1])) for i in range(L - 1)]
    A = []
    for i in range(L):
        a = 1 if i == 0 else bonds[i - 1]
        b = 1 if i == L - 1 else bonds[i]
        d = dims[i]
        A.append(rng.standard_normal((a, d, d, b)) + 1j * rng.standard_normal((a, d, d, b)))
    for i in range(center):
        a, d, _, b = A[i].shape
        Q, R = T.qr_pos(A[i].reshape(a * d * d, b))
        A[i] = Q.reshape(a, d, d, b)
        A[i + 1] = np.tensordot(R, A[i + 1], axes=([1], [0]))
    for i in range(L - 1, center, -1):
        a, d, _, b = A[i].shape
        Lm, Q = T.lq_pos(A[i].reshape(a, d * d * b))
        A[i] = Q.reshape(a, d, d, b)
        A[i - 1] = np.tensordot(A[i - 1], Lm, axes=([3], [0]))
    A[center] /= np.linalg.norm(A[center])
    return T.MPS(A)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def mps_inner(a, b):
    """<a|b> by left-to-right contraction (log_norm factors excluded)."""
    E = np.ones((1, 1), dtype=complex)
    for A, B in zip(a.A, b.A):
        E = np.einsum("xy,xpqa,ypqb->ab", E, A.conj(), B)
    return complex(E[0, 0])


def mps_rel_distance(a, b, n_probe=6, seed=1234):
    """Relative difference of two MPS through linear probes: for random MPS r
    of bond dimension 3, max |<r|a> - <r|b>| / max |<r|b>|.  Linear in a - b,
    so it resolves differences down to rounding (no cancellation)."""
    rng = np.random.default_rng(seed)
    dims = [t.shape[1] for t in b.A]
    L = len(dims)
    num, den = 0.0, 0.0
    for _ in range(n_probe):
        R = []
        for i, d in enumerate(dims):
            x = 1 if i == 0 else 3
            y = 1 if i == L - 1 else 3
            R.append(rng.standard_normal((x, d, d, y)) + 1j * rng.standard_normal((x, d, d, y)))
        from oracle.tdvp import MPS
        r = MPS(R)
        ra, rb = mps_inner(r, a), mps_inner(r, b)
        num = max(num, abs(ra - rb))
        den = max(den, abs(rb))
    return float(num / den)


def download_mps(psi_gpu, dims):
    """Host copy (oracle MPS) of a device MPS, log_norm included."""
    from oracle import tdvp as T
    info = psi_gpu.info()
    bd = info["bond_dims"]
    L = info["n_sites"]
    out = []
    for i in range(L):
        a = 1 if i == 0 else bd[i - 1]
        b = 1 if i == L - 1 else bd[i]
        out.append(psi_gpu.site(i, (a, dims[i], dims[i], b)))
    return T.MPS(out, info["log_norm"])
