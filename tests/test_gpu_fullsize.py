"""Parity at the benchmark's sizes.

* Sampled outputs: the effective-Hamiltonian matvec at a phonon site of the
  benchmark's shape (bond dimension 128, 10 phonon levels, the rubrene-shaped
  Holstein-Peierls MPO channels) on a 3-molecule ring, against the oracle's
  contraction of the same tensors: complex128 and the mixed-precision path.
* Properties at full size: after the benchmark's own preparation of the
  21-molecule ring, one real-time pair step conserves <psi|psi> and
  <psi|H|psi> of both states (one-site projector-splitting TDVP conserves both
  up to the Krylov tolerance and the contraction precision)."""
import numpy as np
import pytest

from helpers import random_mps, rel
from oracle import model as Mdl
from oracle import mpo as OM
from oracle import tdvp as T
from paper_2003_13245_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_heff_at_benchmark_shape(ctx):
    from paper_2003_13245_amd import api
    wl = W.rubrene_shaped(n_mol=3)
    m = wl.model
    dims = Mdl.site_dims(m)
    Hw = OM.hamiltonian_mpo(m)
    H, _ = api.mpo_build(ctx, m)
    # middle phonon site whose bonds both reach D = 128
    site = len(dims) // 2
    while dims[site] == 2:
        site += 1
    rng = np.random.default_rng(5)
    psi = random_mps(dims, 128, rng, site)
    a, _, _, b = psi.A[site].shape
    say(f"[fullsize] H_eff at site {site}: {a} x {dims[site]} x {dims[site]} x {b}")
    assert a == 128 and b == 128
    Lenv = T._boundary(1)
    for i in range(site):
        Lenv = T.left_env(Lenv, psi.A[i], Hw[i], psi.A[i])
    Renv = T._boundary(1)
    for i in range(len(dims) - 1, site, -1):
        Renv = T.right_env(Renv, psi.A[i], Hw[i], psi.A[i])
    x = rng.standard_normal(psi.A[site].shape) + 1j * rng.standard_normal(psi.A[site].shape)
    y_ref = T.heff_apply(Lenv, Hw[site], Renv, x)
    g = api.mps_from_host(ctx, psi.A)
    y = api.heff_apply(ctx, H, g, site, x)
    e64 = rel(y, y_ref)
    # complex-FP32 contractions: K up to (MPO width) x 128 terms, FP32
    # rounding 6e-8 per term with random signs -> ~ 6e-8 * sqrt(K) ~ 2e-6
    g.set_precision("c64")
    y32 = api.heff_apply(ctx, H, g, site, x)
    e32 = rel(y32, y_ref)
    # bf16x3: each real product carries a relative error of order 2^-17
    # (the split of both operands and the dropped lo*lo term), ~1e-5, with
    # the same random-sign growth over K
    g.set_precision("bf16x3")
    yb = api.heff_apply(ctx, H, g, site, x)
    eb = rel(yb, y_ref)
    say(f"[fullsize] H_eff rel err c128 {e64:.1e}, c64 {e32:.1e}, bf16x3 {eb:.1e}")
    assert e64 < 1e-12
    assert e32 < 2e-5
    assert eb < 1e-3


def test_pair_step_conserves_norm_and_energy_at_full_size(ctx):
    from paper_2003_13245_amd import api
    wl = W.headline()
    m, r = wl.model, wl.run
    H, J = api.mpo_build(ctx, m)
    say(f"[fullsize] preparing {wl.name}")
    psi, logz = api.thermal_prep(ctx, H, r.beta, r.n_imag, r.n_grow, r.D, cutoff=r.cutoff,
                                 precision="c64", tol=r.krylov_tol, mmax=r.krylov_mmax)
    phi = api.apply_compress(ctx, J, psi, r.D, r.cutoff)
    phi.set_precision("c64")
    before = [(s.norm2(), api.overlap(ctx, s, H, s).real) for s in (psi, phi)]
    api.tdvp_pair(ctx, H, psi, phi, dt_real=r.dt, tol=r.krylov_tol, mmax=r.krylov_mmax)
    after = [(s.norm2(), api.overlap(ctx, s, H, s).real) for s in (psi, phi)]
    for (n0, e0), (n1, e1) in zip(before, after):
        say(f"[fullsize] norm {n0:.12g} -> {n1:.12g}, energy {e0:.12g} -> {e1:.12g}")
        # Krylov tolerance 1e-8 per exponential over ~500 exponentials, FP32
        # contractions: relative drift well below 1e-5
        assert abs(n1 - n0) <= 1e-5 * abs(n0)
        assert abs(e1 - e0) <= 1e-5 * abs(e0)
