"""Pins of the oracle's mobility sweep (batched runs over temperature,
transfer integral and frequency scale) against exact results:

* the isotope scaling keeps every mode's reorganisation energy g^2 omega and
  multiplies its frequency by s; s = sqrt(m/m') for a mass m -> m';
* one sweep point reproduces the single pipeline run exactly;
* without electron-phonon coupling the current correlation of the ring is the
  constant (2 e0 V R)^2 sum_k sin^2 k e^{-2 beta V cos k} / sum_k e^{-2 beta V
  cos k} (k = 2 pi j / N), so mu = beta C t_max / e0 for every beta, V and s:
  a wrong beta, V or scale anywhere in the orchestration fails it;
* the mobility gradient: exact diagonalisation differentiated in closed form
  (divided differences of the exponentials) against central differences of
  the exact mobility, and the oracle's finite-difference gradient through
  the whole TDVP pipeline at full bond dimension against that exact
  gradient."""
import dataclasses
import math

import numpy as np
import pytest

from helpers import small_model
from oracle import analysis as An
from oracle import ed as ED
from oracle import mpo as OM
from oracle import sweep as S
from oracle import tdvp as T
from paper_2003_13245_amd import workloads as W


def test_scaling_keeps_reorganisation_energies():
    m = small_model(n_mol=3, n_loc=2, n_nl=1, levels=3)
    for s in (0.5, 1.0, math.sqrt(12.0 / 13.0), 2.0):
        ms = S.scaled_model(m, 0.3, s)
        assert ms.V == 0.3 and ms.n_mol == m.n_mol and ms.levels_loc == m.levels_loc
        for w0, g0, w1, g1 in list(zip(m.omega_loc, m.g_loc, ms.omega_loc, ms.g_loc)) + \
                list(zip(m.omega_nl, m.g_nl, ms.omega_nl, ms.g_nl)):
            assert abs(w1 - s * w0) <= 1e-15 * w0
            assert abs(g1 * g1 * w1 - g0 * g0 * w0) <= 1e-14 * g0 * g0 * w0
    assert S.mass_scale(13.0 / 12.0) == pytest.approx(math.sqrt(12.0 / 13.0), rel=1e-15)
    with pytest.raises(ValueError):
        S.scaled_model(m, 1.0, 0.0)


def test_single_point_equals_pipeline():
    m = small_model(n_mol=3, n_loc=1, n_nl=1, levels=3)
    mu, logz = S.mobility_sweep(m, [(1.0, m.V, 1.0)], 6, 6, 12, 0.1, 5)
    Hw, Jw = OM.hamiltonian_mpo(m), OM.current_mpo(m)
    psi, lz = T.thermal_prep(m, Hw, 1.0, 6, 6, 12)
    C = T.corr_current(Hw, Jw, psi, 12, 0.1, 5)
    assert mu[0] == An.mobility(C, 0.1, 1.0, m.e0)[0]
    assert logz[0] == lz


def test_uncoupled_ring_matches_closed_form_at_every_point():
    m = W.Model(n_mol=4, periodic=1, omega_loc=[1.0], g_loc=[0.0], omega_nl=[], g_nl=[],
                levels_loc=2, levels_nl=1, V=1.0)
    pts = [(1.0, 1.0, 1.0), (1.0, 1.0, 0.8), (0.5, 0.7, 1.3)]
    dt, n_steps = 0.1, 10
    mu, _ = S.mobility_sweep(m, pts, 20, 20, 64, dt, n_steps)
    k = 2 * np.pi * np.arange(m.n_mol) / m.n_mol
    for (beta, V, s), got in zip(pts, mu):
        w = np.exp(-2 * beta * V * np.cos(k))
        C = (2 * m.e0 * V * m.R) ** 2 * (np.sin(k) ** 2 * w).sum() / w.sum()
        exact = beta / m.e0 * C * n_steps * dt
        # Taylor-4 preparation and the projector-splitting drift at this
        # rank: measured 1.5e-7 to 1.3e-6 (a wrong beta, V or s is an O(1) error)
        assert abs(got - exact) <= 1e-5 * exact, (beta, V, s, got, exact)


def test_gradient_chain_rule_matches_isotope_slope():
    """The finite-difference gradient and the sweep probe mu along different
    directions; the chain rule through omega -> s omega, g -> g/sqrt(s) ties
    them: -1/2 d mu / d ln s at s = 1 equals -1/2 sum omega d mu/d omega +
    1/4 sum g d mu/d g.  Both are central differences (error O(h^2) plus the
    rounding of mu over h)."""
    m = small_model(n_mol=3, n_loc=1, n_nl=0, levels=3)
    run = dict(n_imag=6, n_grow=6, D=12, dt=0.1, n_steps=5)
    mu, grads = S.mobility_grad(m, 1.0, rel_step=1e-4, **run)
    assert mu == S.mobility_sweep(m, [(1.0, m.V, 1.0)], **run)[0][0]
    iso = S.isotope_derivative(m, grads)
    h = 1e-4
    mus, _ = S.mobility_sweep(m, [(1.0, m.V, 1 + h), (1.0, m.V, 1 - h)], **run)
    slope = -0.5 * (mus[0] - mus[1]) / (math.log(1 + h) - math.log(1 - h))
    # measured 1.3e-9 relative
    assert abs(slope - iso) <= 1e-6 * abs(iso), (slope, iso)


GRAD_MODELS = {"holstein": dict(n_mol=3, n_loc=1, n_nl=0, levels=2, V=0.6),
               "peierls": dict(n_mol=3, n_loc=0, n_nl=1, levels=2, V=0.6)}


def _exact_mu(m, beta, dt, n_steps):
    r = ED.EDResult(m, beta)
    return An.mobility(r.corr(np.arange(n_steps + 1) * dt), dt, beta, m.e0)[0]


@pytest.mark.parametrize("name", ["holstein", "peierls", "both"])
def test_exact_gradient_matches_differences_of_exact_mobility(name):
    """The closed-form derivative of the exact mobility (every term of
    d Tr[e^{-beta H} e^{iHt} j e^{-iHt} j] and of dZ; the Peierls model also
    moves j) against central differences of the exact mobility itself, which
    share none of that formula: a dropped term or a sign fails by far more
    than the difference error (measured 1e-11 to 5e-10 relative)."""
    kw = GRAD_MODELS.get(name, dict(n_mol=3, n_loc=1, n_nl=1, levels=2, V=0.7))
    m = small_model(**kw)
    beta, dt, n_steps = 1.0, 0.1, 20
    mu, grads = ED.mobility_gradient(m, beta, dt, n_steps)
    assert abs(mu - _exact_mu(m, beta, dt, n_steps)) < 1e-13 * abs(mu)
    for key, g in grads.items():
        vals = list(getattr(m, key))
        assert len(g) == len(vals)
        for i, x in enumerate(vals):
            h = 1e-5 * abs(x)
            up = dataclasses.replace(m, **{key: vals[:i] + [x + h] + vals[i + 1:]})
            dn = dataclasses.replace(m, **{key: vals[:i] + [x - h] + vals[i + 1:]})
            fd = (_exact_mu(up, beta, dt, n_steps) - _exact_mu(dn, beta, dt, n_steps)) / (2 * h)
            assert abs(g[i] - fd) <= 1e-8 * abs(fd), (key, i, g[i], fd)


@pytest.mark.parametrize("name", ["holstein", "peierls"])
def test_pipeline_gradient_at_full_rank_matches_exact_gradient(name):
    """At full bond dimension and with no singular value discarded, one
    growth step followed by one-site TDVP is exact, so the oracle's central
    differences of mu through preparation, j|Psi>, real-time steps and the
    Kubo sum must reproduce the exact gradient (measured 1e-9 to 2e-8
    relative; mu itself to 5e-11)."""
    m = small_model(**GRAD_MODELS[name])
    beta, dt, n_steps = 1.0, 0.1, 10
    mu_x, g_x = ED.mobility_gradient(m, beta, dt, n_steps)
    mu, g = S.mobility_grad(m, beta, n_imag=40, n_grow=1, D=64, dt=dt, n_steps=n_steps,
                            cutoff=0.0)
    assert abs(mu - mu_x) <= 1e-9 * abs(mu_x), (mu, mu_x)
    for key in g_x:
        assert len(g[key]) == len(g_x[key])
        for a, b in zip(g[key], g_x[key]):
            assert abs(a - b) <= 1e-6 * abs(b), (key, a, b)
