"""Batched mobility runs over temperature, transfer integral and mode-
frequency scale: the workload of the paper's temperature, coupling and
isotope studies, run point by point through this package's pipeline.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Isotope substitution of a mass m by m' multiplies each mode frequency by
s = sqrt(m/m') with the mode's reorganisation energy g^2 omega held fixed
(isotope-effect passage), hence g -> g / sqrt(s).  The isotope effect is
mu(s) / mu(1) - 1 between two runs that differ only in s."""
import dataclasses
import math

import numpy as np

from . import analysis as An
from . import mpo as OM
from . import tdvp as T


def scaled_model(model, V, s):
    """`model` with transfer integral V and every mode (local and bond)
    scaled: omega -> s omega, g -> g / sqrt(s)."""
    if not (s > 0 and math.isfinite(s)):
        raise ValueError("frequency scale must be positive")
    f = 1.0 / math.sqrt(s)
    return dataclasses.replace(model, V=float(V),
                               omega_loc=[s * w for w in model.omega_loc],
                               g_loc=[f * g for g in model.g_loc],
                               omega_nl=[s * w for w in model.omega_nl],
                               g_nl=[f * g for g in model.g_nl])


def mass_scale(mass_ratio):
    """Frequency scale s of replacing a mass m by m' = mass_ratio * m."""
    return 1.0 / math.sqrt(mass_ratio)


def mobility_sweep(model, points, n_imag, n_grow, D, dt, n_steps, cutoff=1e-10, tol=1e-14,
                   mmax=40):
    """(mu in a.u., ln Z) for each (beta, V, s) point: Psi_beta, C(t) and the
    Kubo mobility of the scaled model."""
    mus, logzs = [], []
    for beta, V, s in points:
        m = scaled_model(model, V, s)
        Hw, Jw = OM.hamiltonian_mpo(m), OM.current_mpo(m)
        psi, logz = T.thermal_prep(m, Hw, beta, n_imag, n_grow, D, cutoff=cutoff, tol=tol,
                                   mmax=mmax)
        C = T.corr_current(Hw, Jw, psi, D, dt, n_steps, cutoff=cutoff, tol=tol, mmax=mmax)
        mus.append(An.mobility(C, dt, beta, m.e0)[0])
        logzs.append(logz)
    return np.array(mus), np.array(logzs)


def mobility_grad(model, beta, n_imag, n_grow, D, dt, n_steps, cutoff=1e-10, tol=1e-14,
                  mmax=40, rel_step=1e-4):
    """mu and its central finite differences in every shared mode parameter:
    {"omega_loc", "g_loc", "omega_nl", "g_nl"} -> arrays of d mu / d x, with
    step rel_step |x| (rel_step for x = 0)."""
    def mu_of(m):
        return mobility_sweep(m, [(beta, m.V, 1.0)], n_imag, n_grow, D, dt, n_steps,
                              cutoff=cutoff, tol=tol, mmax=mmax)[0][0]

    mu0 = mu_of(model)
    grads = {}
    for name in ("omega_loc", "g_loc", "omega_nl", "g_nl"):
        vals = list(getattr(model, name))
        out = []
        for i, x in enumerate(vals):
            h = rel_step * (abs(x) if x != 0 else 1.0)
            up = dataclasses.replace(model, **{name: vals[:i] + [x + h] + vals[i + 1:]})
            dn = dataclasses.replace(model, **{name: vals[:i] + [x - h] + vals[i + 1:]})
            out.append((mu_of(up) - mu_of(dn)) / (2 * h))
        grads[name] = np.array(out)
    return mu0, grads


def isotope_derivative(model, grads):
    """d mu / d ln m when every mode frequency scales as m^(-1/2) with g^2 omega
    fixed (chain rule through omega -> s omega, g -> g / sqrt(s), s = m^(-1/2)):
    -1/2 sum omega d mu/d omega + 1/4 sum g d mu/d g."""
    d = 0.0
    for w_name, g_name in (("omega_loc", "g_loc"), ("omega_nl", "g_nl")):
        d += -0.5 * float(np.dot(getattr(model, w_name), grads[w_name]))
        d += 0.25 * float(np.dot(getattr(model, g_name), grads[g_name]))
    return d
