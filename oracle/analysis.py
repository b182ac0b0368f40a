"""Post-processing of C(t): Kubo mobility, hopping-limit C(t), mean free path.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import math

import numpy as np

# e a0^2 / hbar in m^2/(V s) (CODATA 2018), times 1e4 for cm^2/(V s)
_E = 1.602176634e-19
_A0 = 5.29177210903e-11
_HBAR = 1.054571817e-34
MOBILITY_AU_CM2VS = _E * _A0 ** 2 / _HBAR * 1e4


def mobility(C, dt, beta, e0=1.0):
    """Kubo formula: mu = (1/(2 k_B T e0)) int_{-inf}^{inf} C(t) dt.
    With C(-t) = conj(C(t)) the integral is 2 int_0^tmax Re C dt, cut at the
    last sample (the paper integrates up to the region before the
    recurrence).  Trapezoid rule on the uniform grid.  Returns (a.u., cm^2/Vs)."""
    C = np.asarray(C)
    if C.size < 2:
        raise ValueError("need at least two samples")
    re = C.real
    integral = dt * (re.sum() - 0.5 * (re[0] + re[-1]))
    mu = beta / e0 * integral
    return mu, mu * MOBILITY_AU_CM2VS


def bose(omega, beta):
    return 1.0 / math.expm1(beta * omega) if beta * omega < 700 else 0.0


def fgr_corr(t, V, omega, g, beta, e0=1.0, R=1.0):
    """Hopping-limit (V -> 0) current correlation of the Holstein chain, derived
    for the C(t) and j of the paper: a carrier hops to either neighbour (factor
    2) and the modes of both molecules are displaced (g^2 twice):
      C(t) = 2 (e0 R V)^2 exp(-sum_m 2 g_m^2 [(2n_m+1) - (n_m+1) e^{-i w_m t}
                                               - n_m e^{i w_m t}])
    The printed hopping-limit formula has the complex-conjugate time
    dependence and no factors of 2; its real part, and so the mobility, agrees
    with this form when g^2 there denotes the pair Huang-Rhys factor."""
    t = np.asarray(t, dtype=float)
    expo = np.zeros_like(t, dtype=complex)
    for w, gm in zip(omega, g):
        n = bose(w, beta)
        expo += 2 * gm ** 2 * ((2 * n + 1) - (n + 1) * np.exp(-1j * w * t)
                               - n * np.exp(1j * w * t))
    return 2 * (e0 * R * V) ** 2 * np.exp(-expo)


def tight_binding_corr(N, V, beta, e0=1.0, R=1.0):
    """g = 0: j commutes with H, C(t) = <j^2> = (2 e0 V R)^2 <sin^2 k>."""
    k = 2 * np.pi * np.arange(N) / N
    w = np.exp(-beta * 2 * V * np.cos(k))
    return (2 * e0 * V * R) ** 2 * float((np.sin(k) ** 2 * w).sum() / w.sum())


def mean_free_path(C, dt):
    """l_mfp = v tau with v = sqrt(<j j>) and tau = (1/2) int |Re C/Re C(0)| dt
    over (-tmax, tmax), i.e. int_0^tmax |Re C / Re C(0)| dt (trapezoid)."""
    C = np.asarray(C)
    v = math.sqrt(C[0].real)
    r = np.abs(C.real / C[0].real)
    tau = dt * (r.sum() - 0.5 * (r[0] + r[-1]))
    return v * tau, v, tau


def coherent_length(sigma):
    """L = (sum_ij |sigma_ij|)^2 / (N sum_ij |sigma_ij|^2) of the reduced
    electronic density sigma (N x N): 1 for sigma = I/N (localised), N for
    |sigma_ij| = 1/N (delocalised)."""
    a = np.abs(np.asarray(sigma))
    N = a.shape[0]
    return float(a.sum() ** 2 / (N * (a * a).sum()))
