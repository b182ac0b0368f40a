"""Seeded synthetic workloads for the finite-temperature TD-DMRG mobility path.

This module produces *inputs only*: model parameters in atomic units and run
settings (inverse temperature, step counts, bond dimension).  It holds none of
the method's arithmetic (no operators, no propagation, no observables), so both
the CPU oracle and the HIP library consume exactly the same numbers.

The model is the one-dimensional multi-mode Holstein chain of Eq. (1) of the
paper, optionally with the off-diagonal (Peierls) coupling of the
Holstein-Peierls Hamiltonian given near the end of the main text.  The rubrene
parameter tables live in the paper's supporting information, which is not
available, so the rubrene-shaped workloads draw frequencies log-uniformly over
the span the paper quotes (84-1594 cm^-1 for rubrene's retained modes, widened
to 50-1600 cm^-1 here), fix the total local reorganisation energy, and set the
Peierls couplings from a target transfer-integral fluctuation.

Unit conventions: hbar = e0 = k_B = 1 (atomic units); CODATA 2018 constants.
"""
from __future__ import annotations

import dataclasses
import json
import math
from typing import List, Optional

import numpy as np

SEED = 200313245

# CODATA 2018
HARTREE_MEV = 27211.386245988
HARTREE_CM = 219474.6313632
KB_HARTREE_PER_K = 3.166811563e-6
AU_TIME_FS = 0.024188843265857
BOHR_M = 5.29177210903e-11
HARTREE_EV = 27.211386245988
AU_TIME_S = 2.4188843265857e-17


def mev(x: float) -> float:
    """meV -> Hartree."""
    return x / HARTREE_MEV


def cm1(x: float) -> float:
    """cm^-1 -> Hartree."""
    return x / HARTREE_CM


def fs(x: float) -> float:
    """femtoseconds -> atomic time units."""
    return x / AU_TIME_FS


def beta_of_T(T_kelvin: float) -> float:
    """Inverse temperature 1/(k_B T) in 1/Hartree."""
    return 1.0 / (KB_HARTREE_PER_K * T_kelvin)


@dataclasses.dataclass
class Model:
    """Parameters of the (Holstein-)Peierls chain, atomic units.

    n_mol       number of molecules N on the chain
    periodic    1: periodic chain (wrap bond N-1 -> 0), 0: open
    omega_loc   [M_loc] local-mode frequencies, shared by all molecules
    g_loc       [M_loc] dimensionless local (Holstein) couplings g^(1)
    omega_nl    [M_nl] non-local (bond) mode frequencies, one set per bond
    g_nl        [M_nl] dimensionless Peierls couplings g^(2)
    levels_loc  harmonic-oscillator states kept per local mode
    levels_nl   harmonic-oscillator states kept per non-local mode
    V           transfer integral
    R           inter-molecular distance (enters the current operator)
    e0          carrier charge
    """
    n_mol: int
    periodic: int
    omega_loc: List[float]
    g_loc: List[float]
    omega_nl: List[float]
    g_nl: List[float]
    levels_loc: int
    levels_nl: int
    V: float
    R: float = 1.0
    e0: float = 1.0

    @property
    def n_loc(self) -> int:
        return len(self.omega_loc)

    @property
    def n_nl(self) -> int:
        return len(self.omega_nl)

    def to_json(self) -> str:
        return json.dumps(dataclasses.asdict(self), sort_keys=True)


@dataclasses.dataclass
class Run:
    """Run settings for one C(t) evaluation."""
    beta: float
    n_imag: int          # imaginary-time steps to reach beta/2
    n_grow: int          # of which the first n_grow grow the bond dimension
    D: int               # MPS bond dimension of the purified state and of j|Psi>
    dt: float            # real-time step
    n_steps: int         # real-time steps
    krylov_tol: float = 1e-14
    krylov_mmax: int = 40
    cutoff: float = 1e-10  # relative singular-value cutoff for compression
    expand_tol: float = 0.0  # bond expansion threshold of the one-site TDVP steps (0: off)
    T_K: float = 0.0     # temperature in kelvin (0: model units, beta given directly)
    dt_fs: float = 0.0   # real-time step in femtoseconds (0: model units)
    # the imaginary-time preparation of Psi_beta: contraction precision and
    # Krylov tolerance (expand_tol applies to it)
    prep_precision: str = "c128"
    prep_krylov_tol: float = 1e-14


@dataclasses.dataclass
class Workload:
    name: str
    model: Model
    run: Run
    precision: str       # "c128", "c64" or "bf16x3"
    note: str = ""


def _logu(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))


def tiny_fp64() -> Workload:
    """N=4, one local mode (omega=1, g=1), V=1, 6 levels, D=16, beta=1 in 20
    imaginary steps, t=0..10 with dt=0.1 (model units)."""
    m = Model(n_mol=4, periodic=1, omega_loc=[1.0], g_loc=[1.0], omega_nl=[],
              g_nl=[], levels_loc=6, levels_nl=1, V=1.0)
    r = Run(beta=1.0, n_imag=20, n_grow=1, D=16, dt=0.1, n_steps=100)
    return Workload("holstein_n4_d6_D16", m, r, "c128")


def fp64_chain(beta: float = 1.0) -> Workload:
    """N=11, two local modes with omega 0.5 and 1.5, Huang-Rhys S ~ U[0.2, 1],
    g = sqrt(S), V=1, 8 levels, D=64, dtau=0.025, t=0..40 with dt=0.05."""
    rng = np.random.default_rng(SEED)
    omega = [0.5, 1.5]
    S = rng.uniform(0.2, 1.0, size=2)
    g = [float(math.sqrt(s)) for s in S]
    m = Model(n_mol=11, periodic=1, omega_loc=omega, g_loc=g, omega_nl=[],
              g_nl=[], levels_loc=8, levels_nl=1, V=1.0)
    n_imag = int(round(beta / 2 / 0.025))
    r = Run(beta=beta, n_imag=n_imag, n_grow=1, D=64, dt=0.05, n_steps=800)
    return Workload(f"holstein_n11_d8_D64_beta{beta:g}", m, r, "c128")


def _peierls_g(V, dV_over_V, omega_nl, beta):
    """g^(2) such that the thermal transfer-integral variance
    sum_m (g_m omega_m)^2 coth(beta omega_m / 2) equals (dV_over_V * V)^2,
    split equally over the non-local modes."""
    n = len(omega_nl)
    out = []
    for w in omega_nl:
        coth = 1.0 / math.tanh(beta * w / 2.0)
        out.append(float(dV_over_V * V / math.sqrt(n) / (w * math.sqrt(coth))))
    return out


def rubrene_shaped(n_mol=21, n_loc=4, n_nl=1, levels=10, D=128, T=300.0,
                   t_fs=200.0, dt_fs=0.5, lam_meV=150.0, V_meV=80.0,
                   dV_over_V=0.2, precision="c64", n_imag=40) -> Workload:
    """Rubrene-shaped Holstein-Peierls chain: local frequencies log-uniform in
    [50, 1600] cm^-1 (sorted), total local reorganisation sum g^2 omega =
    lam_meV split equally, one set of non-local modes per bond log-uniform in
    [50, 1600] cm^-1 with couplings from dV/V at temperature T."""
    rng = np.random.default_rng(SEED)
    w_loc = np.sort(_logu(rng, 50.0, 1600.0, n_loc))
    w_nl = _logu(rng, 50.0, 1600.0, n_nl) if n_nl else np.zeros(0)
    omega_loc = [cm1(float(w)) for w in w_loc]
    lam = mev(lam_meV) / n_loc
    g_loc = [float(math.sqrt(lam / w)) for w in omega_loc]
    beta = beta_of_T(T)
    V = mev(V_meV)
    omega_nl = [cm1(float(w)) for w in w_nl]
    g_nl = _peierls_g(V, dV_over_V, omega_nl, beta) if n_nl else []
    m = Model(n_mol=n_mol, periodic=1, omega_loc=omega_loc, g_loc=g_loc,
              omega_nl=omega_nl, g_nl=g_nl, levels_loc=levels,
              levels_nl=levels, V=V)
    dt = fs(dt_fs)
    n_steps = int(round(t_fs / dt_fs))
    # Psi_beta is prepared in float64 whatever the precision of the real-time
    # steps: a preparation with complex-FP32 contractions (Krylov tolerance
    # 1e-8, expansion threshold 1e-5) ends at a state with ln Z about 24 lower
    # on the 21-molecule ring
    r = Run(beta=beta, n_imag=n_imag, n_grow=1, D=D, dt=dt, n_steps=n_steps,
            krylov_tol=1e-14 if precision == "c128" else 1e-8,
            expand_tol=1e-8, T_K=T, dt_fs=dt_fs)
    name = f"hp_n{n_mol}_loc{n_loc}_nl{n_nl}_d{levels}_D{D}_T{T:g}"
    return Workload(name, m, r, precision)


def adjoint_chain() -> Workload:
    """N=11, three local modes log-uniform in [100, 1600] cm^-1, V=80 meV,
    8 levels, D=64, T=300 K, 100 real steps of 0.5 fs."""
    rng = np.random.default_rng(SEED)
    w = np.sort(_logu(rng, 100.0, 1600.0, 3))
    omega = [cm1(float(x)) for x in w]
    lam = mev(150.0) / 3
    g = [float(math.sqrt(lam / x)) for x in omega]
    m = Model(n_mol=11, periodic=1, omega_loc=omega, g_loc=g, omega_nl=[],
              g_nl=[], levels_loc=8, levels_nl=1, V=mev(80.0))
    r = Run(beta=beta_of_T(300.0), n_imag=40, n_grow=1, D=64, dt=fs(0.5),
            n_steps=100, T_K=300.0, dt_fs=0.5)
    return Workload("holstein_n11_loc3_d8_D64_T300", m, r, "c128")


def large_rubrene_shaped(T=300.0) -> Workload:
    """N=31, 6 local + 2 non-local modes per bond, 12 levels, D=256, to 300 fs."""
    return rubrene_shaped(n_mol=31, n_loc=6, n_nl=2, levels=12, D=256, T=T,
                          t_fs=300.0, dt_fs=0.5, precision="c64")


def headline() -> Workload:
    """The workload the throughput figure is quoted on: rubrene-shaped
    Holstein-Peierls chain, N=21, 4 local + 1 non-local mode, 10 levels,
    D=128, T=300 K."""
    return rubrene_shaped()


def random_site_tensor(rng, Dl, d, Dr, dtype=np.complex128):
    """Complex Gaussian tensor [Dl, d, d, Dr] (physical P leg, then Q leg)."""
    shape = (Dl, d, d, Dr)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return x.astype(dtype)


def random_env(rng, w, D, dtype=np.complex128):
    """Complex Gaussian environment block [w, D, D]."""
    x = rng.standard_normal((w, D, D)) + 1j * rng.standard_normal((w, D, D))
    return x.astype(dtype)
