"""End-to-end GPU parity: imaginary-time preparation, j|Psi_beta>, real-time
C(t) and the mobility against the float64 oracle on the same seeded chains.

The pipeline is checked in two stages, each to a tolerance set by what the
oracle itself can resolve:

* preparation: the GPU's |Psi_beta> against the oracle's, as states (linear
  probes) and through ln Z;
* dynamics: C(t) from the *same* |Psi_beta> (the oracle's, uploaded; and the
  GPU's own, downloaded) on both sides.

Why not compare two independent pipelines tightly: the prepared state of the
tiny ring keeps singular values down to ~4e-9 of the largest plus exactly
degenerate pairs, and their directions are fixed by rounding.  One-site TDVP
then populates them.  The oracle shows this against itself: with LAPACK's
gesvd instead of gesdd (two valid SVDs) its own C(t) agrees to 1e-14 for six
steps and then departs to ~1e-4 within three more, while from a common
|Psi_beta> the swap moves C(t) by < 1e-12 over 20 steps.  The independent
pipeline difference is therefore reported and held only to a loose bound:
30x the oracle's own mobility spread between the two drivers (5e-6 to 6e-4
relative on the tiny ring), and at least 1e-3 relative.

Floors per step k are running maxima of |C' - C| / |C(0)| over the oracle
variants: a relative 1e-15 perturbation of the state; the other SVD driver;
and every gauge QR factor perturbed by a fixed relative STEP_DELTA = 1e-13,
the rounding level of one step of two float64 implementations fixed in
advance (about 1000 unit roundoffs: the dependent operations of a sweep).  The last variant is how the oracle itself amplifies differences of
the size by which two implementations differ per step (accumulation order,
CholeskyQR against Householder QR, the Krylov stop test); several steps of
these chains contain bursts that amplify them a hundredfold in one step.
Every floor comes from oracle runs alone; the measured distance between one
GPU step and one oracle step is reported and held below 1e-12 on its own.
The GPU must satisfy err(k) <= max(1e-10, 30 x floor(k)) at every step."""
import numpy as np
import pytest

from helpers import download_mps, mps_rel_distance, small_model
from oracle import analysis as An
from oracle import model as Mdl
from oracle import mpo as OM
from oracle import tdvp as T
from paper_2003_13245_amd import workloads as W

pytestmark = pytest.mark.gpu

# relative perturbation of every oracle gauge factor that stands for the
# per-step rounding difference of two float64 implementations (fixed a
# priori, not measured on the GPU)
STEP_DELTA = 1e-13


def say(*a):
    print(*a, flush=True)


def perturbed(psi, seed, scale=1e-15):
    rng = np.random.default_rng(seed)
    p = psi.copy()
    for k in range(len(p.A)):
        p.A[k] = p.A[k] * (1 + scale * rng.standard_normal(p.A[k].shape))
    return p


CASES = {
    # tiny ring (N=4, 6 levels, D=16), all imaginary steps by
    # propagation-and-compression
    "tiny_pc": dict(wl="tiny", n_imag=20, n_grow=20, steps=20, cutoff=1e-10),
    "tiny_pc_cut6": dict(wl="tiny", n_imag=20, n_grow=20, steps=20, cutoff=1e-6),
    # one growth step, then one-site TDVP in imaginary time
    "tiny_tdvp": dict(wl="tiny", n_imag=20, n_grow=1, steps=10, cutoff=1e-10),
    # adaptive growth (stops by the growth rule), then one-site TDVP
    "tiny_adaptive": dict(wl="tiny", n_imag=20, n_grow=-1, steps=10, cutoff=1e-10),
    # Holstein-Peierls ring
    "peierls": dict(wl="peierls", n_imag=6, n_grow=6, steps=10, cutoff=1e-10),
}


def workload(name):
    if name == "tiny":
        return W.tiny_fp64()
    m = small_model(n_mol=3, n_loc=1, n_nl=1, levels=3)
    return W.Workload("hp_n3", m, W.Run(beta=1.0, n_imag=6, n_grow=6, D=12, dt=0.1,
                                        n_steps=10), "c128")


class Case:
    """Oracle results for one case, computed once per session."""

    def __init__(self, name):
        cfg = CASES[name]
        self.name, self.cfg = name, cfg
        wl = workload(cfg["wl"])
        self.m, self.r = wl.model, wl.run
        self.cut = cfg["cutoff"]
        self.dims = Mdl.site_dims(self.m)
        self.Hw, self.Jw = OM.hamiltonian_mpo(self.m), OM.current_mpo(self.m)
        self.psi, self.logz = self.prep("gesdd")
        self.psi_v, self.logz_v = self.prep("gesvd")
        self.C = self.corr(self.psi)
        # the whole pipeline again with the other SVD driver: the oracle's own
        # spread of mu between two valid implementations
        self.C_v = self.corr(self.psi_v, "gesvd")
        self.mu = An.mobility(self.C, self.r.dt, self.r.beta)[0]
        self.mu_spread = abs(An.mobility(self.C_v, self.r.dt, self.r.beta)[0] - self.mu)
        # floor of the dynamics from a common state: the state perturbed and
        # the other SVD driver; the per-step variant is added by set_step_noise
        self.c0 = abs(self.C[0])
        self.base = np.maximum(np.abs(self.corr(perturbed(self.psi, 1)) - self.C),
                               np.abs(self.corr(self.psi, "gesvd") - self.C)) / self.c0
        self.noise = None
        self.set_floor(self.base)

    def set_floor(self, fl):
        self.floor = np.maximum.accumulate(fl)
        self.bound = np.maximum(1e-10, 30 * self.floor)

    def set_step_noise(self, delta):
        """Add the oracle's response to every gauge QR factor perturbed by a
        relative `delta` to the floor."""
        noise = float(delta)
        if self.noise == noise:
            return
        T.QR_NOISE = noise
        try:
            C_q = self.corr(self.psi)
        finally:
            T.QR_NOISE = 0.0
        self.noise = noise
        self.set_floor(np.maximum(self.base, np.abs(C_q - self.C) / self.c0))

    def prep(self, driver):
        T.SVD_DRIVER = driver
        try:
            c = self.cfg
            return T.thermal_prep(self.m, self.Hw, self.r.beta, c["n_imag"], c["n_grow"],
                                  self.r.D, cutoff=self.cut)
        finally:
            T.SVD_DRIVER = "gesdd"

    def corr(self, psi, driver="gesdd"):
        T.SVD_DRIVER = driver
        try:
            return T.corr_current(self.Hw, self.Jw, psi, self.r.D, self.r.dt,
                                  self.cfg["steps"], cutoff=self.cut)
        finally:
            T.SVD_DRIVER = "gesdd"

    def check_dynamics(self, C_gpu, C_ref, label):
        err = np.abs(np.asarray(C_gpu) - C_ref) / self.c0
        say(f"[e2e] {self.name} {label}: err   " + " ".join(f"{x:.0e}" for x in err))
        say(f"[e2e] {self.name} {label}: floor " + " ".join(f"{x:.0e}" for x in self.floor))
        bad = np.nonzero(err > self.bound)[0]
        assert bad.size == 0, [(int(k), float(err[k]), float(self.bound[k])) for k in bad]
        # mu is the trapezoid of Re C: its error is bounded by the summed bounds
        r = self.r
        w = np.full(err.size, r.dt)
        w[0] = w[-1] = r.dt / 2
        return float((self.bound * w).sum()) * self.c0 * r.beta + 1e-15


_CACHE = {}


def case(name):
    if name not in _CACHE:
        say(f"[e2e] {name}: oracle")
        _CACHE[name] = Case(name)
    return _CACHE[name]


def one_step_difference(ctx, c):
    """Relative distance between one real-time TDVP step on the GPU and one in
    the oracle, both from the oracle's prepared state."""
    from paper_2003_13245_amd import api
    H, _ = api.mpo_build(ctx, c.m)
    g = api.mps_from_host(ctx, c.psi.A)
    api.tdvp_step(ctx, H, g, dt_real=c.r.dt)
    o = c.psi.copy()
    o.log_norm = 0.0
    T.tdvp_step(o, c.Hw, -1j * c.r.dt)
    d = mps_rel_distance(download_mps(g, c.dims), o)
    say(f"[e2e] {c.name}: one-step GPU/oracle distance {d:.1e}")
    assert d < 1e-12, d
    return d


def gpu_prep(ctx, c):
    from paper_2003_13245_amd import api
    H, J = api.mpo_build(ctx, c.m)
    psi, logz = api.thermal_prep(ctx, H, c.r.beta, c.cfg["n_imag"], c.cfg["n_grow"], c.r.D,
                                 cutoff=c.cut)
    return H, J, psi, logz


@pytest.mark.parametrize("name", list(CASES))
def test_prep_vs_oracle(ctx, name):
    """The prepared thermal state and ln Z."""
    c = case(name)
    say(f"[e2e] {name}: gpu prep")
    _, _, psi_g, logz_g = gpu_prep(ctx, c)
    assert psi_g.info()["bond_dims"] == c.psi.bond_dims()
    host = download_mps(psi_g, c.dims)
    dist = mps_rel_distance(host, c.psi)
    spread = mps_rel_distance(c.psi_v, c.psi)
    dlogz = abs(logz_g - c.logz)
    say(f"[e2e] {name}: state distance {dist:.2e} (oracle drivers {spread:.2e}); "
        f"dlnZ {dlogz:.2e} (oracle drivers {abs(c.logz_v - c.logz):.2e})")
    assert dist < max(1e-10, 30 * spread), dist
    assert dlogz < max(1e-10, 30 * abs(c.logz_v - c.logz)), dlogz


@pytest.mark.parametrize("name", list(CASES))
def test_corr_from_common_state(ctx, name):
    """C(t) on the GPU from the oracle's |Psi_beta>, against the oracle."""
    from paper_2003_13245_amd import api
    c = case(name)
    one_step_difference(ctx, c)
    c.set_step_noise(STEP_DELTA)
    H, J = api.mpo_build(ctx, c.m)
    say(f"[e2e] {name}: gpu dynamics from the oracle state")
    psi = api.mps_from_host(ctx, c.psi.A)
    C_g = api.corr_current(ctx, H, J, psi, c.r.D, c.r.dt, c.cfg["steps"], cutoff=c.cut)
    mu_tol = c.check_dynamics(C_g, c.C, "common state")
    mu_o = An.mobility(c.C, c.r.dt, c.r.beta)[0]
    mu_g = api.mobility(C_g, c.r.dt, c.r.beta)[0]
    assert abs(mu_g - mu_o) <= mu_tol, (mu_g, mu_o, mu_tol)


@pytest.mark.parametrize("name", list(CASES))
def test_pipeline(ctx, name):
    """The whole GPU pipeline; dynamics checked against the oracle run from
    the GPU's own prepared state.  The independent-pipeline mobility is
    conditioning-limited (module docstring): it is held to 30x the oracle's
    own spread between the two SVD drivers, and never tighter than 1e-3."""
    from paper_2003_13245_amd import api
    c = case(name)
    one_step_difference(ctx, c)
    c.set_step_noise(STEP_DELTA)
    say(f"[e2e] {name}: gpu pipeline")
    H, J, psi_g, _ = gpu_prep(ctx, c)
    C_g = api.corr_current(ctx, H, J, psi_g, c.r.D, c.r.dt, c.cfg["steps"], cutoff=c.cut)
    host = download_mps(psi_g, c.dims)
    host.log_norm = 0.0
    C_og = c.corr(host)
    mu_tol = c.check_dynamics(C_g, C_og, "gpu state")
    mu_g = api.mobility(C_g, c.r.dt, c.r.beta)[0]
    mu_og = An.mobility(C_og, c.r.dt, c.r.beta)[0]
    assert abs(mu_g - mu_og) <= mu_tol, (mu_g, mu_og, mu_tol)
    mu_o = c.mu
    say(f"[e2e] {name}: mobility gpu {mu_g:.12g}, oracle {mu_o:.12g}, "
        f"rel diff {abs(mu_g - mu_o) / abs(mu_o):.1e} "
        f"(oracle driver spread {c.mu_spread / abs(mu_o):.1e})")
    assert abs(mu_g - mu_o) <= max(1e-3 * abs(mu_o), 30 * c.mu_spread)


def test_mobility_abi_matches_oracle(ctx):
    from paper_2003_13245_amd import api
    rng = np.random.default_rng(3)
    t = np.arange(257) * 0.05
    C = np.exp(-t / 2.0) * (1 + 0.2j * np.sin(t)) + 1e-3 * rng.standard_normal(t.size)
    for beta in (0.5, 1052.58):
        a = An.mobility(C, 0.05, beta)
        b = api.mobility(C, 0.05, beta)
        assert abs(a[0] - b[0]) < 1e-13 * abs(a[0]) and abs(a[1] - b[1]) < 1e-13 * abs(a[1])
