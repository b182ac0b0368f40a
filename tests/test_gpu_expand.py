"""Bond expansion of the one-site TDVP step on the GPU (ftd_tdvp_step_expand
and the expanding imaginary-time preparation) against the float64 oracle.

The expansion adds directions with zero coefficients, whose basis within the
added span is fixed only up to a unitary (the singular vectors' phases), so
tensors are compared through gauge-invariant quantities: the represented
state (linear probes), bond dimensions, norms, energies and ln Z."""
import sys

import numpy as np
import pytest

from helpers import download_mps, mps_rel_distance, random_mps, small_model
from oracle import model as Mdl
from oracle import mpo as OM
from oracle import tdvp as T
from paper_2003_13245_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _start(seed, D0, n_nl=1):
    m = small_model(n_mol=3, n_loc=1, n_nl=n_nl, levels=3)
    dims = Mdl.site_dims(m)
    return m, dims, OM.hamiltonian_mpo(m), random_mps(dims, D0, np.random.default_rng(seed), 0)


def test_expansion_at_zero_time_keeps_the_state(ctx):
    from paper_2003_13245_amd import api
    m, dims, Hw, host = _start(3, 3)
    H, _ = api.mpo_build(ctx, m)
    g = api.mps_from_host(ctx, host.A)
    api.tdvp_step_expand(ctx, H, g, 12, 1e-10, dt_real=0.0)
    o = host.copy()
    T.tdvp_step(o, Hw, 0.0, expand=(12, 1e-10))
    gb = g.info()["bond_dims"]
    say(f"[expand] bonds {host.bond_dims()} -> gpu {gb}, oracle {o.bond_dims()}")
    assert gb == o.bond_dims()
    out = download_mps(g, dims)
    d_state = mps_rel_distance(out, host)
    say(f"[expand] zero-time state change {d_state:.1e}")
    assert d_state < 1e-13


@pytest.mark.parametrize("name,z", [("real", -0.15j), ("imag", -0.05)])
def test_expanded_steps_match_oracle(ctx, name, z):
    """Five steps with expansion from a common low-bond state: the same bond
    dimensions and the same state as the oracle's (1e-11), norm and energy
    conserved in real time."""
    from paper_2003_13245_amd import api
    m, dims, Hw, host = _start(5, 3)
    H, _ = api.mpo_build(ctx, m)
    g = api.mps_from_host(ctx, host.A)
    o = host.copy()
    e0 = T.overlap(o, Hw, o).real
    for k in range(5):
        if z.imag:
            api.tdvp_step_expand(ctx, H, g, 10, 1e-10, dt_real=-z.imag)
        else:
            api.tdvp_step_expand(ctx, H, g, 10, 1e-10, dt_imag=-z.real)
        T.tdvp_step(o, Hw, z, expand=(10, 1e-10))
        assert g.info()["bond_dims"] == o.bond_dims(), k
    out = download_mps(g, dims)
    dist = mps_rel_distance(out, o)
    say(f"[expand] {name}: bonds {o.bond_dims()}, gpu/oracle state distance {dist:.1e}")
    assert dist < 1e-11
    if name == "real":
        n = T.norm(out)
        e = T.overlap(out, Hw, out).real
        assert abs(n - 1.0) < 1e-12 and abs(e - e0) < 1e-10 * max(1.0, abs(e0))


def test_expanding_preparation_reaches_D_and_matches_oracle(ctx):
    """The tiny ring (N = 4, 6 levels) prepared with one growth step and then
    expanding one-site TDVP steps up to D = 16: every bond reaches
    min(D, its full rank) on both sides, and ln Z and the state agree with
    the oracle's within 30x the oracle's own spread between its two SVD
    drivers (and at least 1e-10)."""
    from paper_2003_13245_amd import api
    wl = W.tiny_fp64()
    m, r = wl.model, wl.run
    dims = Mdl.site_dims(m)
    Hw = OM.hamiltonian_mpo(m)
    psi_o, lz_o = T.thermal_prep(m, Hw, r.beta, r.n_imag, 1, r.D, expand_tol=1e-8)
    T.SVD_DRIVER = "gesvd"
    try:
        psi_v, lz_v = T.thermal_prep(m, Hw, r.beta, r.n_imag, 1, r.D, expand_tol=1e-8)
    finally:
        T.SVD_DRIVER = "gesdd"
    H, _ = api.mpo_build(ctx, m)
    psi_g, lz_g = api.thermal_prep(ctx, H, r.beta, r.n_imag, 1, r.D, expand_tol=1e-8)
    full = T.full_bonds(dims)
    gb = psi_g.info()["bond_dims"]
    say(f"[expand] prep bonds gpu {gb} oracle {psi_o.bond_dims()}; dlnZ {abs(lz_g - lz_o):.1e} "
        f"(oracle drivers {abs(lz_v - lz_o):.1e})")
    assert gb == psi_o.bond_dims()
    assert gb == [int(min(r.D, f)) for f in full]
    spread = mps_rel_distance(psi_v, psi_o)
    dist = mps_rel_distance(download_mps(psi_g, dims), psi_o)
    say(f"[expand] prep state distance {dist:.1e} (oracle drivers {spread:.1e})")
    assert abs(lz_g - lz_o) < max(1e-10, 30 * abs(lz_v - lz_o))
    assert dist < max(1e-10, 30 * spread)
