"""The mobility sweep on the GPU (batched runs over temperature, transfer
integral and isotope frequency scale) against the oracle's sweep on the
3-molecule Holstein-Peierls ring, whose single-point pipeline agrees with the
oracle to about 1e-10 in mu: per point mu and ln Z, and the isotope effect
mu(s)/mu(1) - 1 of a 12C -> 13C-like substitution (s = sqrt(12/13))."""
import math

import numpy as np
import pytest

from helpers import small_model
from oracle import sweep as S
from oracle import tdvp as T

pytestmark = pytest.mark.gpu

RUN = dict(n_imag=6, n_grow=6, D=12, dt=0.1, n_steps=10)


def say(*a):
    print(*a, flush=True)


def test_mobility_sweep_matches_oracle(ctx):
    from paper_2003_13245_amd import api
    m = small_model(n_mol=3, n_loc=1, n_nl=1, levels=3)
    s13 = math.sqrt(12.0 / 13.0)
    pts = [(1.0, m.V, 1.0), (1.0, m.V, s13), (2.0, 0.5, 1.0)]
    mu_o, lz_o = S.mobility_sweep(m, pts, **RUN)
    # the oracle's own spread between its two LAPACK SVD drivers
    T.SVD_DRIVER = "gesvd"
    try:
        mu_v, lz_v = S.mobility_sweep(m, pts, **RUN)
    finally:
        T.SVD_DRIVER = "gesdd"
    mu_g, lz_g = api.mobility_sweep(ctx, m, pts, **RUN)
    for i, p in enumerate(pts):
        say(f"[sweep] beta {p[0]} V {p[1]:.3f} s {p[2]:.4f}: mu gpu {mu_g[i]:.12g} oracle "
            f"{mu_o[i]:.12g}; lnZ gpu {lz_g[i]:.12g} oracle {lz_o[i]:.12g}")
        assert abs(mu_g[i] - mu_o[i]) <= max(1e-8 * abs(mu_o[i]), 30 * abs(mu_v[i] - mu_o[i]))
        assert abs(lz_g[i] - lz_o[i]) <= max(1e-10, 30 * abs(lz_v[i] - lz_o[i]))
    iso_g, iso_o = mu_g[1] / mu_g[0] - 1, mu_o[1] / mu_o[0] - 1
    say(f"[sweep] isotope effect gpu {iso_g:.9f} oracle {iso_o:.9f}")
    assert abs(iso_g - iso_o) <= 1e-7


def test_sweep_rejects_bad_points(ctx):
    from paper_2003_13245_amd import api
    m = small_model(n_mol=3, n_loc=1, n_nl=1, levels=3)
    for bad in ([(0.0, 1.0, 1.0)], [(1.0, 1.0, -1.0)], [(1.0, float("nan"), 1.0)]):
        with pytest.raises(api.FtdError):
            api.mobility_sweep(ctx, m, bad, **RUN)
