"""The mobility gradient on the GPU (central finite differences through the
whole GPU path, in every shared mode frequency and coupling) against the
oracle's finite differences with the same steps, on a 3-molecule Holstein
ring with two local modes; and the isotope derivative from the gradient
against the GPU sweep's slope in the frequency scale (chain rule).

Finite differences of the truncated method are meaningful only where its
truncation decisions are stable between the +h and -h runs.  On the
3-molecule Holstein-Peierls ring at D = 12 they are not for the bond-mode
frequency: there the prepared state keeps symmetry-degenerate singular pairs
near s/s_max ~ 1e-5 at the bond-dimension cut, rounding splits them by ~1e-7
relative (above the 1e-8 multiplet rule), and the GPU at omega_nl (1 + 1e-4)
kept a different rank than the oracle (ln Z differs by 1.6e-9, mu by 3.4e-4)."""
import math

import numpy as np
import pytest

from helpers import small_model
from oracle import sweep as S

pytestmark = pytest.mark.gpu

RUN = dict(n_imag=6, n_grow=6, D=12, dt=0.1, n_steps=10)


def say(*a):
    print(*a, flush=True)


def test_mobility_gradient_matches_oracle(ctx):
    from paper_2003_13245_amd import api
    m = small_model(n_mol=3, n_loc=2, n_nl=0, levels=3)
    mu_g, gr_g = api.mobility_grad(ctx, m, 1.0, rel_step=1e-4, **RUN)
    mu_o, gr_o = S.mobility_grad(m, 1.0, rel_step=1e-4, **RUN)
    scale = max(abs(v) for k in gr_o for v in gr_o[k])
    for k in gr_o:
        say(f"[grad] d mu / d {k}: gpu {gr_g[k]}, oracle {gr_o[k]}")
        # each mu agrees to ~1e-10 relative; over a step of 1e-4 |x| that is
        # ~1e-6 of the gradient scale
        assert np.allclose(gr_g[k], gr_o[k], rtol=0, atol=1e-4 * scale), k
    assert abs(mu_g - mu_o) <= 1e-8 * abs(mu_o)
    iso = S.isotope_derivative(m, {k: np.asarray(v) for k, v in gr_g.items()})
    h = 1e-4
    mus, _ = api.mobility_sweep(ctx, m, [(1.0, m.V, 1 + h), (1.0, m.V, 1 - h)], **RUN)
    slope = -0.5 * (mus[0] - mus[1]) / (math.log(1 + h) - math.log(1 - h))
    say(f"[grad] d mu / d ln m: chain rule {iso:.10f}, sweep slope {slope:.10f}")
    assert abs(slope - iso) <= 1e-5 * abs(iso)


def test_gradient_rejects_bad_step(ctx):
    from paper_2003_13245_amd import api
    m = small_model(n_mol=3, n_loc=2, n_nl=0, levels=3)
    for step in (0.0, 0.5, float("nan")):
        with pytest.raises(api.FtdError):
            api.mobility_grad(ctx, m, 1.0, rel_step=step, **RUN)


def test_mobility_autograd_function(ctx):
    """torch autograd through the Mobility function: backward gives mu-bar
    times ftd_mobility_grad's gradient, and the chain rule through
    omega -> s omega, g -> g / sqrt(s) gives the frequency-scaling derivative
    at s = 1, d mu / d s = sum_k omega_k dmu/domega_k - (1/2) sum_k g_k dmu/dg_k."""
    import torch
    from paper_2003_13245_amd import api
    m = small_model(n_mol=3, n_loc=2, n_nl=0, levels=3)
    mu_ref, gr = api.mobility_grad(ctx, m, 1.0, rel_step=1e-4, **RUN)
    w0 = torch.tensor(m.omega_loc, dtype=torch.float64)
    g0 = torch.tensor(m.g_loc, dtype=torch.float64)
    s = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    empty = torch.zeros(0, dtype=torch.float64)
    mu = api.mobility_autograd(ctx, m, 1.0, w0 * s, g0 / torch.sqrt(s), empty, empty,
                               rel_step=1e-4, **RUN)
    assert abs(mu.item() - mu_ref) <= 1e-12 * abs(mu_ref)
    (2.5 * mu).backward()
    expect = 2.5 * (float(np.dot(m.omega_loc, gr["omega_loc"]))
                    - 0.5 * float(np.dot(m.g_loc, gr["g_loc"])))
    say(f"[grad] autograd d(2.5 mu)/ds {s.grad.item():.12g}, expected {expect:.12g}")
    assert abs(s.grad.item() - expect) <= 1e-10 * max(1.0, abs(expect))
