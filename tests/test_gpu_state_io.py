"""Checkpoint and resume, run-to-run determinism and failure handling of the
HIP library (all through the C ABI).

* A state written by ftd_mps_save and read by ftd_mps_load is the same state
  bit for bit, and 2K real-time steps run straight give the same bits as K
  steps, save, load, K steps.
* Two identical runs (preparation, j|Psi>, C(t)) give identical bits: every
  reduction in the library has a fixed order.
* Failures come back as status codes and leave the context usable: a device
  allocator that refuses (FTD_ENOMEM), a non-finite tensor (FTD_ENOCONV), a
  Krylov space too small for the tolerance (FTD_ENOCONV), malformed state
  files (FTD_EINVAL).  No kernel is made to fault: each condition is set up
  from the host and every kernel runs to its normal end."""
import os
import sys

import numpy as np
import pytest

from helpers import download_mps, random_mps, small_model
from oracle import model as Mdl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _tiny(ctx):
    from paper_2003_13245_amd import api
    m = small_model(n_mol=3, n_loc=1, n_nl=1, levels=3)
    H, J = api.mpo_build(ctx, m)
    psi, logz = api.thermal_prep(ctx, H, 1.0, 6, 2, 12)
    return m, H, J, psi


def _same_bits(a, b, dims):
    A, B = download_mps(a, dims), download_mps(b, dims)
    assert A.log_norm == B.log_norm
    for x, y in zip(A.A, B.A):
        assert x.shape == y.shape
        assert np.array_equal(x.view(np.float64), y.view(np.float64))


def test_save_load_roundtrip_is_exact(ctx, tmp_path):
    from paper_2003_13245_amd import api
    m, H, J, psi = _tiny(ctx)
    psi.set_precision("c64")
    path = tmp_path / "psi.ftdmps"
    psi.save(path)
    back = api.mps_load(ctx, path)
    assert back.info() == psi.info()
    _same_bits(psi, back, Mdl.site_dims(m))


def test_checkpoint_resume_gives_the_same_bits(ctx, tmp_path):
    """2K steps straight == K steps + save/load + K steps, bitwise."""
    from paper_2003_13245_amd import api
    m, H, J, psi = _tiny(ctx)
    dims = Mdl.site_dims(m)
    K, dt = 4, 0.1
    straight = psi.copy()
    for _ in range(2 * K):
        api.tdvp_step(ctx, H, straight, dt_real=dt)
    part = psi.copy()
    for _ in range(K):
        api.tdvp_step(ctx, H, part, dt_real=dt)
    path = tmp_path / "ckpt.ftdmps"
    part.save(path)
    del part
    resumed = api.mps_load(ctx, path)
    for _ in range(K):
        api.tdvp_step(ctx, H, resumed, dt_real=dt)
    _same_bits(straight, resumed, dims)
    phi = api.apply_compress(ctx, J, psi, 12)
    assert api.overlap(ctx, straight, J, phi) == api.overlap(ctx, resumed, J, phi)


def test_run_to_run_determinism(ctx):
    """The same preparation and C(t) twice: identical bits."""
    from paper_2003_13245_amd import api
    m = small_model(n_mol=3, n_loc=1, n_nl=1, levels=3)
    out = []
    for _ in range(2):
        H, J = api.mpo_build(ctx, m)
        psi, logz = api.thermal_prep(ctx, H, 1.0, 6, 2, 12)
        C = api.corr_current(ctx, H, J, psi, 12, 0.1, 6)
        out.append((logz, C))
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])


def test_set_site_replaces_one_tensor(ctx):
    from paper_2003_13245_amd import api
    m, H, J, psi = _tiny(ctx)
    dims = Mdl.site_dims(m)
    host = download_mps(psi, dims)
    rng = np.random.default_rng(4)
    t = rng.standard_normal(host.A[2].shape) + 1j * rng.standard_normal(host.A[2].shape)
    psi.set_site(2, t)
    back = download_mps(psi, dims)
    assert np.array_equal(back.A[2], t)
    assert np.array_equal(back.A[1], host.A[1])
    with pytest.raises(api.FtdError) as e:
        psi.set_site(2, t[:, :, :, :-1])
    assert e.value.code == 1
    bad = t.copy()
    bad[0, 0, 0, 0] = np.nan
    with pytest.raises(api.FtdError):
        psi.set_site(2, bad)


def test_malformed_state_files_are_rejected(ctx, tmp_path):
    from paper_2003_13245_amd import api
    m, H, J, psi = _tiny(ctx)
    good = tmp_path / "good.ftdmps"
    psi.save(good)
    raw = good.read_bytes()
    cases = {"missing": None, "short": raw[: len(raw) // 2], "magic": b"XXXXXXXX" + raw[8:],
             "trailing": raw + b"\0"}
    for name, data in cases.items():
        p = tmp_path / f"{name}.ftdmps"
        if data is not None:
            p.write_bytes(data)
        with pytest.raises(api.FtdError) as e:
            api.mps_load(ctx, p)
        assert e.value.code == 1, name


class _LimitedAllocator:
    """torch's caching allocator behind a switch: after `budget` further
    allocations it refuses (returns 0), as a full device would."""

    def __init__(self, device=0):
        import torch
        self.torch, self.device = torch, device
        self.budget = None
        self.count = 0

    def alloc(self, nbytes):
        if self.budget is not None and self.count >= self.budget:
            return 0
        self.count += 1
        stream = self.torch.cuda.current_stream(self.device).cuda_stream
        return self.torch.cuda.caching_allocator_alloc(nbytes, self.device, stream)

    def free(self, ptr):
        self.torch.cuda.caching_allocator_delete(ptr)


def test_allocation_failure_is_reported_and_recovered():
    from paper_2003_13245_amd import api
    al = _LimitedAllocator()
    c = api.Context(0, allocator=al)
    m = small_model(n_mol=3, n_loc=1, n_nl=1, levels=3)
    H, J = api.mpo_build(c, m)
    for budget in (0, 5, 40):
        al.count, al.budget = 0, budget
        with pytest.raises(api.FtdError) as e:
            api.thermal_prep(c, H, 1.0, 6, 2, 12)
        assert e.value.code == 2, (budget, e.value)
        say(f"[io] allocation refused after {budget}: {e.value}")
    al.budget = None
    psi, logz = api.thermal_prep(c, H, 1.0, 6, 2, 12)
    ref = api.Context(0)
    H2, _ = api.mpo_build(ref, m)
    psi2, logz2 = api.thermal_prep(ref, H2, 1.0, 6, 2, 12)
    assert logz == logz2
    c.close()


def test_non_finite_state_and_short_krylov_space(ctx):
    from paper_2003_13245_amd import api
    m = small_model(n_mol=3, n_loc=1, n_nl=0, levels=3)
    dims = Mdl.site_dims(m)
    H, J = api.mpo_build(ctx, m)
    rng = np.random.default_rng(2)
    host = random_mps(dims, 6, rng, 0)
    ok = api.mps_from_host(ctx, host.A)
    with pytest.raises(api.FtdError) as e:
        api.tdvp_step(ctx, H, ok, dt_real=0.1, tol=1e-14, mmax=1)
    assert e.value.code == 4
    host.A[3] = host.A[3].copy()
    host.A[3][0, 0, 0, 0] = np.nan
    bad = api.mps_from_host(ctx, host.A)
    with pytest.raises(api.FtdError) as e:
        api.tdvp_step(ctx, H, bad, dt_real=0.1)
    assert e.value.code == 4
    # the context still works afterwards
    good = api.mps_from_host(ctx, random_mps(dims, 6, rng, 0).A)
    api.tdvp_step(ctx, H, good, dt_real=0.1)
    assert abs(good.norm2() - 1.0) < 1e-12


def test_handles_may_outlive_their_context():
    """ftd_ctx_destroy before the handles made on the context: the context
    stays alive until the last handle is destroyed (no use after free), in
    either order of handle destruction."""
    import gc
    from paper_2003_13245_amd import _abi, api
    for order in (0, 1):
        c = api.Context(0)
        m = small_model(n_mol=3, n_loc=1, n_nl=0, levels=2)
        H, J = api.mpo_build(c, m)
        psi, _ = api.thermal_prep(c, H, 1.0, 4, 1, 6)
        _abi.lib.ftd_ctx_destroy(c.h)
        c.h = None
        objs = [H, J, psi] if order == 0 else [psi, J, H]
        for o in objs:
            o._release()
        del objs, H, J, psi, c
        gc.collect()
