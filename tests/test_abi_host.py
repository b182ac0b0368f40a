"""Host-side checks of the C ABI (no GPU needed): the shared library loads,
exports every function include/ftdmrg.h declares, the Python binding covers
each of them under the same name, and the host-only entry points (mobility
quadrature, argument validation, error reporting) behave as declared."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ftdmrg.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(ftd_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def abi():
    import torch  # noqa: F401  (torch's HIP runtime must be loaded first)
    from paper_2003_13245_amd import build
    if not os.path.exists(build.OUT):
        build.build()
    from paper_2003_13245_amd import _abi
    return _abi


def test_header_declares_the_path():
    names = declared()
    for must in ("ftd_mpo_build", "ftd_thermal_prep", "ftd_tdvp_step", "ftd_apply_compress",
                 "ftd_overlap", "ftd_corr_current", "ftd_mobility", "ftd_heff_apply"):
        assert must in names
    assert len(names) >= 27


def test_library_exports_every_declared_symbol(abi):
    names = declared()
    missing = [n for n in names if not hasattr(abi.lib, n)]
    assert not missing, missing
    unbound = [n for n in names if n not in abi.SIGNATURES]
    assert not unbound, unbound
    extra = [n for n in abi.SIGNATURES if n not in names]
    assert not extra, extra


def test_mobility_host_entry_matches_oracle(abi):
    from oracle import analysis as An
    from paper_2003_13245_amd import api
    rng = np.random.default_rng(7)
    t = np.arange(101) * 0.1
    C = np.exp(-t) * (1 + 0.3j * np.cos(t)) + 1e-3 * rng.standard_normal(t.size)
    for beta, e0 in ((0.5, 1.0), (1052.58, 2.0)):
        a = An.mobility(C, 0.1, beta, e0)
        b = api.mobility(C, 0.1, beta, e0)
        assert abs(a[0] - b[0]) <= 1e-13 * abs(a[0])
        assert abs(a[1] - b[1]) <= 1e-13 * abs(a[1])


def test_mobility_rejects_bad_arguments(abi):
    from paper_2003_13245_amd import api
    with pytest.raises(abi.FtdError) as e:
        api.mobility(np.ones(1), 0.1, 1.0)
    assert e.value.code == abi.FTD_EINVAL
    with pytest.raises(abi.FtdError):
        api.mobility(np.ones(4), -0.1, 1.0)
    with pytest.raises(abi.FtdError):
        api.mobility(np.ones(4), 0.1, 1.0, e0=0.0)


def test_context_without_device_reports_error(abi):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import ctypes as C
    h = C.c_void_p()
    rc = abi.lib.ftd_ctx_create(0, None, None, C.byref(h))
    assert rc in (abi.FTD_EDEVICE, abi.FTD_EINVAL)
    assert not h.value
    assert abi.lib.ftd_last_error()


def test_mean_free_path_matches_oracle(abi):
    from oracle import analysis as An
    from paper_2003_13245_amd import api
    rng = np.random.default_rng(11)
    t = np.arange(301) * 0.05
    C = 2.5 * np.exp(-t / 3.0) * np.cos(0.7 * t) + 0.1j * np.sin(t) + 1e-3 * rng.standard_normal(t.size)
    ref = An.mean_free_path(C, 0.05)
    got = api.mean_free_path(C, 0.05)
    for a, b in zip(got, ref):
        assert abs(a - b) <= 1e-13 * abs(b)
    # e0 scales the velocity (j carries the charge)
    got2 = api.mean_free_path(C, 0.05, e0=2.0)
    assert abs(got2[1] - ref[1] / 2) < 1e-14 and abs(got2[2] - ref[2]) < 1e-13
    with pytest.raises(abi.FtdError):
        api.mean_free_path(-np.ones(4), 0.05)


@pytest.mark.parametrize("beta", [0.7, 40.0, 5000.0])
def test_fgr_corr_matches_oracle(abi, beta):
    from oracle import analysis as An
    from paper_2003_13245_amd import api
    t = np.linspace(0.0, 30.0, 257)
    om, g = [0.3, 1.1, 2.4], [0.8, 0.5, 0.2]
    ref = An.fgr_corr(t, 0.01, om, g, beta, e0=1.3, R=2.0)
    got = api.fgr_corr(t, 0.01, om, g, beta, e0=1.3, R=2.0)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    # t = 0: the exponent vanishes, C(0) = 2 (e0 R V)^2
    assert abs(got[0] - 2 * (1.3 * 2.0 * 0.01) ** 2) < 1e-16
    # no modes: constant
    flat = api.fgr_corr(t, 0.01, [], [], beta)
    assert np.allclose(flat, 2e-4, rtol=0, atol=1e-18)


def test_fgr_corr_rejects_bad_modes(abi):
    from paper_2003_13245_amd import api
    with pytest.raises(abi.FtdError):
        api.fgr_corr(np.zeros(3), 0.1, [0.0], [1.0], 1.0)
    with pytest.raises(abi.FtdError):
        api.fgr_corr(np.zeros(3), 0.1, [1.0], [1.0], 0.0)


def test_coherent_length_host_entry(abi):
    from oracle import analysis as An
    from paper_2003_13245_amd import api
    rng = np.random.default_rng(4)
    for n in (1, 3, 21):
        s = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        s = s @ s.conj().T
        a, b = An.coherent_length(s), api.coherent_length(s)
        assert abs(a - b) <= 1e-13 * a
    # the two limits the coherent-length definition names
    assert abs(api.coherent_length(np.eye(5) / 5) - 1.0) < 1e-14
    assert abs(api.coherent_length(np.full((5, 5), 0.2)) - 5.0) < 1e-13
    for bad in (np.zeros((3, 3)), np.full((2, 2), np.nan)):
        with pytest.raises(api.FtdError):
            api.coherent_length(bad)
    import ctypes
    L = ctypes.c_double()
    assert abi.lib.ftd_coherent_length(abi._dptr(np.zeros(2)), 0, ctypes.byref(L)) != 0


def test_site_vector_size_is_checked_before_the_call():
    """heff_apply / heff_expm hand x to the C ABI without a length: the binding
    refuses an x whose size is not the site's Dl d^2 Dr (an out-of-range site
    is left to the library's own error)."""
    import numpy as np
    from paper_2003_13245_amd import api

    class MpoStub:
        def info(self):
            return np.array([2, 3, 3, 2]), None

    class MpsStub:
        def info(self):
            return {"bond_dims": [4, 5, 6]}

    H, psi = MpoStub(), MpsStub()
    for site, n in ((0, 1 * 4 * 4), (1, 4 * 9 * 5), (2, 5 * 9 * 6), (3, 6 * 4 * 1)):
        api._check_site_vector(H, psi, site, np.zeros(n))
        with pytest.raises(ValueError):
            api._check_site_vector(H, psi, site, np.zeros(n + 1))
    api._check_site_vector(H, psi, 4, np.zeros(3))
