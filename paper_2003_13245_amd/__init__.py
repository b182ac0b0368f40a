"""ftdmrg: finite-temperature TD-DMRG carrier mobility on AMD MI355X.

    from paper_2003_13245_amd import api        # the native library binding
    from paper_2003_13245_amd import workloads  # seeded synthetic inputs

The binding loads libftdmrg.so on first use and raises ImportError when it has
not been built (there is no fallback implementation).
"""
_API = {"Context", "Mpo", "Mps", "mpo_build", "thermal_prep", "tdvp_step", "corr_current",
        "mobility", "apply_compress", "overlap", "heff_apply", "mps_from_host", "FtdError"}


def __getattr__(name):
    if name in _API:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
