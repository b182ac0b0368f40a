"""Writes tests/golden/fp64_chain_common_state.json: the oracle's reference
for the float64 parity of the 11-molecule chain (two local modes with
omega 0.5 and 1.5, seeded Huang-Rhys factors, 8 levels, D = 64).

Everything here is computed by oracle/ alone, from seeded inputs:
  * Psi: a seeded random right-canonical MPS of the chain's site dimensions
    at bond dimension 64 (tests/helpers.random_mps, seed 2003);
  * Phi = j Psi compressed to 64 (oracle apply_current);
  * C_k = <Psi(t_k)| j |Phi(t_k)>, k = 0..10, dt = 0.05, one-site TDVP steps
    of both states (Krylov tolerance 1e-14);
  * linear probes <r|Phi> (random bond-3 MPS r, tests/helpers convention),
    so that a GPU-compressed Phi can be checked against this one.
Run from the repository root: python tests/golden/make_fp64_chain_fixture.py
(about ten minutes on eight cores)."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from helpers import mps_inner, random_mps  # noqa: E402
from oracle import model as Mdl  # noqa: E402
from oracle import mpo as OM  # noqa: E402
from oracle import tdvp as T  # noqa: E402
from paper_2003_13245_amd import workloads as W  # noqa: E402

SEED, D, STEPS, N_PROBE, PROBE_SEED = 2003, 64, 10, 6, 1234


def probes(dims, n, seed):
    rng = np.random.default_rng(seed)
    L = len(dims)
    out = []
    for _ in range(n):
        R = []
        for i, d in enumerate(dims):
            x = 1 if i == 0 else 3
            y = 1 if i == L - 1 else 3
            R.append(rng.standard_normal((x, d, d, y)) + 1j * rng.standard_normal((x, d, d, y)))
        out.append(T.MPS(R))
    return out


def main():
    wl = W.fp64_chain(1.0)
    m, r = wl.model, wl.run
    dims = Mdl.site_dims(m)
    Hw, Jw = OM.hamiltonian_mpo(m), OM.current_mpo(m)
    psi = random_mps(dims, D, np.random.default_rng(SEED), 0)
    phi = T.apply_current(Jw, psi, D)
    phi_bonds = phi.bond_dims()
    pr = [complex(mps_inner(p, phi)) for p in probes(dims, N_PROBE, PROBE_SEED)]
    C = [complex(T.overlap(psi, Jw, phi))]
    for k in range(STEPS):
        T.tdvp_step(psi, Hw, -1j * r.dt)
        T.tdvp_step(phi, Hw, -1j * r.dt)
        C.append(complex(T.overlap(psi, Jw, phi)))
        print(f"step {k + 1}: C = {C[-1]:.15e}", flush=True)
    out = {
        "what": "oracle C(t) of the 11-molecule float64 chain from a seeded common state",
        "workload": wl.name, "seed": SEED, "D": D, "dt": r.dt, "steps": STEPS,
        "krylov_tol": 1e-14, "cutoff": 1e-10, "probe_seed": PROBE_SEED,
        "phi_bonds": phi_bonds,
        "phi_probes": [[z.real, z.imag] for z in pr],
        "C": [[z.real, z.imag] for z in C],
    }
    with open(os.path.join(HERE, "fp64_chain_common_state.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
