"""CPU oracle for the finite-temperature TD-DMRG mobility path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or calls anything in this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark do.

Contents
  model.py    chain layout, local operators, the Hamiltonian and current as
              lists of operator strings (Eq. (1), the current operator below
              the Kubo formula, and the Holstein-Peierls coupling)
  ed.py       exact diagonalisation in the one-carrier sector: Z, C(t)
  mpo.py      matrix-product operators built term by term from model.py
  tdvp.py     purified MPS, imaginary-time preparation, one-site projector-
              splitting TDVP, the current correlation and the mobility
  analysis.py Kubo mobility, Fermi-golden-rule hopping-limit C(t), mean free
              path, coherent length
  sweep.py    batched mobility runs over temperature, transfer integral and
              frequency scale (isotope substitution)

Everything runs in float64 / complex128 with numpy and scipy.
"""
