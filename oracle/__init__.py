"""CPU reference ("oracle") for fermionic state-vector evolution at fixed (N_alpha, N_beta).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package:
only the test suite, the smoke check and the bench's CPU-baseline leg use it.
It shares no code, tables or helpers with the HIP library.

Everything here is plain complex128 / float64 numpy and scipy, written from the
definitions in the paper (ffsim: faster simulation of fermionic quantum
circuits), one function per operation, with no blocking, fusion or merging of
gates:

  strings.py      electronic configurations and their addresses (Sec. 2.2, 2.4, 3.1)
  gates.py        orbital rotation as the compound-matrix action of U (Sec. 2.3,
                  3.2.3), number-operator-sum and diagonal-Coulomb phases
                  (Sec. 3.2.1, 3.2.2), the Givens pair action (Sec. 3.2.3)
  hamiltonian.py  one-body action, double-factorized Hamiltonian action and
                  energy (Eq. double-factorized-hamiltonian, Sec. 4.2),
                  Trotter-Suzuki product formulas S_0, S_1, S_k (Sec. 4.5.3)
  lucj.py         the LUCJ ansatz (Sec. 4.5.1), its energy, finite-difference and
                  adjoint gradients
  sampled.py      single amplitudes of a rotated state at sizes where full
                  compound matrices are too large

Parity status: every function is pinned by the tests in tests/test_oracle_*.py
against brute-force Jordan-Wigner matrices, closed forms or invariants, except
where a function's docstring says "parity unpinned".
"""
