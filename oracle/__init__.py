"""Plain, slow, complex128 CPU oracle for noisy-circuit MPO simulation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
runs this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark may.  It shares no code with the HIP path: the only common
dependency is `mpo_inputs`, which supplies raw seeded Gaussian draws and the
brickwork schedule and holds none of the method's arithmetic.

Method followed (Noh, Jiang, Fefferman, "Efficient classical simulation of
noisy random quantum circuits in one dimension", Quantum 2020):
  * gates.py    Haar U(4) sampling, two-qubit depolarizing channel, the noisy
                gate M = N . U as a 16x16 superoperator (Sec. II.B, Eq. for the
                two-qubit CPTP map in Sec. III.B, App. A definition of M), and
                the change to the normalised Pauli basis.
  * dense.py    brute-force evolution of the 2^n x 2^n density matrix and a
                pure-state simulator (plain definitions, small n).
  * mpo.py      the MPO update with a QR-moved orthogonality centre and a local
                truncated SVD (the "Note added" variant), MPO entanglement
                entropy (Sec. III.C, Eq. for S_l), trace and Pauli expectation
                values by transfer contraction (Sec. III.D).
  * vidal.py    the paper's own global Gamma-lambda update (App. A), used only
                to cross-check mpo.py under truncation.

Every function is pinned by `-m "not gpu"` tests against closed forms,
brute force or values the paper prints; see tests/test_oracle_*.py.
"""
