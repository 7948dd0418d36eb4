"""CPU FP64 oracle for Magnus integrators with exact matrix exponentials.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP path; the only common
module is ``paper_1709_06483_amd.inputs`` (seeded problem data, no method
arithmetic).

Contents
--------
``hamiltonians``  Pauli operators by explicit Kronecker products (Section 4,
                  the definitions of the Pauli matrices and of sigma_j^alpha).
``linop``         a tiny lazy operator algebra (sums, commutators) with dense,
                  matvec and rigorous 2-norm-bound evaluation.
``expm``          exp(Omega) v for skew-Hermitian Omega: by Hermitian
                  eigendecomposition (oracle-E) and by fixed-degree truncated
                  Taylor with an a priori remainder bound (oracle-T).
``magnus``        the one-step schemes of Section 2 (M2, M4, M6, Cf4, Cf4:3)
                  as written there, and time propagation Y_{n+1} = exp(Omega_n) Y_n.
``adjoint``       fidelity loss and its exact gradient with respect to a linear
                  control field (eigenbasis Frechet derivatives).

Every function cites the passage of the paper it follows.  Parity pins (what
fixes each function other than itself) live in ``tests/test_oracle_*.py``.
"""
