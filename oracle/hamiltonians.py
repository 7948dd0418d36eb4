"""Spin operators built literally from Kronecker products.

Section 4 defines the Pauli matrices and sigma_j^alpha = I x ... x sigma^alpha x
... x I with sigma^alpha in slot j of n.  These builders follow that definition
term by term (dense for small n, scipy.sparse.kron for larger n) and are used
to check the bit-operation builders of the inputs module, and as independent
Hamiltonians in the oracle's own tests.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)
PAULI = {"x": SX, "y": SY, "z": SZ}


def sigma(alpha: str, j: int, n: int, sparse: bool = True):
    """sigma_j^alpha on n spins, site j in 1..n (slot j of the Kronecker product)."""
    factors = [I2] * (j - 1) + [PAULI[alpha]] + [I2] * (n - j)
    if sparse:
        out = sp.csr_matrix(factors[0])
        for f in factors[1:]:
            out = sp.kron(out, sp.csr_matrix(f), format="csr")
        return out
    out = factors[0]
    for f in factors[1:]:
        out = np.kron(out, f)
    return out


def xxz_open_chain(n: int, J: float, Delta: float, sparse: bool = True):
    """sum_{i=1}^{n-1} J (X_i X_{i+1} + Y_i Y_{i+1} + Delta Z_i Z_{i+1})."""
    H = None
    for i in range(1, n):
        term = J * (sigma("x", i, n, sparse) @ sigma("x", i + 1, n, sparse)
                    + sigma("y", i, n, sparse) @ sigma("y", i + 1, n, sparse)
                    + Delta * (sigma("z", i, n, sparse) @ sigma("z", i + 1, n, sparse)))
        H = term if H is None else H + term
    return H


def field(axis: str, n: int, sparse: bool = True):
    """sum_{j=1}^n sigma_j^axis."""
    H = None
    for j in range(1, n + 1):
        term = sigma(axis, j, n, sparse)
        H = term if H is None else H + term
    return H


def nonlocal_heisenberg(n: int, sparse: bool = False):
    """The paper's dense example (Example 1): H1 = -sum_i sum_{j != i} J_ij Z_i Z_j,
    J_ij = 1/|i-j|, and H2 = -sum_i X_i, with H(t) = H1 + h(t) H2."""
    H1 = None
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            if i == j:
                continue
            term = -(1.0 / abs(i - j)) * (sigma("z", i, n, sparse) @ sigma("z", j, n, sparse))
            H1 = term if H1 is None else H1 + term
    H2 = -field("x", n, sparse)
    return H1, H2


def single_spin_rabi_terms():
    """Terms of the one-spin Rabi Hamiltonian (w0/2) Z + W (cos(w t) X + sin(w t) Y)."""
    return SZ, SX, SY
