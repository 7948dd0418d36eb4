"""exp(Omega) v for a skew-Hermitian exponent Omega (Omega = -i tau H_hat).

Section 3 needs the action of the matrix exponential of each Magnus exponent
on the state.  The oracle computes it exactly (to rounding), by definition,
two ways:

``expmv_eig``    (oracle-E) i*Omega is Hermitian; with i*Omega = Q diag(mu) Q^H,
                 exp(Omega) = Q diag(exp(-i mu)) Q^H.
``expmv_taylor`` (oracle-T) the exponential series sum_k Omega^k v / k!, split
                 into s equal substeps with rho = ||Omega||/s <= 1 and cut at
                 the degree m where the remainder bound
                 s * rho^(m+1) e^rho / (m+1)! falls below 1e-17.  Non-adaptive
                 (its degree depends only on the norm bound), so it is smooth
                 in the problem data.

Neither uses Leja interpolation; they are the plain definitions the Leja
method approximates.
"""
from __future__ import annotations

import math

import numpy as np

from .linop import Op

TAYLOR_REMAINDER = 1e-17


def expmv_eig(Omega, v: np.ndarray) -> np.ndarray:
    """exp(Omega) v by eigendecomposition of the Hermitian matrix i*Omega."""
    W = Omega.dense() if isinstance(Omega, Op) else np.asarray(Omega)
    G = 1j * W
    G = 0.5 * (G + G.conj().T)
    mu, Q = np.linalg.eigh(G)
    V = np.asarray(v).reshape(v.shape[0], -1)
    out = Q @ (np.exp(-1j * mu)[:, None] * (Q.conj().T @ V))
    return out.reshape(v.shape)


def taylor_plan(norm_bound: float, remainder: float = TAYLOR_REMAINDER):
    """Substeps s and degree m with rho = norm_bound/s <= 1 and
    s * rho^(m+1) e^rho / (m+1)! <= remainder."""
    s = max(1, int(math.ceil(norm_bound)))
    rho = norm_bound / s
    m = 0
    if rho == 0.0:
        return s, 0, rho
    term = rho  # rho^(m+1)/(m+1)! for m = 0
    while s * term * math.exp(rho) > remainder:
        m += 1
        term *= rho / (m + 1)
    return s, m, rho


def expmv_taylor(Omega: Op, v: np.ndarray) -> np.ndarray:
    """exp(Omega) v by a truncated Taylor series with substeps (a priori degree)."""
    s, m, _ = taylor_plan(Omega.norm_bound())
    x = np.array(v, dtype=np.complex128, copy=True)
    for _ in range(s):
        acc = x.copy()
        term = x
        for k in range(1, m + 1):
            term = Omega.matvec(term) / (s * k)
            acc = acc + term
        x = acc
    return x
