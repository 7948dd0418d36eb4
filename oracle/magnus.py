"""One-step Magnus schemes of Section 2, applied step by step.

The ODE is Y' = A(t) Y with A(t) = -i H(t) (Section 1 writes i psi' = H(t) psi;
Section 2 writes Y' = A(t) Y), and H(t) = sum_k f_k(t) H_k (Section 4 uses
H(t) = H1 + h(t) H2).  A step is Y_{n+1} = exp(Omega_n) Y_n (Section 2, the
one-step scheme), or for commutator-free methods a product of exponentials, the
rightmost acting first.  Each method below returns its exponents in the order
the paper writes them (left to right); ``step`` applies them right to left.

Readings (where the paper is ambiguous or garbled):
* M4 in Section 4's pseudocode drops the factor -i; here A_i = -i H(t_n + c_i tau)
  throughout, as the ODE of Sections 1-2 fixes (pinned by the observed order).
* M6 prints the coefficient of B_3 as 1/2; consistency of the three-point Gauss
  quadrature of int A requires 1/12, which is used (pinned by observed order 6).
"""
from __future__ import annotations

import math
from typing import Callable, Sequence

import numpy as np

from .expm import expmv_eig, expmv_taylor
from .linop import Comm, Lin, Mat, Op

SQRT3 = math.sqrt(3.0)
SQRT15 = math.sqrt(15.0)

# Method M4 / Cf4: two-stage Gauss nodes.
GAUSS2 = (0.5 - SQRT3 / 6.0, 0.5 + SQRT3 / 6.0)
# Method Cf4 coefficients.
CF4_ALPHA1 = (3.0 - 2.0 * SQRT3) / 12.0
CF4_ALPHA2 = (3.0 + 2.0 * SQRT3) / 12.0
# Methods M6 / Cf4:3: three-stage Gauss nodes.
GAUSS3 = (0.5 - SQRT15 / 10.0, 0.5, 0.5 + SQRT15 / 10.0)
_a = 37.0 / 240.0
_b = 10.0 * SQRT15 / 261.0
# Method Cf4:3, the 3x3 alpha matrix as printed (row i = exponent i).
CF43_ALPHA = np.array([
    [_a - _b, -1.0 / 30.0, _a + _b],
    [-11.0 / 360.0, 23.0 / 45.0, -11.0 / 360.0],
    [_a + _b, -1.0 / 30.0, _a - _b],
])


class Problem:
    """i psi' = H(t) psi with H(t) = sum_k f_k(t) H_k; A(t) = -i H(t)."""

    def __init__(self, terms: Sequence[tuple]):
        self.mats = [Mat(H) for H, _ in terms]
        self.fs = [f for _, f in terms]

    def A(self, t: float) -> Op:
        return Lin([(-1j * f(t), M) for M, f in zip(self.mats, self.fs)])


def two_term(H1, H2, f: Callable[[float], float]) -> Problem:
    """H(t) = H1 + f(t) H2."""
    return Problem([(H1, lambda t: 1.0), (H2, f)])


# -- Section 2, Method M2 ----------------------------------------------------
def exponents_m2(P: Problem, tn: float, tau: float):
    return [tau * P.A(tn + 0.5 * tau)]


# -- Section 2, Method M4 ----------------------------------------------------
def exponents_m4(P: Problem, tn: float, tau: float):
    A1 = P.A(tn + GAUSS2[0] * tau)
    A2 = P.A(tn + GAUSS2[1] * tau)
    return [(0.5 * tau) * (A1 + A2) + (SQRT3 * tau * tau / 12.0) * Comm(A2, A1)]


# -- Section 2, Method M6 (with the 1/12 reading of the B_3 coefficient) -----
def exponents_m6(P: Problem, tn: float, tau: float):
    A1, A2, A3 = (P.A(tn + c * tau) for c in GAUSS3)
    B1 = tau * A2
    B2 = (SQRT15 / 3.0 * tau) * (A3 - A1)
    B3 = (10.0 / 3.0 * tau) * Lin([(1.0, A3), (-2.0, A2), (1.0, A1)])
    C12 = Comm(B1, B2)
    left = Lin([(-20.0, B1), (-1.0, B3), (1.0, C12)])
    right = Lin([(1.0, B2), (-1.0 / 60.0, Comm(B1, Lin([(2.0, B3), (1.0, C12)])))])
    return [Lin([(1.0, B1), (1.0 / 12.0, B3), (1.0 / 240.0, Comm(left, right))])]


# -- Section 2, Method Cf4 ---------------------------------------------------
def exponents_cf4(P: Problem, tn: float, tau: float):
    A1 = P.A(tn + GAUSS2[0] * tau)
    A2 = P.A(tn + GAUSS2[1] * tau)
    return [tau * Lin([(CF4_ALPHA1, A1), (CF4_ALPHA2, A2)]),
            tau * Lin([(CF4_ALPHA2, A1), (CF4_ALPHA1, A2)])]


# -- Section 2, Method Cf4:3 -------------------------------------------------
def exponents_cf43(P: Problem, tn: float, tau: float):
    A = [P.A(tn + c * tau) for c in GAUSS3]
    return [tau * Lin([(CF43_ALPHA[i, j], A[j]) for j in range(3)]) for i in range(3)]


METHODS = {
    "M2": exponents_m2,
    "M4": exponents_m4,
    "M6": exponents_m6,
    "CF4": exponents_cf4,
    "CF43": exponents_cf43,
}


def apply_exponentials(exponents, y: np.ndarray, expm: str = "eig") -> np.ndarray:
    """exp(Omega^(1)) ... exp(Omega^(s)) y, the rightmost factor first."""
    f = expmv_eig if expm == "eig" else expmv_taylor
    for Om in reversed(exponents):
        y = f(Om, y)
    return y


def step(method: str, P: Problem, tn: float, tau: float, y: np.ndarray, expm: str = "eig"):
    return apply_exponentials(METHODS[method](P, tn, tau), y, expm)


def propagate(method: str, P: Problem, tau: float, nsteps: int, psi0: np.ndarray,
              t0: float = 0.0, expm: str = "eig", every: int | None = None):
    """Y_{n+1} from Y_n for n = 0..nsteps-1 on the grid t_n = t0 + n tau.

    Returns Y_nsteps, or (Y_nsteps, [Y_0, Y_every, ...]) when ``every`` is given.
    """
    y = np.array(psi0, dtype=np.complex128, copy=True)
    snaps = [y.copy()] if every else None
    for n in range(nsteps):
        y = step(method, P, t0 + n * tau, tau, y, expm)
        if every and (n + 1) % every == 0:
            snaps.append(y.copy())
    return (y, snaps) if every else y
