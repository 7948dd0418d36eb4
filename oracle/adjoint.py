"""Fidelity loss of a Cf4 propagation and its exact gradient (FP64, CPU).

Test infrastructure only.  The paper has no adjoint; this follows the plain
definitions.  For psi_{n+1} = E_a(n) E_b(n) psi_n (Method Cf4 of Section 2,
the right factor E_b = exp(-i tau (H1/2 + beta_n H2)) acting first, then
E_a = exp(-i tau (H1/2 + gamma_n H2)), with beta_n = alpha2 f1 + alpha1 f2 and
gamma_n = alpha1 f1 + alpha2 f2 from the field samples f1, f2 of step n):

    L = 1 - |z|^2,  z = psi_tgt^H psi_N,
    dz = sum_n lambda_{n+1}^H dE(n) psi_n,   lambda_{n+1} = (E(N-1) ... E(n+1))^H psi_tgt,
    dE(n) = dgamma_n L_a E_b + dbeta_n E_a L_b,

where L_x = L(-i tau H_x, -i tau H2) is the Frechet derivative of the matrix
exponential at -i tau H_x in the direction -i tau H2.  So with
phi_n = E_b psi_n and mu_n = E_a^H lambda_{n+1}:

    g_a(n) = lambda_{n+1}^H L_a phi_n,   g_b(n) = mu_n^H L_b psi_n,
    dL/dtheta_k = -2 Re( conj(z) sum_n [ dgamma_n/dtheta_k g_a(n) + dbeta_n/dtheta_k g_b(n) ] ).

Frechet derivatives are computed in the eigenbasis (Daleckii-Krein: for
A = Q diag(l) Q^H, L(A, E) = Q (F o (Q^H E Q)) Q^H with F_ij the first divided
difference of exp at l_i, l_j); ``frechet_block`` gives the same quantity
from the exponential of the block matrix [[A, E], [0, A]] for cross-checks.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .magnus import CF4_ALPHA1, CF4_ALPHA2


def _dense(M):
    return M.toarray() if hasattr(M, "toarray") else np.asarray(M)


def exp_eig(Hhat: np.ndarray, tau: float):
    """(Q, l) with exp(-i tau Hhat) = Q diag(exp(l)) Q^H, l = -i tau eig(Hhat)."""
    H = 0.5 * (Hhat + Hhat.conj().T)
    w, Q = np.linalg.eigh(H)
    return Q, -1j * tau * w


def expmv(Q, l, v):
    return Q @ (np.exp(l) * (Q.conj().T @ v))


def frechet_apply(Q, l, E, v):
    """L(A, E) v for A = Q diag(l) Q^H (Daleckii-Krein)."""
    el = np.exp(l)
    dl = l[:, None] - l[None, :]
    same = np.abs(dl) < 1e-12
    with np.errstate(divide="ignore", invalid="ignore"):
        F = np.where(same, el[:, None], (el[:, None] - el[None, :]) / np.where(same, 1.0, dl))
    Et = Q.conj().T @ E @ Q
    return Q @ ((F * Et) @ (Q.conj().T @ v))


def frechet_block(A, E, v):
    """L(A, E) v from exp([[A, E], [0, A]]) [0; v]."""
    n = A.shape[0]
    M = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    M[:n, :n] = A
    M[:n, n:] = E
    M[n:, n:] = A
    x = np.concatenate([np.zeros(n, dtype=np.complex128), v])
    return (sla.expm(M) @ x)[:n]


def cf4_coeffs(f1, f2):
    beta = CF4_ALPHA2 * f1 + CF4_ALPHA1 * f2
    gamma = CF4_ALPHA1 * f1 + CF4_ALPHA2 * f2
    return beta, gamma


def loss_and_gradient(H1, H2, tau: float, f_nodes: np.ndarray, df_nodes: np.ndarray, psi0, psi_tgt):
    """Loss and gradient with respect to the control parameters.

    f_nodes: (nsteps, 2) field samples at the two Gauss nodes of each step.
    df_nodes: (nsteps, 2, P) their derivatives with respect to the P parameters.
    """
    H1 = _dense(H1)
    H2 = _dense(H2)
    nsteps = f_nodes.shape[0]
    E = -1j * tau * H2
    psis, phis, fac = [np.asarray(psi0, dtype=np.complex128)], [], []
    for n in range(nsteps):
        beta, gamma = cf4_coeffs(*f_nodes[n])
        Qb, lb = exp_eig(0.5 * H1 + beta * H2, tau)
        Qa, la = exp_eig(0.5 * H1 + gamma * H2, tau)
        phi = expmv(Qb, lb, psis[-1])
        phis.append(phi)
        psis.append(expmv(Qa, la, phi))
        fac.append((Qb, lb, Qa, la))
    z = np.vdot(psi_tgt, psis[-1])
    loss = 1.0 - abs(z) ** 2
    lam = np.asarray(psi_tgt, dtype=np.complex128)
    ga = np.zeros(nsteps, dtype=np.complex128)
    gb = np.zeros(nsteps, dtype=np.complex128)
    for n in range(nsteps - 1, -1, -1):
        Qb, lb, Qa, la = fac[n]
        ga[n] = np.vdot(lam, frechet_apply(Qa, la, E, phis[n]))
        mu = expmv(Qa, la.conj(), lam)          # E_a^H lambda
        gb[n] = np.vdot(mu, frechet_apply(Qb, lb, E, psis[n]))
        lam = expmv(Qb, lb.conj(), mu)          # E_b^H mu
    dbeta = CF4_ALPHA2 * df_nodes[:, 0, :] + CF4_ALPHA1 * df_nodes[:, 1, :]
    dgamma = CF4_ALPHA1 * df_nodes[:, 0, :] + CF4_ALPHA2 * df_nodes[:, 1, :]
    dz = dgamma.T @ ga + dbeta.T @ gb
    grad = -2.0 * np.real(np.conj(z) * dz)
    return loss, grad, {"z": z, "g_a": ga, "g_b": gb}


def loss(H1, H2, tau: float, f_nodes: np.ndarray, psi0, psi_tgt):
    H1 = _dense(H1)
    H2 = _dense(H2)
    psi = np.asarray(psi0, dtype=np.complex128)
    for n in range(f_nodes.shape[0]):
        beta, gamma = cf4_coeffs(*f_nodes[n])
        Qb, lb = exp_eig(0.5 * H1 + beta * H2, tau)
        Qa, la = exp_eig(0.5 * H1 + gamma * H2, tau)
        psi = expmv(Qa, la, expmv(Qb, lb, psi))
    return 1.0 - abs(np.vdot(psi_tgt, psi)) ** 2
