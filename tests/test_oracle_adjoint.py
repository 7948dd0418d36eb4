"""Pins of the oracle's fidelity gradient (CPU): finite differences of the loss,
the block-matrix form of the Frechet derivative, and the Magnus oracle itself."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import adjoint as oa
from oracle import hamiltonians as hm
from oracle import magnus as mg
from paper_1709_06483_amd import inputs


def _nodes(f, tau, nsteps, t0=0.0):
    t = np.array([[t0 + n * tau + c * tau for c in mg.GAUSS2] for n in range(nsteps)])
    return np.vectorize(f)(t), t


def _problem(n=4, K=8, T=2.0, nsteps=40, seed=40):
    H1 = hm.xxz_open_chain(n, 1.0, 0.5, sparse=False)
    H2 = hm.field("x", n, sparse=False)
    theta = inputs.fourier_theta(K, seed)
    tau = T / nsteps
    psi0 = inputs.random_states(1 << n, seed=41)
    tgt = inputs.random_states(1 << n, seed=42)
    return H1, H2, theta, tau, nsteps, T, psi0, tgt


def _field_data(theta, T, tau, nsteps):
    f = inputs.fourier_field(theta, T)
    fn, t = _nodes(f, tau, nsteps)
    basis = inputs.fourier_basis(len(theta), T)
    dfn = np.stack([np.stack([basis(t[n, j]) for j in range(2)]) for n in range(nsteps)])
    return fn, dfn


def test_frechet_eigenbasis_matches_block_exponential():
    rng = np.random.default_rng(3)
    N = 16
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    H = 0.5 * (X + X.conj().T)
    Y = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    H2 = 0.5 * (Y + Y.conj().T)
    tau = 0.3
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    Q, l = oa.exp_eig(H, tau)
    a = oa.frechet_apply(Q, l, -1j * tau * H2, v)
    b = oa.frechet_block(-1j * tau * H, -1j * tau * H2, v)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)
    # and the definition as a derivative: (exp(A + eps E) - exp(A - eps E)) / (2 eps)
    eps = 1e-6
    A, E = -1j * tau * H, -1j * tau * H2
    fd = (sla.expm(A + eps * E) - sla.expm(A - eps * E)) @ v / (2 * eps)
    assert np.linalg.norm(a - fd) <= 1e-8 * np.linalg.norm(fd)


def test_loss_matches_magnus_oracle():
    H1, H2, theta, tau, nsteps, T, psi0, tgt = _problem()
    fn, _ = _field_data(theta, T, tau, nsteps)
    f = inputs.fourier_field(theta, T)
    y = mg.propagate("CF4", mg.two_term(H1, H2, f), tau, nsteps, psi0)
    assert abs(oa.loss(H1, H2, tau, fn, psi0, tgt) - (1 - abs(np.vdot(tgt, y)) ** 2)) <= 1e-14


def test_gradient_matches_finite_differences():
    H1, H2, theta, tau, nsteps, T, psi0, tgt = _problem()
    fn, dfn = _field_data(theta, T, tau, nsteps)
    L, g, _ = oa.loss_and_gradient(H1, H2, tau, fn, dfn, psi0, tgt)
    eps = 1e-5
    for k in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += eps
        tm[k] -= eps
        fp, _ = _field_data(tp, T, tau, nsteps)
        fm, _ = _field_data(tm, T, tau, nsteps)
        fd = (oa.loss(H1, H2, tau, fp, psi0, tgt) - oa.loss(H1, H2, tau, fm, psi0, tgt)) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-9 + 1e-7 * abs(g[k]), (k, fd, g[k])


def test_planted_swapped_node_derivatives_are_caught():
    H1, H2, theta, tau, nsteps, T, psi0, tgt = _problem()
    fn, dfn = _field_data(theta, T, tau, nsteps)
    _, g, aux = oa.loss_and_gradient(H1, H2, tau, fn, dfn, psi0, tgt)
    # the same contraction with the roles of beta and gamma exchanged
    dbeta = mg.CF4_ALPHA2 * dfn[:, 0, :] + mg.CF4_ALPHA1 * dfn[:, 1, :]
    dgamma = mg.CF4_ALPHA1 * dfn[:, 0, :] + mg.CF4_ALPHA2 * dfn[:, 1, :]
    wrong = -2.0 * np.real(np.conj(aux["z"]) * (dbeta.T @ aux["g_a"] + dgamma.T @ aux["g_b"]))
    assert np.max(np.abs(wrong - g)) > 1e-4 * np.max(np.abs(g))
