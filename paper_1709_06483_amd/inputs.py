"""Seeded synthetic inputs: spin-chain Hamiltonians, dense power-law
Hamiltonians, initial states and control fields.

This module holds no part of the integration method.  It only builds the
problem data that both the HIP path and the CPU oracle consume:

* ``chain_terms``: the open XXZ chain ``H1 = sum_i J (X_i X_{i+1} + Y_i Y_{i+1}
  + Delta Z_i Z_{i+1})`` and the transverse field ``H2 = sum_i X_i`` as
  complex128 CSR arrays, built directly from bit operations on basis indices.
  Site 1 is the leftmost Kronecker factor (the paper's definition of
  sigma_j^alpha in Section 4), i.e. the most significant bit of the index.
  A basis bit 0 is spin up (sigma^z eigenvalue +1).
* ``powerlaw_hermitian``: a dense Hermitian matrix with entries
  ``g_jk / (1 + |j-k|)^alpha``, ``g`` complex normal.
* ``random_states``: seeded random unit vectors.
* ``fourier_field`` / ``cos_field`` / ``sin_field``: the scalar control field f(t)
  of ``H(t) = H1 + f(t) H2`` (Section 4 splits H(t) this way).

Every generator draws from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class CSR:
    """A complex128 CSR matrix as three host arrays (int32 indices)."""

    indptr: np.ndarray
    indices: np.ndarray
    data: np.ndarray
    dim: int

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.dim, self.dim))

    @staticmethod
    def from_scipy(m: sp.spmatrix) -> "CSR":
        m = sp.csr_matrix(m, dtype=np.complex128)
        m.eliminate_zeros()
        m.sort_indices()
        return CSR(m.indptr.astype(np.int32), m.indices.astype(np.int32),
                   np.ascontiguousarray(m.data, dtype=np.complex128), m.shape[0])


def _coo_to_csr(rows, cols, vals, dim) -> CSR:
    m = sp.coo_matrix((vals, (rows, cols)), shape=(dim, dim)).tocsr()
    return CSR.from_scipy(m)


def _site_bit(n: int, j: int) -> int:
    """Bit mask of site j (1-based, site 1 = most significant bit)."""
    return 1 << (n - j)


def xxz_chain(n: int, J: float = 1.0, Delta: float = 0.5) -> CSR:
    """Open XXZ chain, bonds (i, i+1) for i = 1..n-1.

    Diagonal: J*Delta*sum z_i z_{i+1}.  X X + Y Y on an anti-aligned pair flips
    both spins with amplitude 2J and annihilates an aligned pair.
    """
    if n < 2:
        raise ValueError("a chain needs n >= 2 spins")
    N = 1 << n
    s = np.arange(N, dtype=np.int64)
    bits = [((s >> (n - j)) & 1) for j in range(1, n + 1)]
    diag = np.zeros(N)
    rows, cols, vals = [s], [s], []
    for i in range(1, n):
        zi = 1 - 2 * bits[i - 1]
        zj = 1 - 2 * bits[i]
        diag += J * Delta * zi * zj
        anti = bits[i - 1] != bits[i]
        r = s[anti]
        rows.append(r)
        cols.append(r ^ (_site_bit(n, i) | _site_bit(n, i + 1)))
        vals.append(np.full(r.shape, 2.0 * J, dtype=np.complex128))
    vals.insert(0, diag.astype(np.complex128))
    return _coo_to_csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), N)


def pauli_field(n: int, axis: str = "x") -> CSR:
    """sum_j sigma^axis_j for axis in {x, z}."""
    N = 1 << n
    s = np.arange(N, dtype=np.int64)
    if axis == "x":
        rows = np.concatenate([s] * n)
        cols = np.concatenate([s ^ _site_bit(n, j) for j in range(1, n + 1)])
        vals = np.ones(rows.shape, dtype=np.complex128)
        return _coo_to_csr(rows, cols, vals, N)
    if axis == "z":
        diag = np.zeros(N)
        for j in range(1, n + 1):
            diag += 1 - 2 * ((s >> (n - j)) & 1)
        return _coo_to_csr(s, s, diag.astype(np.complex128), N)
    raise ValueError(axis)


def chain_terms(n: int, J: float = 1.0, Delta: float = 0.5, field_axis: str = "x"):
    """(H1, H2) of H(t) = H1 + f(t) H2 for the open XXZ chain with a uniform field."""
    return xxz_chain(n, J, Delta), pauli_field(n, field_axis)


def heisenberg_nonlocal_terms(n: int):
    """(H1, H2) of the paper's dense-case model (Section 4, Example 1):
    H1 = -sum_{i != j} sigma^z_i sigma^z_j / |i - j| (all ordered pairs, so every
    unordered pair twice; diagonal), H2 = -sum_j sigma^x_j.  The paper stores
    both densely; their structure is that of a diagonal plus n flips per row."""
    if n < 2:
        raise ValueError("the model needs n >= 2 spins")
    N = 1 << n
    s = np.arange(N, dtype=np.int64)
    z = [1 - 2 * ((s >> (n - j)) & 1) for j in range(1, n + 1)]
    diag = np.zeros(N)
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            if i != j:
                diag -= z[i - 1] * z[j - 1] / abs(i - j)
    H1 = _coo_to_csr(s, s, diag.astype(np.complex128), N)
    x = pauli_field(n, "x").to_scipy()
    return H1, CSR.from_scipy(-x)


def heisenberg_local_terms(n: int, Jx: float = 1.0, Jy: float = 2.0, Jz: float = 3.0):
    """(H1, H2) of the paper's sparse-case model (Section 4, Example 2):
    H1 = -1/2 sum_{j=1}^{n} (Jx X_j X_{j+1} + Jy Y_j Y_{j+1} + Jz Z_j Z_{j+1}) with
    site n + 1 read as site 1 (a ring; the paper leaves the boundary open to
    reading), H2 = -1/2 sum_j sigma^z_j.  X X + Y Y flips both spins of a bond
    with amplitude Jx - Jy on an aligned pair and Jx + Jy on an anti-aligned one."""
    if n < 3:
        raise ValueError("a ring needs n >= 3 spins")
    N = 1 << n
    s = np.arange(N, dtype=np.int64)
    bits = [((s >> (n - j)) & 1) for j in range(1, n + 1)]
    diag = np.zeros(N)
    rows, cols, vals = [s], [s], []
    for i in range(1, n + 1):
        k = i % n + 1
        zi, zk = 1 - 2 * bits[i - 1], 1 - 2 * bits[k - 1]
        diag += -0.5 * Jz * zi * zk
        anti = bits[i - 1] != bits[k - 1]
        amp = np.where(anti, Jx + Jy, Jx - Jy) * -0.5
        keep = amp != 0.0
        rows.append(s[keep])
        cols.append(s[keep] ^ (_site_bit(n, i) | _site_bit(n, k)))
        vals.append(amp[keep].astype(np.complex128))
    vals.insert(0, diag.astype(np.complex128))
    H1 = _coo_to_csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), N)
    zf = pauli_field(n, "z").to_scipy()
    return H1, CSR.from_scipy(-0.5 * zf)


def powerlaw_hermitian(N: int, alpha: float, seed: int) -> np.ndarray:
    """Dense Hermitian H with H_jk = g_jk / (1 + |j-k|)^alpha, row-major complex128.

    Upper triangle g_jk ~ CN(0, 1) (real and imaginary parts N(0, 1/2)),
    g_kj = conj(g_jk), real diagonal g_jj ~ N(0, 1).
    """
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((N, N))
    im = rng.standard_normal((N, N))
    d = rng.standard_normal(N)
    H = np.empty((N, N), dtype=np.complex128)
    H.real = re
    H.imag = im
    del re, im
    H *= 1.0 / math.sqrt(2.0)
    w = (1.0 + np.arange(N, dtype=np.float64)) ** (-alpha)
    idx = np.arange(N)
    blk = 512
    for r0 in range(0, N, blk):
        r1 = min(N, r0 + blk)
        dist = np.abs(idx[r0:r1, None] - idx[None, :])
        H[r0:r1] *= w[dist]
        # keep only the strict upper triangle of this row block
        H[r0:r1][idx[None, :] <= idx[r0:r1, None]] = 0.0
    H += H.conj().T
    H[idx, idx] = d * w[0]
    return H


def random_states(N: int, seed: int, batch: int | None = None) -> np.ndarray:
    """Seeded complex-normal vectors normalised to unit 2-norm; shape (N,) or (batch, N)."""
    rng = np.random.default_rng(seed)
    B = 1 if batch is None else batch
    x = np.empty((B, N), dtype=np.complex128)
    for b in range(B):  # state b draws its real then imaginary parts in turn
        x[b].real = rng.standard_normal(N)
        x[b].imag = rng.standard_normal(N)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x[0].copy() if batch is None else x


def cos_field(omega: float, amp: float = 1.0):
    return lambda t: amp * math.cos(omega * t)


def sin_field(omega: float, amp: float = 1.0):
    return lambda t: amp * math.sin(omega * t)


def fourier_theta(K: int, seed: int, sigma: float = 0.1) -> np.ndarray:
    return sigma * np.random.default_rng(seed).standard_normal(K)


def fourier_field(theta: np.ndarray, T: float):
    """f(t) = sum_k theta_k sin(k pi t / T), k = 1..K."""
    theta = np.asarray(theta, dtype=np.float64)
    k = np.arange(1, theta.shape[0] + 1, dtype=np.float64)

    def f(t):
        return float(np.dot(theta, np.sin(k * math.pi * t / T)))

    return f


def fourier_basis(K: int, T: float):
    """s_k(t) = sin(k pi t / T): the derivative of the Fourier field with respect to theta_k."""
    k = np.arange(1, K + 1, dtype=np.float64)
    return lambda t: np.sin(k * math.pi * t / T)


# Workload recipes (sizes, seeds, readings of unstated parameters).
CONFIGS = {
    "chain_n10": dict(kind="sparse_chain", n=10, J=1.0, Delta=0.5, omega=2.0, field="cos",
                      psi_seed=0, tau=0.01, nsteps=100, t0=0.0, budget_tol=1e-10),
    "chain_n20": dict(kind="sparse_chain", n=20, J=1.0, Delta=0.5, omega=2.0, field="cos",
                      psi_seed=1, tau=0.01, nsteps=500, t0=0.0, budget_tol=1e-10),
    "dense_8192": dict(kind="dense_powerlaw", N=8192, alpha=1.5, omega=1.0, field="sin",
                       seeds=dict(H0=20, V=21, psi=22), tau=0.005, nsteps=200, t0=0.0,
                       budget_tol=1e-10),
    # 256 states on the dense construction at N = 4096 (one FP64-MFMA GEMM per
    # Leja iteration); step count and tau unstated, taken from dense_8192
    "batched_dense_4096": dict(kind="batched", N=4096, alpha=1.5, omega=1.0, field="sin", batch=256,
                               seeds=dict(H0=31, V=32, psi=30), tau=0.005, nsteps=200, t0=0.0,
                               budget_tol=1e-10),
    # chains of 12, 14, 16 and 18 sites, 16 instances each: instance k has the
    # field amplitude 1 + k/16 on cos(2t) and its own initial state (seed
    # 300 + n, one draw of 16 states); step count and tau taken from chain_n10
    "ragged_chains": dict(kind="ragged", sizes=(12, 14, 16, 18), per_size=16, J=1.0, Delta=0.5, omega=2.0,
                          field="cos", psi_seed_base=300, tau=0.01, nsteps=100, t0=0.0, budget_tol=1e-10),
    # optimal control: f(t) = sum_{k<=32} theta_k sin(k pi t / T), theta ~ N(0, 0.1^2)
    # (seed 40), T = 2, 400 Cf4 steps, loss 1 - |<psi_target, psi(T)>|^2
    "adjoint_chain_n16": dict(kind="adjoint", n=16, J=1.0, Delta=0.5, params=32, theta_seed=40, T=2.0,
                              nsteps=400, psi_seed=41, target_seed=42, budget_tol=1e-10),
    "adjoint_dense_4096": dict(kind="adjoint", N=4096, alpha=1.5, seeds=dict(H0=20, V=21), params=32,
                               theta_seed=40, T=2.0, nsteps=400, psi_seed=41, target_seed=42, budget_tol=1e-10),
}
