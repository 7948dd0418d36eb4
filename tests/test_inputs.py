"""The seeded input builders against the Kronecker-product definitions (CPU)."""
import numpy as np
import pytest

from oracle import hamiltonians as hm
from paper_1709_06483_amd import inputs


@pytest.mark.parametrize("n", [2, 3, 4, 7, 10])
def test_xxz_chain_matches_kronecker(n):
    J, Delta = 1.0, 0.5
    H1 = inputs.xxz_chain(n, J, Delta)
    ref = hm.xxz_open_chain(n, J, Delta, sparse=True)
    assert abs(H1.to_scipy() - ref).max() < 1e-15


@pytest.mark.parametrize("n", [2, 5, 10])
def test_fields_match_kronecker(n):
    assert abs(inputs.pauli_field(n, "x").to_scipy() - hm.field("x", n)).max() < 1e-15
    assert abs(inputs.pauli_field(n, "z").to_scipy() - hm.field("z", n)).max() < 1e-15


@pytest.mark.parametrize("n", [10, 12, 14])
def test_chain_nnz_formula(n):
    # even n: the ZZ diagonal never vanishes; N(n+1)/2 for H1, nN for H2
    H1, H2 = inputs.chain_terms(n)
    N = 1 << n
    assert H1.nnz == N * (n + 1) // 2
    assert H2.nnz == n * N
    for H in (H1, H2):
        assert H.indptr.dtype == np.int32 and H.indices.dtype == np.int32
        assert H.indptr[0] == 0 and H.indptr[-1] == H.nnz
        assert np.all(np.diff(H.indptr) >= 0)
        # sorted columns within each row
        rows = np.repeat(np.arange(N), np.diff(H.indptr))
        key = rows.astype(np.int64) * N + H.indices
        assert np.all(np.diff(key) > 0)
        S = H.to_scipy()
        assert abs(S - S.conj().T).max() == 0


def test_powerlaw_hermitian_structure():
    N, alpha = 64, 1.5
    H = inputs.powerlaw_hermitian(N, alpha, seed=3)
    assert H.flags["C_CONTIGUOUS"] and H.dtype == np.complex128
    assert np.array_equal(H, H.conj().T)
    # the power-law envelope: |H_jk| (1+|j-k|)^alpha is O(1) complex normal
    j, k = np.indices((N, N))
    g = H * (1.0 + np.abs(j - k)) ** alpha
    off = g[j < k]
    assert abs(np.mean(np.abs(off) ** 2) - 1.0) < 0.1
    assert np.all(np.imag(np.diag(H)) == 0)
    # reproducible, seed-dependent
    assert np.array_equal(H, inputs.powerlaw_hermitian(N, alpha, seed=3))
    assert not np.array_equal(H, inputs.powerlaw_hermitian(N, alpha, seed=4))


def test_random_states():
    x = inputs.random_states(128, seed=7)
    assert x.shape == (128,) and abs(np.linalg.norm(x) - 1) < 1e-15
    B = inputs.random_states(128, seed=7, batch=5)
    assert B.shape == (5, 128)
    assert np.allclose(np.linalg.norm(B, axis=1), 1, atol=1e-15)
    assert np.array_equal(B[0], x)


def test_fourier_field():
    th = np.array([0.3, -0.2, 0.1])
    f = inputs.fourier_field(th, 2.0)
    t = 0.37
    assert abs(f(t) - sum(th[k] * np.sin((k + 1) * np.pi * t / 2.0) for k in range(3))) < 1e-15
    assert np.allclose(inputs.fourier_basis(3, 2.0)(t), [np.sin((k + 1) * np.pi * t / 2.0) for k in range(3)])


def _kron_site(n, j, P):
    """sigma^P on site j (1-based, site 1 = the leftmost factor) of n spins, dense."""
    I2 = np.eye(2)
    out = np.array([[1.0 + 0j]])
    for k in range(1, n + 1):
        out = np.kron(out, P if k == j else I2)
    return out


def test_paper_heisenberg_models_match_kronecker_products():
    """The paper's two example models (Section 4) built from explicit tensor products of
    the Pauli matrices, for a few small n, equal the generators' CSR terms."""
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
    Z = np.array([[1, 0], [0, -1]], dtype=complex)
    for n in (3, 4, 5):
        H1, H2 = inputs.heisenberg_nonlocal_terms(n)
        ref1 = sum(-(1.0 / abs(i - j)) * _kron_site(n, i, Z) @ _kron_site(n, j, Z)
                   for i in range(1, n + 1) for j in range(1, n + 1) if i != j)
        ref2 = sum(-_kron_site(n, j, X) for j in range(1, n + 1))
        assert np.allclose(H1.to_scipy().toarray(), ref1, atol=1e-13)
        assert np.allclose(H2.to_scipy().toarray(), ref2, atol=1e-13)
        H1, H2 = inputs.heisenberg_local_terms(n)
        ref1 = sum(-0.5 * (1.0 * _kron_site(n, j, X) @ _kron_site(n, j % n + 1, X)
                           + 2.0 * _kron_site(n, j, Y) @ _kron_site(n, j % n + 1, Y)
                           + 3.0 * _kron_site(n, j, Z) @ _kron_site(n, j % n + 1, Z)) for j in range(1, n + 1))
        ref2 = sum(-0.5 * _kron_site(n, j, Z) for j in range(1, n + 1))
        assert np.allclose(H1.to_scipy().toarray(), ref1, atol=1e-13)
        assert np.allclose(H2.to_scipy().toarray(), ref2, atol=1e-13)
