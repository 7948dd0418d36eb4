"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerance: the Magnus result must match the oracle to 1e-10 in relative
2-norm (Leja tolerance 1e-10 treated as the budget for the whole run, split
over its exponentials).  Single exponentials planned for tol run to 20*tol
(interpolation bound plus FP64 rounding over the Newton terms).
"""
import math

import numpy as np
import pytest

from oracle import expm as oe
from oracle import hamiltonians as hm
from oracle import magnus as mg
from oracle.linop import Comm, Lin, Mat
from paper_1709_06483_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected only where a GPU exists
    pytest.skip("no GPU", allow_module_level=True)

from paper_1709_06483_amd import binding as B  # noqa: E402

BUDGET = 1e-10


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(max_dim=1 << 20, max_batch=4)
    yield c
    c.close()


def chain(n):
    H1, H2 = inputs.chain_terms(n)
    return H1, H2


@pytest.fixture(scope="module")
def chain10(ctx):
    H1, H2 = chain(10)
    ham = B.magnus_spectral_bounds(ctx, B.DeviceHamiltonian.from_csr(H1, H2))
    return H1, H2, ham


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def oracle_exponent(H1, H2, a, b, kappa, tau):
    M1, M2 = Mat(H1), Mat(H2)
    terms = [(-1j * tau * a, M1), (-1j * tau * b, M2)]
    if kappa != 0.0:
        terms.append((-1j * tau * kappa * 1j, Comm(M1, M2)))
    return Lin(terms)


def node_field(t0, tau, f1, f2):
    """A field that takes the values f1, f2 at the two Gauss nodes of the step at t0."""
    t1, t2 = t0 + mg.GAUSS2[0] * tau, t0 + mg.GAUSS2[1] * tau
    return lambda t: f1 + (f2 - f1) * (t - t1) / (t2 - t1)


# ---------------------------------------------------------------------------
def test_spectral_bounds_enclose_spectrum(chain10):
    H1, H2, ham = chain10
    for H, T in ((H1, ham.struct.H1), (H2, ham.struct.H2)):
        ev = np.linalg.eigvalsh(H.to_scipy().toarray())
        assert T.lam_min <= ev[0] + 1e-12 and ev[-1] <= T.lam_max + 1e-12
    K = 1j * (H1.to_scipy() @ H2.to_scipy() - H2.to_scipy() @ H1.to_scipy()).toarray()
    evk = np.linalg.eigvalsh(K)
    assert ham.struct.k_min <= evk[0] and evk[-1] <= ham.struct.k_max


@pytest.mark.parametrize("a,b,kappa,tau", [
    (0.5, 0.3, 0.0, 0.01), (1.0, -0.7, 0.0, 0.05), (0.5, 0.5, 0.0, -0.03), (1.0, 0.2, 1e-3, 0.02),
    (1.0, -0.4, -2e-3, -0.04)])
def test_expmv_matches_oracle(ctx, chain10, a, b, kappa, tau):
    H1, H2, ham = chain10
    v = inputs.random_states(1024, seed=101)
    tol = 1e-12
    w, st = B.expmv_leja(ctx, ham, a, b, kappa, tau, dev(v), opts=B.leja_opts(tol), stats=True)
    ref = oe.expmv_eig(oracle_exponent(H1.to_scipy(), H2.to_scipy(), a, b, kappa, tau), v)
    assert rel(host(w), ref) <= 20 * tol
    assert st["exponentials"] == 1 and 1 <= st["iters"] <= st["planned_iters"]
    assert st["hv_products"] == st["iters"] * (4 if kappa else 2)


def test_expmv_substeps_large_step(ctx):
    H1, H2 = chain(8)
    ham = B.magnus_spectral_bounds(ctx, B.DeviceHamiltonian.from_csr(H1, H2))
    v = inputs.random_states(256, seed=102)
    tol = 1e-11
    w, st = B.expmv_leja(ctx, ham, 1.0, 0.8, 0.0, 0.9, dev(v), opts=B.leja_opts(tol), stats=True)
    assert st["max_substeps_used"] >= 2
    ref = oe.expmv_eig(oracle_exponent(H1.to_scipy(), H2.to_scipy(), 1.0, 0.8, 0.0, 0.9), v)
    assert rel(host(w), ref) <= 20 * tol * st["max_substeps_used"]


def test_expmv_frozen_degree_and_early_termination_agree(ctx, chain10):
    H1, H2, ham = chain10
    v = dev(inputs.random_states(1024, seed=103))
    w1, s1 = B.expmv_leja(ctx, ham, 0.5, 0.2, 0.0, 0.02, v, opts=B.leja_opts(1e-12, early_termination=False),
                          stats=True)
    w2, s2 = B.expmv_leja(ctx, ham, 0.5, 0.2, 0.0, 0.02, v, opts=B.leja_opts(1e-12), stats=True)
    assert s1["iters"] == s1["planned_iters"]
    assert s2["iters"] <= s1["iters"]
    assert rel(host(w2), host(w1)) <= 2e-11


def test_zero_step_and_in_place(ctx, chain10):
    H1, H2, ham = chain10
    v = dev(inputs.random_states(1024, seed=104))
    w = B.expmv_leja(ctx, ham, 1.0, 0.5, 0.0, 0.0, v)
    assert torch.equal(w, v)
    out = B.expmv_leja(ctx, ham, 1.0, 0.5, 0.0, 0.03, v)
    inplace = v.clone()
    B.expmv_leja(ctx, ham, 1.0, 0.5, 0.0, 0.03, inplace, inplace)
    assert torch.equal(out, inplace)


@pytest.mark.parametrize("method", ["CF4", "M4"])
def test_single_step_matches_oracle(ctx, chain10, method):
    H1, H2, ham = chain10
    psi = inputs.random_states(1024, seed=105)
    tau, t0, f1, f2 = 0.02, 0.3, 0.8, -0.35
    fn = B.magnus_step_cf4 if method == "CF4" else B.magnus_step_m4
    out = fn(ctx, ham, tau, f1, f2, dev(psi), opts=B.leja_opts(1e-12))
    P = mg.two_term(H1.to_scipy().toarray(), H2.to_scipy().toarray(), node_field(t0, tau, f1, f2))
    ref = mg.step(method, P, t0, tau, psi)
    assert rel(host(out), ref) <= 4e-11


def _field_nodes(method, f, t0, tau, nsteps):
    t = B.magnus_quadrature_nodes(B.METHODS[method], t0, tau, nsteps)
    return np.vectorize(f)(t)


@pytest.mark.parametrize("method", ["CF4", "M4"])
def test_propagate_chain_n10_matches_oracle(ctx, chain10, method):
    """Chain n = 10 (dim 1024), cos(2t) field, tau = 0.01, 100 steps on [0, 1]."""
    H1, H2, ham = chain10
    cfg = inputs.CONFIGS["chain_n10"]
    f = inputs.cos_field(cfg["omega"])
    psi0 = inputs.random_states(1024, seed=cfg["psi_seed"])
    fn = _field_nodes(method, f, 0.0, cfg["tau"], cfg["nsteps"])
    psi = dev(psi0)
    _, st = B.propagate(ctx, ham, B.METHODS[method], cfg["tau"], fn, psi,
                        opts=B.leja_opts(BUDGET, tol_mode=1), stats=True)
    P = mg.two_term(H1.to_scipy(), H2.to_scipy(), f)
    ref = mg.propagate(method, P, cfg["tau"], cfg["nsteps"], psi0, expm="taylor")
    err = rel(host(psi), ref)
    assert err <= BUDGET, err
    assert st["exponentials"] == cfg["nsteps"] * (2 if method == "CF4" else 1)


def test_propagate_batch_checkpoints_and_determinism(ctx, chain10):
    H1, H2, ham = chain10
    tau, nsteps, k = 0.01, 10, 4
    psi0 = inputs.random_states(1024, seed=7, batch=3)
    fields = [inputs.cos_field(2.0, amp) for amp in (1.0, 0.5, -0.25)]
    fn = np.stack([_field_nodes("CF4", f, 0.0, tau, nsteps) for f in fields])
    nck = (nsteps + k - 1) // k + 1
    ck = torch.zeros((nck, 3, 1024), dtype=torch.complex128, device="cuda")
    psi = dev(psi0)
    B.propagate(ctx, ham, B.CF4, tau, fn, psi, checkpoints=ck, every_k=k, opts=B.leja_opts(1e-12))
    batch_out = host(psi)
    ck = host(ck)
    assert np.array_equal(ck[0], psi0)
    for c in range(3):
        # states 0, 1 run as one group through the multi-state kernel, state 2 alone
        single = dev(psi0[c])
        B.propagate(ctx, ham, B.CF4, tau, fn[c], single, opts=B.leja_opts(1e-12))
        assert rel(host(single), batch_out[c]) <= 1e-13
        mid = dev(psi0[c])
        B.propagate(ctx, ham, B.CF4, tau, fn[c, :k], mid, opts=B.leja_opts(1e-12))
        assert rel(host(mid), ck[1, c]) <= 1e-13
    assert np.array_equal(ck[-1], batch_out)
    again = dev(psi0)
    B.propagate(ctx, ham, B.CF4, tau, fn, again, opts=B.leja_opts(1e-12))
    assert np.array_equal(host(again), batch_out)


def test_time_reversal_on_device(ctx, chain10):
    H1, H2, ham = chain10
    tau, nsteps = 0.02, 15
    f = inputs.cos_field(2.0)
    psi0 = inputs.random_states(1024, seed=9)
    fwd = _field_nodes("CF4", f, 0.0, tau, nsteps)
    bwd = _field_nodes("CF4", f, nsteps * tau, -tau, nsteps)
    psi = dev(psi0)
    B.propagate(ctx, ham, B.CF4, tau, fwd, psi, opts=B.leja_opts(1e-13))
    B.propagate(ctx, ham, B.CF4, -tau, bwd, psi, opts=B.leja_opts(1e-13))
    assert rel(host(psi), psi0) <= 1e-11


def test_dense_powerlaw_ragged_dim(ctx):
    """Dense H0 + sin(t) V, power-law entries, dim 1000 (not a multiple of the row tile)."""
    N, tau, nsteps = 1000, 0.005, 20
    H0 = inputs.powerlaw_hermitian(N, 1.5, seed=20)
    V = inputs.powerlaw_hermitian(N, 1.5, seed=21)
    ham = B.magnus_spectral_bounds(ctx, B.DeviceHamiltonian.from_dense(H0, V))
    f = inputs.sin_field(1.0)
    psi0 = inputs.random_states(N, seed=22)
    psi = dev(psi0)
    B.propagate(ctx, ham, B.CF4, tau, _field_nodes("CF4", f, 0.0, tau, nsteps), psi,
                opts=B.leja_opts(BUDGET, tol_mode=1))
    ref = mg.propagate("CF4", mg.two_term(H0, V, f), tau, nsteps, psi0, expm="taylor")
    assert rel(host(psi), ref) <= BUDGET


def _ragged_hermitian(N, seed, long_rows=(), long_len=0):
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 12, size=N)
    lens[rng.integers(0, N, size=N // 50)] = 0  # some empty rows
    rows = np.repeat(np.arange(N), lens)
    cols = rng.integers(0, N, size=rows.shape[0])
    for r in long_rows:
        c = rng.choice(N, size=long_len, replace=False)
        rows = np.concatenate([rows, np.full(long_len, r)])
        cols = np.concatenate([cols, c])
    vals = rng.standard_normal(rows.shape[0]) + 1j * rng.standard_normal(rows.shape[0])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsr()
    H = (A + A.conj().T) * 0.5
    return inputs.CSR.from_scipy(H)


@pytest.mark.parametrize("N,long_len", [(5000, 3000), (70001, 5000)])
def test_ragged_csr_with_long_rows(ctx, N, long_len):
    """Irregular rows (empty rows, rows longer than one LDS chunk), ragged tail."""
    H1 = _ragged_hermitian(N, 31, long_rows=(3, N // 2), long_len=long_len)
    H2 = _ragged_hermitian(N, 32)
    ham = B.magnus_spectral_bounds(ctx, B.DeviceHamiltonian.from_csr(H1, H2))
    v = inputs.random_states(N, seed=33)
    tol = 1e-12
    w = B.expmv_leja(ctx, ham, 0.6, -0.4, 0.0, 0.01, dev(v), opts=B.leja_opts(tol))
    ref = oe.expmv_taylor(oracle_exponent(H1.to_scipy(), H2.to_scipy(), 0.6, -0.4, 0.0, 0.01), v)
    assert rel(host(w), ref) <= 20 * tol


def test_full_size_chain_n20_sampled_steps(ctx):
    """Chain n = 20 (dim 2^20, 31,981,568 nonzeros) in the bench's launch
    configuration: 2 Cf4 steps and 1 M4 step against the oracle's Taylor series."""
    cfg = inputs.CONFIGS["chain_n20"]
    H1, H2 = chain(20)
    ham = B.magnus_spectral_bounds(ctx, B.DeviceHamiltonian.from_csr(H1, H2))
    f = inputs.cos_field(cfg["omega"])
    psi0 = inputs.random_states(1 << 20, seed=cfg["psi_seed"])
    tol_e = BUDGET / (2 * cfg["nsteps"])  # the per-exponential tolerance of the full run
    S1, S2 = H1.to_scipy(), H2.to_scipy()
    P = mg.two_term(S1, S2, f)
    for method, nsteps in (("CF4", 2), ("M4", 1)):
        psi = dev(psi0)
        B.propagate(ctx, ham, B.METHODS[method], cfg["tau"], _field_nodes(method, f, 0.0, cfg["tau"], nsteps), psi,
                    opts=B.leja_opts(tol_e))
        ref = mg.propagate(method, P, cfg["tau"], nsteps, psi0, expm="taylor")
        assert rel(host(psi), ref) <= 50 * tol_e * nsteps


def test_malformed_csr_rejected(ctx):
    H1, H2 = chain(6)
    bad = inputs.CSR(H1.indptr.copy(), H1.indices.copy(), H1.data.copy(), H1.dim)
    bad.indptr[10] = bad.indptr[11] + 1  # not monotone
    ham = B.DeviceHamiltonian.from_csr(bad, H2)
    with pytest.raises(B.MagnusError) as e:
        B.magnus_spectral_bounds(ctx, ham)
    assert e.value.code == B.EINVAL
    bad2 = inputs.CSR(H1.indptr.copy(), H1.indices.copy(), H1.data.copy(), H1.dim)
    bad2.indices[5] = 64  # column out of range
    ham2 = B.DeviceHamiltonian.from_csr(bad2, H2)
    ham2.struct.H1.lam_min, ham2.struct.H1.lam_max = -1.0, 1.0
    ham2.struct.H2.lam_min, ham2.struct.H2.lam_max = -6.0, 6.0
    with pytest.raises(B.MagnusError) as e:
        B.expmv_leja(ctx, ham2, 1.0, 1.0, 0.0, 0.1, dev(inputs.random_states(64, seed=1)))
    assert e.value.code == B.EINVAL


def test_argument_errors(ctx, chain10):
    H1, H2, ham = chain10
    v = dev(inputs.random_states(1024, seed=1))
    with pytest.raises(B.MagnusError) as e:
        B.expmv_leja(ctx, ham, 1.0, 1.0, 0.0, 0.1, v, opts=B.leja_opts(0.0))
    assert e.value.code == B.EDOMAIN
    with pytest.raises(B.MagnusError) as e:
        B.expmv_leja(ctx, ham, 1.0, float("nan"), 0.0, 0.1, v)
    assert e.value.code == B.EDOMAIN
    with pytest.raises(B.MagnusError) as e:
        B.expmv_leja(ctx, ham, 1.0, 1.0, 0.0, 50.0, v, opts=B.leja_opts(1e-10, max_degree=8, max_substeps=1))
    assert e.value.code == B.ENOCONV
    small = B.Context(max_dim=512)
    with pytest.raises(B.MagnusError) as e:
        B.expmv_leja(small, ham, 1.0, 1.0, 0.0, 0.1, v)
    assert e.value.code == B.ENOMEM
    small.close()


def test_nan_state_reported(ctx, chain10):
    H1, H2, ham = chain10
    x = inputs.random_states(1024, seed=2)
    x[17] = np.nan
    v = dev(x)
    with pytest.raises(B.MagnusError) as e:
        B.expmv_leja(ctx, ham, 1.0, 0.5, 0.0, 0.01, v, stats=True)
    assert e.value.code == B.ENAN
    with pytest.raises(B.MagnusError):
        ctx.check()  # the flag stays set until the next call starts
    B.expmv_leja(ctx, ham, 1.0, 0.5, 0.0, 0.01, dev(inputs.random_states(1024, seed=3)))
    ctx.check()


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7])
def test_csr_kernel_variants_match_oracle(variant, monkeypatch):
    """Every CSR iteration kernel (nonzero-streaming 16/64-row blocks, row-per-lane
    32/64/128-row blocks, wave tiles of 8/16 rows, streamed wave tiles) on irregular rows (empty rows, rows longer than one LDS chunk) and a ragged tail, in
    Leja and commutator modes."""
    monkeypatch.setenv("MAGNUS_CSR_VARIANT", str(variant))
    N = 70001
    H1 = _ragged_hermitian(N, 41, long_rows=(0, 5, N - 1), long_len=6000)
    H2 = _ragged_hermitian(N, 42)
    c = B.Context(max_dim=N)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
    v = inputs.random_states(N, seed=43)
    tol = 1e-12
    S1, S2 = H1.to_scipy(), H2.to_scipy()
    for kappa in (0.0, 1e-4):
        w = B.expmv_leja(c, ham, 0.6, -0.4, kappa, 0.01, dev(v), opts=B.leja_opts(tol))
        ref = oe.expmv_taylor(oracle_exponent(S1, S2, 0.6, -0.4, kappa, 0.01), v)
        assert rel(host(w), ref) <= 20 * tol, (variant, kappa)
    c.close()


@pytest.mark.parametrize("batch", [2, 5, 16, 32])
def test_batched_expmv_matches_oracle(batch):
    """Groups of states through the multi-state CSR kernel (one matrix pass per group)."""
    H1, H2 = chain(9)
    c = B.Context(max_dim=512, max_batch=32)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
    V = inputs.random_states(512, seed=61, batch=batch)
    tol = 1e-12
    W, st = B.expmv_leja(c, ham, 0.7, -0.3, 0.0, 0.04, dev(V), opts=B.leja_opts(tol), stats=True)
    W = host(W)
    Om = oracle_exponent(H1.to_scipy().toarray(), H2.to_scipy().toarray(), 0.7, -0.3, 0.0, 0.04)
    for k in range(batch):
        assert rel(W[k], oe.expmv_eig(Om, V[k])) <= 20 * tol, k
    assert st["exponentials"] >= 1
    c.close()


def test_batched_propagate_per_state_fields():
    """16 states with their own field amplitudes (A_k = 1 + k/16), Cf4, against
    single-state runs and, for two of them, against the oracle."""
    n, Bn, tau, nsteps = 10, 16, 0.01, 40
    H1, H2 = chain(n)
    c = B.Context(max_dim=1 << n, max_batch=Bn)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
    psi0 = inputs.random_states(1 << n, seed=300, batch=Bn)
    fields = [inputs.cos_field(2.0, 1.0 + k / 16) for k in range(Bn)]
    fn = np.stack([_field_nodes("CF4", f, 0.0, tau, nsteps) for f in fields])
    psi = dev(psi0)
    opts = B.leja_opts(BUDGET, tol_mode=1)
    _, st = B.propagate(c, ham, B.CF4, tau, fn, psi, opts=opts, stats=True)
    out = host(psi)
    for k in (0, 7, 15):
        one = dev(psi0[k])
        B.propagate(c, ham, B.CF4, tau, fn[k], one, opts=opts)
        assert rel(host(one), out[k]) <= 1e-12
    for k in (3, 12):
        P = mg.two_term(H1.to_scipy(), H2.to_scipy(), fields[k])
        ref = mg.propagate("CF4", P, tau, nsteps, psi0[k], expm="taylor")
        assert rel(out[k], ref) <= BUDGET
    again = dev(psi0)
    B.propagate(c, ham, B.CF4, tau, fn, again, opts=opts)
    assert np.array_equal(host(again), out)
    c.close()


@pytest.mark.parametrize("reserve,per_state,N", [(True, False, 300), (False, False, 300), (True, True, 300),
                                                 (True, False, 10), (False, True, 10)])
def test_dense_batched_mfma_matches_oracle(reserve, per_state, N):
    """Groups of states on dense terms: FP64 MFMA GEMM (assembled exponent when the
    field is shared and the buffer is reserved, two-term otherwise), ragged dim and batch;
    N = 300 splits 19 K chunks unevenly between the workgroup's two K groups, N = 10
    leaves the second group without a chunk."""
    Bn, tau, nsteps = 70, 0.005, 6
    H0 = inputs.powerlaw_hermitian(N, 1.5, seed=31)
    V = inputs.powerlaw_hermitian(N, 1.5, seed=32)
    c = B.Context(max_dim=N, max_batch=Bn)
    if reserve:
        c.reserve_dense(N)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_dense(H0, V))
    psi0 = inputs.random_states(N, seed=30, batch=Bn)
    amps = [1.0 + (k / Bn if per_state else 0.0) for k in range(Bn)]
    fields = [inputs.sin_field(1.0, a) for a in amps]
    fn = np.stack([_field_nodes("CF4", f, 0.0, tau, nsteps) for f in fields])
    psi = dev(psi0)
    B.propagate(c, ham, B.CF4, tau, fn if per_state else fn[0], psi, opts=B.leja_opts(BUDGET, tol_mode=1))
    out = host(psi)
    for k in (0, 33, Bn - 1):
        ref = mg.propagate("CF4", mg.two_term(H0, V, fields[k]), tau, nsteps, psi0[k], expm="eig")
        assert rel(out[k], ref) <= BUDGET, k
    c.close()


@pytest.mark.parametrize("tile,N,Bn", [(0, 300, 70), (1, 300, 70), (2, 300, 70), (3, 300, 70), (4, 300, 70),
                                        (5, 300, 70), (5, 5, 2), (5, 33, 65), (5, 48, 64),
                                        (6, 300, 70), (6, 5, 2), (6, 33, 65), (6, 128, 64)])
@pytest.mark.parametrize("reserve", [True, False])
def test_dense_mfma_tile_shapes_match_oracle(tile, N, Bn, reserve, monkeypatch):
    """Every FP64-MFMA tile shape the autotuner chooses from (32 x 64 and 64 x 64
    rows x states with and without the K split, 32 x 128 with it, 32 x 64 and
    64 x 64 staged by LDS-DMA) on a ragged dim and batch, one term (assembled)
    and two; the LDS-DMA tiles also on one partial K chunk (N = 5), two chunks
    and a ragged tail (N = 33, one state past a column block) and whole chunks
    and blocks (N = 48 or 128, 64 states)."""
    monkeypatch.setenv("MAGNUS_MFMA_TILE", str(tile))
    tau, nsteps = 0.005, 4
    H0 = inputs.powerlaw_hermitian(N, 1.5, seed=31)
    V = inputs.powerlaw_hermitian(N, 1.5, seed=32)
    c = B.Context(max_dim=N, max_batch=Bn)
    if reserve:
        c.reserve_dense(N)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_dense(H0, V))
    psi0 = inputs.random_states(N, seed=30, batch=Bn)
    f = inputs.sin_field(1.0)
    psi = dev(psi0)
    c.timing(True)
    B.propagate(c, ham, B.CF4, tau, _field_nodes("CF4", f, 0.0, tau, nsteps), psi,
                opts=B.leja_opts(BUDGET, tol_mode=1))
    assert c.timing_read(B.KERNEL_DENSE_MFMA)[1] > 0
    c.timing(False)
    out = host(psi)
    for k in sorted({0, min(37, Bn - 1), Bn - 1}):
        ref = mg.propagate("CF4", mg.two_term(H0, V, f), tau, nsteps, psi0[k], expm="eig")
        assert rel(out[k], ref) <= BUDGET, k
    c.close()


@pytest.mark.parametrize("rpw", [1, 2, 4])
def test_dense_gemv_rows_per_wave_match_oracle(rpw, monkeypatch):
    monkeypatch.setenv("MAGNUS_DENSE_RPW", str(rpw))
    N, tau, nsteps = 1001, 0.005, 6
    H0 = inputs.powerlaw_hermitian(N, 1.5, seed=20)
    V = inputs.powerlaw_hermitian(N, 1.5, seed=21)
    c = B.Context(max_dim=N)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_dense(H0, V))
    f = inputs.sin_field(1.0)
    psi0 = inputs.random_states(N, seed=22)
    ref = mg.propagate("CF4", mg.two_term(H0, V, f), tau, nsteps, psi0, expm="eig")
    for reserve in (False, True):  # two terms, then the assembled exponent
        if reserve:
            c.reserve_dense(N)
        psi = dev(psi0)
        B.propagate(c, ham, B.CF4, tau, _field_nodes("CF4", f, 0.0, tau, nsteps), psi,
                    opts=B.leja_opts(BUDGET, tol_mode=1))
        assert rel(host(psi), ref) <= BUDGET
    c.close()


def test_dense_autotune_choices_are_used_and_match_oracle():
    N, Bn, tau, nsteps = 700, 40, 0.005, 4
    H0 = inputs.powerlaw_hermitian(N, 1.5, seed=31)
    V = inputs.powerlaw_hermitian(N, 1.5, seed=32)
    c = B.Context(max_dim=N, max_batch=Bn)
    c.reserve_dense(N)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_dense(H0, V))
    res = B.magnus_autotune(c, ham, batch=Bn)
    assert res["rows_per_wave"] in (1, 2, 4) and res["mfma_tile"] in B.MFMA_TILES
    assert all(v > 0 for v in res["rows_per_wave_us"].values())
    assert all(v is not None and v > 0 for v in res["mfma_tile_us"].values())
    psi0 = inputs.random_states(N, seed=30, batch=Bn)
    f = inputs.sin_field(1.0)
    psi = dev(psi0)
    B.propagate(c, ham, B.CF4, tau, _field_nodes("CF4", f, 0.0, tau, nsteps), psi,
                opts=B.leja_opts(BUDGET, tol_mode=1))
    one = dev(psi0[5])
    B.propagate(c, ham, B.CF4, tau, _field_nodes("CF4", f, 0.0, tau, nsteps), one,
                opts=B.leja_opts(BUDGET, tol_mode=1))
    out = host(psi)
    for k in (0, Bn - 1):
        ref = mg.propagate("CF4", mg.two_term(H0, V, f), tau, nsteps, psi0[k], expm="eig")
        assert rel(out[k], ref) <= BUDGET
    ref5 = mg.propagate("CF4", mg.two_term(H0, V, f), tau, nsteps, psi0[5], expm="eig")
    assert rel(host(one), ref5) <= BUDGET
    c.close()


@pytest.mark.parametrize("persist", ["1", "0"])
def test_small_state_propagation_paths_agree(persist, monkeypatch):
    """Small states run whole propagations in one workgroup each (MAGNUS_PERSIST=1)
    or as per-iteration launches (0); both match the oracle, with checkpoints."""
    monkeypatch.setenv("MAGNUS_PERSIST", persist)
    n, tau, nsteps, k = 10, 0.01, 30, 7
    H1, H2 = chain(n)
    c = B.Context(max_dim=1 << n, max_batch=3)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
    psi0 = inputs.random_states(1 << n, seed=8, batch=3)
    fields = [inputs.cos_field(2.0, a) for a in (1.0, -0.5, 2.0)]
    fn = np.stack([_field_nodes("CF4", f, 0.0, tau, nsteps) for f in fields])
    nck = (nsteps + k - 1) // k + 1
    ck = torch.zeros((nck, 3, 1 << n), dtype=torch.complex128, device="cuda")
    psi = dev(psi0)
    _, st = B.propagate(c, ham, B.CF4, tau, fn, psi, checkpoints=ck, every_k=k,
                        opts=B.leja_opts(BUDGET, tol_mode=1), stats=True)
    out, ck = host(psi), host(ck)
    for j in range(3):
        P = mg.two_term(H1.to_scipy(), H2.to_scipy(), fields[j])
        ref, snaps = mg.propagate("CF4", P, tau, nsteps, psi0[j], expm="taylor", every=k)
        assert rel(out[j], ref) <= BUDGET
        for q, snap in enumerate(snaps):
            assert rel(ck[q, j], snap) <= BUDGET
        assert rel(ck[-1, j], ref) <= BUDGET
    assert st["exponentials"] == 2 * nsteps * 3
    assert 0 < st["iters"] <= st["planned_iters"]
    c.close()


def test_small_state_kernel_term1_in_lds_is_bitwise_the_uncached(monkeypatch):
    """The one-workgroup kernel keeps term 1 of problems of at most 1024 rows in LDS
    when it fits (chains of 8 and 10 spins in one launch; a random pair of 1000 rows
    whose term 1 holds too many entries, which stays uncached): states equal bit for
    bit those with the cache switched off, and match the oracle."""
    monkeypatch.setenv("MAGNUS_PERSIST", "1")
    tau, nsteps = 0.01, 8
    terms = [chain(8), chain(10), (_ragged_hermitian(1000, 41), _ragged_hermitian(1000, 42))]
    assert terms[2][0].to_scipy().nnz > 6400 >= terms[1][0].to_scipy().nnz
    out = {}
    for cache in ("1", "0"):
        monkeypatch.setenv("MAGNUS_PERSIST_CACHE", cache)
        c = B.Context(max_dim=1024, max_batch=2)
        for idx, (H1, H2) in enumerate(terms):
            N = H1.to_scipy().shape[0]
            ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
            psi0 = inputs.random_states(N, seed=500 + idx, batch=2)
            fields = [inputs.cos_field(2.0, a) for a in (1.0, -0.7)]
            fn = np.stack([_field_nodes("CF4", f, 0.0, tau, nsteps) for f in fields])
            psi = dev(psi0)
            B.propagate(c, ham, B.CF4, tau, fn, psi, opts=B.leja_opts(BUDGET, tol_mode=1))
            out[cache, idx] = host(psi)
            if cache == "1":
                for k in range(2):
                    P = mg.two_term(H1.to_scipy(), H2.to_scipy(), fields[k])
                    ref = mg.propagate("CF4", P, tau, nsteps, psi0[k], expm="taylor")
                    assert rel(out[cache, idx][k], ref) <= BUDGET, (idx, k)
        c.close()
    for idx in range(len(terms)):
        assert np.array_equal(out["1", idx], out["0", idx]), idx


@pytest.mark.parametrize("persist", ["1", "0"])
def test_ragged_batch_matches_oracle(persist, monkeypatch):
    """Chains of 8, 10, 12 and 15 spins with several states each, one call: the
    three problems of at most 4096 rows share one persistent launch and the
    15-spin chain runs batched (persist 0: every problem runs batched)."""
    monkeypatch.setenv("MAGNUS_PERSIST", persist)
    tau, nsteps = 0.01, 12
    c = B.Context(max_dim=1 << 15, max_batch=4)
    probs, refs = [], []
    for n, per in ((8, 3), (10, 2), (12, 4), (15, 2)):
        H1, H2 = chain(n)
        ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
        psi0 = inputs.random_states(1 << n, seed=300 + n, batch=per)
        fields = [inputs.cos_field(2.0, 1.0 + k / 16) for k in range(per)]
        fn = np.stack([_field_nodes("CF4", f, 0.0, tau, nsteps) for f in fields])
        psi = dev(psi0)
        probs.append((ham, psi, fn))
        refs.append((H1, H2, fields, psi0))
    st = B.magnus_propagate_ragged(c, probs, B.CF4, tau, opts=B.leja_opts(BUDGET, tol_mode=1), stats=True)
    for (ham, psi, fn), (H1, H2, fields, psi0) in zip(probs, refs):
        out = host(psi)
        for k in (0, len(fields) - 1):
            P = mg.two_term(H1.to_scipy(), H2.to_scipy(), fields[k])
            ref = mg.propagate("CF4", P, tau, nsteps, psi0[k], expm="taylor")
            assert rel(out[k], ref) <= BUDGET
    assert st["exponentials"] == 2 * nsteps * (3 + 2 + 4 + 2)
    c.close()


def test_ragged_large_problems_in_one_launch_per_iteration(monkeypatch):
    """Chains of 13, 14 and 15 spins with 4 states each (and a 10-spin chain
    in the persistent launch), one call: with a workspace that holds all
    large problems at once they advance together, one launch per Leja
    iteration (MAGNUS_RAGGED_JOINT=1), else one after another (0); both
    against the oracle, the same states either way, fewer launches jointly."""
    tau, nsteps, per = 0.01, 8, 4
    sizes = (10, 13, 14, 15)
    runs = {}
    for joint in ("1", "0"):
        monkeypatch.setenv("MAGNUS_RAGGED_JOINT", joint)
        c = B.Context(max_dim=sum(1 << n for n in sizes), max_batch=per)
        probs, refs = [], []
        for n in sizes:
            H1, H2 = chain(n)
            ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
            psi0 = inputs.random_states(1 << n, seed=400 + n, batch=per)
            fields = [inputs.cos_field(2.0, 1.0 + k / 4) for k in range(per)]
            fn = np.stack([_field_nodes("CF4", f, 0.0, tau, nsteps) for f in fields])
            probs.append((ham, dev(psi0), fn))
            refs.append((H1, H2, fields, psi0))
        c.timing(True)
        st = B.magnus_propagate_ragged(c, probs, B.CF4, tau, opts=B.leja_opts(BUDGET, tol_mode=1), stats=True)
        _, launches = c.timing_read(B.KERNEL_CSR_MULTI)
        c.timing(False)
        runs[joint] = ([host(psi) for _, psi, _ in probs], st, launches)
        c.close()
    (outs, st, lj), (outs0, st0, l0) = runs["1"], runs["0"]
    print(f"ragged 13/14/15 x 4: multi-state launches joint {lj}, one problem after another {l0}", flush=True)
    assert 0 < lj < l0
    assert st["exponentials"] == st0["exponentials"] == 2 * nsteps * per * len(sizes)
    assert st["iters"] == st0["iters"]
    for out, out0, (H1, H2, fields, psi0) in zip(outs, outs0, refs):
        assert rel(out, out0) <= 1e-14
        for k in (0, per - 1):
            P = mg.two_term(H1.to_scipy(), H2.to_scipy(), fields[k])
            ref = mg.propagate("CF4", P, tau, nsteps, psi0[k], expm="taylor")
            assert rel(out[k], ref) <= BUDGET


def test_autotune_choices_are_used_and_match_oracle():
    """The autotuner times every CSR row mapping and multi-state group size on the
    n = 13 chain, keeps the fastest, and later calls with those kernels still match
    the oracle (single state and a group of 6)."""
    n, tau, nsteps = 13, 0.01, 6
    H1, H2 = chain(n)
    c = B.Context(max_dim=1 << n, max_batch=6)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
    res = B.magnus_autotune(c, ham, batch=6)
    assert res["variant"] in B.CSR_VARIANTS
    assert all(v > 0 for v in res["variant_us"].values())
    assert res["group"] in (2, 4)
    assert res["group_us"]["8"] is None and res["group_us"]["2"] > 0
    f = inputs.cos_field(2.0)
    fn = _field_nodes("CF4", f, 0.0, tau, nsteps)
    psi0 = inputs.random_states(1 << n, seed=77, batch=6)
    psi = dev(psi0)
    B.propagate(c, ham, B.CF4, tau, fn, psi, opts=B.leja_opts(BUDGET, tol_mode=1))
    out = host(psi)
    P = mg.two_term(H1.to_scipy(), H2.to_scipy(), f)
    for k in (0, 5):
        assert rel(out[k], mg.propagate("CF4", P, tau, nsteps, psi0[k], expm="taylor")) <= BUDGET
    one = dev(psi0[2])
    B.propagate(c, ham, B.CF4, tau, fn, one, opts=B.leja_opts(BUDGET, tol_mode=1))
    assert rel(host(one), mg.propagate("CF4", P, tau, nsteps, psi0[2], expm="taylor")) <= BUDGET
    c.close()


def _tiny_hermitian(N, seed, density=0.5, empty_rows=()):
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    A = np.zeros((N, N), complex)
    for i in range(N):
        for j in range(i, N):
            if rng.random() < density:
                A[i, j] = rng.standard_normal() + (1j * rng.standard_normal() if i != j else 0.0)
    A = A + np.triu(A, 1).conj().T
    for r in empty_rows:
        A[r, :] = 0.0
        A[:, r] = 0.0
    return inputs.CSR.from_scipy(sp.csr_matrix(A)), A


@pytest.mark.parametrize("persist", ["1", "0"])
@pytest.mark.parametrize("N", [1, 2, 3, 5, 17, 130])
def test_tiny_dims_empty_rows_and_zero_term(N, persist, monkeypatch):
    """Degenerate inputs on every path: dimensions 1..130, rows without entries, and an
    H2 with no entries at all (null column and value arrays); single states (small-state
    kernel or per-iteration launches), a group of 3, and M4."""
    import scipy.sparse as sp
    monkeypatch.setenv("MAGNUS_PERSIST", persist)
    H1, A1 = _tiny_hermitian(N, seed=900 + N, empty_rows=(N // 2,) if N > 2 else ())
    H2z = inputs.CSR(np.zeros(N + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, complex), N)
    H2, A2 = _tiny_hermitian(N, seed=950 + N, density=0.3)
    c = B.Context(max_dim=N, max_batch=3)
    tau, nsteps = 0.05, 7
    f = inputs.cos_field(2.0)
    psi0 = inputs.random_states(N, seed=960 + N, batch=3)
    for second, A2d in ((H2z, np.zeros((N, N))), (H2, A2)):
        ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, second))
        P = mg.two_term(A1, A2d, f)
        for method in ("CF4", "M4"):
            fn = _field_nodes(method, f, 0.0, tau, nsteps)
            one = dev(psi0[0])
            B.propagate(c, ham, B.METHODS[method], tau, fn, one, opts=B.leja_opts(BUDGET, tol_mode=1))
            ref = mg.propagate(method, P, tau, nsteps, psi0[0], expm="eig")
            assert rel(host(one), ref) <= BUDGET, (method, N)
        grp = dev(psi0)
        B.propagate(c, ham, B.CF4, tau, _field_nodes("CF4", f, 0.0, tau, nsteps), grp,
                    opts=B.leja_opts(BUDGET, tol_mode=1))
        out = host(grp)
        for k in range(3):
            assert rel(out[k], mg.propagate("CF4", P, tau, nsteps, psi0[k], expm="eig")) <= BUDGET, (k, N)
    c.close()


def test_term_rewritten_in_place_is_revalidated():
    """A term validated once and then corrupted in place (a column out of range) is
    caught when the caller re-scans it, and stays refused afterwards."""
    H1, H2 = chain(7)
    c = B.Context(max_dim=128, max_batch=1)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
    psi = dev(inputs.random_states(128, seed=3))
    B.expmv_leja(c, ham, 1.0, 0.5, 0.0, 0.05, psi)
    ci = ham.tensors[1]  # H1's column indices on the device
    ci[3] = 1000
    torch.cuda.synchronize()
    with pytest.raises(B.MagnusError) as e:
        B.magnus_spectral_bounds(c, ham)
    assert e.value.code == B.EINVAL
    with pytest.raises(B.MagnusError) as e:
        B.expmv_leja(c, ham, 1.0, 0.5, 0.0, 0.05, psi)
    assert e.value.code == B.EINVAL
    c.close()


@pytest.mark.parametrize("kind", ["chain", "dense"])
def test_lanczos_bounds_enclose_the_spectrum_and_tighten(kind):
    """The Lanczos estimates (60 steps, 1% margin) contain every eigenvalue of each term
    and are no wider than the Gershgorin intervals (narrower for the chain's H1)."""
    if kind == "chain":
        H1, H2 = chain(10)
        A1, A2 = H1.to_scipy().toarray(), H2.to_scipy().toarray()
        mk = lambda: B.DeviceHamiltonian.from_csr(H1, H2)
    else:
        A1 = inputs.powerlaw_hermitian(300, 1.5, seed=5)
        A2 = inputs.powerlaw_hermitian(300, 1.5, seed=6)
        mk = lambda: B.DeviceHamiltonian.from_dense(A1, A2)
    c = B.Context(max_dim=A1.shape[0], max_batch=1)
    g = B.magnus_spectral_bounds(c, mk())
    lz = B.magnus_spectral_bounds_lanczos(c, mk(), steps=60, margin=0.01)
    for term, A in (("H1", A1), ("H2", A2)):
        lam = np.linalg.eigvalsh(A)
        tg, tl = getattr(g.struct, term), getattr(lz.struct, term)
        assert tl.lam_min <= lam[0] and lam[-1] <= tl.lam_max, (term, tl.lam_min, tl.lam_max, lam[0], lam[-1])
        assert tl.lam_max - tl.lam_min <= tg.lam_max - tg.lam_min + 1e-12
    if kind == "chain":
        assert lz.struct.H1.lam_max - lz.struct.H1.lam_min < 0.8 * (g.struct.H1.lam_max - g.struct.H1.lam_min)
    with pytest.raises(B.MagnusError):
        B.magnus_spectral_bounds_lanczos(c, mk(), steps=1)
    c.close()


def test_lanczos_bounds_propagation_matches_oracle(ctx):
    """With the Lanczos estimates the chain n = 10 run (100 Cf4 and M4 steps) and two Cf4
    steps of the full n = 20 chain still match the oracle within the budget."""
    cfg = inputs.CONFIGS["chain_n10"]
    H1, H2 = chain(10)
    ham = B.magnus_spectral_bounds_lanczos(ctx, B.DeviceHamiltonian.from_csr(H1, H2))
    f = inputs.cos_field(cfg["omega"])
    psi0 = inputs.random_states(1024, seed=cfg["psi_seed"])
    P = mg.two_term(H1.to_scipy(), H2.to_scipy(), f)
    for method in ("CF4", "M4"):
        psi = dev(psi0)
        B.propagate(ctx, ham, B.METHODS[method], cfg["tau"], _field_nodes(method, f, 0.0, cfg["tau"], cfg["nsteps"]),
                    psi, opts=B.leja_opts(BUDGET, tol_mode=1))
        ref = mg.propagate(method, P, cfg["tau"], cfg["nsteps"], psi0, expm="taylor")
        assert rel(host(psi), ref) <= BUDGET, method
    cfg = inputs.CONFIGS["chain_n20"]
    H1, H2 = chain(20)
    ham = B.magnus_spectral_bounds_lanczos(ctx, B.DeviceHamiltonian.from_csr(H1, H2))
    f = inputs.cos_field(cfg["omega"])
    psi0 = inputs.random_states(1 << 20, seed=cfg["psi_seed"])
    tol_e = BUDGET / (2 * cfg["nsteps"])
    psi = dev(psi0)
    B.propagate(ctx, ham, B.CF4, cfg["tau"], _field_nodes("CF4", f, 0.0, cfg["tau"], 2), psi, opts=B.leja_opts(tol_e))
    ref = mg.propagate("CF4", mg.two_term(H1.to_scipy(), H2.to_scipy(), f), cfg["tau"], 2, psi0, expm="taylor")
    assert rel(host(psi), ref) <= 50 * tol_e * 2


def test_ragged_more_small_states_than_control_slots():
    """300 small states (more than the context's 256 control slots) run as two
    persistent launches; every state matches its single-state propagation."""
    tau, nsteps = 0.01, 5
    c = B.Context(max_dim=256, max_batch=4)
    H1, H2 = chain(8)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
    psi0 = inputs.random_states(256, seed=601, batch=300)
    fields = [inputs.cos_field(2.0, 1.0 + k / 300) for k in range(300)]
    fn = np.stack([_field_nodes("CF4", f, 0.0, tau, nsteps) for f in fields])
    psi = dev(psi0)
    st = B.magnus_propagate_ragged(c, [(ham, psi, fn)], B.CF4, tau, opts=B.leja_opts(BUDGET, tol_mode=1), stats=True)
    out = host(psi)
    assert st["exponentials"] == 2 * nsteps * 300
    assert st["iters"] > 0
    P0 = mg.two_term(H1.to_scipy(), H2.to_scipy(), fields[0])
    P1 = mg.two_term(H1.to_scipy(), H2.to_scipy(), fields[299])
    assert rel(out[0], mg.propagate("CF4", P0, tau, nsteps, psi0[0], expm="taylor")) <= BUDGET
    assert rel(out[299], mg.propagate("CF4", P1, tau, nsteps, psi0[299], expm="taylor")) <= BUDGET
    c.close()


@pytest.mark.parametrize("n,batch,persistent", [(10, 1, True), (11, 1, False), (11, 4, True),
                                                (12, 16, False), (12, 32, True)])
def test_small_state_path_selection(n, batch, persistent, monkeypatch):
    """The persistent kernel takes a call when the dimension is within the cap for
    its state count (1024; 2048 from 4 states; 4096 from 32), otherwise every
    Leja iteration is a grid launch; both results match the oracle."""
    monkeypatch.setenv("MAGNUS_PERSIST", "1")
    tau, nsteps = 0.01, 3
    H1, H2 = chain(n)
    c = B.Context(max_dim=1 << n, max_batch=batch)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
    psi0 = inputs.random_states(1 << n, seed=700 + n, batch=batch)
    f = inputs.cos_field(2.0)
    psi = dev(psi0)
    c.timing(True)
    B.propagate(c, ham, B.CF4, tau, _field_nodes("CF4", f, 0.0, tau, nsteps), psi,
                opts=B.leja_opts(BUDGET, tol_mode=1))
    launches = c.timing_read(B.KERNEL_PERSIST)[1]
    c.timing(False)
    assert (launches > 0) == persistent
    out = host(psi)
    ref = mg.propagate("CF4", mg.two_term(H1.to_scipy(), H2.to_scipy(), f), tau, nsteps, psi0[batch - 1],
                       expm="taylor")
    assert rel(out[batch - 1], ref) <= BUDGET
    c.close()


@pytest.mark.parametrize("variant", ["7"])
@pytest.mark.parametrize("N", [1, 2, 3, 5, 17, 130, 1000, 5000])
def test_streamed_tiles_small_and_degenerate(N, variant, monkeypatch):
    """The streamed wave-tile kernel on dimensions that leave most tiles and waves of a
    workgroup empty, rows without entries and an H2 without entries (null arrays):
    it matches the oracle and the 8-row wave-tile kernel, which sums in the same order;
    and its two-pass form of the matrix-free commutator matches the oracle."""
    import scipy.sparse as sp
    H1, A1 = _tiny_hermitian(N, seed=1900 + N, density=0.5 if N <= 130 else 0.02,
                             empty_rows=(N // 2,) if N > 2 else ())
    H2z = inputs.CSR(np.zeros(N + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, complex), N)
    H2, A2 = _tiny_hermitian(N, seed=1950 + N, density=0.3 if N <= 130 else 0.01)
    v = inputs.random_states(N, seed=1960 + N)
    tol = 1e-12
    for second, A2d in ((H2z, np.zeros((N, N))), (H2, A2)):
        out = {}
        for var in (variant, "5"):
            monkeypatch.setenv("MAGNUS_CSR_VARIANT", var)
            c = B.Context(max_dim=N)
            ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, second))
            out[var] = host(B.expmv_leja(c, ham, 0.7, -0.3, 0.0, 0.05, dev(v), opts=B.leja_opts(tol)))
            c.close()
        ref = oe.expmv_taylor(oracle_exponent(sp.csr_matrix(A1), sp.csr_matrix(A2d), 0.7, -0.3, 0.0, 0.05), v)
        assert rel(out[variant], ref) <= 20 * tol, N
        assert rel(out[variant], out["5"]) <= 1e-14, N
    # a commutator exponent: the matrix-free commutator's two streamed passes
    monkeypatch.setenv("MAGNUS_CSR_VARIANT", variant)
    c = B.Context(max_dim=N)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
    w = host(B.expmv_leja(c, ham, 0.7, -0.3, 0.02, 0.05, dev(v), opts=B.leja_opts(tol)))
    c.close()
    ref = oe.expmv_taylor(oracle_exponent(sp.csr_matrix(A1), sp.csr_matrix(A2), 0.7, -0.3, 0.02, 0.05), v)
    assert rel(w, ref) <= 20 * tol, N


def test_streamed_tiles_large_ragged(monkeypatch):
    """The streamed kernel on a large irregular matrix (over 2,000 blocks of 256
    rows, the last one ragged, with empty rows and rows longer than two LDS chunks):
    it matches the oracle and the 8-row wave-tile kernel, which sums in the same
    order, in the Leja pass and in the two-pass matrix-free commutator."""
    N = 2 * 1024 * 256 + 12345
    H1 = _ragged_hermitian(N, 2101, long_rows=(7, N - 3), long_len=700)
    H2 = _ragged_hermitian(N, 2102)
    v = inputs.random_states(N, seed=2103)
    tol = 1e-12
    S1, S2 = H1.to_scipy(), H2.to_scipy()
    for kappa in (0.0, 1e-4):
        out = {}
        for var in ("7", "5"):
            monkeypatch.setenv("MAGNUS_CSR_VARIANT", var)
            c = B.Context(max_dim=N)
            ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
            out[var] = host(B.expmv_leja(c, ham, 0.6, -0.4, kappa, 0.01, dev(v), opts=B.leja_opts(tol)))
            c.close()
        ref = oe.expmv_taylor(oracle_exponent(S1, S2, 0.6, -0.4, kappa, 0.01), v)
        assert rel(out["7"], ref) <= 20 * tol, kappa
        assert rel(out["7"], out["5"]) <= 1e-14, kappa


@pytest.mark.parametrize("stride", [1, 3])
def test_kernel_timing_stride(stride):
    """magnus_timing with stride k brackets every k-th launch of a kernel class: the
    number of bracketed iteration launches is ceil(iterations / k)."""
    H1, H2 = chain(12)
    c = B.Context(max_dim=1 << 12)
    ham = B.magnus_spectral_bounds(c, B.DeviceHamiltonian.from_csr(H1, H2))
    v = dev(inputs.random_states(1 << 12, seed=5))
    c.timing(True, stride=stride)
    _, st = B.expmv_leja(c, ham, 1.0, 0.5, 0.0, 0.05, v, opts=B.leja_opts(1e-12, early_termination=False),
                         stats=True)
    ms, n = c.timing_read(B.KERNEL_CSR_LEJA)
    c.timing(False)
    assert st["iters"] > 3
    assert n == -(-st["iters"] // stride)
    assert ms > 0.0
    with pytest.raises(ValueError):
        c.timing(True, stride=0)
    c.close()
