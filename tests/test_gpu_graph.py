"""Magnus steps of one state replayed from a captured HIP graph (one graph
launch per step, every launch reading its Leja coefficients from a device
table indexed by a step counter) against the same steps enqueued launch by
launch (MAGNUS_GRAPH=0): identical states and iteration counts for Cf4, M4,
Cf4:3 and M2 on the kernel families of the graph path, with checkpoints,
table chunks, degrees that change from step to step and early termination;
and against the CPU oracle."""
import numpy as np
import pytest

from oracle import magnus as mg
from paper_1709_06483_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected only where a GPU exists
    pytest.skip("no GPU", allow_module_level=True)

from paper_1709_06483_amd import binding as B  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run(monkeypatch, graph, H1, H2, method, f, tau, nsteps, psi0, tol=1e-12, widen=1.0, every_k=None,
        chunk=None, comm=False):
    monkeypatch.setenv("MAGNUS_GRAPH", str(graph))
    if chunk:
        monkeypatch.setenv("MAGNUS_GRAPH_STEPS", str(chunk))
    else:
        monkeypatch.delenv("MAGNUS_GRAPH_STEPS", raising=False)
    ctx = B.Context(max_dim=psi0.shape[0])
    ham = B.magnus_spectral_bounds(ctx, B.DeviceHamiltonian.from_csr(H1, H2))
    if comm:
        B.magnus_csr_commutator(ctx, ham)
    for T in (ham.struct.H1, ham.struct.H2):
        c, r = 0.5 * (T.lam_min + T.lam_max), 0.5 * (T.lam_max - T.lam_min)
        T.lam_min, T.lam_max = c - widen * r, c + widen * r
    psi = torch.from_numpy(psi0).cuda()
    fn = np.vectorize(f)(B.magnus_quadrature_nodes(B.METHODS[method], 0.0, tau, nsteps))
    ck = None
    if every_k:
        ck = torch.empty(((nsteps + every_k - 1) // every_k + 1, psi0.shape[0]), dtype=torch.complex128,
                         device="cuda")
    _, st = B.propagate(ctx, ham, B.METHODS[method], tau, fn, psi, checkpoints=ck, every_k=every_k or 1,
                        opts=B.leja_opts(tol), stats=True)
    out = psi.cpu().numpy(), st, (ck.cpu().numpy() if ck is not None else None)
    ctx.close()
    return out


@pytest.mark.parametrize("n", [13, 14, 18])
@pytest.mark.parametrize("method", ["CF4", "M4", "CF43", "M2"])
def test_graph_replay_matches_launches(monkeypatch, n, method):
    H1, H2 = inputs.chain_terms(n)
    psi0 = inputs.random_states(1 << n, seed=90 + n)
    f = inputs.cos_field(2.0)
    nsteps = 12
    g, sg, _ = run(monkeypatch, 1, H1, H2, method, f, 0.01, nsteps, psi0)
    l, sl, _ = run(monkeypatch, 0, H1, H2, method, f, 0.01, nsteps, psi0)
    print(f"n={n} {method}: iters graph {sg['iters']} / launches {sl['iters']}, planned {sg['planned_iters']}, "
          f"bitwise {np.array_equal(g, l)}", flush=True)
    assert sg["iters"] == sl["iters"] and sg["planned_iters"] == sl["planned_iters"]
    assert sg["exponentials"] == sl["exponentials"]
    assert rel(g, l) <= 1e-14
    if n == 13:
        ref = mg.propagate(method, mg.two_term(H1.to_scipy(), H2.to_scipy(), f), 0.01, nsteps, psi0, expm="taylor")
        assert rel(g, ref) <= 50 * 1e-12 * 3 * nsteps


def test_graph_replay_checkpoints_chunks_and_varying_degrees(monkeypatch):
    # a field ramping from 0 to 30 changes the degree from step to step (records
    # past a step's degree are inactive); tables uploaded in chunks of 5 steps
    n = 14
    H1, H2 = inputs.chain_terms(n)
    psi0 = inputs.random_states(1 << n, seed=5)
    f = lambda t: 30.0 * t
    g, sg, cg = run(monkeypatch, 1, H1, H2, "CF4", f, 0.02, 23, psi0, every_k=7, chunk=5)
    l, sl, cl = run(monkeypatch, 0, H1, H2, "CF4", f, 0.02, 23, psi0, every_k=7)
    assert sg["iters"] == sl["iters"] and sg["planned_iters"] == sl["planned_iters"]
    assert sg["max_degree_used"] > 0
    assert rel(g, l) <= 1e-14
    for a, b in zip(cg, cl):
        assert rel(a, b) <= 1e-14
    ref = mg.propagate("CF4", mg.two_term(H1.to_scipy(), H2.to_scipy(), f), 0.02, 23, psi0, expm="taylor")
    assert rel(g, ref) <= 50 * 1e-12 * 46


def test_graph_replay_early_termination(monkeypatch):
    # e_0 (all spins up) is an eigenvector of the z-field chain's terms; with the
    # enclosures' upper ends at its eigenvalues and a positive field, w_1 vanishes
    # to rounding and every substep stops after two iterations
    n = 14
    out = {}
    for graph in (1, 0):
        monkeypatch.setenv("MAGNUS_GRAPH", str(graph))
        H1, H2 = inputs.chain_terms(n, field_axis="z")
        ctx = B.Context(max_dim=1 << n)
        ham = B.magnus_spectral_bounds(ctx, B.DeviceHamiltonian.from_csr(H1, H2))
        ham.struct.H1.lam_max = 0.5 * (n - 1)
        ham.struct.H2.lam_max = float(n)
        v = np.zeros(1 << n, dtype=np.complex128)
        v[0] = 1.0
        psi = torch.from_numpy(v).cuda()
        _, st = B.propagate(ctx, ham, B.CF4, 0.02, 1.0 + 0.1 * np.ones((10, 2)), psi, opts=B.leja_opts(1e-12),
                            stats=True)
        out[graph] = (psi.cpu().numpy(), st)
        ctx.close()
    (g, sg), (l, sl) = out[1], out[0]
    assert sg["iters"] == sl["iters"] == 2 * sg["exponentials"] < sg["planned_iters"]
    assert rel(g, l) <= 1e-14


def test_graph_replay_m4_assembled_commutator_and_constant_field(monkeypatch):
    # K assembled (three-term iteration); a constant field makes kappa = 0, which
    # the replayed step carries as a zero coefficient of the same launches
    n = 13
    H1, H2 = inputs.chain_terms(n)
    psi0 = inputs.random_states(1 << n, seed=8)
    for f in (inputs.cos_field(2.0), lambda t: 0.7):
        g, sg, _ = run(monkeypatch, 1, H1, H2, "M4", f, 0.01, 8, psi0, comm=True)
        l, sl, _ = run(monkeypatch, 0, H1, H2, "M4", f, 0.01, 8, psi0, comm=True)
        assert sg["iters"] == sl["iters"]
        assert rel(g, l) <= 1e-13
    ref = mg.propagate("M4", mg.two_term(H1.to_scipy(), H2.to_scipy(), lambda t: 0.7), 0.01, 8, psi0, expm="taylor")
    assert rel(g, ref) <= 50 * 1e-12 * 8
