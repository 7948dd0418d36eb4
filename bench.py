#!/usr/bin/env python3
"""Magnus-Leja propagation benchmark on one MI355X.

Workload (default ``chain_n20``): the open XXZ chain of 20 spins (J = 1,
Delta = 0.5) with a transverse field cos(2t) sum_i X_i, dim 2^20, complex128
CSR (31,981,568 nonzeros over the two terms), psi0 a seeded random unit
vector, tau = 0.01 on [0, 5] (500 steps).  A "step" is one Magnus step (the
Cf4 method, two Leja-interpolated exponentials); M4 (one exponential with the
matrix-free commutator) is timed side by side.  The Leja tolerance 1e-10 is
the budget of the whole 500-step run, i.e. 1e-13 per Cf4 exponential.

Prints one JSON line.  ``value`` is Cf4 Magnus steps per second with inputs
resident in HBM; ``roofline`` covers the dominant kernel (the fused two-term
CSR Leja iteration), timed with HIP events on the library's stream;
``cpu_baseline`` times the CPU oracle (truncated Taylor with scipy CSR) on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def csr_iter_bytes(nnz_total: int, dim: int) -> int:
    """Algorithmic HBM bytes of one fused two-term CSR Leja iteration: 20 B
    per nonzero (4 B column index + 16 B complex128 value), two row-pointer
    arrays (2 x 4 B x (dim+1)), and four complex128 vectors of dim entries
    (gathered w, p read, w_i written, p written)."""
    return 20 * nnz_total + 8 * (dim + 1) + 64 * dim


def comm_iter_bytes(nnz_total: int, dim: int) -> int:
    """Algorithmic bytes of one M4 iteration (two passes): both passes stream
    the CSR terms; pass 1 reads w and writes U, V; pass 2 gathers U, V and
    reads w, p, writes w_i, p."""
    return 2 * (20 * nnz_total + 8 * (dim + 1)) + 48 * dim + 96 * dim


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-m4", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=3)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale the FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (--gpus {args.gpus}, "
              f"WORLD_SIZE {world}); run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1709_06483_amd import binding as B
    from paper_1709_06483_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 16, dtype=torch.complex128, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": True, "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                          "copies": 3}), flush=True)
        return

    cfg = inputs.CONFIGS["chain_n20"]
    n, tau, cfg_steps = cfg["n"], cfg["tau"], cfg["nsteps"]
    dim = 1 << n
    t_build = time.perf_counter()
    H1, H2 = inputs.chain_terms(n, cfg["J"], cfg["Delta"])
    nnz_total = H1.nnz + H2.nnz
    psi0 = inputs.random_states(dim, seed=cfg["psi_seed"])
    f = inputs.cos_field(cfg["omega"])
    print(f"[bench] inputs built in {time.perf_counter() - t_build:.1f}s: dim {dim}, nnz {nnz_total}",
          file=sys.stderr, flush=True)

    ctx = B.Context(max_dim=dim)
    ham = B.magnus_spectral_bounds(ctx, B.DeviceHamiltonian.from_csr(H1, H2))
    W, K = args.warmup, args.steps

    def run(method: str, tol_e: float):
        mid = B.METHODS[method]
        tn = B.magnus_quadrature_nodes(mid, 0.0, tau, W + K)
        fn = np.vectorize(f)(tn)
        psi = torch.from_numpy(psi0).cuda()
        opts = B.leja_opts(tol_e)
        if W:
            B.propagate(ctx, ham, mid, tau, fn[:W], psi, opts=opts)
        torch.cuda.synchronize()
        ctx.timing(True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record()
        _, st = B.propagate(ctx, ham, mid, tau, fn[W:], psi, opts=opts, stats=True)
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = ev0.elapsed_time(ev1)
        kinds = {"leja": B.KERNEL_CSR_LEJA, "split": B.KERNEL_CSR_SPLIT, "comm": B.KERNEL_CSR_COMM}
        kt = {k: ctx.timing_read(v) for k, v in kinds.items()}
        ctx.timing(False)
        ctx.check()
        return ms, wall, st, kt

    out = {}
    # Cf4: two exponentials per step, tolerance budget split over the 500-step run
    tol_cf4 = cfg["budget_tol"] / (2 * cfg_steps)
    ms, wall, st, kt = run("CF4", tol_cf4)
    print(f"[bench] CF4 {K} steps: {ms:.1f} ms (wall {wall:.2f}s), iters {st['iters']}/{st['planned_iters']}",
          file=sys.stderr, flush=True)
    it_bytes = csr_iter_bytes(nnz_total, dim)
    k_ms, k_launch = kt["leja"]
    avg_ms = k_ms / max(k_launch, 1)
    bytes_per_launch = it_bytes * st["iters"] / max(k_launch, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    steps_per_s = K / (ms * 1e-3)
    hv_gbps = it_bytes * st["iters"] / (ms * 1e-3) / 1e9

    if not args.no_m4:
        tol_m4 = cfg["budget_tol"] / cfg_steps
        ms4, wall4, st4, kt4 = run("M4", tol_m4)
        print(f"[bench] M4 {K} steps: {ms4:.1f} ms, iters {st4['iters']}/{st4['planned_iters']}",
              file=sys.stderr, flush=True)
        m4b = comm_iter_bytes(nnz_total, dim)
        out["m4"] = {
            "steps_per_s": K / (ms4 * 1e-3),
            "ms_per_step": ms4 / K,
            "leja_iters_per_step": st4["iters"] / K,
            "hv_gbps": m4b * st4["iters"] / (ms4 * 1e-3) / 1e9,
            "split_kernel_avg_us": 1e3 * kt4["split"][0] / max(kt4["split"][1], 1),
            "comm_kernel_avg_us": 1e3 * kt4["comm"][0] / max(kt4["comm"][1], 1),
            "tol_per_exp": tol_m4,
        }

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(H1, H2, f, tau, psi0, args.cpu_sample_steps)
        print(f"[bench] cpu oracle: {cpu['value']:.3f} steps/s", file=sys.stderr, flush=True)

    line = {
        "metric": "Magnus steps/sec (Cf4) and H*v GB/s at 1e-10 error vs FP64 oracle",
        "value": steps_per_s,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "chain_n20: open XXZ chain J=1 Delta=0.5 + cos(2t) sum X_i, n=20 (dim 1048576), "
                        "complex128 CSR, Cf4, tau=0.01, 500-step run on [0,5], Leja budget 1e-10",
            "dim": dim, "nnz": nnz_total, "tau": tau, "method": "CF4",
            "tol_per_exponential": tol_cf4, "early_termination": True,
        },
        "hv_gbps": hv_gbps,
        "leja_iters_per_step": st["iters"] / K,
        "planned_iters_per_step": st["planned_iters"] / K,
        "roofline": {
            "kernel": "csr2_iter_kernel<64, kLeja>",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "bytes_per_iteration": it_bytes,
            "launches": k_launch,
            "avg_launch_us": avg_ms * 1e3,
        },
        "cpu_baseline": cpu,
        "device": torch.cuda.get_device_name(0),
    }
    line.update(out)
    print(json.dumps(line), flush=True)
    ctx.close()


def cpu_baseline(H1, H2, f, tau, psi0, nsample: int):
    """The CPU oracle (Cf4 with truncated-Taylor exponentials on scipy CSR,
    single-threaded) on the first nsample steps of the same workload."""
    from threadpoolctl import threadpool_limits

    from oracle import magnus as mg

    P = mg.two_term(H1.to_scipy(), H2.to_scipy(), f)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        mg.propagate("CF4", P, tau, nsample, psi0, expm="taylor")
        dt = time.perf_counter() - t0
    return {"value": nsample / dt, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {nsample} Cf4 steps of chain_n20 (oracle-T: Taylor series, a priori remainder "
                      f"1e-17, scipy CSR products, 1 thread), {dt:.1f} s"}


if __name__ == "__main__":
    main()
