"""Thin ctypes binding of libmagnus (include/magnus.h), same names as the C ABI.

Only argument marshalling happens here: torch tensors supply device memory
and the current HIP stream; every step of the computation runs in the
library's kernels.  Loading fails loudly if the library has not been built
(``python -m paper_1709_06483_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmagnus.so")

OK, EINVAL, EDOMAIN, ENOCONV, EHIP, ENOMEM, ENAN = 0, -1, -2, -3, -4, -5, -6
CSR, DENSE = 0, 1
CF4, M4, M2, CF43, M6 = 0, 1, 2, 3, 4
MAX_DEGREE = 64
METHODS = {"CF4": CF4, "M4": M4, "M2": M2, "CF43": CF43, "M6": M6}


class MagnusError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"magnus status {code}: {msg}")
        self.code = code


class Term(C.Structure):
    _fields_ = [("format", C.c_int32), ("reserved", C.c_int32), ("dim", C.c_int64), ("nnz", C.c_int64),
                ("ld", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("lam_min", C.c_double), ("lam_max", C.c_double)]


class Hamiltonian(C.Structure):
    _fields_ = [("H1", Term), ("H2", Term), ("k_min", C.c_double), ("k_max", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("h", Hamiltonian), ("psi", C.c_void_p), ("batch", C.c_int32), ("batch_f", C.c_int32),
                ("f_nodes", C.POINTER(C.c_double))]


class LejaOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_degree", C.c_int32), ("max_substeps", C.c_int32),
                ("early_termination", C.c_int32), ("tol_mode", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("exponentials", C.c_int64), ("substeps", C.c_int64), ("planned_iters", C.c_int64),
                ("iters", C.c_int64), ("hv_products", C.c_int64), ("max_degree_used", C.c_int32),
                ("max_substeps_used", C.c_int32), ("max_err_bound", C.c_double), ("tol_per_exp", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

# Every symbol include/magnus.h declares.
EXPORTS = ("magnus_create", "magnus_destroy", "magnus_last_error", "magnus_check", "magnus_spectral_bounds",
           "expmv_leja", "magnus_step_cf4", "magnus_step_m4", "propagate", "magnus_quadrature_nodes",
           "magnus_leja_points", "magnus_divided_differences", "magnus_leja_error", "magnus_leja_plan",
           "magnus_timing", "magnus_timing_read", "magnus_reserve_dense", "magnus_adjoint_workspace_bytes",
           "magnus_propagate_adjoint", "magnus_propagate_ragged", "magnus_method_nodes",
           "magnus_dense_commutator", "magnus_dense_m6_prepare", "magnus_autotune",
           "magnus_spectral_bounds_lanczos", "magnus_csr_commutator", "magnus_csr_m6_prepare",
           "magnus_step_cf4_noalloc")
KERNEL_PERSIST, KERNEL_CSR_LEJA3 = 6, 7
KERNEL_CSR_LEJA, KERNEL_CSR_SPLIT, KERNEL_CSR_COMM, KERNEL_DENSE_LEJA, KERNEL_CSR_MULTI, KERNEL_DENSE_MFMA = 0, 1, 2, 3, 4, 5


def lib():
    """Load libmagnus.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1709_06483_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "magnus_create": (C.c_int, [P(vp), i64, i32, i32]),
        "magnus_destroy": (C.c_int, [vp]),
        "magnus_last_error": (C.c_char_p, []),
        "magnus_check": (C.c_int, [vp, vp]),
        "magnus_spectral_bounds": (C.c_int, [vp, P(Hamiltonian), vp]),
        "expmv_leja": (C.c_int, [vp, P(Hamiltonian), dbl, dbl, dbl, dbl, vp, vp, i32, P(LejaOpts), P(Stats), vp]),
        "magnus_step_cf4": (C.c_int, [vp, P(Hamiltonian), dbl, dbl, dbl, vp, vp, i32, P(LejaOpts), P(Stats), vp]),
        "magnus_step_m4": (C.c_int, [vp, P(Hamiltonian), dbl, dbl, dbl, vp, vp, i32, P(LejaOpts), P(Stats), vp]),
        "magnus_step_cf4_noalloc": (C.c_int, [P(Hamiltonian), dbl, dbl, dbl, vp, vp, P(LejaOpts), P(Stats), vp]),
        "propagate": (C.c_int, [vp, P(Hamiltonian), i32, dbl, i64, P(dbl), i32, vp, i32, vp, i32, P(LejaOpts),
                                P(Stats), vp]),
        "magnus_quadrature_nodes": (C.c_int, [i32, dbl, dbl, i64, P(dbl)]),
        "magnus_method_nodes": (C.c_int, [i32]),
        "magnus_leja_points": (C.c_int, [i32, P(dbl)]),
        "magnus_divided_differences": (C.c_int, [dbl, i32, P(dbl)]),
        "magnus_leja_error": (dbl, [dbl, i32]),
        "magnus_leja_plan": (C.c_int, [dbl, dbl, i32, i32, P(i32), P(i32), P(dbl)]),
        "magnus_timing": (C.c_int, [vp, i32]),
        "magnus_timing_read": (C.c_int, [vp, i32, P(dbl), P(i64)]),
        "magnus_reserve_dense": (C.c_int, [vp, i64]),
        "magnus_dense_commutator": (C.c_int, [vp, P(Hamiltonian), vp]),
        "magnus_dense_m6_prepare": (C.c_int, [vp, P(Hamiltonian), vp]),
        "magnus_csr_m6_prepare": (C.c_int, [vp, P(Hamiltonian), vp]),
        "magnus_autotune": (C.c_int, [vp, P(Hamiltonian), i32, P(i32), P(i32), P(dbl), P(dbl), vp]),
        "magnus_spectral_bounds_lanczos": (C.c_int, [vp, P(Hamiltonian), i32, dbl, vp]),
        "magnus_csr_commutator": (C.c_int, [vp, P(Hamiltonian), vp]),
        "magnus_adjoint_workspace_bytes": (i64, [i64, i64, i32]),
        "magnus_propagate_ragged": (C.c_int, [vp, P(Problem), i32, i32, dbl, i64, P(LejaOpts), P(Stats), vp]),
        "magnus_propagate_adjoint": (C.c_int, [vp, P(Hamiltonian), dbl, i64, P(dbl), P(dbl), i32, vp, vp, i32, vp,
                                               i64, P(dbl), P(dbl), P(LejaOpts), P(Stats), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise MagnusError(rc, lib().magnus_last_error().decode(errors="replace"))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---------------------------------------------------------------------------
# Host planning helpers
# ---------------------------------------------------------------------------
def magnus_method_nodes(method: int) -> int:
    q = lib().magnus_method_nodes(method)
    _check(q if q < 0 else OK)
    return q


def magnus_quadrature_nodes(method: int, t0: float, tau: float, nsteps: int) -> np.ndarray:
    q = magnus_method_nodes(method)
    out = np.zeros(q * nsteps, dtype=np.float64)
    _check(lib().magnus_quadrature_nodes(method, t0, tau, nsteps, _dptr(out)))
    return out.reshape(nsteps, q)


def magnus_leja_points(m: int) -> np.ndarray:
    out = np.zeros(m + 1)
    _check(lib().magnus_leja_points(m, _dptr(out)))
    return out


def magnus_divided_differences(theta: float, m: int) -> np.ndarray:
    out = np.zeros(2 * (m + 1))
    _check(lib().magnus_divided_differences(theta, m, _dptr(out)))
    return out[0::2] + 1j * out[1::2]


def magnus_leja_error(theta: float, m: int) -> float:
    return lib().magnus_leja_error(theta, m)


def magnus_leja_plan(theta: float, tol: float, max_degree: int = MAX_DEGREE, max_substeps: int = 1 << 20):
    m, s, b = C.c_int32(), C.c_int32(), C.c_double()
    _check(lib().magnus_leja_plan(theta, tol, max_degree, max_substeps, C.byref(m), C.byref(s), C.byref(b)))
    return m.value, s.value, b.value


# ---------------------------------------------------------------------------
# Device objects (torch supplies memory and streams)
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Context:
    """A libmagnus context (workspace for states up to max_dim x max_batch)."""

    def __init__(self, max_dim: int, max_batch: int = 1, device: int = 0):
        h = C.c_void_p()
        _check(lib().magnus_create(C.byref(h), max_dim, max_batch, device))
        self.handle = h
        self.device = device
        self.max_dim = max_dim
        self.max_batch = max_batch

    def close(self):
        if self.handle:
            lib().magnus_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self):
        _check(lib().magnus_check(self.handle, _stream()))

    def reserve_dense(self, dim: int):
        """Let groups of states on dense terms use one assembled exponent per Leja iteration."""
        _check(lib().magnus_reserve_dense(self.handle, dim))

    def timing(self, enable: bool, stride: int = 1):
        """Bracket every stride-th launch of each kernel class with HIP events (or stop)."""
        if stride < 1:
            raise ValueError("stride must be at least 1")
        _check(lib().magnus_timing(self.handle, int(stride) if enable else 0))

    def timing_read(self, kind: int):
        """(total milliseconds, bracketed launches) of one kernel class since timing was enabled."""
        t, n = C.c_double(), C.c_int64()
        _check(lib().magnus_timing_read(self.handle, kind, C.byref(t), C.byref(n)))
        return t.value, n.value


@dataclass
class DeviceHamiltonian:
    """H(t) = H1 + f(t) H2 with both terms resident on the device."""

    struct: Hamiltonian
    tensors: tuple  # keeps the device arrays alive
    dim: int
    fmt: int

    @staticmethod
    def from_csr(H1, H2, device: str = "cuda") -> "DeviceHamiltonian":
        """H1, H2: objects with indptr, indices, data (int32, int32, complex128) and dim."""
        torch = _torch()
        ts = []
        terms = []
        for H in (H1, H2):
            rp = torch.from_numpy(np.ascontiguousarray(H.indptr, dtype=np.int32)).to(device)
            ci = torch.from_numpy(np.ascontiguousarray(H.indices, dtype=np.int32)).to(device)
            va = torch.from_numpy(np.ascontiguousarray(H.data, dtype=np.complex128)).to(device)
            ts += [rp, ci, va]
            terms.append(Term(CSR, 0, H.dim, int(ci.numel()), 0, rp.data_ptr(), ci.data_ptr(), va.data_ptr(),
                              0.0, 0.0))
        st = Hamiltonian(terms[0], terms[1], 0.0, 0.0)
        return DeviceHamiltonian(st, tuple(ts), int(H1.dim), CSR)

    @staticmethod
    def from_dense(H1, H2, device: str = "cuda") -> "DeviceHamiltonian":
        """H1, H2: row-major complex128 arrays (numpy or torch) of shape (dim, dim); a device
        tensor whose rows are contiguous but padded (row stride > dim) is used as it is."""
        torch = _torch()
        ts = []
        terms = []
        for H in (H1, H2):
            t = H if isinstance(H, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(H))
            t = t.to(device=device, dtype=torch.complex128)
            if t.stride(1) != 1 or t.stride(0) < t.shape[1]:
                t = t.contiguous()
            ts.append(t)
            n = t.shape[0]
            terms.append(Term(DENSE, 0, n, 0, t.stride(0), None, None, t.data_ptr(), 0.0, 0.0))
        st = Hamiltonian(terms[0], terms[1], 0.0, 0.0)
        return DeviceHamiltonian(st, tuple(ts), int(ts[0].shape[0]), DENSE)


def magnus_spectral_bounds(ctx: Context, ham: DeviceHamiltonian) -> DeviceHamiltonian:
    _check(lib().magnus_spectral_bounds(ctx.handle, C.byref(ham.struct), _stream()))
    return ham


def magnus_spectral_bounds_lanczos(ctx: Context, ham: DeviceHamiltonian, steps: int = 60,
                                   margin: float = 0.01) -> DeviceHamiltonian:
    """Lanczos estimates of the terms' spectra (tighter than Gershgorin, not rigorous)."""
    _check(lib().magnus_spectral_bounds_lanczos(ctx.handle, C.byref(ham.struct), steps, margin, _stream()))
    return ham


def magnus_csr_commutator(ctx: Context, ham: DeviceHamiltonian) -> DeviceHamiltonian:
    """Assemble K = i[H1, H2] of CSR terms in the context (M4 then runs one pass per iteration)."""
    _check(lib().magnus_csr_commutator(ctx.handle, C.byref(ham.struct), _stream()))
    return ham


def magnus_dense_commutator(ctx: Context, ham: DeviceHamiltonian) -> DeviceHamiltonian:
    """Assemble K = i[H1, H2] of dense terms in the context (needed for M4 on dense terms)."""
    _check(lib().magnus_dense_commutator(ctx.handle, C.byref(ham.struct), _stream()))
    return ham


CSR_VARIANTS = {1: "nonzero streaming", 2: "row per lane, 64 rows", 3: "row per lane, 32 rows",
                4: "row per lane, 128 rows", 5: "wave tiles of 8 rows", 6: "wave tiles of 16 rows",
                7: "streamed wave tiles"}


DENSE_ROWS_PER_WAVE = (1, 2, 4)
MFMA_TILES = {0: "32x64, K split in two", 1: "32x64", 2: "64x64", 3: "64x64, K split in two",
              4: "32x128, K split in two", 5: "32x64, LDS-DMA staging",
              6: "64x64, LDS-DMA staging"}


def magnus_autotune(ctx: Context, ham: DeviceHamiltonian, batch: int = 1) -> dict:
    """Time the kernel variants on these terms and keep the fastest in the context.
    CSR terms: the row mappings of the single-state iteration (and multi-state group
    sizes when batch > 1).  Dense terms: rows per wave of the GEMV iteration (and the
    FP64-MFMA tile shapes of group iterations of `batch` states).  Returns the choices
    and the timings."""
    v, g = C.c_int32(), C.c_int32()
    vus = np.zeros(len(CSR_VARIANTS))
    gus = np.zeros(len(MFMA_TILES))
    _check(lib().magnus_autotune(ctx.handle, C.byref(ham.struct), batch, C.byref(v), C.byref(g), _dptr(vus),
                                 _dptr(gus), _stream()))
    if ham.struct.H1.format == DENSE:
        return {"rows_per_wave": int(v.value), "mfma_tile": int(g.value) if batch > 1 else None,
                "mfma_tile_name": MFMA_TILES[int(g.value)] if batch > 1 else None,
                "rows_per_wave_us": {str(r): float(vus[k]) for k, r in enumerate(DENSE_ROWS_PER_WAVE)},
                "mfma_tile_us": {MFMA_TILES[t]: (None if np.isnan(gus[t]) else float(gus[t])) for t in MFMA_TILES}}
    return {"variant": int(v.value), "variant_name": CSR_VARIANTS[int(v.value)], "group": int(g.value),
            "variant_us": {CSR_VARIANTS[k + 1]: float(vus[k]) for k in range(len(CSR_VARIANTS))},
            "group_us": {str(b): (None if np.isnan(gus[i]) else float(gus[i])) for i, b in enumerate((2, 4, 8, 16, 32))}}


def magnus_dense_m6_prepare(ctx: Context, ham: DeviceHamiltonian) -> DeviceHamiltonian:
    """Assemble the fixed commutator matrices of M6 for dense terms in the context."""
    _check(lib().magnus_dense_m6_prepare(ctx.handle, C.byref(ham.struct), _stream()))
    return ham


def magnus_csr_m6_prepare(ctx: Context, ham: DeviceHamiltonian) -> DeviceHamiltonian:
    """Assemble K and P_1, P_2 of M6 for CSR terms in the context (nested commutators matrix-free)."""
    _check(lib().magnus_csr_m6_prepare(ctx.handle, C.byref(ham.struct), _stream()))
    return ham


def leja_opts(tol: float = 1e-10, max_degree: int = MAX_DEGREE, max_substeps: int = 1 << 20,
              early_termination: bool = True, tol_mode: int = 0) -> LejaOpts:
    return LejaOpts(tol, max_degree, max_substeps, int(bool(early_termination)), tol_mode)


def _states(x, dim):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or x.dtype != torch.complex128 or not x.is_cuda or not x.is_contiguous():
        raise TypeError("states must be contiguous complex128 CUDA tensors")
    if x.shape[-1] != dim or x.dim() not in (1, 2):
        raise ValueError(f"state shape {tuple(x.shape)} does not match dim {dim}")
    return 1 if x.dim() == 1 else x.shape[0]


def _finish(rc, stats, want):
    _check(rc)
    return stats.as_dict() if want else None


def expmv_leja(ctx: Context, ham: DeviceHamiltonian, a: float, b: float, kappa: float, tau: float, v, w=None,
               opts: LejaOpts | None = None, stats: bool = False):
    """w = exp(-i tau (a H1 + b H2 + kappa K)) v.  Returns w (and stats when asked)."""
    torch = _torch()
    batch = _states(v, ham.dim)
    if w is None:
        w = torch.empty_like(v)
    _states(w, ham.dim)
    st = Stats()
    o = opts or leja_opts()
    rc = lib().expmv_leja(ctx.handle, C.byref(ham.struct), a, b, kappa, tau, _ptr(v), _ptr(w), batch, C.byref(o),
                          C.byref(st) if stats else None, _stream())
    s = _finish(rc, st, stats)
    return (w, s) if stats else w


def _step(fn, ctx, ham, tau, f1, f2, psi_in, psi_out, opts, stats):
    torch = _torch()
    batch = _states(psi_in, ham.dim)
    if psi_out is None:
        psi_out = torch.empty_like(psi_in)
    _states(psi_out, ham.dim)
    st = Stats()
    o = opts or leja_opts()
    rc = fn(ctx.handle, C.byref(ham.struct), tau, f1, f2, _ptr(psi_in), _ptr(psi_out), batch, C.byref(o),
            C.byref(st) if stats else None, _stream())
    s = _finish(rc, st, stats)
    return (psi_out, s) if stats else psi_out


def magnus_step_cf4(ctx, ham, tau, f1, f2, psi_in, psi_out=None, opts=None, stats=False):
    return _step(lib().magnus_step_cf4, ctx, ham, tau, f1, f2, psi_in, psi_out, opts, stats)


def magnus_step_m4(ctx, ham, tau, f1, f2, psi_in, psi_out=None, opts=None, stats=False):
    return _step(lib().magnus_step_m4, ctx, ham, tau, f1, f2, psi_in, psi_out, opts, stats)


def magnus_step_cf4_noalloc(ham, tau, f1, f2, psi_in, psi_out, opts=None, stats=False):
    """One Cf4 step of one state without a context: the library's device scratch
    array is the workspace (dim <= 2^17).  psi_out is caller-allocated."""
    if _states(psi_in, ham.dim) != 1 or _states(psi_out, ham.dim) != 1:
        raise ValueError("the allocation-free step takes one state")
    st = Stats()
    o = opts or leja_opts()
    rc = lib().magnus_step_cf4_noalloc(C.byref(ham.struct), tau, f1, f2, _ptr(psi_in), _ptr(psi_out), C.byref(o),
                                       C.byref(st) if stats else None, _stream())
    s = _finish(rc, st, stats)
    return (psi_out, s) if stats else psi_out


def propagate(ctx: Context, ham: DeviceHamiltonian, method: int, tau: float, f_nodes, psi, checkpoints=None,
              every_k: int = 1, opts: LejaOpts | None = None, stats: bool = False):
    """nsteps = len(f_nodes) steps in place on psi.  f_nodes: (nsteps, q) or (batch, nsteps, q) host
    array of the field at the method's q quadrature nodes (magnus_quadrature_nodes)."""
    batch = _states(psi, ham.dim)
    f = np.ascontiguousarray(f_nodes, dtype=np.float64)
    q = magnus_method_nodes(method)
    if f.ndim == 2:
        batch_f, nsteps = 1, f.shape[0]
    elif f.ndim == 3:
        batch_f, nsteps = f.shape[0], f.shape[1]
    else:
        raise ValueError(f"f_nodes must be (nsteps, {q}) or (batch, nsteps, {q})")
    if f.shape[-1] != q:
        raise ValueError(f"f_nodes last axis must hold the method's {q} node samples")
    ck = None
    if checkpoints is not None:
        _states(checkpoints.reshape(-1, ham.dim), ham.dim)
        need = ((nsteps + every_k - 1) // every_k + 1) * batch * ham.dim
        if checkpoints.numel() < need:
            raise ValueError(f"checkpoints hold {checkpoints.numel()} values, need {need}")
        ck = _ptr(checkpoints)
    st = Stats()
    o = opts or leja_opts()
    rc = lib().propagate(ctx.handle, C.byref(ham.struct), method, tau, nsteps, _dptr(f), batch_f, _ptr(psi),
                         batch, ck, every_k, C.byref(o), C.byref(st) if stats else None, _stream())
    s = _finish(rc, st, stats)
    return (psi, s) if stats else psi


def magnus_adjoint_workspace_bytes(dim: int, nsteps: int, every_k: int) -> int:
    return int(lib().magnus_adjoint_workspace_bytes(dim, nsteps, every_k))


def magnus_propagate_adjoint(ctx: Context, ham: DeviceHamiltonian, tau: float, f_nodes, df_nodes, psi0, psi_target,
                             every_k: int = 16, opts: LejaOpts | None = None, stats: bool = False, workspace=None):
    """Loss 1 - |<psi_target, psi_N>|^2 of a Cf4 run and its gradient with respect to the
    parameters behind the field samples.  f_nodes (nsteps, 2); df_nodes (nsteps, 2, P).
    Returns (loss, grad[P]) (and stats when asked)."""
    torch = _torch()
    f = np.ascontiguousarray(f_nodes, dtype=np.float64)
    df = np.ascontiguousarray(df_nodes, dtype=np.float64)
    nsteps = f.shape[0]
    if f.shape != (nsteps, 2) or df.ndim != 3 or df.shape[:2] != (nsteps, 2):
        raise ValueError("f_nodes must be (nsteps, 2) and df_nodes (nsteps, 2, P)")
    P = df.shape[2]
    for t in (psi0, psi_target):
        if _states(t, ham.dim) != 1:
            raise ValueError("psi0 and psi_target are single states")
    need = magnus_adjoint_workspace_bytes(ham.dim, nsteps, every_k)
    if workspace is None or workspace.numel() * workspace.element_size() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=psi0.device)
    loss = C.c_double()
    grad = np.zeros(max(P, 1))
    st = Stats()
    o = opts or leja_opts()
    rc = lib().magnus_propagate_adjoint(ctx.handle, C.byref(ham.struct), tau, nsteps, _dptr(f), _dptr(df), P,
                                        _ptr(psi0), _ptr(psi_target), every_k, _ptr(workspace),
                                        workspace.numel() * workspace.element_size(), C.byref(loss), _dptr(grad),
                                        C.byref(o), C.byref(st) if stats else None, _stream())
    s = _finish(rc, st, stats)
    out = (loss.value, grad[:P].copy())
    return (out + (s,)) if stats else out


def magnus_propagate_ragged(ctx: Context, problems, method: int, tau: float, opts: LejaOpts | None = None,
                            stats: bool = False):
    """problems: list of (DeviceHamiltonian, psi, f_nodes) with psi (batch, dim) or (dim,) device
    states propagated in place and f_nodes (nsteps, q) or (batch, nsteps, q)."""
    arr = (Problem * len(problems))()
    keep = []
    nsteps = None
    q = magnus_method_nodes(method)
    for i, (ham, psi, f_nodes) in enumerate(problems):
        batch = _states(psi, ham.dim)
        f = np.ascontiguousarray(f_nodes, dtype=np.float64)
        if f.shape[-1] != q:
            raise ValueError(f"problem {i}: f_nodes last axis must hold the method's {q} node samples")
        batch_f = 1 if f.ndim == 2 else f.shape[0]
        ns = f.shape[-2]
        if nsteps is None:
            nsteps = ns
        elif ns != nsteps:
            raise ValueError("all problems need the same number of steps")
        keep.append(f)
        arr[i] = Problem(ham.struct, psi.data_ptr(), batch, batch_f, _dptr(f))
    st = Stats()
    o = opts or leja_opts()
    rc = lib().magnus_propagate_ragged(ctx.handle, arr, len(problems), method, tau, nsteps, C.byref(o),
                                       C.byref(st) if stats else None, _stream())
    del keep
    return _finish(rc, st, stats)
