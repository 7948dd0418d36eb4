// Device helpers shared by the HIP kernels of libmagnus (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace magnus {
namespace dev {

using d2 = double __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;

__device__ __forceinline__ d2 cmul(d2 a, d2 b) { return d2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ d2 rmul(double s, d2 a) { return d2{s * a.x, s * a.y}; }
__device__ __forceinline__ d2 tod2(double2 v) { return d2{v.x, v.y}; }
__device__ __forceinline__ double2 fromd2(d2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double nrm2(d2 v) { return v.x * v.x + v.y * v.y; }

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of row blocks so rows that share gathered vector entries
// share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7, x = b & 7, k = b >> 3;
  return x * q + min(x, rem) + k;
}

__device__ __forceinline__ int load_stopped(const Slot* s) {
  return __hip_atomic_load(&s->stopped, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Cross-lane exchange through a wave-private LDS slice: wait for this wave's
// LDS traffic and keep the compiler from moving memory operations across.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

// Early-termination verdict of one Leja substep from the reduced norms of the
// iteration just finished (Section 3; our reading: stop once
// |d_i| |w_i| + |d_{i-1}| |w_{i-1}| <= tol |v|).
__device__ __forceinline__ void leja_verdict(Slot* S, bool first, bool early, double tol, double dabs,
                                             double d0abs, double wsq, double vsq) {
  const double wn = sqrt(wsq);
  const double vn = first ? sqrt(vsq) : S->vnorm;
  const double prev = first ? d0abs * vn : S->prev_term;
  const double term = dabs * wn;
  const double est = term + prev;
  const bool bad = !isfinite(wsq) || !isfinite(vn);
  if (bad) S->status |= 1;
  S->vnorm = vn;
  S->prev_term = term;
  S->last_est = est;
  S->iters_sub = first ? 1 : S->iters_sub + 1;
  S->stopped = (bad || (early && est <= tol * vn)) ? 1 : 0;
  S->iters_total += 1;
}

// The launch's arguments with the coefficients of the current step read from
// its table column when it runs from a replayed graph (uniform scalar loads).
__device__ __forceinline__ IterArgs resolve_args(const IterArgs& in) {
  IterArgs a = in;
  if (!in.coef) return a;
  const IterCoef* c = in.coef + (long long)(*in.step) * in.coef_stride;
  if (!in.unit_a) {
    a.a1 = c->a1;
    a.a2 = c->a2;
  }
  a.kap = c->kap;
  a.sigma = c->sigma;
  a.d = make_double2(c->dre, c->dim);
  a.d0 = make_double2(c->d0re, c->d0im);
  a.dabs = c->dabs;
  a.d0abs = c->d0abs;
  a.prev_dabs = c->prev_dabs;
  a.tol = c->tol;
  a.skip = !c->active;
  return a;
}

// Whether an iteration launch must return at once because its substep has
// stopped.  Without a.fused the verdict of the previous iteration is in the
// slot (written by the decide kernel launched after it).  With a.fused, every
// workgroup reduces the previous iteration's partials itself in one fixed
// order (each thread a fixed subset in order, then the waves in order), so
// every workgroup reaches the same verdict; workgroup 0 records it in the
// slot and counts the iteration.  Called by every thread of the workgroup;
// the result is uniform over it.  Slot fields written here are never read by
// the same launch: term[] is double-buffered by iteration parity, vnorm is
// written on the second iteration only, when every workgroup computes it.
// lds: kFuseLds doubles of the caller's LDS, free to reuse once this returns.
constexpr int kFuseLds = 40;
__device__ __forceinline__ bool iteration_stopped(const IterArgs& a, double* lds) {
  if (!a.fused) return a.skip || (a.check_stop && load_stopped(a.slot));
  Slot* S = a.slot;
  const int tid = threadIdx.x;
  if (!a.check_stop) {  // a substep's first iteration: it always runs
    if (blockIdx.x == 0 && tid == 0) {
      S->stopped = 0;
      S->iters_sub = 1;
      S->iters_total += 1;
    }
    return false;
  }
  // The partial sums are loaded before a replayed launch's record (which
  // says whether the iteration is past its step's degree) is looked at, so
  // the two latencies overlap; a skipped iteration discards the sums.
  double* fz_w = lds;       // per-wave sums (at most 16 waves)
  double* fz_v = lds + 16;
  if (tid == 0) lds[32] = load_stopped(S) ? 1.0 : 0.0;
  const int n = a.prev_grid, nt = blockDim.x;
  const bool vfirst = a.iter == 2;  // the previous iteration was the substep's first
  const double* P = a.prev_partials;
  constexpr int kU = 8;
  double sw = 0.0, sv = 0.0;
  for (int k0 = 0; k0 < n; k0 += kU * nt) {
    double w[kU], v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + u * nt + tid;
      w[u] = k < n ? P[k] : 0.0;
      v[u] = (vfirst && k < n) ? P[n + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      sw += w[u];
      sv += v[u];
    }
  }
  sw = wave_sum(sw);
  sv = wave_sum(sv);
  const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
  if (lane == 0) {
    fz_w[wv] = sw;
    fz_v[wv] = sv;
  }
  __syncthreads();
  // past this step's degree (uniform: scalar loads), or stopped by an earlier verdict of this substep
  if (a.skip || lds[32] != 0.0) return true;
  double tw = 0.0, tv = 0.0;
  for (int w = 0; w < nw; ++w) {
    tw += fz_w[w];
    tv += fz_v[w];
  }
  __syncthreads();  // every wave has read the sums: the caller may reuse lds
  const double vn = vfirst ? sqrt(tv) : S->vnorm;
  const double prev = vfirst ? a.d0abs * vn : S->term[a.iter & 1];  // iteration iter-2's term
  const double term = a.prev_dabs * sqrt(tw);
  const double est = term + prev;
  const bool bad = !isfinite(tw) || !isfinite(vn);
  const bool stop = bad || (a.early && est <= a.tol * vn);
  if (blockIdx.x == 0 && tid == 0) {
    if (bad) S->status |= 1;
    if (vfirst) S->vnorm = vn;
    S->term[(a.iter - 1) & 1] = term;
    S->last_est = est;
    if (stop) {
      S->stopped = 1;
    } else {
      S->iters_sub = a.iter;
      S->iters_total += 1;
    }
  }
  return stop;
}

}  // namespace dev
}  // namespace magnus
