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

}  // namespace dev
}  // namespace magnus
