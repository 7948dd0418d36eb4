// Whole propagations inside one workgroup, for states of small dimension.
//
// At a few thousand rows a Leja iteration moves well under a megabyte, so
// the cost of separate kernel launches (and of a grid-wide reduction for
// the stop test) dominates.  Here one 1024-thread workgroup carries one state
// through every exponential of the call, with the state's vectors in LDS and
// registers: each Leja iteration is the workgroup's threads over the rows
// (two-term CSR product gathering from LDS, shift, Newton accumulation, norm
// partials), one workgroup barrier, a fixed-order sum of the partials that
// every thread does and the stop verdict, all without leaving the kernel.
// The parameters of every iteration come from the per-call table; the states
// of a call (or several problems of a ragged batch) are separate workgroups of
// one launch.
#include "device_common.h"

namespace magnus {
namespace {

using namespace dev;

constexpr int kPT = 1024;  // threads per workgroup

// sum_k val[k] X[col[k]] over one row, the vector X resident in LDS.
__device__ __forceinline__ d2 row_product(int k0, int k1, const int* __restrict__ col, const d2* __restrict__ val,
                                          const d2* X) {
  d2 s = {0.0, 0.0};
#pragma unroll 4
  for (int k = k0; k < k1; ++k) s += cmul(val[k], X[col[k]]);
  return s;
}

// CAP: the largest dimension the LDS buffers hold.  CACHE (CAP = 1024 only):
// term 1's column indices and values are copied into LDS once, beside the two
// vectors (160 KiB then, one workgroup per CU), and read from there by every
// iteration; n = 10 chain: 5.21 against 6.48 us per iteration, as the
// iteration's time goes mostly to the value loads through the workgroup's one
// CU.  Thread t owns rows
// t, t + kPT, ... (at most CAP / kPT of them); the Newton accumulator and the
// vector each substep starts from stay in its registers, the basis vectors
// w_i in two LDS buffers (iteration i gathers from one and writes the other),
// so the only global traffic of an iteration is the CSR data itself.
template <int CAP, bool CACHE>
__global__ __launch_bounds__(kPT) void persist_propagate_kernel(PersistArgs a) {
  constexpr int R = CAP / kPT;
  __shared__ d2 X[2][CAP];
  __shared__ double red[2][2][kPT / 64];
  __shared__ d2 cval[CACHE ? kPersistCache : 1];
  __shared__ int ccol[CACHE ? kPersistCache : 1];
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const PersistProblem pb = a.probs[a.state_prob[b]];
  const int dim = pb.dim;
  const d2* v1 = reinterpret_cast<const d2*>(pb.t1.val);
  const d2* v2 = reinterpret_cast<const d2*>(pb.t2.val);
  const int* c1 = pb.t1.ci;
  if constexpr (CACHE) {  // term 1's entries in LDS (published by the first barrier below)
    const int nnz1 = min(pb.t1.rp[dim], kPersistCache);  // the host checked that they fit
    for (int k = threadIdx.x; k < nnz1; k += kPT) {
      cval[k] = v1[k];
      ccol[k] = pb.t1.ci[k];
    }
    v1 = cval;
    c1 = ccol;
  }
  d2* state = reinterpret_cast<d2*>(a.state[b]);
  const PersistExp* exps = a.exps + (long long)b * a.nexp;

  // row bounds: kept in registers for one row per thread, re-read (from
  // cache) every iteration for several, which keeps the kernel spill-free
  constexpr int RR = R == 1 ? 1 : 0;
  int s1[1] = {0}, e1[1] = {0}, s2[1] = {0}, e2[1] = {0};
  d2 cur[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int r = tid + k * kPT;
    cur[k] = r < dim ? state[r] : d2{0.0, 0.0};
  }
  if (RR && tid < dim) {
    s1[0] = pb.t1.rp[tid];
    e1[0] = pb.t1.rp[tid + 1];
    s2[0] = pb.t2.rp[tid];
    e2[0] = pb.t2.rp[tid + 1];
  }

  // control state of the stop test, identical in every thread
  Slot* S = &a.slots[b];
  long long iters = 0;
  int status = 0, stopped = 0, iters_sub = 0;
  double vnorm = 0.0, prev = 0.0, est = 0.0;
  int par = 0, rpar = 0;

  for (int e = 0; e < a.nexp; ++e) {
    const PersistExp E = exps[e];
    for (int sub = 0; sub < E.s; ++sub) {
#pragma unroll
      for (int k = 0; k < R; ++k)
        if (tid + k * kPT < dim) X[par][tid + k * kPT] = cur[k];
      __syncthreads();
      d2 P[R];
#pragma unroll
      for (int k = 0; k < R; ++k) P[k] = d2{0.0, 0.0};
      for (int i = 1; i <= E.m; ++i) {
        const ColParam prm = a.table[E.table_off + (i - 1)];
        const bool first = (i == 1);
        const d2 dd = {prm.dre, prm.dim};
        double pw = 0.0, pv = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const int r = tid + k * kPT;
          if (r >= dim) continue;
          const int a1 = RR ? s1[0] : pb.t1.rp[r], b1 = RR ? e1[0] : pb.t1.rp[r + 1];
          const int a2 = RR ? s2[0] : pb.t2.rp[r], b2 = RR ? e2[0] : pb.t2.rp[r + 1];
          const d2 y1 = row_product(a1, b1, c1, v1, X[par]);
          const d2 y2 = row_product(a2, b2, pb.t2.ci, v2, X[par]);
          const d2 xr = X[par][r];
          const d2 wn = rmul(prm.a1, y1) + rmul(prm.a2, y2) - rmul(prm.sigma, xr);
          if (first) {
            P[k] = cmul(d2{prm.d0re, prm.d0im}, xr) + cmul(dd, wn);
            pv += nrm2(xr);
          } else {
            P[k] += cmul(dd, wn);
          }
          X[par ^ 1][r] = wn;
          pw += nrm2(wn);
        }
        pw = wave_sum(pw);
        pv = wave_sum(pv);
        if (lane == 0) { red[rpar][0][wv] = pw; red[rpar][1][wv] = pv; }
        __syncthreads();  // publishes w_i and the partial sums
        double tw = 0.0, tv = 0.0;
        for (int w = 0; w < kPT / 64; ++w) { tw += red[rpar][0][w]; tv += red[rpar][1][w]; }
        rpar ^= 1;
        par ^= 1;
        // the early-termination test (same rule as the grid path's decide kernel)
        const double wnrm = sqrt(tw);
        const double vn = first ? sqrt(tv) : vnorm;
        const double pt = first ? prm.d0abs * vn : prev;
        const double term = prm.dabs * wnrm;
        const bool bad = !isfinite(tw) || !isfinite(vn);
        est = term + pt;
        status |= bad ? 1 : 0;
        vnorm = vn;
        prev = term;
        iters_sub = first ? 1 : iters_sub + 1;
        stopped = (bad || (a.early && est <= E.tol_sub * vn)) ? 1 : 0;
        ++iters;
        if (stopped && i < E.m) break;  // uniform: the remaining terms are below tolerance
      }
#pragma unroll
      for (int k = 0; k < R; ++k) cur[k] = P[k];
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k)
    if (tid + k * kPT < dim) state[tid + k * kPT] = cur[k];
  if (tid == 0) {
    S->stopped = stopped;
    S->iters_sub = iters_sub;
    S->status |= status;
    S->iters_total += iters;
    S->vnorm = vnorm;
    S->prev_term = prev;
    S->last_est = est;
  }
}

}  // namespace

hipError_t launch_persist_propagate(const PersistArgs& a, int nstates, int max_dim, hipStream_t s) {
  if (max_dim <= 1024 && a.cache1) persist_propagate_kernel<1024, true><<<nstates, kPT, 0, s>>>(a);
  else if (max_dim <= 1024) persist_propagate_kernel<1024, false><<<nstates, kPT, 0, s>>>(a);
  else if (max_dim <= kPersistMaxDim) persist_propagate_kernel<kPersistMaxDim, false><<<nstates, kPT, 0, s>>>(a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace magnus
