// HIP kernels of libmagnus for gfx950 (CDNA4, wave64).
//
// The hot loop is one Leja iteration (Section 3, the Newton-form recurrence
// w <- A w - xi_{i-1} w, p <- p + d_i w), fused into a single pass over the
// Hamiltonian: the matrix-vector product of both terms of H(t) = H1 + f H2
// (Section 4), the shift, the accumulation into p, and the partial sums of
// |w_i|^2 (and |v|^2 on the first iteration) for the error control.  A
// one-workgroup kernel that follows reduces the partials in a fixed order and
// writes the early-termination verdict for the next iteration to read, so the
// host never waits.
#include "device_common.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace magnus {
namespace {

using namespace dev;

// Leja update for one row; y = (scale-folded) H_hat w at that row.
__device__ __forceinline__ void leja_row(const IterArgs& a, int r, d2 y, double& pw, double& pv) {
  const d2 w_old = tod2(a.wcur[r]);
  const d2 wn = y - rmul(a.sigma, w_old);
  d2 p;
  if (a.first) {
    p = cmul(tod2(a.d0), w_old) + cmul(tod2(a.d), wn);
    pv += nrm2(w_old);
  } else {
    p = tod2(a.pacc[r]) + cmul(tod2(a.d), wn);
  }
  a.wout[r] = fromd2(wn);
  a.pacc[r] = fromd2(p);
  pw += nrm2(wn);
}

// |w_i|^2 of the workgroup at partials[blockIdx.x]; on a substep's first
// iteration also |v|^2 at partials[gridDim.x + blockIdx.x].
__device__ __forceinline__ void store_partials(const IterArgs& a, double bw, double bv) {
  a.partials[blockIdx.x] = bw;
  if (a.first) a.partials[gridDim.x + blockIdx.x] = bv;
}

// Block sums of the norm partials, one pair per workgroup (plain stores: the
// reduction across workgroups happens in leja_decide_kernel, after this
// kernel has finished, so no device-scope atomics or fences are needed).
__device__ void block_partials(const IterArgs& a, double pw, double pv) {
  __shared__ double red[2][kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  pw = wave_sum(pw);
  pv = wave_sum(pv);
  if (lane == 0) { red[0][wv] = pw; red[1][wv] = pv; }
  __syncthreads();
  if (tid == 0) {
    double bw = 0.0, bv = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) { bw += red[0][w]; bv += red[1][w]; }
    store_partials(a, bw, bv);
  }
}

// One workgroup: reduce the partials of the iteration just finished in a
// fixed order, then the early-termination test of Section 3 (our reading:
// stop once |d_i w_i| + |d_{i-1} w_{i-1}| <= tol |v|).  Every thread issues
// all of its loads before summing, so the kernel costs about one memory
// round trip.  The kernel sits between every two iterations, so its own
// dispatch and completion matter on small grids: four waves dispatch and
// finish sooner than sixteen (measured, Cf4 on chains: n = 13 6,531 -> 7,548
// steps/s, n = 16 3,579 -> 3,829, n = 20 unchanged).
constexpr int kDecideThreads = 256;
constexpr int kDecidePer = 16;
// sum of p[0..n) over the workgroup's threads (each thread's loads all issued first)
__device__ __forceinline__ double decide_sum(const double* p, int n, int tid) {
  double s = 0.0;
  for (int k0 = 0; k0 < n; k0 += kDecideThreads * kDecidePer) {
    double v[kDecidePer];
#pragma unroll
    for (int u = 0; u < kDecidePer; ++u) {
      const int k = k0 + u * kDecideThreads + tid;
      v[u] = k < n ? p[k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kDecidePer; ++u) s += v[u];
  }
  return s;
}

__global__ __launch_bounds__(kDecideThreads) void leja_decide_kernel(IterArgs a, int grid) {
  __shared__ double red[2][kDecideThreads / 64];
  if (a.check_stop && load_stopped(a.slot)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // |v|^2 partials exist (and matter) only on a substep's first iteration
  double sw = decide_sum(a.partials, grid, tid);
  double sv = a.first ? decide_sum(a.partials + grid, grid, tid) : 0.0;
  sw = wave_sum(sw);
  sv = wave_sum(sv);
  if (lane == 0) { red[0][wv] = sw; red[1][wv] = sv; }
  __syncthreads();
  if (tid == 0) {
    double tw = 0.0, tv = 0.0;
    for (int w = 0; w < kDecideThreads / 64; ++w) { tw += red[0][w]; tv += red[1][w]; }
    leja_verdict(a.slot, a.first, a.early, a.tol, a.dabs, a.d0abs, tw, tv);
  }
}

// After the last iteration of a call whose stop tests were fused into the
// iteration kernels: no later launch reduces that iteration's partials, so
// this one checks them for non-finite norms (unless the substep had stopped
// before it, leaving stale partials).
__global__ __launch_bounds__(kDecideThreads) void leja_final_check_kernel(IterArgs a) {
  __shared__ double red[2][kDecideThreads / 64];
  if (load_stopped(a.slot)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double sw = decide_sum(a.prev_partials, a.prev_grid, tid);
  double sv = a.iter == 2 ? decide_sum(a.prev_partials + a.prev_grid, a.prev_grid, tid) : 0.0;
  sw = wave_sum(sw);
  sv = wave_sum(sv);
  if (lane == 0) { red[0][wv] = sw; red[1][wv] = sv; }
  __syncthreads();
  if (tid == 0) {
    double tw = 0.0, tv = 0.0;
    for (int w = 0; w < kDecideThreads / 64; ++w) { tw += red[0][w]; tv += red[1][w]; }
    if (!isfinite(tw) || !isfinite(tv)) a.slot->status |= 1;
  }
}

// ---------------------------------------------------------------------------
// Two-term CSR iteration.  A workgroup owns ROWS consecutive rows; all of its
// threads stream the rows' nonzeros of both terms (coalesced, non-temporal,
// so the gathered vectors keep the caches), multiply by the gathered vector
// entries and stage the products in LDS; then LPR threads per row sum the
// row's products in a fixed order.  Any nonzero distribution is handled by
// processing the workgroup's nonzeros in chunks of CAP.
// ---------------------------------------------------------------------------
template <int ROWS, int MODE>
__global__ __launch_bounds__(kThreads) void csr2_iter_kernel(CsrDev t1, CsrDev t2, int dim, IterArgs a_in) {
  const IterArgs a = resolve_args(a_in);
  constexpr int LPR = kThreads / ROWS;
  constexpr int CAP = ROWS * 32;
  constexpr int U = 4;
  __shared__ d2 prod[CAP];
  __shared__ int rps[2][ROWS + 1];
  static_assert(2 * CAP >= kFuseLds, "stop-test scratch");
  if (iteration_stopped(a, reinterpret_cast<double*>(prod))) return;

  const int tid = threadIdx.x;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int row0 = L * ROWS;
  const int nrows = min(ROWS, dim - row0);
  for (int i = tid; i <= nrows; i += kThreads) {
    rps[0][i] = t1.rp[row0 + i];
    rps[1][i] = t2.rp[row0 + i];
  }
  __syncthreads();
  const int base1 = rps[0][0], n1 = rps[0][nrows] - base1;
  const int base2 = rps[1][0], n2 = rps[1][nrows] - base2;
  const int total = n1 + n2;
  const int rr = tid / LPR, q = tid % LPR;
  int s1 = 0, e1 = 0, s2 = 0, e2 = 0;
  if (rr < nrows) {
    s1 = rps[0][rr] - base1;
    e1 = rps[0][rr + 1] - base1;
    s2 = n1 + rps[1][rr] - base2;
    e2 = n1 + rps[1][rr + 1] - base2;
  }
  const d2* x1 = reinterpret_cast<const d2*>(a.x1);
  const d2* x2 = reinterpret_cast<const d2*>(a.x2);
  const d2* v1 = reinterpret_cast<const d2*>(t1.val);
  const d2* v2 = reinterpret_cast<const d2*>(t2.val);
  d2 acc1 = {0.0, 0.0}, acc2 = {0.0, 0.0};

  for (int c0 = 0; c0 < total; c0 += CAP) {
    const int cn = min(CAP, total - c0);
    for (int kb = 0; kb < cn; kb += kThreads * U) {
      int col[U];
      d2 val[U];
      bool in1[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = kb + u * kThreads + tid;
        const int g = c0 + k;
        in1[u] = g < n1;
        col[u] = 0;
        val[u] = d2{0.0, 0.0};
        if (k < cn) {
          if (in1[u]) {
            col[u] = __builtin_nontemporal_load(t1.ci + base1 + g);
            val[u] = __builtin_nontemporal_load(v1 + base1 + g);
          } else {
            col[u] = __builtin_nontemporal_load(t2.ci + base2 + (g - n1));
            val[u] = __builtin_nontemporal_load(v2 + base2 + (g - n1));
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = kb + u * kThreads + tid;
        if (k < cn) {
          const d2 x = in1[u] ? x1[col[u]] : x2[col[u]];
          prod[k] = cmul(val[u], x);
        }
      }
    }
    __syncthreads();
    if (rr < nrows) {
      const int hi = c0 + cn;
      for (int k = max(s1, c0) + q; k < min(e1, hi); k += LPR) acc1 += prod[k - c0];
      for (int k = max(s2, c0) + q; k < min(e2, hi); k += LPR) acc2 += prod[k - c0];
    }
    __syncthreads();
  }
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) {
    acc1.x += __shfl_xor(acc1.x, off, 64);
    acc1.y += __shfl_xor(acc1.y, off, 64);
    acc2.x += __shfl_xor(acc2.x, off, 64);
    acc2.y += __shfl_xor(acc2.y, off, 64);
  }
  const bool owner = (q == 0) && (rr < nrows);
  const int r = row0 + rr;
  if constexpr (MODE == kSplit) {
    if (owner) {
      a.wout[r] = fromd2(acc1);
      a.pacc[r] = fromd2(acc2);
    }
    return;
  } else {
    double pw = 0.0, pv = 0.0;
    if (owner) {
      d2 y;
      if constexpr (MODE == kLeja) {
        y = rmul(a.a1, acc1) + rmul(a.a2, acc2);
      } else {
        const d2 Ur = x2[r], Vr = x1[r];
        const d2 dl = acc1 - acc2;
        y = rmul(a.a1, Ur) + rmul(a.a2, Vr) + d2{-a.kap * dl.y, a.kap * dl.x};
      }
      leja_row(a, r, y, pw, pv);
    }
    block_partials(a, pw, pv);
  }
}

// ---------------------------------------------------------------------------
// Two-term CSR iteration, row-per-lane variant.  The workgroup first copies
// its rows' column indices and values (both terms) into LDS with coalesced,
// non-temporal loads; then lane l of every wave owns row row0 + l and wave q
// walks the row's entries k = q, q + 4, ... .  Neighbouring lanes therefore
// gather x at the same position of neighbouring rows, which for structured
// Hamiltonians (neighbouring basis states couple to neighbouring states) turns
// most gathers into contiguous 1 KiB loads.  The four partial sums per row are
// combined in LDS in a fixed order and wave 0 applies the Leja update to 64
// consecutive rows with coalesced stores.
// ---------------------------------------------------------------------------
template <int ROWS, int MODE>
__global__ __launch_bounds__(kThreads) void csr2_rowlane_kernel(CsrDev t1, CsrDev t2, int dim, IterArgs a_in) {
  const IterArgs a = resolve_args(a_in);
  constexpr int NW = kThreads / ROWS;  // entry groups per row
  constexpr int CAP = ROWS * 32;
  constexpr int U = CAP / kThreads;
  __shared__ d2 sval[CAP];
  __shared__ int scol[CAP];
  __shared__ int rps[2][ROWS + 1];
  __shared__ d2 part[2][NW][ROWS];
  __shared__ double wred[2][kThreads / 64];
  static_assert(2 * CAP >= kFuseLds, "stop-test scratch");
  if (iteration_stopped(a, reinterpret_cast<double*>(sval))) return;

  const int tid = threadIdx.x;
  const int lane = tid % ROWS, wv = tid / ROWS;  // row within the block, entry group
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int row0 = L * ROWS;
  const int nrows = min(ROWS, dim - row0);
  for (int i = tid; i <= nrows; i += kThreads) {
    rps[0][i] = t1.rp[row0 + i];
    rps[1][i] = t2.rp[row0 + i];
  }
  __syncthreads();
  const int base1 = rps[0][0], n1 = rps[0][nrows] - base1;
  const int base2 = rps[1][0], n2 = rps[1][nrows] - base2;
  const int total = n1 + n2;
  // this lane's row segments in the concatenated (term 1, term 2) sequence
  int s1 = 0, e1 = 0, s2 = 0, e2 = 0;
  if (lane < nrows) {
    s1 = rps[0][lane] - base1;
    e1 = rps[0][lane + 1] - base1;
    s2 = n1 + rps[1][lane] - base2;
    e2 = n1 + rps[1][lane + 1] - base2;
  }
  const d2* x1 = reinterpret_cast<const d2*>(a.x1);
  const d2* x2 = reinterpret_cast<const d2*>(a.x2);
  const d2* v1 = reinterpret_cast<const d2*>(t1.val);
  const d2* v2 = reinterpret_cast<const d2*>(t2.val);
  d2 acc1 = {0.0, 0.0}, acc2 = {0.0, 0.0};

  for (int c0 = 0; c0 < total; c0 += CAP) {
    const int cn = min(CAP, total - c0);
    int col[U];
    d2 val[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = u * kThreads + tid;
      const int g = c0 + k;
      col[u] = 0;
      val[u] = d2{0.0, 0.0};
      if (k < cn) {
        if (g < n1) {
          col[u] = __builtin_nontemporal_load(t1.ci + base1 + g);
          val[u] = __builtin_nontemporal_load(v1 + base1 + g);
        } else {
          col[u] = __builtin_nontemporal_load(t2.ci + base2 + (g - n1));
          val[u] = __builtin_nontemporal_load(v2 + base2 + (g - n1));
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = u * kThreads + tid;
      if (k < cn) {
        scol[k] = col[u];
        sval[k] = val[u];
      }
    }
    __syncthreads();
    const int hi = c0 + cn;
    {
      const int lo = max(s1, c0) + wv, end = min(e1, hi);
#pragma unroll 4
      for (int k = lo; k < end; k += NW) acc1 += cmul(sval[k - c0], x1[scol[k - c0]]);
    }
    {
      const int lo = max(s2, c0) + wv, end = min(e2, hi);
#pragma unroll 4
      for (int k = lo; k < end; k += NW) acc2 += cmul(sval[k - c0], x2[scol[k - c0]]);
    }
    __syncthreads();
  }
  part[0][wv][lane] = acc1;
  part[1][wv][lane] = acc2;
  __syncthreads();
  // threads 0..ROWS-1 finish one row each (lane == tid there)
  const bool owner = tid < ROWS && lane < nrows;
  const int r = row0 + lane;
  d2 r1 = {0.0, 0.0}, r2 = {0.0, 0.0};
  if (tid < ROWS) {
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      r1 += part[0][w][lane];
      r2 += part[1][w][lane];
    }
  }
  if constexpr (MODE == kSplit) {
    if (owner) {
      a.wout[r] = fromd2(r1);
      a.pacc[r] = fromd2(r2);
    }
  } else {
    double pw = 0.0, pv = 0.0;
    if (owner) {
      d2 y;
      if constexpr (MODE == kLeja) {
        y = rmul(a.a1, r1) + rmul(a.a2, r2);
      } else {
        const d2 Ur = x2[r], Vr = x1[r];
        const d2 dl = r1 - r2;
        y = rmul(a.a1, Ur) + rmul(a.a2, Vr) + d2{-a.kap * dl.y, a.kap * dl.x};
      }
      leja_row(a, r, y, pw, pv);
    }
    pw = wave_sum(pw);
    pv = wave_sum(pv);
    if ((tid & 63) == 0) { wred[0][tid >> 6] = pw; wred[1][tid >> 6] = pv; }
    __syncthreads();
    if (tid == 0) {
      double bw = 0.0, bv = 0.0;
      for (int k = 0; k < kThreads / 64; ++k) { bw += wred[0][k]; bv += wred[1][k]; }
      store_partials(a, bw, bv);
    }
  }
}

// ---------------------------------------------------------------------------
// Two-term CSR iteration, wave-tile variant.  Every wave owns RPW consecutive
// rows and works through them on its own: it stages its rows' column indices
// and values (both terms) in a private LDS slice with coalesced non-temporal
// loads, gathers x with lanes laid out row-fastest (lane = g * RPW + r, so
// neighbouring lanes gather the same entry position of neighbouring rows),
// sums each row's G = 64 / RPW groups with shuffles in a fixed order and
// applies the Leja update to its RPW rows.  No block-wide barrier separates
// the phases, so the waves of a CU overlap freely; the only barrier combines
// the four waves' norm partials at the end.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wave's LDS accesses are done
  __builtin_amdgcn_wave_barrier();
}

// Seven waves per SIMD (at most 72 VGPRs): enough independent tiles in flight
// per CU to cover the memory latency of each tile's load -> gather chain.  The
// commutator pass holds two more own-row vectors and gets six (no spills).
// keep_entries: tiles whose entries start within the first keep_entries of the
// two terms together are read with normal loads, so that they stay in the
// memory-side cache (MALL) until the next pass over the matrix; the rest are
// read non-temporally.
template <int RPW, int MODE>
__global__ __launch_bounds__(kThreads, MODE == kLejaComm ? 6 : 7) void csr2_wave_kernel(CsrDev t1, CsrDev t2, int dim, IterArgs a_in,
                                                                                      int keep_entries) {
  const IterArgs a = resolve_args(a_in);
  constexpr int NWAVE = kThreads / 64;
  constexpr int G = 64 / RPW;      // entry groups per row
  constexpr int CAPW = RPW * 32;   // entries staged per chunk
  constexpr int U = CAPW / 64;     // entries per lane per chunk
  static_assert(RPW + 1 <= 32, "row pointers are loaded by half-waves");
  __shared__ d2 sval[NWAVE][CAPW];
  __shared__ int scol[NWAVE][CAPW];
  __shared__ int srp[NWAVE][2][RPW + 1];
  __shared__ double wred[2][NWAVE];
  // The stop flag is the same for every wave of the launch; it is tested only
  // once the row pointers and own-row operands are in flight, so its latency
  // overlaps theirs (the fused test reduces the partials first).
  const bool stopped = iteration_stopped(a, reinterpret_cast<double*>(&sval[0][0]));

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int row0 = (L * NWAVE + wv) * RPW;
  const int nrows = max(0, min(RPW, dim - row0));
  const int r = lane % RPW, g = lane / RPW;
  const bool owner = (lane < RPW) && (r < nrows);
  const int row = row0 + r;
  double pw = 0.0, pv = 0.0;

  int rpa = 0, rpb = 0;
  d2 w_old = {0.0, 0.0}, p_old = {0.0, 0.0}, own1 = {0.0, 0.0}, own2 = {0.0, 0.0};
  if (nrows > 0) {
    if (lane <= nrows) rpa = t1.rp[row0 + lane];
    if (lane >= 32 && lane - 32 <= nrows) rpb = t2.rp[row0 + lane - 32];
    // own-row operands of the update, fetched early
    if (owner) {
      if constexpr (MODE != kSplit) {
        w_old = tod2(a.wcur[row]);
        if (!a.first) p_old = tod2(a.pacc[row]);
      }
      if constexpr (MODE == kLejaComm) {
        own1 = tod2(a.x1[row]);
        own2 = tod2(a.x2[row]);
      }
    }
  }
  if (stopped) return;  // uniform over the workgroup

  if (nrows > 0) {
    if (lane <= nrows) srp[wv][0][lane] = rpa;
    if (lane >= 32 && lane - 32 <= nrows) srp[wv][1][lane - 32] = rpb;
    wave_lds_sync();
    const int base1 = srp[wv][0][0], n1 = srp[wv][0][nrows] - base1;
    const int base2 = srp[wv][1][0], n2 = srp[wv][1][nrows] - base2;
    const int total = n1 + n2;
    int s1 = 0, e1 = 0, s2 = 0, e2 = 0;
    if (r < nrows) {
      s1 = srp[wv][0][r] - base1;
      e1 = srp[wv][0][r + 1] - base1;
      s2 = n1 + srp[wv][1][r] - base2;
      e2 = n1 + srp[wv][1][r + 1] - base2;
    }
    const d2* x1 = reinterpret_cast<const d2*>(a.x1);
    const d2* x2 = reinterpret_cast<const d2*>(a.x2);
    const d2* v1 = reinterpret_cast<const d2*>(t1.val);
    const d2* v2 = reinterpret_cast<const d2*>(t2.val);
    d2 acc1 = {0.0, 0.0}, acc2 = {0.0, 0.0};
    const bool keep = (long long)base1 + base2 < keep_entries;  // uniform over the wave (no int overflow)
    for (int c0 = 0; c0 < total; c0 += CAPW) {
      const int cn = min(CAPW, total - c0);
      int col[U];
      d2 val[U];
      auto load_chunk = [&](auto streaming) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = u * 64 + lane;
          const int gk = c0 + k;
          col[u] = 0;
          val[u] = d2{0.0, 0.0};
          auto ld = [&](const auto* p) {
            if constexpr (decltype(streaming)::value) return __builtin_nontemporal_load(p);
            else return *p;
          };
          if (k < cn) {
            if (gk < n1) {
              col[u] = ld(t1.ci + base1 + gk);
              val[u] = ld(v1 + base1 + gk);
            } else {
              col[u] = ld(t2.ci + base2 + (gk - n1));
              val[u] = ld(v2 + base2 + (gk - n1));
            }
          }
        }
      };
      if (keep) load_chunk(std::false_type{});
      else load_chunk(std::true_type{});
      wave_lds_sync();  // the previous chunk's LDS reads are done
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = u * 64 + lane;
        if (k < cn) {
          scol[wv][k] = col[u];
          sval[wv][k] = val[u];
        }
      }
      wave_lds_sync();
      const int hi = c0 + cn;
      {
        const int lo = max(s1, c0) + g, end = min(e1, hi);
#pragma unroll 4
        for (int k = lo; k < end; k += G) acc1 += cmul(sval[wv][k - c0], x1[scol[wv][k - c0]]);
      }
      {
        const int lo = max(s2, c0) + g, end = min(e2, hi);
#pragma unroll 4
        for (int k = lo; k < end; k += G) acc2 += cmul(sval[wv][k - c0], x2[scol[wv][k - c0]]);
      }
    }
#pragma unroll
    for (int off = 32; off >= RPW; off >>= 1) {
      acc1.x += __shfl_xor(acc1.x, off, 64);
      acc1.y += __shfl_xor(acc1.y, off, 64);
      acc2.x += __shfl_xor(acc2.x, off, 64);
      acc2.y += __shfl_xor(acc2.y, off, 64);
    }
    if (owner) {
      if constexpr (MODE == kSplit) {
        a.wout[row] = fromd2(acc1);
        a.pacc[row] = fromd2(acc2);
      } else {
        d2 y;
        if constexpr (MODE == kLeja) {
          y = rmul(a.a1, acc1) + rmul(a.a2, acc2);
        } else {
          // own2 = U_r (term-2 gather vector), own1 = V_r (term-1 gather vector)
          const d2 dl = acc1 - acc2;
          y = rmul(a.a1, own2) + rmul(a.a2, own1) + d2{-a.kap * dl.y, a.kap * dl.x};
        }
        const d2 wn = y - rmul(a.sigma, w_old);
        d2 p;
        if (a.first) {
          p = cmul(tod2(a.d0), w_old) + cmul(tod2(a.d), wn);
          pv = nrm2(w_old);
        } else {
          p = p_old + cmul(tod2(a.d), wn);
        }
        a.wout[row] = fromd2(wn);
        a.pacc[row] = fromd2(p);
        pw = nrm2(wn);
      }
    }
  }
  if constexpr (MODE != kSplit) {
    pw = wave_sum(pw);
    pv = wave_sum(pv);
    if (lane == 0) { wred[0][wv] = pw; wred[1][wv] = pv; }
    __syncthreads();
    if (tid == 0) {
      double bw = 0.0, bv = 0.0;
      for (int k = 0; k < NWAVE; ++k) { bw += wred[0][k]; bv += wred[1][k]; }
      store_partials(a, bw, bv);
    }
  }
}

// ---------------------------------------------------------------------------
// Two-term dense iteration (row-major H1, H2).  A wave owns RPW rows; its
// lanes stride over columns so every matrix load is a coalesced 1 KiB
// transaction, and each gathered x_j is loaded once per lane for RPW rows and
// both terms.
// ---------------------------------------------------------------------------
// Rows below keep_rows are read with normal loads so that they stay in the
// memory-side cache (MALL) from one iteration to the next (the matrix is read
// again by every iteration); the rest stream through non-temporally.
template <int RPW, int NT>
__global__ __launch_bounds__(kThreads) void dense2_iter_kernel(const double2* H1, const double2* H2,
                                                              int dim, long long ld, IterArgs a, int keep_rows) {
  __shared__ double fz[kFuseLds];
  if (iteration_stopped(a, fz)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int rbase = (L * (kThreads / 64) + wv) * RPW;
  const d2* x = reinterpret_cast<const d2*>(a.x1);
  const d2* A1 = reinterpret_cast<const d2*>(H1);
  const d2* A2 = reinterpret_cast<const d2*>(H2);
  d2 acc1[RPW], acc2[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) { acc1[r] = d2{0.0, 0.0}; acc2[r] = d2{0.0, 0.0}; }
  int nr = min(RPW, dim - rbase);
  if (nr < 0) nr = 0;
  // columns in groups of UNR per lane: the same matrix bytes in flight per wave for one term or two
  constexpr int UNR = NT == 2 ? 2 : 4;
  auto run = [&](auto streaming) {
    for (int j0 = lane; j0 < dim; j0 += 64 * UNR) {
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int j = j0 + 64 * u;
        if (j < dim) {
          const d2 xj = x[j];
#pragma unroll
          for (int r = 0; r < RPW; ++r) {
            if (r < nr) {
              const long long off = (long long)(rbase + r) * ld + j;
              if constexpr (decltype(streaming)::value) {
                acc1[r] += cmul(__builtin_nontemporal_load(A1 + off), xj);
                if constexpr (NT == 2) acc2[r] += cmul(__builtin_nontemporal_load(A2 + off), xj);
              } else {
                acc1[r] += cmul(A1[off], xj);
                if constexpr (NT == 2) acc2[r] += cmul(A2[off], xj);
              }
            }
          }
        }
      }
    }
  };
  if (rbase < keep_rows) run(std::false_type{});
  else run(std::true_type{});
  double pw = 0.0, pv = 0.0;
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    d2 s1 = acc1[r], s2 = acc2[r];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s1.x += __shfl_xor(s1.x, off, 64);
      s1.y += __shfl_xor(s1.y, off, 64);
      if constexpr (NT == 2) {
        s2.x += __shfl_xor(s2.x, off, 64);
        s2.y += __shfl_xor(s2.y, off, 64);
      }
    }
    if (lane == r && r < nr) {
      const d2 y = NT == 2 ? rmul(a.a1, s1) + rmul(a.a2, s2) : rmul(a.a1, s1);
      leja_row(a, rbase + r, y, pw, pv);
    }
  }
  block_partials(a, pw, pv);
}

// The first iteration of an exponential on dense terms fused with the
// assembly of its exponent: while it streams H1 and H2 (and K) it stores
// Hs = ca H1 + cb H2 (+ ck K) into the assembly buffer (row stride dim, all
// stores non-temporal: dim 8192 Cf4 382 steps/s, against 367 with the rows
// that the next iterations keep in the MALL stored normally and 354 with all
// stores normal) and multiplies Hs x.  Hs is
// formed by the same expression as dense_assemble_kernel, and every lane
// sums the same columns in the same order as the one-term iteration, so the
// result is bitwise that of assembling first and iterating on the assembled
// matrix; the separate assembly pass and one full read of the assembled
// matrix disappear.
template <int RPW, bool WITH_K>
__global__ __launch_bounds__(kThreads) void dense_assemble_iter_kernel(DenseAssembly D, int dim, IterArgs a) {
  __shared__ double fz[kFuseLds];
  if (iteration_stopped(a, fz)) return;  // a first iteration always runs
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int rbase = (L * (kThreads / 64) + wv) * RPW;
  const d2* x = reinterpret_cast<const d2*>(a.x1);
  const d2* A1 = reinterpret_cast<const d2*>(D.H1);
  const d2* A2 = reinterpret_cast<const d2*>(D.H2);
  const d2* Kp = reinterpret_cast<const d2*>(D.K);
  d2 acc[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) acc[r] = d2{0.0, 0.0};
  int nr = min(RPW, dim - rbase);
  if (nr < 0) nr = 0;
  constexpr int UNR = 2;
  for (int j0 = lane; j0 < dim; j0 += 64 * UNR) {
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int j = j0 + 64 * u;
      if (j < dim) {
        const d2 xj = x[j];
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          if (r < nr) {
            const long long row = rbase + r;
            d2 h = rmul(D.ca, __builtin_nontemporal_load(A1 + row * D.ld + j)) +
                   rmul(D.cb, __builtin_nontemporal_load(A2 + row * D.ld + j));
            if constexpr (WITH_K) h += rmul(D.ck, __builtin_nontemporal_load(Kp + row * dim + j));
            __builtin_nontemporal_store(h, reinterpret_cast<d2*>(D.out) + row * dim + j);
            acc[r] += cmul(h, xj);
          }
        }
      }
    }
  }
  double pw = 0.0, pv = 0.0;
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    d2 s1 = acc[r];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s1.x += __shfl_xor(s1.x, off, 64);
      s1.y += __shfl_xor(s1.y, off, 64);
    }
    if (lane == r && r < nr) leja_row(a, rbase + r, rmul(a.a1, s1), pw, pv);
  }
  block_partials(a, pw, pv);
}

// ---------------------------------------------------------------------------
// The Method M6 iteration on CSR terms (the exponent's nested commutators
// applied to vectors as commutators of assembled CSR matrices), in two
// passes over the five matrices M = (H1, H2, K, P1, P2), 8 lanes per row,
// each term's products summed in a fixed order:
//   stage A: s_k = (M_k w)[r] for the row, then on the row itself y0 and the
//            five vectors u_k that stage B multiplies (see M6Vecs);
//   stage B: y = y0 + sum_k M_k u_k, then the Leja update and norm partials.
// Grouping the products by matrix reads P1 and P2 twice per iteration where
// applying each commutator product separately reads them three and four times.
// A lane loads its row's bounds in all five matrices before the first product,
// so those loads are in flight together (n = 16: 2,263 against 2,197 steps/s).
// ---------------------------------------------------------------------------
constexpr int kM6Lanes = 8;  // lanes per row

__device__ __forceinline__ d2 times_i(d2 v) { return d2{-v.y, v.x}; }

__global__ __launch_bounds__(kThreads) void m6_stage_a_kernel(M6Terms T, const double2* __restrict__ w, M6Coef C,
                                                             M6Vecs V, int dim, const Slot* slot, int check_stop) {
  if (check_stop && load_stopped(slot)) return;
  const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
  const int r = (int)(t / kM6Lanes), q = (int)(t % kM6Lanes);
  const d2* wv = reinterpret_cast<const d2*>(w);
  d2 sk[kM6Terms];
  int rs[kM6Terms], re[kM6Terms];
#pragma unroll
  for (int k = 0; k < kM6Terms; ++k) {
    rs[k] = r < dim ? T.m[k].rp[r] : 0;
    re[k] = r < dim ? T.m[k].rp[r + 1] : 0;
  }
#pragma unroll
  for (int k = 0; k < kM6Terms; ++k) {
    d2 acc = {0.0, 0.0};
    {
      const d2* av = reinterpret_cast<const d2*>(T.m[k].val);
      for (int e = rs[k] + q; e < re[k]; e += kM6Lanes) acc += cmul(av[e], wv[T.m[k].ci[e]]);
    }
#pragma unroll
    for (int off = kM6Lanes / 2; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off, 64);
      acc.y += __shfl_xor(acc.y, off, 64);
    }
    sk[k] = acc;
  }
  if (r >= dim) return;
  const double* c = C.c;
  // lane q of the row writes output q (all lanes hold the five sums)
  d2 out;
  switch (q) {
    case 0: out = rmul(c[0], sk[0]) + rmul(c[1], sk[1]) + rmul(c[2], sk[2]) + rmul(c[3], sk[3]) + rmul(c[4], sk[4]); break;
    case 1: out = times_i(rmul(c[5], sk[3]) + rmul(c[6], sk[4])); break;
    case 2: out = times_i(rmul(c[7], sk[4])); break;
    case 3: out = times_i(rmul(-c[8], sk[3]) - rmul(c[9], sk[4])); break;
    case 4: out = times_i(rmul(c[8], sk[2]) - rmul(c[5], sk[0])); break;
    case 5: out = times_i(rmul(c[9], sk[2]) - rmul(c[6], sk[0]) - rmul(c[7], sk[1])); break;
    default: return;
  }
  double2* dst = q == 0 ? V.y0 : V.u[q - 1];
  dst[r] = fromd2(out);
}

__global__ __launch_bounds__(kThreads) void m6_stage_b_kernel(M6Terms T, M6Vecs V, double scale, int dim, IterArgs a) {
  if (a.check_stop && load_stopped(a.slot)) return;
  const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
  // rows in reverse order: stage A ends on the last rows, whose matrix entries
  // are still in the MALL when stage B starts on them (and stage B ends on the
  // first rows, where the next iteration's stage A starts)
  const int r0 = (int)(t / kM6Lanes), q = (int)(t % kM6Lanes);
  const int r = r0 < dim ? dim - 1 - r0 : r0;
  d2 acc = {0.0, 0.0};
  if (r < dim) {
    int rs[kM6Terms], re[kM6Terms];
#pragma unroll
    for (int k = 0; k < kM6Terms; ++k) {
      rs[k] = T.m[k].rp[r];
      re[k] = T.m[k].rp[r + 1];
    }
#pragma unroll
    for (int k = 0; k < kM6Terms; ++k) {
      const d2* av = reinterpret_cast<const d2*>(T.m[k].val);
      const d2* uv = reinterpret_cast<const d2*>(V.u[k]);
      for (int e = rs[k] + q; e < re[k]; e += kM6Lanes) acc += cmul(av[e], uv[T.m[k].ci[e]]);
    }
  }
#pragma unroll
  for (int off = kM6Lanes / 2; off > 0; off >>= 1) {
    acc.x += __shfl_xor(acc.x, off, 64);
    acc.y += __shfl_xor(acc.y, off, 64);
  }
  double pw = 0.0, pv = 0.0;
  if (r < dim && q == 0) leja_row(a, r, rmul(scale, tod2(V.y0[r]) + acc), pw, pv);
  block_partials(a, pw, pv);
}

// ---------------------------------------------------------------------------
// Gershgorin discs + structure check (CSR), one thread per row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void csr_gershgorin_kernel(CsrDev t, int dim, long long nnz,
                                                                double* out) {
  __shared__ double smin[kThreads], smax[kThreads];
  __shared__ int sbad[kThreads];
  const int tid = threadIdx.x;
  const int r = blockIdx.x * kThreads + tid;
  double lo = INFINITY, hi = -INFINITY;
  int bad = 0;
  if (r < dim) {
    const long long rs = t.rp[r], re = t.rp[r + 1];
    if (r == 0 && rs != 0) bad = 1;
    if (r == dim - 1 && re != nnz) bad = 1;
    if (rs < 0 || re < rs || re > nnz) bad = 1;
    double diag = 0.0, rad = 0.0;
    if (!bad) {
      for (long long j = rs; j < re; ++j) {
        const int c = t.ci[j];
        const double2 v = t.val[j];
        if (c < 0 || c >= dim) { bad = 1; break; }
        if (c == r) { diag += v.x; rad += fabs(v.y); }
        else rad += sqrt(v.x * v.x + v.y * v.y);
      }
    }
    lo = diag - rad;
    hi = diag + rad;
  }
  smin[tid] = lo; smax[tid] = hi; sbad[tid] = bad;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      smin[tid] = fmin(smin[tid], smin[tid + s]);
      smax[tid] = fmax(smax[tid], smax[tid + s]);
      sbad[tid] |= sbad[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[3 * blockIdx.x] = smin[0];
    out[3 * blockIdx.x + 1] = smax[0];
    out[3 * blockIdx.x + 2] = (double)sbad[0];
  }
}

// Gershgorin discs of a dense row-major term, one wave per row.
__global__ __launch_bounds__(kThreads) void dense_gershgorin_kernel(const double2* H, int dim, long long ld,
                                                                  double* out) {
  __shared__ double smin[kThreads / 64], smax[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = blockIdx.x * (kThreads / 64) + wv;
  double lo = INFINITY, hi = -INFINITY;
  if (r < dim) {
    double rad = 0.0, diag = 0.0;
    for (int j = lane; j < dim; j += 64) {
      const double2 v = H[(long long)r * ld + j];
      if (j == r) { diag += v.x; rad += fabs(v.y); }
      else rad += sqrt(v.x * v.x + v.y * v.y);
    }
    rad = wave_sum(rad);
    diag = wave_sum(diag);
    lo = diag - rad;
    hi = diag + rad;
  }
  if (lane == 0) { smin[wv] = lo; smax[wv] = hi; }
  __syncthreads();
  if (tid == 0) {
    double a = INFINITY, b = -INFINITY;
    for (int w = 0; w < kThreads / 64; ++w) { a = fmin(a, smin[w]); b = fmax(b, smax[w]); }
    out[2 * blockIdx.x] = a;
    out[2 * blockIdx.x + 1] = b;
  }
}

__global__ void copy_kernel(const double2* __restrict__ src, double2* __restrict__ dst, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void step_set_kernel(int* ctr, int value) { *ctr = value; }
__global__ void step_advance_kernel(int* ctr) { *ctr += 1; }

__global__ void slot_reset_kernel(Slot* s, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    s[i].counter = 0u;
    s[i].stopped = 0;
    s[i].iters_sub = 0;
    s[i].status = 0;
    s[i].iters_total = 0;
    s[i].vnorm = 0.0;
    s[i].prev_term = 0.0;
    s[i].last_est = 0.0;
    s[i].term[0] = 0.0;
    s[i].term[1] = 0.0;
  }
}

}  // namespace

int csr_keep_entries(int dim) {
  // the MALL's 256 MiB less a margin and the vectors an iteration touches
  // (about 80 bytes per row), in 20-byte CSR entries
  const long long keep = std::max(0LL, (240LL << 20) - 80LL * dim) / 20;
  return (int)std::min<long long>(keep, 1LL << 30);
}

int csr2_grid(int dim, int rows_per_block) {
  if (rows_per_block == kStreamTile) return csr2_stream_grid(dim);
  int rows = rows_per_block < 0 ? -rows_per_block : rows_per_block;
  if (rows_per_block > kWaveTile) rows = (rows_per_block - kWaveTile) * (kThreads / 64);
  return (dim + rows - 1) / rows;
}

hipError_t launch_csr2_iter(int mode, const CsrDev& t1, const CsrDev& t2, int dim, const IterArgs& a,
                            int rows_per_block, hipStream_t s) {
  if (rows_per_block == kStreamTile) return launch_csr2_stream(mode, t1, t2, dim, a, s);
  if (mode == kSplitComm) return hipErrorInvalidValue;
  const int grid = csr2_grid(dim, rows_per_block);
#define MAGNUS_CSR_CASE(R, M) \
  if (rows_per_block == R && mode == M) { csr2_iter_kernel<R, M><<<grid, kThreads, 0, s>>>(t1, t2, dim, a); return hipGetLastError(); }
  MAGNUS_CSR_CASE(64, kLeja)
  MAGNUS_CSR_CASE(64, kSplit)
  MAGNUS_CSR_CASE(64, kLejaComm)
  MAGNUS_CSR_CASE(16, kLeja)
  MAGNUS_CSR_CASE(16, kSplit)
  MAGNUS_CSR_CASE(16, kLejaComm)
#undef MAGNUS_CSR_CASE
#define MAGNUS_ROWLANE_CASE(R)                                                                     \
  if (rows_per_block == -R) {                                                                      \
    const int g = csr2_grid(dim, -R);                                                              \
    if (mode == kLeja) csr2_rowlane_kernel<R, kLeja><<<g, kThreads, 0, s>>>(t1, t2, dim, a);       \
    else if (mode == kSplit) csr2_rowlane_kernel<R, kSplit><<<g, kThreads, 0, s>>>(t1, t2, dim, a); \
    else csr2_rowlane_kernel<R, kLejaComm><<<g, kThreads, 0, s>>>(t1, t2, dim, a);                 \
    return hipGetLastError();                                                                      \
  }
  MAGNUS_ROWLANE_CASE(32)
  MAGNUS_ROWLANE_CASE(64)
  MAGNUS_ROWLANE_CASE(128)
#undef MAGNUS_ROWLANE_CASE
#define MAGNUS_WAVE_CASE(R)                                                                         \
  if (rows_per_block == kWaveTile + R) {                                                            \
    const int g = csr2_grid(dim, rows_per_block);                                                   \
    const int ke = csr_keep_entries(dim);                                                           \
    if (mode == kLeja) csr2_wave_kernel<R, kLeja><<<g, kThreads, 0, s>>>(t1, t2, dim, a, ke);       \
    else if (mode == kSplit) csr2_wave_kernel<R, kSplit><<<g, kThreads, 0, s>>>(t1, t2, dim, a, ke); \
    else csr2_wave_kernel<R, kLejaComm><<<g, kThreads, 0, s>>>(t1, t2, dim, a, ke);                 \
    return hipGetLastError();                                                                       \
  }
  MAGNUS_WAVE_CASE(8)
  MAGNUS_WAVE_CASE(16)
#undef MAGNUS_WAVE_CASE
  return hipErrorInvalidValue;
}

int csr_gershgorin_grid(int dim) { return (dim + kThreads - 1) / kThreads; }

hipError_t launch_csr_gershgorin(const CsrDev& t, int dim, long long nnz, double* out, int grid, hipStream_t s) {
  csr_gershgorin_kernel<<<grid, kThreads, 0, s>>>(t, dim, nnz, out);
  return hipGetLastError();
}

int dense_gershgorin_grid(int dim) { return (dim + kThreads / 64 - 1) / (kThreads / 64); }

hipError_t launch_dense_gershgorin(const double2* H, int dim, long long ld, double* out, int grid,
                                   hipStream_t s) {
  dense_gershgorin_kernel<<<grid, kThreads, 0, s>>>(H, dim, ld, out);
  return hipGetLastError();
}

// Rows per wave: 1, 2 or 4 (magnus_autotune times them on the caller's
// terms; 2 by default: with 8192 rows that is 16 waves per CU, and more rows
// per wave leave too few waves to cover the memory latency).
int dense2_grid(int dim, int nterms, int rpw) {
  (void)nterms;
  const int rows_per_block = rpw * (kThreads / 64);
  return (dim + rows_per_block - 1) / rows_per_block;
}

// MALL budget kept for matrix rows: its 256 MiB less a margin and the vectors
// an iteration touches (x, w and p read, w and p written).
constexpr long long kDenseMallKeepBytes = 240LL << 20;

hipError_t launch_dense_assemble_iter(const DenseAssembly& D, int dim, const IterArgs& a, hipStream_t s, int rpw) {
  const int g = dense2_grid(dim, 1, rpw);
#define MAGNUS_DENSE_ASM_CASE(R)                                                        \
  case R:                                                                               \
    if (D.K) dense_assemble_iter_kernel<R, true><<<g, kThreads, 0, s>>>(D, dim, a);      \
    else dense_assemble_iter_kernel<R, false><<<g, kThreads, 0, s>>>(D, dim, a);         \
    break;
  switch (rpw) {
    MAGNUS_DENSE_ASM_CASE(1)
    MAGNUS_DENSE_ASM_CASE(2)
    MAGNUS_DENSE_ASM_CASE(4)
    default: return hipErrorInvalidValue;
  }
#undef MAGNUS_DENSE_ASM_CASE
  return hipGetLastError();
}

hipError_t launch_dense2_iter(const double2* H1, const double2* H2, int dim, long long ld,
                              const IterArgs& a, hipStream_t s, int rpw) {
  const long long row_bytes = 16LL * ld * (H2 ? 2 : 1);
  const long long keep = std::max(0LL, kDenseMallKeepBytes - 80LL * dim) / std::max(1LL, row_bytes);
  const int keep_rows = (int)std::min<long long>(keep, dim);
  const int g = dense2_grid(dim, H2 ? 2 : 1, rpw);
#define MAGNUS_DENSE_CASE(R)                                                             \
  case R:                                                                                \
    if (H2) dense2_iter_kernel<R, 2><<<g, kThreads, 0, s>>>(H1, H2, dim, ld, a, keep_rows); \
    else dense2_iter_kernel<R, 1><<<g, kThreads, 0, s>>>(H1, H1, dim, ld, a, keep_rows);    \
    break;
  switch (rpw) {
    MAGNUS_DENSE_CASE(1)
    MAGNUS_DENSE_CASE(2)
    MAGNUS_DENSE_CASE(4)
    default: return hipErrorInvalidValue;
  }
#undef MAGNUS_DENSE_CASE
  return hipGetLastError();
}

int m6_grid(int dim) { return (int)(((long long)dim * kM6Lanes + kThreads - 1) / kThreads); }

hipError_t launch_m6_stage_a(const M6Terms& T, const double2* w, const M6Coef& C, const M6Vecs& V, int dim,
                             const Slot* slot, int check_stop, hipStream_t s) {
  if (dim <= 0) return hipSuccess;
  m6_stage_a_kernel<<<m6_grid(dim), kThreads, 0, s>>>(T, w, C, V, dim, slot, check_stop);
  return hipGetLastError();
}

hipError_t launch_m6_stage_b(const M6Terms& T, const M6Vecs& V, double scale, int dim, const IterArgs& a,
                             hipStream_t s) {
  if (dim <= 0) return hipSuccess;
  m6_stage_b_kernel<<<m6_grid(dim), kThreads, 0, s>>>(T, V, scale, dim, a);
  return hipGetLastError();
}

hipError_t launch_copy(const double2* src, double2* dst, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long grid = (n + kThreads - 1) / kThreads;
  copy_kernel<<<(unsigned)grid, kThreads, 0, s>>>(src, dst, n);
  return hipGetLastError();
}

hipError_t launch_leja_final_check(const IterArgs& a, hipStream_t s) {
  leja_final_check_kernel<<<1, kDecideThreads, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_leja_decide(const IterArgs& a, int grid, hipStream_t s) {
  leja_decide_kernel<<<1, kDecideThreads, 0, s>>>(a, grid);
  return hipGetLastError();
}

hipError_t launch_step_set(int* ctr, int value, hipStream_t s) {
  step_set_kernel<<<1, 1, 0, s>>>(ctr, value);
  return hipGetLastError();
}

hipError_t launch_step_advance(int* ctr, hipStream_t s) {
  step_advance_kernel<<<1, 1, 0, s>>>(ctr);
  return hipGetLastError();
}

hipError_t launch_slot_reset(Slot* slot, int n, hipStream_t s) {
  slot_reset_kernel<<<(n + 63) / 64, 64, 0, s>>>(slot, n);
  return hipGetLastError();
}

}  // namespace magnus
