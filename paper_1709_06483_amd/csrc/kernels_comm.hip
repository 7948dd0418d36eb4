// The commutator K = i [H1, H2] of two CSR terms, assembled once for Method
// M4 (Section 2; Section 4 forms the M4 commutator explicitly), and the Leja
// iteration on the three-term exponent a1 H1 + a2 H2 + a3 K.
//
// Assembly: one wave per row r.  The wave lists every product of row r of
// H1 H2 (H1[r,k] H2[k,c]) and of -H2 H1 (-H2[r,k] H1[k,c]) in LDS, sorts them
// by (column, position in the list) with a bitonic network, and lane 0 sums
// equal columns in that order (deterministic), drops exact zeros and scales
// by i.  A count pass sizes the rows; a fill pass writes them.
//
// Iteration: the wave-tile mapping of the two-term kernel (8 rows per wave,
// 8 lanes per row, each tile's entries of the three terms staged in LDS
// with coalesced non-temporal loads, fixed-order shuffle sums).  Large
// matrices take the streamed three-term kernel instead (LDS-DMA copies one
// chunk ahead), which sums in the same order.
#include <climits>
#include <type_traits>

#include "device_common.h"

namespace magnus {
namespace {

using namespace dev;

constexpr int kCommWaves = 4;

__device__ __forceinline__ void comm_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

template <bool FILL>
__global__ __launch_bounds__(kCommWaves * 64) void csr_commutator_kernel(CsrDev A, CsrDev Bm, int dim, int* counts,
                                                                          const int* rp_out, int* ci_out,
                                                                          double2* val_out, int* overflow) {
  __shared__ long long skey[kCommWaves][kCommCap];
  __shared__ d2 sval[kCommWaves][kCommCap];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = blockIdx.x * kCommWaves + wv;
  if (r >= dim) return;  // whole wave; no workgroup barrier below
  const d2* av = reinterpret_cast<const d2*>(A.val);
  const d2* bv = reinterpret_cast<const d2*>(Bm.val);

  // list the products of row r: first A B, then -(B A)
  int n = 0;
  for (int side = 0; side < 2; ++side) {
    const CsrDev& L = side == 0 ? A : Bm;
    const CsrDev& R = side == 0 ? Bm : A;
    const d2* lv = side == 0 ? av : bv;
    const d2* rv = side == 0 ? bv : av;
    const double sg = side == 0 ? 1.0 : -1.0;
    for (int e = L.rp[r]; e < L.rp[r + 1]; ++e) {
      const int k = L.ci[e];
      const d2 lval = lv[e];
      const int b0 = R.rp[k], b1 = R.rp[k + 1];
      for (int j = b0 + lane; j < b1; j += 64) {
        const int idx = n + (j - b0);
        if (idx < kCommCap) {
          skey[wv][idx] = ((long long)R.ci[j] << 32) | (long long)idx;
          sval[wv][idx] = rmul(sg, cmul(lval, rv[j]));
        }
      }
      n += b1 - b0;
    }
  }
  if (n > kCommCap) {
    if (lane == 0) *overflow = 1;  // plain vector store; any writer sets the same value
    return;
  }
  int np2 = 1;
  while (np2 < n) np2 <<= 1;
  for (int i = n + lane; i < np2; i += 64) skey[wv][i] = LLONG_MAX;
  comm_lds_sync();
  // bitonic sort of skey (with sval) ascending
  for (int k = 2; k <= np2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < np2; i += 64) {
        const int p = i ^ j;
        if (p > i) {
          const bool up = (i & k) == 0;
          const long long ki = skey[wv][i], kp = skey[wv][p];
          if ((ki > kp) == up) {
            skey[wv][i] = kp;
            skey[wv][p] = ki;
            const d2 t = sval[wv][i];
            sval[wv][i] = sval[wv][p];
            sval[wv][p] = t;
          }
        }
      }
      comm_lds_sync();
    }
  if (lane != 0) return;
  int out = 0;
  const int base = FILL ? rp_out[r] : 0;
  for (int i = 0; i < n;) {
    const int c = (int)(skey[wv][i] >> 32);
    d2 s = {0.0, 0.0};
    for (; i < n && (int)(skey[wv][i] >> 32) == c; ++i) s += sval[wv][i];
    if (s.x != 0.0 || s.y != 0.0) {
      if (FILL) {
        ci_out[base + out] = c;
        val_out[base + out] = make_double2(-s.y, s.x);  // i s
      }
      ++out;
    }
  }
  if (!FILL) counts[r] = out;
}

// ---------------------------------------------------------------------------
// Three-term Leja iteration: y = a1 H1 x + a2 H2 x + a3 K x, then the update.
// ---------------------------------------------------------------------------
constexpr int kRPW3 = 8;

__global__ __launch_bounds__(kThreads, 5) void csr3_wave_kernel(CsrDev t1, CsrDev t2, CsrDev t3, int dim, IterArgs a_in,
                                                               double a3_arg, int keep_entries) {
  const IterArgs a = resolve_args(a_in);
  const double a3 = a_in.coef ? a.kap : a3_arg;  // replayed: scale * kappa from the table
  constexpr int NWAVE = kThreads / 64;
  constexpr int RPW = kRPW3;
  constexpr int G = 64 / RPW;
  constexpr int CAPW = RPW * 32;
  constexpr int U = CAPW / 64;
  __shared__ d2 sval[NWAVE][CAPW];
  __shared__ int scol[NWAVE][CAPW];
  __shared__ int srp[NWAVE][3][RPW + 1];
  __shared__ double wred[2][NWAVE];
  const bool stopped = iteration_stopped(a, reinterpret_cast<double*>(&sval[0][0]));
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int row0 = (L * NWAVE + wv) * RPW;
  const int nrows = max(0, min(RPW, dim - row0));
  const int r = lane % RPW, g = lane / RPW;
  const bool owner = (lane < RPW) && (r < nrows);
  const int row = row0 + r;
  double pw = 0.0, pv = 0.0;
  // lanes 0..8, 16..24, 32..40 fetch the row pointers of the three terms
  const int tsel = lane >> 4, tl = lane & 15;
  int rpv = 0;
  d2 w_old = {0.0, 0.0}, p_old = {0.0, 0.0};
  if (nrows > 0) {
    if (tsel < 3 && tl <= nrows) rpv = (tsel == 0 ? t1 : tsel == 1 ? t2 : t3).rp[row0 + tl];
    if (owner) {
      w_old = tod2(a.wcur[row]);
      if (!a.first) p_old = tod2(a.pacc[row]);
    }
  }
  if (stopped) return;  // uniform over the workgroup

  if (nrows > 0) {
    if (tsel < 3 && tl <= nrows) srp[wv][tsel][tl] = rpv;
    comm_lds_sync();
    int base[3], len[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      base[t] = srp[wv][t][0];
      len[t] = srp[wv][t][nrows] - base[t];
    }
    const int off2 = len[0], off3 = len[0] + len[1];
    const int total = off3 + len[2];
    int s[3] = {0, 0, 0}, e[3] = {0, 0, 0};
    if (r < nrows) {
      const int offs[3] = {0, off2, off3};
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        s[t] = offs[t] + srp[wv][t][r] - base[t];
        e[t] = offs[t] + srp[wv][t][r + 1] - base[t];
      }
    }
    const d2* x = reinterpret_cast<const d2*>(a.x1);
    const d2* v1 = reinterpret_cast<const d2*>(t1.val);
    const d2* v2 = reinterpret_cast<const d2*>(t2.val);
    const d2* v3 = reinterpret_cast<const d2*>(t3.val);
    d2 acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    // the front of the matrix is read with normal loads and stays in the MALL
    // until the next iteration; the rest streams through (uniform per wave)
    const bool keep = (long long)base[0] + base[1] + base[2] < keep_entries;  // no int overflow
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
            if (gk < off2) {
              col[u] = ld(t1.ci + base[0] + gk);
              val[u] = ld(v1 + base[0] + gk);
            } else if (gk < off3) {
              col[u] = ld(t2.ci + base[1] + (gk - off2));
              val[u] = ld(v2 + base[1] + (gk - off2));
            } else {
              col[u] = ld(t3.ci + base[2] + (gk - off3));
              val[u] = ld(v3 + base[2] + (gk - off3));
            }
          }
        }
      };
      if (keep) load_chunk(std::false_type{});
      else load_chunk(std::true_type{});
      comm_lds_sync();  // the previous chunk's LDS reads are done
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = u * 64 + lane;
        if (k < cn) {
          scol[wv][k] = col[u];
          sval[wv][k] = val[u];
        }
      }
      comm_lds_sync();
      const int hi = c0 + cn;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int lo = max(s[t], c0) + g, end = min(e[t], hi);
#pragma unroll 4
        for (int k = lo; k < end; k += G) acc[t] += cmul(sval[wv][k - c0], x[scol[wv][k - c0]]);
      }
    }
#pragma unroll
    for (int off = 32; off >= RPW; off >>= 1)
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        acc[t].x += __shfl_xor(acc[t].x, off, 64);
        acc[t].y += __shfl_xor(acc[t].y, off, 64);
      }
    if (owner) {
      const d2 y = rmul(a.a1, acc[0]) + rmul(a.a2, acc[1]) + rmul(a3, acc[2]);
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
  pw = wave_sum(pw);
  pv = wave_sum(pv);
  if (lane == 0) { wred[0][wv] = pw; wred[1][wv] = pv; }
  __syncthreads();
  if (tid == 0) {
    double bw = 0.0, bv = 0.0;
    for (int k = 0; k < NWAVE; ++k) { bw += wred[0][k]; bv += wred[1][k]; }
    a.partials[blockIdx.x] = bw;
    if (a.first) a.partials[gridDim.x + blockIdx.x] = bv;
  }
}

}  // namespace

hipError_t launch_csr_commutator(bool fill, const CsrDev& A, const CsrDev& Bm, int dim, int* counts,
                                 const int* rp_out, int* ci_out, double2* val_out, int* overflow, hipStream_t s) {
  const int grid = (dim + kCommWaves - 1) / kCommWaves;
  if (fill) csr_commutator_kernel<true><<<grid, kCommWaves * 64, 0, s>>>(A, Bm, dim, counts, rp_out, ci_out, val_out, overflow);
  else csr_commutator_kernel<false><<<grid, kCommWaves * 64, 0, s>>>(A, Bm, dim, counts, rp_out, ci_out, val_out, overflow);
  return hipGetLastError();
}

int csr3_grid(int dim, bool streamed) {
  if (streamed) return csr2_stream_grid(dim);
  const int rows = kRPW3 * (kThreads / 64);
  return (dim + rows - 1) / rows;
}

hipError_t launch_csr3_iter(const CsrDev& t1, const CsrDev& t2, const CsrDev& t3, int dim, const IterArgs& a,
                            double a3, bool streamed, hipStream_t s) {
  if (streamed) return launch_csr3_stream(t1, t2, t3, dim, a, a3, s);
  csr3_wave_kernel<<<csr3_grid(dim, false), kThreads, 0, s>>>(t1, t2, t3, dim, a, a3, csr_keep_entries(dim));
  return hipGetLastError();
}

}  // namespace magnus
