// Several states per Leja iteration (gfx950, wave64).
//
// B states sharing H1, H2 are stored interleaved (element (row, b) at
// row * B + b), so one pass over the CSR terms serves all B states: each
// matrix entry is streamed once and its B gathers are one contiguous run.
// Each state carries its own coefficients, shift and divided differences (its
// own field value), and its own stop flag.  The same kernel with B = 2 and a
// coupling term runs the Leja recurrence on the block vector of
// [[H, H2], [0, H]], whose exponential carries the Frechet derivative of the
// matrix exponential in its upper-right block.
#include <algorithm>
#include <type_traits>

#include "device_common.h"

namespace magnus {
namespace {

using namespace dev;

// keep_entries: tiles whose entries start within the first keep_entries of the
// two terms are read with normal loads (they stay in the MALL until the next
// iteration), the rest non-temporally.
//
// The body takes the workgroup's block index bid among nb blocks of its
// problem, so that one launch can serve several problems (ragged batches).
template <int B, int MODE>
__device__ __forceinline__ void multi_body(const CsrDev& t1, const CsrDev& t2, int dim, const MultiArgs& a,
                                           int keep_entries, int bid, int nb) {
  constexpr int NWAVE = kThreads / 64;
  constexpr int RP = 64 / B;                // rows per pass: lane = rr * B + b
  constexpr int RPW = RP;                   // rows per wave: one pass (with many states the
                                            // gathers, not the matrix stream, dominate)
  constexpr int NPASS = RPW / RP;
  constexpr int CAPW = 256;                 // entries staged per chunk
  constexpr int U = CAPW / 64;
  static_assert(MODE != kMultiFrechet || B == 2, "the Frechet block vector has two columns");
  __shared__ d2 sval[NWAVE][CAPW];
  __shared__ int scol[NWAVE][CAPW];
  __shared__ int srp[NWAVE][2][RPW + 1];
  __shared__ double wsum[NWAVE][B][2];
  __shared__ int sstop[B];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid < B) sstop[tid] = a.check_stop ? load_stopped(&a.slots[tid]) : 0;
  __syncthreads();
  if (a.check_stop) {
    bool all = true;
    for (int k = 0; k < B; ++k) all = all && sstop[k];
    if (all) return;  // uniform over the workgroup
  }
  const int L = xcd_remap(bid, nb);
  const int row0 = (L * NWAVE + wv) * RPW;
  const int nrows = max(0, min(RPW, dim - row0));
  const int rr = lane / B, b = lane % B;
  const ColParam P = a.prm[b];
  const bool stopped_b = sstop[b] != 0;
  const d2* x = reinterpret_cast<const d2*>(a.x);
  const d2* v1 = reinterpret_cast<const d2*>(t1.val);
  const d2* v2 = reinterpret_cast<const d2*>(t2.val);
  double pw = 0.0, pv = 0.0;

  d2 acc1[NPASS], acc2[NPASS];
#pragma unroll
  for (int q = 0; q < NPASS; ++q) { acc1[q] = d2{0.0, 0.0}; acc2[q] = d2{0.0, 0.0}; }
  if (nrows > 0) {
    for (int i = lane; i <= nrows; i += 64) {
      srp[wv][0][i] = t1.rp[row0 + i];
      srp[wv][1][i] = t2.rp[row0 + i];
    }
    wave_lds_sync();
    const int base1 = srp[wv][0][0], n1 = srp[wv][0][nrows] - base1;
    const int base2 = srp[wv][1][0], n2 = srp[wv][1][nrows] - base2;
    const int total = n1 + n2;
    const bool keep = (long long)base1 + base2 < keep_entries;  // uniform over the wave (no int overflow)
    for (int c0 = 0; c0 < total; c0 += CAPW) {
      const int cn = min(CAPW, total - c0);
      int col[U];
      d2 val[U];
      auto load_chunk = [&](auto streaming) {
        auto ld = [&](const auto* p) {
          if constexpr (decltype(streaming)::value) return __builtin_nontemporal_load(p);
          else return *p;
        };
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = u * 64 + lane;
          const int gk = c0 + k;
          col[u] = 0;
          val[u] = d2{0.0, 0.0};
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
#pragma unroll
      for (int q = 0; q < NPASS; ++q) {
        const int r = q * RP + rr;
        if (r < nrows) {
          const int s1 = srp[wv][0][r] - base1, e1 = srp[wv][0][r + 1] - base1;
          const int s2 = n1 + srp[wv][1][r] - base2, e2 = n1 + srp[wv][1][r + 1] - base2;
          // unrolled so several gathers are in flight per lane
#pragma unroll 8
          for (int k = max(s1, c0); k < min(e1, hi); ++k)
            acc1[q] += cmul(sval[wv][k - c0], x[(long long)scol[wv][k - c0] * B + b]);
#pragma unroll 8
          for (int k = max(s2, c0); k < min(e2, hi); ++k)
            acc2[q] += cmul(sval[wv][k - c0], x[(long long)scol[wv][k - c0] * B + b]);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NPASS; ++q) {
    const int r = q * RP + rr;
    d2 h2y = {0.0, 0.0};
    if constexpr (MODE == kMultiFrechet) {
      // lane rr*2 + 1 holds H2 y of the same row; the top lane (b = 0) couples it in
      h2y.x = __shfl_down(acc2[q].x, 1, 64);
      h2y.y = __shfl_down(acc2[q].y, 1, 64);
    }
    if (r < nrows) {
      const long long idx = (long long)(row0 + r) * B + b;
      d2 y = rmul(P.a1, acc1[q]) + rmul(P.a2, acc2[q]);
      if constexpr (MODE == kMultiFrechet) {
        if (b == 0) y += rmul(P.coup, h2y);
      }
      const d2 w_old = x[idx];
      const d2 wn = y - rmul(P.sigma, w_old);
      const d2 dd = {P.dre, P.dim};
      d2 p;
      if (a.first) {
        p = cmul(d2{P.d0re, P.d0im}, w_old) + cmul(dd, wn);
        pv += nrm2(w_old);
      } else {
        p = tod2(a.pacc[idx]);
        if (!stopped_b) p += cmul(dd, wn);
      }
      a.wout[idx] = fromd2(wn);
      a.pacc[idx] = fromd2(p);
      pw += nrm2(wn);
    }
  }
  // per-column sums: lanes b, b + B, b + 2B, ... share a column
#pragma unroll
  for (int off = 32; off >= B; off >>= 1) {
    pw += __shfl_xor(pw, off, 64);
    pv += __shfl_xor(pv, off, 64);
  }
  if (lane < B) {
    wsum[wv][lane][0] = pw;
    wsum[wv][lane][1] = pv;
  }
  __syncthreads();
  if (tid < B) {
    double bw = 0.0, bv = 0.0;
    for (int w = 0; w < NWAVE; ++w) { bw += wsum[w][tid][0]; bv += wsum[w][tid][1]; }
    // column-major (column tid, workgroup bid), so each column's decide reads contiguously
    a.partials[((long long)tid * nb + bid) * 2] = bw;
    a.partials[((long long)tid * nb + bid) * 2 + 1] = bv;
  }
}

template <int B, int MODE>
__global__ __launch_bounds__(kThreads) void csr2_multi_kernel(CsrDev t1, CsrDev t2, int dim, MultiArgs a,
                                                             int keep_entries) {
  multi_body<B, MODE>(t1, t2, dim, a, keep_entries, blockIdx.x, gridDim.x);
}

// Several problems (own terms, states, coefficients, slots and partials) in
// one launch: problem q owns blocks [block0[q], block0[q + 1]).
template <int B>
__global__ __launch_bounds__(kThreads) void csr2_ragged_kernel(RaggedArgs r) {
  int q = 0;
  while (q + 1 < r.np && (int)blockIdx.x >= r.p[q + 1].block0) ++q;  // uniform
  const int nb = (q + 1 < r.np ? r.p[q + 1].block0 : (int)gridDim.x) - r.p[q].block0;
  multi_body<B, kMultiLeja>(r.p[q].t1, r.p[q].t2, r.p[q].dim, r.p[q].a, r.p[q].keep_entries,
                            (int)blockIdx.x - r.p[q].block0, nb);
}

// One workgroup per column (or one for the joint block vector): fixed-order
// reduction over workgroups, then the stop verdict.
constexpr int kDecideThreads = 1024;
__device__ __forceinline__ void multi_decide_body(const MultiArgs& a, int grid, int col) {
  __shared__ double red[2][kDecideThreads / 64];
  Slot* S = &a.slots[col];
  if (a.check_stop && load_stopped(S)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int c_lo = a.joint ? 0 : col, c_hi = a.joint ? a.B : col + 1;
  // partials are column-major: column c's per-workgroup pairs are contiguous
  constexpr int kPer = 8;
  double sw = 0.0, sv = 0.0;
  for (int c = c_lo; c < c_hi; ++c) {
    const d2* P = reinterpret_cast<const d2*>(a.partials) + (long long)c * grid;
    for (int k0 = 0; k0 < grid; k0 += kDecideThreads * kPer) {
      d2 v[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int k = k0 + u * kDecideThreads + tid;
        v[u] = k < grid ? P[k] : d2{0.0, 0.0};
      }
#pragma unroll
      for (int u = 0; u < kPer; ++u) { sw += v[u].x; sv += v[u].y; }
    }
  }
  sw = wave_sum(sw);
  sv = wave_sum(sv);
  if (lane == 0) { red[0][wv] = sw; red[1][wv] = sv; }
  __syncthreads();
  if (tid == 0) {
    double tw = 0.0, tv = 0.0;
    for (int w = 0; w < kDecideThreads / 64; ++w) { tw += red[0][w]; tv += red[1][w]; }
    const ColParam P = a.prm[col];
    leja_verdict(S, a.first != 0, a.early != 0, a.tol, P.dabs, P.d0abs, tw, tv);
    if (a.joint)
      for (int c = 1; c < a.B; ++c) a.slots[c] = *S;
  }
}

__global__ __launch_bounds__(kDecideThreads) void multi_decide_kernel(MultiArgs a, int grid) {
  multi_decide_body(a, grid, blockIdx.x);
}

// Column decisions of a ragged launch: workgroup col0[q] + c decides column c
// of problem q over that problem's grid.
__global__ __launch_bounds__(kDecideThreads) void ragged_decide_kernel(RaggedArgs r) {
  int q = 0;
  while (q + 1 < r.np && (int)blockIdx.x >= r.p[q + 1].col0) ++q;  // uniform
  const int nb = (q + 1 < r.np ? r.p[q + 1].block0 : r.nblocks) - r.p[q].block0;
  multi_decide_body(r.p[q].a, nb, (int)blockIdx.x - r.p[q].col0);
}

__global__ void pack_kernel(const double2* __restrict__ src, double2* __restrict__ dst, int dim, int B) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // destination index
  if (i < (long long)dim * B) {
    const long long row = i / B, b = i % B;
    dst[i] = src[b * dim + row];
  }
}

__global__ void unpack_kernel(const double2* __restrict__ src, double2* __restrict__ dst, int dim, int B) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // destination index
  if (i < (long long)dim * B) {
    const long long b = i / dim, row = i % dim;
    dst[i] = src[row * B + b];
  }
}

// Dense block (Frechet) iteration on the interleaved pair (x, y) of the
// block vector of [[H, H2], [0, H]], H = a1 H1 + a2 H2 (scaled): a wave owns
// RPW rows, its lanes stride over the columns, so each matrix element is
// loaded once (coalesced, non-temporal) for both x and y.
template <int RPW>
__global__ __launch_bounds__(kThreads) void dense_frechet_kernel(const double2* H1, const double2* H2, int dim,
                                                                long long ld, MultiArgs a) {
  __shared__ double wsum[kThreads / 64][2][2];
  if (a.check_stop && load_stopped(&a.slots[0])) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int rbase = (L * (kThreads / 64) + wv) * RPW;
  const int nr = max(0, min(RPW, dim - rbase));
  const d2* X = reinterpret_cast<const d2*>(a.x);
  const d2* A1 = reinterpret_cast<const d2*>(H1);
  const d2* A2 = reinterpret_cast<const d2*>(H2);
  d2 acc[RPW][4];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[r][q] = d2{0.0, 0.0};
  for (int j = lane; j < dim; j += 64) {
    const d2 xj = X[2 * (long long)j], yj = X[2 * (long long)j + 1];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      if (r < nr) {
        const long long off = (long long)(rbase + r) * ld + j;
        const d2 h1 = __builtin_nontemporal_load(A1 + off), h2 = __builtin_nontemporal_load(A2 + off);
        acc[r][0] += cmul(h1, xj);
        acc[r][1] += cmul(h2, xj);
        acc[r][2] += cmul(h1, yj);
        acc[r][3] += cmul(h2, yj);
      }
    }
  }
  const ColParam P0 = a.prm[0], P1 = a.prm[1];
  double pw[2] = {0.0, 0.0}, pv[2] = {0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        acc[r][q].x += __shfl_xor(acc[r][q].x, off, 64);
        acc[r][q].y += __shfl_xor(acc[r][q].y, off, 64);
      }
    if (lane == r && r < nr) {
      const long long row = rbase + r;
      const d2 ys[2] = {rmul(P0.a1, acc[r][0]) + rmul(P0.a2, acc[r][1]) + rmul(P0.coup, acc[r][3]),
                        rmul(P1.a1, acc[r][2]) + rmul(P1.a2, acc[r][3])};
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const ColParam& P = c == 0 ? P0 : P1;
        const long long idx = 2 * row + c;
        const d2 w_old = X[idx];
        const d2 wn = ys[c] - rmul(P.sigma, w_old);
        const d2 dd = {P.dre, P.dim};
        d2 p;
        if (a.first) {
          p = cmul(d2{P.d0re, P.d0im}, w_old) + cmul(dd, wn);
          pv[c] += nrm2(w_old);
        } else {
          p = tod2(a.pacc[idx]) + cmul(dd, wn);
        }
        a.wout[idx] = fromd2(wn);
        a.pacc[idx] = fromd2(p);
        pw[c] += nrm2(wn);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    pw[c] = wave_sum(pw[c]);
    pv[c] = wave_sum(pv[c]);
  }
  if (lane == 0)
    for (int c = 0; c < 2; ++c) { wsum[wv][c][0] = pw[c]; wsum[wv][c][1] = pv[c]; }
  __syncthreads();
  if (tid < 2) {
    double bw = 0.0, bv = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) { bw += wsum[w][tid][0]; bv += wsum[w][tid][1]; }
    a.partials[((long long)tid * gridDim.x + blockIdx.x) * 2] = bw;
    a.partials[((long long)tid * gridDim.x + blockIdx.x) * 2 + 1] = bv;
  }
}

// Fixed-order complex dot product sum_i conj(x_i) y_i (strided operands).
constexpr int kDotBlocks = kDotPartials / 2;
__global__ __launch_bounds__(kThreads) void cdot_partial_kernel(const double2* x, long long sx, const double2* y,
                                                               long long sy, long long n, double* partials) {
  __shared__ double red[2][kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double re = 0.0, im = 0.0;
  for (long long i = (long long)blockIdx.x * kThreads + tid; i < n; i += (long long)gridDim.x * kThreads) {
    const d2 a = tod2(x[i * sx]), b = tod2(y[i * sy]);
    re += a.x * b.x + a.y * b.y;
    im += a.x * b.y - a.y * b.x;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) { red[0][wv] = re; red[1][wv] = im; }
  __syncthreads();
  if (tid == 0) {
    double r = 0.0, q = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) { r += red[0][w]; q += red[1][w]; }
    partials[2 * blockIdx.x] = r;
    partials[2 * blockIdx.x + 1] = q;
  }
}

__global__ __launch_bounds__(kThreads) void cdot_final_kernel(const double* partials, int grid, double2* out) {
  __shared__ double red[2][kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double re = 0.0, im = 0.0;
  for (int k = tid; k < grid; k += kThreads) {
    re += partials[2 * k];
    im += partials[2 * k + 1];
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) { red[0][wv] = re; red[1][wv] = im; }
  __syncthreads();
  if (tid == 0) {
    double r = 0.0, q = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) { r += red[0][w]; q += red[1][w]; }
    *out = make_double2(r, q);
  }
}

// One Lanczos orthogonalisation: w <- w - alpha v - beta u (w holds H v on entry).
__global__ void lanczos_orth_kernel(double2* __restrict__ w, const double2* __restrict__ v,
                                    const double2* __restrict__ u, double alpha, double beta, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    w[i] = fromd2(tod2(w[i]) - rmul(alpha, tod2(v[i])) - rmul(beta, tod2(u[i])));
}

__global__ void scale_kernel(const double2* __restrict__ x, double sc, double2* __restrict__ y, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = fromd2(rmul(sc, tod2(x[i])));
}

// Block vector [0; v] of the Frechet exponential, interleaved (element (row, b) at 2 row + b).
__global__ void frechet_init_kernel(const double2* __restrict__ v, double2* __restrict__ dst, int dim) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < dim) {
    dst[2 * i] = make_double2(0.0, 0.0);
    dst[2 * i + 1] = v[i];
  }
}

// Must match csr2_multi_kernel's rows per wave (64 / B) times its waves.
template <int B>
int multi_rows_per_block() {
  return (64 / B) * (kThreads / 64);
}

}  // namespace

int csr2_multi_grid(int dim, int B) {
  int rpb = 0;
  switch (B) {
    case 2: rpb = multi_rows_per_block<2>(); break;
    case 4: rpb = multi_rows_per_block<4>(); break;
    case 8: rpb = multi_rows_per_block<8>(); break;
    case 16: rpb = multi_rows_per_block<16>(); break;
    case 32: rpb = multi_rows_per_block<32>(); break;
    default: return 0;
  }
  return (dim + rpb - 1) / rpb;
}

hipError_t launch_csr2_multi(int mode, const CsrDev& t1, const CsrDev& t2, int dim, const MultiArgs& a,
                             hipStream_t s) {
  const int grid = csr2_multi_grid(dim, a.B);
  if (grid <= 0) return hipErrorInvalidValue;
  // the MALL's 256 MiB less a margin and the vectors of all B states
  const long long keep = std::max(0LL, (240LL << 20) - 80LL * dim * a.B) / 20;
  const int ke = (int)std::min<long long>(keep, 1LL << 30);
  if (mode == kMultiFrechet) {
    if (a.B != 2) return hipErrorInvalidValue;
    csr2_multi_kernel<2, kMultiFrechet><<<grid, kThreads, 0, s>>>(t1, t2, dim, a, ke);
    return hipGetLastError();
  }
  switch (a.B) {
    case 2: csr2_multi_kernel<2, kMultiLeja><<<grid, kThreads, 0, s>>>(t1, t2, dim, a, ke); break;
    case 4: csr2_multi_kernel<4, kMultiLeja><<<grid, kThreads, 0, s>>>(t1, t2, dim, a, ke); break;
    case 8: csr2_multi_kernel<8, kMultiLeja><<<grid, kThreads, 0, s>>>(t1, t2, dim, a, ke); break;
    case 16: csr2_multi_kernel<16, kMultiLeja><<<grid, kThreads, 0, s>>>(t1, t2, dim, a, ke); break;
    case 32: csr2_multi_kernel<32, kMultiLeja><<<grid, kThreads, 0, s>>>(t1, t2, dim, a, ke); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_multi_decide(const MultiArgs& a, int grid, hipStream_t s) {
  multi_decide_kernel<<<a.joint ? 1 : a.B, kDecideThreads, 0, s>>>(a, grid);
  return hipGetLastError();
}

int ragged_grid(int dim, int B) {
  const int g = csr2_multi_grid(dim, B);
  return (g + 7) / 8 * 8;  // whole rounds of the 8 XCDs, so the XCD-aware row order holds per problem
}

hipError_t launch_csr2_ragged(RaggedArgs r, int B, hipStream_t s) {
  if (r.np < 1 || r.np > kMaxRagged) return hipErrorInvalidValue;
  int blocks = 0, cols = 0;
  for (int q = 0; q < r.np; ++q) {
    if (r.p[q].a.B != B || r.p[q].a.joint) return hipErrorInvalidValue;
    r.p[q].block0 = blocks;
    r.p[q].col0 = cols;
    // the MALL's 256 MiB less a margin and the vectors of all B states (per problem)
    const long long keep = std::max(0LL, (240LL << 20) - 80LL * r.p[q].dim * B) / 20;
    r.p[q].keep_entries = (int)std::min<long long>(keep, 1LL << 30);
    blocks += ragged_grid(r.p[q].dim, B);
    cols += B;
  }
  r.nblocks = blocks;
  switch (B) {
    case 2: csr2_ragged_kernel<2><<<blocks, kThreads, 0, s>>>(r); break;
    case 4: csr2_ragged_kernel<4><<<blocks, kThreads, 0, s>>>(r); break;
    case 8: csr2_ragged_kernel<8><<<blocks, kThreads, 0, s>>>(r); break;
    case 16: csr2_ragged_kernel<16><<<blocks, kThreads, 0, s>>>(r); break;
    case 32: csr2_ragged_kernel<32><<<blocks, kThreads, 0, s>>>(r); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  ragged_decide_kernel<<<cols, kDecideThreads, 0, s>>>(r);
  return hipGetLastError();
}

constexpr int kFrechetRPW = 2;
int dense_frechet_grid(int dim) {
  const int rows = kFrechetRPW * (kThreads / 64);
  return (dim + rows - 1) / rows;
}

hipError_t launch_dense_frechet(const double2* H1, const double2* H2, int dim, long long ld, const MultiArgs& a,
                                hipStream_t s) {
  if (a.B != 2) return hipErrorInvalidValue;
  dense_frechet_kernel<kFrechetRPW><<<dense_frechet_grid(dim), kThreads, 0, s>>>(H1, H2, dim, ld, a);
  return hipGetLastError();
}

hipError_t launch_lanczos_orth(double2* w, const double2* v, const double2* u, double alpha, double beta, long long n,
                               hipStream_t s) {
  const long long g = std::min<long long>((n + kThreads - 1) / kThreads, 4096);
  lanczos_orth_kernel<<<(unsigned)std::max<long long>(g, 1), kThreads, 0, s>>>(w, v, u, alpha, beta, n);
  return hipGetLastError();
}

hipError_t launch_scale(const double2* x, double sc, double2* y, long long n, hipStream_t s) {
  const long long g = std::min<long long>((n + kThreads - 1) / kThreads, 4096);
  scale_kernel<<<(unsigned)std::max<long long>(g, 1), kThreads, 0, s>>>(x, sc, y, n);
  return hipGetLastError();
}

hipError_t launch_cdot(const double2* x, long long sx, const double2* y, long long sy, long long n, double* partials,
                       double2* out, hipStream_t s) {
  cdot_partial_kernel<<<kDotBlocks, kThreads, 0, s>>>(x, sx, y, sy, n, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  cdot_final_kernel<<<1, kThreads, 0, s>>>(partials, kDotBlocks, out);
  return hipGetLastError();
}

hipError_t launch_frechet_init(const double2* v, double2* dst, int dim, hipStream_t s) {
  frechet_init_kernel<<<(dim + 255) / 256, 256, 0, s>>>(v, dst, dim);
  return hipGetLastError();
}

hipError_t launch_pack(const double2* src, double2* dst, int dim, int B, hipStream_t s) {
  const long long n = (long long)dim * B;
  pack_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, dst, dim, B);
  return hipGetLastError();
}

hipError_t launch_unpack(const double2* src, double2* dst, int dim, int B, hipStream_t s) {
  const long long n = (long long)dim * B;
  unpack_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, dst, dim, B);
  return hipGetLastError();
}

}  // namespace magnus
