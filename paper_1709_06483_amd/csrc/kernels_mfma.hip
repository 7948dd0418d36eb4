// Dense Leja iteration for a group of states: Y = H W as an FP64 MFMA GEMM
// (gfx950 v_mfma_f64_16x16x4f64), fused with the Leja update.
//
// W holds B states interleaved (element (k, b) at k * B + b); H is row-major.
// The complex product uses four real MFMAs per 16x16x4 step:
//   Yre += Hre Wre - Him Wim,   Yim += Hre Wim + Him Wre.
// NT = 1: one (assembled) matrix, y_b = a1_b (H w_b).
// NT = 2: two terms with per-state coefficients folded into the W operand,
//         y_b = H1 (a1_b w_b) + H2 (a2_b w_b).
// Several tile shapes (kMfmaTiles, chosen per problem by magnus_autotune;
// the LDS-DMA variants further down are the sixth and seventh):
// a wave computes TI x TJ MFMA tiles, four waves per K group a 32 TI x 32 TJ
// block of rows x states; K is staged through LDS 16 at a time with the next
// chunk prefetched into registers while the MFMAs run.
#include <type_traits>

#include "device_common.h"
#include "mfma_dma.h"

namespace magnus {
namespace {

using namespace dev;
using dma_gemm::v4d;

constexpr int TK = 16;

// Tile shape of one instantiation: a wave computes TI x TJ MFMA tiles of
// 16 x 16 (16 TI rows, 16 TJ states), four waves per K group in a 2 x 2
// arrangement make the workgroup tile TM x TN = 32 TI x 32 TJ, and K is
// split between KS groups of four waves: group g accumulates the K chunks
// g, g + KS, ... of the workgroup's tile in its own LDS slice, and the
// groups' accumulators are added in a fixed order at the end.  Larger wave
// tiles read fewer LDS operands per MFMA; the split gives each SIMD more
// waves to overlap the MFMA chains with the staging of the next chunk.
template <int TI_, int TJ_, int KS_>
struct MfmaTile {
  static constexpr int TI = TI_, TJ = TJ_, KS = KS_;
  static constexpr int WM = 16 * TI, WN = 16 * TJ;
  static constexpr int TM = 2 * WM, TN = 2 * WN;
  static constexpr int THREADS = KS * kThreads;
  static constexpr int HU = TM * TK / kThreads;  // H elements per thread and term (consecutive along K)
  static constexpr int WU = TK * TN / kThreads;  // W elements per thread (consecutive states)
};

// Epilogue of a group iteration, called by every thread: the Leja update of
// the workgroup's TM x TN block from the accumulators (element j of a lane's
// v4d is row lane/16 + 4 j of its 16-row tile, state lane % 16, the
// v_mfma_f64_16x16x4f64 output layout), and the per-state norm partials of
// the block, stored column-major (state, 32-row block) as the decide kernel
// reads them (a tile of TM rows writes its sums at its first 32-row block,
// zeros at the others).  epi: this thread's accumulators hold the sums.
template <int NT, int TI, int TJ, int WM, int WN, int TM, int TN>
__device__ __forceinline__ void group_epilogue(const MultiArgs& a, int dim, int row0, int col0, int wr, int wc,
                                               bool epi, const v4d (&are)[TI][TJ], const v4d (&aim)[TI][TJ],
                                               double (&csum)[TM / WM][2][TN]) {
  const int B = a.B;
  const int tid = threadIdx.x, lane = tid & 63;
  const d2* W = reinterpret_cast<const d2*>(a.x);
  double pw[TJ], pv[TJ];
#pragma unroll
  for (int tj = 0; tj < TJ; ++tj) {
    pw[tj] = 0.0;
    pv[tj] = 0.0;
    const int c = col0 + wc * WN + tj * 16 + (lane & 15);
    if (!epi || c >= B) continue;
    const ColParam P = a.prm[c];
    const bool stopped_c = a.check_stop ? load_stopped(&a.slots[c]) != 0 : false;
    const double ys = NT == 2 ? 1.0 : P.a1;
#pragma unroll
    for (int ti = 0; ti < TI; ++ti)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = row0 + wr * WM + ti * 16 + (lane >> 4) + 4 * j;
        if (r >= dim) continue;
        const long long idx = (long long)r * B + c;
        const d2 y = d2{ys * are[ti][tj][j], ys * aim[ti][tj][j]};
        const d2 w_old = W[idx];
        const d2 wn = y - rmul(P.sigma, w_old);
        const d2 dd = {P.dre, P.dim};
        d2 p;
        if (a.first) {
          p = cmul(d2{P.d0re, P.d0im}, w_old) + cmul(dd, wn);
          pv[tj] += nrm2(w_old);
        } else {
          p = tod2(a.pacc[idx]);
          if (!stopped_c) p += cmul(dd, wn);
        }
        a.wout[idx] = fromd2(wn);
        a.pacc[idx] = fromd2(p);
        pw[tj] += nrm2(wn);
      }
  }
  // per-state sums: lanes l, l + 16, l + 32, l + 48 share a state
#pragma unroll
  for (int tj = 0; tj < TJ; ++tj) {
    pw[tj] += __shfl_xor(pw[tj], 16, 64);
    pw[tj] += __shfl_xor(pw[tj], 32, 64);
    pv[tj] += __shfl_xor(pv[tj], 16, 64);
    pv[tj] += __shfl_xor(pv[tj], 32, 64);
    if (epi && lane < 16) {
      csum[wr][0][wc * WN + tj * 16 + lane] = pw[tj];
      csum[wr][1][wc * WN + tj * 16 + lane] = pv[tj];
    }
  }
  __syncthreads();
  if (tid < TN && col0 + tid < B) {
    const int rb32 = row0 / 32, nrb32 = (dim + 31) / 32;
    const long long o = ((long long)(col0 + tid) * nrb32 + rb32) * 2;
    if constexpr (TM / WM == 2) {  // two rows of waves: the tile's sums in its first 32-row block
      a.partials[o] = csum[0][0][tid] + csum[1][0][tid];
      a.partials[o + 1] = csum[0][1][tid] + csum[1][1][tid];
      for (int q = 1; q < TM / 32 && rb32 + q < nrb32; ++q) {
        a.partials[o + 2 * q] = 0.0;
        a.partials[o + 2 * q + 1] = 0.0;
      }
    } else {  // rows of 16-row waves: two of them per 32-row block
      static_assert(WM == 16, "two rows of waves per 32-row block");
      for (int q = 0; q < TM / 32 && rb32 + q < nrb32; ++q) {
        a.partials[o + 2 * q] = csum[2 * q][0][tid] + csum[2 * q + 1][0][tid];
        a.partials[o + 2 * q + 1] = csum[2 * q][1][tid] + csum[2 * q + 1][1][tid];
      }
    }
  }
}

template <int NT, class T>
__global__ __launch_bounds__(T::THREADS) void dense_mfma_leja_kernel(const double2* H1, const double2* H2,
                                                                     long long ld, int dim, MultiArgs a) {
  constexpr int TI = T::TI, TJ = T::TJ, KS = T::KS, WM = T::WM, WN = T::WN, TM = T::TM, TN = T::TN;
  constexpr int HU = T::HU, WU = T::WU;
  // Row strides chosen so that the operand reads of one MFMA step hit distinct
  // LDS banks (64 banks of 4 bytes, 32 lanes of 8-byte reads per pass).  W:
  // lanes l and l + 16 read rows kk and kk + 1, 16 consecutive states each,
  // so the stride is 16 doubles past a multiple of 32 (with TN + 1 nearly
  // every lane of the second half met one of the first).  H: the 16 rows of
  // an operand start a stride apart, and a stride of 2 mod 4 doubles with an
  // odd half (18 for TK = 16) puts them on sixteen distinct multiples of 4
  // banks, the next k (lanes 16..31) on the pairs in between.
  constexpr int kHStride = TK + 2, kWStride = TN + 16;
  static_assert(kHStride % 4 == 2 && (kHStride / 2) % 2 == 1, "H operand reads free of bank conflicts");
  static_assert(kWStride % 32 == 16, "W operand reads free of bank conflicts");
  __shared__ double sHre[KS][NT][TM][kHStride], sHim[KS][NT][TM][kHStride];
  __shared__ double sWre[KS][TK][kWStride], sWim[KS][TK][kWStride];
  __shared__ double csum[2][2][TN];  // [row half][w|v][state]
  __shared__ int sstop_any;
  const int B = a.B;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int kg = wv >> 2;               // K group
  const int gtid = tid & (kThreads - 1);  // thread within the group
  const int wq = wv & 3;
  const int wr = wq >> 1, wc = wq & 1;  // wave position in the 2 x 2 arrangement

  // block coordinates: the column blocks of one row block share an XCD
  const int gx = (B + TN - 1) / TN;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int rb = L / gx, cb = L % gx;
  const int row0 = rb * TM, col0 = cb * TN;

  if (tid == 0) {
    int any_running = 0;
    for (int c = col0; c < min(B, col0 + TN); ++c)
      any_running |= a.check_stop ? !load_stopped(&a.slots[c]) : 1;
    sstop_any = any_running;
  }
  __syncthreads();
  if (!sstop_any) return;  // every state of this block has stopped (uniform)

  // per-lane operand scale factors (NT = 2): columns of this lane's B operands
  double sc[NT][TJ];
#pragma unroll
  for (int tj = 0; tj < TJ; ++tj) {
    const int c = col0 + wc * WN + tj * 16 + (lane & 15);
    const ColParam P = a.prm[c < B ? c : 0];
    sc[0][tj] = NT == 2 ? P.a1 : 1.0;
    if constexpr (NT == 2) sc[1][tj] = P.a2;
  }

  // staging assignment within the group: the H tile TM x TK per term (HU
  // consecutive K entries per thread), the W tile TK x TN (WU consecutive
  // states per thread)
  const int h_r = gtid / (TK / HU), h_k = (gtid % (TK / HU)) * HU;
  const int w_k = gtid / (TN / WU), w_c = (gtid % (TN / WU)) * WU;
  const d2* W = reinterpret_cast<const d2*>(a.x);
  const d2* Hp[2] = {reinterpret_cast<const d2*>(H1), reinterpret_cast<const d2*>(H2)};
  // PD chunks of each group are in flight in registers (slot s holds the
  // chunks of rounds s, s + PD, ...): two when the staging registers leave
  // room for them (one term, small tiles), else one
  constexpr int PD = (NT == 1 && HU + WU <= 6) ? 2 : 1;
  d2 hreg[PD][NT][HU], wreg[PD][WU];
  // Loads without branches (every index clamped into the matrix), so the
  // compiler can count them and wait for one slot while the next is in
  // flight.  Rows past dim and states past B only reach outputs that are
  // never stored; entries past dim along K are zeroed on the W side when the
  // chunk is staged, which also cancels the clamped H columns.
  auto load_chunk = [&](auto slot, int k0) {
    constexpr int S = decltype(slot)::value;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int u = 0; u < HU; ++u) {
        const int r = min(row0 + h_r, dim - 1), k = min(k0 + h_k + u, dim - 1);
        hreg[S][t][u] = __builtin_nontemporal_load(Hp[t] + (long long)r * ld + k);
      }
#pragma unroll
    for (int u = 0; u < WU; ++u) {
      const int k = min(k0 + w_k, dim - 1), c = min(col0 + w_c + u, B - 1);
      wreg[S][u] = W[(long long)k * B + c];
    }
  };
  auto store_chunk = [&](auto slot, int k0) {
    constexpr int S = decltype(slot)::value;
    const bool k_in = k0 + w_k < dim;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int u = 0; u < HU; ++u) {
        sHre[kg][t][h_r][h_k + u] = hreg[S][t][u].x;
        sHim[kg][t][h_r][h_k + u] = hreg[S][t][u].y;
      }
#pragma unroll
    for (int u = 0; u < WU; ++u) {
      sWre[kg][w_k][w_c + u] = k_in ? wreg[S][u].x : 0.0;
      sWim[kg][w_k][w_c + u] = k_in ? wreg[S][u].y : 0.0;
    }
  };

  v4d are[TI][TJ], aim[TI][TJ];
#pragma unroll
  for (int ti = 0; ti < TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) {
      are[ti][tj] = v4d{0.0, 0.0, 0.0, 0.0};
      aim[ti][tj] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  const int nk = (dim + TK - 1) / TK;
  const int rounds = (nk + KS - 1) / KS;  // the same barrier count for every group
  // one round: stage this round's chunk from its slot, refill the slot with
  // the chunk PD rounds ahead, multiply
  auto round = [&](auto slot, int it) {
    const int kc = it * KS + kg;
    __syncthreads();  // previous chunk's operands consumed
    store_chunk(slot, kc * TK);
    __syncthreads();
    // refilled unconditionally (past the end the clamped loads are discarded)
    load_chunk(slot, (kc + PD * KS) * TK);  // in flight during the MFMAs
    if (kc >= nk) return;  // this group has no chunk left (uniform per wave)
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        double hre[TI], him[TI], wre[TJ], wim[TJ];
#pragma unroll
        for (int ti = 0; ti < TI; ++ti) {
          const int ar = wr * WM + ti * 16 + (lane & 15);
          hre[ti] = sHre[kg][t][ar][kk];
          him[ti] = sHim[kg][t][ar][kk];
        }
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) {
          const int bc = wc * WN + tj * 16 + (lane & 15);
          wre[tj] = sWre[kg][kk][bc] * sc[t][tj];
          wim[tj] = sWim[kg][kk][bc] * sc[t][tj];
        }
        // the 2 TI TJ accumulators are independent chains: issue one product into
        // each before the second product of any, so dependent MFMAs are never back to back
#pragma unroll
        for (int ti = 0; ti < TI; ++ti)
#pragma unroll
          for (int tj = 0; tj < TJ; ++tj) {
            are[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(hre[ti], wre[tj], are[ti][tj], 0, 0, 0);
            aim[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(hre[ti], wim[tj], aim[ti][tj], 0, 0, 0);
          }
#pragma unroll
        for (int ti = 0; ti < TI; ++ti)
#pragma unroll
          for (int tj = 0; tj < TJ; ++tj) {
            are[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-him[ti], wim[tj], are[ti][tj], 0, 0, 0);
            aim[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(him[ti], wre[tj], aim[ti][tj], 0, 0, 0);
          }
      }
    }
  };
  load_chunk(std::integral_constant<int, 0>{}, kg * TK);
  if constexpr (PD == 2) {
    load_chunk(std::integral_constant<int, 1>{}, (KS + kg) * TK);
    for (int it = 0; it < rounds; it += 2) {
      round(std::integral_constant<int, 0>{}, it);
      if (it + 1 < rounds) round(std::integral_constant<int, 1>{}, it + 1);
    }
  } else {
    for (int it = 0; it < rounds; ++it) round(std::integral_constant<int, 0>{}, it);
  }

  // the groups' accumulators, added in group order, one MFMA tile at a time:
  // group g > 0 parks its values in the (now idle) W staging buffers, group 0
  // adds them
  if constexpr (KS > 1) {
    static_assert(sizeof(sWre) >= sizeof(double) * 4 * kThreads, "accumulator exchange space");
    double* xre = &sWre[0][0][0];
    double* xim = &sWim[0][0][0];
    __syncthreads();  // every group's last chunk has been read
#pragma unroll
    for (int ti = 0; ti < TI; ++ti)
#pragma unroll
      for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
        for (int g = 1; g < KS; ++g) {
          if (kg == g) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              xre[j * kThreads + gtid] = are[ti][tj][j];
              xim[j * kThreads + gtid] = aim[ti][tj][j];
            }
          }
          __syncthreads();
          if (kg == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              are[ti][tj][j] += xre[j * kThreads + gtid];
              aim[ti][tj][j] += xim[j * kThreads + gtid];
            }
          }
          __syncthreads();
        }
  }
  const bool epi = kg == 0;  // group 0 holds the sums; the others only keep the barrier count
  group_epilogue<NT, TI, TJ, WM, WN, TM, TN>(a, dim, row0, col0, wr, wc, epi, are, aim, csum);
}

// ---------------------------------------------------------------------------
// The same iteration on the LDS-DMA tile product (mfma_dma.h): TM rows (32 or
// 64) x 64 states per workgroup of TM / 8 waves, each wave 16 rows x 32
// states.  TAIL: dim is not a multiple of the K chunk.
template <int NT, int TM, bool TAIL>
__global__ __launch_bounds__(TM * 8) void dense_mfma_dma_kernel(const double2* H1, const double2* H2, long long ld,
                                                                int dim, MultiArgs a) {
  constexpr int TI = 1, TJ = 2, WM = 16, WN = 32, TN = dma_gemm::kTN;
  __shared__ double csum[TM / WM][2][TN];  // [row of waves][w|v][state]
  __shared__ int sstop_any;
  const int B = a.B;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wv >> 1, wc = wv & 1;  // wave position: TM / 16 rows x 2 columns of waves

  // block coordinates: the column blocks of one row block share an XCD
  const int gx = (B + TN - 1) / TN;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int rb = L / gx, cb = L % gx;
  const int row0 = rb * TM, col0 = cb * TN;

  if (tid == 0) {
    int any_running = 0;
    for (int c = col0; c < min(B, col0 + TN); ++c)
      any_running |= a.check_stop ? !load_stopped(&a.slots[c]) : 1;
    sstop_any = any_running;
  }
  __syncthreads();
  if (!sstop_any) return;  // every state of this block has stopped (uniform)

  // per-lane operand scale factors (NT = 2): columns of this lane's B operands
  double sc[NT][TJ];
#pragma unroll
  for (int tj = 0; tj < TJ; ++tj) {
    const int c = col0 + wc * WN + tj * 16 + (lane & 15);
    const ColParam P = a.prm[c < B ? c : 0];
    sc[0][tj] = NT == 2 ? P.a1 : 1.0;
    if constexpr (NT == 2) sc[1][tj] = P.a2;
  }
  v4d are[TI][TJ], aim[TI][TJ];
  dma_gemm::tile_product<NT, TM, TAIL>(reinterpret_cast<const d2*>(H1), reinterpret_cast<const d2*>(H2), ld,
                                       reinterpret_cast<const d2*>(a.x), B, B, dim, row0, col0, sc, are[0], aim[0]);
  group_epilogue<NT, TI, TJ, WM, WN, TM, TN>(a, dim, row0, col0, wr, wc, true, are, aim, csum);
}

// H = a H1 + b H2 (+ k K) (row-major, row stride ld for H1, H2, dim for K and out).
template <bool WITH_K>
__global__ void dense_assemble_kernel(const double2* __restrict__ H1, const double2* __restrict__ H2, long long ld,
                                      int dim, double ca, double cb, const double2* __restrict__ K, double ck,
                                      double2* __restrict__ out) {
  // rows over the grid, columns over the threads (no index division)
  for (long long r = blockIdx.x; r < dim; r += gridDim.x) {
    const d2* h1 = reinterpret_cast<const d2*>(H1) + r * ld;
    const d2* h2 = reinterpret_cast<const d2*>(H2) + r * ld;
    double2* o = out + r * dim;
    for (int c = threadIdx.x; c < dim; c += blockDim.x) {
      d2 h = rmul(ca, __builtin_nontemporal_load(h1 + c)) + rmul(cb, __builtin_nontemporal_load(h2 + c));
      if constexpr (WITH_K) h += rmul(ck, __builtin_nontemporal_load(reinterpret_cast<const d2*>(K) + r * dim + c));
      o[c] = fromd2(h);
    }
  }
}

}  // namespace

// Partial sums are kept per 32-row block whatever the tile's height.
int dense_mfma_row_blocks(int dim) { return (dim + 31) / 32; }

namespace {
template <class T>
hipError_t launch_mfma_tile(int nterms, const double2* H1, const double2* H2, long long ld, int dim,
                            const MultiArgs& a, hipStream_t s) {
  const int gx = (a.B + T::TN - 1) / T::TN;
  const int grid = (dim + T::TM - 1) / T::TM * gx;
  if (nterms == 1) dense_mfma_leja_kernel<1, T><<<grid, T::THREADS, 0, s>>>(H1, H2, ld, dim, a);
  else dense_mfma_leja_kernel<2, T><<<grid, T::THREADS, 0, s>>>(H1, H2, ld, dim, a);
  return hipGetLastError();
}

template <int TM>
hipError_t launch_dma_tile(int nterms, const double2* H1, const double2* H2, long long ld, int dim,
                           const MultiArgs& a, hipStream_t s) {
  const int grid = (dim + TM - 1) / TM * ((a.B + 63) / 64);
  const bool tail = dim % dma_gemm::kTK != 0;
  if (nterms == 1 && tail) dense_mfma_dma_kernel<1, TM, true><<<grid, TM * 8, 0, s>>>(H1, H2, ld, dim, a);
  else if (nterms == 1) dense_mfma_dma_kernel<1, TM, false><<<grid, TM * 8, 0, s>>>(H1, H2, ld, dim, a);
  else if (tail) dense_mfma_dma_kernel<2, TM, true><<<grid, TM * 8, 0, s>>>(H1, H2, ld, dim, a);
  else dense_mfma_dma_kernel<2, TM, false><<<grid, TM * 8, 0, s>>>(H1, H2, ld, dim, a);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_dense_mfma(int nterms, const double2* H1, const double2* H2, long long ld, int dim,
                             const MultiArgs& a, hipStream_t s, int tile) {
  switch (tile) {
    case 0: return launch_mfma_tile<MfmaTile<1, 2, 2>>(nterms, H1, H2, ld, dim, a, s);  // 32 x 64, K split in two
    case 1: return launch_mfma_tile<MfmaTile<1, 2, 1>>(nterms, H1, H2, ld, dim, a, s);  // 32 x 64
    case 2: return launch_mfma_tile<MfmaTile<2, 2, 1>>(nterms, H1, H2, ld, dim, a, s);  // 64 x 64
    case 3: return launch_mfma_tile<MfmaTile<2, 2, 2>>(nterms, H1, H2, ld, dim, a, s);  // 64 x 64, K split in two
    case 4: return launch_mfma_tile<MfmaTile<1, 4, 2>>(nterms, H1, H2, ld, dim, a, s);  // 32 x 128, K split in two
    case 5: return launch_dma_tile<32>(nterms, H1, H2, ld, dim, a, s);  // 32 x 64, LDS-DMA staging
    case 6: return launch_dma_tile<64>(nterms, H1, H2, ld, dim, a, s);  // 64 x 64, LDS-DMA staging
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_dense_assemble(const double2* H1, const double2* H2, long long ld, int dim, double ca, double cb,
                                 const double2* K, double ck, double2* out, hipStream_t s) {
  if (K) dense_assemble_kernel<true><<<4096, kThreads, 0, s>>>(H1, H2, ld, dim, ca, cb, K, ck, out);
  else dense_assemble_kernel<false><<<4096, kThreads, 0, s>>>(H1, H2, ld, dim, ca, cb, nullptr, 0.0, out);
  return hipGetLastError();
}

}  // namespace magnus
