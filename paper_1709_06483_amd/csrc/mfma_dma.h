// Complex FP64 matrix-core tile product with its operands staged by LDS-DMA,
// shared by the dense Leja group iteration (Y = H W for a group of states)
// and the commutator GEMM (C = A B).
//
// A workgroup of TM / 8 waves (TM = 32 or 64) computes a TM x 64 block of
// rows x columns of  sum_t H_t (sc_t W)  (NT = 1 or 2 terms, sc_t a per-column
// scale), each wave 16 rows x 32 columns as two 16 x 16 tiles of
// v_mfma_f64_16x16x4f64, four real MFMAs per complex step:
//   Yre += Hre Wre - Him Wim,   Yim += Hre Wim + Him Wre.
//
// Each K chunk of 16 of the H block (TM rows x 16) and of the W block
// (16 x 64 columns) goes from memory straight into LDS with global_load_lds
// (no registers held while in flight), three chunks deep, so a workgroup
// passes one barrier per chunk: at the top of chunk c every wave waits until
// its own copies of chunk c have landed (only chunk c + 1's remain in
// flight), the barrier then covers everybody's copies and everybody's reads
// of chunk c - 1, whose buffer takes chunk c + 2's copies.  The copies place
// complex elements k-major (slot k * TM + r for H, k * 64 + c for W; a copy's
// lanes may load any addresses, so the transposition of the row-major H is
// free), which makes each MFMA step's operand reads 16-byte reads of 16
// consecutive slots: one read gives a lane both halves of its complex
// operand, free of bank conflicts.  The copies are issued from inline asm,
// so the compiler, which does not see them, neither makes every LDS read wait
// for all copies in flight (it cannot tell the buffers apart) nor keeps the
// operand reads in place: it schedules them as ordinary LDS loads ahead of
// the MFMAs that use them.  The waits for the copies are explicit (before
// each barrier, for all of them before the first copy, so the compiler's own
// count of outstanding loads stays an upper bound, and after the last chunk).
// The three buffers are separate LDS arrays and the chunk loop is unrolled by
// three, so every buffer index is a constant; a chunk's body has no branch
// (past the last chunk the copies repeat it), so the compiler may move
// operand reads ahead across its steps.
#pragma once

#include <type_traits>

#include "device_common.h"

namespace magnus {
namespace {
namespace dma_gemm {

using namespace dev;
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kTK = 16;  // K chunk
constexpr int kTN = 64;  // columns per workgroup

__device__ __forceinline__ unsigned lds_offset(const void* p) {
  return (unsigned)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// One 16-byte-per-lane copy from memory into LDS at lds + 16 * lane (lds
// wave-uniform); M0 takes the LDS address, and the copy reads M0 one wait
// state after it was written.
__device__ __forceinline__ void copy16(const void* src, unsigned lds) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "s"(lds) : "memory", "m0");
}

// The LDS staging buffers, one pair of arrays per buffer.
template <int NT, int TM, int BUF>
struct Buf {
  static __device__ __forceinline__ d2 (&h())[NT][kTK][TM] {
    __shared__ d2 a[NT][kTK][TM];
    return a;
  }
  static __device__ __forceinline__ d2 (&w())[kTK][kTN] {
    __shared__ d2 a[kTK][kTN];
    return a;
  }
};

// The workgroup's block at rows row0.., columns col0..: H_t is dim x dim
// (row stride ld), W is dim x ncols (row stride ldw).  Rows past dim and
// columns past ncols are read clamped (they reach only outputs the caller
// does not store); TAIL (dim not a multiple of 16) zeroes the W entries past
// dim along K as they are read.  On return are/aim hold this wave's two
// 16 x 16 tiles (element j of a lane: row lane / 16 + 4 j, column lane % 16
// of its tile; wave wv covers rows (wv / 2) * 16.., columns (wv % 2) * 32 +
// 16 tj..) and no copy is in flight.  sc[t][tj]: scale of this lane's W
// column in term t.  All waves of the workgroup call it.
template <int NT, int TM, bool TAIL>
__device__ __forceinline__ void tile_product(const d2* H1, const d2* H2, long long ld, const d2* W, long long ldw,
                                             int ncols, int dim, int row0, int col0, const double (&sc)[NT][2],
                                             v4d (&are)[2], v4d (&aim)[2]) {
  constexpr int TK = kTK, TN = kTN, WM = 16, WN = 32;
  constexpr int NW = TM / 8;                  // waves
  constexpr int kHCopies = TM * TK / 64;      // copies of one term's H chunk per workgroup
  constexpr int kHOps = NT * kHCopies / NW;   // copy instructions per wave and chunk: H
  constexpr int kWOps = TK * TN / 64 / NW;    // and W
  constexpr int kOps = kHOps + kWOps;
  static_assert(kOps < 16, "vmcnt field");
  static_assert(kHCopies % NW == 0 && (TK * TN / 64) % NW == 0, "copies spread evenly over the waves");
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wv >> 1, wc = wv & 1;
  const d2* Hp[2] = {H1, H2};
  // This wave's copies: H copy u of the workgroup covers term u / kHCopies,
  // slots (u % kHCopies) * 64 + lane = k * TM + r, at LDS offset hdst; W copy
  // k covers row k of the chunk.
  unsigned hdst[kHOps];
#pragma unroll
  for (int i = 0; i < kHOps; ++i) {
    const int u = wv * kHOps + i;
    hdst[i] = (unsigned)(((u / kHCopies) * TK * TM + (u % kHCopies) * 64) * sizeof(d2));
  }
  const int wcol = min(col0 + lane, ncols - 1);
  const int nk = (dim + TK - 1) / TK;
  // copies of K chunk kc into buffer buf, indices clamped into the matrices
  auto copy_chunk = [&](int kc, auto buf) {
    constexpr int BF = decltype(buf)::value;
    const unsigned hb = lds_offset(&Buf<NT, TM, BF>::h()[0][0][0]);
    const unsigned wb = lds_offset(&Buf<NT, TM, BF>::w()[0][0]);
    const int k0 = min(kc, nk - 1) * TK;
#pragma unroll
    for (int i = 0; i < kHOps; ++i) {
      const int u = wv * kHOps + i;
      const int t = u / kHCopies, sl = (u % kHCopies) * 64 + lane;
      const int row = min(row0 + sl % TM, dim - 1), col = min(k0 + sl / TM, dim - 1);
      copy16(Hp[t] + (long long)row * ld + col, hb + hdst[i]);
    }
#pragma unroll
    for (int i = 0; i < kWOps; ++i) {
      const int k = wv * kWOps + i;
      const int kr = min(k0 + k, dim - 1);
      copy16(W + (long long)kr * ldw + wcol, wb + (unsigned)(k * TN * sizeof(d2)));
    }
  };

#pragma unroll
  for (int tj = 0; tj < 2; ++tj) {
    are[tj] = v4d{0.0, 0.0, 0.0, 0.0};
    aim[tj] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the caller's loads are done before the first copy
  copy_chunk(0, std::integral_constant<int, 0>{});
  copy_chunk(1, std::integral_constant<int, 1>{});
  // this lane's operands: H row hr, W columns wc * WN + tj * 16 + lane % 16, K offset kq
  const int hr = wr * WM + (lane & 15), kq = lane >> 4;
  // chunk kc from buffer buf: wait for it (with chunk kc + 1's copies still
  // in flight), release chunk kc - 1's buffer to chunk kc + 2's copies
  // (issued after the first step's operand reads, which then wait on nothing
  // but LDS), multiply
  auto chunk = [&](int kc, auto buf) {
    constexpr int BF = decltype(buf)::value;
    auto& sh = Buf<NT, TM, BF>::h();
    auto& sw = Buf<NT, TM, BF>::w();
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(kOps) : "memory");
    const int k0 = kc * TK;
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      const bool k_in = !TAIL || k0 + ks * 4 + kq < dim;
      d2 h[NT], wv2[2];
#pragma unroll
      for (int t = 0; t < NT; ++t) h[t] = sh[t][ks * 4 + kq][hr];
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        wv2[tj] = sw[ks * 4 + kq][wc * WN + tj * 16 + (lane & 15)];
        if (!k_in) wv2[tj] = d2{0.0, 0.0};
      }
      if (ks == 0) copy_chunk(kc + 2, std::integral_constant<int, (BF + 2) % 3>{});
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        double wre[2], wim[2];
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          wre[tj] = wv2[tj].x * sc[t][tj];
          wim[tj] = wv2[tj].y * sc[t][tj];
        }
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          are[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(h[t].x, wre[tj], are[tj], 0, 0, 0);
          aim[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(h[t].x, wim[tj], aim[tj], 0, 0, 0);
        }
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          // the last argument sets the MFMA's negate modifier on A: -Him Wim
          are[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(h[t].y, wim[tj], are[tj], 0, 0, 1);
          aim[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(h[t].y, wre[tj], aim[tj], 0, 0, 0);
        }
      }
    }
  };
  for (int kc = 0; kc < nk; kc += 3) {
    chunk(kc, std::integral_constant<int, 0>{});
    if (kc + 1 < nk) chunk(kc + 1, std::integral_constant<int, 1>{});
    if (kc + 2 < nk) chunk(kc + 2, std::integral_constant<int, 2>{});
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): no copy into this workgroup's LDS is still in flight
}

}  // namespace dma_gemm
}  // namespace
}  // namespace magnus
