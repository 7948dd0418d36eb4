// Commutators of dense Hermitian matrices, assembled once per pair of terms
// for Methods M4 and M6 (Section 2) on dense terms.  For Hermitian A, B the
// products A B and B A are adjoint to each other, so one complex GEMM
// C = A B gives the Hermitian i [A, B] = i (C - C^H).
//
// The GEMM runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64, four real
// products per complex 16x16x4 step) with the operands copied into LDS by
// LDS-DMA (mfma_dma.h).  The combine pass reads C and its transpose through
// 32 x 32 LDS tiles so both reads are coalesced.
#include "device_common.h"
#include "mfma_dma.h"

namespace magnus {
namespace {

using namespace dev;

// C = A B on the LDS-DMA tile product (mfma_dma.h): 64 x 64 of C per
// workgroup of eight waves (each 16 x 32).  TAIL: n is not a multiple of the
// K chunk.
template <bool TAIL>
__global__ __launch_bounds__(512) void zgemm_kernel(const double2* A, long long lda, const double2* Bm, long long ldb,
                                                   double2* C, int n) {
  constexpr int TM = 64, TN = dma_gemm::kTN;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wv >> 1, wc = wv & 1;
  // block coordinates: the column blocks of one row block share an XCD
  const int nb = (n + TN - 1) / TN;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int row0 = (L / nb) * TM, col0 = (L % nb) * TN;
  const double sc[1][2] = {{1.0, 1.0}};
  dma_gemm::v4d cre[2], cim[2];
  const d2* Ap = reinterpret_cast<const d2*>(A);
  dma_gemm::tile_product<1, TM, TAIL>(Ap, Ap, lda, reinterpret_cast<const d2*>(Bm), ldb, n, n, row0, col0, sc, cre,
                                      cim);
  // accumulator element q of a lane: row lane / 16 + 4 q, column lane % 16 of its 16 x 16 tile
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = row0 + wr * 16 + (lane >> 4) + 4 * q;
      const int c = col0 + wc * 32 + j * 16 + (lane & 15);
      if (r < n && c < n) C[(long long)r * n + c] = make_double2(cre[j][q], cim[j][q]);
    }
}

// K[r][c] = s i (C[r][c] - conj(C[c][r])), C and K n x n with row stride n.
__global__ __launch_bounds__(256) void commutator_combine_kernel(const double2* C, int n, double sc, double2* K) {
  __shared__ double2 t[32][33];
  const int tx = threadIdx.x & 31, ty0 = threadIdx.x >> 5;  // 32 x 8 threads
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int ty = ty0; ty < 32; ty += 8) {
    const int r = bx + ty, c = by + tx;
    t[ty][tx] = (r < n && c < n) ? C[(long long)r * n + c] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int ty = ty0; ty < 32; ty += 8) {
    const int r = by + ty, c = bx + tx;
    if (r < n && c < n) {
      const double2 a = C[(long long)r * n + c];
      const double2 b = t[tx][ty];  // C[c][r]
      K[(long long)r * n + c] = make_double2(-sc * (a.y + b.y), sc * (a.x - b.x));
    }
  }
}

// out = sum_t c_t M_t (out row stride n).
__global__ __launch_bounds__(kThreads) void assemble_terms_kernel(AssembleTerms T, int n, double2* __restrict__ out) {
  // rows over the grid, columns over the threads (no index division)
  for (long long r = blockIdx.x; r < n; r += gridDim.x)
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
      d2 h = {0.0, 0.0};
      for (int t = 0; t < T.nterms; ++t)
        h += rmul(T.c[t], __builtin_nontemporal_load(reinterpret_cast<const d2*>(T.m[t]) + r * T.ld[t] + c));
      out[r * n + c] = fromd2(h);
    }
}

}  // namespace

hipError_t launch_assemble_terms(const AssembleTerms& T, int n, double2* out, hipStream_t s) {
  if (T.nterms < 1 || T.nterms > kMaxAssembleTerms) return hipErrorInvalidValue;
  assemble_terms_kernel<<<4096, kThreads, 0, s>>>(T, n, out);
  return hipGetLastError();
}

hipError_t launch_zgemm(const double2* A, long long lda, const double2* B, long long ldb, double2* C, int n,
                        hipStream_t s) {
  const long long nb = (n + dma_gemm::kTN - 1) / dma_gemm::kTN;
  if (n % dma_gemm::kTK) zgemm_kernel<true><<<(unsigned)(nb * nb), 512, 0, s>>>(A, lda, B, ldb, C, n);
  else zgemm_kernel<false><<<(unsigned)(nb * nb), 512, 0, s>>>(A, lda, B, ldb, C, n);
  return hipGetLastError();
}

hipError_t launch_commutator_combine(const double2* C, int n, double scale, double2* K, hipStream_t s) {
  const unsigned g = (unsigned)((n + 31) / 32);
  commutator_combine_kernel<<<dim3(g, g), 256, 0, s>>>(C, n, scale, K);
  return hipGetLastError();
}

}  // namespace magnus
