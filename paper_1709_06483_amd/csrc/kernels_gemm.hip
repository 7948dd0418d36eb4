// Commutators of dense Hermitian matrices, assembled once per pair of terms
// for Methods M4 and M6 (Section 2) on dense terms.  For Hermitian A, B the
// products A B and B A are adjoint to each other, so one complex GEMM
// C = A B gives the Hermitian i [A, B] = i (C - C^H).
//
// The GEMM runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64, four real
// products per complex 16x16x4 step).  A workgroup of four waves computes a
// 64 x 64 tile of C (each wave 32 x 32 = 2 x 2 MFMA tiles); K is staged
// through LDS 16 at a time.  The combine pass reads C and its transpose
// through 32 x 32 LDS tiles so both reads are coalesced.
#include "device_common.h"

namespace magnus {
namespace {

using namespace dev;
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int GM = 64, GN = 64, GK = 16;

__global__ __launch_bounds__(kThreads) void zgemm_kernel(const double2* A, long long lda, const double2* Bm,
                                                        long long ldb, double2* C, int n) {
  __shared__ double sAre[GM][GK + 1], sAim[GM][GK + 1];
  __shared__ double sBre[GK][GN + 1], sBim[GK][GN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  const int nb = (n + GN - 1) / GN;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int row0 = (L / nb) * GM, col0 = (L % nb) * GN;
  const d2* Ap = reinterpret_cast<const d2*>(A);
  const d2* Bp = reinterpret_cast<const d2*>(Bm);
  // staging: A tile 64 x 16 (row tid / 4, four k), B tile 16 x 64 (k tid / 16, four columns)
  const int a_r = tid >> 2, a_k = (tid & 3) * 4;
  const int b_k = tid >> 4, b_c = (tid & 15) * 4;

  v4d cre[2][2], cim[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cre[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      cim[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  for (int k0 = 0; k0 < n; k0 += GK) {
    d2 ar[4], br[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = row0 + a_r, k = k0 + a_k + u;
      ar[u] = (r < n && k < n) ? Ap[(long long)r * lda + k] : d2{0.0, 0.0};
      const int kb = k0 + b_k, c = col0 + b_c + u;
      br[u] = (kb < n && c < n) ? Bp[(long long)kb * ldb + c] : d2{0.0, 0.0};
    }
    __syncthreads();  // the previous chunk has been consumed
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      sAre[a_r][a_k + u] = ar[u].x;
      sAim[a_r][a_k + u] = ar[u].y;
      sBre[b_k][b_c + u] = br[u].x;
      sBim[b_k][b_c + u] = br[u].y;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      double are[2], aim[2], bre[2], bim[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int r = wr * 32 + t * 16 + (lane & 15);
        are[t] = sAre[r][kk];
        aim[t] = sAim[r][kk];
        const int c = wc * 32 + t * 16 + (lane & 15);
        bre[t] = sBre[kk][c];
        bim[t] = sBim[kk][c];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cre[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[i], bre[j], cre[i][j], 0, 0, 0);
          cre[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-aim[i], bim[j], cre[i][j], 0, 0, 0);
          cim[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[i], bim[j], cim[i][j], 0, 0, 0);
          cim[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim[i], bre[j], cim[i][j], 0, 0, 0);
        }
    }
  }
  // accumulator element q of a lane: row lane / 16 + 4 q, column lane % 16 of its 16 x 16 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = row0 + wr * 32 + i * 16 + (lane >> 4) + 4 * q;
        const int c = col0 + wc * 32 + j * 16 + (lane & 15);
        if (r < n && c < n) C[(long long)r * n + c] = make_double2(cre[i][j][q], cim[i][j][q]);
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
  const long long nb = (n + GN - 1) / GN;
  zgemm_kernel<<<(unsigned)(nb * nb), kThreads, 0, s>>>(A, lda, B, ldb, C, n);
  return hipGetLastError();
}

hipError_t launch_commutator_combine(const double2* C, int n, double scale, double2* K, hipStream_t s) {
  const unsigned g = (unsigned)((n + 31) / 32);
  commutator_combine_kernel<<<dim3(g, g), 256, 0, s>>>(C, n, scale, K);
  return hipGetLastError();
}

}  // namespace magnus
