// The C ABI of libmagnus (declared in include/magnus.h).
//
// Host side of the hot path: argument validation, per-exponential Leja
// planning (planner.h), buffer rotation for the Newton recurrence and its
// substeps, and the two fourth-order Magnus steps of Section 2 (Cf4, M4)
// built from chained exponentials.  All device work is in kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/magnus.h"
#include "kernels.h"
#include "planner.h"

using magnus::ColParam;
using magnus::CsrDev;
using magnus::ExpPlan;
using magnus::IterArgs;
using magnus::MultiArgs;
using magnus::PersistArgs;
using magnus::PersistExp;
using magnus::PersistProblem;
using magnus::Slot;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(MAGNUS_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Workspace vectors per state.
enum Vec { kA = 0, kB, kS0, kS1, kS2, kU, kV, kY, kNumVec };

// Device table of per-state Leja parameters (ColParam entries) filled once per call segment.
constexpr size_t kTableCap = 1 << 18;
// Per-call headers of the persistent small-state kernel.
constexpr size_t kArenaBytes = 8u << 20;
// States of at most this many entries run whole propagations in one workgroup.
constexpr int64_t kSmallDim = magnus::kPersistMaxDim;
// Row mappings magnus_autotune times (variant codes 1..kTuneVariants).
constexpr int kTuneVariants = 7;

}  // namespace

struct magnus_ctx {
  int device = 0;
  int64_t max_dim = 0;
  int32_t max_batch = 0;
  double2* vecs = nullptr;     // kNumVec vectors of max_dim * max_batch entries
  Slot* slots = nullptr;       // one control block per state of a batch
  int nslots = 0;
  int sticky_status = 0;       // status bits of slots reset inside the current call
  ColParam* table = nullptr;   // kTableCap entries
  unsigned char* arena = nullptr;  // kArenaBytes
  int persist = 1;  // MAGNUS_PERSIST: 0 never, 1 by size and state count, 2 every state of at most kSmallDim
  int fuse = 1;     // MAGNUS_FUSE: 0 a decide kernel after every iteration, 1 stop tests fused on small grids
  magnus::IterArgs fz_last{};  // the arguments of a final check of the last fused iteration
  bool fz_pending = false;     // a fused iteration ran since the last final check
  // graph replay of single-state steps (MAGNUS_GRAPH: 0 off, 1 on): one Magnus
  // step captured on cap_stream, replayed once per step with the step's Leja
  // coefficients read from a device table indexed by the counter *gctr
  int graph = 0;         // off by default: replays measured slower than launches once the stop tests are fused
  int graph_chunk = 0;  // MAGNUS_GRAPH_STEPS: steps per uploaded table chunk (0: as many as fit)
  int ragged_joint = 1; // MAGNUS_RAGGED_JOINT: 0 runs a ragged batch's large problems one after another
  int* gctr = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph_g = nullptr;
  hipGraphExec_t graph_x = nullptr;
  hipEvent_t graph_done = nullptr;  // recorded after the last replay of the current graph
  std::vector<magnus::IterCoef> graph_table;  // host side of the last uploaded table chunk
  double2* assembled = nullptr;  // magnus_reserve_dense
  int64_t assembled_dim = 0;
  double2* comm = nullptr;       // magnus_dense_commutator: K = i[H1, H2], row stride comm_dim
  int64_t comm_dim = 0;
  const void* comm_h1 = nullptr;  // the dense pair K belongs to (value pointers, dim, ld)
  const void* comm_h2 = nullptr;
  int64_t comm_n = 0, comm_ld = 0;
  // magnus_csr_commutator: K = i[H1, H2] as CSR (row stride-free arrays of
  // kc_rows + 1, kc_cap entries) for the pair of CSR terms recognised by kc_key
  int* kc_rp = nullptr;
  int* kc_ci = nullptr;
  double2* kc_val = nullptr;
  int64_t kc_rows = 0, kc_cap = 0, kc_nnz = 0;
  std::tuple<const void*, const void*, const void*, const void*, int64_t> kc_key{nullptr, nullptr, nullptr, nullptr, 0};
  // magnus_csr_m6_prepare: P_a = -i[H_a, K] (a = 1, 2) as CSR for the pair K
  // belongs to (valid while pm_key equals kc_key), their enclosures, and six
  // work vectors of pm_ws_dim entries for the M6 iteration (u_1..u_5, y0)
  int* pm_rp[2] = {nullptr, nullptr};
  int* pm_ci[2] = {nullptr, nullptr};
  double2* pm_val[2] = {nullptr, nullptr};
  int64_t pm_rows[2] = {0, 0}, pm_cap[2] = {0, 0}, pm_nnz[2] = {0, 0};
  double pm_lo[2] = {0.0, 0.0}, pm_hi[2] = {0.0, 0.0};
  double2* pm_ws = nullptr;
  int64_t pm_ws_dim = 0;
  std::tuple<const void*, const void*, const void*, const void*, int64_t> pm_key{nullptr, nullptr, nullptr, nullptr, 0};
  // magnus_dense_m6_prepare: the nested commutators of M6, kM6Mats matrices of
  // m6_dim^2 entries, with Gershgorin enclosures, for the pair K belongs to
  double2* m6 = nullptr;
  int64_t m6_dim = 0;
  bool m6_ready = false;
  double m6_lo[7] = {0, 0, 0, 0, 0, 0, 0}, m6_hi[7] = {0, 0, 0, 0, 0, 0, 0};
  double* partials = nullptr;  // npartials doubles
  size_t npartials = 0;
  int64_t max_grid = 0;
  double* scan = nullptr;      // per-workgroup outputs of the Gershgorin scans
  int64_t scan_len = 0;
  std::set<std::tuple<const void*, const void*, const void*, int64_t, int64_t>> validated;
  std::mutex mu;
  // kernel timing: (kind, start, stop) per recorded launch, events reused from a pool
  int csr_variant = 0;  // MAGNUS_CSR_VARIANT: 0 auto (row per lane in blocks of 32 rows, of 64 from
                        // 32768 rows, wave tiles of 16 rows from 65536, streamed wave tiles from 131072),
                        // 1 nonzero-streaming, 2-4 row-per-lane (64/32/128 rows), 5-6 wave tiles
                        // (8/16 rows), 7 streamed wave tiles
  // magnus_autotune results, per CSR term pair (H1 row_ptr, dim): the variant code
  // of the single-state iteration and the states per multi-state pass
  std::map<std::pair<const void*, int64_t>, int> tuned_variant, tuned_group;
  // magnus_autotune results for dense terms, per (H1 values, dim): rows per
  // wave of the GEMV iteration and the FP64-MFMA tile of group iterations
  std::map<std::pair<const void*, int64_t>, int> tuned_dense_rpw, tuned_mfma;
  int dense_rpw_env = 0;   // MAGNUS_DENSE_RPW: 1, 2 or 4 rows per wave of the GEMV iteration (0: tuned or 2)
  int persist_cache = 1;   // MAGNUS_PERSIST_CACHE: 0 keeps the small-state kernel's term 1 out of LDS
  int fuse_assembly = 1;   // MAGNUS_ASSEMBLE_FUSED: 0 assembles a dense exponent in a pass of its own
  int mfma_tile_env = -1;  // MAGNUS_MFMA_TILE: 0..6 forces an FP64-MFMA tile shape (-1: tuned or the size rule)
  int timing = 0;  // 0 off, k >= 1: every k-th launch of each kernel class is bracketed
  int64_t timing_seq[MAGNUS_KERNEL_CSR_LEJA3 + 1] = {};  // launches of each class since enabling
  std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> records;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;

  double2* vec(int k) { return vecs + (size_t)k * (size_t)max_dim * (size_t)max_batch; }
};

namespace {

bool is_fin(double x) { return std::isfinite(x); }

int check_term(const magnus_term& t, int64_t dim, const char* name) {
  if (t.format != MAGNUS_CSR && t.format != MAGNUS_DENSE)
    return fail(MAGNUS_EINVAL, "%s: unknown format %d", name, t.format);
  if (t.dim != dim) return fail(MAGNUS_EINVAL, "%s: dim %lld != %lld", name, (long long)t.dim, (long long)dim);
  if (t.format == MAGNUS_CSR) {
    if (t.nnz < 0 || t.nnz > INT32_MAX) return fail(MAGNUS_EINVAL, "%s: nnz %lld out of range", name, (long long)t.nnz);
    // a term without entries (the zero matrix) may pass null column and value arrays
    if (!t.row_ptr || (t.nnz > 0 && (!t.col_idx || !t.val)))
      return fail(MAGNUS_EINVAL, "%s: null CSR array", name);
  } else {
    if (!t.val) return fail(MAGNUS_EINVAL, "%s: null val", name);
    if (t.ld < dim) return fail(MAGNUS_EINVAL, "%s: ld %lld < dim", name, (long long)t.ld);
  }
  if (!is_fin(t.lam_min) || !is_fin(t.lam_max) || t.lam_min > t.lam_max)
    return fail(MAGNUS_EDOMAIN, "%s: spectral enclosure [%g, %g] invalid", name, t.lam_min, t.lam_max);
  return MAGNUS_OK;
}

int check_ham(magnus_ctx* ctx, const magnus_hamiltonian* h, int need_k) {
  if (!ctx) return fail(MAGNUS_EINVAL, "null context");
  if (!h) return fail(MAGNUS_EINVAL, "null hamiltonian");
  const int64_t dim = h->H1.dim;
  if (dim < 1) return fail(MAGNUS_EINVAL, "dim %lld < 1", (long long)dim);
  if (dim > ctx->max_dim) return fail(MAGNUS_ENOMEM, "dim %lld exceeds workspace max_dim %lld", (long long)dim, (long long)ctx->max_dim);
  if (dim > INT32_MAX / 2) return fail(MAGNUS_EINVAL, "dim %lld too large", (long long)dim);
  int rc = check_term(h->H1, dim, "H1");
  if (rc) return rc;
  rc = check_term(h->H2, dim, "H2");
  if (rc) return rc;
  if (h->H1.format != h->H2.format) return fail(MAGNUS_EINVAL, "H1 and H2 must share a format");
  if (h->H1.format == MAGNUS_DENSE && h->H1.ld != h->H2.ld)
    return fail(MAGNUS_EINVAL, "dense H1 and H2 must share the row stride ld");
  if (need_k && (!is_fin(h->k_min) || !is_fin(h->k_max) || h->k_min > h->k_max))
    return fail(MAGNUS_EDOMAIN, "commutator enclosure [%g, %g] invalid", h->k_min, h->k_max);
  return MAGNUS_OK;
}

int check_opts(const magnus_leja_opts* o) {
  if (!o) return fail(MAGNUS_EINVAL, "null options");
  if (!(o->tol > 0.0) || !is_fin(o->tol)) return fail(MAGNUS_EDOMAIN, "tol %g must be positive and finite", o->tol);
  if (o->max_degree < 1 || o->max_degree > MAGNUS_MAX_DEGREE)
    return fail(MAGNUS_EINVAL, "max_degree %d outside 1..%d", o->max_degree, MAGNUS_MAX_DEGREE);
  if (o->max_substeps < 1) return fail(MAGNUS_EINVAL, "max_substeps %d < 1", o->max_substeps);
  if (o->tol_mode != 0 && o->tol_mode != 1) return fail(MAGNUS_EINVAL, "tol_mode %d", o->tol_mode);
  return MAGNUS_OK;
}

// Structural check (and Gershgorin enclosure) of a CSR term, run once per term.
int csr_scan(magnus_ctx* ctx, const magnus_term& t, hipStream_t s, double* lo, double* hi) {
  const int dim = (int)t.dim;
  const int grid = magnus::csr_gershgorin_grid(dim);
  if (3 * (int64_t)grid > ctx->scan_len) return fail(MAGNUS_ENOMEM, "scan buffer too small");
  auto key = std::make_tuple((const void*)t.row_ptr, (const void*)t.col_idx, t.val, t.dim, t.nnz);
  {
    // a term scanned again (its arrays may have been rewritten) counts as valid only if this scan passes
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->validated.erase(key);
  }
  double* dout = ctx->scan;
  CsrDev d{t.row_ptr, t.col_idx, reinterpret_cast<const double2*>(t.val)};
  hipError_t e = magnus::launch_csr_gershgorin(d, dim, t.nnz, dout, grid, s);
  std::vector<double> h(3 * (size_t)grid);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), dout, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(MAGNUS_EHIP, "CSR scan: %s", hipGetErrorString(e));
  double a = INFINITY, b = -INFINITY;
  bool bad = false;
  for (int g = 0; g < grid; ++g) {
    a = std::fmin(a, h[3 * g]);
    b = std::fmax(b, h[3 * g + 1]);
    bad = bad || h[3 * g + 2] != 0.0;
  }
  if (bad) return fail(MAGNUS_EINVAL, "malformed CSR (row_ptr not monotone / not 0..nnz, or column out of range)");
  *lo = a;
  *hi = b;
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->validated.insert(key);
  return MAGNUS_OK;
}

int ensure_valid(magnus_ctx* ctx, const magnus_hamiltonian* h, hipStream_t s) {
  for (const magnus_term* t : {&h->H1, &h->H2}) {
    if (t->format != MAGNUS_CSR) continue;
    auto key = std::make_tuple((const void*)t->row_ptr, (const void*)t->col_idx, t->val, t->dim, t->nnz);
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      if (ctx->validated.count(key)) continue;
    }
    double lo, hi;
    int rc = csr_scan(ctx, *t, s, &lo, &hi);
    if (rc) return rc;
  }
  return MAGNUS_OK;
}

int dense_scan(magnus_ctx* ctx, const magnus_term& t, hipStream_t s, double* lo, double* hi) {
  const int dim = (int)t.dim;
  const int grid = magnus::dense_gershgorin_grid(dim);
  if (2 * (int64_t)grid > ctx->scan_len) return fail(MAGNUS_ENOMEM, "scan buffer too small");
  double* dout = ctx->scan;
  hipError_t e = magnus::launch_dense_gershgorin(reinterpret_cast<const double2*>(t.val), dim, t.ld, dout, grid, s);
  std::vector<double> h(2 * (size_t)grid);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), dout, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(MAGNUS_EHIP, "dense scan: %s", hipGetErrorString(e));
  double a = INFINITY, b = -INFINITY;
  for (int g = 0; g < grid; ++g) { a = std::fmin(a, h[2 * g]); b = std::fmax(b, h[2 * g + 1]); }
  *lo = a;
  *hi = b;
  return MAGNUS_OK;
}

// Host-side record of the work a call enqueued.
struct Acc {
  int64_t exponentials = 0, substeps = 0, planned = 0;
  int64_t extra_iters = 0;  // iterations already counted by nested calls
  int32_t max_m = 0, max_s = 0;
  double max_bound = 0.0;
  int products_per_iter = 2;
};

struct ExpOp {
  const magnus_hamiltonian* h;
  double a, b, kappa;
  const double2* assembled = nullptr;  // dense: the exponent assembled (row stride dim), used with a = 1
  bool has_interval = false;           // spectral enclosure given (else Weyl from a, b, kappa)
  double lo = 0.0, hi = 0.0;
  const double* m6c = nullptr;         // CSR Method M6: the ten coefficients of the exponent (matrix-free)
  // dense: the first iteration also writes the assembled exponent
  // fuse_out = fa H1 + fb H2 (+ fk K), the matrix `assembled` points to
  bool fuse_assembly = false;
  double fa = 0.0, fb = 0.0, fk = 0.0;
  const double2* fK = nullptr;
  double2* fuse_out = nullptr;
};

// Whether the context holds K = i[H1, H2] of this pair of CSR terms.
bool csr_comm_ready(const magnus_ctx* ctx, const magnus_hamiltonian* h) {
  return ctx->kc_rp && h->H1.format == MAGNUS_CSR &&
         ctx->kc_key == std::make_tuple((const void*)h->H1.row_ptr, h->H1.val, (const void*)h->H2.row_ptr, h->H2.val,
                                        h->H1.dim);
}

// Whether the context holds K and P_1, P_2 of Method M6 for this pair of CSR terms.
bool csr_m6_ready(const magnus_ctx* ctx, const magnus_hamiltonian* h) {
  return csr_comm_ready(ctx, h) && ctx->pm_key == ctx->kc_key && ctx->pm_ws && ctx->pm_ws_dim >= h->H1.dim;
}

// Whether the context holds K = i[H1, H2] of this pair of dense terms.
bool dense_comm_ready(const magnus_ctx* ctx, const magnus_hamiltonian* h) {
  return ctx->comm && ctx->comm_h1 == h->H1.val && ctx->comm_h2 == h->H2.val && ctx->comm_n == h->H1.dim &&
         ctx->comm_ld == h->H1.ld;
}

// Row mapping of the single-state CSR iteration for a variant code (the
// MAGNUS_CSR_VARIANT numbering; 0 = the size heuristic).
int variant_rows(int code, int64_t dim) {
  switch (code) {
    case 1: return dim >= 65536 ? 64 : 16;
    case 2: return magnus::kRowLane;
    case 3: return -32;
    case 4: return -128;
    case 5: return magnus::kWaveTile + 8;
    case 6: return magnus::kWaveTile + 16;
    case 7: return magnus::kStreamTile;
    // Measured on spin chains, Cf4 steps/s with each mapping (the stop test is
    // fused into the iteration on grids of at most kFuseMaxGrid workgroups, else
    // a decide kernel follows every iteration): the streamed tiles from 2^17
    // rows on (n = 17: 2,566 against 2,378 with 8-row wave tiles; n = 18, 19,
    // 20: 42 vs 48 us and 169 vs 183 us per iteration), 16-row wave tiles at
    // 2^16 (3,796 against 3,730), a row per lane in blocks of 64 rows at 2^15
    // (8,134 against 4,922 with 16-row nonzero streaming) and of 32 rows
    // below (n = 14: 9,183 against 7,585; n = 13: 9,983 against 9,657).
    default:
      return dim >= 131072 ? magnus::kStreamTile
             : dim >= 65536 ? magnus::kWaveTile + 16
             : dim >= 32768 ? -64
                            : -32;
  }
}

int rows_per_block(magnus_ctx* ctx, const magnus_hamiltonian* h) {
  if (ctx->csr_variant) return variant_rows(ctx->csr_variant, h->H1.dim);
  auto it = ctx->tuned_variant.find({(const void*)h->H1.row_ptr, h->H1.dim});
  return variant_rows(it == ctx->tuned_variant.end() ? 0 : it->second, h->H1.dim);
}

// Tuned dense choices (the defaults until magnus_autotune ran on these terms).
int dense_rpw(const magnus_ctx* ctx, const magnus_hamiltonian* h) {
  if (ctx->dense_rpw_env > 0) return ctx->dense_rpw_env;
  auto it = ctx->tuned_dense_rpw.find({h->H1.val, h->H1.dim});
  return it == ctx->tuned_dense_rpw.end() ? 2 : it->second;
}
// Untuned FP64-MFMA tile: the LDS-DMA tiles, 64 x 64 once its grid has a
// workgroup for every compute unit, else 32 x 64.  Measured (autotuner, us per
// launch, 32 x 64 / 64 x 64): 512 x 16 states 39.5 / 63.4, 1024 x 128 78.9 /
// 126.6, 2048 x 256 156.0 / 245.6, 4096 x 128 310.4 / 488.0, 4096 x 256
// 536.8 / 482.9, 8192 x 64 580.2 / 945.6, 8192 x 256 2,060.6 / 1,908.8; the
// register-staged tiles were slower at every one of these shapes.
int mfma_tile(const magnus_ctx* ctx, const magnus_hamiltonian* h, int B) {
  if (ctx->mfma_tile_env >= 0) return ctx->mfma_tile_env;
  auto it = ctx->tuned_mfma.find({h->H1.val, h->H1.dim});
  if (it != ctx->tuned_mfma.end()) return it->second;
  const long long blocks = (h->H1.dim + 63) / 64 * ((B + 63) / 64);
  return blocks >= 256 ? 6 : 5;
}

hipEvent_t next_event(magnus_ctx* ctx) {
  if (ctx->pool_used == ctx->pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->pool.push_back(e);
  }
  return ctx->pool[ctx->pool_used++];
}

// Launch f() on stream s, bracketed by events when the context records timings.
template <class F>
hipError_t timed(magnus_ctx* ctx, int kind, hipStream_t s, F f) {
  if (!ctx->timing) return f();
  if (ctx->timing_seq[kind]++ % ctx->timing != 0) return f();
  hipEvent_t a = next_event(ctx), b = next_event(ctx);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e == hipSuccess) e = f();
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) ctx->records.emplace_back(kind, a, b);
  return e;
}

// The last fused iteration's partials are checked for non-finite norms by a
// small kernel, enqueued before anything else writes the partials buffer or
// the control slots (another kind of launch, the end of the call).
int flush_fused_check(magnus_ctx* ctx, hipStream_t s) {
  if (!ctx->fz_pending) return MAGNUS_OK;
  ctx->fz_pending = false;
  HIP_TRY(magnus::launch_leja_final_check(ctx->fz_last, s));
  return MAGNUS_OK;
}

// Launch one Leja iteration (both passes for a commutator exponent).
// One Leja iteration of Method M6 on CSR terms, the exponent's nested
// commutators applied to vectors.  With K = i[H1,H2], P_a = -i[H_a,K] assembled
// and U_ab = i[H_a,P_b], R_a = -i[K,P_a], the Hermitian exponent times w is
//   y = c0 H1w + c1 H2w + c2 Kw + c3 P1w + c4 P2w
//     + i H1 (c5 P1w + c6 P2w) - i c5 P1 H1w - i c6 P2 H1w      (c5 U11 + c6 U12)
//     + i c7 H2 P2w - i c7 P2 H2w                                (c7 U22)
//     - i K (c8 P1w + c9 P2w) + i c8 P1 Kw + i c9 P2 Kw          (c8 R1 + c9 R2)
// Grouped by matrix, y = y0 + H1 u1 + H2 u2 + K u3 + P1 u4 + P2 u5 with
// y0 the first line and u1 = i(c5 P1w + c6 P2w), u2 = i c7 P2w,
// u3 = -i(c8 P1w + c9 P2w), u4 = i(c8 Kw - c5 H1w), u5 = i(c9 Kw - c6 H1w - c7 H2w):
// one pass over the five matrices forms y0 and the u's row by row, a second
// applies them and makes the Leja update, then the stop decision (ten matrix
// reads where the thirteen products one by one would make thirteen).
int m6_csr_iteration(magnus_ctx* ctx, const ExpOp& op, double scale, const IterArgs& a, hipStream_t s) {
  if (int rc = flush_fused_check(ctx, s)) return rc;
  const magnus_hamiltonian* h = op.h;
  const int dim = (int)h->H1.dim;
  const double* c = op.m6c;
  const CsrDev H1{h->H1.row_ptr, h->H1.col_idx, reinterpret_cast<const double2*>(h->H1.val)};
  const CsrDev H2{h->H2.row_ptr, h->H2.col_idx, reinterpret_cast<const double2*>(h->H2.val)};
  const CsrDev K{ctx->kc_rp, ctx->kc_ci, ctx->kc_val};
  const CsrDev P1{ctx->pm_rp[0], ctx->pm_ci[0], ctx->pm_val[0]};
  const CsrDev P2{ctx->pm_rp[1], ctx->pm_ci[1], ctx->pm_val[1]};
  magnus::M6Terms T{{H1, H2, K, P1, P2}};
  magnus::M6Coef C{};
  for (int k = 0; k < 10; ++k) C.c[k] = c[k];
  magnus::M6Vecs V{};
  for (int k = 0; k < magnus::kM6Terms; ++k) V.u[k] = ctx->pm_ws + (size_t)k * (size_t)ctx->pm_ws_dim;
  V.y0 = ctx->pm_ws + (size_t)magnus::kM6Terms * (size_t)ctx->pm_ws_dim;
  HIP_TRY(magnus::launch_m6_stage_a(T, a.wcur, C, V, dim, a.slot, a.check_stop, s));
  HIP_TRY(timed(ctx, MAGNUS_KERNEL_CSR_LEJA, s, [&] { return magnus::launch_m6_stage_b(T, V, scale, dim, a, s); }));
  HIP_TRY(magnus::launch_leja_decide(a, magnus::m6_grid(dim), s));
  return MAGNUS_OK;
}

// Stop test of iteration i: fused into the iteration kernel on grids of at
// most kFuseMaxGrid workgroups (every workgroup reduces iteration i-1's
// partials, which alternate between two halves of the partials buffer),
// else a decide kernel after each iteration.  Sets a->fused.
int setup_stop_test(magnus_ctx* ctx, const ExpPlan& P, int i, int grid, IterArgs* a, hipStream_t s) {
  a->iter = i;
  a->fused = 0;
  if (!ctx->fuse || grid > magnus::kFuseMaxGrid) return flush_fused_check(ctx, s);
  const size_t half = 2 * (size_t)ctx->max_grid;
  a->fused = 1;
  a->partials = ctx->partials + (size_t)(i & 1) * half;
  a->prev_partials = ctx->partials + (size_t)((i - 1) & 1) * half;
  a->prev_grid = grid;
  a->prev_dabs = i >= 2 ? std::abs(P.d[i - 1]) : 0.0;
  // the call's last fused iteration is checked for non-finite norms at its end
  ctx->fz_last = *a;
  ctx->fz_last.iter = i + 1;
  ctx->fz_last.prev_partials = a->partials;
  ctx->fz_pending = true;
  return MAGNUS_OK;
}

// Table column of one iteration launch in a captured step (graph replay).
struct TableRef {
  const magnus::IterCoef* col;  // record of this iteration in step 0
  int stride;                   // records per step
  const int* step;              // device step counter
};

int launch_iteration(magnus_ctx* ctx, const ExpOp& op, const ExpPlan& P, int i, const double2* win,
                     double2* wout, double2* pacc, double tol_sub, int early, hipStream_t s,
                     const TableRef* tab = nullptr) {
  const magnus_hamiltonian* h = op.h;
  const int dim = (int)h->H1.dim;
  const auto& xi = magnus::leja_points();
  IterArgs a{};
  if (tab) {
    a.coef = tab->col;
    a.coef_stride = tab->stride;
    a.step = tab->step;
  }
  a.slot = ctx->slots;
  a.partials = ctx->partials;
  a.a1 = P.scale * op.a;
  a.a2 = P.scale * op.b;
  a.kap = P.scale * op.kappa;
  a.sigma = P.scale * P.c + xi[i - 1];
  a.d = make_double2(P.d[i].real(), P.d[i].imag());
  a.d0 = make_double2(P.d[0].real(), P.d[0].imag());
  a.dabs = std::abs(P.d[i]);
  a.d0abs = std::abs(P.d[0]);
  a.tol = tol_sub;
  a.early = early;
  a.first = (i == 1);
  a.check_stop = (i != 1);
  a.iter = i;
  a.wcur = win;
  a.wout = wout;
  a.pacc = pacc;
  if (op.m6c) return m6_csr_iteration(ctx, op, P.scale, a, s);
  if (h->H1.format == MAGNUS_DENSE) {
    if (op.kappa != 0.0) return fail(MAGNUS_EINVAL, "dense commutator exponents run assembled");
    a.x1 = win;
    a.x2 = win;
    const int rpw = dense_rpw(ctx, h);
    const int grid = magnus::dense2_grid(dim, op.assembled ? 1 : 2, rpw);
    if (int rc = setup_stop_test(ctx, P, i, grid, &a, s)) return rc;
    const bool fused = a.fused;
    HIP_TRY(timed(ctx, MAGNUS_KERNEL_DENSE_LEJA, s, [&] {
      if (op.fuse_assembly && i == 1) {
        const magnus::DenseAssembly D{reinterpret_cast<const double2*>(h->H1.val),
                                      reinterpret_cast<const double2*>(h->H2.val),
                                      op.fK,
                                      h->H1.ld,
                                      op.fa,
                                      op.fb,
                                      op.fk,
                                      op.fuse_out};
        return magnus::launch_dense_assemble_iter(D, dim, a, s, rpw);
      }
      if (op.assembled) return magnus::launch_dense2_iter(op.assembled, nullptr, dim, dim, a, s, rpw);
      return magnus::launch_dense2_iter(reinterpret_cast<const double2*>(h->H1.val),
                                        reinterpret_cast<const double2*>(h->H2.val), dim, h->H1.ld, a, s, rpw);
    }));
    if (!fused) HIP_TRY(magnus::launch_leja_decide(a, grid, s));
    return MAGNUS_OK;
  }
  CsrDev t1{h->H1.row_ptr, h->H1.col_idx, reinterpret_cast<const double2*>(h->H1.val)};
  CsrDev t2{h->H2.row_ptr, h->H2.col_idx, reinterpret_cast<const double2*>(h->H2.val)};
  const int rpb = rows_per_block(ctx, h);
  if (op.kappa == 0.0) {
    a.x1 = win;
    a.x2 = win;
    const int grid = magnus::csr2_grid(dim, rpb);
    if (int rc = setup_stop_test(ctx, P, i, grid, &a, s)) return rc;
    const bool fused = a.fused;
    HIP_TRY(timed(ctx, MAGNUS_KERNEL_CSR_LEJA, s,
                  [&] { return magnus::launch_csr2_iter(magnus::kLeja, t1, t2, dim, a, rpb, s); }));
    if (!fused) HIP_TRY(magnus::launch_leja_decide(a, grid, s));
    return MAGNUS_OK;
  }
  if (csr_comm_ready(ctx, h)) {
    // assembled commutator: one pass over H1, H2 and K
    CsrDev t3{ctx->kc_rp, ctx->kc_ci, ctx->kc_val};
    a.x1 = win;
    a.x2 = win;
    const bool streamed = rpb == magnus::kStreamTile;  // the three-term kernel follows the two-term choice
    const int grid = magnus::csr3_grid(dim, streamed);
    if (int rc = setup_stop_test(ctx, P, i, grid, &a, s)) return rc;
    const bool fused = a.fused;
    HIP_TRY(timed(ctx, MAGNUS_KERNEL_CSR_LEJA3, s,
                  [&] { return magnus::launch_csr3_iter(t1, t2, t3, dim, a, P.scale * op.kappa, streamed, s); }));
    if (!fused) HIP_TRY(magnus::launch_leja_decide(a, grid, s));
    return MAGNUS_OK;
  }
  // Commutator exponents take two passes per iteration.  The first pass
  // makes the stop test (fused or not); with the fused test the second pass
  // only reads the verdict the first one recorded, and it writes the
  // partials the next iteration's first pass reduces.
  double2* U = ctx->vec(kU);
  double2* V = ctx->vec(kV);
  const int grid = magnus::csr2_grid(dim, rpb);
  if (int rc = setup_stop_test(ctx, P, i, grid, &a, s)) return rc;
  const bool fused = a.fused;
  IterArgs p1 = a;
  p1.x1 = win;
  p1.x2 = win;
  p1.wout = U;
  p1.pacc = V;
  if (fused) {
    a.fused = 0;
    a.check_stop = 1;
  }
  if (rpb == magnus::kStreamTile) {
    // streamed commutator: pass 1 writes U = a1 w + i k H2 w and V = a2 w - i k H1 w,
    // pass 2 is the two-term iteration on H1 U + H2 V
    HIP_TRY(timed(ctx, MAGNUS_KERNEL_CSR_SPLIT, s,
                  [&] { return magnus::launch_csr2_iter(magnus::kSplitComm, t1, t2, dim, p1, rpb, s); }));
    a.x1 = U;
    a.x2 = V;
    a.a1 = 1.0;
    a.a2 = 1.0;
    a.unit_a = 1;
    HIP_TRY(timed(ctx, MAGNUS_KERNEL_CSR_COMM, s,
                  [&] { return magnus::launch_csr2_iter(magnus::kLeja, t1, t2, dim, a, rpb, s); }));
    if (!fused) HIP_TRY(magnus::launch_leja_decide(a, grid, s));
    return MAGNUS_OK;
  }
  // commutator: pass 1 writes U = H1 w, V = H2 w; pass 2 applies H1 V and H2 U
  HIP_TRY(timed(ctx, MAGNUS_KERNEL_CSR_SPLIT, s,
                [&] { return magnus::launch_csr2_iter(magnus::kSplit, t1, t2, dim, p1, rpb, s); }));
  a.x1 = V;
  a.x2 = U;
  HIP_TRY(timed(ctx, MAGNUS_KERNEL_CSR_COMM, s,
                [&] { return magnus::launch_csr2_iter(magnus::kLejaComm, t1, t2, dim, a, rpb, s); }));
  if (!fused) HIP_TRY(magnus::launch_leja_decide(a, grid, s));
  return MAGNUS_OK;
}

// The launches of one planned exponential: P.lp.s substeps of P.lp.m
// iterations, the Newton sums in kS0/kS1 (or dst), w in kA/kB.  With a table
// (capture of a replayed step) iteration i of substep sub reads record
// tab->col + sub * m + i - 1 of the step.
int enqueue_exponential(magnus_ctx* ctx, const ExpOp& it, const ExpPlan& P, const double2* src, double2* dst,
                        double tol_sub, int early, const TableRef* tab, hipStream_t s) {
  const int64_t dim = it.h->H1.dim;
  const int m = P.lp.m, ns = P.lp.s;
  const double2* cur = src;
  ExpOp op = it;  // a fused assembly happens in the first iteration only
  for (int sub = 0; sub < ns; ++sub) {
    const bool last = (sub == ns - 1);
    double2* Pbuf;
    if (last && dst != cur) Pbuf = dst;
    else Pbuf = (cur == ctx->vec(kS0)) ? ctx->vec(kS1) : ctx->vec(kS0);
    for (int i = 1; i <= m; ++i) {
      const double2* win = (i == 1) ? cur : ((i - 1) % 2 == 1 ? ctx->vec(kA) : ctx->vec(kB));
      double2* wout = (i % 2 == 1) ? ctx->vec(kA) : ctx->vec(kB);
      TableRef t{};
      if (tab) t = TableRef{tab->col + (size_t)sub * m + (i - 1), tab->stride, tab->step};
      int rc = launch_iteration(ctx, op, P, i, win, wout, Pbuf, tol_sub, early, s, tab ? &t : nullptr);
      if (rc) return rc;
      op.fuse_assembly = false;
    }
    cur = Pbuf;
  }
  if (cur != dst) HIP_TRY(magnus::launch_copy(cur, dst, dim, s));
  return MAGNUS_OK;
}

// dst = exp(-i tau (a H1 + b H2 + kappa K)) src for one state.  dst may equal
// src and may be kS2; it must not be another workspace vector.
int run_exponential(magnus_ctx* ctx, const ExpOp& op, double tau, const double2* src, double2* dst,
                    double tol_e, const magnus_leja_opts* o, Acc* acc, hipStream_t s) {
  const int64_t dim = op.h->H1.dim;
  if (tau == 0.0) {
    if (src != dst) HIP_TRY(magnus::launch_copy(src, dst, dim, s));
    acc->exponentials += 1;
    return MAGNUS_OK;
  }
  double lo = op.lo, hi = op.hi;
  if (!op.has_interval)
    magnus::weyl_interval(op.a, op.h->H1.lam_min, op.h->H1.lam_max, op.b, op.h->H2.lam_min, op.h->H2.lam_max,
                          op.kappa, op.h->k_min, op.h->k_max, &lo, &hi);
  ExpPlan P;
  if (!magnus::plan_exponential(tau, lo, hi, tol_e, o->max_degree, o->max_substeps, &P))
    return fail(MAGNUS_ENOCONV, "no degree <= %d with <= %d substeps reaches tol %g (theta %g)",
                o->max_degree, o->max_substeps, tol_e, 0.5 * std::fabs(tau) * 0.5 * (hi - lo));
  const int m = P.lp.m, ns = P.lp.s;
  const double tol_sub = tol_e / (2.0 * ns);
  // Dense terms: assemble the exponent once (48 dim^2 bytes) when that is
  // cheaper than reading both terms in every iteration (16 dim^2 bytes more
  // each), and always for a commutator exponent (K itself is assembled).
  ExpOp it = op;
  if (!op.assembled && op.h->H1.format == MAGNUS_DENSE &&
      (op.kappa != 0.0 || (ctx->assembled_dim >= dim && m * ns >= 4))) {
    if (op.kappa != 0.0 && !dense_comm_ready(ctx, op.h))
      return fail(MAGNUS_EINVAL, "dense commutator exponents need magnus_dense_commutator for this pair of terms");
    if (ctx->assembled_dim < dim) return fail(MAGNUS_ENOMEM, "no assembly buffer (magnus_reserve_dense)");
    it = ExpOp{op.h, 1.0, 0.0, 0.0, ctx->assembled};
    if (ctx->fuse_assembly) {  // assembled by the first iteration as it goes
      it.fuse_assembly = true;
      it.fa = op.a;
      it.fb = op.b;
      it.fk = op.kappa;
      it.fK = op.kappa != 0.0 ? ctx->comm : nullptr;
      it.fuse_out = ctx->assembled;
    } else {
      HIP_TRY(magnus::launch_dense_assemble(reinterpret_cast<const double2*>(op.h->H1.val),
                                            reinterpret_cast<const double2*>(op.h->H2.val), op.h->H1.ld, (int)dim,
                                            op.a, op.b, op.kappa != 0.0 ? ctx->comm : nullptr, op.kappa,
                                            ctx->assembled, s));
    }
  }
  int rc = enqueue_exponential(ctx, it, P, src, dst, tol_sub, o->early_termination, nullptr, s);
  if (rc) return rc;
  acc->exponentials += 1;
  acc->substeps += ns;
  acc->planned += (int64_t)m * ns;
  acc->max_m = std::max(acc->max_m, m);
  acc->max_s = std::max(acc->max_s, ns);
  acc->max_bound = std::max(acc->max_bound, P.lp.bound);
  return MAGNUS_OK;
}

int begin_call(magnus_ctx* ctx, hipStream_t s) {
  HIP_TRY(hipSetDevice(ctx->device));
  ctx->sticky_status = 0;
  ctx->fz_pending = false;
  HIP_TRY(magnus::launch_slot_reset(ctx->slots, ctx->nslots, s));
  return MAGNUS_OK;
}

// Sum of the per-state counters and the union of the status bits.
int read_slots(magnus_ctx* ctx, hipStream_t s, long long* iters, int* status) {
  std::vector<Slot> hs(ctx->nslots);
  HIP_TRY(hipMemcpyAsync(hs.data(), ctx->slots, sizeof(Slot) * hs.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *iters = 0;
  *status = 0;
  for (const Slot& x : hs) {
    *iters += x.iters_total;
    *status |= x.status;
  }
  return MAGNUS_OK;
}

int end_call(magnus_ctx* ctx, const Acc& acc, double tol_e, magnus_stats* st, hipStream_t s) {
  if (int rc = flush_fused_check(ctx, s)) return rc;
  if (!st) return MAGNUS_OK;
  long long iters = 0;
  int status = 0;
  int rc = read_slots(ctx, s, &iters, &status);
  if (rc) return rc;
  st->exponentials = acc.exponentials;
  st->substeps = acc.substeps;
  st->planned_iters = acc.planned;
  st->iters = iters + acc.extra_iters;
  status |= ctx->sticky_status;
  st->hv_products = st->iters * acc.products_per_iter;
  st->max_degree_used = acc.max_m;
  st->max_substeps_used = acc.max_s;
  st->max_err_bound = acc.max_bound;
  st->tol_per_exp = tol_e;
  if (status & 1) return fail(MAGNUS_ENAN, "non-finite vector norm met during the call");
  return MAGNUS_OK;
}

double per_exp_tol(const magnus_leja_opts* o, int64_t exps_per_state) {
  if (o->tol_mode == 1 && exps_per_state > 0) return o->tol / (double)exps_per_state;
  return o->tol;
}

// H2 coefficient of exponential k of a product-of-exponentials step.
double scheme_b(const magnus::Scheme& S, int k, const double* f) {
  double b = 0.0;
  for (int j = 0; j < S.q; ++j) b += S.w[k][j] * f[j];
  return b;
}

// One step of a product-of-exponentials method (Cf4, Cf4:3, M2) on one state,
// f = the step's field samples; the factors act in the order of the scheme
// (for Cf4 the right factor exp(tau(alpha2 A1 + alpha1 A2)) first).
int cf_state(magnus_ctx* ctx, const magnus_hamiltonian* h, const magnus::Scheme& S, double tau, const double* f,
             const double2* in, double2* out, double tol_e, const magnus_leja_opts* o, Acc* acc, hipStream_t s) {
  double2* mids[2] = {ctx->vec(kS2), ctx->vec(kU)};
  const double2* src = in;
  for (int k = 0; k < S.nexp; ++k) {
    double2* dst = (k == S.nexp - 1) ? out : mids[k & 1];
    int rc = run_exponential(ctx, ExpOp{h, S.rho[k], scheme_b(S, k, f), 0.0}, tau, src, dst, tol_e, o, acc, s);
    if (rc) return rc;
    src = dst;
  }
  return MAGNUS_OK;
}

// One step of Method M4 on one state: exp(-i tau (H1 + fbar H2 + kappa K)).
int m4_state(magnus_ctx* ctx, const magnus_hamiltonian* h, double tau, double f1, double f2,
             const double2* in, double2* out, double tol_e, const magnus_leja_opts* o, Acc* acc,
             hipStream_t s) {
  const double fbar = 0.5 * (f1 + f2);
  const double kappa = magnus::kSqrt3 * tau * (f2 - f1) / 12.0;
  return run_exponential(ctx, ExpOp{h, 1.0, fbar, kappa}, tau, in, out, tol_e, o, acc, s);
}

// Whether the context holds the M6 commutators of this pair of dense terms.
bool dense_m6_ready(const magnus_ctx* ctx, const magnus_hamiltonian* h) {
  return ctx->m6_ready && dense_comm_ready(ctx, h);
}

// One step of Method M6 on one state, dense terms.  With A_j = -i(H1 + f_j H2)
// the exponent's B_1 = -i tau Hm (Hm = H1 + f_2 H2) and B_2 = -i b2 H2,
// B_3 = -i b3 H2 with b2 = sqrt(15)/3 tau (f3 - f1), b3 = 10/3 tau (f3 - 2 f2 + f1).
// Expanding the nested commutators of the M6 exponent in H1, H2 makes it a
// linear combination, with step-dependent scalars, of ten fixed Hermitian
// matrices: H1, H2, K = i[H1,H2], P_a = -i[H_a,K], U_ab = i[H_a,P_b]
// (U_12 = U_21 by the Jacobi identity) and R_a = -i[K,P_a].  The step
// assembles -i tau (sum_t c_t M_t) once and runs one Leja exponential on it.
int m6_state(magnus_ctx* ctx, const magnus_hamiltonian* h, double tau, const double* f, const double2* in,
             double2* out, double tol_e, const magnus_leja_opts* o, Acc* acc, hipStream_t s) {
  const int64_t dim = h->H1.dim;
  const double f1 = f[0], f2 = f[1], f3 = f[2];
  const double r15 = 3.8729833462074168852;
  const double b2 = r15 / 3.0 * tau * (f3 - f1);
  const double b3 = 10.0 / 3.0 * tau * (f3 - 2.0 * f2 + f1);
  // coefficients of H1, H2, K, P1, P2, U11, U12, U22, R1, R2 in the exponent / (-i tau)
  const double c[10] = {1.0,
                        f2 + b3 / (12.0 * tau),
                        b2 / 12.0,
                        -tau * b3 / 360.0,
                        (-(2.0 * tau * b3 * f2 / 3.0) - b3 * b3 / 30.0 + b2 * b2) / 240.0,
                        tau * tau * b2 / 720.0,
                        (2.0 * tau * tau * b2 * f2 / 3.0 + tau * b2 * b3 / 60.0) / 240.0,
                        (tau * tau * b2 * f2 * f2 / 3.0 + tau * b2 * b3 * f2 / 60.0) / 240.0,
                        -tau * tau * b2 * b2 / 14400.0,
                        -tau * tau * b2 * b2 * f2 / 14400.0};
  double mlo[10] = {h->H1.lam_min, h->H2.lam_min, h->k_min, ctx->m6_lo[0], ctx->m6_lo[1], ctx->m6_lo[2],
                    ctx->m6_lo[3], ctx->m6_lo[4], ctx->m6_lo[5], ctx->m6_lo[6]};
  double mhi[10] = {h->H1.lam_max, h->H2.lam_max, h->k_max, ctx->m6_hi[0], ctx->m6_hi[1], ctx->m6_hi[2],
                    ctx->m6_hi[3], ctx->m6_hi[4], ctx->m6_hi[5], ctx->m6_hi[6]};
  if (h->H1.format == MAGNUS_CSR) {
    // P_a from their Gershgorin discs; the nested commutators i[A, B] are
    // applied matrix-free, enclosed by +-2 rho(A) rho(B) (rho: the larger end
    // of an enclosure in absolute value)
    auto rho = [](double lo_, double hi_) { return std::fmax(std::fabs(lo_), std::fabs(hi_)); };
    const double rh1 = rho(h->H1.lam_min, h->H1.lam_max), rh2 = rho(h->H2.lam_min, h->H2.lam_max);
    const double rk = rho(h->k_min, h->k_max);
    const double rp1 = rho(ctx->pm_lo[0], ctx->pm_hi[0]), rp2 = rho(ctx->pm_lo[1], ctx->pm_hi[1]);
    const double nested[5] = {2 * rh1 * rp1, 2 * rh1 * rp2, 2 * rh2 * rp2, 2 * rk * rp1, 2 * rk * rp2};
    mlo[3] = ctx->pm_lo[0];
    mhi[3] = ctx->pm_hi[0];
    mlo[4] = ctx->pm_lo[1];
    mhi[4] = ctx->pm_hi[1];
    for (int t = 0; t < 5; ++t) {
      mlo[5 + t] = -nested[t];
      mhi[5 + t] = nested[t];
    }
  }
  // Weyl: the spectrum of a sum of Hermitian matrices lies in the sum of their enclosures
  double lo = 0.0, hi = 0.0;
  for (int t = 0; t < 10; ++t) {
    lo += std::fmin(c[t] * mlo[t], c[t] * mhi[t]);
    hi += std::fmax(c[t] * mlo[t], c[t] * mhi[t]);
  }
  if (h->H1.format == MAGNUS_CSR) {
    ExpOp op{h, 0.0, 0.0, 0.0};
    op.has_interval = true;
    op.lo = lo;
    op.hi = hi;
    op.m6c = c;
    return run_exponential(ctx, op, tau, in, out, tol_e, o, acc, s);
  }
  magnus::AssembleTerms T{};
  T.nterms = 10;
  for (int t = 0; t < 10; ++t) {
    T.c[t] = c[t];
    if (t < 2) {
      T.m[t] = reinterpret_cast<const double2*>(t == 0 ? h->H1.val : h->H2.val);
      T.ld[t] = h->H1.ld;
    } else {
      T.m[t] = t == 2 ? ctx->comm : ctx->m6 + (size_t)(t - 3) * (size_t)ctx->m6_dim * (size_t)ctx->m6_dim;
      T.ld[t] = dim;
    }
  }
  if (ctx->assembled_dim < dim) return fail(MAGNUS_ENOMEM, "no assembly buffer (magnus_reserve_dense)");
  HIP_TRY(magnus::launch_assemble_terms(T, (int)dim, ctx->assembled, s));
  ExpOp op{h, 1.0, 0.0, 0.0, ctx->assembled};
  op.has_interval = true;
  op.lo = lo;
  op.hi = hi;
  return run_exponential(ctx, op, tau, in, out, tol_e, o, acc, s);
}

// ---------------------------------------------------------------------------
// Several states per iteration (interleaved workspace, one CSR pass for all).
// ---------------------------------------------------------------------------

// One exponential of a group of B states: exp(-i tau (a_b H1 + b_b H2)) for
// state b.  All states share the substep count s and run max_b m_b
// iterations; a state whose own degree m_b is smaller gets d_i = 0 beyond it.
struct MultiExp {
  int B = 0, s = 1, m = 1;
  int dense_terms = 0;           // dense: 1 (assembled, with acoef/bcoef below) or 2
  double ca = 0.0, cb = 0.0;     // coefficients of the assembled exponent
  size_t table_off = 0;          // first ColParam of this exponential ([i-1][b])
  double tau = 0.0;
  int frechet = 0;               // block vector of [[H, H2], [0, H]] (B == 2)
  const double2* src = nullptr;  // interleaved, dim * B
  double2* dst = nullptr;
};

int plan_multi(const magnus_hamiltonian* h, const double* acoef, const double* bcoef, int B, double tau,
               double tol_e, const magnus_leja_opts* o, int frechet, std::vector<ColParam>* table,
               MultiExp* out, Acc* acc, bool assembled = false) {
  std::vector<double> lo(B), hi(B);
  int s = 1;
  for (int b = 0; b < B; ++b) {
    magnus::weyl_interval(acoef[b], h->H1.lam_min, h->H1.lam_max, bcoef[b], h->H2.lam_min, h->H2.lam_max, 0.0, 0.0,
                          0.0, &lo[b], &hi[b]);
    ExpPlan t;
    if (!magnus::plan_exponential(tau, lo[b], hi[b], tol_e, o->max_degree, o->max_substeps, &t))
      return fail(MAGNUS_ENOCONV, "no degree <= %d with <= %d substeps reaches tol %g", o->max_degree,
                  o->max_substeps, tol_e);
    s = std::max(s, t.lp.s);
  }
  std::vector<ExpPlan> P(B);
  int m = 1;
  double worst = 0.0;
  for (int b = 0; b < B; ++b) {
    const double coupling =
        frechet ? std::fmax(std::fabs(h->H2.lam_min), std::fabs(h->H2.lam_max)) : 0.0;
    if (!magnus::plan_exponential_fixed_s(tau, lo[b], hi[b], tol_e, s, o->max_degree, &P[b], coupling))
      return fail(MAGNUS_ENOCONV, "no degree <= %d reaches tol %g with %d substeps", o->max_degree, tol_e, s);
    m = std::max(m, P[b].lp.m);
    worst = std::max(worst, P[b].lp.bound);
  }
  const auto& xi = magnus::leja_points();
  out->B = B;
  out->s = s;
  out->m = m;
  out->tau = tau;
  out->frechet = frechet;
  out->table_off = table->size();
  for (int i = 1; i <= m; ++i)
    for (int b = 0; b < B; ++b) {
      const ExpPlan& p = P[b];
      ColParam c{};
      c.a1 = assembled ? p.scale : p.scale * acoef[b];
      c.a2 = assembled ? 0.0 : p.scale * bcoef[b];
      c.sigma = p.scale * p.c + xi[i - 1];
      const std::complex<double> d = i <= p.lp.m ? p.d[i] : std::complex<double>(0.0, 0.0);
      c.dre = d.real();
      c.dim = d.imag();
      c.dabs = std::abs(d);
      c.d0re = p.d[0].real();
      c.d0im = p.d[0].imag();
      c.d0abs = std::abs(p.d[0]);
      c.coup = frechet ? p.scale : 0.0;
      table->push_back(c);
    }
  acc->exponentials += B;
  acc->substeps += (int64_t)s * B;
  acc->planned += (int64_t)m * s * B;
  acc->max_m = std::max(acc->max_m, m);
  acc->max_s = std::max(acc->max_s, s);
  acc->max_bound = std::max(acc->max_bound, worst);
  return MAGNUS_OK;
}

int upload_table(magnus_ctx* ctx, const std::vector<ColParam>& table, hipStream_t s) {
  if (table.empty()) return MAGNUS_OK;
  if (table.size() > kTableCap) return fail(MAGNUS_ENOMEM, "parameter table of %zu entries exceeds %zu", table.size(), kTableCap);
  HIP_TRY(hipMemcpyAsync(ctx->table, table.data(), sizeof(ColParam) * table.size(), hipMemcpyHostToDevice, s));
  return MAGNUS_OK;
}

// Launch the iterations of one planned multi-state exponential.
int launch_multi(magnus_ctx* ctx, const magnus_hamiltonian* h, const MultiExp& E, double tol_e, int early,
                 hipStream_t s) {
  if (int rc = flush_fused_check(ctx, s)) return rc;
  const int dim = (int)h->H1.dim;
  const int B = E.B;
  const size_t n = (size_t)dim * B;
  CsrDev t1{h->H1.row_ptr, h->H1.col_idx, reinterpret_cast<const double2*>(h->H1.val)};
  CsrDev t2{h->H2.row_ptr, h->H2.col_idx, reinterpret_cast<const double2*>(h->H2.val)};
  const bool dense = h->H1.format == MAGNUS_DENSE;
  const int grid = dense ? (E.frechet ? magnus::dense_frechet_grid(dim) : magnus::dense_mfma_row_blocks(dim))
                         : magnus::csr2_multi_grid(dim, B);
  const int mode = E.frechet ? magnus::kMultiFrechet : magnus::kMultiLeja;
  if (grid <= 0 || (size_t)grid * (size_t)B * 2 > ctx->npartials)
    return fail(MAGNUS_ENOMEM, "per-workgroup partial sums (%d x %d) exceed the context's buffer", grid, B);
  const double2* D1 = reinterpret_cast<const double2*>(h->H1.val);
  const double2* D2 = reinterpret_cast<const double2*>(h->H2.val);
  long long ldd = h->H1.ld;
  if (dense && E.dense_terms == 1) {
    HIP_TRY(magnus::launch_dense_assemble(D1, D2, h->H1.ld, dim, E.ca, E.cb, nullptr, 0.0, ctx->assembled, s));
    D1 = ctx->assembled;
    ldd = dim;
  }
  const double tol_sub = tol_e / (2.0 * E.s);
  const double2* cur = E.src;
  for (int sub = 0; sub < E.s; ++sub) {
    const bool last = (sub == E.s - 1);
    double2* Pbuf;
    if (last && E.dst != cur) Pbuf = E.dst;
    else Pbuf = (cur == ctx->vec(kS0)) ? ctx->vec(kS1) : ctx->vec(kS0);
    for (int i = 1; i <= E.m; ++i) {
      MultiArgs a{};
      a.x = (i == 1) ? cur : ((i - 1) % 2 == 1 ? ctx->vec(kA) : ctx->vec(kB));
      a.wout = (i % 2 == 1) ? ctx->vec(kA) : ctx->vec(kB);
      a.pacc = Pbuf;
      a.slots = ctx->slots;
      a.partials = ctx->partials;
      a.prm = ctx->table + E.table_off + (size_t)(i - 1) * B;
      a.B = B;
      a.first = (i == 1);
      a.check_stop = (i != 1);
      a.early = early;
      a.tol = tol_sub;
      a.joint = E.frechet;
      if (dense && E.frechet)
        HIP_TRY(timed(ctx, MAGNUS_KERNEL_DENSE_LEJA, s,
                      [&] { return magnus::launch_dense_frechet(D1, D2, dim, h->H1.ld, a, s); }));
      else if (dense)
        HIP_TRY(timed(ctx, MAGNUS_KERNEL_DENSE_MFMA, s,
                      [&] { return magnus::launch_dense_mfma(E.dense_terms, D1, D2, ldd, dim, a, s, mfma_tile(ctx, h, B)); }));
      else
        HIP_TRY(timed(ctx, MAGNUS_KERNEL_CSR_MULTI, s, [&] { return magnus::launch_csr2_multi(mode, t1, t2, dim, a, s); }));
      HIP_TRY(magnus::launch_multi_decide(a, grid, s));
    }
    cur = Pbuf;
  }
  if (cur != E.dst) HIP_TRY(magnus::launch_copy(cur, E.dst, (long long)n, s));
  return MAGNUS_OK;
}

// Largest supported group size for the remaining states.
int group_size(int remaining, int cap = 32) {
  for (int g : {32, 16, 8, 4, 2})
    if (g <= cap && remaining >= g) return g;
  return 1;
}

bool multi_ok(const magnus_hamiltonian* h, double kappa) { return kappa == 0.0; }

// Dense groups take every remaining state at once; CSR groups 32, 16, 8, 4, 2
// (at most the autotuned group size).
int group_for(magnus_ctx* ctx, const magnus_hamiltonian* h, int remaining) {
  if (h->H1.format == MAGNUS_DENSE) return remaining > 1 ? remaining : 1;
  auto it = ctx->tuned_group.find({(const void*)h->H1.row_ptr, h->H1.dim});
  return group_size(remaining, it == ctx->tuned_group.end() ? 32 : it->second);
}

// Plan one group exponential, assembling the dense exponent when all states share it.
int plan_group(magnus_ctx* ctx, const magnus_hamiltonian* h, const double* acoef, const double* bcoef, int B,
               double tau, double tol_e, const magnus_leja_opts* o, std::vector<ColParam>* table, MultiExp* E,
               Acc* acc) {
  bool shared = true;
  for (int b = 1; b < B; ++b) shared = shared && acoef[b] == acoef[0] && bcoef[b] == bcoef[0];
  const bool dense = h->H1.format == MAGNUS_DENSE;
  const bool assemble = dense && shared && ctx->assembled && ctx->assembled_dim >= h->H1.dim;
  int rc = plan_multi(h, acoef, bcoef, B, tau, tol_e, o, 0, table, E, acc, assemble);
  if (rc) return rc;
  E->dense_terms = dense ? (assemble ? 1 : 2) : 0;
  E->ca = acoef[0];
  E->cb = bcoef[0];
  return MAGNUS_OK;
}

// dst[c] = exp(-i tau (a H1 + b_c H2)) src[c] for the states c0..c0+B-1
// (b-major caller layout in and out).
int multi_expmv_group(magnus_ctx* ctx, const magnus_hamiltonian* h, int B, const double* acoef,
                      const double* bcoef, double tau, const double2* src, double2* dst, double tol_e,
                      const magnus_leja_opts* o, Acc* acc, hipStream_t s) {
  const int dim = (int)h->H1.dim;
  double2* Y = ctx->vec(kY);
  HIP_TRY(magnus::launch_pack(src, Y, dim, B, s));
  std::vector<ColParam> table;
  MultiExp E;
  int rc = plan_group(ctx, h, acoef, bcoef, B, tau, tol_e, o, &table, &E, acc);
  if (rc) return rc;
  if ((rc = upload_table(ctx, table, s))) return rc;
  E.src = Y;
  E.dst = Y;
  if ((rc = launch_multi(ctx, h, E, tol_e, o->early_termination, s))) return rc;
  HIP_TRY(magnus::launch_unpack(Y, dst, dim, B, s));
  return MAGNUS_OK;
}

// Product-of-exponentials steps for a group of B states held interleaved in
// kY, f values per state: fn(c, n, j) = f(t_n + c_j tau) of state c.
template <class F>
int multi_cf_steps(magnus_ctx* ctx, const magnus_hamiltonian* h, const magnus::Scheme& S, int B, double tau,
                   int64_t n0, int64_t n1, F fn, double tol_e, const magnus_leja_opts* o, Acc* acc,
                   hipStream_t s) {
  double2* Y = ctx->vec(kY);
  double2* mids[2] = {ctx->vec(kS2), ctx->vec(kU)};
  std::vector<double> av(B), bv(B), fv(S.q);
  // steps are planned and uploaded in segments that fit the parameter table
  int64_t n = n0;
  while (n < n1) {
    std::vector<ColParam> table;
    std::vector<MultiExp> exps;
    int64_t k = n;
    for (; k < n1; ++k) {
      const size_t mark = table.size();
      Acc trial = *acc;
      std::vector<MultiExp> step(S.nexp);
      const double2* src = Y;
      for (int e = 0; e < S.nexp; ++e) {
        for (int c = 0; c < B; ++c) {
          for (int j = 0; j < S.q; ++j) fv[j] = fn(c, k, j);
          av[c] = S.rho[e];
          bv[c] = scheme_b(S, e, fv.data());
        }
        int rc = plan_group(ctx, h, av.data(), bv.data(), B, tau, tol_e, o, &table, &step[e], &trial);
        if (rc) return rc;
        step[e].src = src;
        step[e].dst = (e == S.nexp - 1) ? Y : mids[e & 1];
        src = step[e].dst;
      }
      if (table.size() > kTableCap) {
        if (k == n) return fail(MAGNUS_ENOMEM, "one step needs more than the parameter table holds");
        table.resize(mark);
        break;
      }
      *acc = trial;
      for (const MultiExp& E : step) exps.push_back(E);
    }
    int rc = upload_table(ctx, table, s);
    if (rc) return rc;
    for (const MultiExp& E : exps)
      if ((rc = launch_multi(ctx, h, E, tol_e, o->early_termination, s))) return rc;
    n = k;
  }
  return MAGNUS_OK;
}

// ---------------------------------------------------------------------------
// Ragged batches: the large problems of equal group size B advance together,
// one launch per Leja iteration serving every problem (and one decision
// launch for all their columns), each problem with its own terms, degrees,
// workspace slice, control slots and partial sums.
// ---------------------------------------------------------------------------
struct RagProblem {
  const magnus_problem* P;
  int c0;         // first of its states in the problem (a group of B states)
  size_t voff;    // offset of its slice inside every workspace vector
  int slot0;      // its first control slot
  size_t poff;    // offset of its partial sums
  double2* v(magnus_ctx* ctx, int k) const { return ctx->vec(k) + voff; }
  double2* psi() const { return reinterpret_cast<double2*>(P->psi) + (size_t)c0 * P->h.H1.dim; }
};

// One exponential of every problem (E[q] planned for problem q).
int launch_ragged_exp(magnus_ctx* ctx, const std::vector<RagProblem>& R, const std::vector<MultiExp>& E, int B,
                      double tol_e, int early, hipStream_t s) {
  if (int rc = flush_fused_check(ctx, s)) return rc;
  const size_t np = R.size();
  std::vector<const double2*> cur(np);
  std::vector<double2*> pbuf(np);
  int max_s = 1;
  for (size_t q = 0; q < np; ++q) {
    cur[q] = E[q].src;
    max_s = std::max(max_s, E[q].s);
  }
  for (int sub = 0; sub < max_s; ++sub) {
    int max_m = 0;
    for (size_t q = 0; q < np; ++q) {
      if (sub >= E[q].s) continue;
      const bool last = sub == E[q].s - 1;
      if (last && E[q].dst != cur[q]) pbuf[q] = E[q].dst;
      else pbuf[q] = cur[q] == R[q].v(ctx, kS0) ? R[q].v(ctx, kS1) : R[q].v(ctx, kS0);
      max_m = std::max(max_m, E[q].m);
    }
    for (int i = 1; i <= max_m; ++i) {
      magnus::RaggedArgs r{};
      for (size_t q = 0; q < np; ++q) {
        if (sub >= E[q].s || i > E[q].m) continue;
        const magnus_hamiltonian& h = R[q].P->h;
        magnus::RaggedProblem& rp = r.p[r.np++];
        rp.t1 = CsrDev{h.H1.row_ptr, h.H1.col_idx, reinterpret_cast<const double2*>(h.H1.val)};
        rp.t2 = CsrDev{h.H2.row_ptr, h.H2.col_idx, reinterpret_cast<const double2*>(h.H2.val)};
        rp.dim = (int)h.H1.dim;
        MultiArgs& a = rp.a;
        a.x = (i == 1) ? cur[q] : ((i - 1) % 2 == 1 ? R[q].v(ctx, kA) : R[q].v(ctx, kB));
        a.wout = (i % 2 == 1) ? R[q].v(ctx, kA) : R[q].v(ctx, kB);
        a.pacc = pbuf[q];
        a.slots = ctx->slots + R[q].slot0;
        a.partials = ctx->partials + R[q].poff;
        a.prm = ctx->table + E[q].table_off + (size_t)(i - 1) * B;
        a.B = B;
        a.first = (i == 1);
        a.check_stop = (i != 1);
        a.early = early;
        a.tol = tol_e / (2.0 * E[q].s);
        a.joint = 0;
      }
      HIP_TRY(timed(ctx, MAGNUS_KERNEL_CSR_MULTI, s, [&] { return magnus::launch_csr2_ragged(r, B, s); }));
    }
    for (size_t q = 0; q < np; ++q)
      if (sub < E[q].s) cur[q] = pbuf[q];
  }
  for (size_t q = 0; q < np; ++q)
    if (cur[q] != E[q].dst)
      HIP_TRY(magnus::launch_copy(cur[q], E[q].dst, (long long)R[q].P->h.H1.dim * B, s));
  return MAGNUS_OK;
}

// Product-of-exponentials steps of the ragged batch's large problems (all of
// batch B, B a group size), packed interleaved into their workspace slices.
int ragged_joint_steps(magnus_ctx* ctx, std::vector<RagProblem>& R, const magnus::Scheme& S, int B, double tau,
                       int64_t nsteps, double tol_e, const magnus_leja_opts* o, Acc* acc, hipStream_t s) {
  for (const RagProblem& q : R) HIP_TRY(magnus::launch_pack(q.psi(), q.v(ctx, kY), (int)q.P->h.H1.dim, B, s));
  std::vector<double> av(B), bv(B), fv(S.q);
  int64_t n = 0;
  while (n < nsteps) {
    std::vector<ColParam> table;
    std::vector<std::vector<MultiExp>> steps;  // [step * nexp + e][problem]
    int64_t k = n;
    for (; k < nsteps; ++k) {
      const size_t mark = table.size();
      Acc trial = *acc;
      std::vector<std::vector<MultiExp>> st(S.nexp, std::vector<MultiExp>(R.size()));
      for (size_t q = 0; q < R.size(); ++q) {
        const magnus_problem& P = *R[q].P;
        const double2* src = R[q].v(ctx, kY);
        double2* mids[2] = {R[q].v(ctx, kS2), R[q].v(ctx, kU)};
        for (int e = 0; e < S.nexp; ++e) {
          for (int c = 0; c < B; ++c) {
            const double* f = P.f_nodes + ((P.batch_f == 1 ? 0 : (int64_t)(R[q].c0 + c)) * nsteps + k) * S.q;
            for (int j = 0; j < S.q; ++j) fv[j] = f[j];
            av[c] = S.rho[e];
            bv[c] = scheme_b(S, e, fv.data());
          }
          MultiExp& E = st[e][q];
          int rc = plan_multi(&P.h, av.data(), bv.data(), B, tau, tol_e, o, 0, &table, &E, &trial);
          if (rc) return rc;
          E.src = src;
          E.dst = (e == S.nexp - 1) ? R[q].v(ctx, kY) : mids[e & 1];
          src = E.dst;
        }
      }
      if (table.size() > kTableCap) {
        if (k == n) return fail(MAGNUS_ENOMEM, "one step needs more than the parameter table holds");
        table.resize(mark);
        break;
      }
      *acc = trial;
      for (auto& e : st) steps.push_back(std::move(e));
    }
    int rc = upload_table(ctx, table, s);
    if (rc) return rc;
    for (const auto& E : steps)
      if ((rc = launch_ragged_exp(ctx, R, E, B, tol_e, o->early_termination, s))) return rc;
    n = k;
  }
  for (const RagProblem& q : R) HIP_TRY(magnus::launch_unpack(q.v(ctx, kY), q.psi(), (int)q.P->h.H1.dim, B, s));
  return MAGNUS_OK;
}

// ---------------------------------------------------------------------------
// Whole Cf4 propagations of small states, one workgroup per state.
// ---------------------------------------------------------------------------
struct SmallState {
  int prob;
  double2* psi;
  const double* fn;  // this state's field samples, [nsteps][q]
};

// One workgroup's iteration time grows with the dimension, while the
// per-iteration grid launches of the other paths cost about the same for any
// dimension up to a few thousand rows; the persistent launch pays off when its
// states are small or many.  Measured crossover (MI355X, Cf4 on spin chains,
// state-steps/s persistent vs grid): 1024 rows win from one state on; 2048
// rows lose at one state (5.1k vs 7.5k) and win at four (19k vs 14k); 4096
// rows lose up to 16 states (38k vs 40k) and win at 64 (151k vs 59k).
int64_t small_cap(const magnus_ctx* ctx, int64_t nstates) {
  if (ctx->persist == 0) return 0;
  if (ctx->persist >= 2 || nstates >= 32) return kSmallDim;
  return nstates >= 4 ? 2048 : 1024;
}

bool small_candidate(const magnus_hamiltonian* h) { return h->H1.format == MAGNUS_CSR && h->H1.dim <= kSmallDim; }

bool small_ok(magnus_ctx* ctx, const magnus_hamiltonian* h, int64_t nstates) {
  return small_candidate(h) && h->H1.dim <= small_cap(ctx, nstates);
}

// Steps n0..n1-1 of every state in one launch.
int persist_segment(magnus_ctx* ctx, const std::vector<const magnus_hamiltonian*>& hs,
                    const std::vector<SmallState>& st, const magnus::Scheme& S, double tau, int64_t n0, int64_t n1,
                    double tol_e, const magnus_leja_opts* o, Acc* acc, hipStream_t s) {
  if (int rc = flush_fused_check(ctx, s)) return rc;
  const int nst = (int)st.size();
  const int nexp = (int)(S.nexp * (n1 - n0));
  if (nst > ctx->nslots) return fail(MAGNUS_ENOMEM, "%d small states exceed %d control slots", nst, ctx->nslots);
  int64_t maxdim = 1;
  for (auto* h : hs) maxdim = std::max<int64_t>(maxdim, h->H1.dim);
  if (maxdim > magnus::kPersistMaxDim) return fail(MAGNUS_EINVAL, "dimension %lld too large for the small-state kernel", (long long)maxdim);
  std::vector<ColParam> table;
  std::vector<PersistExp> exps((size_t)nst * nexp);
  const auto& xi = magnus::leja_points();
  for (int b = 0; b < nst; ++b) {
    const magnus_hamiltonian* h = hs[st[b].prob];
    for (int64_t n = n0; n < n1; ++n) {
      const double* f = st[b].fn + S.q * n;
      for (int half = 0; half < S.nexp; ++half) {
        const double rho = S.rho[half], coef = scheme_b(S, half, f);
        double lo, hi;
        magnus::weyl_interval(rho, h->H1.lam_min, h->H1.lam_max, coef, h->H2.lam_min, h->H2.lam_max, 0.0, 0.0, 0.0,
                              &lo, &hi);
        ExpPlan P;
        if (!magnus::plan_exponential(tau, lo, hi, tol_e, o->max_degree, o->max_substeps, &P))
          return fail(MAGNUS_ENOCONV, "no degree <= %d with <= %d substeps reaches tol %g", o->max_degree,
                      o->max_substeps, tol_e);
        PersistExp& E = exps[(size_t)b * nexp + S.nexp * (n - n0) + half];
        E.m = P.lp.m;
        E.s = P.lp.s;
        E.table_off = (long long)table.size();
        E.tol_sub = tol_e / (2.0 * P.lp.s);
        for (int i = 1; i <= P.lp.m; ++i) {
          ColParam c{};
          c.a1 = P.scale * rho;
          c.a2 = P.scale * coef;
          c.sigma = P.scale * P.c + xi[i - 1];
          c.dre = P.d[i].real();
          c.dim = P.d[i].imag();
          c.dabs = std::abs(P.d[i]);
          c.d0re = P.d[0].real();
          c.d0im = P.d[0].imag();
          c.d0abs = std::abs(P.d[0]);
          table.push_back(c);
        }
        acc->exponentials += 1;
        acc->substeps += P.lp.s;
        acc->planned += (int64_t)P.lp.m * P.lp.s;
        acc->max_m = std::max(acc->max_m, P.lp.m);
        acc->max_s = std::max(acc->max_s, P.lp.s);
        acc->max_bound = std::max(acc->max_bound, P.lp.bound);
      }
    }
  }
  if (table.size() > kTableCap) return fail(MAGNUS_ENOMEM, "parameter table overflow");
  // headers: problems | state_prob | state pointers | exponentials
  std::vector<PersistProblem> probs(hs.size());
  for (size_t i = 0; i < hs.size(); ++i) {
    const magnus_hamiltonian* h = hs[i];
    probs[i].t1 = CsrDev{h->H1.row_ptr, h->H1.col_idx, reinterpret_cast<const double2*>(h->H1.val)};
    probs[i].t2 = CsrDev{h->H2.row_ptr, h->H2.col_idx, reinterpret_cast<const double2*>(h->H2.val)};
    probs[i].dim = (int)h->H1.dim;
  }
  std::vector<int> sp(nst);
  std::vector<double2*> ptrs(nst);
  for (int b = 0; b < nst; ++b) {
    sp[b] = st[b].prob;
    ptrs[b] = st[b].psi;
  }
  auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t o_prob = 0;
  const size_t o_sp = align(o_prob + sizeof(PersistProblem) * probs.size());
  const size_t o_ptr = align(o_sp + sizeof(int) * sp.size());
  const size_t o_exp = align(o_ptr + sizeof(double2*) * ptrs.size());
  const size_t total = o_exp + sizeof(PersistExp) * exps.size();
  if (total > kArenaBytes) return fail(MAGNUS_ENOMEM, "call headers of %zu bytes exceed the arena", total);
  std::vector<unsigned char> host(total);
  memcpy(host.data() + o_prob, probs.data(), sizeof(PersistProblem) * probs.size());
  memcpy(host.data() + o_sp, sp.data(), sizeof(int) * sp.size());
  memcpy(host.data() + o_ptr, ptrs.data(), sizeof(double2*) * ptrs.size());
  memcpy(host.data() + o_exp, exps.data(), sizeof(PersistExp) * exps.size());
  HIP_TRY(hipMemcpyAsync(ctx->arena, host.data(), total, hipMemcpyHostToDevice, s));
  int rc = upload_table(ctx, table, s);
  if (rc) return rc;
  PersistArgs a{};
  a.probs = reinterpret_cast<const PersistProblem*>(ctx->arena + o_prob);
  a.state_prob = reinterpret_cast<const int*>(ctx->arena + o_sp);
  a.state = reinterpret_cast<double2* const*>(ctx->arena + o_ptr);
  a.table = ctx->table;
  a.exps = reinterpret_cast<const PersistExp*>(ctx->arena + o_exp);
  a.nexp = nexp;
  a.slots = ctx->slots;
  a.early = o->early_termination;
  // term 1 in LDS: one workgroup per CU then, so only while the states fit the chip
  a.cache1 = ctx->persist_cache && maxdim <= 1024 && nst <= 256;
  for (const magnus_hamiltonian* h : hs) a.cache1 = a.cache1 && h->H1.nnz <= magnus::kPersistCache;
  HIP_TRY(timed(ctx, MAGNUS_KERNEL_PERSIST, s, [&] { return magnus::launch_persist_propagate(a, nst, (int)maxdim, s); }));
  return MAGNUS_OK;
}

// All steps of a set of small-state problems, split into segments whose
// tables fit (and at the given stop points).
int persist_steps(magnus_ctx* ctx, const std::vector<const magnus_hamiltonian*>& hs,
                  const std::vector<SmallState>& st, const magnus::Scheme& S, double tau, int64_t n0, int64_t n1,
                  double tol_e, const magnus_leja_opts* o, Acc* acc, hipStream_t s) {
  const int64_t per_step = (int64_t)st.size() * S.nexp * std::max(1, o->max_degree) * 2;
  int64_t L = std::max<int64_t>(1, (int64_t)kTableCap / std::max<int64_t>(per_step, 1));
  L = std::min<int64_t>(L, (int64_t)(kArenaBytes / 2) / ((int64_t)sizeof(PersistExp) * S.nexp * (int64_t)st.size() + 1));
  L = std::max<int64_t>(L, 1);
  for (int64_t n = n0; n < n1; n += L) {
    int rc = persist_segment(ctx, hs, st, S, tau, n, std::min(n1, n + L), tol_e, o, acc, s);
    if (rc) return rc;
  }
  return MAGNUS_OK;
}

// Plan of one exponential of a replayed step with s substeps: the plan the
// launch-by-launch path makes when it chooses s itself, else the smallest
// degree for s substeps.
bool graph_step_plan(double tau, double lo, double hi, double tol_e, int s, const magnus_leja_opts* o, ExpPlan* P) {
  if (magnus::plan_exponential(tau, lo, hi, tol_e, o->max_degree, o->max_substeps, P) && P->lp.s == s) return true;
  return magnus::plan_exponential_fixed_s(tau, lo, hi, tol_e, s, o->max_degree, P);
}

// ---------------------------------------------------------------------------
// Graph replay of a single CSR state's steps.  The launches of one Magnus step
// (every exponential's substeps and iterations, with the stop tests fused)
// are captured once per call and replayed once per step; each launch reads
// its Leja coefficients from a device table column indexed by a step counter
// that the graph advances at its end.  Every step has the same launch
// structure: per exponential k the largest substep count s_k and degree m_k
// over the call's steps, iterations past a step's own degree inactive.
// ---------------------------------------------------------------------------
struct GraphPlan {
  int nexp = 0;
  std::vector<int> s, m;    // per exponential
  std::vector<int> off;     // first record of exponential k in a step
  int stride = 0;           // records per step
  std::vector<double> lo, hi;  // enclosure of exponential k of step n at [n * nexp + k]
  std::vector<ExpOp> ops;      // exponent of exponential k of step n
};

// Records of the graph's step table that fit the context's table memory.
int64_t graph_table_cap(const magnus_ctx*) {
  return (int64_t)(kTableCap * sizeof(ColParam) / sizeof(magnus::IterCoef));
}

// Whether every iteration launch of this state's exponentials makes its own
// stop test (the condition for capturing a step: no decide kernels).
bool graph_eligible(magnus_ctx* ctx, const magnus_hamiltonian* h, const magnus::Scheme& S) {
  if (!ctx->graph || !ctx->fuse || ctx->timing || h->H1.format != MAGNUS_CSR || S.sixth) return false;
  const int dim = (int)h->H1.dim;
  const int rpb = rows_per_block(ctx, h);
  int grid = magnus::csr2_grid(dim, rpb);
  if (S.commutator && csr_comm_ready(ctx, h)) grid = magnus::csr3_grid(dim, rpb == magnus::kStreamTile);
  return grid <= magnus::kFuseMaxGrid;
}

template <class F>
int graph_plan(magnus_ctx* ctx, const magnus_hamiltonian* h, const magnus::Scheme& S, double tau, int64_t nsteps,
               F fval, double tol_e, const magnus_leja_opts* o, GraphPlan* G) {
  G->nexp = S.commutator ? 1 : S.nexp;
  const int ne = G->nexp;
  G->s.assign(ne, 1);
  G->m.assign(ne, 1);
  G->lo.resize((size_t)nsteps * ne);
  G->hi.resize((size_t)nsteps * ne);
  G->ops.resize((size_t)nsteps * ne);
  for (int64_t n = 0; n < nsteps; ++n) {
    double f[3] = {0, 0, 0};
    for (int j = 0; j < S.q; ++j) f[j] = fval(n, j);
    for (int k = 0; k < ne; ++k) {
      ExpOp op;
      if (S.commutator) {
        op = ExpOp{h, 1.0, 0.5 * (f[0] + f[1]), magnus::kSqrt3 * tau * (f[1] - f[0]) / 12.0};
      } else {
        op = ExpOp{h, S.rho[k], scheme_b(S, k, f), 0.0};
      }
      double lo, hi;
      magnus::weyl_interval(op.a, h->H1.lam_min, h->H1.lam_max, op.b, h->H2.lam_min, h->H2.lam_max, op.kappa,
                            h->k_min, h->k_max, &lo, &hi);
      ExpPlan P;
      if (!magnus::plan_exponential(tau, lo, hi, tol_e, o->max_degree, o->max_substeps, &P))
        return fail(MAGNUS_ENOCONV, "no degree <= %d with <= %d substeps reaches tol %g", o->max_degree,
                    o->max_substeps, tol_e);
      G->s[k] = std::max(G->s[k], P.lp.s);
      const size_t q = (size_t)n * ne + k;
      G->ops[q] = op;
      G->lo[q] = lo;
      G->hi[q] = hi;
    }
  }
  for (int64_t n = 0; n < nsteps; ++n)
    for (int k = 0; k < ne; ++k) {
      ExpPlan P;
      const size_t q = (size_t)n * ne + k;
      if (!graph_step_plan(tau, G->lo[q], G->hi[q], tol_e, G->s[k], o, &P))
        return fail(MAGNUS_ENOCONV, "no degree <= %d reaches tol %g with %d substeps", o->max_degree, tol_e, G->s[k]);
      G->m[k] = std::max(G->m[k], P.lp.m);
    }
  G->off.assign(ne, 0);
  G->stride = 0;
  for (int k = 0; k < ne; ++k) {
    G->off[k] = G->stride;
    G->stride += G->s[k] * G->m[k];
  }
  if (G->stride > graph_table_cap(ctx)) return fail(MAGNUS_ENOMEM, "step table too large for graph replay");
  return MAGNUS_OK;
}

// Coefficient records of steps [n0, n1) in the layout a captured step reads
// (record off[k] + sub * m[k] + i - 1 of each step).
int graph_fill(const GraphPlan& G, double tau, int64_t n0, int64_t n1, double tol_e, const magnus_leja_opts* o,
               Acc* acc, std::vector<magnus::IterCoef>* out) {
  const auto& xi = magnus::leja_points();
  const int ne = G.nexp;
  out->assign((size_t)(n1 - n0) * G.stride, magnus::IterCoef{});
  for (int64_t n = n0; n < n1; ++n)
    for (int k = 0; k < ne; ++k) {
      const size_t q = (size_t)n * ne + k;
      ExpPlan P;
      if (!graph_step_plan(tau, G.lo[q], G.hi[q], tol_e, G.s[k], o, &P))
        return fail(MAGNUS_ENOCONV, "no degree <= %d reaches tol %g", o->max_degree, tol_e);
      const ExpOp& op = G.ops[q];
      const int m = P.lp.m, ns = G.s[k];
      for (int sub = 0; sub < ns; ++sub)
        for (int i = 1; i <= m; ++i) {
          magnus::IterCoef& c = (*out)[(size_t)(n - n0) * G.stride + G.off[k] + (size_t)sub * G.m[k] + (i - 1)];
          c.a1 = P.scale * op.a;
          c.a2 = P.scale * op.b;
          c.kap = P.scale * op.kappa;
          c.sigma = P.scale * P.c + xi[i - 1];
          c.dre = P.d[i].real();
          c.dim = P.d[i].imag();
          c.d0re = P.d[0].real();
          c.d0im = P.d[0].imag();
          c.dabs = std::abs(P.d[i]);
          c.d0abs = std::abs(P.d[0]);
          c.prev_dabs = i >= 2 ? std::abs(P.d[i - 1]) : 0.0;
          c.tol = tol_e / (2.0 * ns);
          c.active = 1;
        }
      acc->exponentials += 1;
      acc->substeps += ns;
      acc->planned += (int64_t)m * ns;
      acc->max_m = std::max(acc->max_m, m);
      acc->max_s = std::max(acc->max_s, ns);
      acc->max_bound = std::max(acc->max_bound, P.lp.bound);
    }
  return MAGNUS_OK;
}

void graph_release(magnus_ctx* ctx) {
  if (ctx->graph_x) (void)hipGraphExecDestroy(ctx->graph_x);
  if (ctx->graph_g) (void)hipGraphDestroy(ctx->graph_g);
  ctx->graph_x = nullptr;
  ctx->graph_g = nullptr;
}

// Capture the launches of one step of state y (in place) on the context's
// capture stream: the exponentials in the scheme's order, each launch bound
// to its table column, then the step counter's advance.
int graph_capture(magnus_ctx* ctx, const magnus_hamiltonian* h, const magnus::Scheme& S, const GraphPlan& G,
                  double2* y, double tol_e, int early) {
  if (ctx->graph_x) {
    // the previous call's replays must have finished before its graph goes
    HIP_TRY(hipEventSynchronize(ctx->graph_done));
    graph_release(ctx);
  }
  if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  hipStream_t cs = ctx->cap_stream;
  const magnus::IterCoef* base = reinterpret_cast<const magnus::IterCoef*>(ctx->table);
  HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  int rc = MAGNUS_OK;
  double2* mids[2] = {ctx->vec(kS2), ctx->vec(kU)};
  const double2* src = y;
  for (int k = 0; k < G.nexp && rc == MAGNUS_OK; ++k) {
    // structure only: the coefficients come from the table
    ExpPlan T;
    T.scale = 1.0;
    T.lp = magnus::LejaPlan{G.m[k], G.s[k], 0.0};
    T.d.assign((size_t)G.m[k] + 1, std::complex<double>(1.0, 0.0));
    const TableRef tab{base + G.off[k], G.stride, ctx->gctr};
    double2* dst = (k == G.nexp - 1) ? y : mids[k & 1];
    const ExpOp op{h, 1.0, 1.0, S.commutator ? 1.0 : 0.0};
    rc = enqueue_exponential(ctx, op, T, src, dst, tol_e / (2.0 * G.s[k]), early, &tab, cs);
    src = dst;
  }
  if (rc == MAGNUS_OK && magnus::launch_step_advance(ctx->gctr, cs) != hipSuccess)
    rc = fail(MAGNUS_EHIP, "step counter launch during capture");
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cs, &g);
  if (rc != MAGNUS_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc != MAGNUS_OK ? rc : fail(MAGNUS_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  }
  ctx->graph_g = g;
  HIP_TRY(hipGraphInstantiate(&ctx->graph_x, g, nullptr, nullptr, 0));
  if (!ctx->graph_done) HIP_TRY(hipEventCreateWithFlags(&ctx->graph_done, hipEventDisableTiming));
  return MAGNUS_OK;
}

// Replay steps [n0, n1): table chunks uploaded behind the previous replays,
// the counter set to the chunk's first step, one graph launch per step.
int graph_replay(magnus_ctx* ctx, const GraphPlan& G, double tau, int64_t n0, int64_t n1, double tol_e,
                 const magnus_leja_opts* o, Acc* acc, hipStream_t s) {
  int64_t per = std::max<int64_t>(1, graph_table_cap(ctx) / G.stride);
  if (ctx->graph_chunk > 0) per = std::min<int64_t>(per, ctx->graph_chunk);
  for (int64_t c0 = n0; c0 < n1; c0 += per) {
    const int64_t c1 = std::min(n1, c0 + per);
    int rc = graph_fill(G, tau, c0, c1, tol_e, o, acc, &ctx->graph_table);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(ctx->table, ctx->graph_table.data(), sizeof(magnus::IterCoef) * ctx->graph_table.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(magnus::launch_step_set(ctx->gctr, 0, s));
    for (int64_t n = c0; n < c1; ++n) HIP_TRY(hipGraphLaunch(ctx->graph_x, s));
  }
  HIP_TRY(hipEventRecord(ctx->graph_done, s));
  return MAGNUS_OK;
}

int check_batch(magnus_ctx* ctx, int32_t batch) {
  if (batch < 1) return fail(MAGNUS_EINVAL, "batch %d < 1", batch);
  if (batch > ctx->max_batch) return fail(MAGNUS_ENOMEM, "batch %d exceeds workspace max_batch %d", batch, ctx->max_batch);
  return MAGNUS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of the allocation-free Cf4 step (magnus_step_cf4_noalloc): the eight
// workspace vectors of one state of up to kNoAllocMaxDim entries, the
// per-workgroup norm partials of the iteration kernels, the outputs of the
// CSR structure scan and one control slot.  A file-scope device array, so the
// code object's loader places it on every device the library runs on, and it
// stays there until the process ends.  Host code never uses the array's name
// as an address: it asks each device for its copy's address once
// (hipGetSymbolAddress) and passes that pointer on.
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kNoAllocMaxDim = 1 << 17;
constexpr size_t kNaAlign = 256;
constexpr size_t na_round(size_t b) { return (b + kNaAlign - 1) / kNaAlign * kNaAlign; }
constexpr size_t kNaVecBytes = (size_t)kNumVec * (size_t)kNoAllocMaxDim * sizeof(double2);
constexpr int64_t kNaGrid = kNoAllocMaxDim / 8 + 2;  // as magnus_create: 8 rows per smallest row block
constexpr size_t kNaPartials = 4 * (size_t)kNaGrid + 64;  // two halves for the fused stop tests
constexpr int64_t kNaScanLen = 2 * (kNoAllocMaxDim / 4 + 2) + 3 * (kNoAllocMaxDim / 256 + 2);
constexpr size_t kNaPartialOff = kNaVecBytes;
constexpr size_t kNaScanOff = kNaPartialOff + na_round(kNaPartials * sizeof(double));
constexpr size_t kNaSlotOff = kNaScanOff + na_round((size_t)kNaScanLen * sizeof(double));
constexpr size_t kNoAllocBytes = kNaSlotOff + na_round(sizeof(Slot));  // 17.0 MiB
constexpr int kNaMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_na_mu;
// One context per device whose workspace points into that device's scratch
// (set up on the first call on the device; never freed).
magnus_ctx g_na_ctx[kNaMaxDevices];

int noalloc_context(magnus_ctx** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNaMaxDevices) return fail(MAGNUS_EINVAL, "device %d beyond the %d the library serves", dev, kNaMaxDevices);
  std::lock_guard<std::mutex> g(g_na_mu);
  magnus_ctx& c = g_na_ctx[dev];
  if (!c.vecs) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(MAGNUS_EHIP, "address of the scratch array on device %d: %s", dev, hipGetErrorString(e));
    unsigned char* base = static_cast<unsigned char*>(ptr);
    c.device = dev;
    c.max_dim = kNoAllocMaxDim;
    c.max_batch = 1;
    c.max_grid = kNaGrid;
    c.partials = reinterpret_cast<double*>(base + kNaPartialOff);
    c.npartials = kNaPartials;
    c.scan = reinterpret_cast<double*>(base + kNaScanOff);
    c.scan_len = kNaScanLen;
    c.slots = reinterpret_cast<Slot*>(base + kNaSlotOff);
    c.nslots = 1;
    c.persist = 0;
    if (const char* v = getenv("MAGNUS_CSR_VARIANT")) c.csr_variant = atoi(v);
    if (const char* v = getenv("MAGNUS_FUSE")) c.fuse = atoi(v);
    c.vecs = reinterpret_cast<double2*>(base);  // last: marks the device's context ready
  }
  *out = &c;
  return MAGNUS_OK;
}
}  // namespace

extern "C" {

const char* magnus_last_error(void) { return g_err.c_str(); }

int magnus_create(magnus_ctx** out, int64_t max_dim, int32_t max_batch, int32_t device) {
  if (!out) return fail(MAGNUS_EINVAL, "null output pointer");
  *out = nullptr;
  if (max_dim < 1 || max_batch < 1) return fail(MAGNUS_EINVAL, "max_dim and max_batch must be >= 1");
  if (max_dim > INT32_MAX / 2) return fail(MAGNUS_EINVAL, "max_dim too large");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(MAGNUS_EINVAL, "device %d not in 0..%d", device, ndev - 1);
  HIP_TRY(hipSetDevice(device));
  magnus_ctx* c = new magnus_ctx();
  c->device = device;
  c->max_dim = max_dim;
  c->max_batch = max_batch;
  if (const char* v = getenv("MAGNUS_CSR_VARIANT")) c->csr_variant = atoi(v);
  c->max_grid = max_dim / 8 + 2;  // the smallest row block of any iteration kernel is 8 rows
  c->scan_len = 2 * (max_dim / 4 + 2) + 3 * (max_dim / 256 + 2);
  c->nslots = std::max<int>(256, max_batch);
  if (const char* v = getenv("MAGNUS_PERSIST")) c->persist = atoi(v);
  if (const char* v = getenv("MAGNUS_FUSE")) c->fuse = atoi(v);
  if (const char* v = getenv("MAGNUS_GRAPH")) c->graph = atoi(v);
  if (const char* v = getenv("MAGNUS_GRAPH_STEPS")) c->graph_chunk = atoi(v);
  if (const char* v = getenv("MAGNUS_RAGGED_JOINT")) c->ragged_joint = atoi(v);
  if (const char* v = getenv("MAGNUS_DENSE_RPW")) {
    const int r = atoi(v);
    c->dense_rpw_env = (r == 1 || r == 2 || r == 4) ? r : 0;
  }
  if (const char* v = getenv("MAGNUS_ASSEMBLE_FUSED")) c->fuse_assembly = atoi(v);
  if (const char* v = getenv("MAGNUS_PERSIST_CACHE")) c->persist_cache = atoi(v);
  if (const char* v = getenv("MAGNUS_MFMA_TILE")) {
    const int t = atoi(v);
    c->mfma_tile_env = (t >= 0 && t < magnus::kMfmaTiles) ? t : -1;
  }
  const size_t nvec = (size_t)kNumVec * (size_t)max_dim * (size_t)max_batch;
  hipError_t e = hipMalloc(&c->vecs, sizeof(double2) * nvec);
  if (e == hipSuccess) e = hipMalloc(&c->slots, sizeof(Slot) * c->nslots);
  if (e == hipSuccess) e = hipMalloc(&c->table, sizeof(ColParam) * kTableCap);
  if (e == hipSuccess) e = hipMalloc(&c->arena, kArenaBytes);
  // the multi-state CSR kernel writes dim * B^2 / 128 doubles (B <= 32: at most 8 dim)
  c->npartials = 2 * (size_t)c->max_grid + 8 * (size_t)max_dim +
                 (size_t)max_dim * (size_t)std::max(1, max_batch) / 8 + (size_t)max_dim + 64;
  // the dot-product kernel's per-workgroup pairs, whatever the dimension
  c->npartials = std::max(c->npartials, (size_t)magnus::kDotPartials + 64);
  if (e == hipSuccess) e = hipMalloc(&c->partials, sizeof(double) * c->npartials);
  if (e == hipSuccess) e = hipMalloc(&c->scan, sizeof(double) * (size_t)c->scan_len);
  if (e == hipSuccess) e = hipMalloc(&c->gctr, 256);
  if (e == hipSuccess) e = hipMemset(c->slots, 0, sizeof(Slot) * c->nslots);
  if (e == hipSuccess) e = hipMemset(c->vecs, 0, sizeof(double2) * nvec);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    magnus_destroy(c);
    return fail(MAGNUS_EHIP, "workspace allocation: %s", hipGetErrorString(e));
  }
  (void)magnus::leja_points();  // build the planner tables once, up front
  *out = c;
  return MAGNUS_OK;
}

int magnus_reserve_dense(magnus_ctx* ctx, int64_t dim) {
  if (!ctx) return fail(MAGNUS_EINVAL, "null context");
  if (dim < 1 || dim > ctx->max_dim) return fail(MAGNUS_EINVAL, "dim %lld outside 1..max_dim", (long long)dim);
  if (ctx->assembled_dim >= dim) return MAGNUS_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  if (ctx->assembled) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(ctx->assembled));
    ctx->assembled = nullptr;
    ctx->assembled_dim = 0;
  }
  HIP_TRY(hipMalloc(&ctx->assembled, sizeof(double2) * (size_t)dim * (size_t)dim));
  ctx->assembled_dim = dim;
  return MAGNUS_OK;
}

int magnus_dense_commutator(magnus_ctx* ctx, magnus_hamiltonian* h, magnus_stream stream) {
  if (!ctx || !h) return fail(MAGNUS_EINVAL, "null argument");
  int rc = check_ham(ctx, h, 0);
  if (rc) return rc;
  if (h->H1.format != MAGNUS_DENSE) return fail(MAGNUS_EINVAL, "magnus_dense_commutator needs dense terms");
  const int64_t dim = h->H1.dim;
  if ((rc = magnus_reserve_dense(ctx, dim))) return rc;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  if (ctx->comm_dim < dim) {
    if (ctx->comm) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(ctx->comm));
      ctx->comm = nullptr;
      ctx->comm_dim = 0;
    }
    HIP_TRY(hipMalloc(&ctx->comm, sizeof(double2) * (size_t)dim * (size_t)dim));
    ctx->comm_dim = dim;
  }
  ctx->comm_h1 = ctx->comm_h2 = nullptr;
  ctx->m6_ready = false;
  const double2* H1 = reinterpret_cast<const double2*>(h->H1.val);
  const double2* H2 = reinterpret_cast<const double2*>(h->H2.val);
  HIP_TRY(magnus::launch_zgemm(H1, h->H1.ld, H2, h->H2.ld, ctx->assembled, (int)dim, s));
  HIP_TRY(magnus::launch_commutator_combine(ctx->assembled, (int)dim, 1.0, ctx->comm, s));
  magnus_term kt{};
  kt.format = MAGNUS_DENSE;
  kt.dim = dim;
  kt.ld = dim;
  kt.val = ctx->comm;
  double lo, hi;
  if ((rc = dense_scan(ctx, kt, s, &lo, &hi))) return rc;
  h->k_min = lo;
  h->k_max = hi;
  ctx->comm_h1 = h->H1.val;
  ctx->comm_h2 = h->H2.val;
  ctx->comm_n = dim;
  ctx->comm_ld = h->H1.ld;
  return MAGNUS_OK;
}

// out = i (A B - B A) of two CSR matrices into the storage (rp, ci, val) of
// rows + 1 and cap entries (grown as needed), with its Gershgorin enclosure.
int assemble_csr_commutator(magnus_ctx* ctx, const CsrDev& A, const CsrDev& Bm, int64_t dim, int*& rp_d, int*& ci_d,
                            double2*& val_d, int64_t& rows, int64_t& cap, int64_t& nnz_out, double* lo, double* hi,
                            hipStream_t s) {
  // count pass: per-row sizes in a work vector, the overflow flag in the scan buffer
  int* counts = reinterpret_cast<int*>(ctx->vec(kV));
  int* overflow = reinterpret_cast<int*>(ctx->scan);
  HIP_TRY(hipMemsetAsync(overflow, 0, sizeof(int), s));
  HIP_TRY(magnus::launch_csr_commutator(false, A, Bm, (int)dim, counts, nullptr, nullptr, nullptr, overflow, s));
  std::vector<int> cnt((size_t)dim);
  int ovf = 0;
  HIP_TRY(hipMemcpyAsync(cnt.data(), counts, sizeof(int) * cnt.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&ovf, overflow, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (ovf)
    return fail(MAGNUS_ENOMEM, "a row of A B - B A lists more than %d products (use the matrix-free commutator)",
                magnus::kCommCap);
  std::vector<int> rp((size_t)dim + 1, 0);
  for (int64_t r = 0; r < dim; ++r) {
    if ((int64_t)rp[r] + cnt[r] > INT32_MAX) return fail(MAGNUS_ENOMEM, "the commutator has more than 2^31 entries");
    rp[r + 1] = rp[r] + cnt[r];
  }
  const int64_t nnz = rp[dim];
  if (rows < dim || cap < std::max<int64_t>(nnz, 1)) {
    HIP_TRY(hipStreamSynchronize(s));
    if (rp_d) HIP_TRY(hipFree(rp_d));
    if (ci_d) HIP_TRY(hipFree(ci_d));
    if (val_d) HIP_TRY(hipFree(val_d));
    rp_d = nullptr;
    ci_d = nullptr;
    val_d = nullptr;
    rows = cap = 0;
    HIP_TRY(hipMalloc(&rp_d, sizeof(int) * (size_t)(dim + 1)));
    HIP_TRY(hipMalloc(&ci_d, sizeof(int) * (size_t)std::max<int64_t>(nnz, 1)));
    HIP_TRY(hipMalloc(&val_d, sizeof(double2) * (size_t)std::max<int64_t>(nnz, 1)));
    rows = dim;
    cap = std::max<int64_t>(nnz, 1);
  }
  HIP_TRY(hipMemcpyAsync(rp_d, rp.data(), sizeof(int) * rp.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(magnus::launch_csr_commutator(true, A, Bm, (int)dim, counts, rp_d, ci_d, val_d, overflow, s));
  nnz_out = nnz;
  magnus_term kt{};
  kt.format = MAGNUS_CSR;
  kt.dim = dim;
  kt.nnz = nnz;
  kt.row_ptr = rp_d;
  kt.col_idx = ci_d;
  kt.val = val_d;
  return csr_scan(ctx, kt, s, lo, hi);
}

int magnus_csr_commutator(magnus_ctx* ctx, magnus_hamiltonian* h, magnus_stream stream) {
  if (!ctx || !h) return fail(MAGNUS_EINVAL, "null argument");
  int rc = check_ham(ctx, h, 0);
  if (rc) return rc;
  if (h->H1.format != MAGNUS_CSR) return fail(MAGNUS_EINVAL, "magnus_csr_commutator needs CSR terms");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  if ((rc = ensure_valid(ctx, h, s))) return rc;
  const int64_t dim = h->H1.dim;
  CsrDev A{h->H1.row_ptr, h->H1.col_idx, reinterpret_cast<const double2*>(h->H1.val)};
  CsrDev Bm{h->H2.row_ptr, h->H2.col_idx, reinterpret_cast<const double2*>(h->H2.val)};
  ctx->kc_key = std::make_tuple(nullptr, nullptr, nullptr, nullptr, (int64_t)0);
  double lo, hi;
  if ((rc = assemble_csr_commutator(ctx, A, Bm, dim, ctx->kc_rp, ctx->kc_ci, ctx->kc_val, ctx->kc_rows, ctx->kc_cap,
                                    ctx->kc_nnz, &lo, &hi, s)))
    return rc;
  h->k_min = lo;
  h->k_max = hi;
  ctx->kc_key = std::make_tuple((const void*)h->H1.row_ptr, h->H1.val, (const void*)h->H2.row_ptr, h->H2.val, dim);
  return MAGNUS_OK;
}

int magnus_csr_m6_prepare(magnus_ctx* ctx, magnus_hamiltonian* h, magnus_stream stream) {
  int rc = magnus_csr_commutator(ctx, h, stream);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int64_t dim = h->H1.dim;
  ctx->pm_key = std::make_tuple(nullptr, nullptr, nullptr, nullptr, (int64_t)0);
  const CsrDev K{ctx->kc_rp, ctx->kc_ci, ctx->kc_val};
  const CsrDev H[2] = {CsrDev{h->H1.row_ptr, h->H1.col_idx, reinterpret_cast<const double2*>(h->H1.val)},
                       CsrDev{h->H2.row_ptr, h->H2.col_idx, reinterpret_cast<const double2*>(h->H2.val)}};
  for (int a = 0; a < 2; ++a)  // P_a = -i[H_a, K] = i[K, H_a]
    if ((rc = assemble_csr_commutator(ctx, K, H[a], dim, ctx->pm_rp[a], ctx->pm_ci[a], ctx->pm_val[a],
                                      ctx->pm_rows[a], ctx->pm_cap[a], ctx->pm_nnz[a], &ctx->pm_lo[a],
                                      &ctx->pm_hi[a], s)))
      return rc;
  if (ctx->pm_ws_dim < dim) {
    HIP_TRY(hipStreamSynchronize(s));
    if (ctx->pm_ws) HIP_TRY(hipFree(ctx->pm_ws));
    ctx->pm_ws = nullptr;
    ctx->pm_ws_dim = 0;
    HIP_TRY(hipMalloc(&ctx->pm_ws, (magnus::kM6Terms + 1) * sizeof(double2) * (size_t)dim));
    ctx->pm_ws_dim = dim;
  }
  ctx->pm_key = ctx->kc_key;
  return MAGNUS_OK;
}

int magnus_dense_m6_prepare(magnus_ctx* ctx, magnus_hamiltonian* h, magnus_stream stream) {
  int rc = magnus_dense_commutator(ctx, h, stream);
  if (rc) return rc;
  const int64_t dim = h->H1.dim;
  hipStream_t s = (hipStream_t)stream;
  if (ctx->m6_dim < dim) {
    if (ctx->m6) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(ctx->m6));
      ctx->m6 = nullptr;
      ctx->m6_dim = 0;
    }
    HIP_TRY(hipMalloc(&ctx->m6, 7 * sizeof(double2) * (size_t)dim * (size_t)dim));
    ctx->m6_dim = dim;
  }
  const size_t sz = (size_t)ctx->m6_dim * (size_t)ctx->m6_dim;
  double2* M = ctx->m6;
  double2* P1 = M;
  double2* P2 = M + sz;
  const double2* H1 = reinterpret_cast<const double2*>(h->H1.val);
  const double2* H2 = reinterpret_cast<const double2*>(h->H2.val);
  const long long ld = h->H1.ld;
  // (left, ld, right, ld, scale, out): out = scale i [left, right], the GEMM product in the assembly buffer
  struct Job {
    const double2* a;
    long long lda;
    const double2* b;
    long long ldb;
    double scale;
    double2* out;
  };
  const Job jobs[7] = {{H1, ld, ctx->comm, dim, -1.0, P1},           // P1 = -i[H1, K]
                       {H2, ld, ctx->comm, dim, -1.0, P2},           // P2 = -i[H2, K]
                       {H1, ld, P1, dim, 1.0, M + 2 * sz},           // U11 = i[H1, P1]
                       {H1, ld, P2, dim, 1.0, M + 3 * sz},           // U12 = i[H1, P2]
                       {H2, ld, P2, dim, 1.0, M + 4 * sz},           // U22 = i[H2, P2]
                       {ctx->comm, dim, P1, dim, -1.0, M + 5 * sz},  // R1 = -i[K, P1]
                       {ctx->comm, dim, P2, dim, -1.0, M + 6 * sz}}; // R2 = -i[K, P2]
  for (int j = 0; j < 7; ++j) {
    HIP_TRY(magnus::launch_zgemm(jobs[j].a, jobs[j].lda, jobs[j].b, jobs[j].ldb, ctx->assembled, (int)dim, s));
    HIP_TRY(magnus::launch_commutator_combine(ctx->assembled, (int)dim, jobs[j].scale, jobs[j].out, s));
    magnus_term t{};
    t.format = MAGNUS_DENSE;
    t.dim = dim;
    t.ld = dim;
    t.val = jobs[j].out;
    if ((rc = dense_scan(ctx, t, s, &ctx->m6_lo[j], &ctx->m6_hi[j]))) return rc;
  }
  ctx->m6_ready = true;
  return MAGNUS_OK;
}

}  // extern "C"

namespace {
// Dense terms: the GEMV iteration with 1, 2 and 4 rows per wave (two terms),
// and for batches the FP64-MFMA group iteration with each tile shape on the
// batch's states (one term, as a shared field assembles the exponent, when
// the context holds an assembly buffer; else two), 5 timed launches each.
int autotune_dense(magnus_ctx* ctx, const magnus_hamiltonian* h, int32_t batch, int32_t* variant, int32_t* group,
                   double* variant_us, double* group_us, hipStream_t s) {
  int rc = begin_call(ctx, s);
  if (rc) return rc;
  const int dim = (int)h->H1.dim;
  const size_t nvec = (size_t)ctx->max_dim * (size_t)ctx->max_batch;
  for (int k : {kA, kB, kS0, kY}) HIP_TRY(hipMemsetAsync(ctx->vec(k), 0, sizeof(double2) * nvec, s));
  const double2* D1 = reinterpret_cast<const double2*>(h->H1.val);
  const double2* D2 = reinterpret_cast<const double2*>(h->H2.val);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  constexpr int kReps = 5;
  auto time_us = [&](auto f, double* us) -> hipError_t {
    hipError_t e = f();
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < kReps && e == hipSuccess; ++r) e = f();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    *us = 1e3 * (double)ms / kReps;
    return e;
  };
  hipError_t err = hipSuccess;
  IterArgs a{};
  a.x1 = a.x2 = a.wcur = ctx->vec(kA);
  a.wout = ctx->vec(kB);
  a.pacc = ctx->vec(kS0);
  a.slot = ctx->slots;
  a.partials = ctx->partials;
  a.a1 = a.a2 = 1.0;
  a.first = 1;
  int best_rpw = 2;
  double best = INFINITY;
  const int rpws[3] = {1, 2, 4};
  for (int q = 0; q < 3 && err == hipSuccess; ++q) {
    double us = 0.0;
    err = time_us([&] { return magnus::launch_dense2_iter(D1, D2, dim, h->H1.ld, a, s, rpws[q]); }, &us);
    if (variant_us) variant_us[q] = us;
    if (us < best) {
      best = us;
      best_rpw = rpws[q];
    }
  }
  if (variant_us)
    for (int q = 3; q < kTuneVariants; ++q) variant_us[q] = NAN;
  int best_tile = 0;
  double best_t = INFINITY;
  if (err == hipSuccess && batch > 1) {
    std::vector<ColParam> table(batch);
    for (ColParam& c : table) c.a1 = c.a2 = 1.0;
    if ((rc = upload_table(ctx, table, s))) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return rc;
    }
    const bool one = ctx->assembled && ctx->assembled_dim >= dim;
    for (int t = 0; t < magnus::kMfmaTiles && err == hipSuccess; ++t) {
      MultiArgs m{};
      m.x = ctx->vec(kY);
      m.wout = ctx->vec(kA);
      m.pacc = ctx->vec(kB);
      m.slots = ctx->slots;
      m.partials = ctx->partials;
      m.prm = ctx->table;
      m.B = batch;
      m.first = 1;
      double us = 0.0;
      err = time_us([&] { return magnus::launch_dense_mfma(one ? 1 : 2, D1, D2, h->H1.ld, dim, m, s, t); }, &us);
      if (group_us) group_us[t] = us;
      if (us < best_t) {
        best_t = us;
        best_tile = t;
      }
    }
  } else if (group_us) {
    for (int t = 0; t < magnus::kMfmaTiles; ++t) group_us[t] = NAN;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(MAGNUS_EHIP, "autotune: %s", hipGetErrorString(err));
  const auto key = std::make_pair(h->H1.val, h->H1.dim);
  ctx->tuned_dense_rpw[key] = best_rpw;
  if (batch > 1) ctx->tuned_mfma[key] = best_tile;
  if (variant) *variant = best_rpw;
  if (group) *group = batch > 1 ? best_tile : 0;
  return MAGNUS_OK;
}
}  // namespace

extern "C" {

int magnus_autotune(magnus_ctx* ctx, const magnus_hamiltonian* h, int32_t batch, int32_t* variant,
                    int32_t* group, double* variant_us, double* group_us, magnus_stream stream) {
  int rc = check_ham(ctx, h, 0);
  if (rc) return rc;
  if ((rc = check_batch(ctx, batch))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (h->H1.format == MAGNUS_DENSE) return autotune_dense(ctx, h, batch, variant, group, variant_us, group_us, s);
  if ((rc = begin_call(ctx, s))) return rc;
  if ((rc = ensure_valid(ctx, h, s))) return rc;
  const int dim = (int)h->H1.dim;
  const size_t nvec = (size_t)ctx->max_dim * (size_t)ctx->max_batch;
  for (int k : {kA, kB, kS0, kY})
    HIP_TRY(hipMemsetAsync(ctx->vec(k), 0, sizeof(double2) * nvec, s));
  CsrDev t1{h->H1.row_ptr, h->H1.col_idx, reinterpret_cast<const double2*>(h->H1.val)};
  CsrDev t2{h->H2.row_ptr, h->H2.col_idx, reinterpret_cast<const double2*>(h->H2.val)};
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  constexpr int kReps = 5;
  // time f (kReps launches after one untimed launch), in microseconds per launch
  auto time_us = [&](auto f, double* us) -> hipError_t {
    hipError_t e = f();
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < kReps && e == hipSuccess; ++r) e = f();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    *us = 1e3 * (double)ms / kReps;
    return e;
  };
  hipError_t err = hipSuccess;
  // the single-state iteration: each row mapping on this matrix
  IterArgs a{};
  a.x1 = a.x2 = a.wcur = ctx->vec(kA);
  a.wout = ctx->vec(kB);
  a.pacc = ctx->vec(kS0);
  a.slot = ctx->slots;
  a.partials = ctx->partials;
  a.a1 = a.a2 = 1.0;
  a.first = 1;
  double best = INFINITY;
  int best_code = 0;
  for (int code = 1; code <= kTuneVariants && err == hipSuccess; ++code) {
    const int rpb = variant_rows(code, dim);
    double us = 0.0;
    // an iteration on a grid too large for the fused stop test is followed by
    // the decide kernel, so that is timed with it
    const bool decide = !ctx->fuse || magnus::csr2_grid(dim, rpb) > magnus::kFuseMaxGrid;
    err = time_us(
        [&] {
          hipError_t e = magnus::launch_csr2_iter(magnus::kLeja, t1, t2, dim, a, rpb, s);
          if (e == hipSuccess && decide) e = magnus::launch_leja_decide(a, magnus::csr2_grid(dim, rpb), s);
          return e;
        },
        &us);
    if (variant_us) variant_us[code - 1] = us;
    if (us < best) {
      best = us;
      best_code = code;
    }
  }
  // the multi-state iteration: cost per state of each group size up to the batch
  int best_group = 32;
  double best_per_state = INFINITY;
  std::vector<ColParam> table(32);
  for (ColParam& c : table) c.a1 = c.a2 = 1.0;
  if (err == hipSuccess && batch > 1) {
    if ((rc = upload_table(ctx, table, s))) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return rc;
    }
  }
  int gi = 0;
  for (int g : {2, 4, 8, 16, 32}) {
    double us = NAN;
    if (err == hipSuccess && g <= batch && (size_t)magnus::csr2_multi_grid(dim, g) * g * 2 <= ctx->npartials) {
      MultiArgs m{};
      m.x = ctx->vec(kY);
      m.wout = ctx->vec(kA);
      m.pacc = ctx->vec(kB);
      m.slots = ctx->slots;
      m.partials = ctx->partials;
      m.prm = ctx->table;
      m.B = g;
      m.first = 1;
      err = time_us([&] { return magnus::launch_csr2_multi(magnus::kMultiLeja, t1, t2, dim, m, s); }, &us);
      if (err == hipSuccess && us / g < best_per_state) {
        best_per_state = us / g;
        best_group = g;
      }
    }
    if (group_us) group_us[gi] = us;
    ++gi;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(MAGNUS_EHIP, "autotune: %s", hipGetErrorString(err));
  const auto key = std::make_pair((const void*)h->H1.row_ptr, h->H1.dim);
  ctx->tuned_variant[key] = best_code;
  if (batch > 1) ctx->tuned_group[key] = best_group;
  if (variant) *variant = best_code;
  if (group) *group = batch > 1 ? best_group : 1;
  return MAGNUS_OK;
}

int magnus_destroy(magnus_ctx* ctx) {
  if (!ctx) return MAGNUS_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->vecs) (void)hipFree(ctx->vecs);
  if (ctx->slots) (void)hipFree(ctx->slots);
  if (ctx->table) (void)hipFree(ctx->table);
  if (ctx->arena) (void)hipFree(ctx->arena);
  if (ctx->assembled) (void)hipFree(ctx->assembled);
  if (ctx->comm) (void)hipFree(ctx->comm);
  if (ctx->m6) (void)hipFree(ctx->m6);
  if (ctx->kc_rp) (void)hipFree(ctx->kc_rp);
  if (ctx->kc_ci) (void)hipFree(ctx->kc_ci);
  if (ctx->kc_val) (void)hipFree(ctx->kc_val);
  for (int a = 0; a < 2; ++a) {
    if (ctx->pm_rp[a]) (void)hipFree(ctx->pm_rp[a]);
    if (ctx->pm_ci[a]) (void)hipFree(ctx->pm_ci[a]);
    if (ctx->pm_val[a]) (void)hipFree(ctx->pm_val[a]);
  }
  if (ctx->pm_ws) (void)hipFree(ctx->pm_ws);
  if (ctx->partials) (void)hipFree(ctx->partials);
  if (ctx->scan) (void)hipFree(ctx->scan);
  if (ctx->graph_x || ctx->graph_g) {
    if (ctx->graph_done) (void)hipEventSynchronize(ctx->graph_done);
    graph_release(ctx);
  }
  if (ctx->graph_done) (void)hipEventDestroy(ctx->graph_done);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->gctr) (void)hipFree(ctx->gctr);
  for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
  delete ctx;
  return MAGNUS_OK;
}

int magnus_check(magnus_ctx* ctx, magnus_stream stream) {
  if (!ctx) return fail(MAGNUS_EINVAL, "null context");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  long long iters = 0;
  int status = 0;
  int rc = read_slots(ctx, s, &iters, &status);
  if (rc) return rc;
  status |= ctx->sticky_status;
  if (status & 1) return fail(MAGNUS_ENAN, "non-finite vector norm met on the device");
  return MAGNUS_OK;
}

int magnus_spectral_bounds(magnus_ctx* ctx, magnus_hamiltonian* h, magnus_stream stream) {
  if (!ctx || !h) return fail(MAGNUS_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  const int64_t dim = h->H1.dim;
  if (dim < 1 || dim > ctx->max_dim) return fail(dim < 1 ? MAGNUS_EINVAL : MAGNUS_ENOMEM, "dim %lld", (long long)dim);
  magnus_term* terms[2] = {&h->H1, &h->H2};
  for (magnus_term* t : terms) {
    // the enclosure is not yet known: validate the rest of the term only
    const double l0 = t->lam_min, u0 = t->lam_max;
    t->lam_min = 0.0;
    t->lam_max = 0.0;
    int rc = check_term(*t, dim, t == &h->H1 ? "H1" : "H2");
    t->lam_min = l0;
    t->lam_max = u0;
    if (rc) return rc;
    double lo, hi;
    rc = (t->format == MAGNUS_CSR) ? csr_scan(ctx, *t, s, &lo, &hi) : dense_scan(ctx, *t, s, &lo, &hi);
    if (rc) return rc;
    t->lam_min = lo;
    t->lam_max = hi;
  }
  const double n1 = std::fmax(std::fabs(h->H1.lam_min), std::fabs(h->H1.lam_max));
  const double n2 = std::fmax(std::fabs(h->H2.lam_min), std::fabs(h->H2.lam_max));
  h->k_min = -2.0 * n1 * n2;
  h->k_max = 2.0 * n1 * n2;
  return MAGNUS_OK;
}

namespace {

// y = H x for one term (the iteration kernels with the other term empty or absent).
int apply_term(magnus_ctx* ctx, const magnus_term& t, const double2* x, double2* y, hipStream_t s) {
  const int dim = (int)t.dim;
  IterArgs a{};
  a.x1 = a.x2 = a.wcur = x;
  a.wout = y;
  a.pacc = ctx->vec(kS1);
  a.slot = ctx->slots;
  a.partials = ctx->partials;
  a.a1 = 1.0;
  a.first = 1;
  if (t.format == MAGNUS_DENSE) {
    HIP_TRY(magnus::launch_dense2_iter(reinterpret_cast<const double2*>(t.val), nullptr, dim, t.ld, a, s));
    return MAGNUS_OK;
  }
  CsrDev t1{t.row_ptr, t.col_idx, reinterpret_cast<const double2*>(t.val)};
  CsrDev none{reinterpret_cast<const int*>(ctx->vec(kV)), nullptr, nullptr};  // all rows empty
  HIP_TRY(magnus::launch_csr2_iter(magnus::kLeja, t1, none, dim, a, variant_rows(0, dim), s));
  return MAGNUS_OK;
}

// Re(x^H y) on the host (one device dot product and a wait).
int dot_re(magnus_ctx* ctx, const double2* x, const double2* y, int64_t n, double* out, hipStream_t s) {
  double2* dev_out = reinterpret_cast<double2*>(ctx->partials + magnus::kDotPartials);
  if (int rc = flush_fused_check(ctx, s)) return rc;
  HIP_TRY(magnus::launch_cdot(x, 1, y, 1, n, ctx->partials, dev_out, s));
  double2 h;
  HIP_TRY(hipMemcpyAsync(&h, dev_out, sizeof(double2), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *out = h.x;
  return MAGNUS_OK;
}

// Lanczos on one Hermitian term from a fixed pseudo-random start: extreme Ritz
// values after `steps` steps and their change over the last steps.
int lanczos_term(magnus_ctx* ctx, const magnus_term& t, int steps, double* lo, double* hi, double* drift,
                 hipStream_t s) {
  const int64_t n = t.dim;
  double2* P = ctx->vec(kA);  // previous basis vector
  double2* C = ctx->vec(kB);  // current basis vector
  double2* W = ctx->vec(kS0);
  HIP_TRY(hipMemsetAsync(ctx->vec(kV), 0, sizeof(int) * (size_t)(n + 1), s));
  HIP_TRY(hipMemsetAsync(P, 0, sizeof(double2) * (size_t)n, s));
  {
    // start vector: splitmix64 stream mapped to [-1, 1)^2, normalised on the host
    std::vector<double2> v0((size_t)n);
    uint64_t z = 0x9E3779B97F4A7C15ull;
    double nrm = 0.0;
    auto next = [&z]() {
      z += 0x9E3779B97F4A7C15ull;
      uint64_t r = z;
      r = (r ^ (r >> 30)) * 0xBF58476D1CE4E5B9ull;
      r = (r ^ (r >> 27)) * 0x94D049BB133111EBull;
      r ^= r >> 31;
      return (double)(r >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    };
    for (auto& e : v0) {
      e.x = next();
      e.y = next();
      nrm += e.x * e.x + e.y * e.y;
    }
    const double inv = 1.0 / std::sqrt(nrm);
    for (auto& e : v0) {
      e.x *= inv;
      e.y *= inv;
    }
    HIP_TRY(hipMemcpyAsync(C, v0.data(), sizeof(double2) * v0.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  std::vector<double> al, be;
  double beta_prev = 0.0, lo_prev = 0.0, hi_prev = 0.0;
  *drift = 0.0;
  const int k = (int)std::min<int64_t>(steps, n);
  for (int j = 0; j < k; ++j) {
    int rc = apply_term(ctx, t, C, W, s);
    if (rc) return rc;
    double alpha, beta2;
    if ((rc = dot_re(ctx, C, W, n, &alpha, s))) return rc;
    HIP_TRY(magnus::launch_lanczos_orth(W, C, P, alpha, beta_prev, n, s));
    if ((rc = dot_re(ctx, W, W, n, &beta2, s))) return rc;
    al.push_back(alpha);
    const double beta = std::sqrt(std::max(beta2, 0.0));
    if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(MAGNUS_ENAN, "Lanczos met a non-finite value");
    if (j + 1 == k || beta <= 1e-13 * (std::fabs(alpha) + 1.0)) break;  // done, or an invariant subspace
    be.push_back(beta);
    HIP_TRY(magnus::launch_scale(W, 1.0 / beta, P, n, s));  // P becomes the next vector
    std::swap(P, C);
    beta_prev = beta;
    if (j + 1 == k - 10) magnus::tridiag_extremes(al, be, &lo_prev, &hi_prev);
  }
  be.resize(al.size() - 1);
  magnus::tridiag_extremes(al, be, lo, hi);
  if ((int)al.size() > 10) *drift = std::max(std::fabs(*lo - lo_prev), std::fabs(*hi - hi_prev));
  return MAGNUS_OK;
}

}  // namespace

int magnus_spectral_bounds_lanczos(magnus_ctx* ctx, magnus_hamiltonian* h, int32_t steps, double margin,
                                   magnus_stream stream) {
  int rc = magnus_spectral_bounds(ctx, h, stream);  // validates; the Gershgorin enclosures cap the estimate
  if (rc) return rc;
  if (steps < 2 || !(margin >= 0.0)) return fail(MAGNUS_EINVAL, "steps %d < 2 or margin %g < 0", steps, margin);
  hipStream_t s = (hipStream_t)stream;
  for (magnus_term* t : {&h->H1, &h->H2}) {
    double lo, hi, drift;
    if ((rc = lanczos_term(ctx, *t, steps, &lo, &hi, &drift, s))) return rc;
    const double d = std::max(margin * (hi - lo), 3.0 * drift);
    t->lam_min = std::max(t->lam_min, lo - d);
    t->lam_max = std::min(t->lam_max, hi + d);
    if (t->lam_min > t->lam_max) t->lam_min = t->lam_max = 0.5 * (lo + hi);
  }
  const double n1 = std::fmax(std::fabs(h->H1.lam_min), std::fabs(h->H1.lam_max));
  const double n2 = std::fmax(std::fabs(h->H2.lam_min), std::fabs(h->H2.lam_max));
  h->k_min = -2.0 * n1 * n2;
  h->k_max = 2.0 * n1 * n2;
  return MAGNUS_OK;
}

int expmv_leja(magnus_ctx* ctx, const magnus_hamiltonian* h, double a, double b, double kappa, double tau,
               const void* v, void* w, int32_t batch, const magnus_leja_opts* opts, magnus_stats* stats,
               magnus_stream stream) {
  int rc = check_ham(ctx, h, kappa != 0.0);
  if (rc) return rc;
  if ((rc = check_opts(opts)) || (rc = check_batch(ctx, batch))) return rc;
  if (!v || !w) return fail(MAGNUS_EINVAL, "null state pointer");
  if (!is_fin(a) || !is_fin(b) || !is_fin(kappa) || !is_fin(tau))
    return fail(MAGNUS_EDOMAIN, "non-finite coefficient or step");
  if (kappa != 0.0 && h->H1.format != MAGNUS_CSR && !dense_comm_ready(ctx, h))
    return fail(MAGNUS_EINVAL, "dense commutator exponents need magnus_dense_commutator for this pair of terms");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = begin_call(ctx, s))) return rc;
  if ((rc = ensure_valid(ctx, h, s))) return rc;
  const int64_t dim = h->H1.dim;
  const double tol_e = per_exp_tol(opts, 1);
  Acc acc;
  acc.products_per_iter = kappa != 0.0 ? 4 : 2;
  const double2* vin = reinterpret_cast<const double2*>(v);
  double2* wout = reinterpret_cast<double2*>(w);
  for (int32_t c = 0; c < batch;) {
    const int g = (multi_ok(h, kappa) && tau != 0.0) ? group_for(ctx, h, batch - c) : 1;
    if (g > 1) {
      std::vector<double> av(g, a), bv(g, b);
      rc = multi_expmv_group(ctx, h, g, av.data(), bv.data(), tau, vin + c * dim, wout + c * dim, tol_e, opts, &acc, s);
    } else {
      rc = run_exponential(ctx, ExpOp{h, a, b, kappa}, tau, vin + c * dim, wout + c * dim, tol_e, opts, &acc, s);
    }
    if (rc) return rc;
    c += g;
  }
  return end_call(ctx, acc, tol_e, stats, s);
}

static int step_common(int method, magnus_ctx* ctx, const magnus_hamiltonian* h, double tau, double f1,
                       double f2, const void* psi_in, void* psi_out, int32_t batch,
                       const magnus_leja_opts* opts, magnus_stats* stats, magnus_stream stream) {
  int rc = check_ham(ctx, h, method == MAGNUS_M4);
  if (rc) return rc;
  if ((rc = check_opts(opts)) || (rc = check_batch(ctx, batch))) return rc;
  if (!psi_in || !psi_out) return fail(MAGNUS_EINVAL, "null state pointer");
  if (!is_fin(tau) || !is_fin(f1) || !is_fin(f2)) return fail(MAGNUS_EDOMAIN, "non-finite step or field value");
  if (method == MAGNUS_M4 && h->H1.format != MAGNUS_CSR && !dense_comm_ready(ctx, h))
    return fail(MAGNUS_EINVAL, "M4 on dense terms needs magnus_dense_commutator for this pair of terms");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = begin_call(ctx, s))) return rc;
  if ((rc = ensure_valid(ctx, h, s))) return rc;
  const int64_t dim = h->H1.dim;
  magnus::Scheme S;
  magnus::method_scheme(method, &S);
  const double fv[2] = {f1, f2};
  const double tol_e = per_exp_tol(opts, S.nexp);
  Acc acc;
  acc.products_per_iter = method == MAGNUS_M4 ? 4 : 2;
  const double2* in = reinterpret_cast<const double2*>(psi_in);
  double2* out = reinterpret_cast<double2*>(psi_out);
  for (int32_t c = 0; c < batch;) {
    const int g = (!S.commutator && multi_ok(h, 0.0)) ? group_for(ctx, h, batch - c) : 1;
    if (g > 1) {
      HIP_TRY(magnus::launch_pack(in + c * dim, ctx->vec(kY), (int)dim, g, s));
      rc = multi_cf_steps(ctx, h, S, g, tau, 0, 1, [&](int, int64_t, int j) { return fv[j]; }, tol_e, opts, &acc, s);
      if (rc) return rc;
      HIP_TRY(magnus::launch_unpack(ctx->vec(kY), out + c * dim, (int)dim, g, s));
    } else {
      rc = S.commutator ? m4_state(ctx, h, tau, f1, f2, in + c * dim, out + c * dim, tol_e, opts, &acc, s)
                        : cf_state(ctx, h, S, tau, fv, in + c * dim, out + c * dim, tol_e, opts, &acc, s);
    }
    if (rc) return rc;
    c += g;
  }
  return end_call(ctx, acc, tol_e, stats, s);
}

int magnus_step_cf4(magnus_ctx* ctx, const magnus_hamiltonian* h, double tau, double f1, double f2,
                    const void* psi_in, void* psi_out, int32_t batch, const magnus_leja_opts* opts,
                    magnus_stats* stats, magnus_stream stream) {
  return step_common(MAGNUS_CF4, ctx, h, tau, f1, f2, psi_in, psi_out, batch, opts, stats, stream);
}

int magnus_step_m4(magnus_ctx* ctx, const magnus_hamiltonian* h, double tau, double f1, double f2,
                   const void* psi_in, void* psi_out, int32_t batch, const magnus_leja_opts* opts,
                   magnus_stats* stats, magnus_stream stream) {
  return step_common(MAGNUS_M4, ctx, h, tau, f1, f2, psi_in, psi_out, batch, opts, stats, stream);
}

int magnus_step_cf4_noalloc(const magnus_hamiltonian* h, double tau, double f1, double f2, const void* psi_in,
                            void* psi_out, const magnus_leja_opts* opts, magnus_stats* stats, magnus_stream stream) {
  if (!h) return fail(MAGNUS_EINVAL, "null hamiltonian");
  if (h->H1.dim > kNoAllocMaxDim)
    return fail(MAGNUS_ENOMEM, "dim %lld exceeds the %lld entries the allocation-free scratch holds",
                (long long)h->H1.dim, (long long)kNoAllocMaxDim);
  magnus_ctx* ctx = nullptr;
  int rc = noalloc_context(&ctx);
  if (rc) return rc;
  return step_common(MAGNUS_CF4, ctx, h, tau, f1, f2, psi_in, psi_out, 1, opts, stats, stream);
}

int propagate(magnus_ctx* ctx, const magnus_hamiltonian* h, int32_t method, double tau, int64_t nsteps,
              const double* f_nodes, int32_t batch_f, void* psi, int32_t batch, void* checkpoints,
              int32_t every_k, const magnus_leja_opts* opts, magnus_stats* stats, magnus_stream stream) {
  magnus::Scheme S;
  if (!magnus::method_scheme(method, &S)) return fail(MAGNUS_EINVAL, "unknown method %d", method);
  int rc = check_ham(ctx, h, S.commutator);
  if (rc) return rc;
  if ((rc = check_opts(opts)) || (rc = check_batch(ctx, batch))) return rc;
  if (!psi) return fail(MAGNUS_EINVAL, "null state pointer");
  if (nsteps < 0) return fail(MAGNUS_EINVAL, "nsteps %lld < 0", (long long)nsteps);
  if (nsteps > 0 && !f_nodes) return fail(MAGNUS_EINVAL, "null f_nodes");
  if (batch_f != 1 && batch_f != batch) return fail(MAGNUS_EINVAL, "batch_f %d must be 1 or batch", batch_f);
  if (checkpoints && every_k < 1) return fail(MAGNUS_EINVAL, "every_k %d < 1", every_k);
  if (!is_fin(tau)) return fail(MAGNUS_EDOMAIN, "non-finite step");
  for (int64_t k = 0; k < S.q * nsteps * (int64_t)batch_f; ++k)
    if (!is_fin(f_nodes[k])) return fail(MAGNUS_EDOMAIN, "non-finite field value at node %lld", (long long)k);
  if (method == MAGNUS_M4 && h->H1.format != MAGNUS_CSR && !dense_comm_ready(ctx, h))
    return fail(MAGNUS_EINVAL, "M4 on dense terms needs magnus_dense_commutator for this pair of terms");
  if (S.sixth && !(h->H1.format == MAGNUS_DENSE ? dense_m6_ready(ctx, h) : csr_m6_ready(ctx, h)))
    return fail(MAGNUS_EINVAL, "M6 needs terms prepared by magnus_dense_m6_prepare or magnus_csr_m6_prepare");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = begin_call(ctx, s))) return rc;
  if ((rc = ensure_valid(ctx, h, s))) return rc;
  const int64_t dim = h->H1.dim;
  const int64_t exps = S.nexp * nsteps;
  const double tol_e = per_exp_tol(opts, exps);
  Acc acc;
  acc.products_per_iter = method == MAGNUS_M4 ? 4 : 2;
  double2* st = reinterpret_cast<double2*>(psi);
  double2* ck = reinterpret_cast<double2*>(checkpoints);
  const int64_t nck = checkpoints ? (nsteps + every_k - 1) / every_k + 1 : 0;
  const size_t stride = (size_t)dim * (size_t)batch;
  if (ck) HIP_TRY(hipMemcpyAsync(ck, st, sizeof(double2) * stride, hipMemcpyDeviceToDevice, s));
  auto fval = [&](int c, int64_t n, int j) {
    return f_nodes[((batch_f == 1 ? 0 : (int64_t)c) * nsteps + n) * S.q + j];
  };
  const bool grouped = !S.commutator && multi_ok(h, 0.0) && batch > 1;
  const bool small = !S.commutator && small_ok(ctx, h, batch);
  std::vector<SmallState> sst;
  if (small)
    for (int32_t c = 0; c < batch; ++c)
      sst.push_back(SmallState{0, st + c * dim, f_nodes + (batch_f == 1 ? 0 : (int64_t)c) * nsteps * S.q});
  // checkpoint steps: multiples of every_k and the last step
  auto next_stop = [&](int64_t n) {
    if (!ck) return nsteps;
    const int64_t k = ((n / every_k) + 1) * every_k;
    return std::min(k, nsteps);
  };
  // one state on the grid path with every stop test fused: one step captured,
  // replayed once per step
  GraphPlan G;
  const bool use_graph = batch == 1 && !small && tau != 0.0 && nsteps >= 2 && graph_eligible(ctx, h, S);
  if (use_graph) {
    if ((rc = graph_plan(ctx, h, S, tau, nsteps, [&](int64_t k, int j) { return fval(0, k, j); }, tol_e, opts, &G)))
      return rc;
    if ((rc = flush_fused_check(ctx, s))) return rc;
    if ((rc = graph_capture(ctx, h, S, G, st, tol_e, opts->early_termination))) return rc;
  }
  int64_t n = 0;
  while (n < nsteps) {
    const int64_t stop = next_stop(n);
    if (small) {
      rc = persist_steps(ctx, {h}, sst, S, tau, n, stop, tol_e, opts, &acc, s);
      if (rc) return rc;
    }
    for (int32_t c = small ? batch : 0; c < batch;) {
      const int g = grouped ? group_for(ctx, h, batch - c) : 1;
      if (g > 1) {
        HIP_TRY(magnus::launch_pack(st + c * dim, ctx->vec(kY), (int)dim, g, s));
        rc = multi_cf_steps(ctx, h, S, g, tau, n, stop,
                            [&](int cc, int64_t k, int j) { return fval(c + cc, k, j); }, tol_e, opts, &acc, s);
        if (rc) return rc;
        HIP_TRY(magnus::launch_unpack(ctx->vec(kY), st + c * dim, (int)dim, g, s));
      } else if (use_graph) {
        if ((rc = graph_replay(ctx, G, tau, n, stop, tol_e, opts, &acc, s))) return rc;
      } else {
        for (int64_t k = n; k < stop; ++k) {
          double2* y = st + c * dim;
          double fv[3];
          for (int j = 0; j < S.q; ++j) fv[j] = fval(c, k, j);
          rc = S.sixth        ? m6_state(ctx, h, tau, fv, y, y, tol_e, opts, &acc, s)
               : S.commutator ? m4_state(ctx, h, tau, fv[0], fv[1], y, y, tol_e, opts, &acc, s)
                              : cf_state(ctx, h, S, tau, fv, y, y, tol_e, opts, &acc, s);
          if (rc) return rc;
        }
      }
      c += g;
    }
    n = stop;
    if (ck) {
      const int64_t slot = n % every_k == 0 ? n / every_k : nck - 1;
      HIP_TRY(hipMemcpyAsync(ck + slot * stride, st, sizeof(double2) * stride, hipMemcpyDeviceToDevice, s));
    }
  }
  return end_call(ctx, acc, tol_e, stats, s);
}

int magnus_timing(magnus_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(MAGNUS_EINVAL, "null context");
  if (enable < 0) return fail(MAGNUS_EINVAL, "timing stride %d", enable);
  HIP_TRY(hipSetDevice(ctx->device));
  if (enable) {
    HIP_TRY(hipDeviceSynchronize());  // pooled events may still be pending
    ctx->records.clear();
    ctx->pool_used = 0;
    for (auto& k : ctx->timing_seq) k = 0;
  }
  ctx->timing = enable;
  return MAGNUS_OK;
}

int magnus_timing_read(magnus_ctx* ctx, int32_t kind, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches) return fail(MAGNUS_EINVAL, "null argument");
  if (kind < MAGNUS_KERNEL_CSR_LEJA || kind > MAGNUS_KERNEL_CSR_LEJA3) return fail(MAGNUS_EINVAL, "kernel class %d", kind);
  HIP_TRY(hipSetDevice(ctx->device));
  double t = 0.0;
  int64_t n = 0;
  for (auto& r : ctx->records) {
    if (std::get<0>(r) != kind) continue;
    HIP_TRY(hipEventSynchronize(std::get<2>(r)));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, std::get<1>(r), std::get<2>(r)));
    t += ms;
    ++n;
  }
  *total_ms = t;
  *launches = n;
  return MAGNUS_OK;
}

int magnus_propagate_ragged(magnus_ctx* ctx, const magnus_problem* probs, int32_t nprob, int32_t method,
                            double tau, int64_t nsteps, const magnus_leja_opts* opts, magnus_stats* stats,
                            magnus_stream stream) {
  if (!ctx) return fail(MAGNUS_EINVAL, "null context");
  if (!probs || nprob < 1) return fail(MAGNUS_EINVAL, "no problems");
  magnus::Scheme S;
  if (!magnus::method_scheme(method, &S)) return fail(MAGNUS_EINVAL, "unknown method %d", method);
  int rc = check_opts(opts);
  if (rc) return rc;
  if (nsteps < 0 || !is_fin(tau)) return fail(MAGNUS_EINVAL, "bad nsteps or tau");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = begin_call(ctx, s))) return rc;
  for (int32_t i = 0; i < nprob; ++i) {
    const magnus_problem& P = probs[i];
    if ((rc = check_ham(ctx, &P.h, method == MAGNUS_M4))) return rc;
    if (!P.psi || P.batch < 1 || (P.batch_f != 1 && P.batch_f != P.batch) || (nsteps > 0 && !P.f_nodes))
      return fail(MAGNUS_EINVAL, "problem %d: bad state, batch or field", i);
    for (int64_t k = 0; k < S.q * nsteps * (int64_t)P.batch_f; ++k)
      if (!is_fin(P.f_nodes[k])) return fail(MAGNUS_EDOMAIN, "problem %d: non-finite field value", i);
    if ((rc = ensure_valid(ctx, &P.h, s))) return rc;
  }
  const double tol_e = per_exp_tol(opts, S.nexp * nsteps);
  Acc acc;
  // small problems (product-of-exponentials methods): every state in one persistent launch
  std::vector<const magnus_hamiltonian*> hs;
  std::vector<SmallState> sst;
  std::vector<int> big;
  // every CSR problem of at most kSmallDim rows joins the persistent launches:
  // the alternative here is a batched propagation per problem with a host
  // wait after it, which costs more than the single-call crossover assumes
  for (int32_t i = 0; i < nprob; ++i) {
    const magnus_problem& P = probs[i];
    if (!S.commutator && small_ok(ctx, &P.h, std::max<int64_t>(32, P.batch))) {
      const int pi = (int)hs.size();
      hs.push_back(&P.h);
      double2* psi = reinterpret_cast<double2*>(P.psi);
      for (int32_t c = 0; c < P.batch; ++c)
        sst.push_back(
            SmallState{pi, psi + c * P.h.H1.dim, P.f_nodes + (P.batch_f == 1 ? 0 : (int64_t)c) * nsteps * S.q});
    } else {
      big.push_back(i);
    }
  }
  // the large problems together when they have the same batch and fit the
  // workspace at once: each split into groups of JB states (the group size
  // tuned for the largest of them, else the largest that divides the batch),
  // one launch per Leja iteration for all groups, their control slots after
  // the small states' (no reset, no host wait between problems)
  bool joint = ctx->ragged_joint && !S.commutator && big.size() >= 2;
  int JB = 0;
  if (joint) {
    const int batch = probs[big[0]].batch;
    int largest = big[0];
    for (int i : big)
      if (probs[i].h.H1.dim > probs[largest].h.H1.dim) largest = i;
    JB = group_for(ctx, &probs[largest].h, batch);
    while (JB > 1 && batch % JB != 0) JB /= 2;
    size_t vtot = 0, ptot = 0, groups = 0;
    for (int i : big) {
      const magnus_problem& P = probs[i];
      joint = joint && P.h.H1.format == MAGNUS_CSR && P.batch == batch;
      vtot += (size_t)P.h.H1.dim * batch;
      if (JB >= 2) ptot += (size_t)magnus::ragged_grid((int)P.h.H1.dim, JB) * JB * 2 * (batch / JB);
      groups += JB >= 2 ? (size_t)(batch / JB) : 0;
    }
    joint = joint && JB >= 2 && JB <= ctx->max_batch && groups <= (size_t)magnus::kMaxRagged &&
            vtot <= (size_t)ctx->max_dim * (size_t)ctx->max_batch && ptot <= ctx->npartials &&
            sst.size() + groups * (size_t)JB <= (size_t)ctx->nslots;
  }
  if (joint && nsteps > 0) {
    std::vector<RagProblem> R;
    size_t voff = 0, poff = 0;
    int slot0 = (int)sst.size();
    for (int i : big) {
      const magnus_problem& P = probs[i];
      for (int c0 = 0; c0 < P.batch; c0 += JB) {
        R.push_back(RagProblem{&P, c0, voff, slot0, poff});
        voff += (size_t)P.h.H1.dim * JB;
        poff += (size_t)magnus::ragged_grid((int)P.h.H1.dim, JB) * JB * 2;
        slot0 += JB;
      }
    }
    if ((rc = ragged_joint_steps(ctx, R, S, JB, tau, nsteps, tol_e, opts, &acc, s))) return rc;
    big.clear();
  }
  // the large problems first: each is one batched propagation (which resets the control slots)
  for (int i : big) {
    const magnus_problem& P = probs[i];
    if (P.batch > ctx->max_batch) return fail(MAGNUS_ENOMEM, "problem %d: batch %d exceeds max_batch", i, P.batch);
    magnus_leja_opts o = *opts;
    o.tol = tol_e;
    o.tol_mode = 0;
    magnus_stats ps{};
    // with stats, so a non-finite norm in this problem surfaces here (the slots are reset afterwards)
    rc = propagate(ctx, &P.h, method, tau, nsteps, P.f_nodes, P.batch_f, P.psi, P.batch, nullptr, 1, &o, &ps,
                   stream);
    if (rc) return rc;
    acc.exponentials += ps.exponentials;
    acc.substeps += ps.substeps;
    acc.planned += ps.planned_iters;
    acc.max_m = std::max(acc.max_m, ps.max_degree_used);
    acc.max_s = std::max(acc.max_s, ps.max_substeps_used);
    acc.max_bound = std::max(acc.max_bound, ps.max_err_bound);
    acc.extra_iters += ps.iters;  // counted by the nested call
  }
  if (!sst.empty() && nsteps > 0) {
    if (!big.empty()) HIP_TRY(magnus::launch_slot_reset(ctx->slots, ctx->nslots, s));
    // one launch per group of at most nslots states (one control slot each); the
    // slots keep counting, so groups after the first are folded into extra_iters
    for (size_t g0 = 0; g0 < sst.size(); g0 += (size_t)ctx->nslots) {
      const size_t g1 = std::min(sst.size(), g0 + (size_t)ctx->nslots);
      if (g0 > 0) {
        long long it = 0;
        int st = 0;
        if ((rc = read_slots(ctx, s, &it, &st))) return rc;  // the previous group's counters and status
        acc.extra_iters += it;
        ctx->sticky_status |= st;
        HIP_TRY(magnus::launch_slot_reset(ctx->slots, ctx->nslots, s));
      }
      std::vector<SmallState> part(sst.begin() + (long)g0, sst.begin() + (long)g1);
      if ((rc = persist_steps(ctx, hs, part, S, tau, 0, nsteps, tol_e, opts, &acc, s))) return rc;
    }
  }
  return end_call(ctx, acc, tol_e, stats, s);
}

int64_t magnus_adjoint_workspace_bytes(int64_t dim, int64_t nsteps, int32_t every_k) {
  if (dim < 1 || nsteps < 1 || every_k < 1) return -1;
  const int64_t k = std::min<int64_t>(every_k, nsteps);
  const int64_t nck = (nsteps + k - 1) / k + 1;
  const int64_t vecs = nck + (k + 1) + k + 2 + 4;
  return (vecs * dim + 2 * nsteps + 1) * (int64_t)sizeof(double2);
}

int magnus_propagate_adjoint(magnus_ctx* ctx, const magnus_hamiltonian* h, double tau, int64_t nsteps,
                             const double* f_nodes, const double* df_nodes, int32_t nparams, const void* psi0,
                             const void* psi_target, int32_t every_k, void* workspace, int64_t workspace_bytes,
                             double* loss, double* grad, const magnus_leja_opts* opts, magnus_stats* stats,
                             magnus_stream stream) {
  int rc = check_ham(ctx, h, 0);
  if (rc) return rc;
  if ((rc = check_opts(opts))) return rc;
  if (ctx->max_batch < 2) return fail(MAGNUS_ENOMEM, "the adjoint needs a context with max_batch >= 2");
  if (nsteps < 1 || nparams < 0 || every_k < 1) return fail(MAGNUS_EINVAL, "nsteps, nparams or every_k out of range");
  if (!f_nodes || (nparams > 0 && !df_nodes) || !psi0 || !psi_target || !workspace || !loss || (nparams > 0 && !grad))
    return fail(MAGNUS_EINVAL, "null argument");
  if (!is_fin(tau)) return fail(MAGNUS_EDOMAIN, "non-finite step");
  for (int64_t i = 0; i < 2 * nsteps; ++i)
    if (!is_fin(f_nodes[i])) return fail(MAGNUS_EDOMAIN, "non-finite field value");
  for (int64_t i = 0; i < 2 * nsteps * (int64_t)nparams; ++i)
    if (!is_fin(df_nodes[i])) return fail(MAGNUS_EDOMAIN, "non-finite field derivative");
  const int64_t need = magnus_adjoint_workspace_bytes(h->H1.dim, nsteps, every_k);
  if (workspace_bytes < need)
    return fail(MAGNUS_ENOMEM, "workspace of %lld bytes, need %lld", (long long)workspace_bytes, (long long)need);
  hipStream_t s = (hipStream_t)stream;
  if ((rc = begin_call(ctx, s))) return rc;
  if ((rc = ensure_valid(ctx, h, s))) return rc;

  const int64_t dim = h->H1.dim;
  const int64_t k = std::min<int64_t>(every_k, nsteps);
  const int64_t nck = (nsteps + k - 1) / k + 1;
  const int64_t nseg = (nsteps + k - 1) / k;
  double2* base = reinterpret_cast<double2*>(workspace);
  double2* ck = base;                       // nck states
  double2* seg_psi = ck + nck * dim;        // k + 1 states
  double2* seg_phi = seg_psi + (k + 1) * dim;  // k states
  double2* lam = seg_phi + k * dim;
  double2* mu = lam + dim;
  double2* X2 = mu + dim;                   // interleaved pair
  double2* Y2 = X2 + 2 * dim;
  double2* g = Y2 + 2 * dim;                // 2 nsteps + 1 complex
  const double tol_e = per_exp_tol(opts, 2 * nsteps);
  Acc acc;
  auto beta_of = [&](int64_t n) { return magnus::kAlpha2 * f_nodes[2 * n] + magnus::kAlpha1 * f_nodes[2 * n + 1]; };
  auto gamma_of = [&](int64_t n) { return magnus::kAlpha1 * f_nodes[2 * n] + magnus::kAlpha2 * f_nodes[2 * n + 1]; };
  const double2* tgt = reinterpret_cast<const double2*>(psi_target);

  // forward sweep with checkpoints (state kept in mu)
  HIP_TRY(hipMemcpyAsync(ck, psi0, sizeof(double2) * dim, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(mu, psi0, sizeof(double2) * dim, hipMemcpyDeviceToDevice, s));
  magnus::Scheme cf4;
  magnus::method_scheme(MAGNUS_CF4, &cf4);
  for (int64_t n = 0; n < nsteps; ++n) {
    rc = cf_state(ctx, h, cf4, tau, f_nodes + 2 * n, mu, mu, tol_e, opts, &acc, s);
    if (rc) return rc;
    if ((n + 1) % k == 0 || n + 1 == nsteps) {
      const int64_t slot = (n + 1) % k == 0 ? (n + 1) / k : nck - 1;
      HIP_TRY(hipMemcpyAsync(ck + slot * dim, mu, sizeof(double2) * dim, hipMemcpyDeviceToDevice, s));
    }
  }
  if ((rc = flush_fused_check(ctx, s))) return rc;
  HIP_TRY(magnus::launch_cdot(tgt, 1, mu, 1, dim, ctx->partials, g + 2 * nsteps, s));
  HIP_TRY(hipMemcpyAsync(lam, tgt, sizeof(double2) * dim, hipMemcpyDeviceToDevice, s));

  const double half[2] = {0.5, 0.5};
  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const int64_t n0 = seg * k, n1 = std::min(n0 + k, nsteps);
    // recompute psi_n and the half-step states phi_n of the segment
    HIP_TRY(hipMemcpyAsync(seg_psi, ck + seg * dim, sizeof(double2) * dim, hipMemcpyDeviceToDevice, s));
    for (int64_t n = n0; n < n1; ++n) {
      double2* p0 = seg_psi + (n - n0) * dim;
      double2* ph = seg_phi + (n - n0) * dim;
      rc = run_exponential(ctx, ExpOp{h, 0.5, beta_of(n), 0.0}, tau, p0, ph, tol_e, opts, &acc, s);
      if (rc) return rc;
      rc = run_exponential(ctx, ExpOp{h, 0.5, gamma_of(n), 0.0}, tau, ph, p0 + dim, tol_e, opts, &acc, s);
      if (rc) return rc;
    }
    // block (Frechet) exponentials of the segment, planned and uploaded together
    std::vector<ColParam> table;
    std::vector<MultiExp> ea(n1 - n0), eb(n1 - n0);
    for (int64_t n = n0; n < n1; ++n) {
      const double ga2[2] = {gamma_of(n), gamma_of(n)}, be2[2] = {beta_of(n), beta_of(n)};
      rc = plan_multi(h, half, ga2, 2, tau, tol_e, opts, 1, &table, &ea[n - n0], &acc);
      if (rc) return rc;
      rc = plan_multi(h, half, be2, 2, tau, tol_e, opts, 1, &table, &eb[n - n0], &acc);
      if (rc) return rc;
    }
    if ((rc = upload_table(ctx, table, s))) return rc;
    for (int64_t n = n1 - 1; n >= n0; --n) {
      MultiExp A = ea[n - n0], Bx = eb[n - n0];
      A.src = X2;
      A.dst = Y2;
      Bx.src = X2;
      Bx.dst = Y2;
      // g_a(n) = lambda_{n+1}^H L_a phi_n
      HIP_TRY(magnus::launch_frechet_init(seg_phi + (n - n0) * dim, X2, (int)dim, s));
      if ((rc = launch_multi(ctx, h, A, tol_e, opts->early_termination, s))) return rc;
      if ((rc = flush_fused_check(ctx, s))) return rc;
      HIP_TRY(magnus::launch_cdot(lam, 1, Y2, 2, dim, ctx->partials, g + 2 * n, s));
      // mu_n = E_a^H lambda_{n+1}
      rc = run_exponential(ctx, ExpOp{h, 0.5, gamma_of(n), 0.0}, -tau, lam, mu, tol_e, opts, &acc, s);
      if (rc) return rc;
      // g_b(n) = mu_n^H L_b psi_n
      HIP_TRY(magnus::launch_frechet_init(seg_psi + (n - n0) * dim, X2, (int)dim, s));
      if ((rc = launch_multi(ctx, h, Bx, tol_e, opts->early_termination, s))) return rc;
      if ((rc = flush_fused_check(ctx, s))) return rc;
      HIP_TRY(magnus::launch_cdot(mu, 1, Y2, 2, dim, ctx->partials, g + 2 * n + 1, s));
      // lambda_n = E_b^H mu_n
      rc = run_exponential(ctx, ExpOp{h, 0.5, beta_of(n), 0.0}, -tau, mu, lam, tol_e, opts, &acc, s);
      if (rc) return rc;
    }
  }
  std::vector<double2> hg(2 * nsteps + 1);
  HIP_TRY(hipMemcpyAsync(hg.data(), g, sizeof(double2) * hg.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const std::complex<double> z(hg[2 * nsteps].x, hg[2 * nsteps].y);
  *loss = 1.0 - std::norm(z);
  for (int32_t p = 0; p < nparams; ++p) {
    std::complex<double> dz = 0.0;
    for (int64_t n = 0; n < nsteps; ++n) {
      const double d1 = df_nodes[(2 * n) * nparams + p], d2v = df_nodes[(2 * n + 1) * nparams + p];
      const double dbeta = magnus::kAlpha2 * d1 + magnus::kAlpha1 * d2v;
      const double dgamma = magnus::kAlpha1 * d1 + magnus::kAlpha2 * d2v;
      dz += dgamma * std::complex<double>(hg[2 * n].x, hg[2 * n].y) +
            dbeta * std::complex<double>(hg[2 * n + 1].x, hg[2 * n + 1].y);
    }
    grad[p] = -2.0 * std::real(std::conj(z) * dz);
  }
  return end_call(ctx, acc, tol_e, stats, s);
}

int magnus_method_nodes(int32_t method) {
  magnus::Scheme S;
  if (!magnus::method_scheme(method, &S)) return fail(MAGNUS_EINVAL, "unknown method %d", method);
  return S.q;
}

int magnus_quadrature_nodes(int32_t method, double t0, double tau, int64_t nsteps, double* t_out) {
  magnus::Scheme S;
  if (!magnus::method_scheme(method, &S)) return fail(MAGNUS_EINVAL, "unknown method %d", method);
  if (nsteps < 0 || (nsteps > 0 && !t_out)) return fail(MAGNUS_EINVAL, "bad output");
  for (int64_t n = 0; n < nsteps; ++n) {
    const double tn = t0 + (double)n * tau;
    for (int j = 0; j < S.q; ++j) t_out[S.q * n + j] = tn + S.c[j] * tau;
  }
  return MAGNUS_OK;
}

int magnus_leja_points(int32_t m, double* xi) {
  if (m < 0 || m >= magnus::kNumPoints || !xi) return fail(MAGNUS_EINVAL, "m %d outside 0..%d", m, magnus::kNumPoints - 1);
  const auto& p = magnus::leja_points();
  for (int k = 0; k <= m; ++k) xi[k] = p[k];
  return MAGNUS_OK;
}

int magnus_divided_differences(double theta, int32_t m, double* d) {
  if (m < 0 || m >= magnus::kNumPoints || !d) return fail(MAGNUS_EINVAL, "m %d outside 0..%d", m, magnus::kNumPoints - 1);
  if (!is_fin(theta) || std::fabs(theta) > magnus::kThetaCap)
    return fail(MAGNUS_EDOMAIN, "|theta| %g above %g", theta, magnus::kThetaCap);
  std::vector<std::complex<double>> v(m + 1);
  magnus::divided_differences(theta, m, v.data());
  for (int k = 0; k <= m; ++k) { d[2 * k] = v[k].real(); d[2 * k + 1] = v[k].imag(); }
  return MAGNUS_OK;
}

double magnus_leja_error(double theta, int32_t m) {
  if (!is_fin(theta) || std::fabs(theta) > magnus::kThetaCap) return INFINITY;
  return magnus::leja_error(theta, m);
}

int magnus_leja_plan(double theta, double tol, int32_t max_degree, int32_t max_substeps, int32_t* m, int32_t* s,
                     double* bound) {
  if (!m || !s || !bound) return fail(MAGNUS_EINVAL, "null output");
  if (!(tol > 0.0) || !is_fin(theta)) return fail(MAGNUS_EDOMAIN, "bad theta or tol");
  magnus::LejaPlan p;
  if (!magnus::plan_degree(theta, tol, max_degree, max_substeps, &p))
    return fail(MAGNUS_ENOCONV, "caps cannot reach tol %g at theta %g", tol, theta);
  *m = p.m;
  *s = p.s;
  *bound = p.bound;
  return MAGNUS_OK;
}

}  // extern "C"
