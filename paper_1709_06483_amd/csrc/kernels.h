// Internal device-side interface of libmagnus: kernel launchers used by the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace magnus {

// Per-state control block in device memory.  One Leja substep runs as a
// sequence of iteration kernels, each followed by a one-workgroup kernel that
// reduces the norm partials in a fixed order, evaluates the early-termination
// test and writes the verdict here for the next iteration to read; or, on
// small grids, with that reduction and test made at the start of the next
// iteration kernel by each of its workgroups (IterArgs::fused).
struct Slot {
  unsigned int counter;   // unused (kept zero)
  int stopped;            // 1: the current substep has terminated early
  int iters_sub;          // iterations done in the current substep
  int status;             // sticky: bit 0 = non-finite norm seen
  long long iters_total;  // sticky: Leja iterations executed since the last reset
  double vnorm;           // |v| of the current substep
  double prev_term;       // |d_{i-1}| |w_{i-1}|
  double last_est;        // last early-termination estimate
  double term[2];         // fused stop test: |d_i| |w_i| of iteration i at term[i & 1]
};

struct CsrDev {
  const int* rp;
  const int* ci;
  const double2* val;
};

enum IterMode : int {
  kLeja = 0,       // y = a1 H1 x1 + a2 H2 x2, then the Leja update
  kSplit = 1,      // out1 = H1 x1, out2 = H2 x2 (first half of a commutator pass)
  kLejaComm = 2,   // y = a1 x2 + a2 x1 + i k (H1 x1 - H2 x2), then the Leja update
  kSplitComm = 3,  // out1 = a1 x + i k H2 x, out2 = a2 x - i k H1 x with x = x1 = x2 = wcur
                   // (streamed kernel only; kLeja over out1, out2 with a1 = a2 = 1 completes it)
};

// The coefficients of one Leja iteration of one Magnus step, read from device
// memory by launches that a captured graph replays once per step: record
// coef[step * stride] of the launch's table column, with `step` a device
// counter the graph advances at its end.  Iterations past the step's own
// degree (the graph holds the largest degree of the call) are inactive.
struct IterCoef {
  double a1, a2, kap, sigma;
  double dre, dim, d0re, d0im;
  double dabs, d0abs, prev_dabs, tol;
  int active;
  int pad;
};

// One Leja iteration: w_i = X w_{i-1} - xi_{i-1} w_{i-1}, p += d_i w_i, where
// X w = a1 (H1 w) + a2 (H2 w) [+ k K w] - c' w has been folded into the
// coefficients below (sigma = scale * c + xi_{i-1}).
struct IterArgs {
  const double2* x1;    // vector gathered by term 1
  const double2* x2;    // vector gathered by term 2
  const double2* wcur;  // w_{i-1} (own rows); v for the first iteration
  double2* wout;        // w_i            (kSplit: H1 x1)
  double2* pacc;        // p accumulator  (kSplit: H2 x2)
  Slot* slot;
  double* partials;     // 2 * grid doubles
  double a1, a2, kap;
  double sigma;
  double2 d;            // d_i
  double2 d0;           // d_0 (first iteration)
  double dabs;          // |d_i|
  double d0abs;         // |d_0|
  double tol;           // early-termination threshold relative to |v|
  int early;            // early termination enabled
  int first;            // first iteration of a substep
  int check_stop;       // return at once if the substep has stopped
  // Fused stop test (no decide kernel between iterations): every workgroup of
  // iteration `iter` reduces iteration iter-1's partials itself, in one fixed
  // order, and applies the early-termination test; workgroup 0 records the
  // verdict and counts the iteration in the slot.
  int fused;
  int iter;                    // iteration index within the substep (1-based)
  const double* prev_partials; // iteration iter-1's partials (its |v|^2 partials follow when iter == 2)
  int prev_grid;               // workgroups of iteration iter-1
  double prev_dabs;            // |d_{iter-1}|
  // Table mode (graph replay): the coefficients above come from
  // coef[*step * coef_stride]; unit_a keeps a1 = a2 = 1 (the second pass of a
  // streamed commutator iteration); skip is set for an inactive record.
  const IterCoef* coef;
  const int* step;
  int coef_stride;
  int unit_a;
  int skip;
};

// Row-block selector of launch_csr2_iter: 16 or 64 rows per workgroup with
// the nonzero-streaming kernel, or -32, -64, -128 for the row-per-lane kernel
// with that many rows per workgroup.
constexpr int kRowLane = -64;
// kWaveTile + R selects the wave-tile kernel with R rows per wave (R = 8, 16;
// four waves per workgroup).
constexpr int kWaveTile = 1000;
// kStreamTile selects the streaming wave-tile kernel (modes kLeja and kSplitComm): every
// wave walks 8 tiles of 8 rows, copying each tile's entries into LDS one tile
// ahead.
constexpr int kStreamTile = 2000;

// Launch one iteration over `dim` rows of the two CSR terms.
hipError_t launch_csr2_iter(int mode, const CsrDev& t1, const CsrDev& t2, int dim,
                            const IterArgs& a, int rows_per_block, hipStream_t s);

// Grid size (workgroups) of launch_csr2_iter for `dim` rows.
int csr2_grid(int dim, int rows_per_block);

// CSR entries (both terms, from the start of the matrix) that the iteration
// kernels read with normal loads so that they stay in the 256 MiB MALL from
// one pass over the matrix to the next; the rest are read non-temporally.
int csr_keep_entries(int dim);

// Method M6 on CSR terms, one Leja iteration in two passes over the five
// matrices (H1, H2, K, P1, P2).  Stage A: with s_k = M_k w,
//   y0 = sum_k c_k s_k, u1 = i(c5 s3 + c6 s4), u2 = i c7 s4,
//   u3 = -i(c8 s3 + c9 s4), u4 = i(c8 s2 - c5 s0), u5 = i(c9 s2 - c6 s0 - c7 s1);
// stage B: y = y0 + sum_k M_k u_{k+1}, then the Leja update from y (the
// Hermitian exponent times w_{i-1}) with its norm partials (grid m6_grid for
// the decide kernel).  Both return at once when check_stop and the slot's
// substep has stopped.
constexpr int kM6Terms = 5;
struct M6Terms {
  CsrDev m[kM6Terms];
};
struct M6Coef {
  double c[10];
};
struct M6Vecs {
  double2* u[kM6Terms];  // stage B's input vectors, in the order of M6Terms
  double2* y0;
};
hipError_t launch_m6_stage_a(const M6Terms& T, const double2* w, const M6Coef& C, const M6Vecs& V, int dim,
                             const Slot* slot, int check_stop, hipStream_t s);
hipError_t launch_m6_stage_b(const M6Terms& T, const M6Vecs& V, double scale, int dim, const IterArgs& a,
                             hipStream_t s);
int m6_grid(int dim);

// The streaming kernel (kernels_stream.hip).
hipError_t launch_csr2_stream(int mode, const CsrDev& t1, const CsrDev& t2, int dim, const IterArgs& a,
                              hipStream_t s);
int csr2_stream_grid(int dim);

// Gershgorin enclosure and structural check of one CSR term.  Writes per
// workgroup min, max and a "malformed" flag into out[3 * grid].
hipError_t launch_csr_gershgorin(const CsrDev& t, int dim, long long nnz, double* out, int grid,
                                 hipStream_t s);
int csr_gershgorin_grid(int dim);

// Gershgorin enclosure of a dense row-major term (out[2 * grid]).
hipError_t launch_dense_gershgorin(const double2* H, int dim, long long ld, double* out, int grid,
                                   hipStream_t s);
int dense_gershgorin_grid(int dim);

// Inputs of the first dense iteration fused with the assembly of its exponent:
// out = ca H1 + cb H2 (+ ck K), H1 and H2 with row stride ld, K (optional)
// and out with row stride dim.
struct DenseAssembly {
  const double2* H1;
  const double2* H2;
  const double2* K;
  long long ld;
  double ca, cb, ck;
  double2* out;
};
hipError_t launch_dense_assemble_iter(const DenseAssembly& D, int dim, const IterArgs& a, hipStream_t s, int rpw);
// Dense Leja iteration (mode kLeja only): two terms, or one (an assembled
// exponent) when H2 is null.
// rpw: rows per wave (1, 2 or 4).
hipError_t launch_dense2_iter(const double2* H1, const double2* H2, int dim, long long ld,
                              const IterArgs& a, hipStream_t s, int rpw = 2);
int dense2_grid(int dim, int nterms, int rpw = 2);

// Reduce the norm partials of the iteration launched just before (grid
// workgroups) and write the early-termination verdict into the slot.
hipError_t launch_leja_decide(const IterArgs& a, int grid, hipStream_t s);
// After the last fused iteration of a call: flag a non-finite norm of that
// iteration (a.prev_partials, a.prev_grid, a.iter = the iteration after it)
// unless its substep had stopped.
hipError_t launch_leja_final_check(const IterArgs& a, hipStream_t s);
// Largest grid of an iteration launch that makes its own stop decision
// (each workgroup reads every partial sum of the previous iteration; measured
// on chains, Cf4 steps/s with the decide kernel / fused: n = 13 (512
// workgroups) 7,786 / 9,448, n = 14 (1,024) 6,664 / 7,525, n = 15 (2,048)
// 4,987 / 5,095, n = 16 (2,048 wave tiles) 3,796 / 3,640).
constexpr int kFuseMaxGrid = 1024;
// Step counter of graph replays: set to zero, advanced by one.
hipError_t launch_step_set(int* ctr, int value, hipStream_t s);
hipError_t launch_step_advance(int* ctr, hipStream_t s);

// ---- several states at once (states interleaved: element (row, b) at row*B + b) ----

constexpr int kMaxCols = 32;

// Leja parameters of one state (column) for one iteration.
struct ColParam {
  double a1, a2;        // scale * a, scale * b
  double sigma;         // scale * c + xi_{i-1}
  double dre, dim;      // d_i
  double dabs;          // |d_i|
  double d0re, d0im;    // d_0
  double d0abs;         // |d_0|
  double coup;          // Frechet coupling (scale * 1 for the H2 block), 0 otherwise
};

struct MultiArgs {
  const double2* x;     // w_{i-1} (v on the first iteration), interleaved
  double2* wout;        // w_i
  double2* pacc;        // p
  Slot* slots;          // one per column
  double* partials;     // [grid][B][2]
  const ColParam* prm;  // B entries for this iteration
  int B;
  int first;
  int check_stop;
  int early;
  double tol;
  int joint;            // 1: the B columns form one block vector (shared stop test)
};

enum MultiMode : int { kMultiLeja = 0, kMultiFrechet = 1 };

int csr2_multi_grid(int dim, int B);
// One Leja iteration for B interleaved states sharing H1, H2 (B in 2, 4, 8, 16, 32).
// kMultiFrechet (B == 2): columns (x, y) of the block vector of [[H, H2], [0, H]].
hipError_t launch_csr2_multi(int mode, const CsrDev& t1, const CsrDev& t2, int dim, const MultiArgs& a,
                             hipStream_t s);
// Per-column (or joint) reduction of the partials and stop verdicts.
hipError_t launch_multi_decide(const MultiArgs& a, int grid, hipStream_t s);

// Several problems of B interleaved states each (own CSR terms, states,
// coefficients, slots and partials) in one launch per Leja iteration, then
// one decision launch for all their columns.  block0, col0, keep_entries and
// nblocks are filled by launch_csr2_ragged; problem q's partials take
// ragged_grid(dim, B) * B * 2 doubles.
constexpr int kMaxRagged = 8;
struct RaggedProblem {
  CsrDev t1, t2;
  int dim;
  int block0;        // first workgroup of the problem
  int col0;          // first decision workgroup of the problem
  int keep_entries;  // matrix entries read with normal loads (MALL-resident)
  MultiArgs a;
};
struct RaggedArgs {
  RaggedProblem p[kMaxRagged];
  int np;
  int nblocks;
};
int ragged_grid(int dim, int B);
hipError_t launch_csr2_ragged(RaggedArgs r, int B, hipStream_t s);
// Interleave / de-interleave B states of dim entries (optionally scaling by a
// per-state phase is not needed: plain copies).
hipError_t launch_pack(const double2* src, double2* dst, int dim, int B, hipStream_t s);
hipError_t launch_unpack(const double2* src, double2* dst, int dim, int B, hipStream_t s);

// Dense group iteration as an FP64 MFMA GEMM fused with the Leja update
// (nterms = 1: H1 only, y_b = a1_b H1 w_b; nterms = 2: y_b = H1 (a1_b w_b) + H2 (a2_b w_b)).
// Partials are written per 32-row block: decide with dense_mfma_row_blocks(dim).
// tile: 0 32 x 64 with K split in two (default), 1 32 x 64, 2 64 x 64,
// 3 64 x 64 with K split in two, 4 32 x 128 with K split in two (rows x states).
constexpr int kMfmaTiles = 7;
hipError_t launch_dense_mfma(int nterms, const double2* H1, const double2* H2, long long ld, int dim,
                             const MultiArgs& a, hipStream_t s, int tile = 0);
int dense_mfma_row_blocks(int dim);
// out = ca H1 + cb H2 (dim x dim, row stride ld in, dim out).
// out = ca H1 + cb H2 + ck K (H1, H2 with row stride ld; K, if not null, and
// out with row stride dim).
hipError_t launch_dense_assemble(const double2* H1, const double2* H2, long long ld, int dim, double ca, double cb,
                                 const double2* K, double ck, double2* out, hipStream_t s);

// C = A B (n x n complex128, row strides lda, ldb in, n out) on the FP64 matrix cores.
hipError_t launch_zgemm(const double2* A, long long lda, const double2* B, long long ldb, double2* C, int n,
                        hipStream_t s);
// K = scale i (C - C^H), n x n with row stride n.
hipError_t launch_commutator_combine(const double2* C, int n, double scale, double2* K, hipStream_t s);

// out = sum_t c[t] m[t] (m[t] with row stride ld[t], out with row stride n).
constexpr int kMaxAssembleTerms = 10;
struct AssembleTerms {
  const double2* m[kMaxAssembleTerms];
  long long ld[kMaxAssembleTerms];
  double c[kMaxAssembleTerms];
  int nterms;
};
hipError_t launch_assemble_terms(const AssembleTerms& T, int n, double2* out, hipStream_t s);

// Dense Frechet block iteration (B == 2 interleaved pair, joint stop test);
// decide with dense_frechet_grid(dim) workgroups.
hipError_t launch_dense_frechet(const double2* H1, const double2* H2, int dim, long long ld, const MultiArgs& a,
                                hipStream_t s);
int dense_frechet_grid(int dim);

// out = sum_i conj(x[i*sx]) y[i*sy] (fixed order; partials: kDotPartials doubles).
constexpr int kDotPartials = 1024;
hipError_t launch_cdot(const double2* x, long long sx, const double2* y, long long sy, long long n, double* partials,
                       double2* out, hipStream_t s);
// Lanczos helpers: w <- w - alpha v - beta u; y = sc x.
hipError_t launch_lanczos_orth(double2* w, const double2* v, const double2* u, double alpha, double beta, long long n,
                               hipStream_t s);
hipError_t launch_scale(const double2* x, double sc, double2* y, long long n, hipStream_t s);
// dst (interleaved pair) = [0; v].
hipError_t launch_frechet_init(const double2* v, double2* dst, int dim, hipStream_t s);

// ---- assembled CSR commutator (Method M4 on CSR terms) ----
// Products of one row of H1 H2 and H2 H1 that the assembly kernel holds.
constexpr int kCommCap = 1024;
// K = i (A B - B A), one wave per row.  Count pass (fill = false): counts[r] =
// entries of row r, *overflow = 1 if a row lists more than kCommCap products.
// Fill pass: column indices and values at rp_out[r].
hipError_t launch_csr_commutator(bool fill, const CsrDev& A, const CsrDev& Bm, int dim, int* counts,
                                 const int* rp_out, int* ci_out, double2* val_out, int* overflow, hipStream_t s);
// One Leja iteration on a1 H1 + a2 H2 + a3 K (kLeja semantics, x = a.x1).
// streamed: the three-term kernel streamed through LDS like kStreamTile (grid
// csr2_stream_grid), else the 8-row wave tiles.
int csr3_grid(int dim, bool streamed);
hipError_t launch_csr3_iter(const CsrDev& t1, const CsrDev& t2, const CsrDev& t3, int dim, const IterArgs& a,
                            double a3, bool streamed, hipStream_t s);
hipError_t launch_csr3_stream(const CsrDev& t1, const CsrDev& t2, const CsrDev& t3, int dim, const IterArgs& a,
                              double a3, hipStream_t s);

// ---- whole propagations in one workgroup per state (small dimensions) ----

struct PersistProblem {
  CsrDev t1, t2;
  int dim;
};

// One exponential of one state: m iterations per substep, s substeps, the
// parameters of iteration i at table[table_off + i - 1].
struct PersistExp {
  int m, s;
  long long table_off;
  double tol_sub;
};

struct PersistArgs {
  const PersistProblem* probs;
  const int* state_prob;   // problem of each state (workgroup)
  double2* const* state;   // state vector of each workgroup (in place)
  const ColParam* table;
  const PersistExp* exps;  // nexp per state, state-major
  int nexp;                // exponentials per state (even: Cf4 pairs)
  Slot* slots;             // one per state
  int early;
  int cache1;              // every problem's term 1 fits kPersistCache entries (dim <= 1024)
};

// Largest dimension of the one-workgroup-per-state kernel (two LDS vectors).
constexpr int kPersistMaxDim = 4096;
// Entries of term 1 the dim <= 1024 kernel keeps in LDS beside its two vectors.
constexpr int kPersistCache = 6400;
hipError_t launch_persist_propagate(const PersistArgs& a, int nstates, int max_dim, hipStream_t s);

// Small helpers.
hipError_t launch_copy(const double2* src, double2* dst, long long n, hipStream_t s);
hipError_t launch_slot_reset(Slot* slot, int n, hipStream_t s);

}  // namespace magnus
