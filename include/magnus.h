/*
 * magnus.h -- C ABI of the MI355X Magnus-Leja propagator.
 *
 * Problem (Section 1, the Schroedinger equation; Section 4, the split of the
 * Hamiltonian):  i dpsi/dt = H(t) psi,  H(t) = H1 + f(t) H2,  H1, H2 Hermitian,
 * psi(t0) = psi0.  With A(t) = -i H(t) (Section 2 writes Y' = A(t) Y), one step
 * of size tau is Y_{n+1} = exp(Omega_n) Y_n (Section 2, the one-step scheme),
 * and every exponential is applied to the state by Newton interpolation at
 * Leja points (Section 3).  Each exponent handled here has the form
 *
 *     Omega = -i tau H_hat,   H_hat = a H1 + b H2 + kappa K,   K = i [H1, H2],
 *
 * so exp(Omega) v = exp(-i tau H_hat) v with a Hermitian H_hat.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Complex numbers are complex128, interleaved (re, im) pairs of IEEE
 *   doubles, the layout of torch.complex128 / numpy complex128 / hipDoubleComplex.
 * - A state of dimension dim is dim contiguous complex128 values; a batch of
 *   `batch` states is batch*dim values, state b starting at element b*dim.
 * - All vector and matrix pointers are DEVICE pointers on the context's device,
 *   allocated and freed by the caller; the library never frees them, keeps no
 *   reference to them after a call returns, and never writes to inputs.
 * - Scalars, option structs, f-node arrays and stats are HOST memory.
 * - Calls enqueue work on `stream` (a hipStream_t; NULL = the default stream)
 *   and return without synchronising, unless a non-NULL `stats` is passed, in
 *   which case the call synchronises `stream` before returning.  A context
 *   owns one workspace: calls that share a context must be ordered on one
 *   stream (calls on different streams through one context race).
 * - Return value: MAGNUS_OK (0) or a negative status; magnus_last_error()
 *   returns a thread-local message describing the last failure.
 * - Precision: all arithmetic is FP64 (device and host).
 * - Device memory is allocated by magnus_create (the workspace) and, on
 *   request only, by the preparation calls that build matrices the hot path
 *   then reuses (magnus_reserve_dense, magnus_dense_commutator,
 *   magnus_csr_commutator, magnus_dense_m6_prepare, magnus_csr_m6_prepare):
 *   their sizes depend on the terms (dim^2 per dense matrix, the commutator's
 *   nonzeros), which a context created for a dimension cannot know.  Every
 *   other call allocates nothing on the device; magnus_step_cf4_noalloc needs
 *   no context at all.
 * - Dense terms are row-major (each row contiguous, stride ld): the GEMV and
 *   GEMM kernels stream rows, and a Hermitian term's column-major layout is
 *   its conjugate's row-major one.
 * - Spectral enclosures come from magnus_spectral_bounds (rigorous
 *   Gershgorin discs) or magnus_spectral_bounds_lanczos (Lanczos estimates,
 *   with a step count); one entry point per method.
 */
#ifndef MAGNUS_H
#define MAGNUS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define MAGNUS_OK        0
#define MAGNUS_EINVAL   -1  /* null pointer, size mismatch, bad format, malformed CSR */
#define MAGNUS_EDOMAIN  -2  /* tol <= 0, non-finite tau/f/a/b/kappa, lam_min > lam_max */
#define MAGNUS_ENOCONV  -3  /* the degree/substep caps cannot meet tol (nothing enqueued) */
#define MAGNUS_EHIP     -4  /* HIP runtime error */
#define MAGNUS_ENOMEM   -5  /* dim or batch larger than the context workspace */
#define MAGNUS_ENAN     -6  /* non-finite value met on the device (magnus_check) */

/* ---- term formats -------------------------------------------------------- */
#define MAGNUS_CSR    0
#define MAGNUS_DENSE  1

/* ---- methods ---------------------------------------------------------------- */
#define MAGNUS_CF4  0   /* Section 2, Method Cf4: 2 Gauss nodes, 2 exponentials */
#define MAGNUS_M4   1   /* Section 2, Method M4: 2 Gauss nodes, 1 exponential with the commutator */
#define MAGNUS_M2   2   /* Section 2, exponential midpoint rule (order 2): 1 node, 1 exponential */
#define MAGNUS_CF43 3   /* Section 2, Method Cf4:3: 3 Gauss nodes, 3 exponentials */
#define MAGNUS_M6   4   /* Section 2, Method M6: 3 Gauss nodes, 1 exponential with nested commutators
                           (after magnus_dense_m6_prepare or magnus_csr_m6_prepare) */

/* Largest interpolation degree per substep the library plans for. */
#define MAGNUS_MAX_DEGREE 64

typedef struct magnus_ctx magnus_ctx;
typedef void* magnus_stream;   /* hipStream_t */

/*
 * One Hermitian term of the Hamiltonian.
 *   format  MAGNUS_CSR: row_ptr[dim+1] (row_ptr[0] = 0, non-decreasing,
 *           row_ptr[dim] = nnz), col_idx[nnz] (0 <= col < dim), val[nnz]
 *           complex128 (both may be NULL when nnz = 0; rows may be empty).
 *           Section 3 fixes CSR as the sparse format.
 *           MAGNUS_DENSE: val is a row-major dim x dim complex128 matrix with
 *           row stride ld >= dim elements (element (i, j) at val[i*ld + j]),
 *           the same ld for H1 and H2;
 *           row_ptr, col_idx, nnz unused.
 *   lam_min, lam_max  an enclosure of the term's spectrum (Section 3: the Leja
 *           method needs an estimate of the spectrum).  Fill them with
 *           magnus_spectral_bounds or supply them; lam_min <= lam_max.
 */
typedef struct {
  int32_t format;
  int32_t reserved;
  int64_t dim;
  int64_t nnz;
  int64_t ld;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const void* val;
  double lam_min;
  double lam_max;
} magnus_term;

/* H(t) = H1 + f(t) H2 (Section 4).  k_min, k_max enclose the spectrum of the
 * Hermitian K = i [H1, H2] (needed by M4 only; magnus_spectral_bounds fills
 * them with the rigorous bound |K| <= 2 |H1| |H2|). */
typedef struct {
  magnus_term H1;
  magnus_term H2;
  double k_min;
  double k_max;
} magnus_hamiltonian;

/* Leja options (Section 4 runs with relative and absolute tolerance 1e-10 and
 * early termination on).
 *   tol               error allowed per exponential, relative to |v|_2
 *                     (tol_mode 0), or for the whole call, split evenly over
 *                     its exponentials (tol_mode 1).
 *   max_degree        cap on the degree per substep (1..MAGNUS_MAX_DEGREE).
 *   max_substeps      cap on the number of substeps per exponential (>= 1).
 *   early_termination 1: stop a substep once two consecutive Newton terms
 *                     are below tol |v| (Section 3); 0: always run the a
 *                     priori degree (a result that is smooth in the data). */
typedef struct {
  double tol;
  int32_t max_degree;
  int32_t max_substeps;
  int32_t early_termination;
  int32_t tol_mode;
} magnus_leja_opts;

/* Work done by one call (filled when non-NULL; implies a stream sync). */
typedef struct {
  int64_t exponentials;     /* exponentials applied (per state) */
  int64_t substeps;         /* substeps over all exponentials */
  int64_t planned_iters;    /* Leja iterations planned a priori */
  int64_t iters;            /* Leja iterations executed (early termination) */
  int64_t hv_products;      /* products of a CSR/dense term with a vector */
  int32_t max_degree_used;
  int32_t max_substeps_used;
  double max_err_bound;     /* largest a priori interpolation bound per exponential */
  double tol_per_exp;       /* tolerance each exponential was planned for */
} magnus_stats;

/* ---- context -------------------------------------------------------------- */

/* Create a context on `device` owning a workspace for states of up to
 * max_dim entries and batches of up to max_batch states (allocated here; later
 * allocations happen only in magnus_reserve_dense, magnus_dense_commutator,
 * magnus_dense_m6_prepare, magnus_csr_commutator and magnus_csr_m6_prepare;
 * about 8 vectors per state).  *out receives the
 * context.  Calls on one context share its workspace: they must not run
 * concurrently from several host threads, and work they enqueue on different
 * streams must not overlap on the device (one stream per context, or the
 * caller orders them).  Errors: EINVAL (null out, max_dim < 1, max_batch < 1),
 * EHIP (device or allocation failure). */
int magnus_create(magnus_ctx** out, int64_t max_dim, int32_t max_batch, int32_t device);

/* Reserve (once) a dim x dim complex128 device buffer in the context for the
 * assembled exponent H_hat = a H1 + b H2 of dense terms.  With it, groups of
 * states that share the field run one MFMA GEMM per Leja iteration instead of
 * two, and a single state whose exponential needs at least 4 iterations
 * assembles H_hat once (48 dim^2 bytes) and then reads one matrix per
 * iteration instead of two (Section 4 assembles H(t) on the device likewise).
 * An explicit allocation entry point: calls made without it work, reading
 * both terms in every iteration.
 * Errors: EINVAL (dim < 1), EHIP (allocation failure). */
int magnus_reserve_dense(magnus_ctx* ctx, int64_t dim);

/* Assemble the commutator K = i [H1, H2] of two dense terms in the context
 * (Section 2, Method M4; Section 4 forms the commutator of the M4 exponent
 * with matrix products): one complex GEMM C = H1 H2 on the FP64 matrix cores,
 * then K = i (C - C^H), since H2 H1 = (H1 H2)^H for Hermitian terms.  Sets
 * h->k_min, h->k_max from K's Gershgorin discs (tighter than the
 * 2 |H1| |H2| of magnus_spectral_bounds).  Needed before M4 steps or
 * commutator exponents (kappa != 0) on dense terms, which then assemble
 * H1 + b H2 + kappa K once per exponential.  The context keeps K (it
 * allocates dim^2 complex128 for it, and reserves the magnus_reserve_dense
 * buffer) for this pair of terms, recognised by their value pointers, dim
 * and ld; a later call for another pair replaces it.  Synchronous.
 * Errors: EINVAL (null or non-dense terms), EDOMAIN, ENOMEM (dim above
 * max_dim), EHIP. */
int magnus_dense_commutator(magnus_ctx* ctx, magnus_hamiltonian* h, magnus_stream stream);

/* Assemble the commutator K = i [H1, H2] of two CSR terms in the context
 * (Section 2, Method M4; Section 4 forms the M4 commutator explicitly) and set
 * h->k_min, h->k_max from K's Gershgorin discs.  Every row of H1 H2 - H2 H1 is
 * formed on the device from its products (one wave per row: at most 1024
 * products per row, else ENOMEM), equal columns summed in a fixed order,
 * exact zeros dropped.  Afterwards M4 steps and commutator exponents on these
 * terms run one pass over H1, H2 and K per Leja iteration instead of the two
 * matrix-free passes.  The context keeps K (allocating its arrays) for this
 * pair of terms, recognised by their row_ptr and val pointers and dim; a
 * later call for another pair replaces it.  Synchronous.
 * Errors: EINVAL (null or non-CSR terms, malformed CSR), EDOMAIN, ENOMEM, EHIP. */
int magnus_csr_commutator(magnus_ctx* ctx, magnus_hamiltonian* h, magnus_stream stream);

/* Prepare Method M6 (Section 2) on two dense terms.  For H(t) = H1 + f(t) H2
 * the nested commutators of the M6 exponent expand into a linear combination,
 * with scalars that depend on the step's three field samples, of ten fixed
 * Hermitian matrices: H1, H2, K = i[H1,H2], P_a = -i[H_a,K] (a = 1, 2),
 * U_11 = i[H1,P_1], U_12 = i[H1,P_2] (= i[H2,P_1]), U_22 = i[H2,P_2],
 * R_a = -i[K,P_a].  This call forms K as magnus_dense_commutator does and the
 * seven others with one FP64-MFMA GEMM each, plus their Gershgorin
 * enclosures, and keeps them in the context (it allocates 7 dim^2 complex128
 * more); each M6 step then assembles its exponent from the ten (one pass
 * over them) and runs one Leja exponential, the spectral enclosure summed
 * over the ten (Weyl).  The matrices belong to this pair of terms, as for
 * magnus_dense_commutator.  Synchronous.  Errors as magnus_dense_commutator. */
int magnus_dense_m6_prepare(magnus_ctx* ctx, magnus_hamiltonian* h, magnus_stream stream);

/* Prepare Method M6 (Section 2) on two CSR terms: K = i[H1,H2] as
 * magnus_csr_commutator forms it, then P_a = -i[H_a,K] (a = 1, 2) by the same
 * device assembly (at most 1024 products per row of each, else ENOMEM), with
 * Gershgorin enclosures, kept in the context with six work vectors of dim
 * entries.  The nested commutators U_ab = i[H_a,P_b] and R_a = -i[K,P_a] fill
 * in too quickly to assemble; each Leja iteration of an M6 step applies them
 * to the iterate as commutators of the assembled matrices (with the ten
 * scalars of the dense case, the products grouped by matrix: two passes over
 * H1, H2, K, P1 and P2 per iteration), and the
 * spectral enclosure is the Weyl sum of the assembled matrices' discs and
 * +-2 rho(A) rho(B) for each nested [A, B].  The matrices belong to this pair
 * of terms, as for magnus_csr_commutator.  Synchronous.  Errors as
 * magnus_csr_commutator. */
int magnus_csr_m6_prepare(magnus_ctx* ctx, magnus_hamiltonian* h, magnus_stream stream);

/* Free the workspace and the context (NULL is accepted). */
int magnus_destroy(magnus_ctx* ctx);

/* Thread-local description of the last non-OK status. */
const char* magnus_last_error(void);

/* Synchronise `stream` and report device-side failures since the last check:
 * MAGNUS_ENAN if a non-finite vector norm was met, else MAGNUS_OK. */
int magnus_check(magnus_ctx* ctx, magnus_stream stream);

/* ---- spectral bounds (Section 3: the parameters of the Leja method need an
 * estimate of the spectrum) --------------------------------------------------- */

/* Fill h->H1.lam_min/lam_max, h->H2.lam_min/lam_max (Gershgorin discs, rigorous
 * for Hermitian terms) and h->k_min/k_max (|K| <= 2 |H1| |H2|).  Also validates
 * CSR structure (row_ptr monotone, row_ptr[0] = 0, row_ptr[dim] = nnz, columns
 * in range) and returns EINVAL if it is malformed.  Synchronous.
 * Every call that takes CSR terms validates a term once per context (recognised
 * by its three array pointers, dim and nnz) before any kernel gathers through
 * it; a caller that rewrites a term's arrays in place calls this function
 * again, which re-validates it (a failed re-validation leaves it invalid). */
int magnus_spectral_bounds(magnus_ctx* ctx, magnus_hamiltonian* h, magnus_stream stream);

/* Tighter spectral estimates by the Lanczos process (Section 3 needs only an
 * estimate of the spectrum): first as magnus_spectral_bounds (which also
 * validates), then `steps` Lanczos steps on each term from a fixed
 * pseudo-random start vector (the term's products run on the device), and
 * each term's enclosure becomes [theta_min - d, theta_max + d] intersected with
 * its Gershgorin interval, theta_min/max the extreme Ritz values and
 * d = max(margin (theta_max - theta_min), 3 x their change over the last 10
 * steps); k_min/k_max = -+2 |H1| |H2| with the new norms.  Unlike the
 * Gershgorin discs this is an estimate, not a proof: the a priori Leja error
 * bound assumes the spectrum lies inside.  Uses the context's work vectors.
 * Synchronous (one host wait per dot product).
 * Errors: as magnus_spectral_bounds; EINVAL (steps < 2, margin < 0); ENAN. */
int magnus_spectral_bounds_lanczos(magnus_ctx* ctx, magnus_hamiltonian* h, int32_t steps, double margin,
                                   magnus_stream stream);

/* ---- the hot path ------------------------------------------------------------ */

/* w = exp(-i tau (a H1 + b H2 + kappa K)) v for `batch` states
 * (Section 3: the Leja interpolant sum_i d_i prod_{j<i} (A - xi_j I) v and its
 * recurrence).  v and w hold batch*dim complex128; w may equal v.
 * tau may be negative or zero (zero copies v).  kappa != 0 applies
 * K w = i (H1 (H2 w) - H2 (H1 w)) matrix-free.
 * Errors: EINVAL, EDOMAIN, ENOMEM, ENOCONV (before any work is enqueued), EHIP. */
int expmv_leja(magnus_ctx* ctx, const magnus_hamiltonian* h, double a, double b, double kappa,
               double tau, const void* v, void* w, int32_t batch, const magnus_leja_opts* opts,
               magnus_stats* stats, magnus_stream stream);

/* One step of Method Cf4 (Section 2):
 *   psi_out = exp(tau(alpha1 A1 + alpha2 A2)) exp(tau(alpha2 A1 + alpha1 A2)) psi_in,
 * the right factor acting first, with A_j = -i (H1 + f_j H2), f1 = f(t_n + c1 tau),
 * f2 = f(t_n + c2 tau), c_{1,2} = 1/2 -+ sqrt(3)/6, alpha_{1,2} = (3 -+ 2 sqrt(3))/12.
 * The caller evaluates f at the nodes (magnus_quadrature_nodes gives them).
 * psi_in may equal psi_out.  Errors as expmv_leja. */
int magnus_step_cf4(magnus_ctx* ctx, const magnus_hamiltonian* h, double tau, double f1, double f2,
                    const void* psi_in, void* psi_out, int32_t batch, const magnus_leja_opts* opts,
                    magnus_stats* stats, magnus_stream stream);

/* One step of Method M4 (Section 2):
 *   psi_out = exp(tau/2 (A1 + A2) + sqrt(3) tau^2 / 12 [A2, A1]) psi_in,
 * i.e. exp(-i tau (H1 + fbar H2 + kappa K)) with fbar = (f1 + f2)/2,
 * kappa = sqrt(3) tau (f2 - f1) / 12, K = i [H1, H2]; the commutator is
 * applied to vectors, never assembled.  Arguments as magnus_step_cf4. */
int magnus_step_m4(magnus_ctx* ctx, const magnus_hamiltonian* h, double tau, double f1, double f2,
                   const void* psi_in, void* psi_out, int32_t batch, const magnus_leja_opts* opts,
                   magnus_stats* stats, magnus_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one Cf4 step
 * of one state, as magnus_step_cf4 with batch = 1, without a context and
 * without allocating.  Its workspace is a device array of the library of
 * 17.0 MiB per device (eight vectors of up to 131072 = 2^17 entries, the norm
 * partials, the CSR scan outputs and one control slot), set up on the first
 * call on the current device and held until the process ends.
 *   h             as magnus_step_cf4 (CSR or dense two-term terms, dim <= 2^17;
 *                 dense terms run the two-term iteration, never assembled).
 *   other args    as magnus_step_cf4; the call runs on the current device.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents (the control slot is cleared at the start of each call):
 * calls that overlap on one device, from several host threads or on several
 * streams, race.  The first call with a given CSR term scans its structure
 * (a stream sync), as the context entry points do once per term.
 * Errors: ENOMEM (dim > 2^17), EHIP (no address for the array on this
 * device), otherwise as magnus_step_cf4. */
int magnus_step_cf4_noalloc(const magnus_hamiltonian* h, double tau, double f1, double f2,
                            const void* psi_in, void* psi_out, const magnus_leja_opts* opts,
                            magnus_stats* stats, magnus_stream stream);

/* nsteps steps of `method` in place on psi (batch*dim complex128, device) on
 * the grid t_n = t0 + n tau (the one-step scheme of Section 2 repeated;
 * control flow stays on the host, Section 3).  Methods: MAGNUS_CF4, MAGNUS_M4,
 * MAGNUS_M2 (exp(tau A(t_n + tau/2))), MAGNUS_CF43 (Method Cf4:3: three
 * exponentials exp(tau sum_j alpha_ij A_j) on the three Gauss nodes
 * c = 1/2 -+ sqrt(15)/10, 1/2, the factor of the last row acting first),
 * MAGNUS_M6 (terms prepared by magnus_dense_m6_prepare or magnus_csr_m6_prepare;
 * states in turn).
 *   f_nodes     HOST double[batch_f][nsteps][q]: f(t_n + c_j tau), j < q, with
 *               q = magnus_method_nodes(method) (2, 2, 1, 3, 3).
 *   batch_f     1 (one field for all states) or batch (one field per state).
 *   checkpoints NULL, or DEVICE storage for ceil(nsteps/every_k)+1 copies of psi:
 *               slot j receives psi after j*every_k steps (slot 0 = psi0), and
 *               the last slot psi after nsteps steps.
 *   every_k     checkpoint spacing (>= 1; ignored when checkpoints is NULL).
 * CSR states of the product-of-exponentials methods run the whole call in one
 * persistent launch (one workgroup per state, vectors in LDS) when the
 * dimension is at most 1024, 2048 with 4 or more states, 4096 with 32 or more
 * (environment MAGNUS_PERSIST, read at magnus_create: 0 never, 2 always up to
 * 4096); larger ones launch each Leja iteration over the grid.
 * Errors as expmv_leja. */
int propagate(magnus_ctx* ctx, const magnus_hamiltonian* h, int32_t method, double tau,
              int64_t nsteps, const double* f_nodes, int32_t batch_f, void* psi, int32_t batch,
              void* checkpoints, int32_t every_k, const magnus_leja_opts* opts,
              magnus_stats* stats, magnus_stream stream);

/* One problem of a ragged batch: its own Hamiltonian, states and fields. */
typedef struct {
  magnus_hamiltonian h;   /* spectral enclosures filled */
  void* psi;              /* DEVICE, batch * h.H1.dim complex128, propagated in place */
  int32_t batch;          /* states of this problem */
  int32_t batch_f;        /* 1 or batch */
  const double* f_nodes;  /* HOST [batch_f][nsteps][q], q = magnus_method_nodes(method) */
} magnus_problem;

/* nsteps steps of `method` for several independent problems of different
 * sizes (the one-step scheme of Section 2 on each).  CSR problems of the
 * product-of-exponentials methods (Cf4, Cf4:3, M2) run in persistent launches
 * (one workgroup per state carries every step with its vectors in LDS; up to
 * 256 or max_batch states per launch) when their dimension is at most 4096
 * (none with MAGNUS_PERSIST=0).  The larger CSR problems advance together
 * when there are at least 2 of them, all with the same batch, split into
 * groups of G states (G the group size magnus_autotune chose for the largest
 * of them, else the largest of 32, 16, 8, 4, 2 within the batch, halved until
 * it divides the batch; at most 8 groups), their states fit the context's
 * workspace at once (sum of dim * batch at most max_dim * max_batch) and
 * their control slots fit beside the small states': one launch per Leja
 * iteration serves every group (each problem with its own degree,
 * coefficients and stop tests), then one launch makes all their columns'
 * stop decisions; no host wait.  Otherwise they run first, as
 * batched propagations, each followed by a host wait that reports a
 * non-finite norm (ENAN) at once.  Tolerances as in propagate (tol_mode 1:
 * budget over the exponentials of each state).  Errors as propagate. */
int magnus_propagate_ragged(magnus_ctx* ctx, const magnus_problem* probs, int32_t nprob, int32_t method,
                            double tau, int64_t nsteps, const magnus_leja_opts* opts, magnus_stats* stats,
                            magnus_stream stream);

/* ---- adjoint (gradient of a final-state fidelity) ------------------------------ */

/* Bytes of device workspace magnus_propagate_adjoint needs (or -1 for bad
 * arguments): checkpoints every every_k steps, one segment of recomputed
 * states, and a few vectors. */
int64_t magnus_adjoint_workspace_bytes(int64_t dim, int64_t nsteps, int32_t every_k);

/* Loss L = 1 - |psi_target^H psi_N|^2 of an nsteps-step Cf4 propagation from
 * psi0 (Method Cf4, Section 2; t_n = n tau with the caller's field samples)
 * and its gradient with respect to P control parameters, by a backward sweep:
 * lambda_N = psi_target, lambda_n = E(n)^H lambda_{n+1} (exponentials with
 * -tau), and for each step the two scalars lambda^H L(A, E) phi, where the
 * Frechet derivative L of the matrix exponential at A = -i tau H_hat in the
 * direction E = -i tau H2 is the upper-right block of the exponential of the
 * block matrix [[A, E], [0, A]] (Leja recurrence on 2-vectors).
 *   f_nodes   HOST double[nsteps][2]: f(t_n + c_1 tau), f(t_n + c_2 tau).
 *   df_nodes  HOST double[nsteps][2][P]: derivatives of those samples with respect
 *             to each parameter.
 *   psi0, psi_target  DEVICE, dim complex128 each (not modified).
 *   every_k   checkpoint spacing: states are stored every every_k steps and each
 *             segment is recomputed during the backward sweep.
 *   workspace DEVICE scratch of at least magnus_adjoint_workspace_bytes bytes,
 *             caller-owned.
 *   loss      HOST double; grad HOST double[P].
 * CSR or dense terms; the context needs max_batch >= 2.  Synchronous.
 * Errors: EINVAL, EDOMAIN, ENOMEM (workspace or context too small), ENOCONV, EHIP, ENAN. */
int magnus_propagate_adjoint(magnus_ctx* ctx, const magnus_hamiltonian* h, double tau, int64_t nsteps,
                             const double* f_nodes, const double* df_nodes, int32_t nparams, const void* psi0,
                             const void* psi_target, int32_t every_k, void* workspace, int64_t workspace_bytes,
                             double* loss, double* grad, const magnus_leja_opts* opts, magnus_stats* stats,
                             magnus_stream stream);

/* ---- autotuning ----------------------------------------------------------------- */

/* Autotuner for the H·v stream that Section 3 reduces the method's cost to:
 * times, on the device, each row mapping of the single-state CSR Leja
 * iteration on these terms (variant codes 1 nonzero streaming, 2-4 a row per
 * lane in blocks of 64/32/128 rows, 5-6 wave tiles of 8/16 rows, 7 runs of 8
 * wave tiles of 8 rows streamed through LDS one tile ahead;
 * 5 timed launches each) and, when batch > 1, the multi-state iteration with 2, 4, 8,
 * 16 and 32 states per pass (up to batch; cost per state), and keeps the
 * fastest for these terms (recognised by H1's row_ptr and dim) in the
 * context: later calls use them.  Results differ from untuned calls only in
 * rounding (another summation order); the MAGNUS_CSR_VARIANT environment
 * variable, when set, still wins.  Overwrites the context's work vectors.
 *   variant, group       HOST out (may be NULL): the chosen code and group size
 *   variant_us[7], group_us[7]  HOST out (may be NULL): measured microseconds per
 *                        iteration (a mapping whose grid is too large for the
 *                        stop test fused into the iteration is timed with the
 *                        decide kernel that then follows each iteration; group
 *                        entries NAN where not tried).
 * Dense terms: times the two-term GEMV iteration with 1, 2 and 4 rows per
 * wave and, when batch > 1, the FP64-MFMA group iteration of batch states
 * with each tile shape (0: 32 rows x 64 states with K split between two
 * groups of four waves, 1: 32 x 64, 2: 64 x 64, 3: 64 x 64 with K split,
 * 4: 32 x 128 with K split, 5: 32 x 64 and 6: 64 x 64 with the operands
 * copied into LDS by LDS-DMA three chunks deep; one term when the context holds an assembly
 * buffer, else two), and keeps the fastest for these terms (H1's values and
 * dim); then variant receives the rows per wave, group the tile code,
 * variant_us[0..2] and group_us[0..6] the timings (CSR terms: group_us[0..4]).
 * Synchronous.  Errors: EINVAL, ENOMEM, EHIP. */
int magnus_autotune(magnus_ctx* ctx, const magnus_hamiltonian* h, int32_t batch, int32_t* variant,
                    int32_t* group, double* variant_us, double* group_us, magnus_stream stream);

/* ---- kernel timing (profiling aid) ---------------------------------------------- */

/* Kernel classes timed by magnus_timing. */
#define MAGNUS_KERNEL_CSR_LEJA   0  /* two-term CSR Leja iteration */
#define MAGNUS_KERNEL_CSR_SPLIT  1  /* first pass of a commutator iteration */
#define MAGNUS_KERNEL_CSR_COMM   2  /* second pass of a commutator iteration */
#define MAGNUS_KERNEL_DENSE_LEJA 3  /* two-term dense Leja iteration */
#define MAGNUS_KERNEL_CSR_MULTI  4  /* two-term CSR Leja iteration on a group of states */
#define MAGNUS_KERNEL_DENSE_MFMA 5  /* dense group Leja iteration (FP64 MFMA GEMM) */
#define MAGNUS_KERNEL_PERSIST    6  /* whole small-state propagations, one workgroup per state */
#define MAGNUS_KERNEL_CSR_LEJA3  7  /* three-term CSR Leja iteration (assembled commutator) */

/* enable = k >= 1: from now on bracket every k-th launch of each kernel class
 * (k = 1: every iteration kernel the context launches) with a pair of HIP
 * events on the call's stream, previous records dropped; a larger k keeps the
 * events' own cost (a few percent of a 150 us launch at k = 1) out of the
 * launches in between.  enable = 0: stop recording.  Errors: EINVAL (k < 0),
 * EHIP. */
int magnus_timing(magnus_ctx* ctx, int32_t enable);

/* Wait for the recorded events and report, for one kernel class, the summed
 * event-to-event time in milliseconds and the number of bracketed launches.
 * Errors: EINVAL (bad class), EHIP. */
int magnus_timing_read(magnus_ctx* ctx, int32_t kind, double* total_ms, int64_t* launches);

/* ---- host planning helpers (pure host code, no device needed) ------------------- */

/* Field samples per step of `method` (Section 2): 2 for Cf4 and M4 (two
 * Gauss nodes), 1 for M2 (midpoint), 3 for Cf4:3 and M6 (three Gauss nodes);
 * EINVAL for an unknown method. */
int magnus_method_nodes(int32_t method);

/* t_out[q n + j] = t0 + n tau + c_j tau for n < nsteps, j < q: the quadrature
 * nodes of `method` (Section 2), q = magnus_method_nodes(method). */
int magnus_quadrature_nodes(int32_t method, double t0, double tau, int64_t nsteps, double* t_out);

/* The first m+1 Leja points of [-2, 2]: xi_0 = 2, then each point maximises
 * the product of distances to the previous ones (ties to the left). */
int magnus_leja_points(int32_t m, double* xi);

/* Divided differences d_k = f[xi_0, ..., xi_k], k = 0..m, of f(x) = exp(-i theta x)
 * at the Leja points (Section 3), written as m+1 interleaved complex values. */
int magnus_divided_differences(double theta, int32_t m, double* d);

/* sup over x in [-2, 2] of |exp(-i theta x) - p_m(x)| (p_m the degree-m Leja
 * interpolant), evaluated on the planner's grid from the tail of the Newton series. */
double magnus_leja_error(double theta, int32_t m);

/* Degree m and substeps s chosen for exp(-i theta X), spec(X) in [-2, 2], so
 * that s * err(theta/s, m) <= tol / 2 at least cost m*s; *bound receives the
 * achieved s * err.  Returns ENOCONV if the caps cannot meet tol. */
int magnus_leja_plan(double theta, double tol, int32_t max_degree, int32_t max_substeps,
                     int32_t* m, int32_t* s, double* bound);

#ifdef __cplusplus
}
#endif
#endif /* MAGNUS_H */
