/*
 * rdm.h -- C ABI of the MI355X (gfx950) library for the equilibrium reduced
 * density matrix of a spin system strongly coupled to a spin bath, by the
 * partial-trace typicality estimator of Chen & Cheng, "Numerical computation
 * of the equilibrium-reduced density matrix for strongly coupled open quantum
 * systems" (arXiv:2204.08147).
 *
 * All functions have C linkage; no C++ exception crosses this boundary.  Every
 * function returning rdm_status leaves a human-readable message retrievable
 * with rdm_last_error() when it fails.  Unless stated otherwise, pointers
 * named host_* or documented as "host" point to host memory owned by the
 * caller, and pointers documented as "device" point to device memory on the
 * current HIP device, also owned by the caller.
 *
 * Physics conventions (the paper's eqn:Ht and the site operators of Section
 * "Spin systems"):
 *   - N = n_s + n_b spin-1/2 sites, 0-based; site 0 is the leftmost Kronecker
 *     factor, the system is sites 0..n_s-1.  Site i is bit (N-1-i) of a basis
 *     index, so the system index of basis state idx is idx >> n_b, and bit
 *     value 0 means sigma^z = +1.
 *   - H_t = sum_pairs (jx sx_i sx_j + jy sy_i sy_j + jz sz_i sz_j)
 *           + sum_i (hx_i sx_i + hz_i sz_i)              (Pauli matrices)
 *     Each pair is given once (unordered); a pair listed several times has its
 *     coefficients summed.  The paper's field "(h/2) sigma^z" is hz_i = h/2.
 *   - H_s / H_b / H_sb follow the paper's split: terms with all sites in the
 *     system / all in the bath / mixed.
 *
 * Estimator (Section "Algorithm"): n_v real Rademacher bath vectors v_j of
 * unit norm are drawn from the seed by the SplitMix64 rule
 *     key_j = sm64(seed ^ sm64(j)),  word = sm64(key_j ^ (b >> 6)),
 *     v_j[b] = (1 - 2*((word >> (b & 63)) & 1)) * sqrt(2^-n_b),
 * where sm64(x) is one SplitMix64 output from state x (golden-gamma add, then
 * the 30/27/31 xor-shift-multiply finaliser).  Every start column
 * |m> (x) |v_j> (column c = j*d_s + m) runs k steps of the scalar Lanczos
 * recurrence (Algorithm 1 with block size one, no reorthogonalisation);
 * psi = Lanczos approximation of exp(-beta (H_t - E0)/2) |m>(x)|v_j>; the
 * averaged Gram M(beta) = (1/n_v) sum_j Psi_j^T Psi_j estimates
 * exp(beta E0) tr_b exp(-beta H_t) / d_b (eqn:trace_est, eqn:fT, eqn:trB_est).
 * A second Lanczos run on H_b from the same v_j gives Z_b (eqn:H_est).  E0 /
 * E0b are the smallest Ritz values over all columns (the overflow shift of the
 * section on the mean force Hamiltonian).
 */
#ifndef RDM_H
#define RDM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RDM_OK = 0,
  RDM_E_INVALID = -1,   /* argument out of range; nothing was written       */
  RDM_E_NOMEM = -2,     /* not enough device memory even for the two-pass plan */
  RDM_E_DEVICE = -3,    /* a HIP runtime call failed                         */
  RDM_E_NONFINITE = -4, /* a non-finite value appeared during the solve      */
  RDM_E_BUSY = -5,      /* serving queue full                                */
  RDM_E_CANCELLED = -6  /* serving: the request was cancelled                */
} rdm_status;

enum { RDM_FP64 = 0, RDM_MIXED = 1 };                 /* rdm_options.precision */
enum { RDM_AUTO = 0, RDM_STORED_Q = 1, RDM_TWO_PASS = 2 };  /* rdm_options.mode */
enum { RDM_PER_COLUMN = 0, RDM_BLOCK = 1, RDM_METHOD_AUTO = 2 };  /* rdm_options.method */
enum { RDM_APPLY_AUTO = 0, RDM_APPLY_HOPS = 1, RDM_APPLY_TRANSFORM = 2, RDM_APPLY_HOPS_ROWS = 3 };  /* rdm_hamiltonian_create_ex */

/* One two-site term: jx sx_i sx_j + jy sy_i sy_j + jz sz_i sz_j (Pauli),
 * eqn:Ht.  0 <= i, j < N, i != j; (i, j) and (j, i) denote the same pair. */
typedef struct {
  int32_t i, j;
  double jx, jy, jz;
} rdm_coupling;

typedef struct rdm_hamiltonian rdm_hamiltonian; /* opaque, immutable */

/* Solver options; a NULL pointer means all defaults (zeros). */
typedef struct {
  int32_t precision;   /* RDM_FP64: vectors and arithmetic in FP64.
                          RDM_MIXED: vectors, the Hamiltonian apply and the
                          three-term recurrence in FP32; every dot product and
                          norm accumulated in FP64; tridiagonal eigenproblems,
                          exponentials, cross-tile Gram sums, the n_v average
                          and the finalisation in FP64.                      */
  int32_t mode;        /* RDM_AUTO: stored Lanczos basis if it fits in
                          hbm_budget, else two-pass.  RDM_STORED_Q: keep all
                          k Lanczos vectors.  RDM_TWO_PASS: keep two; a second
                          pass regenerates them bit-identically from the stored
                          recurrence coefficients.                           */
  uint64_t hbm_budget; /* bytes of device memory the solve may use; 0 = free
                          device memory minus a 2 GiB reserve                */
  int32_t slab;        /* apply/norm kernels: 16-byte panels per lane, 1, 2 or
                          4 (0 = tuned); results do not depend on it         */
  int32_t rows_per_lane;/* Gram kernel: rows per lane (0 = tuned)             */
  double tau;          /* breakdown threshold (0 = 1e-12 FP64, 1e-5 mixed)    */
  int32_t profile;      /* 1: time the step kernels with HIP events on
                           hip_stream (results in rdm_result.diag; the steps
                           are then launched one by one).  2: keep the graph
                           replay and time each replayed phase with HIP
                           events on the replay stream (diag[11..12])        */
  int32_t eager;        /* 1: launch every Lanczos step's kernels one by one;
                           by default the steps of a solve or batch run as one
                           captured hipGraph, replayed by later calls with
                           the same workspace and shape (same kernels and
                           arguments, identical results)                      */
  int32_t method;       /* RDM_PER_COLUMN (0): Lanczos on every start column
                           and exp(-beta H/2) by function approximation, then
                           the Gram of the recombined columns (the hot path).
                           RDM_BLOCK (1): the block Lanczos of Algorithm 1 on
                           each bath vector's d_s start columns and the block
                           Gauss quadrature E_1^T exp(-beta T) E_1 (eqn:fT,
                           eqn:trB_est); single solves only (rdm_solve,
                           rdm_solve_ws), no Lanczos basis is kept; n_s <= 3.
                           RDM_METHOD_AUTO (2): per-column when its plan
                           keeps the Lanczos basis within the budget, block
                           when the basis would not fit (with mode RDM_AUTO;
                           otherwise per-column); rdm_workspace_size and
                           rdm_solve_ws decide alike for the same budget;
                           batches use per-column                             */
  int32_t reserved;     /* must be 0                                          */
} rdm_options;

/* Outputs of a solve, per inverse temperature (caller-owned host arrays). */
typedef struct {
  double* rho;      /* n_beta x d_s x d_s, row-major: rho*(beta) = M / tr M   */
  double* h_star;   /* n_beta x d_s x d_s: mean force Hamiltonian (eqn:HMF)  */
  double* log_z;    /* n_beta: ln Z* = ln Z_t - ln Z_b                       */
  double* entropy;  /* n_beta: -tr rho* ln rho*                              */
  double* diag;     /* optional (NULL ok), 16 + 2*n_beta doubles:
                       [0] E0, [1] E0b, [2] columns of H_t that hit breakdown,
                       [3] columns of H_b that hit breakdown, [4] 1 if the
                       two-pass plan was used, [5] device bytes of the plan,
                       [6] mu_min/mu_max of the last beta, [7] mean apply
                       time per Lanczos step (ms; hop-table apply kernel
                       and transform pass 2), [8] mean norm kernel time
                       (ms; hop-table operators), [9] mean Gram kernel time
                       (ms), [10] mean transform pass 1 time (ms; norm step
                       and high-bit transform) -- [7..10] only when
                       rdm_options.profile = 1 (event timing), else 0 --
                       [11] mean time of a replayed Lanczos step (ms: all
                       its kernels, as they ran), [12] steps replayed --
                       only when rdm_options.profile = 2 (for a batch:
                       the steps of all its instances together) --
                       [13..15] zero; then per beta {ln Z_t, ln Z_b}.        */
} rdm_result;

/* Build a Hamiltonian (eqn:Ht) and its bath part.  hx, hz: host arrays of
 * length n_s + n_b, coefficients of sx_i and sz_i; NULL means all zero.
 * Validation: 1 <= n_s <= 4, 1 <= n_b, n_s + n_b <= 28 (a 16-byte panel of
 * one vector is addressed with 32-bit byte offsets: at most 2^28 rows),
 * every coefficient finite, 0 <= i,j < N, i != j.  The library copies all inputs; device tables
 * are built lazily on first use on the current device. */
rdm_status rdm_hamiltonian_create(int32_t n_s, int32_t n_b, const rdm_coupling* couplings,
                                  int64_t n_couplings, const double* hx, const double* hz,
                                  rdm_hamiltonian** out);
/* As rdm_hamiltonian_create, choosing how products with H_t and H_b are
 * computed (the results agree to rounding either way):
 *   RDM_APPLY_HOPS: gathers of the partner rows idx ^ f from hop tables.
 *     Tiles of 256 consecutive rows, or, on 12 sites and more, tiles of
 *     the 4096 rows that differ only in 12 row bits chosen
 *     per operator (the 4 lowest and those that leave the fewest distinct
 *     partner tiles), when that form reads fewer partner tiles per tile
 *     than the other reads partner rows per row;
 *   RDM_APPLY_HOPS_ROWS: hop tables with 256-row tiles only;
 *   RDM_APPLY_TRANSFORM: on 16..28 sites, H = D_Z + W D_X W + T W D_Y W T
 *     (W the Walsh-Hadamard transform, in whose basis XX couplings and
 *     x-fields are diagonal, D_X; YY couplings are T (XX) T with
 *     T = diag((-1)^floor(popcount(idx)/2)), D_Y), streamed in tiles;
 *     other sizes use hop tables;
 *   RDM_APPLY_AUTO (what rdm_hamiltonian_create does): the transform where
 *     available, unless a hop table would read fewer partner rows per row
 *     than the transform streams vectors (sparse operators with YY terms);
 *     hop tables as under RDM_APPLY_HOPS otherwise.
 * rdm_hamiltonian_info reports the choice for H_t and H_b.  RDM_E_INVALID
 * for another value of apply. */
rdm_status rdm_hamiltonian_create_ex(int32_t n_s, int32_t n_b, const rdm_coupling* couplings,
                                     int64_t n_couplings, const double* hx, const double* hz,
                                     int32_t apply, rdm_hamiltonian** out);
void rdm_hamiltonian_destroy(rdm_hamiltonian* h);

/* H_s, the system part of the split H_t = H_s (x) I + I (x) H_b + H_sb
 * (Section "Spin systems"): the couplings and fields of system sites only,
 * as a dense d_s x d_s matrix (out: host, row-major, d_s = 2^n_s; system
 * state m has site s < n_s at bit n_s-1-s).  Used by observables such as the
 * internal-energy deviation tr(H* rho*) - tr(H_s rho_s). */
rdm_status rdm_system_hamiltonian(const rdm_hamiltonian* h, double* out);

/* The internal-energy deviation of Section "Deviation in internal energy"
 * (formula:deviation_of_Hamiltonian): out[b] = tr(H*(beta_b) rho*(beta_b)) -
 * tr(H_s rho_s(beta_b)), rho_s = exp(-beta H_s) / tr exp(-beta H_s) the bare
 * system's thermal state (H_s as rdm_system_hamiltonian).  rho, h_star: host,
 * n_beta x d_s x d_s row-major, the outputs of a solve at the n_beta inverse
 * temperatures beta (host, each > 0 and finite); out: host, n_beta.  Zero
 * when H_sb = 0, where H* = H_s.  RDM_E_INVALID for NULL or bad arguments,
 * RDM_E_NONFINITE for a non-finite input. */
rdm_status rdm_energy_deviation(const rdm_hamiltonian* h, int32_t n_beta, const double* beta, const double* rho,
                                const double* h_star, double* out);

/* Table sizes of a built Hamiltonian: out[0]=N, [1]=n_s, [2]=n_b,
 * [3]=uniform-coefficient hops, [4]=parity-dependent hops, [5]=diagonal terms,
 * [6..8] the same three counts for H_b, [9] / [10] partner-tile groups the
 * 256-row-tile apply stages in LDS for H_t / H_b (hops grouped by their flip bits
 * above a 256-row tile; the own tile plus every tile read by at least three
 * hops), [11] / [12] hops it gathers directly from memory instead, [13] /
 * [14] 1 when H_t / H_b is applied by the transform (rdm_hamiltonian_create_ex)
 * instead, [15] / [16] 1 when that transform has a YY part, [17] / [18] 1
 * when products with H_t / H_b take the 4096-row tiles of chosen
 * row bits, [19] / [20] partner tiles one such tile reads (staged tiles other
 * than its own plus hops gathered directly; 0 under 12 sites).
 * out: host array of 21 int64. */
rdm_status rdm_hamiltonian_info(const rdm_hamiltonian* h, int64_t* out);

/* Full solve (blocking; results on the host).  beta: host array of n_beta
 * inverse temperatures, each > 0 and finite.  n_v >= 1 bath vectors, k >= 1
 * Lanczos steps (capped at 2^N).  hip_stream: a hipStream_t or NULL for the
 * null stream.  Device workspace is allocated and freed by the library. */
rdm_status rdm_solve(const rdm_hamiltonian* h, const double* beta, int32_t n_beta, int32_t n_v,
                     int32_t k, uint64_t seed, const rdm_options* opt, void* hip_stream,
                     rdm_result* out);

/* Device bytes rdm_solve_ws needs for these arguments (host output). */
rdm_status rdm_workspace_size(const rdm_hamiltonian* h, int32_t n_beta, int32_t n_v, int32_t k,
                              const rdm_options* opt, uint64_t* bytes);

/* As rdm_solve, but all device memory comes from the caller's workspace
 * (device pointer, 256-byte aligned, at least rdm_workspace_size bytes,
 * borrowed for the duration of the call).  Device tables of the Hamiltonian
 * are still cached inside the handle. */
rdm_status rdm_solve_ws(const rdm_hamiltonian* h, const double* beta, int32_t n_beta, int32_t n_v,
                        int32_t k, uint64_t seed, const rdm_options* opt, void* hip_stream,
                        rdm_result* out, void* dev_workspace, uint64_t ws_bytes);

/* For callers that cannot allocate device memory (code that may not call
 * hipMalloc or an allocating library routine: tight serving loops, harnesses
 * that forbid allocation).  As rdm_solve with the per-column method, but the
 * device workspace is a fixed array inside this library of
 * RDM_NOALLOC_MAX_BYTES bytes per device (held by every device the library
 * runs on until the process ends); the call allocates no device memory.
 * The plan must fit the array: with mode RDM_AUTO a basis that does not fit
 * takes the two-pass plan; RDM_E_NOMEM (and nothing run) if even that does
 * not fit.  The Hamiltonian's device tables for this precision must already
 * be resident on the current device (any earlier rdm_solve, rdm_solve_ws or
 * rdm_apply with it builds them); otherwise RDM_E_INVALID and nothing run.
 * The Lanczos steps are launched one by one (no graph capture, no slab
 * timing); results equal rdm_solve's with the same options and an
 * hbm_budget of RDM_NOALLOC_MAX_BYTES.  The array keeps the last call's
 * contents, and the solve initialises everything it reads.  Calls share the
 * device's array: the library serialises the calls of one process (a second
 * caller blocks until the first returns), and calls that overlapped on one
 * device would race.  Blocking; results on the host.  method must be
 * RDM_PER_COLUMN or RDM_METHOD_AUTO (taken as per-column) and profile 0. */
#define RDM_NOALLOC_MAX_BYTES (64ull << 20)
rdm_status rdm_solve_noalloc(const rdm_hamiltonian* h, const double* beta, int32_t n_beta, int32_t n_v,
                             int32_t k, uint64_t seed, const rdm_options* opt, void* hip_stream,
                             rdm_result* out);

/* One instance of a batched solve. */
typedef struct {
  const rdm_hamiltonian* h;
  const double* beta;   /* host, n_beta entries */
  int32_t n_beta, n_v, k;
  uint64_t seed;
  rdm_result out;
  rdm_status status;    /* written by rdm_solve_batch */
} rdm_batch_item;

/* Solve independent instances of different sizes together: all instances
 * advance their Lanczos recurrences in the same kernel launches (one launch per
 * kernel per step for the whole batch), grouped into waves that fit in
 * hbm_budget.  Each instance's result is bitwise identical to its own
 * rdm_solve with the same options (fixed per-instance reduction order).
 * Returns the first failing item's status, RDM_OK if all succeeded. */
rdm_status rdm_solve_batch(int32_t n_items, rdm_batch_item* items, const rdm_options* opt,
                           void* hip_stream);

/* As rdm_solve_batch with caller-owned device memory (device pointer,
 * 256-byte aligned, borrowed for the call): the waves are planned to fit
 * ws_bytes (unless hbm_budget is smaller) and all reuse the same workspace.
 * ws_bytes must be at least the min_bytes of rdm_batch_workspace_size. */
rdm_status rdm_solve_batch_ws(int32_t n_items, rdm_batch_item* items, const rdm_options* opt,
                              void* hip_stream, void* dev_workspace, uint64_t ws_bytes);

/* Workspace bounds of a batch (host outputs): min_bytes runs the largest
 * instance alone; all_bytes runs every valid instance in one wave.  Items
 * failing validation get their status written and are left out. */
rdm_status rdm_batch_workspace_size(int32_t n_items, rdm_batch_item* items, const rdm_options* opt,
                                    uint64_t* min_bytes, uint64_t* all_bytes);

/* ---- Kernel-level entry points (device pointers; used by tests/bench) ---- */

/* Block layout used by the library ("panels"): a block of C columns of length
 * dim = 2^n is stored as ceil(C / w) panels of w = 16 / sizeof(scalar)
 * columns (w = 2 FP64, 4 FP32); panel p holds rows 0..dim-1 of columns
 * p*w .. p*w+w-1, row-major with the w values of one row contiguous (16 bytes),
 * and the panels follow each other: element (row, c) is at offset
 * ((c / w) * dim + row) * w + c % w.  Columns past C in the last panel are
 * padding. */

/* Y = H X (which = 0: H_t on 2^N rows; which = 1: H_b on 2^n_b rows), the
 * matrix-free spin-Hamiltonian apply of the hot path (H is accessed only
 * through such products, Section "Past algorithms").  x, y: device, panel
 * layout above with n_cols columns, FP64 (precision RDM_FP64) or FP32
 * (RDM_MIXED); x and y must not overlap.  Runs on hip_stream and returns
 * after it completes (blocking). */
rdm_status rdm_apply(const rdm_hamiltonian* h, int32_t which, int32_t precision, int32_t n_cols,
                     const void* x, void* y, const rdm_options* opt, void* hip_stream);

/* The start block of a solve: column c = j*d_s + m is |m> (x) |v_j> (which = 0,
 * 2^N rows, d_s*n_v columns), v_j itself (which = 1, 2^n_b rows, n_v
 * columns), or the product vector |v_s^(j)> (x) |v_j> of rdm_product_trace
 * (which = 2, 2^N rows, n_v columns), in the panel layout.  out: device.
 * Asynchronous. */
rdm_status rdm_start_block(const rdm_hamiltonian* h, int32_t which, int32_t precision, int32_t n_v,
                           uint64_t seed, void* out, void* hip_stream);

/* Run only the Lanczos recurrences of a solve (k steps on every start column
 * of H_t, or of H_b if which = 1) and return their coefficients (blocking):
 * host_alpha, host_beta: k x n_cols doubles (row j holds alpha_{j+1} /
 * beta_{j+1} of every column), host_kc: n_cols int32 Krylov sizes after
 * breakdown truncation.  n_cols = d_s*n_v (which = 0) or n_v (which = 1). */
rdm_status rdm_lanczos(const rdm_hamiltonian* h, int32_t which, int32_t n_v, int32_t k,
                       uint64_t seed, const rdm_options* opt, void* hip_stream,
                       double* host_alpha, double* host_beta, int32_t* host_kc);

/* Host routine of the hot path's step "eigendecomposition of T_k and function
 * approximation weights" (eqn:fT): for one symmetric tridiagonal matrix with
 * diagonal alpha[0..kk-1] and off-diagonal beta[0..kk-2] (host arrays) compute
 * its eigenvalues theta (host out, kk) and, for each of n_beta inverse
 * temperatures b, y_b = exp(-b (T - e0)/2) e_1 (host out, n_beta x kk) and the
 * Gauss quadrature e_1^T exp(-b (T - e0)) e_1 (host out, n_beta).  Any output
 * pointer may be NULL.  Implicit symmetric QR with Wilkinson shifts; the
 * rotations are replayed on e_1 instead of forming the eigenvectors. */
rdm_status rdm_tridiag_fa(int32_t kk, const double* alpha, const double* beta, int32_t n_beta,
                          const double* betas, double e0, double* theta, double* y, double* quad);

/* Host routine of the block variant (Algorithm 1 + eqn:fT): for a symmetric
 * n x n matrix t (host, row-major; the block tridiagonal T of a block
 * Lanczos run with blocks of b columns) form E_1^T exp(-beta (t - e0)) E_1,
 * the leading b x b block, for each of n_beta inverse temperatures
 * (f: host out, n_beta x b x b row-major), and the smallest eigenvalue of t
 * (min_eig: host out, may be NULL).  Householder reduction to tridiagonal
 * form, then implicit symmetric QR; the eigenvectors are never formed. */
rdm_status rdm_block_quadrature(int32_t n, int32_t b, const double* t, int32_t n_beta,
                                const double* betas, double e0, double* min_eig, double* f);

/* Low-temperature limit (Section "High and low temperature limits"):
 * rho*(inf) = (1/r) sum_i tr_b |psi_i><psi_i| over the r ground states of H_t,
 * and the ground energies E_t, E_b of H_t and H_b, so that
 * H*(inf) = (E_t - E_b) I.  n_v (1..8) Lanczos runs of k steps on seeded
 * full-space Rademacher vectors (vector c is the bath-vector rule of the hot
 * path with n_b replaced by N); the columns whose lowest Ritz value reached
 * the smallest one span the ground space (r = the eigenvalues of their Ritz
 * vectors' Gram matrix above 1e-6 (FP64) / 1e-3 (mixed) of the largest;
 * r <= 4).  Outputs (host, any may be NULL): rho d_s x d_s row-major,
 * e_total, e_bath, entropy -tr rho ln rho, degeneracy r.  opt: precision,
 * hbm_budget, tau and eager are used (NULL = FP64).  Any output pointer,
 * the residual included, may be NULL.  Blocking; the library allocates its
 * workspace. */
typedef struct {
  double* rho;
  double* e_total;
  double* e_bath;
  double* entropy;
  int32_t* degeneracy;
  double* residual;   /* convergence measure: the largest, over the columns
                         that span the ground space, Ritz residual norm
                         |H y - theta y| (y of unit norm) of the lowest Ritz
                         pair after k - 1 steps; 0 when a column reached an
                         invariant subspace.  Small against the gap to the
                         next eigenvalue means a converged ground space. */
} rdm_ground_result;
/* (n_s <= 3: RDM_E_INVALID otherwise.) */
rdm_status rdm_ground_state(const rdm_hamiltonian* h, int32_t n_v, int32_t k, uint64_t seed,
                            const rdm_options* opt, void* hip_stream, rdm_ground_result* out);

/* Outputs of rdm_product_trace, per inverse temperature (caller-owned host
 * arrays; any may be NULL). */
typedef struct {
  double* log_z;    /* n_beta: ln Z* = ln Z_t - ln Z_b                        */
  double* log_z_t;  /* n_beta: ln Z_t from the product samples                */
  double* log_z_b;  /* n_beta: ln Z_b from the bath vectors                   */
  double* samples;  /* n_beta x n_v: per-sample ln(2^N <x_j|exp(-beta H_t)|x_j>) */
} rdm_product_result;

/* Product-state (rank-one) estimator of Z_t (appendix "A consistent partial
 * trace estimator").  Sample j is the unit product vector
 * x_j = |v_s^(j)> (x) |v_j>, where v_j is bath vector j of rdm_solve with the
 * same seed and v_s^(j) is the same sign rule over the n_s system bits with
 * the seed XOR 0x9E3779B97F4A7C15.  2^N <x_j|exp(-beta H_t)|x_j> is unbiased
 * for Z_t; its means over the bath factor (system factor) are the quadratic
 * forms of tr_b exp(-beta H_t) (tr_s exp(-beta H_t)), so the trace estimate
 * is consistent with the partial-trace estimates, and with the same bath
 * vector it equals <v_s|M_j|v_s> for the partial-trace sample M_j of
 * rdm_solve.  One Lanczos column per sample (k steps, the hot-path kernels),
 * Gauss quadrature from each T (eqn:fT with block size one), Z_b from the
 * bath vectors as in rdm_solve.  ln Z_t = ln mean_j(2^N e_1^T exp(-beta
 * (T_j - E0)) e_1) - beta E0 with E0 the smallest Ritz value over the
 * columns.  betas: host, n_beta values >= 0.  Options as for rdm_solve
 * (precision, tau, hbm_budget, eager; the rest ignored).  Allocates its
 * device workspace, runs on hip_stream and returns when done.
 * Errors: RDM_E_INVALID for NULL arguments, n_v or k outside 1..4096 or a
 * negative or non-finite beta; RDM_E_NOMEM beyond the budget; RDM_E_DEVICE;
 * RDM_E_NONFINITE for a failed quadrature. */
rdm_status rdm_product_trace(const rdm_hamiltonian* h, const double* betas, int32_t n_beta, int32_t n_v,
                             int32_t k, uint64_t seed, const rdm_options* opt, void* hip_stream,
                             rdm_product_result* out);

/* High-temperature offset of the estimator (Section "A note on high
 * temperatures"; the appendix deriving the high-temperature limit).  As
 * beta -> 0 the exact H*(beta) tends to H_s, while the estimate built from
 * the bath vectors v_0 .. v_{n_v-1} of a solve with this seed tends to
 * H_s + C,
 *     C = (1/n_v) sum_j (I_s (x) <v_j|) H_sb (I_s (x) |v_j>).
 * C has zero mean over the random vectors: its size indicates the sampling
 * error of that solve, and subtracting it from the estimated H*(beta)
 * removes the estimator's offset at high temperature.
 *   c_out   host, d_s x d_s row-major (system state m has site s < n_s at
 *           bit n_s-1-s): C.
 *   sx_out  host, n_b doubles, or NULL: (1/n_v) sum_j <v_j| sx_c |v_j> for
 *           bath site c = n_s .. N-1 (the only bath expectations C needs:
 *           the sy ones vanish for real vectors, the sz ones because all
 *           entries of a bath vector have the same magnitude).
 * The device computes the bath sign correlations as exact integer sums on
 * hip_stream (NULL: the null stream); the call allocates and frees a small
 * device buffer and returns after the stream has finished it.
 * Errors: RDM_E_INVALID for a NULL h or c_out or n_v outside 1..65535;
 * RDM_E_DEVICE for a failed HIP call. */
rdm_status rdm_high_temperature_term(const rdm_hamiltonian* h, int32_t n_v, uint64_t seed, void* hip_stream,
                                     double* c_out, double* sx_out);

/* Device memory bandwidth probe (a measurement utility, not part of the
 * method): the reference points for the streaming kernels.  pattern 0 reads
 * one array, 1 copies one array into another, 2 reads three arrays and
 * writes a fourth, 3 reads two and writes two; every array holds `bytes`
 * (a positive multiple of 4096), each workgroup moves one 4 KiB chunk per
 * array with nontemporal loads and stores, as the transform passes do.
 * gbs (host): bytes moved per second / 1e9, best of reps timed launches
 * after one warm-up.  Allocates and frees its arrays; runs on hip_stream and
 * returns when done.  Errors: RDM_E_INVALID (pattern, reps < 1, bytes),
 * RDM_E_NOMEM, RDM_E_DEVICE. */
rdm_status rdm_stream_probe(int32_t pattern, uint64_t bytes, int32_t reps, void* hip_stream, double* gbs);

/* ---- Serving: continuous batching over one device stream ---- */

typedef struct rdm_server rdm_server;

/* Start a serving engine on the current device.  hbm_budget: device bytes the
 * engine may hold for admitted requests (0 = free memory minus a reserve);
 * max_active: most requests resident at once (0 = 64).  precision: as
 * rdm_options.  A worker thread owns the device work. */
rdm_status rdm_server_create(uint64_t hbm_budget, int32_t max_active, int32_t precision,
                             rdm_server** out);
/* Queue a solve (non-blocking).  The Hamiltonian must outlive the request;
 * beta is copied.  ticket: host out.  Outputs are written into the caller's
 * result buffers when the request completes. */
rdm_status rdm_server_submit(rdm_server* s, const rdm_hamiltonian* h, const double* beta,
                             int32_t n_beta, int32_t n_v, int32_t k, uint64_t seed,
                             rdm_result out, uint64_t* ticket);
/* done = 1 once the ticket's results are in its buffers; status = the solve's
 * status.  Non-blocking.  A ticket has one owner: the poll that reports it
 * done retires it, and a ticket retired or being waited for by
 * rdm_server_wait gives RDM_E_INVALID. */
rdm_status rdm_server_poll(rdm_server* s, uint64_t ticket, int32_t* done, rdm_status* status);
/* Block until the ticket completes, then retire it.  RDM_E_INVALID for an
 * unknown or retired ticket, or one another thread already waits for. */
rdm_status rdm_server_wait(rdm_server* s, uint64_t ticket, rdm_status* status);
/* Cancel a request: one still queued completes at once, one resident leaves
 * the engine at its next step boundary (its memory returns once the steps
 * already launched for it are done), one being finished is finished unless
 * it still has a regeneration pass to run.  A cancelled request completes
 * with status RDM_E_CANCELLED and its result buffers are not written.
 * RDM_OK also when the request had completed already (its status tells);
 * RDM_E_INVALID for an unknown or retired ticket or one being waited for. */
rdm_status rdm_server_cancel(rdm_server* s, uint64_t ticket);
/* Counters: out[0] submitted, [1] completed, [2] active, [3] queued, [4] engine
 * steps, [5] peak active, [6] peak device bytes.  host out, 7 int64. */
rdm_status rdm_server_stats(rdm_server* s, int64_t* out);
/* Drain outstanding work and stop the engine. */
void rdm_server_destroy(rdm_server* s);

/* Message of the calling thread's last failure (valid until its next call). */
const char* rdm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RDM_H */
