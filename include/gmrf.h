/*
 * gmrf.h -- C ABI of the MI355X (gfx950) Krylov sampler and log-determinant library.
 *
 * Method: Simpson, Turner, Strickland & Pettitt, "Scalable iterative methods for sampling
 * from massive Gaussian random vectors" (arXiv 1312.1476).
 *   - Algorithm 1 (Section 4): Lanczos approximation x_m = ||z|| V_m T_m^{-1/2} e_1 of
 *     x = Q^{-1/2} z for a sparse SPD precision Q, only products Q v being needed (Section 2).
 *   - Theorem 1 (Section 4): the error is bounded by lambda_min^{-1/2} ||r_m||, r_m the
 *     conjugate-gradient residual of Q y = z; its relative size rho_m is the stopping test.
 *   - Proposition 1 (Section 5): sampling with a factored preconditioner M = F F^T; here M is
 *     the periodic (block-circulant) version of a lattice Q, applied with 2D FFTs (Section 5.1).
 *   - Section 6: Hutchinson estimate of log det Q with Rademacher probes, each quadratic form
 *     v^T log(Q) v evaluated by Lanczos (Gauss) quadrature; Section 6.2: preconditioned split
 *     log det Q = log det(F^{-1} Q F^{-T}) + 2 log det F.
 *
 * Conventions shared by every entry point
 *   - Functions never abort or throw; they return a gmrf_status.  A thread-local message for
 *     the last failure is available from gmrf_last_error().
 *   - Vectors are column-major blocks: n rows (lattice points, row-major lattice order
 *     i = (i1*N2 + i2)*N3 + i3) times k columns (right-hand sides, probes).
 *   - "Device" pointers are HIP device allocations on the current device; "host" pointers
 *     are ordinary host memory.  The caller owns every buffer it passes; the library owns
 *     the memory behind a gmrf_op handle and its own scratch.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are stream-ordered: their
 *     kernels run after the work already queued on `stream` (a call that spreads its columns
 *     over side streams forks them from `stream` with an event and joins them back), and work
 *     queued on `stream` afterwards runs after them.  Sample, solve and log-det calls also
 *     synchronise their own work before returning -- the stop polls read rho_j from the device,
 *     and `info` and the host outputs are written after that internal sync -- so X is complete
 *     on return; Z and X need to stay valid only for the duration of the call.
 *   - Calls that share one gmrf_op may run concurrently; each call has its own scratch.
 */
#ifndef GMRF_H
#define GMRF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GMRF_OK = 0,
    GMRF_EINVAL = 1,        /* bad argument; outputs untouched                              */
    GMRF_ENOTSPD = 2,       /* alpha_j <= 0, a pivot d_j <= 0 or T_m not positive definite   */
    GMRF_ENOCONV = 3,       /* per right-hand side: rho_m > tol at m = m_max (X holds x_m)   */
    GMRF_ENOMEM = 4,        /* device allocation failed or the HBM budget would be exceeded  */
    GMRF_EDEVICE = 5,       /* no usable gfx950 device, or a HIP runtime error               */
    GMRF_EUNSUPPORTED = 6   /* valid request outside this build (e.g. FFT on non-2^p sides)   */
} gmrf_status;

typedef enum { GMRF_F64 = 0, GMRF_F32 = 1 } gmrf_dtype;   /* storage of Krylov vectors + Q */
typedef enum { GMRF_FREE = 0, GMRF_PERIODIC = 1 } gmrf_boundary;

typedef struct gmrf_op gmrf_op;       /* opaque, device resident */

/* Per right-hand-side result of gmrf_sample.
 *   m_used       Krylov dimension m of the returned x_m
 *   status       GMRF_OK, GMRF_ENOCONV, GMRF_ENOTSPD or GMRF_EINVAL (non-finite column of Z)
 *   rel_residual rho_m = ||r_m|| / ||z||, r_m the CG residual of Theorem 1 (of A = F^{-1}QF^{-T}
 *                when preconditioned), from the LDL^T pivots of T_m
 *   err_bound    lambda_lb^{-1/2} rho_m: Theorem 1's a posteriori bound on ||x - x_m|| / ||z||
 *                (on ||u - u_m|| / ||z|| when preconditioned) using an analytic lower bound
 *                lambda_lb on lambda_min (tau*kappa2 for first-order lattices, tau*kappa2^2 for
 *                second order); NaN when no bound is known (CSR, preconditioned).          */
typedef struct {
    int32_t m_used;
    int32_t status;
    double rel_residual;
    double err_bound;
} gmrf_info;

/* ---- operators (Section 2: Q is only accessed through products Q v) -------------------- */

/* Lattice precision on a regular 1D/2D/3D lattice with shape[0..ndim-1] points per axis:
 *   order 1:  Q = tau (kappa2 I + L)        (5-point in 2D, 7-point in 3D)
 *   order 2:  Q = tau (kappa2 I + L)^2      (13-point in 2D)
 * L is the graph Laplacian of the grid (bc = GMRF_FREE) or torus (bc = GMRF_PERIODIC) graph.
 * Matrix free: no coefficients are stored.  storage selects FP64 or FP32 Krylov vectors
 * (Lanczos scalars, reductions and the tridiagonal step are FP64 in both).
 * EINVAL: ndim not in 1..3, a side < 1, order not 1/2, tau <= 0, non-finite kappa2.        */
gmrf_status gmrf_op_create_lattice(int ndim, const int64_t* shape, int order, double kappa2,
                                   double tau, gmrf_boundary bc, gmrf_dtype storage,
                                   gmrf_op** out);

/* General sparse SPD Q in CSR form (host arrays, copied to the device; 0-based indices,
 * row_ptr[n] = nnz).  Symmetry is the caller's responsibility; a non-SPD Q is reported as
 * GMRF_ENOTSPD by the sampling calls.  EINVAL: n < 1, bad row_ptr or out-of-range column. */
gmrf_status gmrf_op_create_csr(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                               const double* values, gmrf_dtype storage, gmrf_op** out);

/* Proposition 1 with M = the periodic version of a 2D lattice Q (block circulant), F = M^{1/2}
 * its symmetric root, applied with 2D FFTs (Section 5.1).  Sampling then runs Algorithm 1 on
 * A = M^{-1/2} Q M^{-1/2} and returns x = M^{-1/2} u_m; log det adds log det M (Section 6.2).
 * EUNSUPPORTED: not a 2D lattice, or a side that is not a power of two in [8, 4096].      */
gmrf_status gmrf_op_set_circulant_precond(gmrf_op* Q, int enable);

/* Q <- Q + diag(d) for a lattice operator: d is a host array of n finite values (copied; NULL
 * removes the term).  The log-Gaussian Cox process proposal of Section 3 samples
 * N(0, (Q + H)^{-1}) with Q the periodic prior and H the diagonal Fisher information; Section 5.1
 * (Theorem 2, alpha_n = 0) preconditions it with M = Q.  With circulant preconditioning enabled
 * the operator must be periodic, M stays the lattice part, and sampling runs Algorithm 1 on
 * A = I + M^{-1/2} H M^{-1/2} (two 2D FFTs per step); log det adds log det M.  Sampling or log det
 * of Q + diag(d) without preconditioning returns EUNSUPPORTED (pass such a Q as CSR);
 * gmrf_op_apply includes the term.  EINVAL: non-finite value.  EUNSUPPORTED: CSR operator, or
 * preconditioning on a free-boundary lattice.                                                 */
gmrf_status gmrf_op_set_diagonal(gmrf_op* Q, const double* d);

/* Proposition 1 with M = L L^T from an incomplete Cholesky factorisation of a CSR operator and
 * F = L (Section 5.2, Figure 3): sampling runs Algorithm 1 on A = L^{-1} Q L^{-T} and returns
 * x = L^{-T} u_m; log det adds 2 sum log l_ii.  The factorisation runs on the host when the
 * preconditioner is set (left looking on C = Q + shift diag(Q)):
 *   droptol >= 0: an off-diagonal entry is dropped when its numerator c_ij - sum_k l_ik l_jk is
 *                 below droptol * ||Q[:, j]||_2 in magnitude (droptol = 0: complete Cholesky);
 *   droptol <  0: zero fill, IC(0) (entries only where Q_ij != 0).
 * A non-positive pivot restarts with the next shift of 0, 1e-3, 2e-3, 4e-3, ...; *shift_used (may
 * be NULL) receives the shift.  Each step then costs two level-scheduled triangular solves (one
 * block per column, a barrier between levels; the number of levels bounds the speed).
 * enable = 0 removes the preconditioner.  EUNSUPPORTED: not a CSR operator.  ENOTSPD: breakdown
 * at every shift.  EINVAL: NaN droptol.                                                         */
gmrf_status gmrf_op_set_ichol_precond(gmrf_op* Q, int enable, double droptol, double* shift_used);

/* Size of the incomplete-Cholesky factor of a handle: nonzeros of L (with the diagonal), number
 * of levels of the forward solve, the diagonal shift used.  EINVAL without the preconditioner.  */
gmrf_status gmrf_ichol_info(const gmrf_op* Q, int64_t* nnz_L, int32_t* levels, double* shift);

/* Device bytes one gmrf_sample call needs for k right-hand sides and m_max steps (Krylov
 * basis, work vectors, partial sums, FFT scratch, the tridiagonal step; each allocation rounded
 * up to the scratch pool's 2 MiB granularity), plus what the handle keeps resident.        */
gmrf_status gmrf_op_bytes(const gmrf_op* Q, int64_t k, int32_t m_max, int reorth, size_t* bytes);

/* The same for gmrf_sample_two_pass: three Krylov slots, both passes' scalars, the tridiagonal
 * step and, when preconditioned, the accumulator of u_m.                                    */
gmrf_status gmrf_op_bytes_two_pass(const gmrf_op* Q, int64_t k, int32_t m_max, size_t* bytes);

/* Lattice size n of the operator. */
gmrf_status gmrf_op_size(const gmrf_op* Q, int64_t* n);

/* Y = Q X for k columns, X and Y device buffers in the operator's storage dtype (n x k,
 * column-major).  The SpMV/SpMM kernel of the sampler on its own (Section 2).            */
gmrf_status gmrf_op_apply(const gmrf_op* Q, const void* X, void* Y, int64_t k, void* stream);

/* Y = M^{-1/2} X (real space, storage dtype, device) for a handle with circulant
 * preconditioning enabled: the FFT multiplier of Proposition 1 on its own.              */
gmrf_status gmrf_precond_apply(const gmrf_op* Q, const void* X, void* Y, int64_t k, void* stream);

void gmrf_op_destroy(gmrf_op* Q);

/* ---- sampling: Algorithm 1 (Section 4), Proposition 1 (Section 5) ---------------------- */

/* X[:, r] = x_m for each column z = Z[:, r] (Z, X: device FP64, n x k column-major).
 * tol > 0: stop at the first m with rho_m <= tol (or at breakdown), else at m_max with
 *          status GMRF_ENOCONV for that column;  tol <= 0: exactly m_max steps.
 * reorth:  0 = plain three-term recurrence, 1 = full reorthogonalisation (classical
 *          Gram-Schmidt applied twice against all stored basis vectors).
 * info:    host array of k entries (may be NULL).
 * Returns GMRF_OK when every column ended OK or ENOCONV; GMRF_ENOTSPD if some column was
 * not positive definite (its X column is NaN); EINVAL/ENOMEM/EDEVICE on call failure.    */
gmrf_status gmrf_sample(const gmrf_op* Q, const double* Z, int64_t k, double tol,
                        int32_t m_max, int reorth, double* X, gmrf_info* info, void* stream);

/* As gmrf_sample, and also copies the Lanczos coefficients out (host arrays, may be NULL):
 * alpha[r * m_max + j - 1] = alpha_j (j = 1..m_used), beta[r * (m_max + 1) + j] = beta_j
 * (j = 0..m_used, beta_0 = ||z||).                                                         */
gmrf_status gmrf_sample_ex(const gmrf_op* Q, const double* Z, int64_t k, double tol,
                           int32_t m_max, int reorth, double* X, gmrf_info* info,
                           double* alpha, double* beta, void* stream);

/* X[:, r] = x_m ~= Q^{-1} B[:, r] by the same recurrence: x_m = ||b|| V_m T_m^{-1} e_1, the Lanczos
 * form of the conjugate-gradient iterate, whose relative residual ||b - Q x_m|| / ||b|| is the
 * rho_m of Theorem 1 (so tol is a residual tolerance).  With a preconditioner F (circulant,
 * diagonal term, incomplete Cholesky) it solves A u = F^{-1} b and returns F^{-T} u: preconditioned
 * conjugate gradients on the sampler's kernels, e.g. the sMMALA proposal mean (Q + H)^{-1} grad
 * of Section 3 with M = Q.  Arguments, info and return as for gmrf_sample (B, X: device FP64).  */
gmrf_status gmrf_solve(const gmrf_op* Q, const double* B, int64_t k, double tol, int32_t m_max,
                       int reorth, double* X, gmrf_info* info, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): gmrf_sample with every scratch buffer (Krylov basis,
 * work vectors, Lanczos scalars, partial sums, tridiagonal scratch) carved from one static device
 * array of 128 MiB that the library holds on each GPU it runs on until the process ends.  The call
 * makes no hipMalloc, hipFree or other allocating call; the caller still owns Z, X and info.
 * The columns run as one group on `stream` (results equal gmrf_sample's, whose preconditioned
 * calls split the columns over two streams).  Arguments, info and return as for gmrf_sample, with
 * k <= 256.  ENOMEM (before any kernel runs) when the call's scratch exceeds 128 MiB, e.g.
 * (m_max + 2) k n s bytes of Krylov basis with s = 8 (FP64) or 4 (FP32) must fit.  Every call on
 * a GPU shares that GPU's array and leaves its contents behind (each call clears what must start
 * at zero).  Overlapping calls on one GPU would race on it, so the library serialises the calls of
 * a process (each returns after its work on the device has finished); each process has its own
 * copy of the array.                                                                             */
gmrf_status gmrf_sample_noalloc(const gmrf_op* Q, const double* Z, int64_t k, double tol,
                                int32_t m_max, int reorth, double* X, gmrf_info* info,
                                void* stream);

/* As gmrf_sample without reorthogonalisation, in O(n k) device memory instead of O(n k m_max):
 * the sampler keeps three Krylov vectors (the O(n) storage Section 1 claims for the method).
 * Pass 1 runs the recurrence with the stopping rule and keeps only alpha_j, beta_j; after
 * y = T_m^{-1/2} e_1 pass 2 runs the same recurrence from z again and adds beta_0 y_t v_{t+1}
 * into X as each vector appears (x_m = ||z|| V_m y, Algorithm 1).  Every reduction has a fixed
 * order, so pass 2 reproduces pass 1's vectors bit for bit.  Twice the recurrence's traffic; no
 * reorthogonalisation (it needs the basis).  Arguments, info and return as for gmrf_sample
 * (err_bound NaN).                                                                             */
gmrf_status gmrf_sample_two_pass(const gmrf_op* Q, const double* Z, int64_t k, double tol,
                                 int32_t m_max, double* X, gmrf_info* info, void* stream);

/* Uneven batch: Algorithm 1 for many independent lattice fields in one set of launches per
 * Lanczos step (every kernel of the iteration covers all fields' columns).  Field f is
 * ops[f] with k[f] right-hand sides; all fields share ndim, order and storage (shape, kappa2,
 * tau and boundary may differ); no preconditioning (EUNSUPPORTED) and no reorthogonalisation.
 * Z and X (device FP64) are the concatenation of the fields' n_f x k_f column-major blocks;
 * info (host, may be NULL) has sum_f k[f] entries in the same order.  tol, m_max and the
 * return value as for gmrf_sample.                                                          */
gmrf_status gmrf_sample_batch(int32_t n_fields, const gmrf_op* const* ops, const int64_t* k,
                              const double* Z, double tol, int32_t m_max, double* X,
                              gmrf_info* info, void* stream);

/* ---- log-determinant: Section 6 (Hutchinson + Lanczos quadrature) ---------------------- */

/* log det Q ~= N^{-1} sum_p Gamma_p with Gamma_p = ||v_p||^2 e_1^T log(T_m) e_1 from m steps
 * of the recurrence started at probe v_p (no reorthogonalisation).
 * probes: NULL = Rademacher probes from `seed` (Philox4x64-10 rule, see gmrf_rademacher),
 *         else a device int8 n x n_probes block of +-1 entries.
 * Outputs (host): *logdet = mean, *std_err = sd(Gamma)/sqrt(N) (NaN for N = 1),
 * per_probe[p] = Gamma_p (may be NULL).  With circulant preconditioning the estimate is
 * Hutchinson on A = M^{-1/2} Q M^{-1/2} plus the closed-form log det M (Section 6.2, with the
 * sign that makes det(F^{-1} Q F^{-T}) = det Q / det(F)^2 hold).                            */
gmrf_status gmrf_logdet(const gmrf_op* Q, int32_t n_probes, int32_t m, uint64_t seed,
                        const int8_t* probes, double* logdet, double* std_err,
                        double* per_probe, void* stream);

/* Coloured Hutchinson (Section 6.1): colour (host, n entries in 0..n_colours-1) partitions the
 * lattice points; probe p is the Rademacher probe of gmrf_logdet's rule split by class, and each
 * class runs its own quadrature: Gamma_p = sum_c ||v_pc||^2 e_1^T log(T_m,c) e_1 (+ log det M when
 * preconditioned).  Unbiased for any partition; a colouring of the graph of Q^p
 * (gmrf_distance_colouring) keeps nodes within p steps in different classes and so removes the
 * largest off-diagonal terms of log(Q) from the variance.  Runs n_probes * n_colours Lanczos columns
 * (at most 65535).  Outputs as for gmrf_logdet (per_probe[p] = Gamma_p).  EINVAL: a colour out of
 * range.                                                                                      */
gmrf_status gmrf_logdet_coloured(const gmrf_op* Q, int32_t n_probes, int32_t m, uint64_t seed,
                                 const int32_t* colour, int32_t n_colours, double* logdet,
                                 double* std_err, double* per_probe, void* stream);

/* Distance-p colouring for the coloured estimator (Section 6.1): first fit in lattice-point order,
 * each point taking the smallest colour not used by an already coloured point within p steps of
 * it in the graph of Q (i.e. adjacent in the graph of Q^p).  Lattice handles: points within L1
 * distance p * order (wrapped on periodic lattices); CSR handles: breadth-first search on the
 * pattern.  colour: host array of n entries; *n_colours: number of classes.  p = 0: one class.  */
gmrf_status gmrf_distance_colouring(const gmrf_op* Q, int32_t p, int32_t* colour, int32_t* n_colours);

/* Rademacher probes (Section 6) into a device int8 n x n_probes block:
 *   v_p[i] = +1 if bit (i mod 256) mod 64 of word (i mod 256) / 64 of
 *            Philox4x64-10(counter = (i / 256, p, 0, 0), key = (seed, 0)) is 0, else -1.
 * Philox4x64-10 is the counter-based generator of Salmon et al. (SC'11).                    */
gmrf_status gmrf_rademacher(uint64_t seed, int64_t n, int32_t n_probes, int8_t* out,
                            void* stream);

/* ---- the tridiagonal step on its own (Algorithm 1, final step; Section 6 quadrature) --- */

/* For each of k tridiagonal matrices T_r = tridiag(beta_r, alpha_r, beta_r) of size m[r]
 * (device arrays: alpha[r * ld + i], beta[r * ld + i] the off-diagonal (i < m[r] - 1),
 * m[r] <= ld):  y[r * ld + i] = (T_r^{-1/2} e_1)_i.  Computed by a trapezoidal rule for
 * lambda^{-1/2} = (2/pi) int exp(s) / (exp(2s) + lambda) ds on the real line: the rational
 * approximation of T^{-1/2} that the caption of Algorithm 1 suggests.  status[r] (device)
 * = GMRF_OK or GMRF_ENOTSPD.  ld <= 16384 (EINVAL otherwise); this is also the longest
 * recurrence (m_max, quadrature m) the samplers and the log-det estimators accept.  Up to
 * ld = 1024 T is staged on chip, beyond that read from device memory: the same bits.      */
gmrf_status gmrf_tridiag_invsqrt_e1(const double* alpha, const double* beta, const int32_t* m,
                                    int32_t k, int32_t ld, double* y, int32_t* status,
                                    void* stream);

/* out[r] = e_1^T log(T_r) e_1 (device), same layout; log(lambda) =
 * int exp(s) (1/(1 + exp(s)) - 1/(lambda + exp(s))) ds by the trapezoidal rule.            */
gmrf_status gmrf_tridiag_log_e1(const double* alpha, const double* beta, const int32_t* m,
                                int32_t k, int32_t ld, double* out, int32_t* status,
                                void* stream);

/* ---- measurement ------------------------------------------------------------------------ */

/* Times one kernel of the sampling path on its own: `reps` launches between two HIP events
 * recorded on `stream`, on scratch buffers of the handle's shape with k columns.
 *   which 0: Y = Q X (the operator's SpMV/SpMM kernel),  1: step kernel of the
 *   preconditioned step (writes w_j from v_j, v_{j-1} and the boundary tables, with the dot
 *   products the next step needs),  2: dot-product kernel of the preconditioned step (one read
 *   of a vector),  3: the update w = q - alpha v of the unpreconditioned step,  4: band kernel
 *   of the preconditioned step,  5: row pass and 6: column pass of the preconditioned step of
 *   Q + diag(d) (gmrf_op_set_diagonal),  7: one-pass Lanczos step of a 2D lattice without
 *   preconditioning (w_j from v_j and v_{j-1} with the sums the next step needs).
 * Krylov slots are filled with seeded +-1 values and the scalar state with ones (every column
 * active, no stop decision triggers), other scratch with zeros, before the first event.
 * Outputs (host): *avg_us = mean duration of one launch,
 * *bytes = algorithmic bytes of one launch (inputs read once, outputs written once; 0 for the
 * band kernel, whose traffic is the small boundary tables).  EINVAL for 1, 2, 4 without
 * preconditioning or with a diagonal term, for 5, 6 without both, for 7 on other operators.                            */
gmrf_status gmrf_kernel_bench(const gmrf_op* Q, int which, int64_t k, int32_t reps, double* avg_us,
                              double* bytes, void* stream);

/* Autotuner (for the batching and sampling paths): times, with `reps` launches between HIP events
 * on scratch data of Q's shape with k columns, every candidate set of launch options of the
 * kernels such calls launch on a 2D lattice -- the operator's SpMM (gmrf_op_apply) and, without
 * preconditioning or diagonal term, the one-pass Lanczos step -- and records the fastest in a
 * process-wide table keyed by (kernel, order, storage, ceil(log2) of each side, ceil(log2 k)).
 * The options are the tile order (linear, or XCD-contiguous so that each of the 8 XCDs, each with
 * its own L2, works through one range of neighbouring tiles) and the store policy of the output
 * (ordinary or non-temporal), and for the SpMM alone its tile shape: rows per wave and columns
 * per lane.  No option changes what is computed or the order of any sum (the SpMM has no sums
 * across points, so its tiling is free; the Lanczos step's partial sums follow its tiles, so its
 * shape stays the lattice's rule), so results are bitwise the same under every table state.
 * chosen (host, may be NULL): [2] chosen option bits (1 = XCD-contiguous, 2 = non-temporal
 * stores; bits 2-3 rows per wave 0 = rule / 8 / 16 / 32, bits 4-5 columns per lane 0 = rule /
 * 1 / 2 / 4; -1 = kernel not used by Q).  Other operators are left untuned (GMRF_OK, chosen = -1). */
gmrf_status gmrf_autotune(const gmrf_op* Q, int64_t k, int32_t reps, int32_t* chosen, void* stream);

/* The tuning table as `count` entries of 7 int32 (kernel 0 = SpMM, 1 = one-pass step; order;
 * storage; ceil(log2 N1); ceil(log2 N2); ceil(log2 k); option bits); at most `cap` are written
 * to entries (host), *count receives the table size.  gmrf_tune_import adds or replaces entries
 * in the same format (EINVAL for an invalid entry, the table then unchanged); gmrf_tune_clear
 * empties the table (every launch then takes no options).                                       */
gmrf_status gmrf_tune_export(int32_t* entries, int32_t cap, int32_t* count);
gmrf_status gmrf_tune_import(const int32_t* entries, int32_t count);
gmrf_status gmrf_tune_clear(void);

/* Achievable HBM bandwidth of the device (the roofline denominator beside the published peak):
 * `reps` launches of a streaming kernel over freshly allocated arrays of `bytes` bytes each
 * (a multiple of 16, at least 1 MiB; use 1 GiB or more to stay beyond the 256 MB Infinity
 * Cache), non-temporal 16-byte accesses, `blocks` workgroups of 256 threads (0: 32 per compute
 * unit), each streaming one contiguous chunk of the arrays.
 *   which 0: read (sum of a),  1: copy (b = a),  2: triad (a = b + q c).
 * Outputs (host): *avg_us = mean launch duration, *gbs = bytes moved (1, 2 or 3 arrays) per
 * launch / *avg_us, in GB/s.  The arrays are freed before returning.                          */
gmrf_status gmrf_bandwidth_bench(int which, size_t bytes, int32_t blocks, int32_t reps, double* gbs,
                                 double* avg_us, void* stream);

/* ---- memory budget and errors ---------------------------------------------------------- */

/* Cap on device bytes held by the library's scratch pool (0 = no cap).  Calls that would
 * exceed it return GMRF_ENOMEM without running.  Every call also returns the pool's cached
 * free blocks (scratch of finished calls kept for reuse) to the device.                     */
gmrf_status gmrf_set_hbm_budget(size_t bytes);
size_t gmrf_hbm_in_use(void);

/* Reserve one device region of `bytes` (rounded up to 2 MiB) for the scratch pool: from then on
 * every call's scratch is carved from it (blocks above 64 MiB best fit from the bottom, smaller
 * ones from the top end; free ranges merged when blocks return)
 * and the pool makes no further device allocations or releases, whose cost on this part is
 * irregular (up to seconds for 100 GB, and a release waits for the whole device).  For servers
 * whose request sizes vary.  A call whose scratch finds no free range large enough returns
 * GMRF_ENOMEM without running (it may succeed once running calls have returned theirs).
 * bytes = 0 releases the region.  Reserving or releasing while calls hold scratch from the
 * region returns GMRF_EINVAL; cached blocks outside the region are returned to the device
 * first.  The budget (gmrf_set_hbm_budget) still applies to what calls hold.                 */
gmrf_status gmrf_pool_reserve(size_t bytes);

typedef struct {
  size_t reserved_bytes;       /* size of the reserved region (0: none)                      */
  size_t largest_free_range;   /* largest free range in the region                           */
  size_t in_use;               /* scratch bytes held by running calls                        */
  size_t cached;               /* freed blocks kept for reuse outside the region             */
  uint64_t device_allocs;      /* hipMalloc calls made by the pool since load                */
  uint64_t device_frees;       /* hipFree calls made by the pool since load                  */
  double alloc_seconds;        /* wall time spent in them                                    */
  double free_seconds;
} gmrf_pool_info;

/* The pool's state and its device-allocator counters (host struct, filled in).               */
gmrf_status gmrf_pool_query(gmrf_pool_info* info);

const char* gmrf_strerror(gmrf_status s);
const char* gmrf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GMRF_H */
