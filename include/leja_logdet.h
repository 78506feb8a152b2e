/*
 * leja_logdet.h -- C ABI of the MI355X (gfx950) Léja + Hutch++ log-determinant
 * library.
 *
 * The method is that of "Novel technique based on Léja Points Approximation for
 * Log-determinant Estimation of Large matrices" (arXiv 2603.02207):
 *   - log det Q = tr log Q (Sec. 2, Eqs. Léja1-Léja2);
 *   - the spectral interval [lmin, lmax] is mapped from [-2, 2] (Sec. 3.1,
 *     Eqs. z_mapping, eq_centre, eq_gamma) and log is interpolated at real fast
 *     Léja points (Eq. Léja5) in Newton form (Eq. Léja6);
 *   - the divided differences come from the scaled Taylor expansion of the
 *     matrix logarithm of the Léja bidiagonal matrix (Alg. 1);
 *   - log(Q~)v is applied by the Newton recurrence (Alg. 2);
 *   - the trace is estimated by Hutch++ (Sec. 4.1, Alg. 3), after the scaling
 *     Q~ = Q/sigma (Eq. scaled_sigma_matrix).
 *
 * Conventions for every entry point:
 *   - Return value: LD_OK (0) on success, a negative LD_E* code on failure; no
 *     exception crosses the ABI.  ld_error_string() names the code; the
 *     thread-local ld_last_error_detail() gives a human-readable reason.
 *   - Matrix and vector data are DEVICE pointers owned by the caller; the
 *     library never frees them.  Dense blocks are row-major n x ncols
 *     (row r holds its ncols entries contiguously), element type = the
 *     matrix dtype.
 *   - Work is ordered on the caller's HIP stream (`stream`, a hipStream_t
 *     passed as void*; NULL = the default stream).  Calls that return host
 *     scalars synchronise that stream before returning.
 *   - Scratch memory comes from the caller's workspace (ld_workspace_size),
 *     which must be 256-byte aligned (LD_EINVAL otherwise); with
 *     workspace == NULL the library allocates and frees it itself.
 *   - The matrix must be symmetric positive definite with sorted column
 *     indices in each row (CSR, int32 indices).  Symmetry of the values is
 *     assumed, not checked (the gradient refuses a sparsity pattern that is
 *     not symmetric); the CSR structure is checked unless
 *     opts->trusted_csr != 0.
 *   - Results are deterministic for fixed inputs and options (no atomics in
 *     any reduction).
 */
#ifndef LEJA_LOGDET_H
#define LEJA_LOGDET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define LD_OK 0
#define LD_EINVAL (-1)      /* bad scalar argument or null pointer            */
#define LD_ECSR (-2)        /* row_ptr / col_idx not a valid CSR structure     */
#define LD_EBREAKDOWN (-3)  /* CholQR Gram matrix not positive definite        */
#define LD_EWORKSPACE (-4)  /* caller's workspace too small                    */
#define LD_EHIP (-5)        /* a HIP runtime call failed                       */
#define LD_EINDEF (-6)      /* Gershgorin lower bound <= 0                      */
#define LD_ENOMEM (-7)      /* internal allocation failed                      */

/* ---- element types -------------------------------------------------------- */
#define LD_F32 0            /* float values; bulk recurrence in FP32            */
#define LD_F64 1            /* double values; bulk recurrence in FP64           */

/* ---- scaling value of Alg. 1 (Sec. 3.1) ----------------------------------- */
#define LD_SVAL_CENTER 0    /* s = (lo+hi)/2, optimal by the Lemma of Sec. 3.1 */
#define LD_SVAL_HALF_LMAX 1 /* s = hi/2, the paper's other variant             */

/* ---- how the quadratic forms x^T P_m(Q~) x are accumulated ---------------- */
#define LD_DOT_AUTO 0       /* SQUARED unless its coefficients are ill-conditioned */
#define LD_DOT_FORWARD 1    /* Alg. 2 forward: m steps, <x, w_j> every step    */
#define LD_DOT_SQUARED 2    /* ceil(m/2) steps: <w_a,w_a>, <w_a,w_a+1>          */

/* ld_options.probe_dist */
#define LD_PROBE_RADEMACHER 0  /* +-1: sign of SplitMix64 output (col*n + row + 1)  */
#define LD_PROBE_GAUSSIAN   1  /* Box-Muller on the two 32-bit halves of that output */

/* ld_options.tile_order */
#define LD_TILES_AUTO        0
#define LD_TILES_XCD_BANDS   1  /* XCD x walks the x-th contiguous band of tiles */
#define LD_TILES_INTERLEAVED 2  /* workgroup w takes tiles w, w + grid, ...      */

typedef struct {
    int64_t n;               /* rows = columns                                 */
    int64_t nnz;             /* stored entries, < 2^31                         */
    const int32_t* row_ptr;  /* device, n+1 entries, row_ptr[0] = 0            */
    const int32_t* col_idx;  /* device, nnz entries in [0, n), sorted per row   */
    const void* val;         /* device, nnz entries of float or double         */
    int32_t dtype;           /* LD_F32 or LD_F64                               */
} ld_csr;

typedef struct {
    int32_t s_val_mode;      /* LD_SVAL_CENTER (default) or LD_SVAL_HALF_LMAX  */
    int32_t block_cols;      /* columns per Newton-step launch, rounded up to
                                whole 16-byte vectors.  0 = the library's
                                choice: ld_apply_log takes up to 64 columns at
                                once; the estimate splits the sketch and
                                [Q_b | U] into equal column blocks as wide as
                                the two blocks a step reads and writes allow
                                within 170 MB and, with the matrix as stored,
                                within 240 MB (the Infinity Cache), else one
                                block of at most 64 columns (the gradient's
                                blocks are always of that kind).  The blocks
                                set how the quadratic forms' sums are
                                grouped, hence their last bits              */
    int64_t taylor_cap;      /* max Taylor order of Alg. 1; 0 = 100000000      */
    int32_t ckpt_stride;     /* gradient checkpoint stride; 0 = auto: 1 (every
                                forward vector kept, no recomputation) when the
                                vectors fit 64 GiB, else the smallest stride that
                                fits, at least ceil(sqrt(m))                    */
    int32_t dot_mode;        /* LD_DOT_AUTO / LD_DOT_FORWARD / LD_DOT_SQUARED  */
    int32_t trusted_csr;     /* nonzero: skip the device CSR structure check    */
    int32_t csr_only;        /* nonzero: never use the diagonal storage (the
                                library otherwise builds it, once per call, when
                                every entry lies on one of at most 9 diagonals,
                                and gathers from it instead of the CSR arrays,
                                keeping one value per diagonal when each
                                diagonal's entries are all equal; the same sums
                                in the same order at the same column blocks,
                                but the default blocks follow the stored bytes
                                (see block_cols) and the gradient groups its
                                per-entry sums differently: equal to rounding
                                there)                                         */
    int32_t tile_order;      /* LD_TILES_AUTO / LD_TILES_XCD_BANDS /
                                LD_TILES_INTERLEAVED: how the workgroups of a
                                Newton-step launch walk the row tiles (auto:
                                XCD bands, unless some eighth of the rows holds
                                more than 1.25x its share of the entries, then
                                interleaved); the sums' grouping, hence the
                                last bits of the quadratic forms, depend on it */
    int32_t probe_dist;      /* LD_PROBE_RADEMACHER (default) / LD_PROBE_GAUSSIAN:
                                the distribution of the probe entries of S and
                                G (Alg. 3 step 2 allows either); ld_logdet_estimate
                                gives the generator                           */
} ld_options;

typedef struct {
    double ms_total;         /* wall time of the call (host clock)             */
    double ms_phase1;        /* sketch Y = P_m(Q~) S                           */
    double ms_qr;            /* CholQR2 + deflation                            */
    double ms_phase23;       /* quadratic forms on [Q_b | U] (not run by a
                                gradient call that takes the Newton form)      */
    double ms_adjoint;       /* gradient only: the reverse sweeps and the
                                k-column algebra (in the Newton form also its
                                forward pass over [Q_b, U, S])                 */
    double bytes_alg;        /* algorithmic HBM bytes of the recurrence kernels */
    int64_t taylor_terms;    /* Taylor order used by Alg. 1                    */
    double sigma, lo, hi;    /* scaling and interval of Q~                     */
    int32_t k, k_G;          /* sketch width and residual probe count          */
    int32_t dot_mode_used;   /* LD_DOT_FORWARD or LD_DOT_SQUARED                */
    int32_t spmm_launches;   /* recurrence kernel launches                     */
    double t_low, t_res;     /* the two traces of Alg. 3 steps 5 and 6         */
    /* Recurrence kernels only, timed with HIP events on `stream` around the
     * back-to-back step launches of each phase: */
    double ms_steps1;        /* phase-1 step launches (sketch)                 */
    double ms_steps23;       /* phase-2+3 step launches (quadratic forms)      */
    int32_t launches1, launches23;
    double bytes1, bytes23;  /* algorithmic bytes of those launches            */
    int32_t dia_diagonals;   /* diagonals of the diagonal storage used, 0: CSR */
    int32_t tile_order_used; /* LD_TILES_XCD_BANDS or LD_TILES_INTERLEAVED      */
    int32_t dia_constant;    /* 1: every diagonal holds one value (stored once,
                                with 16 presence bits per row)                */
    int32_t xcd_chunk_rows;  /* with XCD bands: 0 = one contiguous band of rows
                                per XCD; > 0 = the bands are cut into chunks of
                                this many rows dealt to the XCDs in turn (a
                                launch that streams from HBM, or a 3-D stencil
                                whose plane neighbours would not stay in an
                                XCD's L2), as the quadratic-form launches took
                                them (0 when a chunk is not a whole number of
                                their tiles)                                   */
    int32_t block_cols1;     /* column block width of the sketch's launches    */
    int32_t block_cols23;    /* and of the quadratic forms' (see block_cols)   */
    int32_t ranges23;        /* launches per quadratic-form step: 1, or the
                                consecutive row ranges a step that streams
                                from HBM on a far-reaching stencil takes      */
} ld_stats;

/* Defaults for ld_options (all zero except as documented). */
void ld_default_options(ld_options* opts);

/* Library version string: "leja_logdet <version> (gfx950) src=<hash>", the hash
 * being the first 16 hex digits of SHA-256 over the source files the library
 * was built from (the build script computes it). */
const char* ld_version(void);

/* Name of an error code. */
const char* ld_error_string(int code);

/* Detail of the last error raised on the calling thread ("" if none). */
const char* ld_last_error_detail(void);

/* ---- host-side pieces of the method (no GPU needed) ----------------------- */

/* First `count` real fast Léja points on [-2, 2] (Sec. 3, Eq. Léja5, computed by
 * the fast Léja algorithm the paper cites: maximise prod |x - xi_k| over the
 * midpoints of adjacent points; xi_0 = +2, xi_1 = -2; products equal within a
 * relative 1e-12 are tied and the larger x wins).  xi_host: host, count doubles.
 * Errors: LD_EINVAL if count < 0 or xi_host is NULL with count > 0. */
int ld_leja_points(int32_t count, double* xi_host);

/* Divided differences d_0..d_degree of g(xi) = log(c + gamma*xi) at the Léja
 * points, c = (lo+hi)/2, gamma = (hi-lo)/4 (Sec. 3.1), by the paper's Alg. 1:
 * the first column of log(Q_m) for the Léja bidiagonal matrix Q_m = cI +
 * gamma*Q^_m (Eq. eq_leja_matrix), via log(s) + Taylor series of log(I + W),
 * W = (Q_m - sI)/s, summed until the largest term falls below 2^-60 of the
 * largest entry (at most taylor_cap terms, 0 = 1e8).
 * d_host: host, degree+1 doubles.  terms: host, may be NULL.
 * Errors: LD_EINVAL unless 0 < lo < hi, degree >= 0, valid s_val_mode. */
int ld_divided_differences(double lo, double hi, int32_t degree, int32_t s_val_mode,
                           int64_t taylor_cap, double* d_host, int64_t* terms);

/* Probe entries of the counter-based SplitMix64 generator (Sec. 4.1, Alg. 3
 * step 2 draws +-1 entries with probability 1/2; the generator is a reading):
 * entry (row, col) of stream `stream` = sign of output (col*n + row + 1) of
 * SplitMix64 seeded with key = output (stream+1) of SplitMix64(seed).
 * Writes rows [row0, row0+nrows) x cols [col0, col0+ncols) as int8 +-1,
 * row-major, into out_host.  Errors: LD_EINVAL on negative sizes / NULL. */
int ld_rademacher_host(uint64_t seed, int32_t stream, int64_t n, int64_t row0, int64_t nrows,
                       int64_t col0, int64_t ncols, int8_t* out_host);

/* Coefficients c_0..c_m of the same polynomial in the basis of products
 * q_2a = pi_a^2, q_2a+1 = pi_a pi_a+1 (pi_j = Newton basis at the Léja points),
 * used by LD_DOT_SQUARED so that x^T P(T) x = sum_i c_i nu_i with
 * nu_2a = <w_a, w_a>, nu_2a+1 = <w_a, w_a+1>, w_a = pi_a(T) x.  Computed by
 * repeated change of Newton centres in double-double arithmetic.
 * d_host: in, degree+1; c_host: out, degree+1.  Errors: LD_EINVAL. */
int ld_squared_basis_coefficients(int32_t degree, const double* d_host, double* c_host);

/* ---- device entry points -------------------------------------------------- */

/* Bytes of workspace needed by ld_logdet_estimate (want_grad = 0) or
 * ld_logdet_grad (want_grad = 1) for this matrix, degree and query count, or,
 * when n_matvec is negative (-n_matvec = number of columns), by ld_apply_log
 * (want_grad = 0) or ld_apply_log_adaptive (want_grad = 1).
 * opts may be NULL.  Errors: LD_EINVAL. */
int ld_workspace_size(const ld_csr* A, int32_t degree, int32_t n_matvec, int32_t want_grad,
                      const ld_options* opts, size_t* bytes);

/* PV = P_m(Q~) V + log(sigma) V ~= log(Q) V for a block of ncols vectors
 * (Alg. 2, run in the mapped variable T = (Q~ - cI)/gamma, Horner order;
 * sigma = lmin if lmin < 1 else 1, Eq. scaled_sigma_matrix).
 * V, PV: device, n x ncols row-major, dtype of A, must not overlap.
 * Errors: LD_EINVAL (0 < lmin < lmax, degree >= 1, ncols >= 0), LD_ECSR,
 * LD_EWORKSPACE, LD_EHIP. */
int ld_apply_log(const ld_csr* A, double lmin, double lmax, int32_t degree, const void* V,
                 void* PV, int64_t ncols, const ld_options* opts, void* workspace,
                 size_t ws_bytes, void* stream);

/* Alg. 2 with its adaptive degree, per column: column c starts from w_0 = v,
 * P = d_0 w_0, m = 0 and, while |d_m| ||w_m||_2 > tol and m < max_degree,
 * takes w_{m+1} = (T - xi_m) w_m, m += 1, P += d_m w_m (mapped variable
 * T = (Q~ - cI)/gamma, forward order; tol absolute, as in Alg. 2).  Returns
 * PV = P + log(sigma) V and, in degrees (host, ncols entries, may be NULL),
 * the degree m at which each column stopped (max_degree if it never met tol).
 * The norms are FP64 sums of the column's squares; the stopping test runs on
 * the device after every step, and the host stops launching steps once every
 * column has stopped (checked before the first step, after steps 1, 2 and 4,
 * then every 8 steps).
 * V, PV: device, n x ncols row-major, dtype of A, must not overlap.
 * Errors: LD_EINVAL (0 < lmin < lmax, max_degree >= 1, ncols >= 0, tol finite
 * and >= 0), LD_ECSR, LD_EWORKSPACE, LD_EHIP. */
int ld_apply_log_adaptive(const ld_csr* A, double lmin, double lmax, int32_t max_degree, double tol,
                          const void* V, void* PV, int64_t ncols, const ld_options* opts,
                          void* workspace, size_t ws_bytes, void* stream, int32_t* degrees);

/* Bytes of workspace needed by ld_logdet_estimate_adaptive for this matrix,
 * largest degree and query count.  opts may be NULL.  Errors: LD_EINVAL. */
int ld_adaptive_workspace_size(const ld_csr* A, int32_t max_degree, int32_t n_matvec,
                               const ld_options* opts, size_t* bytes);

/* Alg. 3 with Alg. 2's stopping rule in each of its three applications of
 * log(Q~) (Alg. 3 steps 3, 5 and 6, Sec. 4.1): Y = F S, Q_b = orth(Y) (CholQR2),
 * U = (I - Q_b Q_b^T) G, estimate = n log(sigma) + sum_i q_i^T F q_i +
 * (1/k_G) sum_j u_j^T F u_j, where F x is ld_apply_log_adaptive's P for the
 * column x (forward Newton order, each column its own degree: it stops at the
 * first m with |d_m| ||w_m||_2 <= tol, tol absolute, or at max_degree).
 * Probes, k, k_G, seeds and limits as ld_logdet_estimate.
 * degrees: host, n_matvec int32 (may be NULL): the degree each column stopped
 * at, in the order the columns of S (k), of Q_b (k) and of U (k_G).
 * out_logdet: host double.  stats: host, may be NULL (launches1/launches23 =
 * Newton steps of step 3 / steps 5 and 6; no byte counts).
 * Errors: LD_EINVAL (as ld_logdet_estimate, tol finite and >= 0), LD_ECSR,
 * LD_EBREAKDOWN, LD_EWORKSPACE, LD_EHIP. */
int ld_logdet_estimate_adaptive(const ld_csr* A, double lmin, double lmax, int32_t max_degree, double tol,
                                int32_t n_matvec, uint64_t seed, const ld_options* opts, void* workspace,
                                size_t ws_bytes, void* stream, double* out_logdet, int32_t* degrees,
                                ld_stats* stats);

/* Léja + Hutch++ estimate of log det A (Alg. 3) with n_matvec queries:
 * k = floor(n_matvec/3) sketch columns (probe stream 0), k_G = n_matvec - 2k
 * residual probes (stream 1), degree = number of recurrence steps m.  Probe
 * entry (row, col) of a stream comes from SplitMix64 output x = number
 * (col*n + row + 1) of the stream (see ld_rademacher_host): Rademacher: the
 * sign of x's top bit; Gaussian (opts->probe_dist): sqrt(-2 ln u1) cos(2 pi u2)
 * in FP64 with u1, u2 = (high, low 32 bits of x + 1/2) / 2^32.
 * out_logdet: host double.  stats: host, may be NULL.
 * Limits: 3 <= n_matvec <= 192, i.e. k, k_G <= 64 (the k x k Gram matrices
 * of CholQR are factored by one workgroup on the device, and the quadratic
 * forms take at most 64 columns per launch); k <= n.
 * Errors: LD_EINVAL (0 < lmin < lmax, degree >= 1, the limits above),
 * LD_ECSR, LD_EBREAKDOWN, LD_EWORKSPACE, LD_EHIP. */
int ld_logdet_estimate(const ld_csr* A, double lmin, double lmax, int32_t degree,
                       int32_t n_matvec, uint64_t seed, const ld_options* opts,
                       void* workspace, size_t ws_bytes, void* stream, double* out_logdet,
                       ld_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): ld_logdet_estimate
 * with the library's own static scratch instead of a workspace.  The scratch
 * is a 64 MiB device array of the library, one per GPU, held until the
 * process ends; an estimate whose workspace (ld_workspace_size with
 * want_grad = 0) exceeds 64 MiB returns LD_EWORKSPACE.  The call makes no
 * device allocation and creates no HIP events (so stats carries no kernel
 * timings: its ms_phase and ms_steps fields are 0).  `stream` must belong to
 * the current device (LD_EINVAL otherwise).  All calls on one GPU share its
 * scratch: calls that overlap in time on the same GPU (other host threads,
 * other streams) race and must be serialised by the caller.  Results are
 * those of ld_logdet_estimate with the same arguments.
 * Errors: as ld_logdet_estimate. */
int ld_logdet_estimate_noalloc(const ld_csr* A, double lmin, double lmax, int32_t degree,
                               int32_t n_matvec, uint64_t seed, const ld_options* opts, void* stream,
                               double* out_logdet, ld_stats* stats);

/* As ld_logdet_estimate, and the exact derivative of the returned estimate
 * with respect to each stored value of A (same probes, interval and sigma
 * held fixed; includes the dependence of the sketch basis on A: the
 * estimate's method is Alg. 3 of Sec. 4.1, the derivative is not in the
 * paper).  When the estimate takes the squared basis for its quadratic forms
 * (opts->dot_mode) and k + k_G <= 64, the forward vectors of the estimate's
 * own passes are kept and swept in reverse (the returned estimate is then
 * bit-identical to ld_logdet_estimate's); otherwise one forward pass in the
 * Newton form and one reverse sweep (estimates agree to rounding).  Vectors
 * are kept every opts->ckpt_stride steps (0: all of them while they fit
 * 64 GiB, else the smallest stride that does) and recomputed in between.
 * The quadratic forms' per-entry derivative is symmetric in (r, c) for a
 * symmetric A, so mirrored entries take their mean: A's sparsity pattern
 * must be symmetric.  Sums in FP64 (an FP32 matrix's gradient is rounded to
 * FP32 once).  grad_val: device, nnz entries of A's dtype, overwritten.
 * Errors: as ld_logdet_estimate; LD_EINVAL also when an entry has no mirror. */
int ld_logdet_grad(const ld_csr* A, double lmin, double lmax, int32_t degree, int32_t n_matvec,
                   uint64_t seed, const ld_options* opts, void* workspace, size_t ws_bytes,
                   void* stream, double* out_logdet, void* grad_val, ld_stats* stats);

/* Gershgorin interval [min_i a_ii - r_i, max_i a_ii + r_i], r_i = sum_{j!=i}
 * |a_ij| (Sec. 3; Alg. 1/2 step 1), reduced in FP64 on the device.  With
 * 0 < lanczos_steps <= 512 the upper end is refined as in App. A: that many
 * Lanczos steps (A symmetric; in FP64, an FP32 matrix's values widened
 * once; start vector the unit Rademacher vector of generator stream 2,
 * seed 0; no reorthogonalisation), then the largest Ritz
 * value plus its residual norm beta_k |s_k| plus a rounding margin, and never
 * raised above Gershgorin's bound.  The residual term is the usual practical
 * upper bound, not a guaranteed one.  The lower end is always Gershgorin's.
 * The call allocates its Lanczos vectors (4n doubles, plus nnz doubles for
 * an FP32 matrix).
 * lmin, lmax: host doubles.  Returns LD_EINDEF (with both bounds written) when
 * the lower bound is <= 0.  Errors: LD_EINVAL (null pointers, steps out of
 * range, non-finite values), LD_ECSR, LD_ENOMEM, LD_EHIP. */
int ld_spectral_bounds(const ld_csr* A, int32_t lanczos_steps, void* stream, double* lmin,
                       double* lmax);

#ifdef __cplusplus
}
#endif

#endif /* LEJA_LOGDET_H */
