/*
 * mm.h - C-ABI of the MI355X (gfx950) GLS map-making hot path.
 *
 * Solves A m = b with A = P^T N^-1 P and b = P^T N^-1 d by preconditioned
 * conjugate gradients, after Szydlarski, Grigori & Stompor, "Accelerating the
 * cosmic microwave background map-making procedure through preconditioning",
 * A&A 2014 (arXiv 1408.3048).  Paper references below name the section and
 * the equation's LaTeX label.
 *
 *   P      pointing matrix: row t holds (1, cos 2phi_t, sin 2phi_t) at the
 *          pixel seen at sample t (IQU), or 1 (I only)
 *          [Sect. 2, eq. signal_with_polarization]
 *   N^-1   block-diagonal, one symmetric band-limited Toeplitz block per
 *          stationary interval, built from the interval's noise PSD
 *          [Sect. 2.1, eq. N_def; Sect. 4.1.4, eq. fknee; App. D, eq. apodDef]
 *   M_BD   block-Jacobi preconditioner (P^T diag(N^-1) P)^-1 [Sect. 3.1, eq. stdPrec]
 *   M_2lvl two-level A-DEF1 preconditioner with the a priori coarse space Z_S
 *          [Sect. 3.2, eqs. projection and 2; Sect. 3.3.1, eqs. strofZ, strofZ_polar;
 *           App. C]
 *
 * Conventions for every call:
 *   - Map-domain vectors ("maps") are device arrays of n_obs * n_stokes
 *     doubles in the compact observed-pixel space: compact pixel c is the
 *     c-th smallest original pixel id that occurs in the pointing (Sect. 2:
 *     only observed pixels are solved for), its Stokes parameters I,Q,U are
 *     adjacent.  mm_obs_pixels() returns the compact -> original map.
 *   - Time-domain vectors ("TOD") are device arrays of n_samples values, FP32
 *     or FP64 as stated by a dtype argument (MM_F32 / MM_F64).
 *   - All device work is ordered on the stream given in mm_opts.stream
 *     (a hipStream_t, NULL = the default stream).  Calls return after
 *     enqueueing, except mm_plan and mm_pcg_solve, which synchronise.
 *   - Return value: MM_OK (0) or a negative mm_status.  No call aborts or
 *     throws; on error mm_last_error() returns a message (thread-local,
 *     valid until the next call on the same thread).  Arguments are
 *     validated on the host before any device work is enqueued.
 *   - Caller-owned buffers stay caller-owned; a plan owns deep copies of
 *     everything it needs, so the inputs of mm_plan may be freed after it
 *     returns.  Calls that overlap on one plan from several host threads race.
 *   - Device memory comes from the device's stream-ordered pool.  Blocks the
 *     library frees (mm_destroy, plan-time scratch) are kept for its own later
 *     allocations, up to 16 GiB per device, until the process ends; a block is
 *     reused only after the reusing stream has waited for the work enqueued
 *     before its release, and an allocation the device cannot serve first hands
 *     the kept blocks back to the pool.
 */
#ifndef MM_H
#define MM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_plan_s* mm_plan_t;

enum mm_status {
    MM_OK = 0,
    MM_ERR_ARG = -1,        /* invalid argument (sizes, offsets, pixel ids, NULL pointers) */
    MM_ERR_DEVICE = -2,     /* a HIP runtime call failed */
    MM_ERR_RANK = -3,       /* a pixel's n_s x n_s block has rcond < rcond_min (P not full rank) */
    MM_ERR_NOT_SPD = -4,    /* a Toeplitz block's symbol min <= 0 (N^-1 not positive definite) */
    MM_ERR_BREAKDOWN = -5,  /* PCG: p^T A p <= 0 or not finite; x holds the last iterate */
    MM_ERR_NOCONV = -6,     /* PCG: max_iter reached; x holds the last iterate */
    MM_ERR_STATE = -7       /* the plan was not built with what the call needs */
};

enum { MM_F32 = 0, MM_F64 = 1 };                               /* element types */
enum { MM_WIN_GAUSS = 0, MM_WIN_GAUSS2 = 1, MM_WIN_RECT = 2 };  /* apodisation windows */
enum { MM_FP64 = 0, MM_MIXED = 1, MM_MIXED_IR = 2 };          /* arithmetic of the operator */
enum { MM_COARSE_NONE = 0, MM_COARSE_ZS = 1 };                 /* coarse space built by mm_plan */
enum { MM_BJ = 0, MM_2LVL = 1, MM_ADEF2 = 2 };                 /* preconditioner of mm_pcg_solve */

/* Noise model of one stationary interval: per-sample PSD
 * P(f) = sigma^2 (1 + (f_knee / f)^alpha)  [Sect. 4.1.4, eq. fknee with the
 * slope alpha free; alpha = 2 is the paper's case].  f_knee = 0 is white noise. */
typedef struct { double sigma, f_knee, alpha; } mm_psd;

typedef struct {
    int n_stokes;      /* 1 (I) or 3 (I,Q,U) */
    int lambda;        /* Toeplitz half bandwidth: lags |k| <= lambda kept [Sect. 4.1.4] */
    double f_samp;     /* sampling frequency in Hz (> 0) */
    int window;        /* apodisation of the Toeplitz row [App. D]:
                          MM_WIN_GAUSS w(k) = exp(-(k/lambda)^2) (default),
                          MM_WIN_GAUSS2 exp(-2 (k/lambda)^2), MM_WIN_RECT 1 */
    int precision;     /* MM_FP64: FP64 operator only; MM_MIXED: also FP32 copies of the
                          time-domain data, enabling the FP32 operator and mixed solves */
    int coarse;        /* MM_COARSE_ZS builds Z_S, AZ and E for mm_precond_2lvl */
    double rank_tol;   /* E: columns whose pivoted-Cholesky residual falls below
                          rank_tol * max diag(E) are dropped (span-preserving), default 1e-10 */
    double rcond_min;  /* minimum reciprocal 1-norm condition of a pixel block, default 1e-8 */
    int fft_len_f64;   /* overlap-save FFT length (real samples, power of two) for the FP64
                          operator; 0 = automatic */
    int fft_len_f32;   /* same for the FP32 operator; 0 = automatic */
    void* stream;      /* hipStream_t; NULL = default stream */
    int graph;         /* 1 (default): mm_pcg_solve captures one PCG iteration in a HIP graph
                          on a plan-owned non-blocking stream and replays it; 0: plain
                          launches on the caller's stream */
    int autotune;      /* 1: mm_plan times the candidate FFT lengths on the plan's own data
                          and keeps the fastest (when fft_len_* is 0); 0 (default): cost model */
    int az_fp16;       /* mixed plans with Z_S: 1 (default) the two-level (A-DEF1) apply reads
                          AZ in FP16 with a power-of-two scale per column (half the bytes of
                          FP32; each entry rounded once, relative error <= 2^-11); 0: FP32.
                          E, A-DEF2 and the coarse start keep the FP32 AZ */
    int pt_range;      /* samples per work range of the P^T segmented reduction (a wave takes
                          the whole pixels starting in its range), a power of two in
                          [256, 65536]; 0 = automatic: 2048, or with autotune the fastest of
                          512 / 1024 / 2048 / 4096 timed on the plan's own data.  Results depend on
                          it at rounding level (the order of additions within a pixel) */
} mm_opts;

/* Fill *opts with the defaults above (n_stokes 3, lambda 1024, f_samp 200, graph 1,
 * az_fp16 1). */
void mm_default_opts(mm_opts* opts);

/* Build a plan for one problem [Sect. 2, Sect. 3, App. C]; the same as mm_plan_batched
 * with one problem.
 *   n_samples           N_t, 1 <= N_t < 2^31
 *   pix                 device int32 [N_t], original pixel id in [0, n_pix)
 *   weights             device [N_t][2] = (cos 2phi_t, sin 2phi_t) of type weights_dtype
 *                       for n_stokes = 3 (the I weight is exactly 1 and not passed);
 *                       ignored (may be NULL) for n_stokes = 1
 *   n_pix               size of the original pixel grid
 *   n_intervals         K >= 1 stationary intervals
 *   interval_offsets    host int64 [K+1]: 0 = o_0 < o_1 < ... < o_K = N_t
 *   psd                 host [K] noise model per interval (sigma > 0, f_knee >= 0, alpha > 0)
 * Errors: MM_ERR_ARG (bad sizes/offsets/PSD, pixel id out of range, lambda too large for
 * the FFT tile), MM_ERR_NOT_SPD, MM_ERR_RANK, MM_ERR_DEVICE.  *out is NULL on error. */
int mm_plan(mm_plan_t* out, int64_t n_samples, const int32_t* pix, const void* weights,
            int weights_dtype, int64_t n_pix, int32_t n_intervals,
            const int64_t* interval_offsets, const mm_psd* psd, const mm_opts* opts);

/* Build one plan for n_problems independent problems solved together (many noise
 * realisations or scans of uneven length): A, M_BD and the coarse space are block
 * diagonal over the problems, every operator launch covers all problems at once, and
 * mm_pcg_solve iterates each problem under its own scalars, convergence test and mask
 * (a problem that has converged takes no further part in the launches).
 *   problem_intervals   host int32 [n_problems+1]: problem b owns the intervals
 *                       [problem_intervals[b], problem_intervals[b+1]) and hence the samples
 *                       [interval_offsets[problem_intervals[b]], ...); 0 = first < ... =
 *                       n_intervals
 *   pix                 pixel ids must be disjoint and increasing across problems (every id
 *                       of problem b below every id of problem b+1; e.g. b * n_pix_b + local
 *                       id), so that problem b's observed pixels form the compact block
 *                       [off_b, off_{b+1}) (mm_problem_pixels)
 * Other arguments as mm_plan.  Each problem's results equal, bit for bit, those of a plan
 * built for that problem alone with the same FFT lengths.  Errors as mm_plan; MM_ERR_ARG
 * also for overlapping pixel ranges. */
int mm_plan_batched(mm_plan_t* out, int32_t n_problems, const int32_t* problem_intervals,
                    int64_t n_samples, const int32_t* pix, const void* weights,
                    int weights_dtype, int64_t n_pix, int32_t n_intervals,
                    const int64_t* interval_offsets, const mm_psd* psd, const mm_opts* opts);

/* Number of problems of the plan (1 for mm_plan); -1 on NULL. */
int mm_n_problems(mm_plan_t plan);
/* Host int64 [n_problems+1]: first compact pixel of every problem (map vector entries of
 * problem b: [n_stokes * off_b, n_stokes * off_{b+1})). */
int mm_problem_pixels(mm_plan_t plan, int64_t* host_out);

/* Release a plan and all its device memory (NULL is a no-op; the memory stays with the
 * library for reuse, see above). */
void mm_destroy(mm_plan_t plan);

/* Number of observed pixels n_obs (map vectors hold n_obs * n_stokes doubles); -1 on NULL. */
int64_t mm_n_obs(mm_plan_t plan);
/* n_stokes of the plan; -1 on NULL. */
int mm_n_stokes(mm_plan_t plan);
/* Device int32 [n_obs]: original pixel id of every compact pixel (ascending). */
int mm_obs_pixels(mm_plan_t plan, int32_t* dev_out);
/* Device int32 [n_obs]: hit count s_p of every compact pixel (exact integers). */
int mm_hits(mm_plan_t plan, int32_t* dev_out);
/* Device int32 [N_t]: perm[i] = sample index of the i-th sample in pixel-sorted order
 * (compact pixel ascending, then time ascending; a stable counting sort). */
int mm_sorted_samples(mm_plan_t plan, int32_t* dev_out);

/* Toeplitz taps of interval j (t_0..t_K, K = min(lambda, t_j - 1)) as FP64 on the host
 * [App. D]; returns K+1 or a negative status; at most cap values are written. */
int mm_interval_taps(mm_plan_t plan, int32_t interval, double* host_out, int cap);

/* Coarse space [App. C]: number of columns kept after removing duplicate and dependent
 * columns of Z_S (or of Z_D after mm_coarse_from_krylov) (r_eff), or a negative status. */
int mm_coarse_rank(mm_plan_t plan);
/* Host int32 [r_eff]: interval index of every kept column of Z_S. */
int mm_coarse_columns(mm_plan_t plan, int32_t* host_out, int cap);
/* Host FP64: E = Z^T A Z restricted to the kept columns, row-major; for a batched plan the
 * diagonal block of every problem, concatenated (sum of r_b^2 values). */
int mm_coarse_matrix(mm_plan_t plan, double* host_out, int64_t cap);
/* Host int32 [n_problems+1]: first kept column of every problem. */
int mm_coarse_problem_columns(mm_plan_t plan, int32_t* host_out, int cap);

/* ----- operators (all device pointers; see conventions above) ----- */

/* y = P x  (de-pointing) [Sect. 2].  x: map (FP64); y: TOD of y_dtype. */
int mm_apply_P(mm_plan_t plan, const double* x, void* y, int y_dtype);
/* z = N^-1 y [eq. N_def] with the FP64 (precision MM_FP64, y/z FP64) or FP32 (MM_MIXED,
 * y/z FP32) overlap-save operator.  y and z may not alias. */
int mm_apply_Ninv(mm_plan_t plan, const void* y, void* z, int precision);
/* x = P^T z  (pointing) [Sect. 2]: deterministic segmented reduction over pixel-sorted
 * samples, in ascending sample order per pixel.  z: TOD of z_dtype; x: map (FP64). */
int mm_apply_PT(mm_plan_t plan, const void* z, int z_dtype, double* x);
/* b = P^T N^-1 d [eq. rhs].  d: TOD of d_dtype (FP64 operator). */
int mm_rhs(mm_plan_t plan, const void* d, int d_dtype, double* b);
/* y = A x = P^T N^-1 P x [eq. a_times_x].  precision MM_FP64: FP64 kernels; MM_MIXED:
 * FP32 gather, FFT and scatter with FP32 accumulation (plan must be MM_MIXED).
 * x and y may not alias. */
int mm_apply_A(mm_plan_t plan, const double* x, double* y, int precision);
/* z = M_BD r [eq. stdPrec]. r and z may alias. */
int mm_precond_bj(mm_plan_t plan, const double* r, double* z);
/* z = M_2lvl r = M_BD (r - AZ E^-1 Z^T r) + Z E^-1 Z^T r [eq. 2] with the plan's coarse
 * space (Z_S from MM_COARSE_ZS, or Z_D from mm_coarse_from_krylov; none: MM_ERR_STATE).
 * r and z may not alias. */
int mm_precond_2lvl(mm_plan_t plan, const double* r, double* z);

/* z = M_alt r = R^T M_BD r + Z E^-1 Z^T r, R^T = I - Z E^-1 (AZ)^T [App. B, eq. ADEF2]
 * (A-DEF2) with the plan's coarse space (none: MM_ERR_STATE).  Same spectrum of M A as
 * MM_2LVL; PCG with it starts from x0 + Z E^-1 Z^T (b - A x0), for which it is
 * equivalent to CG with an SPD preconditioner.  r and z may not alias. */
int mm_precond_adef2(mm_plan_t plan, const double* r, double* z);

/* ----- solver ----- */

typedef struct {
    int iterations;        /* total PCG iterations (inner iterations for MM_MIXED) */
    int outer_iterations;  /* iterative-refinement steps (1 for MM_FP64) */
    int replacements;      /* recursive -> true residual replacements */
    int status;            /* MM_OK, MM_ERR_BREAKDOWN or MM_ERR_NOCONV */
    double rel_residual;   /* final true ||b - A x|| / ||b|| with the FP64 operator */
    double solve_ms;       /* wall time of the solve (host clock around device work) */
    double* history;       /* optional caller-owned host buffer for the recursive relative
                              residual of every iteration, or NULL */
    int history_cap;       /* its capacity */
    int history_len;       /* entries written */
} mm_solve_info;

/* Solve A x = b by PCG [Sect. 3] from the initial guess in x (pass zeros for x0 = 0);
 * for a batched plan every problem b solves A_b x_b = b_b (its block of the vectors).
 *   precond    MM_BJ, MM_2LVL (A-DEF1) or MM_ADEF2 (which first replaces x by
 *              x + Z E^-1 Z^T (b - A x))
 *   precision  MM_FP64: FP64 operator; convergence when the recursive and then the true
 *              relative residual are <= tol (otherwise the recursive residual is replaced
 *              by the true one and the iteration continues).
 *              MM_MIXED: PCG with the FP32 operator (FP64 vectors, scalars and coarse
 *              solve) whose recursive residual is replaced by the FP64 true residual
 *              b - A x each time it has dropped by 10^4 since the last replacement and
 *              when it reaches tol (the search direction is kept); stops when the true
 *              relative residual is <= tol.
 *              MM_MIXED_IR: classic iterative refinement; each step solves A d = r with
 *              the FP32-operator PCG from d = 0 and updates x += d; r = b - A x is formed
 *              with the FP64 operator; stops when it is <= tol (single-problem plans).
 *   tol        relative residual target (> 0) of every problem;
 *   max_iter   cap on PCG iterations (per problem).
 *   info       NULL or host array of mm_n_problems(plan) entries, one per problem.
 * Returns MM_OK when every problem converged, else the status of the first that did not
 * (MM_ERR_NOCONV, MM_ERR_BREAKDOWN; x holds the last iterates; info filled), or
 * MM_ERR_ARG / MM_ERR_STATE.  Synchronises the plan's stream before returning. */
int mm_pcg_solve(mm_plan_t plan, const double* b, double* x, int precond, int precision,
                 double tol, int max_iter, mm_solve_info* info);

/* ----- a posteriori coarse space Z_D [Sect. 3.3.2; App. A] ----- */

/* Solve A x = b by block-Jacobi PCG (FP64 operator, from x0 = 0 regardless of x's
 * contents, every problem of a batched plan at once) and build the two-level
 * preconditioner's coarse space from what the solve learns about M_BD A: PCG is the
 * Lanczos process on M_BD A, so its step lengths and preconditioned residuals give the
 * Lanczos matrix T (symmetric tridiagonal) and the basis W (columns (-1)^k z_k /
 * sqrt(r_k^T z_k)); the Ritz pairs (theta_i, y_i = W s_i), T s_i = theta_i s_i [App. A,
 * eq. approxEigen with B = M_BD A], with theta_i < eps_tol become the columns of Z_D
 * (dense, every Stokes row), per problem.  AZ_D and E_D = Z_D^T A Z_D are then formed
 * as for Z_S (pivoted-Cholesky selection with opts.rank_tol), and Z_D replaces the plan's
 * coarse space: later mm_pcg_solve / mm_precond_2lvl calls with MM_2LVL use
 * M_2lvl,D [eq. 2 with Z = Z_D].  Mixed plans keep Z_D and AZ_D in FP32.
 *   b, x        device maps: right-hand side, and the solution of this first system
 *   tol, max_iter   of the recording solve, as in mm_pcg_solve
 *   krylov_dim  basis vectors kept (the first krylov_dim PCG steps; 0: max_iter); the
 *               library holds krylov_dim * n_map FP64 values of device memory during
 *               the call
 *   eps_tol     Ritz-value threshold (the paper uses 0.2)
 *   max_cols    at most this many columns per problem (the smallest Ritz values; 0: no cap)
 *   info        NULL or host array of mm_n_problems(plan) entries (the recording solve)
 * Returns MM_OK; MM_ERR_NOCONV when the solve stopped at max_iter (Z_D is still built
 * from the recorded steps); MM_ERR_RANK when no problem has a Ritz value below eps_tol
 * (the coarse space is then unchanged); MM_ERR_BREAKDOWN, MM_ERR_ARG, MM_ERR_DEVICE.
 * Synchronises the plan's stream. */
int mm_coarse_from_krylov(mm_plan_t plan, const double* b, double* x, double tol, int max_iter,
                          int krylov_dim, double eps_tol, int max_cols, mm_solve_info* info);

/* Host-only helper of mm_coarse_from_krylov (no device work): the Ritz values below
 * eps_tol (ascending, at most max_cols) of the Lanczos matrix of m PCG steps with step
 * lengths alpha[0..m) and products rz[0..m) = r_k^T z_k, T[k][k] = 1/alpha_k +
 * beta_k/alpha_{k-1}, T[k][k+1] = sqrt(beta_{k+1})/alpha_k, beta_k = rz_k/rz_{k-1}
 * [App. A]; theta_out[max_cols]; s_out (or NULL) receives the unit eigenvectors,
 * row-major [m][r] (largest-magnitude entry positive).  Returns r >= 0 or an error. */
int mm_lanczos_ritz(const double* alpha, const double* rz, int m, double eps_tol, int max_cols,
                    double* theta_out, double* s_out);

/* Kind of the plan's coarse space: 0 none, 1 Z_S (mm_plan, MM_COARSE_ZS), 2 Z_D. */
int mm_coarse_kind(mm_plan_t plan);
/* Host FP64 [r_eff]: Ritz value of every kept Z_D column (mm_coarse_columns gives its
 * index among its problem's Ritz values below eps_tol).  MM_ERR_STATE unless Z_D. */
int mm_coarse_ritz_values(mm_plan_t plan, double* host_out, int cap);
/* The kept Z_D columns, FP64, into device dev_out: problem after problem, each block
 * column-major [r_b][n_stokes * pixels_b]; returns the number of values (dev_out NULL:
 * only the count).  MM_ERR_STATE unless Z_D. */
int64_t mm_coarse_dense_columns(mm_plan_t plan, double* dev_out);

/* FFT lengths (real samples per overlap-save tile) the plan uses for the FP64 and the
 * FP32 operator (0 for an operator the plan does not have). */
int mm_fft_lengths(mm_plan_t plan, int* n_r_f64, int* n_r_f32);

/* Samples per P^T work range the plan uses (opts.pt_range, or the autotuned / default
 * value), or a negative status. */
int mm_pt_range(mm_plan_t plan);

/* ----- adjoint (gradients of a loss of the map) ----- */

/* Lag cross-correlations per stationary interval j of two TOD vectors u, v (device FP64
 * [N_t]): c_j(0) = sum_t u_t v_t and c_j(k) = sum_t (u_t v_{t+k} + u_{t+k} v_t) for
 * k = 1..K_j = min(lambda, t_j - 1), t and t+k in interval j, so that u_j^T T_j v_j =
 * sum_k t_k c_j(k) for the band Toeplitz block T_j [Sect. 2.1, eq. N_def].  dev_out:
 * device FP64 [n_intervals][lambda+1], zero past K_j.  Deterministic.  Synchronises. */
int mm_lag_correlations(mm_plan_t plan, const double* u, const double* v, double* dev_out);

/* Derivatives of the windowed Toeplitz taps of every interval with respect to its noise
 * parameters (sigma, f_knee, alpha) [Sect. 4.1.4, eq. fknee; App. D]: host FP64
 * [n_intervals][3][lambda+1], zero past K_j; at most cap values written.  The f_knee and
 * alpha derivatives of a white-noise interval (f_knee = 0) are 0. */
int mm_tap_derivatives(mm_plan_t plan, double* host_out, int64_t cap);

/* Gradients of a loss L(m_hat) of the GLS map m_hat = A^-1 P^T N^-1 d [Sect. 2.1, eq.
 * glsSol] given g = dL/dm_hat, by one more PCG solve mu = A^-1 g (A is symmetric):
 *   dL/dd        = N^-1 P mu                                   (FP64 operator)
 *   dL/dtheta_j  = (P mu)_j^T (dT_j/dtheta_j) (d - P m_hat)_j,  theta_j = (sigma, f_knee, alpha)
 *   m_hat, g       device maps (m_hat as returned by mm_pcg_solve for the same d)
 *   d              device TOD of d_dtype
 *   precond, precision, tol, max_iter   of the mu solve, as in mm_pcg_solve
 *   mu_out         device map receiving mu, or NULL
 *   grad_d         device TOD of grad_d_dtype, or NULL
 *   grad_psd       host FP64 [n_intervals][3], or NULL
 *   info           as in mm_pcg_solve (the mu solve), or NULL
 * Returns the status of the mu solve (gradients are formed only when it is MM_OK), or
 * MM_ERR_ARG / MM_ERR_STATE / MM_ERR_DEVICE.  Synchronises. */
int mm_adjoint(mm_plan_t plan, const double* m_hat, const double* g, const void* d, int d_dtype,
               int precond, int precision, double tol, int max_iter, double* mu_out,
               void* grad_d, int grad_d_dtype, double* grad_psd, mm_solve_info* info);

/* Wall time in ms that mm_plan took for this plan (host clock around all its device work);
 * -1 on NULL. */
double mm_plan_time_ms(mm_plan_t plan);

/* C = A^T B in FP64 on the matrix cores (the product that forms the coarse matrix
 * E = Z^T (AZ) [App. C]).  A: device row-major [n][ra]; B: device row-major [n][rb];
 * C: device row-major [ra][rb].  n must be a positive multiple of 4, ra and rb positive
 * multiples of 16.  Deterministic (fixed split of the n dimension, fixed-order sum).
 * Synchronises the stream (a hipStream_t, NULL = default).  Returns MM_OK or MM_ERR_ARG /
 * MM_ERR_DEVICE. */
int mm_gemm_tn_f64(void* stream, const double* A, const double* B, int64_t n, int32_t ra,
                   int32_t rb, double* C);

/* mm_gemm_tn_f64 for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same product with
 * the same kernels and the same fixed-order sums (bitwise the result of mm_gemm_tn_f64),
 * with its slab partials in a fixed array of 2^20 FP64 values (8 MiB) that the library
 * holds on every device it runs on until the process ends, instead of a buffer allocated
 * per call.  Calls no hipMalloc, hipFree or allocating library routine.
 *   stream  a hipStream_t of the current device (NULL = default stream); the work is
 *           enqueued on it and the call returns without synchronising
 *   A, B, C, n, ra, rb   as mm_gemm_tn_f64
 * Limit: the partials, ksplit * ra * rb values with ksplit = max(1, min(n / 256,
 * 4096 / (ra/16 * rb/16))), must fit the array; every product with ra * rb <= 2^20 does.
 * Calls that overlap on one device share its array and race: order them on one stream.
 * Returns MM_OK, MM_ERR_ARG (shapes as mm_gemm_tn_f64, partials beyond the limit, a
 * stream of another device) or MM_ERR_DEVICE. */
int mm_gemm_tn_f64_noalloc(void* stream, const double* A, const double* B, int64_t n,
                           int32_t ra, int32_t rb, double* C);

/* Kernel timing with HIP events recorded on the plan's stream around every launch of the
 * hot-path kernels (for measurements; off by default).  enable = 1 starts a fresh window,
 * 0 stops recording.  Kernel ids: MM_K_NINV32 / MM_K_NINV64 (overlap-save N^-1 with the
 * de-pointing gather fused, FP32 / FP64), MM_K_PT32 / MM_K_PT64 (P^T segmented reduction),
 * MM_K_PRECOND (block-Jacobi or two-level application), MM_K_VEC (CG vector updates).
 * mm_profile_read synchronises the stream and returns the number of launches and their
 * summed duration in ms. */
enum { MM_K_NINV32 = 0, MM_K_NINV64 = 1, MM_K_PT32 = 2, MM_K_PT64 = 3, MM_K_PRECOND = 4,
       MM_K_VEC = 5, MM_K_COUNT = 6 };
int mm_profile(mm_plan_t plan, int enable);
int mm_profile_read(mm_plan_t plan, int kernel, int64_t* launches, double* total_ms);

/* Message describing the last error on this thread ("" if none). */
const char* mm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MM_H */
