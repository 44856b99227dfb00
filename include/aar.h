/*
 * aar.h — C ABI of the MI355X (gfx950) Alternating Anderson-Richardson solver.
 *
 * Method: Suryanarayana, Pratapa and Pask, "Alternating Anderson-Richardson
 * method: an efficient alternative to preconditioned Krylov methods for
 * large, sparse linear systems", arXiv:1606.08740.  The solver applies the
 * fixed-point iteration x_{k+1} = x_k + B_k f_k of Sec. 2, Eqs. 2-3, with the
 * left-preconditioned residual f_k = M^{-1}(b - A x_k) (Eq. 6) and, for the
 * stencil systems, the Jacobi preconditioner M = D = diag(A) (Sec. 2, the AAJ
 * special case; Secs. 3.2-3.3; general sparse systems, aar_create_csr, also
 * take block ILU(0), Secs. 3.1-3.3):
 *   - Richardson, B_k = omega I, when (k+1)/p is not a natural number;
 *   - Anderson, B_k = beta I - (X_k + beta F_k)(F_k^T F_k)^+ F_k^T, when it is,
 *     with X_k, F_k the last m iterate and residual differences (Eqs. 4-5)
 *     and (.)^+ the Moore-Penrose pseudoinverse (Sec. 3.2).
 * Convergence, r_k = ||b - A x_k||_2 / ||b||_2 < tol (Sec. 2, text after
 * Eq. 6), is tested at Anderson steps only.  The vector tested is D f_k for
 * the f_k of that step.  For the first step of each cycle of p iterations f
 * is formed from x and b; for the later steps of a cycle (the Anderson step
 * included) the solver may form it from the previous one by the identity
 * f_{j+1} = f_j - omega D^-1 A f_j, which a Richardson step x_{j+1} = x_j +
 * omega f_j implies (see AAR_FP64 below).  The iteration count reported is
 * the number of residual evaluations k+1, a multiple of p on convergence.
 *
 * The operator is a finite-difference stencil on a 3D grid (the paper's
 * Poisson and Helmholtz problems, Eqs. 7-8, use sixth-order central
 * differences on a uniform grid):
 *   A u = -a Lap_h u + v . grad_h u + sigma u
 * with the order-2r central second difference along each axis (weights of
 * the standard central formula) and optional first-order upwind convection.
 * Zero Dirichlet axes read zero outside the grid; periodic axes wrap indices
 * modulo n, so on an axis shorter than the stencil (n < 2r+1) several taps
 * land on one point and add up (a circulant), and D includes the taps that
 * land on the point itself.
 *
 * Conventions for every entry point:
 *   - All functions are extern "C", never throw, and return aar_status.
 *   - A negative status means nothing was computed and no output was
 *     written; aar_last_error() then describes the problem (thread-local).
 *   - A positive status (not converged, breakdown) means x holds the last
 *     iterate, whose residual is reported.
 *   - Vector arguments b, x, y are caller-owned FP64 device pointers,
 *     contiguous, one value per grid point in the order i + n0*(j + n1*k).
 *     The library never keeps them past the call.
 *   - Work runs on the HIP stream given at creation; the solve calls return
 *     after their results have reached the host.
 *   - A solver handle is not thread-safe; use one handle per stream.
 */
#ifndef AAR_H
#define AAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aar_solver_t *aar_solver;

typedef enum {
    AAR_OK = 0,                 /* converged: x_k with r_k < tol                        */
    AAR_NOT_CONVERGED = 1,      /* max_iter (or max_outer) reached                      */
    AAR_BREAKDOWN = 2,          /* NaN or Inf in the residual or the Gram matrix        */
    AAR_ERR_INVALID_ARG = -1,   /* bad pointer, size or parameter                       */
    AAR_ERR_UNSUPPORTED = -2,   /* valid request outside what the library implements    */
    AAR_ERR_DEVICE = -3,        /* HIP runtime error                                    */
    AAR_ERR_OUT_OF_MEMORY = -4  /* device allocation failed                             */
} aar_status;

enum { AAR_BC_ZERO_DIRICHLET = 0, AAR_BC_PERIODIC = 1 };

/* Arithmetic of the iteration.
 *   AAR_FP64: every value and every operation in FP64.  When the history
 *     ring holds a whole cycle (m + 1 >= p, p >= 2) the Richardson steps of
 *     a cycle after its first do not read x and b: they form
 *     f_{j+1} = f_j - omega D^-1 A f_j from the previous f (Eq. 6 after the
 *     first case of Eq. 3), and the iterate x_j = x_c + omega sum f_i is
 *     formed from the cycle's first iterate x_c where it is needed (the
 *     Anderson update, the end of a run).  Each cycle's first f is formed
 *     from x and b, so the recursion's rounding (about u ||f|| per step)
 *     does not accumulate across cycles.  The convergence test and the
 *     reported rel_residual are then ||D f_k|| / ||b|| for the recursed
 *     f_k; they equal ||b - A x_k|| / ||b|| for the returned x_k to within
 *     about p u kappa(D^-1 A) relative (1e-6 or better on the evaluation
 *     grids).  With m + 1 < p every f is formed from x and b.
 *   AAR_FP64_FP32HIST / AAR_FP64_BF16HIST: x and b in FP64, the history
 *     ring (the f_j of Eqs. 4-5) stored in FP32 / bfloat16; Gram products
 *     accumulated in FP64.  No refinement is needed: the iterate and the
 *     residual of each cycle's first step are FP64; the extrapolation
 *     directions are rounded.  With an FP32 ring the Anderson update also
 *     takes f_k from the ring and the increments of Anderson steps (the X_k
 *     columns of Eq. 4) are stored in FP32: perturbations of the step
 *     relative to the current residual, which leave the fixed point exact.
 *     The FP32-ring mode runs the recursion described for AAR_FP64 in FP32
 *     on the ring; it restarts from the FP64 residual every cycle, so the
 *     convergence test holds to ~1e-6 relative.  With a bfloat16 ring every
 *     residual is FP64, f_k comes from an FP64 copy and the increments stay
 *     FP64.
 *   AAR_MIXED_FP32: FP32 sweeps, history and Gram products (accumulated in
 *     FP64), FP64 m x m solve, and an outer FP64 iterative refinement:
 *     r = b - A x (FP64), inner FP32 AAR on A d = r/||r|| to inner_tol,
 *     x += ||r|| d, until ||b - A x|| / ||b|| < tol.  With inner_tol = 0 each
 *     step's inner tolerance is max(3e-4, tol / (2 rel)), rel the FP64
 *     relative residual the step starts from (three steps reach 1e-10; a
 *     deeper FP32 target runs into the FP32 accuracy floor).  The outer test and the
 *     reported rel_residual use r formed from x and b in FP64.
 *   AAR_MIXED_FP32_BF16HIST: as AAR_MIXED_FP32 with the history columns
 *     stored in bfloat16 (round to nearest even). */
enum { AAR_FP64 = 0, AAR_MIXED_FP32 = 1, AAR_MIXED_FP32_BF16HIST = 2, AAR_FP64_FP32HIST = 3, AAR_FP64_BF16HIST = 4 };

enum {
    AAR_FLAG_RECORD_RESIDUALS = 1, /* keep r_k and the kept rank of every Anderson step          */
    AAR_FLAG_DEFLATE_CONSTANT = 2, /* exact FP64 removal of the constant mode, see below        */
    AAR_FLAG_NO_GRAPH = 4,         /* launch kernels one by one instead of replaying HIP graphs */
    AAR_FLAG_NO_AUTOTUNE = 8,      /* use the default tile shape instead of timing candidates   */
    AAR_FLAG_FORCE_PINV = 16,      /* every m x m solve by the eigendecomposition, see below    */
    AAR_FLAG_RECYCLE_HISTORY = 32  /* mixed modes: inner runs keep the previous run's history     */
};
/* AAR_FLAG_DEFLATE_CONSTANT: when every axis is periodic and sigma > 0, the
 * constant vector is an exact eigenvector, A 1 = sigma 1 (upwind convection
 * included).  With the flag, each FP64 residual r = b - A x is followed by
 * x += mean(r) / sigma, r -= mean(r) (once before the iteration in FP64
 * mode, at every refinement step in mixed mode), so the iteration only sees
 * the mean-free part.  This removes the near-null mode of small shifts,
 * which FP32 cannot resolve.  It is not part of the paper's method; the
 * answer is the same solution of A x = b.  aar_create returns
 * AAR_ERR_UNSUPPORTED for the flag on any system with a Dirichlet axis or
 * sigma == 0.
 *
 * AAR_FLAG_FORCE_PINV (a check of the solver, for tests): the m x m solve
 * gamma = (F^T F)^+ F^T f_k normally takes a Cholesky solve when a bound
 * proves every eigenvalue of F^T F above the pseudoinverse threshold (the
 * pseudoinverse is then the inverse), and the Jacobi eigendecomposition
 * otherwise.  With the flag every solve takes the eigendecomposition. */

/* AAR_FLAG_RECYCLE_HISTORY (mixed precision modes, single solves): each inner
 * FP32 run after the first starts with the history of the previous run
 * instead of an empty one.  The history is never cleared within a run
 * (Sec. 2); its difference pairs satisfy dF = -D^-1 A dX for any right-hand
 * side, so they stay valid extrapolation directions for the next correction
 * equation A d = r / ||r||.  The one difference that spans the restart pairs
 * residuals of two right-hand sides and enters as a null column (its rows of
 * F^T F and F^T f are zero; the pseudoinverse gives it no weight, as the
 * footnote to Eq. 5 allows).  aar_create returns AAR_ERR_UNSUPPORTED for the
 * flag with an FP64 mode or a batch. */

/* One linear system A x = b (Sec. 2, Eq. 1). */
typedef struct {
    int32_t n[3];            /* grid points per axis (>= 1)                                  */
    double h[3];             /* grid spacing per axis (> 0)                                   */
    int32_t bc[3];           /* AAR_BC_* per axis                                            */
    int32_t radius;          /* r in 1..6: order-2r central second difference, 6r+1 points   */
    double diffusion;        /* a (> 0)                                                      */
    double shift;            /* sigma (>= 0)                                                 */
    const double *velocity;  /* NULL, or device FP64 planar [vx | vy | vz] (3 N values);     */
                             /* radius must be 1 and periodic axes n >= 2; copied at creation */
} aar_problem;

/* Parameters of the iteration (Sec. 2, Eqs. 2-5; the paper's defaults are
 * in Sec. 2, after the description of the method). */
typedef struct {
    double omega;            /* Richardson relaxation (Eq. 3)                    paper: 0.6  */
    double beta;             /* Anderson relaxation (Eq. 3)                      paper: 0.6  */
    int32_t m;               /* history length, 1..32 (Eqs. 4-5)                 paper: 9    */
    int32_t p;               /* Anderson every p iterations, >= 1                paper: 8    */
    double tol;              /* on r_k = ||b - A x|| / ||b||, > 0                            */
    int64_t max_iter;        /* cap on iterations (inner iterations in mixed mode), >= 1    */
    int32_t precision;       /* AAR_FP64, AAR_MIXED_FP32(_BF16HIST), AAR_FP64_*HIST           */
    double inner_tol;        /* mixed: inner FP32 tolerance (0: per step, see AAR_MIXED_FP32) */
    int32_t max_outer;       /* mixed: cap on refinement steps (0 selects 30)                */
    uint32_t flags;          /* AAR_FLAG_*                                                   */
} aar_params;

/* Outcome of one system. */
typedef struct {
    int32_t status;          /* aar_status of this instance                                  */
    int64_t iterations;      /* residual evaluations k+1 (all inner ones in mixed mode)      */
    int32_t outer_steps;     /* refinement steps (mixed), 0 in FP64 mode                     */
    double rel_residual;     /* last tested r_k (see above; FP64 from x and b in mixed mode) */
} aar_result;

/* Create a solver for `count` systems A_i x_i = b_i (Eq. 1) sharing the
 * iteration parameters of Eqs. 2-5.  Validates the descriptions (before any
 * device work), allocates the device workspace (history ring of Eqs. 4-5,
 * partial sums, descriptors; aar_workspace_bytes gives its size), copies
 * velocities, and picks tile shapes (timing candidates unless
 * AAR_FLAG_NO_AUTOTUNE or a tile file lists the grid).  hip_stream is a
 * hipStream_t (NULL: the default stream).  *out receives the handle, which
 * the caller releases with aar_destroy; on failure *out is NULL. */
aar_status aar_create(aar_solver *out, const aar_problem *problems, int32_t count,
                      const aar_params *params, void *hip_stream);

/* Create a solver for one complex-valued system A x = b (Sec. 2, Eq. 1 over C;
 * the periodic Helmholtz problem of Sec. 3.2, Eq. 7, has a complex shift and
 * right-hand side): A = A_r + i shift_imag I, with A_r the real operator of
 * `problem` (its real shift included), and the complex relaxation parameters
 * omega = params->omega + i omega_imag, beta = params->beta + i beta_imag of
 * Eq. 3.  The Anderson step solves with F^H F (the paper's T is the conjugate
 * transpose), its Moore-Penrose pseudoinverse computed on the real form
 * [[Re, -Im], [Im, Re]] of the Hermitian matrix, eigenvalues <=
 * l lambda_max 2^-52 dropped; D = diag(A) is complex.  Every Richardson step
 * forms f from x and b.  The handle then takes complex vectors in aar_solve
 * and aar_apply: b, x, y hold 2N doubles, (re, im) interleaved per grid point.
 * Supported: precision AAR_FP64, m <= 8, no velocity, no deflation
 * (AAR_ERR_UNSUPPORTED otherwise); aar_solve_batched is not. */
aar_status aar_create_complex(aar_solver *out, const aar_problem *problem, const aar_params *params,
                              double shift_imag, double omega_imag, double beta_imag, void *hip_stream);

/* Preconditioners of a general sparse system (aar_create_csr). */
enum { AAR_PRECOND_JACOBI = 0, AAR_PRECOND_ILU0 = 1 };

/* Create a solver for one general sparse system A x = b (Sec. 2, Eq. 1, with
 * any preconditioner M in Eq. 6: Sec. 3.1 solves nonsymmetric sparse systems
 * with the Jacobi and the ILU(0) preconditioner; Secs. 3.2-3.3 use block
 * Jacobi with ILU(0) on each block in parallel).
 *   n                  rows (1 .. 2^31 - 1)
 *   rowptr, col, val   host arrays of A in compressed sparse rows: row i
 *                      holds val[rowptr[i] .. rowptr[i+1]-1] in columns
 *                      col[...], strictly increasing, diagonal present,
 *                      values finite (n + 1, nnz and nnz entries; copied at
 *                      creation, not kept)
 *   preconditioner     AAR_PRECOND_JACOBI: M = diag(A);
 *                      AAR_PRECOND_ILU0: M = block diagonal of the ILU(0)
 *                      factors of the `nblocks` diagonal blocks of A, block
 *                      t holding rows floor(t n / nblocks) ..
 *                      floor((t+1) n / nblocks) - 1 (nblocks = 1: ILU(0) of
 *                      A).  ILU(0): L unit lower and U upper triangular in
 *                      the pattern of the block, (L U)_ij = a_ij on that
 *                      pattern, by elimination in row order with fill outside
 *                      the pattern dropped; entries of A that couple two
 *                      blocks do not enter M.  The factors are formed on the
 *                      device at creation.
 *   nblocks            1 .. n for ILU(0), each block at most 16384 rows
 *                      (AAR_ERR_UNSUPPORTED beyond); ignored for Jacobi
 * The handle then takes vectors of n doubles (one value per row) in
 * aar_solve, aar_apply and aar_precondition.  Every Richardson step forms f
 * from x and b.  Supported: precision AAR_FP64 and the flags
 * AAR_FLAG_RECORD_RESIDUALS, AAR_FLAG_NO_GRAPH, AAR_FLAG_FORCE_PINV
 * (AAR_ERR_UNSUPPORTED for the others); aar_solve_batched is not.  A zero or
 * non-finite ILU(0) pivot returns AAR_ERR_UNSUPPORTED. */
aar_status aar_create_csr(aar_solver *out, int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                          int32_t preconditioner, int32_t nblocks, const aar_params *params, void *hip_stream);

/* z = M^{-1} r for the preconditioner of a solver from aar_create_csr (the
 * M^{-1} of Eq. 6; a check of the factors and substitutions).  r and z are
 * device vectors of n doubles and must not overlap. */
aar_status aar_precondition(aar_solver s, const double *r, double *z);

/* Solve system 0 (count must be 1) by AAR (Sec. 2, Eqs. 2-6).  x holds x_0
 * on entry and the answer on return (the iterate x_k whose test passed, or
 * the last iterate); b is read only.  r receives the outcome (may be NULL). */
aar_status aar_solve(aar_solver s, const double *b, double *x, aar_result *r);

/* Solve all `count` systems by AAR (Sec. 2, Eqs. 2-6), advanced together,
 * each stopping at its own test (Sec. 1: many independent solves).  System i
 * reads b + offsets[i] and updates x + offsets[i] (offsets: count + 1 host
 * int64 values, offsets[i+1] - offsets[i] equal to that system's size).
 * results[i] (host, count entries) receives each outcome; the return value is
 * the worst status. */
aar_status aar_solve_batched(aar_solver s, const double *b, double *x, const int64_t *offsets,
                             aar_result *results);

/* y = A x in FP64 for system `instance` (the operator of Eq. 1; a check of
 * the stencil, or of the sparse product for a solver from aar_create_csr).
 * x and y are device vectors of that system's size and must not overlap. */
aar_status aar_apply(aar_solver s, int32_t instance, const double *x, double *y);

/* Copy up to `cap` recorded Anderson-step residuals r_k (Sec. 2, text after
 * Eq. 6) of system `instance` from the last solve (needs
 * AAR_FLAG_RECORD_RESIDUALS) into host `out`; *count receives the number
 * recorded.  In mixed mode these are the inner residuals of the last
 * refinement step. */
aar_status aar_residual_log(aar_solver s, int32_t instance, double *out, int64_t cap,
                            int64_t *count);

/* Copy up to `cap` ranks kept by the pseudoinverse solve of each Anderson
 * step (Sec. 3.2; the number of eigenvalues of F^T F above the threshold),
 * index for index beside aar_residual_log, into host `out`: -1 for the step
 * whose convergence test ended the run (no solve), l = min(k, m) whenever the
 * Cholesky shortcut proved full rank.  Needs AAR_FLAG_RECORD_RESIDUALS. */
aar_status aar_rank_log(aar_solver s, int32_t instance, int32_t *out, int64_t cap, int64_t *count);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * FP64 solve as aar_solve (precision AAR_FP64, default tile shapes, as with
 * AAR_FLAG_NO_AUTOTUNE) of one system, with no handle.  The workspace (run
 * state, partial sums, two copies of x, b, the m + 1 history slots and the
 * floor(m/p) increment slots) lives in a fixed device array of 32 MiB that
 * the library holds on every GPU it runs on until the process ends; no device
 * memory is allocated or freed.  Systems whose workspace exceeds that limit
 * (about 8 (m + 4 + floor(m/p)) N bytes: a 70^3 grid fits at m = 7, p = 6)
 * return AAR_ERR_UNSUPPORTED before any device work, as do other precisions
 * and AAR_FLAG_RECORD_RESIDUALS.  The velocity array, if any, is read in place
 * and must stay valid for the call.  Work runs on hip_stream (NULL: the
 * default stream) and the call returns after r has reached the host.  Every
 * call on one GPU uses that GPU's array: calls that overlap on one GPU (from
 * several threads or streams) race and must be serialized by the caller. */
aar_status aar_solve_noalloc(const aar_problem *problem, const aar_params *params, const double *b, double *x,
                             aar_result *r, void *hip_stream);

/* Choose the Anderson relaxation beta and the period p for one real system
 * by timing short trial solves (a setup call: it creates and destroys a
 * solver per candidate and allocates one vector).  The paper fixes
 * {omega, beta, m, p} = {0.6, 0.6, 9, 8} and notes that the method is
 * insensitive to them over a broad range but that a larger beta can speed up
 * well-conditioned problems (Sec. 2, closing paragraphs; Sec. 3.1 tunes beta
 * per matrix).  For every pair (betas[i], ps[j]) the solve of `problem` with
 * right-hand side b (device FP64) from x_0 = 0 runs trial_iterations
 * iterations (rounded up to a multiple of that p) twice, and the second run is
 * scored by the decimal digits its residual fell per second,
 * -log10(r_last) / seconds (0 after a breakdown).  The best pair is written to
 * *beta_out, *p_out; scores (may be NULL) receives all of them, index
 * j * nbeta + i.  Other fields of params are used as given (its beta and p are
 * ignored). */
aar_status aar_select_parameters(const aar_problem *problem, const aar_params *params, const double *b,
                                 const double *betas, int32_t nbeta, const int32_t *ps, int32_t np,
                                 int64_t trial_iterations, void *hip_stream, double *beta_out, int32_t *p_out,
                                 double *scores);

/* Device bytes aar_create would allocate for these arguments. */
aar_status aar_workspace_bytes(const aar_problem *problems, int32_t count, const aar_params *params,
                               size_t *bytes);

/* Release the handle and its device memory (NULL is accepted). */
aar_status aar_destroy(aar_solver s);

/* Description of the last error on this thread ("" if none). */
const char *aar_last_error(void);

/* Kernel timing for measurement: when enabled, the solver brackets each
 * cycle's p - 1 consecutive Richardson sweep launches with one pair of HIP
 * events on its stream (graphs are not used while enabled) and accumulates
 * their durations.  aar_sweep_time returns the total milliseconds and the
 * number of sweep launches timed since the last reset. */
aar_status aar_set_timing(aar_solver s, int32_t enable);
aar_status aar_sweep_time(aar_solver s, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* AAR_H */
