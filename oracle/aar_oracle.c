/*
 * Plain FP64 CPU oracle for the Alternating Anderson-Richardson (AAR) method
 * of Suryanarayana, Pratapa and Pask, "Alternating Anderson-Richardson
 * method: an efficient alternative to preconditioned Krylov methods for
 * large, sparse linear systems" (arXiv:1606.08740).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU solver is checked against.  Only the tests, the
 * package smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or constant with the GPU path.
 *
 * What it computes, and where each piece comes from:
 *   - the linear system A x = b (Sec. 2, Eq. 1), real-valued, for a
 *     finite-difference operator on a 3D grid:
 *         A u = -a * Lap_h u + v . grad_h u + sigma * u
 *     with the order-2r central second difference per axis (the paper uses
 *     sixth order, r = 3, for its Helmholtz and Poisson problems, Eqs. 7-8)
 *     and first-order upwind convection (radius 1 only);
 *   - the Jacobi preconditioner M = D = diag(A) (Sec. 2, the AAJ special
 *     case; Sec. 3.2-3.3);
 *   - the AAR iteration x_{k+1} = x_k + B_k f_k (Eqs. 2-3) with the
 *     left-preconditioned residual f_k = M^{-1}(b - A x_k) (Eq. 6), histories
 *     X_k, F_k of the last m differences (Eqs. 4-5), Anderson extrapolation
 *     when (k+1)/p is a natural number and Richardson otherwise, and the
 *     convergence test ||A x_k - b|| / ||b|| < tol made only at Anderson
 *     steps (Sec. 2, text after Eq. 6);
 *   - (F^T F)^{-1} as the Moore-Penrose pseudoinverse (Sec. 3.2), here by a
 *     cyclic Jacobi eigendecomposition of the symmetric matrix F^T F.
 *
 * Readings where the paper is silent (its flowchart, Fig. 1, is not
 * available in the text):
 *   - step order at iteration k: residual; history push of x_k - x_{k-1} and
 *     f_k - f_{k-1}; if Anderson: convergence test on the unpreconditioned
 *     residual just computed, then the update; else the Richardson update;
 *   - history columns with negative index are omitted (footnote to Eq. 5):
 *     at iteration k the history has min(k, m) columns; it is never cleared;
 *   - pseudoinverse threshold: eigenvalues <= l * lambda_max * 2^-52 of the
 *     l x l matrix F^T F are dropped (the usual default of a pseudoinverse);
 *   - the convergence test is strict (<) and the returned x is the iterate
 *     x_k whose residual passed; the reported iteration count is k + 1;
 *   - b = 0 returns x = 0 after zero iterations;
 *   - the iteration cap returns the iterate after max_iter updates.
 *
 * Stencil conventions: unknown (i, j, k) is stored at i + n0*(j + n1*k).
 * Zero Dirichlet boundaries treat points outside the grid as zero.  Periodic
 * boundaries wrap indices modulo n (taps that land on the same point add up).
 * Central weights of order 2r (closed form of the standard central
 * difference, checked by the tests against the moment conditions):
 *     w_s = 2 (-1)^{s+1} (r!)^2 / (s^2 (r-s)! (r+s)!),  s = 1..r,
 *     w_0 = -2 sum_s w_s,
 *     d2u/dx2 at i ~= h^-2 (w_0 u_i + sum_s w_s (u_{i+s} + u_{i-s})).
 * Upwind convection per axis c with velocity v = v_c at the point:
 *     v > 0:  v (u_i - u_{i-1}) / h_c;   otherwise  v (u_{i+1} - u_i) / h_c.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n[3];
    double h[3];
    int32_t bc[3];          /* 0 zero Dirichlet, 1 periodic */
    int32_t radius;         /* 1..6 */
    double diffusion;       /* a */
    double shift;           /* sigma */
    const double *velocity; /* NULL or planar [vx | vy | vz], each of size N */
} oracle_problem;

enum { ORACLE_OK = 0, ORACLE_NOT_CONVERGED = 1, ORACLE_BREAKDOWN = 2, ORACLE_BAD_ARG = -1 };

static int64_t problem_size(const oracle_problem *P)
{
    return (int64_t)P->n[0] * P->n[1] * P->n[2];
}

/* ---------------------------------------------------------------------- */
/* Finite-difference weights                                               */
/* ---------------------------------------------------------------------- */
static double factorial(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i)
        f *= i;
    return f;
}

/* w[0..r]: the order-2r central second-difference weights (unit spacing). */
void oracle_fd_weights(int r, double *w)
{
    double sum = 0.0;
    for (int s = 1; s <= r; ++s) {
        double sign = (s % 2 == 1) ? 1.0 : -1.0;
        w[s] = 2.0 * sign * factorial(r) * factorial(r) /
               ((double)s * s * factorial(r - s) * factorial(r + s));
        sum += w[s];
    }
    w[0] = -2.0 * sum;
}

/* Value of u at index (i, j, k) shifted by d along `axis`, with the boundary
 * rule of that axis; *ok is cleared when the point is outside a Dirichlet
 * boundary (value zero). */
static int64_t neighbour(const oracle_problem *P, int i, int j, int k, int axis, int d, int *ok)
{
    int c[3] = {i, j, k};
    int n = P->n[axis];
    int t = c[axis] + d;
    if (P->bc[axis] == 1) {
        t %= n;
        if (t < 0)
            t += n;
    } else if (t < 0 || t >= n) {
        *ok = 0;
        return 0;
    }
    c[axis] = t;
    *ok = 1;
    return c[0] + (int64_t)P->n[0] * (c[1] + (int64_t)P->n[1] * c[2]);
}

/* y = A x  (standard form: weights times values, summed per axis). */
void oracle_apply(const oracle_problem *P, const double *x, double *y)
{
    double w[7];
    oracle_fd_weights(P->radius, w);
    const int n0 = P->n[0], n1 = P->n[1], n2 = P->n[2];
    const int64_t N = problem_size(P);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n2; ++k) {
        for (int j = 0; j < n1; ++j) {
            for (int i = 0; i < n0; ++i) {
                int64_t id = i + (int64_t)n0 * (j + (int64_t)n1 * k);
                double acc = P->shift * x[id];
                for (int axis = 0; axis < 3; ++axis) {
                    double lap = w[0] * x[id];
                    for (int s = 1; s <= P->radius; ++s) {
                        int ok;
                        int64_t q = neighbour(P, i, j, k, axis, s, &ok);
                        if (ok)
                            lap += w[s] * x[q];
                        q = neighbour(P, i, j, k, axis, -s, &ok);
                        if (ok)
                            lap += w[s] * x[q];
                    }
                    acc += -P->diffusion * lap / (P->h[axis] * P->h[axis]);
                    if (P->velocity) {
                        double v = P->velocity[axis * N + id];
                        int ok;
                        if (v > 0.0) {
                            int64_t q = neighbour(P, i, j, k, axis, -1, &ok);
                            acc += v * (x[id] - (ok ? x[q] : 0.0)) / P->h[axis];
                        } else {
                            int64_t q = neighbour(P, i, j, k, axis, 1, &ok);
                            acc += v * ((ok ? x[q] : 0.0) - x[id]) / P->h[axis];
                        }
                    }
                }
                y[id] = acc;
            }
        }
    }
}

/* d = diag(A): the coefficient of x_i in (A x)_i.  With periodic wrap on a
 * short axis (n < 2r+1) some taps land on i itself and add to the diagonal;
 * the diagonal is therefore read off the operator by applying A to the unit
 * vector pattern of each point's own value, computed directly here. */
void oracle_diagonal(const oracle_problem *P, double *d)
{
    double w[7];
    oracle_fd_weights(P->radius, w);
    const int n0 = P->n[0], n1 = P->n[1], n2 = P->n[2];
    const int64_t N = problem_size(P);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n2; ++k) {
        for (int j = 0; j < n1; ++j) {
            for (int i = 0; i < n0; ++i) {
                int64_t id = i + (int64_t)n0 * (j + (int64_t)n1 * k);
                double acc = P->shift;
                for (int axis = 0; axis < 3; ++axis) {
                    double lap = w[0];
                    for (int s = 1; s <= P->radius; ++s) {
                        int ok;
                        int64_t q = neighbour(P, i, j, k, axis, s, &ok);
                        if (ok && q == id)
                            lap += w[s];
                        q = neighbour(P, i, j, k, axis, -s, &ok);
                        if (ok && q == id)
                            lap += w[s];
                    }
                    acc += -P->diffusion * lap / (P->h[axis] * P->h[axis]);
                    if (P->velocity) {
                        double v = P->velocity[axis * N + id];
                        int ok;
                        if (v > 0.0) {
                            int64_t q = neighbour(P, i, j, k, axis, -1, &ok);
                            acc += v * (1.0 - ((ok && q == id) ? 1.0 : 0.0)) / P->h[axis];
                        } else {
                            int64_t q = neighbour(P, i, j, k, axis, 1, &ok);
                            acc += v * (((ok && q == id) ? 1.0 : 0.0) - 1.0) / P->h[axis];
                        }
                    }
                }
                d[id] = acc;
            }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Pseudoinverse solve of the small normal equations                       */
/* ---------------------------------------------------------------------- */

/* Cyclic Jacobi eigendecomposition of the symmetric l x l matrix S (row
 * major, overwritten by its eigenvalues on the diagonal); V receives the
 * eigenvectors as columns.  Rotations are skipped once the off-diagonal
 * element is negligible against both diagonal entries; the sweeps stop when
 * a full sweep applies no rotation. */
void oracle_jacobi_eigen(int l, double *S, double *V)
{
    for (int i = 0; i < l; ++i)
        for (int j = 0; j < l; ++j)
            V[i * l + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < l - 1; ++p) {
            for (int q = p + 1; q < l; ++q) {
                double apq = S[p * l + q];
                double app = S[p * l + p], aqq = S[q * l + q];
                if (apq == 0.0)
                    continue;
                if (fabs(app) + 1e3 * fabs(apq) == fabs(app) &&
                    fabs(aqq) + 1e3 * fabs(apq) == fabs(aqq)) {
                    S[p * l + q] = S[q * l + p] = 0.0;
                    continue;
                }
                /* angle that zeroes S[p][q]: tan(2 phi) = 2 apq / (aqq - app) */
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0);
                double s = t * c;
                /* S <- J^T S J with J the rotation in the (p, q) plane */
                for (int r = 0; r < l; ++r) {
                    double srp = S[r * l + p], srq = S[r * l + q];
                    S[r * l + p] = c * srp - s * srq;
                    S[r * l + q] = s * srp + c * srq;
                }
                for (int r = 0; r < l; ++r) {
                    double spr = S[p * l + r], sqr = S[q * l + r];
                    S[p * l + r] = c * spr - s * sqr;
                    S[q * l + r] = s * spr + c * sqr;
                }
                S[p * l + q] = S[q * l + p] = 0.0;
                for (int r = 0; r < l; ++r) {
                    double vrp = V[r * l + p], vrq = V[r * l + q];
                    V[r * l + p] = c * vrp - s * vrq;
                    V[r * l + q] = s * vrp + c * vrq;
                }
                rotated = 1;
            }
        }
        if (!rotated)
            break;
    }
}

/* gamma = pinv(G) c for the symmetric positive semidefinite l x l matrix G.
 * Returns the number of eigenvalues kept (the numerical rank); *cond (if not
 * NULL) receives lambda_max / lambda_min over the kept eigenvalues. */
static int pinv_solve_cond(int l, const double *G, const double *c, double *gamma, double *cond);

int oracle_pinv_solve(int l, const double *G, const double *c, double *gamma)
{
    return pinv_solve_cond(l, G, c, gamma, NULL);
}

static int pinv_solve_cond(int l, const double *G, const double *c, double *gamma, double *cond)
{
    if (cond)
        *cond = 1.0;
    if (l <= 0)
        return 0;
    double *S = malloc(sizeof(double) * l * l);
    double *V = malloc(sizeof(double) * l * l);
    memcpy(S, G, sizeof(double) * l * l);
    oracle_jacobi_eigen(l, S, V);
    double lmax = 0.0;
    for (int i = 0; i < l; ++i)
        if (S[i * l + i] > lmax)
            lmax = S[i * l + i];
    double thresh = l * lmax * ldexp(1.0, -52);
    int rank = 0;
    double lmin_kept = lmax;
    for (int i = 0; i < l; ++i)
        gamma[i] = 0.0;
    for (int e = 0; e < l; ++e) {
        double lam = S[e * l + e];
        if (!(lam > thresh))
            continue;
        ++rank;
        if (lam < lmin_kept)
            lmin_kept = lam;
        double proj = 0.0; /* v_e . c */
        for (int i = 0; i < l; ++i)
            proj += V[i * l + e] * c[i];
        for (int i = 0; i < l; ++i)
            gamma[i] += V[i * l + e] * proj / lam;
    }
    if (cond && rank > 0)
        *cond = lmax / lmin_kept;
    free(S);
    free(V);
    return rank;
}

/* ---------------------------------------------------------------------- */
/* The AAR iteration                                                       */
/* ---------------------------------------------------------------------- */
/* Sums are formed over fixed blocks of REDUCE_BLOCK elements, each block
 * summed in index order, and the block sums added in block order, so the
 * result does not depend on the number of threads or their timing. */
#define REDUCE_BLOCK 4096

static double blocked_sum(int64_t N, const double *a, const double *b, int square_diff)
{
    int64_t nblk = (N + REDUCE_BLOCK - 1) / REDUCE_BLOCK;
    double *part = malloc(sizeof(double) * (nblk > 0 ? nblk : 1));
#pragma omp parallel for schedule(static)
    for (int64_t blk = 0; blk < nblk; ++blk) {
        int64_t lo = blk * REDUCE_BLOCK, hi = lo + REDUCE_BLOCK < N ? lo + REDUCE_BLOCK : N;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i)
            s += square_diff ? (a[i] - b[i]) * (a[i] - b[i]) : a[i] * b[i];
        part[blk] = s;
    }
    double s = 0.0;
    for (int64_t blk = 0; blk < nblk; ++blk)
        s += part[blk];
    free(part);
    return s;
}

static double dot(int64_t N, const double *a, const double *b)
{
    return blocked_sum(N, a, b, 0);
}

/*
 * Solve A x = b by preconditioned AAR with M = diag(A).
 *   x        in: x_0, out: the returned iterate (length N)
 *   omega    Richardson relaxation (Eq. 3, first case)
 *   beta     Anderson relaxation (Eq. 3, second case)
 *   m        history length: m+1 iterates enter each extrapolation (Eqs. 4-5)
 *   p        extrapolate when (k+1) is a multiple of p
 *   tol      on ||b - A x_k|| / ||b||, tested at Anderson steps only
 *   max_iter cap on the number of iterations (updates)
 *   trace    optional [trace_cap x 6] rows, one per Anderson step:
 *            k, r_k, ||f_k||, ||f_k - F_k gamma_k|| (0 if converged), rank,
 *            condition number of F_k^T F_k over the kept eigenvalues
 * Returns ORACLE_OK, ORACLE_NOT_CONVERGED, ORACLE_BREAKDOWN (NaN/Inf residual)
 * or ORACLE_BAD_ARG.
 */
/* The residual step of one iteration for whichever operator and
 * preconditioner the caller holds: res = b - A x_k and f_k = M^{-1} res
 * (Eq. 6). */
typedef void (*residual_step)(void *ctx, const double *x, double *res, double *f);

/* The AAR iteration itself (Eqs. 2-5, Sec. 2) over vectors of length N, with
 * the residual step supplied by the caller; arguments and return values as
 * described above. */
static int aar_iterate(int64_t N, residual_step step, void *ctx, const double *b, double *x,
                       double omega, double beta, int m, int p, double tol, int64_t max_iter,
                       int64_t *iters_out, double *relres_out,
                       double *trace, int64_t trace_cap, int64_t *trace_len)
{
    if (N <= 0 || m < 1 || p < 1 || !(tol > 0.0) || max_iter < 1)
        return ORACLE_BAD_ARG;
    if (trace_len)
        *trace_len = 0;
    *iters_out = 0;
    *relres_out = 0.0;

    double nb = sqrt(dot(N, b, b));
    if (nb == 0.0) {
        memset(x, 0, sizeof(double) * N);
        return ORACLE_OK;
    }

    double *res = malloc(sizeof(double) * N);
    double *f = malloc(sizeof(double) * N);
    double *x_prev = malloc(sizeof(double) * N);
    double *f_prev = malloc(sizeof(double) * N);
    double *DX = malloc(sizeof(double) * N * m); /* column slot s at DX + s*N */
    double *DF = malloc(sizeof(double) * N * m);
    int *order = malloc(sizeof(int) * m);        /* order[0] oldest .. order[cols-1] newest */
    double *G = malloc(sizeof(double) * m * m);
    double *c = malloc(sizeof(double) * m);
    double *gamma = malloc(sizeof(double) * m);
    int cols = 0;
    int status = ORACLE_NOT_CONVERGED;
    double r = 0.0;

    for (int64_t k = 0;; ++k) {
        /* residual and preconditioned residual f_k = M^{-1}(b - A x_k)  (Eq. 6) */
        step(ctx, x, res, f);

        /* history push: x_k - x_{k-1} and f_k - f_{k-1}  (Eqs. 4-5) */
        if (k >= 1) {
            int slot;
            if (cols < m) {
                slot = cols;
                order[cols++] = slot;
            } else {
                slot = order[0];
                for (int t = 0; t < m - 1; ++t)
                    order[t] = order[t + 1];
                order[m - 1] = slot;
            }
            double *dx = DX + (int64_t)slot * N, *df = DF + (int64_t)slot * N;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) {
                dx[i] = x[i] - x_prev[i];
                df[i] = f[i] - f_prev[i];
            }
        }
        memcpy(x_prev, x, sizeof(double) * N);
        memcpy(f_prev, f, sizeof(double) * N);

        if ((k + 1) % p == 0) {
            /* Anderson step (Eq. 3, second case), preceded by the convergence test */
            r = sqrt(dot(N, res, res)) / nb;
            int64_t row = -1;
            if (trace && trace_len && *trace_len < trace_cap) {
                row = (*trace_len)++;
                trace[row * 6 + 0] = (double)k;
                trace[row * 6 + 1] = r;
                trace[row * 6 + 2] = sqrt(dot(N, f, f));
                trace[row * 6 + 3] = 0.0;
                trace[row * 6 + 4] = 0.0;
                trace[row * 6 + 5] = 1.0;
            }
            if (!isfinite(r)) {
                status = ORACLE_BREAKDOWN;
                *iters_out = k + 1;
                break;
            }
            if (r < tol) {
                status = ORACLE_OK;
                *iters_out = k + 1;
                break;
            }
            /* G = F^T F, c = F^T f_k */
            for (int a = 0; a < cols; ++a) {
                const double *fa = DF + (int64_t)order[a] * N;
                for (int bb = a; bb < cols; ++bb) {
                    const double *fb = DF + (int64_t)order[bb] * N;
                    G[a * cols + bb] = G[bb * cols + a] = dot(N, fa, fb);
                }
                c[a] = dot(N, fa, f);
            }
            double cond = 1.0;
            int rank = pinv_solve_cond(cols, G, c, gamma, &cond);
            /* x_{k+1} = x_k + beta f_k - (X_k + beta F_k) gamma */
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) {
                double corr = 0.0;
                for (int a = 0; a < cols; ++a)
                    corr += (DX[(int64_t)order[a] * N + i] + beta * DF[(int64_t)order[a] * N + i]) *
                            gamma[a];
                x[i] = x[i] + beta * f[i] - corr;
            }
            if (row >= 0) {
                /* ||f_k - F_k gamma||: the residual of the least-squares problem
                 * (res is free again: it is recomputed at the next iteration) */
#pragma omp parallel for schedule(static)
                for (int64_t i = 0; i < N; ++i) {
                    double e = f[i];
                    for (int a = 0; a < cols; ++a)
                        e -= DF[(int64_t)order[a] * N + i] * gamma[a];
                    res[i] = e;
                }
                trace[row * 6 + 3] = sqrt(dot(N, res, res));
                trace[row * 6 + 4] = rank;
                trace[row * 6 + 5] = cond;
            }
        } else {
            /* Richardson step (Eq. 3, first case) */
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i)
                x[i] = x[i] + omega * f[i];
        }

        if (k + 1 == max_iter) {
            *iters_out = max_iter;
            status = ORACLE_NOT_CONVERGED;
            break;
        }
    }
    *relres_out = r;

    free(res);
    free(f);
    free(x_prev);
    free(f_prev);
    free(DX);
    free(DF);
    free(order);
    free(G);
    free(c);
    free(gamma);
    return status;
}

/* Residual step of the stencil operator with the Jacobi preconditioner
 * M = D = diag(A): f_k = D^{-1}(b - A x_k). */
typedef struct {
    const oracle_problem *P;
    const double *b;
    const double *D;
} stencil_ctx;

static void stencil_residual(void *c, const double *x, double *res, double *f)
{
    const stencil_ctx *S = (const stencil_ctx *)c;
    const int64_t N = problem_size(S->P);
    oracle_apply(S->P, x, res);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        res[i] = S->b[i] - res[i];
        f[i] = res[i] / S->D[i];
    }
}

int oracle_aar_solve(const oracle_problem *P, const double *b, double *x,
                     double omega, double beta, int m, int p, double tol, int64_t max_iter,
                     int64_t *iters_out, double *relres_out,
                     double *trace, int64_t trace_cap, int64_t *trace_len)
{
    const int64_t N = problem_size(P);
    if (N <= 0)
        return ORACLE_BAD_ARG;
    double *D = malloc(sizeof(double) * N);
    oracle_diagonal(P, D);
    stencil_ctx c = {P, b, D};
    int st = aar_iterate(N, stencil_residual, &c, b, x, omega, beta, m, p, tol, max_iter, iters_out, relres_out,
                         trace, trace_cap, trace_len);
    free(D);
    return st;
}

/* ||b - A x|| / ||b|| in FP64 (used to check any solver's final answer). */
double oracle_relative_residual(const oracle_problem *P, const double *b, const double *x)
{
    const int64_t N = problem_size(P);
    double *y = malloc(sizeof(double) * N);
    oracle_apply(P, x, y);
    double num = blocked_sum(N, b, y, 1);
    double den = dot(N, b, b);
    free(y);
    return den > 0.0 ? sqrt(num) / sqrt(den) : sqrt(num);
}

/*
 * The constant-mode step of the solver's optional deflation (not part of the
 * paper's method).  When every axis is periodic the constant vector 1 is an
 * eigenvector of A with eigenvalue sigma: each row of the central second
 * difference sums to zero (w_0 = -2 sum w_s) and the upwind differences of a
 * constant vanish, so A 1 = sigma 1.  For sigma > 0, with r = b - A x, the
 * step x <- x + (mean r / sigma) 1 changes the residual to r - (mean r) 1,
 * whose mean is zero; the solution of A x = b is unchanged.  Written out from
 * that definition: one application of A, the mean as a plain sum over the
 * grid, and the shift of every value.  Returns ORACLE_BAD_ARG unless every
 * axis is periodic and sigma > 0.
 */
int oracle_deflate_constant(const oracle_problem *P, const double *b, double *x)
{
    if (P->bc[0] != 1 || P->bc[1] != 1 || P->bc[2] != 1 || !(P->shift > 0.0))
        return ORACLE_BAD_ARG;
    const int64_t N = problem_size(P);
    double *ax = malloc(sizeof(double) * N);
    oracle_apply(P, x, ax);
    double sum = 0.0;
    for (int64_t i = 0; i < N; ++i)
        sum += b[i] - ax[i];
    const double shift = (sum / (double)N) / P->shift;
    for (int64_t i = 0; i < N; ++i)
        x[i] += shift;
    free(ax);
    return ORACLE_OK;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ====================================================================== */
/* Complex-valued systems                                                  */
/* ====================================================================== */
/*
 * The method is stated for A, x, b complex (Sec. 2, Eq. 1), with complex
 * relaxation parameters omega, beta and T the conjugate transpose (Eq. 3);
 * the paper's periodic Helmholtz problem (Sec. 3.2, Eq. 7) has a complex
 * shift Q and a complex right-hand side P rho^alpha.  Here A = A_r + i s I:
 * the real finite-difference operator of P (with its real shift) plus an
 * imaginary shift s.  Complex vectors are stored interleaved (re, im) per
 * grid point.  Plain C99 complex arithmetic; the steps are those of
 * oracle_aar_solve in the same order.
 */
#include <complex.h>

typedef double complex cplx;

/* y = A x = A_r x + i s x. */
void oracle_apply_complex(const oracle_problem *P, double shift_im, const double *x, double *y)
{
    const int64_t N = problem_size(P);
    double *xr = malloc(sizeof(double) * N), *xi = malloc(sizeof(double) * N);
    double *yr = malloc(sizeof(double) * N), *yi = malloc(sizeof(double) * N);
    for (int64_t i = 0; i < N; ++i) {
        xr[i] = x[2 * i];
        xi[i] = x[2 * i + 1];
    }
    oracle_apply(P, xr, yr);
    oracle_apply(P, xi, yi);
    for (int64_t i = 0; i < N; ++i) {
        y[2 * i] = yr[i] - shift_im * xi[i];
        y[2 * i + 1] = yi[i] + shift_im * xr[i];
    }
    free(xr);
    free(xi);
    free(yr);
    free(yi);
}

/* sum_i conj(a_i) b_i */
static cplx cdot(int64_t N, const cplx *a, const cplx *b)
{
    cplx s = 0.0;
    for (int64_t i = 0; i < N; ++i)
        s += conj(a[i]) * b[i];
    return s;
}

/* gamma = pinv(G) c for a Hermitian positive semidefinite l x l matrix G,
 * through its real form [[Re G, -Im G], [Im G, Re G]] (symmetric, the same
 * eigenvalues each twice): eigenvalues <= l lambda_max 2^-52 are dropped,
 * with l the complex order.  Returns the complex rank; *cond the condition
 * number over the kept eigenvalues. */
static int pinv_solve_hermitian(int l, const cplx *G, const cplx *c, cplx *gamma, double *cond)
{
    *cond = 1.0;
    if (l <= 0)
        return 0;
    const int L = 2 * l;
    double *S = malloc(sizeof(double) * L * L), *V = malloc(sizeof(double) * L * L), *cc = malloc(sizeof(double) * L);
    for (int a = 0; a < l; ++a) {
        for (int b = 0; b < l; ++b) {
            const double gr = creal(G[a * l + b]), gi = cimag(G[a * l + b]);
            S[a * L + b] = gr;
            S[a * L + (b + l)] = -gi;
            S[(a + l) * L + b] = gi;
            S[(a + l) * L + (b + l)] = gr;
        }
        cc[a] = creal(c[a]);
        cc[a + l] = cimag(c[a]);
    }
    oracle_jacobi_eigen(L, S, V);
    double lmax = 0.0;
    for (int i = 0; i < L; ++i)
        if (S[i * L + i] > lmax)
            lmax = S[i * L + i];
    const double thresh = l * lmax * ldexp(1.0, -52);
    double *g = calloc(L, sizeof(double));
    int kept = 0;
    double lmin = lmax;
    for (int e = 0; e < L; ++e) {
        const double lam = S[e * L + e];
        if (!(lam > thresh))
            continue;
        ++kept;
        if (lam < lmin)
            lmin = lam;
        double proj = 0.0;
        for (int i = 0; i < L; ++i)
            proj += V[i * L + e] * cc[i];
        for (int i = 0; i < L; ++i)
            g[i] += V[i * L + e] * proj / lam;
    }
    for (int a = 0; a < l; ++a)
        gamma[a] = g[a] + I * g[a + l];
    if (kept > 0)
        *cond = lmax / lmin;
    free(S);
    free(V);
    free(cc);
    free(g);
    return kept / 2;
}

/*
 * Complex AAR with M = diag(A) (complex): the steps of oracle_aar_solve with
 * complex values.  b, x interleaved complex (length 2N); omega, beta complex
 * (re, im); trace rows as there (k, r_k, ||f_k||, 0, rank, cond).
 */
int oracle_aar_solve_complex(const oracle_problem *P, double shift_im, const double *b_in, double *x_io,
                             double omega_re, double omega_im, double beta_re, double beta_im, int m, int p,
                             double tol, int64_t max_iter, int64_t *iters_out, double *relres_out, double *trace,
                             int64_t trace_cap, int64_t *trace_len)
{
    const int64_t N = problem_size(P);
    if (N <= 0 || m < 1 || p < 1 || !(tol > 0.0) || max_iter < 1)
        return ORACLE_BAD_ARG;
    if (trace_len)
        *trace_len = 0;
    *iters_out = 0;
    *relres_out = 0.0;
    const cplx omega = omega_re + I * omega_im, beta = beta_re + I * beta_im;
    const cplx *b = (const cplx *)b_in;
    cplx *x = (cplx *)x_io;
    const double nb = sqrt(creal(cdot(N, b, b)));
    if (nb == 0.0) {
        for (int64_t i = 0; i < N; ++i)
            x[i] = 0.0;
        return ORACLE_OK;
    }
    double *Dr = malloc(sizeof(double) * N);
    oracle_diagonal(P, Dr);
    cplx *D = malloc(sizeof(cplx) * N), *res = malloc(sizeof(cplx) * N), *f = malloc(sizeof(cplx) * N);
    cplx *x_prev = malloc(sizeof(cplx) * N), *f_prev = malloc(sizeof(cplx) * N);
    cplx *DX = malloc(sizeof(cplx) * N * m), *DF = malloc(sizeof(cplx) * N * m);
    cplx *G = malloc(sizeof(cplx) * m * m), *c = malloc(sizeof(cplx) * m), *gamma = malloc(sizeof(cplx) * m);
    int *order = malloc(sizeof(int) * m);
    for (int64_t i = 0; i < N; ++i)
        D[i] = Dr[i] + I * shift_im;
    int cols = 0, status = ORACLE_NOT_CONVERGED;
    double r = 0.0;
    for (int64_t k = 0;; ++k) {
        /* f_k = D^{-1}(b - A x_k)  (Eq. 6) */
        oracle_apply_complex(P, shift_im, (const double *)x, (double *)res);
        for (int64_t i = 0; i < N; ++i) {
            res[i] = b[i] - res[i];
            f[i] = res[i] / D[i];
        }
        /* history push (Eqs. 4-5) */
        if (k >= 1) {
            int slot;
            if (cols < m) {
                slot = cols;
                order[cols++] = slot;
            } else {
                slot = order[0];
                for (int t = 0; t < m - 1; ++t)
                    order[t] = order[t + 1];
                order[m - 1] = slot;
            }
            for (int64_t i = 0; i < N; ++i) {
                DX[(int64_t)slot * N + i] = x[i] - x_prev[i];
                DF[(int64_t)slot * N + i] = f[i] - f_prev[i];
            }
        }
        memcpy(x_prev, x, sizeof(cplx) * N);
        memcpy(f_prev, f, sizeof(cplx) * N);
        if ((k + 1) % p == 0) {
            r = sqrt(creal(cdot(N, res, res))) / nb;
            int64_t row = -1;
            if (trace && trace_len && *trace_len < trace_cap) {
                row = (*trace_len)++;
                trace[row * 6 + 0] = (double)k;
                trace[row * 6 + 1] = r;
                trace[row * 6 + 2] = sqrt(creal(cdot(N, f, f)));
                trace[row * 6 + 3] = 0.0;
                trace[row * 6 + 4] = 0.0;
                trace[row * 6 + 5] = 1.0;
            }
            if (!isfinite(r)) {
                status = ORACLE_BREAKDOWN;
                *iters_out = k + 1;
                break;
            }
            if (r < tol) {
                status = ORACLE_OK;
                *iters_out = k + 1;
                break;
            }
            /* G = F^H F, c = F^H f_k (T is the conjugate transpose, Eq. 3) */
            for (int a = 0; a < cols; ++a) {
                const cplx *fa = DF + (int64_t)order[a] * N;
                for (int bb = 0; bb < cols; ++bb)
                    G[a * cols + bb] = cdot(N, fa, DF + (int64_t)order[bb] * N);
                c[a] = cdot(N, fa, f);
            }
            double cond = 1.0;
            const int rank = pinv_solve_hermitian(cols, G, c, gamma, &cond);
            /* x_{k+1} = x_k + beta f_k - (X_k + beta F_k) gamma */
            for (int64_t i = 0; i < N; ++i) {
                cplx corr = 0.0;
                for (int a = 0; a < cols; ++a)
                    corr += (DX[(int64_t)order[a] * N + i] + beta * DF[(int64_t)order[a] * N + i]) * gamma[a];
                x[i] = x[i] + beta * f[i] - corr;
            }
            if (row >= 0) {
                /* ||f_k - F_k gamma||, the least-squares residual */
                for (int64_t i = 0; i < N; ++i) {
                    cplx e = f[i];
                    for (int a = 0; a < cols; ++a)
                        e -= DF[(int64_t)order[a] * N + i] * gamma[a];
                    res[i] = e;
                }
                trace[row * 6 + 3] = sqrt(creal(cdot(N, res, res)));
                trace[row * 6 + 4] = rank;
                trace[row * 6 + 5] = cond;
            }
        } else {
            /* Richardson step (Eq. 3, first case) */
            for (int64_t i = 0; i < N; ++i)
                x[i] = x[i] + omega * f[i];
        }
        if (k + 1 >= max_iter) {
            *iters_out = max_iter;
            break;
        }
    }
    *relres_out = r;
    free(Dr);
    free(D);
    free(res);
    free(f);
    free(x_prev);
    free(f_prev);
    free(DX);
    free(DF);
    free(G);
    free(c);
    free(gamma);
    free(order);
    return status;
}

/* ------------------------------------------------------------------------
 * General sparse A (Sec. 3.1: nonsymmetric systems with Jacobi and ILU(0)
 * preconditioning; Secs. 3.2-3.3: block-Jacobi with ILU(0) on each block,
 * the parallel preconditioner of the Helmholtz and Poisson runs).
 *
 * A is held in compressed sparse rows: the entries of row i are
 * val[rowptr[i] .. rowptr[i+1]-1] in columns col[...], strictly increasing,
 * the diagonal present.  Block Jacobi splits the rows into `nblocks`
 * contiguous ranges, block t holding rows floor(t n / nblocks) ..
 * floor((t+1) n / nblocks) - 1; its preconditioner M is block diagonal with
 * the ILU(0) factors of each diagonal block of A, and entries of A that
 * couple two blocks do not enter M.  nblocks = 1 is ILU(0) of A itself.
 *
 * ILU(0): L unit lower triangular and U upper triangular, both with the
 * sparsity pattern of (the block of) A, such that (L U)_ij = a_ij wherever a_ij
 * is in the pattern.  They come from Gaussian elimination in row order that
 * drops every fill-in outside the pattern: for row i and each k < i of its
 * pattern in increasing order, l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for
 * each j > k with both (i, j) and (k, j) in the pattern.  L and U overwrite a
 * copy of A's values (the unit diagonal of L is not stored).
 * ------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    const int64_t *rowptr;  /* n + 1 */
    const int32_t *col;
    const double *val;
} oracle_csr;

enum { ORACLE_PRECOND_JACOBI = 0, ORACLE_PRECOND_ILU0 = 1 };

static int64_t block_first_row(int64_t n, int nblocks, int64_t t)
{
    return t * n / nblocks;
}

/* Position of the diagonal entry of row i, or -1. */
static int64_t diag_pos(const oracle_csr *A, int64_t i)
{
    for (int64_t e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e)
        if (A->col[e] == i)
            return e;
    return -1;
}

/* ORACLE_OK when the arrays describe a valid matrix as above. */
int oracle_csr_check(const oracle_csr *A)
{
    if (A->n < 1 || A->rowptr[0] != 0)
        return ORACLE_BAD_ARG;
    for (int64_t i = 0; i < A->n; ++i) {
        if (A->rowptr[i + 1] < A->rowptr[i])
            return ORACLE_BAD_ARG;
        for (int64_t e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e) {
            if (A->col[e] < 0 || A->col[e] >= A->n)
                return ORACLE_BAD_ARG;
            if (e > A->rowptr[i] && A->col[e] <= A->col[e - 1])
                return ORACLE_BAD_ARG;
        }
        if (diag_pos(A, i) < 0)
            return ORACLE_BAD_ARG;
    }
    return ORACLE_OK;
}

/* y = A x, each row summed in stored order. */
void oracle_csr_apply(const oracle_csr *A, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < A->n; ++i) {
        double s = 0.0;
        for (int64_t e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e)
            s += A->val[e] * x[A->col[e]];
        y[i] = s;
    }
}

/* ILU(0) factors of each diagonal block into lu (a copy of A's values on
 * entry is not needed: lu is written whole).  Entries of lu outside their
 * row's block keep A's values and are never used.  Returns ORACLE_BREAKDOWN
 * when a pivot u_kk is zero or not finite. */
int oracle_ilu0(const oracle_csr *A, int nblocks, double *lu)
{
    const int64_t n = A->n;
    if (nblocks < 1 || nblocks > n)
        return ORACLE_BAD_ARG;
    memcpy(lu, A->val, sizeof(double) * (size_t)A->rowptr[n]);
    int bad = 0;
#pragma omp parallel for schedule(dynamic) reduction(| : bad)
    for (int t = 0; t < nblocks; ++t) {
        const int64_t lo = block_first_row(n, nblocks, t), hi = block_first_row(n, nblocks, t + 1);
        for (int64_t i = lo; i < hi; ++i) {
            const int64_t end = A->rowptr[i + 1];
            for (int64_t e = A->rowptr[i]; e < end && A->col[e] < i; ++e) {
                const int64_t k = A->col[e];
                if (k < lo)
                    continue;                    /* couples two blocks: not in M */
                const double lik = lu[e] / lu[diag_pos(A, k)];
                lu[e] = lik;
                for (int64_t e2 = e + 1; e2 < end; ++e2) {
                    const int64_t j = A->col[e2];
                    if (j >= hi)
                        break;                   /* later columns lie outside the block */
                    /* u_kj, if (k, j) is in the pattern */
                    for (int64_t ek = A->rowptr[k]; ek < A->rowptr[k + 1]; ++ek)
                        if (A->col[ek] == j) {
                            lu[e2] -= lik * lu[ek];
                            break;
                        }
                }
            }
            const double u = lu[diag_pos(A, i)];
            if (u == 0.0 || !isfinite(u))
                bad = 1;
        }
    }
    return bad ? ORACLE_BREAKDOWN : ORACLE_OK;
}

/* z = M^{-1} r for the block ILU(0) factors in lu: L y = r by forward
 * substitution, then U z = y by backward substitution, within each block. */
void oracle_ilu0_solve(const oracle_csr *A, int nblocks, const double *lu, const double *r, double *z)
{
    const int64_t n = A->n;
#pragma omp parallel for schedule(dynamic)
    for (int t = 0; t < nblocks; ++t) {
        const int64_t lo = block_first_row(n, nblocks, t), hi = block_first_row(n, nblocks, t + 1);
        for (int64_t i = lo; i < hi; ++i) {
            double y = r[i];
            for (int64_t e = A->rowptr[i]; e < A->rowptr[i + 1] && A->col[e] < i; ++e)
                if (A->col[e] >= lo)
                    y -= lu[e] * z[A->col[e]];
            z[i] = y;
        }
        for (int64_t i = hi - 1; i >= lo; --i) {
            const int64_t d = diag_pos(A, i);
            double v = z[i];
            for (int64_t e = d + 1; e < A->rowptr[i + 1] && A->col[e] < hi; ++e)
                v -= lu[e] * z[A->col[e]];
            z[i] = v / lu[d];
        }
    }
}

typedef struct {
    const oracle_csr *A;
    const double *b;
    int precond;
    int nblocks;
    const double *lu;    /* ILU(0) factors, or NULL for Jacobi */
} csr_ctx;

/* Residual step of a sparse A: res = b - A x, f = M^{-1} res with M the
 * Jacobi diagonal or the block ILU(0) factors. */
static void csr_residual(void *c, const double *x, double *res, double *f)
{
    const csr_ctx *C = (const csr_ctx *)c;
    const oracle_csr *A = C->A;
    oracle_csr_apply(A, x, res);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < A->n; ++i)
        res[i] = C->b[i] - res[i];
    if (C->precond == ORACLE_PRECOND_JACOBI) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < A->n; ++i)
            f[i] = res[i] / A->val[diag_pos(A, i)];
    } else {
        oracle_ilu0_solve(A, C->nblocks, C->lu, res, f);
    }
}

/* z = M^{-1} r for the preconditioner `precond` (Jacobi, or block ILU(0)
 * with nblocks blocks).  Returns ORACLE_BREAKDOWN when the factorization
 * meets a zero pivot. */
int oracle_csr_precondition(const oracle_csr *A, int precond, int nblocks, const double *r, double *z)
{
    if (oracle_csr_check(A) != ORACLE_OK)
        return ORACLE_BAD_ARG;
    if (precond == ORACLE_PRECOND_JACOBI) {
        for (int64_t i = 0; i < A->n; ++i)
            z[i] = r[i] / A->val[diag_pos(A, i)];
        return ORACLE_OK;
    }
    if (precond != ORACLE_PRECOND_ILU0)
        return ORACLE_BAD_ARG;
    double *lu = malloc(sizeof(double) * (size_t)A->rowptr[A->n]);
    int st = oracle_ilu0(A, nblocks, lu);
    if (st == ORACLE_OK)
        oracle_ilu0_solve(A, nblocks, lu, r, z);
    free(lu);
    return st;
}

/* Preconditioned AAR for a sparse A (Sec. 2 with M from Sec. 3.1 / 3.2):
 * the same iteration, arguments and trace as oracle_aar_solve, with M the
 * Jacobi diagonal (precond 0) or block ILU(0) with nblocks blocks
 * (precond 1).  A zero ILU(0) pivot returns ORACLE_BREAKDOWN before any
 * iteration. */
int oracle_aar_solve_csr(const oracle_csr *A, int precond, int nblocks, const double *b, double *x,
                         double omega, double beta, int m, int p, double tol, int64_t max_iter,
                         int64_t *iters_out, double *relres_out,
                         double *trace, int64_t trace_cap, int64_t *trace_len)
{
    if (oracle_csr_check(A) != ORACLE_OK)
        return ORACLE_BAD_ARG;
    if (precond != ORACLE_PRECOND_JACOBI && precond != ORACLE_PRECOND_ILU0)
        return ORACLE_BAD_ARG;
    if (precond == ORACLE_PRECOND_ILU0 && (nblocks < 1 || nblocks > A->n))
        return ORACLE_BAD_ARG;
    *iters_out = 0;
    *relres_out = 0.0;
    if (trace_len)
        *trace_len = 0;
    double *lu = NULL;
    if (precond == ORACLE_PRECOND_ILU0) {
        lu = malloc(sizeof(double) * (size_t)A->rowptr[A->n]);
        int st = oracle_ilu0(A, nblocks, lu);
        if (st != ORACLE_OK) {
            free(lu);
            return st;
        }
    }
    csr_ctx c = {A, b, precond, nblocks, lu};
    int st = aar_iterate(A->n, csr_residual, &c, b, x, omega, beta, m, p, tol, max_iter, iters_out, relres_out,
                         trace, trace_cap, trace_len);
    free(lu);
    return st;
}

/* ||b - A x|| / ||b|| for a sparse A. */
double oracle_relative_residual_csr(const oracle_csr *A, const double *b, const double *x)
{
    double *r = malloc(sizeof(double) * (size_t)A->n);
    oracle_csr_apply(A, x, r);
    for (int64_t i = 0; i < A->n; ++i)
        r[i] = b[i] - r[i];
    const double out = sqrt(dot(A->n, r, r)) / sqrt(dot(A->n, b, b));
    free(r);
    return out;
}
