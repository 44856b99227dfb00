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
int oracle_aar_solve(const oracle_problem *P, const double *b, double *x,
                     double omega, double beta, int m, int p, double tol, int64_t max_iter,
                     int64_t *iters_out, double *relres_out,
                     double *trace, int64_t trace_cap, int64_t *trace_len)
{
    const int64_t N = problem_size(P);
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

    double *D = malloc(sizeof(double) * N);
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

    oracle_diagonal(P, D);

    for (int64_t k = 0;; ++k) {
        /* residual and preconditioned residual f_k = D^{-1}(b - A x_k)  (Eq. 6) */
        oracle_apply(P, x, res);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            res[i] = b[i] - res[i];
            f[i] = res[i] / D[i];
        }

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

    free(D);
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
