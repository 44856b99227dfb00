/* Drives every entry point of oracle/aar_oracle.c on small problems, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): out
 * of bounds accesses, leaks, signed overflow or misaligned loads in the
 * oracle abort the run.  Exit status 0 means every call returned normally. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t n[3];
    double h[3];
    int32_t bc[3];
    int32_t radius;
    double diffusion;
    double shift;
    const double *velocity;
} oracle_problem;

void oracle_fd_weights(int r, double *w);
void oracle_apply(const oracle_problem *P, const double *x, double *y);
void oracle_diagonal(const oracle_problem *P, double *d);
void oracle_jacobi_eigen(int n, double *S, double *V);
int oracle_pinv_solve(int l, const double *G, const double *c, double *gamma);
int oracle_aar_solve(const oracle_problem *P, const double *b, double *x, double omega, double beta, int m, int p,
                     double tol, int64_t max_iter, int64_t *iters, double *relres, double *trace, int64_t cap,
                     int64_t *len);
double oracle_relative_residual(const oracle_problem *P, const double *b, const double *x);
int oracle_deflate_constant(const oracle_problem *P, const double *b, double *x);

static double rnd(uint64_t *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) * 0x1.0p-53 - 0.5;
}

static int run(const oracle_problem *P, int m, int p, int64_t cap, uint64_t seed)
{
    const int64_t N = (int64_t)P->n[0] * P->n[1] * P->n[2];
    double *b = malloc(sizeof(double) * N), *x = calloc(N, sizeof(double)), *y = malloc(sizeof(double) * N);
    double trace[6 * 64];
    for (int64_t i = 0; i < N; ++i)
        b[i] = rnd(&seed);
    oracle_apply(P, b, y);
    oracle_diagonal(P, y);
    int64_t it = 0, len = 0;
    double rr = 0.0;
    int st = oracle_aar_solve(P, b, x, 0.6, 0.6, m, p, 1e-8, cap, &it, &rr, trace, 64, &len);
    double rel = oracle_relative_residual(P, b, x);
    if (P->bc[0] == 1 && P->bc[1] == 1 && P->bc[2] == 1 && P->shift > 0.0)
        oracle_deflate_constant(P, b, x);
    printf("n=%dx%dx%d r=%d m=%d p=%d status=%d iterations=%lld relres=%.3e check=%.3e trace=%lld\n", P->n[0],
           P->n[1], P->n[2], P->radius, m, p, st, (long long)it, rr, rel, (long long)len);
    free(b);
    free(x);
    free(y);
    return st < 0;
}

int main(void)
{
    int bad = 0;
    double w[7];
    for (int r = 1; r <= 6; ++r)
        oracle_fd_weights(r, w);
    /* pseudoinverse on a rank-deficient Gram (two equal columns) and l = 0 */
    double G[9] = {4, 4, 2, 4, 4, 2, 2, 2, 5}, c[3] = {1, 1, 2}, g[3];
    bad |= oracle_pinv_solve(3, G, c, g) != 2;
    bad |= oracle_pinv_solve(0, G, c, g) != 0;
    double S[4] = {2, 1, 1, 2}, V[4];
    oracle_jacobi_eigen(2, S, V);

    oracle_problem d = {{9, 7, 5}, {0.1, 0.125, 1.0 / 6}, {0, 0, 0}, 1, 1.0, 0.0, NULL};
    bad |= run(&d, 7, 6, 400, 1);
    bad |= run(&d, 20, 1, 60, 2);               /* history longer than the run */
    oracle_problem q = {{4, 6, 5}, {0.25, 1.0 / 6, 0.2}, {1, 1, 1}, 6, 1.0, 0.7, NULL};
    bad |= run(&q, 7, 6, 400, 3);               /* periodic axes shorter than the stencil */
    oracle_problem mix = {{8, 3, 11}, {0.1, 0.3, 0.09}, {1, 0, 1}, 3, 0.7, 0.2, NULL};
    bad |= run(&mix, 3, 5, 300, 4);             /* p > m */
    const int64_t Nc = 6 * 5 * 7;
    double *vel = malloc(sizeof(double) * 3 * Nc);
    uint64_t s = 9;
    for (int64_t i = 0; i < 3 * Nc; ++i)
        vel[i] = 40.0 * rnd(&s);
    oracle_problem cd = {{6, 5, 7}, {1.0 / 7, 1.0 / 6, 1.0 / 8}, {0, 0, 0}, 1, 1.0, 0.0, vel};
    bad |= run(&cd, 10, 4, 400, 5);             /* upwind convection */
    oracle_problem cdp = {{6, 5, 7}, {1.0 / 6, 1.0 / 5, 1.0 / 7}, {1, 1, 1}, 1, 1.0, 0.3, vel};
    bad |= run(&cdp, 10, 4, 400, 6);
    free(vel);
    return bad;
}
