// Device-side math of the Anderson step, shared by the single-system and the
// batched kernels: vector packs, the least-squares core (convergence test,
// pseudoinverse solve, update plan).
#pragma once

#include <math.h>

#include "aar_device.h"

namespace aar {

template <typename T> __device__ inline T wave_sum_a(T v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// Wave sums of E (<= 64) values held by every lane, transposed: lane l
// returns the sum over the wave of entry l (0 for l >= E).  Each of the six
// butterfly rounds halves the entries a lane carries: the lane keeps the half
// selected by its bit o and adds the partner's copy of that half, so the
// rounds exchange 32 + 16 + ... + 1 = 63 values instead of 6 E.
template <int E> __device__ inline double wave_transpose_sum(const double (&v)[E])
{
    static_assert(E <= 64, "at most one entry per lane");
    double a[64];
#pragma unroll
    for (int i = 0; i < 64; ++i)
        a[i] = i < E ? v[i] : 0.0;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const bool hi = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < o; ++i) {
            const double keep = hi ? a[i + o] : a[i];
            const double send = hi ? a[i] : a[i + o];
            a[i] = keep + __shfl_xor(send, o, 64);
        }
    }
    return a[0];
}

// Wave totals of E per-lane values written to dst[0 .. E) (lane e mod 64
// writes entry e), 64 entries per transposed reduction.
template <int E, int B = 0> __device__ inline void wave_sums_to(const double (&v)[E], double *dst)
{
    constexpr int C = E - B < 64 ? E - B : 64;
    double part[C];
#pragma unroll
    for (int i = 0; i < C; ++i)
        part[i] = v[B + i];
    const double t = wave_transpose_sum<C>(part);
    const int lane = threadIdx.x & 63;
    if (lane < C)
        dst[B + lane] = t;
    if constexpr (B + 64 < E)
        wave_sums_to<E, B + 64>(v, dst);
}

// V consecutive elements moved by one 16-byte (8-byte for bf16) access.
template <typename E, int V> struct alignas(sizeof(E) * V) Pack {
    E v[V];
};

template <typename H> struct VecWidth {
    static constexpr int value = 16 / (int)sizeof(H) > 8 ? 8 : 16 / (int)sizeof(H);
};
template <> struct VecWidth<bf16_t> {
    static constexpr int value = 4;
};

template <typename H, int V>
__device__ inline void load_vec(const H *p, int64_t i, double *out)
{
    const Pack<H, V> pk = *reinterpret_cast<const Pack<H, V> *>(p + i);
#pragma unroll
    for (int u = 0; u < V; ++u)
        out[u] = (double)Hist<H>::load(pk.v, u);
}

// Gram contributions of one grid point: col[t] = f at history position t
// (t = 0 oldest, t = l holds f_k); columns c < l are col[c+1] - col[c].
// acc holds the MC(MC+1)/2 upper-triangle products, then the MC products with f_k.
template <int MC> __device__ inline void gram_point(const double *col, int l, double *acc)
{
    constexpr int NP = MC * (MC + 1) / 2;
    double fk = 0.0;
#pragma unroll
    for (int t = 0; t <= MC; ++t)
        fk = t == l ? col[t] : fk;
    double d[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c)
        d[c] = c < l ? col[c + 1] - col[c] : 0.0;
    int e = 0;
#pragma unroll
    for (int c = 0; c < MC; ++c) {
#pragma unroll
        for (int c2 = c; c2 < MC; ++c2)
            acc[e++] += d[c] * d[c2];
    }
#pragma unroll
    for (int c = 0; c < MC; ++c)
        acc[NP + c] += d[c] * fk;
}

constexpr int kLsqThreads = 64;   // one wave: barriers are cheap
constexpr int kRegM = 8;          // history lengths whose m x m solve runs in registers

// Position of entry (i, j), i <= j, in the upper triangle of an m x m matrix
// stored row by row.
__device__ inline int tri_index(int i, int j, int m)
{
    return i * m - i * (i - 1) / 2 + (j - i);
}

// gamma = pinv(S) c for the symmetric l x l matrix held in S (LDS; rows and
// columns from l on are scratch), run by one wave: parallel cyclic Jacobi
// rotations with the round-robin ordering, then eigenvalues at or below
// rcond * thresh_order * lambda_max are dropped (thresh_order is the order
// the threshold counts: l for a real matrix, the complex order for the real
// form of a Hermitian one).  Leaves the eigenvalues on the diagonal of S, the
// eigenvectors in V and the threshold in sh_off; gamma goes to gam.
__device__ inline void jacobi_pinv(int l, double rcond, double thresh_order, double (*S)[kMaxM + 1],
                                   double (*V)[kMaxM + 1], const double *cvec, double *wvec, double *gam,
                                   double *rot_c, double *rot_s, int *pair_p, int *pair_q, double &sh_off,
                                   int &sh_stop)
{
    const int tid = threadIdx.x;
    // ---- gamma = pinv(S) c by parallel cyclic Jacobi (round-robin pairs) ----
    const int L = l + (l & 1);   // even order; index l is a dummy when l is odd
    for (int i = tid; i < kMaxM * kMaxM; i += kLsqThreads) {
        const int row = i / kMaxM, col = i % kMaxM;
        if (row < L && col < L) {
            V[row][col] = row == col ? 1.0 : 0.0;
            if (row >= l || col >= l)
                S[row][col] = 0.0;
        }
    }
    __syncthreads();
    const int half = L / 2;
    const int M1 = L - 1;
    // Sweeps stop when one applies no rotation: a pair is rotated only while
    // |s_pq| > 1e-15 sqrt(|s_pp s_qq|) (negligible against both diagonals).
    for (int sweep = 0; sweep < 40 && L >= 2; ++sweep) {
        if (tid == 0)
            sh_stop = 1;
        __syncthreads();
        for (int round = 0; round < M1; ++round) {
            if (tid < half) {
                // circle method: index L-1 meets `round`; the others pair
                // (round + i) mod (L-1) with (round - i) mod (L-1)
                int p, qq;
                if (tid == 0) {
                    p = round;
                    qq = L - 1;
                } else {
                    p = (round + tid) % M1;
                    qq = (round - tid + M1) % M1;
                }
                if (p > qq) {
                    const int t = p;
                    p = qq;
                    qq = t;
                }
                double c = 1.0, sn = 0.0;
                if (qq < l) {
                    const double apq = S[p][qq];
                    const double app = S[p][p], aqq = S[qq][qq];
                    if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > 1e-300) {
                        const double theta = (aqq - app) / (2.0 * apq);
                        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        sn = t * c;
                        sh_stop = 0;
                    }
                }
                pair_p[tid] = p;
                pair_q[tid] = qq;
                rot_c[tid] = c;
                rot_s[tid] = sn;
            }
            __syncthreads();
            // rows: S <- J^T S
            for (int it = tid; it < half * L; it += kLsqThreads) {
                const int pi = it / L, col = it % L;
                const int p = pair_p[pi], qq = pair_q[pi];
                const double c = rot_c[pi], sn = rot_s[pi];
                const double sp = S[p][col], sq = S[qq][col];
                S[p][col] = c * sp - sn * sq;
                S[qq][col] = sn * sp + c * sq;
            }
            __syncthreads();
            // columns: S <- S J, V <- V J
            for (int it = tid; it < half * L; it += kLsqThreads) {
                const int pi = it / L, row = it % L;
                const int p = pair_p[pi], qq = pair_q[pi];
                const double c = rot_c[pi], sn = rot_s[pi];
                const double sp = S[row][p], sq = S[row][qq];
                S[row][p] = c * sp - sn * sq;
                S[row][qq] = sn * sp + c * sq;
                const double vp = V[row][p], vq = V[row][qq];
                V[row][p] = c * vp - sn * vq;
                V[row][qq] = sn * vp + c * vq;
            }
            __syncthreads();
            // the annihilated pairs are zero in exact arithmetic
            if (tid < half) {
                const int p = pair_p[tid], qq = pair_q[tid];
                if (qq < l && rot_s[tid] != 0.0) {
                    S[p][qq] = 0.0;
                    S[qq][p] = 0.0;
                }
            }
            __syncthreads();
        }
        if (sh_stop)
            break;
    }
    // eigenvalues on the diagonal; drop those <= rcond * l * lambda_max
    if (tid == 0) {
        double lmax = 0.0;
        for (int i = 0; i < l; ++i)
            lmax = fmax(lmax, S[i][i]);
        sh_off = rcond * thresh_order * lmax;
    }
    __syncthreads();
    const double thresh = sh_off;
    for (int e = tid; e < l; e += kLsqThreads) {
        const double lam = S[e][e];
        double proj = 0.0;
        for (int i = 0; i < l; ++i)
            proj += V[i][e] * cvec[i];
        wvec[e] = lam > thresh ? proj / lam : 0.0;
    }
    __syncthreads();
    for (int i = tid; i < l; i += kLsqThreads) {
        double g = 0.0;
        for (int e = 0; e < l; ++e)
            g += V[i][e] * wvec[e];
        gam[i] = g;
    }
    __syncthreads();
}

// Cholesky solve of the symmetric l x l matrix S (LDS) when it provably
// equals the pseudoinverse solve: S = L L^T succeeds and every eigenvalue
// exceeds rcond * thresh_order * lambda_max, shown by lambda_min >=
// 1 / ||L^-1||_F^2 and lambda_max <= trace_scale * trace(S) (trace_scale 1 for
// a real matrix; 1/2 for the real form of a Hermitian one, whose eigenvalues
// come in pairs).  One wave; V receives L, Li its inverse; gamma goes to gam.
// Returns whether the solve was taken.
__device__ inline bool cholesky_proved_solve(int l, double rcond, double thresh_order, double trace_scale,
                                             double (*S)[kMaxM + 1], double (*V)[kMaxM + 1],
                                             double (*Li)[kMaxM + 1], const double *cvec, double *wvec,
                                             double *gam, int &sh_fail)
{
    const int tid = threadIdx.x;
    bool fast = false;
    for (int i = tid; i < l * l; i += kLsqThreads)
        V[i / l][i % l] = S[i / l][i % l];
    if (tid == 0)
        sh_fail = 0;
    __syncthreads();
    for (int j = 0; j < l; ++j) {
        if (tid == 0) {
            const double piv = V[j][j];
            if (!(piv > 0.0))
                sh_fail = 1;
            else
                V[j][j] = sqrt(piv);
        }
        __syncthreads();
        if (sh_fail)
            break;
        for (int i = j + 1 + tid; i < l; i += kLsqThreads)
            V[i][j] /= V[j][j];
        __syncthreads();
        const int w = l - j - 1;   // trailing block (j+1 .. l-1)^2, lower part
        for (int idx = tid; idx < w * w; idx += kLsqThreads) {
            const int i = j + 1 + idx / w, kk = j + 1 + idx % w;
            if (kk <= i)
                V[i][kk] -= V[i][j] * V[kk][j];
        }
        __syncthreads();
    }
    if (!sh_fail) {
        // columns of L^-1, one lane per column
        for (int c = tid; c < l; c += kLsqThreads) {
            for (int i = 0; i < c; ++i)
                Li[i][c] = 0.0;
            for (int i = c; i < l; ++i) {
                double acc = i == c ? 1.0 : 0.0;
                for (int kk = c; kk < i; ++kk)
                    acc -= V[i][kk] * Li[kk][c];
                Li[i][c] = acc / V[i][i];
            }
        }
        __syncthreads();
        double fro = 0.0, tr = 0.0;
        for (int i = tid; i < l * l; i += kLsqThreads)
            fro += Li[i / l][i % l] * Li[i / l][i % l];
        for (int i = tid; i < l; i += kLsqThreads)
            tr += S[i][i];
        fro = __shfl(wave_sum_a(fro), 0, 64);
        tr = __shfl(wave_sum_a(tr), 0, 64);
        fast = (1.0 / fro > rcond * thresh_order * (tr * trace_scale)) && fro == fro;
        if (fast) {
            for (int i = tid; i < l; i += kLsqThreads) {   // y = L^-1 c
                double y = 0.0;
                for (int kk = 0; kk <= i; ++kk)
                    y += Li[i][kk] * cvec[kk];
                wvec[i] = y;
            }
            __syncthreads();
            for (int i = tid; i < l; i += kLsqThreads) {   // gamma = L^-T y
                double g = 0.0;
                for (int kk = i; kk < l; ++kk)
                    g += Li[kk][i] * wvec[kk];
                gam[i] = g;
            }
            __syncthreads();
        }
    }
    return fast;
}

// The least-squares step of one system: convergence test, gamma and the
// update plan.  rho2 = ||b - A x_k||^2 and gram_vals (the m(m+1)/2 entries of
// the upper triangle of F^T F, then F^T f_k) are already summed.  Run by one
// wave; every early return is uniform across it.
//
// For m <= kRegM every lane holds the whole matrix and factors it in
// registers (no LDS traffic, no barriers); larger m use LDS.  Either way the
// Cholesky solve is taken only when it provably equals the pseudoinverse
// solve, else the Jacobi eigendecomposition runs.
__device__ inline void lsq_core(const LsqArgs &a, InstState *st, double rho2, const double *gram_vals)
{
    __shared__ double S[kMaxM][kMaxM + 1];
    __shared__ double V[kMaxM][kMaxM + 1];
    __shared__ double cvec[kMaxM];
    __shared__ double wvec[kMaxM];
    __shared__ double gam[kMaxM];
    __shared__ double rot_c[kMaxM / 2], rot_s[kMaxM / 2];
    __shared__ int pair_p[kMaxM / 2], pair_q[kMaxM / 2];
    __shared__ double Li[kMaxM][kMaxM + 1];
    __shared__ double sh_off;
    __shared__ int sh_stop;
    __shared__ int sh_fail;

    const int tid = threadIdx.x;
    const bool small = a.m <= kRegM;
    const int np = a.m * (a.m + 1) / 2;
    // Every input is read up front, before the first branch on the run
    // state, so the kernel waits for one memory round trip: in registers the
    // lower triangle of S and c (small m, every lane), else the Gram entries
    // spread over the lanes (one to nine each), and the run state.
    double R[kRegM][kRegM];
    double cr[kRegM];
    constexpr int kNeMax = kMaxM * (kMaxM + 1) / 2 + kMaxM;
    constexpr int kPer = (kNeMax + kLsqThreads - 1) / kLsqThreads;
    double gv[kPer];
    if (small) {
#pragma unroll
        for (int i = 0; i < kRegM; ++i) {
#pragma unroll
            for (int j = 0; j <= i; ++j)
                R[i][j] = i < a.m ? gram_vals[tri_index(j, i, a.m)] : 0.0;
            cr[i] = i < a.m ? gram_vals[np + i] : 0.0;
        }
    } else {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + u * kLsqThreads;
            gv[u] = e < a.ne ? gram_vals[e] : 0.0;
        }
    }
    const int status0 = st->status;
    const int64_t cycle0 = st->cycle, max_iter0 = st->max_iter;
    const double nb0 = st->nb, tol0 = st->tol, best_r0 = st->best_r;
    const int log_count0 = st->log_count, since_best0 = st->since_best;
    const int64_t restart0 = st->restart_pos;
    if (status0 != kRunning)
        return;
    const int64_t k = cycle0 * a.p + a.p - 1;
    if (k >= max_iter0) {
        if (tid == 0) {
            st->iters = max_iter0;
            st->status = kMaxIter;
        }
        return;
    }
    const int l = (int)(k < a.m ? k : a.m);
    // the column k - l + cb -> k - l + cb + 1 that spans a carried-over
    // history's restart (its two residuals belong to different right-hand
    // sides) is a null column: its row and column of F^T F and its entry of
    // F^T f are zero, so the pseudoinverse gives it no weight (footnote to Eq. 5)
    const int64_t cb64 = restart0 > 0 ? restart0 - 1 - (k - l) : -1;
    const int cb = (cb64 >= 0 && cb64 < l) ? (int)cb64 : -1;
    if (cb >= 0) {
        if (small) {
#pragma unroll
            for (int i = 0; i < kRegM; ++i) {
#pragma unroll
                for (int j = 0; j <= i; ++j)
                    R[i][j] = (i == cb || j == cb) ? 0.0 : R[i][j];
                cr[i] = i == cb ? 0.0 : cr[i];
            }
        } else {
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int e = tid + u * kLsqThreads;
                if (e < np) {
                    int row = 0, rem = e;
                    while (rem >= a.m - row) {
                        rem -= a.m - row;
                        ++row;
                    }
                    if (row == cb || row + rem == cb)
                        gv[u] = 0.0;
                } else if (e - np == cb) {
                    gv[u] = 0.0;
                }
            }
        }
    }

    const double rel = sqrt(rho2) / nb0;
    if (tid == 0) {
        st->last_r = rel;
        if (a.log && log_count0 < a.log_cap)
            a.log[log_count0] = rel;
        if (a.rank_log && log_count0 < a.log_cap)
            a.rank_log[log_count0] = -1;   // overwritten below when the step extrapolates
        st->log_count = log_count0 + 1;
    }
    // breakdown: a NaN or Inf in the residual or in the l x l Gram system
    bool bad = !isfinite(rel);
    if (small) {
#pragma unroll
        for (int i = 0; i < kRegM; ++i) {
#pragma unroll
            for (int j = 0; j <= i; ++j)
                bad = bad || (i < l && !isfinite(R[i][j]));
            bad = bad || (i < l && !isfinite(cr[i]));
        }
    } else {
        // G (upper triangle, row-major over the m x m layout) and c into LDS
        bool mine = false;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + u * kLsqThreads;
            if (e >= a.ne)
                continue;
            const double v = gv[u];
            if (e < np) {
                int row = 0, rem = e;
                while (rem >= a.m - row) {
                    rem -= a.m - row;
                    ++row;
                }
                const int col = row + rem;
                if (row < l && col < l) {
                    S[row][col] = v;
                    S[col][row] = v;
                    mine = mine || !isfinite(v);
                }
            } else if (e - np < l) {
                cvec[e - np] = v;
                mine = mine || !isfinite(v);
            }
        }
        bad = bad || __any(mine);
        __syncthreads();
    }
    if (bad || rel < tol0) {
        if (tid == 0) {
            st->iters = k + 1;
            st->status = bad ? kBreakdown : kConverged;
        }
        return;
    }
    if (a.stagnation_window > 0) {
        // inner solves of the refinement stop when the best residual has not
        // fallen by the given factor over the last `window` Anderson steps
        if (tid == 0) {
            int since = since_best0 + 1;
            if (rel < a.stagnation_factor * best_r0) {
                st->best_r = rel;
                since = 0;
            }
            st->since_best = since;
            sh_stop = since >= a.stagnation_window;
        }
        __syncthreads();
        if (sh_stop) {
            if (tid == 0) {
                st->iters = k + 1;
                st->status = kStagnated;
            }
            return;
        }
    }

    // ---- fast path: Cholesky S = L L^T ----
    // When every eigenvalue of S provably exceeds the pseudoinverse threshold
    // rcond * l * lambda_max, the pseudoinverse is the inverse and
    // gamma = L^-T L^-1 c.  The proof: lambda_min >= 1 / ||L^-1||_F^2 and
    // lambda_max <= trace(S).  Otherwise the eigendecomposition below runs.
    int fast = 0;
    double gr[kRegM];   // gamma of the register path (every lane)
    if (small) {
        // rows and columns l .. kRegM-1 become the identity, so the factor
        // and its inverse are block diagonal and the padding adds nothing
        double tr = 0.0;
#pragma unroll
        for (int i = 0; i < kRegM; ++i) {
#pragma unroll
            for (int j = 0; j <= i; ++j)
                R[i][j] = i < l ? R[i][j] : (i == j ? 1.0 : 0.0);
            cr[i] = i < l ? cr[i] : 0.0;
            tr += i < l ? R[i][i] : 0.0;
        }
        bool ok = true;
        double id[kRegM];   // 1 / L_jj
#pragma unroll
        for (int j = 0; j < kRegM; ++j) {
            const double piv = R[j][j];
            ok = ok && piv > 0.0;
            const double d = sqrt(piv);
            R[j][j] = d;
            id[j] = 1.0 / d;
#pragma unroll
            for (int i = j + 1; i < kRegM; ++i)
                R[i][j] *= id[j];
#pragma unroll
            for (int i = j + 1; i < kRegM; ++i)
#pragma unroll
                for (int kk = j + 1; kk <= i; ++kk)
                    R[i][kk] -= R[i][j] * R[kk][j];
        }
        // L^-1 column by column (forward substitution) and ||L^-1||_F^2
        double Lr[kRegM][kRegM];
        double fro = 0.0;
#pragma unroll
        for (int c = 0; c < kRegM; ++c)
#pragma unroll
            for (int i = c; i < kRegM; ++i) {
                double acc = i == c ? 1.0 : 0.0;
#pragma unroll
                for (int kk = c; kk < i; ++kk)
                    acc -= R[i][kk] * Lr[kk][c];
                Lr[i][c] = acc * id[i];
                fro += i < l ? Lr[i][c] * Lr[i][c] : 0.0;
            }
        fast = l > 0 && ok && (1.0 / fro > a.rcond * (double)l * tr) && fro == fro && !a.force_pinv;
        if (fast) {
            double y[kRegM];   // y = L^-1 c, gamma = L^-T y
#pragma unroll
            for (int i = 0; i < kRegM; ++i) {
                double v = 0.0;
#pragma unroll
                for (int kk = 0; kk <= i; ++kk)
                    v += Lr[i][kk] * cr[kk];
                y[i] = v;
            }
#pragma unroll
            for (int i = 0; i < kRegM; ++i) {
                double g = 0.0;
#pragma unroll
                for (int kk = i; kk < kRegM; ++kk)
                    g += Lr[kk][i] * y[kk];
                gr[i] = g;
            }
        } else {
            // the Jacobi path works on S and c in LDS
            for (int idx = tid; idx < l * l; idx += kLsqThreads) {
                const int i = idx / l, j = idx % l;
                S[i][j] = (i == cb || j == cb) ? 0.0 : gram_vals[i <= j ? tri_index(i, j, a.m) : tri_index(j, i, a.m)];
            }
            for (int i = tid; i < l; i += kLsqThreads)
                cvec[i] = i == cb ? 0.0 : gram_vals[np + i];
            __syncthreads();
        }
    } else if (l > 0 && !a.force_pinv) {
        fast = cholesky_proved_solve(l, a.rcond, (double)l, 1.0, S, V, Li, cvec, wvec, gam, sh_fail);
    }

    if (!fast)
        jacobi_pinv(l, a.rcond, (double)l, S, V, cvec, wvec, gam, rot_c, rot_s, pair_p, pair_q, sh_off, sh_stop);

    // ---- update plan ----
    // x_{k+1} = x_k + beta f_k - sum_i gamma_i (dX_i + beta dF_i), column i
    // covering iteration j_i = k - l + i:  dF_i = f_{j_i+1} - f_{j_i},
    // dX_i = omega f_{j_i} (Richardson j_i) or the stored increment (Anderson j_i).
    // Lane t writes the coefficient of history position t (t <= l).
    const bool regs = small && fast;
    const int t = tid;
    double gcur = 0.0, gprev = 0.0;
    if (regs) {
#pragma unroll
        for (int u = 0; u < kRegM; ++u) {
            gcur = u == t ? gr[u] : gcur;
            gprev = u + 1 == t ? gr[u] : gprev;
        }
    } else {
        gcur = t < l ? gam[t] : 0.0;
        gprev = t >= 1 && t <= l ? gam[t - 1] : 0.0;
    }
    // k + 1 is a multiple of p, so (j_0 + 1) mod p = (p - l) mod p, and an
    // Anderson column i (j_i + 1 a multiple of p) belongs to the cycle
    // (j_i + 1) / p - 1 = cycle0 - 1 + (p - l + i) / p, an exact division.
    const int pos0 = ((a.p - l) % a.p + a.p) % a.p;
    const int slot0 = (int)((k - l) % a.nslots);     // ring slot of column 0
    const int cyc0 = a.q > 0 ? (int)(cycle0 % a.q) : 0;
    const bool anderson = t < l && a.q > 0 && (pos0 + t) % a.p == 0;
    double al = (t == l ? a.beta : 0.0) - a.beta * (gprev - gcur);
    if (t < l && !anderson)
        al -= a.omega * gcur;
    const unsigned long long amask = __ballot(anderson);
    if (anderson) {
        const int nd = __popcll(amask & ((1ull << t) - 1ull));
        const int c = cyc0 - 1 + (a.p - l + t) / a.p;   // (cycle mod q) up to a multiple of q
        st->dslot[nd] = ((c % a.q) + a.q) % a.q;
        st->delta[nd] = -gcur;
    }
    if (t <= l) {
        st->alpha[t] = al;
        st->fslot[t] = (slot0 + t) % a.nslots;
    }
    if (tid == 0) {
        int rank = l;
        if (!fast) {
            rank = 0;
            for (int e = 0; e < l; ++e)
                rank += S[e][e] > sh_off;
        }
        st->rank = rank;
        if (a.rank_log && log_count0 < a.log_cap)
            a.rank_log[log_count0] = rank;
        st->nf = l + 1;
        st->nd = __popcll(amask);
        st->wslot = a.q > 0 ? cyc0 : -1;
        st->cycle = cycle0 + 1;
    }
}


}  // namespace aar
