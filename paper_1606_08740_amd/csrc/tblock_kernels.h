#pragma once
// Temporal blocking of the Richardson sweeps (Sec. 2: between two Anderson
// steps the iteration is p - 1 purely local Richardson steps, with no global
// reduction), on gfx950.
//
// With the residual recursion a Richardson step needs only the previous
// residual: f_{j+1} = f_j - omega D^-1 A f_j.  A temporal block runs NT such
// steps in one pass: it reads f_{j0-1} once, and writes f_{j0} .. f_{j0+NT-1}
// to their history slots (every one is a column of the history, Eqs. 4-5).
// Optionally its last stage is the Anderson step's residual (kFk: the norm
// partial of ||b - A x_k|| = ||D f_k|| for the convergence test).
//
// Layout: a workgroup of 64 x 4 threads owns a 64 x TY tile of each xy-plane
// and marches through `cz` planes along z.  Stage s (1..NT) computes its step
// on the tile grown by (NT - s) R on every side (the halo the later stages
// read), so stage NT produces the tile itself; neighbouring tiles recompute
// the same halo values (bit for bit the same arithmetic).  The stages are
// pipelined along z: at march step t the input plane L = z0 - NT R + t is
// loaded, and stage s computes plane L - s R.  Every stage keeps its output
// in an LDS ring of 2R + 1 planes over its region, from which the next stage
// reads all its x, y and z taps; stage 0's ring holds the input.  The LDS
// footprint is sum_s (2R + 1) |region_s| values, which confines the blocks to
// small radii (R <= 2) and a few stages; the driver picks NT (or none) per
// grid by timing.
//
// Per point the arithmetic is that of the one-point sweep pass with the
// recursion (same operand order), so a block's outputs equal those of NT
// single sweeps exactly.
#include "aar_device.h"

namespace aar {

constexpr int kTbMaxStages = kTbMaxDepth;

// LDS bytes of a block with NT stages (rings of stages 0 .. NT-1).
inline size_t tblock_lds_bytes(int R, int NT, int TY, size_t esize)
{
    size_t n = 0;
    for (int s = 0; s < NT; ++s) {
        const int g = (NT - s) * R;
        n += (size_t)(2 * R + 1) * (size_t)(kTX + 2 * g) * (size_t)(TY + 2 * g);
    }
    return n * esize;
}

template <typename T, int R, bool CONV, int TY>
__global__ __launch_bounds__(kThreads) void k_tblock(const StencilArgs<T> a, int NT, int last_fk)
{
    extern __shared__ __align__(16) unsigned char tb_smem[];
    constexpr bool kStd = sizeof(T) == 8;   // FP64: weighted-sum taps; FP32: difference form
    constexpr int Q = 2 * R + 1;
    T *ring = reinterpret_cast<T *>(tb_smem);
    __shared__ double red[kWY];

    const StencilDev<T> &st = a.st;
    const InstState *sp = a.state;
    if (sp->status != kRunning)
        return;
    const int64_t k0 = sp->cycle * a.p + a.j;   // position of stage 1's output
    const int64_t max_iter = sp->max_iter;
    if (k0 >= max_iter)
        return;

    const int tid = threadIdx.x + kTX * threadIdx.y;
    int lin = xcd_tile(blockIdx.x, gridDim.x);
    int bx, by, bz;
    if (a.order & kOrderZFast) {
        bz = lin % a.tiles_z;
        lin /= a.tiles_z;
        bx = lin % a.tiles_x;
        by = lin / a.tiles_x;
    } else {
        bx = lin % a.tiles_x;
        lin /= a.tiles_x;
        by = lin % a.tiles_y;
        bz = lin / a.tiles_y;
    }
    const int x0 = bx * kTX, y0 = by * TY;
    const int z0 = bz * a.cz;
    const int z1 = min(z0 + a.cz, st.n2);
    const int nz = z1 - z0;
    const int64_t plane = (int64_t)st.n0 * st.n1;
    const T *fin = reinterpret_cast<const T *>(a.fring) + (int64_t)((k0 - 1) % a.nslots) * a.slot_stride;

    // region of stage s: the tile grown by g_s = (NT - s) R; ring s at ring + off[s]
    int W[kTbMaxStages + 1], H[kTbMaxStages + 1], off[kTbMaxStages + 1];
    {
        int o = 0;
        for (int s = 0; s <= NT; ++s) {
            const int g = (NT - s) * R;
            W[s] = kTX + 2 * g;
            H[s] = TY + 2 * g;
            off[s] = o;
            o += Q * W[s] * H[s];
        }
    }
    // grid offset of an in-plane position (x, y) under the boundary rules;
    // -1 outside a zero Dirichlet boundary
    auto inplane = [&](int x, int y) -> int {
        if (x < 0 || x >= st.n0) {
            if (!st.per0)
                return -1;
            x = x % st.n0;
            x += x < 0 ? st.n0 : 0;
        }
        if (y < 0 || y >= st.n1) {
            if (!st.per1)
                return -1;
            y = y % st.n1;
            y += y < 0 ? st.n1 : 0;
        }
        return x + st.n0 * y;
    };
    auto zplane = [&](int z) -> int {
        if (z < 0 || z >= st.n2) {
            if (!st.per2)
                return -1;
            z = z % st.n2;
            z += z < 0 ? st.n2 : 0;
        }
        return z;
    };

    // stage 0: the input columns this thread loads (region 0), prefetched one
    // march step ahead
    constexpr int kMaxLoad = ((kTX + 2 * kTbMaxStages * R) * (TY + 2 * kTbMaxStages * R) + kThreads - 1) / kThreads;
    const int n_in = W[0] * H[0];
    const int nld = (n_in + kThreads - 1) / kThreads;
    int ldoff[kMaxLoad];
#pragma unroll
    for (int u = 0; u < kMaxLoad; ++u) {
        const int c = tid + u * kThreads;
        ldoff[u] = -1;
        if (u < nld && c < n_in)
            ldoff[u] = inplane(x0 - NT * R + c % W[0], y0 - NT * R + c / W[0]);
    }
    T pre[kMaxLoad];
    const int zbase = z0 - NT * R;   // plane of march step 0's load
    auto fetch = [&](int t) {
        const int zp = zplane(zbase + t);
#pragma unroll
        for (int u = 0; u < kMaxLoad; ++u)
            pre[u] = (u < nld && ldoff[u] >= 0 && zp >= 0) ? fin[ldoff[u] + plane * zp] : T(0);
    };

    const int tmax = nz - 1 + 2 * NT * R;
    double acc = 0.0;
    fetch(0);
    for (int t = 0; t <= tmax; ++t) {
        // stage 0: plane zbase + t into its ring slot t mod Q
        {
            T *r0 = ring + off[0] + (t % Q) * (W[0] * H[0]);
#pragma unroll
            for (int u = 0; u < kMaxLoad; ++u) {
                const int c = tid + u * kThreads;
                if (u < nld && c < n_in)
                    r0[c] = pre[u];
            }
        }
        if (t < tmax)
            fetch(t + 1);
        __syncthreads();
        for (int s = 1; s <= NT; ++s) {
            if (t < 2 * s * R)
                break;   // later stages start later (uniform)
            const int zc = zbase + t - s * R;          // this stage's plane
            const int zg = zplane(zc);
            const int64_t ks = k0 + s - 1;           // its iteration index
            const bool fk = last_fk && s == NT;
            const bool out_ok = zc >= z0 && zc < z1 && ks < max_iter;
            T *dst = s < NT ? ring + off[s] + ((t - s * R) % Q) * (W[s] * H[s]) : nullptr;
            const T *src = ring + off[s - 1];
            const int Ws = W[s - 1];
            const int psz = Ws * H[s - 1];
            // every ring keeps plane zbase + tau in slot tau mod Q; this
            // stage's plane zc is tau = t - s R (>= (s - 1) R + R here)
            const int tin = t - s * R;
            T *fout = reinterpret_cast<T *>(a.fring) + (int64_t)(ks % a.nslots) * a.slot_stride;
            const int gs = (NT - s) * R;
            // the whole region inside the grid: no boundary rule to apply
            const bool inside = x0 - gs >= 0 && x0 + kTX + gs <= st.n0 && y0 - gs >= 0 && y0 + TY + gs <= st.n1;
            const int nout = W[s] * H[s];
            for (int c = tid; c < nout; c += kThreads) {
                const int ex = c % W[s], ey = c / W[s];
                const int gx = x0 - gs + ex, gy = y0 - gs + ey;
                const int io = inside ? gx + st.n0 * gy : inplane(gx, gy);
                T f = T(0);
                if (io >= 0 && zg >= 0) {
                    const int lx = ex + R, ly = ey + R;      // position in region s - 1
                    auto at = [&](int d, int dx, int dy) -> T {
                        return src[((tin + d) % Q) * psz + (ly + dy) * Ws + (lx + dx)];
                    };
                    const T cv = at(0, 0, 0);
                    T ax, dg = st.jdiag;
                    if constexpr (kStd) {
                        ax = st.diag * cv;
#pragma unroll
                        for (int sh = 1; sh <= R; ++sh) {
                            ax += st.c0[sh] * (at(0, sh, 0) + at(0, -sh, 0));
                            ax += st.c1[sh] * (at(0, 0, sh) + at(0, 0, -sh));
                            ax += st.c2[sh] * (at(sh, 0, 0) + at(-sh, 0, 0));
                        }
                    } else {
                        ax = st.sigma * cv;
#pragma unroll
                        for (int sh = 1; sh <= R; ++sh) {
                            ax += st.c0[sh] * ((at(0, sh, 0) - cv) + (at(0, -sh, 0) - cv));
                            ax += st.c1[sh] * ((at(0, 0, sh) - cv) + (at(0, 0, -sh) - cv));
                            ax += st.c2[sh] * ((at(sh, 0, 0) - cv) + (at(-sh, 0, 0) - cv));
                        }
                    }
                    if constexpr (CONV) {
                        const int64_t id = io + plane * zg;
                        const T v0 = st.vel[id], v1 = st.vel[st.N + id], v2 = st.vel[2 * st.N + id];
                        ax += v0 > T(0) ? -v0 * st.ih0 * (at(0, -1, 0) - cv) : v0 * st.ih0 * (at(0, 1, 0) - cv);
                        ax += v1 > T(0) ? -v1 * st.ih1 * (at(0, 0, -1) - cv) : v1 * st.ih1 * (at(0, 0, 1) - cv);
                        ax += v2 > T(0) ? -v2 * st.ih2 * (at(-1, 0, 0) - cv) : v2 * st.ih2 * (at(1, 0, 0) - cv);
                        dg += fabs(v0) * st.ih0 + fabs(v1) * st.ih1 + fabs(v2) * st.ih2;
                    }
                    f = cv - a.omega * (CONV ? ax / dg : ax * st.inv_diag);
                    // own points: inside the tile, written to the history slot
                    const int tx = gx - x0, ty = gy - y0;
                    if (out_ok && tx >= 0 && tx < kTX && ty >= 0 && ty < TY && gx < st.n0 && gy < st.n1) {
                        fout[io + plane * zg] = f;
                        if (fk) {
                            const T res = dg * f;
                            acc += (double)res * (double)res;
                        }
                    }
                }
                if (dst)
                    dst[c] = f;
            }
            __syncthreads();
        }
    }
    if (last_fk) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
            acc += __shfl_down(acc, o, 64);
        if (threadIdx.x == 0)
            red[threadIdx.y] = acc;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < kWY; ++w)
                sum += red[w];
            a.partial[blockIdx.x] = sum;
        }
    }
}

}  // namespace aar
