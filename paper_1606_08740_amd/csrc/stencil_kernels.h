#pragma once
// Stencil passes of the AAR iteration on gfx950: kernels and launch templates.
// The launch entry points are compiled in three units by iterate and history
// precision (stencil.hip: FP64 iterate with FP64 history, the grid helper and
// the FP64 residual and apply passes; stencil_narrow.hip: FP64 iterate with an
// FP32 or bfloat16 history; stencil_f32.hip: FP32 iterate).
//
// One kernel template covers the four passes that apply the operator:
//   kSweep  the Richardson iteration of Eq. 3 (first case) fused with the
//           Jacobi-preconditioned residual of Eq. 6 and the history write:
//           f_j = D^{-1}(b - A x_j), x_{j+1} = x_j + omega f_j, ring <- f_j;
//   kFk     the residual of an Anderson step: ring <- f_k, and the partial
//           sums of ||b - A x_k||^2 for the convergence test (Sec. 2);
//   kResid  r = b - A x and ||r||^2 (FP64 iterative refinement);
//   kApply  y = A x.
//
// The operator is A u = -a Lap_h u + v . grad_h u + sigma u with order-2r
// central differences per axis, written in difference form
//   sum_s c_s [(u_{i+s} - u_i) + (u_{i-s} - u_i)],  c_s = -a w_s / h^2,
// which equals the usual weighted sum because w_0 = -2 sum_s w_s, and keeps
// A 1 = sigma 1 exact in FP32 (the near-null constant mode of the shifted
// periodic problems).  Upwind convection (radius 1): v (u_i - u_{i-1}) / h for
// v > 0, else v (u_{i+1} - u_i) / h.
//
// Tiling (2.5D): a workgroup of 64 x 4 threads owns a 64 x (4 RY) tile of one
// xy-plane and marches through `cz` planes along z.  Each thread keeps its
// column's 2r+1 z-values in registers (a queue advanced once per plane), and
// the current plane plus an r-wide halo sits in LDS for the x and y taps (two
// plane buffers used in turn, so each plane step needs one barrier).  So
// every interior value is fetched from global memory once per pass; halos
// are re-fetched from L2.  The loads of the next plane steps are in flight
// while plane z is computed, so memory latency overlaps the taps.  Tiles are
// assigned so that each XCD works on a contiguous block of tiles (shared
// halos stay in its L2); optionally the block runs along z and odd z chunks
// march downwards, so neighbouring chunks read their shared boundary planes
// at the same moment.  FP64 hot passes use the weighted-sum form of the taps
// (half the flops of the difference form).  The paired layout (stencil_tile2)
// is described at its definition.
#include "aar_device.h"
#include "anderson_core.h"

namespace aar {

__device__ inline int wrap_index(int g, int n)
{
    g %= n;
    return g < 0 ? g + n : g;
}

template <typename T> __device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// One tile (64 x 4 RY columns, planes [bz*cz, bz*cz + cz)) of a stencil pass.
// `lin` is the tile's linear index (x fastest, then y, then z chunk); the
// reduction partial (kFk, kResid) goes to *partial_out.
template <typename T, typename H, int R, bool CONV, int MODE, int RY>
__device__ __forceinline__ void stencil_tile(const StencilArgs<T> &a, int lin, double *partial_out)
{
    // FP64 hot passes use the weighted-sum form (half the flops); FP32 passes
    // and the FP64 refinement residual keep the difference form.
    constexpr bool kStd = (std::is_same<T, double>::value || std::is_same<T, zd>::value) && MODE != kResid;
    constexpr int TY = kWY * RY;
    constexpr int LX = kTX + 2 * R;
    constexpr int LY = TY + 2 * R;
    constexpr int kHaloRows = 2 * R * LX;
    constexpr int kHalo = kHaloRows + TY * 2 * R;
    constexpr int NH = (kHalo + kThreads - 1) / kThreads;
    // two plane buffers: step i writes buffer i & 1 (see the step below)
    __shared__ T sh[2][LY][LX];
    __shared__ double red[kWY];

    const StencilDev<T> &st = a.st;
    int64_t k = 0;
    if constexpr (MODE == kSweep || MODE == kFk) {
        const InstState *s = a.state;
        if (s->status != kRunning)
            return;
        k = s->cycle * a.p + a.j;
        if (k >= s->max_iter)
            return;
    }

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = tx + kTX * ty;
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
    // march direction along z: the queue slot d holds plane z + dir (d - R)
    const int dir = ((a.order & kOrderAltZ) && (bz & 1)) ? -1 : 1;
    const int zs = dir > 0 ? z0 : z1 - 1;
    const int nz = z1 - z0;
    const int gx = x0 + tx;
    const int64_t plane = (int64_t)st.n0 * st.n1;

    H *fout = nullptr;
    if constexpr (MODE == kSweep || MODE == kFk)
        fout = reinterpret_cast<H *>(a.fring) + (int64_t)(k % a.nslots) * a.slot_stride;
    // the stencil's input: x, or f_{k-1} from the ring for the recursion
    bool recur = false;
    const T *xin = a.x;
    if constexpr (std::is_same<T, H>::value && (MODE == kSweep || MODE == kFk)) {
        recur = a.recur != 0;
        if (recur)
            xin = reinterpret_cast<const T *>(a.fring) + (int64_t)((k - 1) % a.nslots) * a.slot_stride;
    }

    // In-plane offsets (boundary rule applied; -1: outside a Dirichlet
    // boundary, value 0) of this thread's columns and of its halo cells.
    int coff[RY];
    bool own[RY];
#pragma unroll
    for (int ry = 0; ry < RY; ++ry) {
        int cx = gx, cy = y0 + ty + ry * kWY;
        own[ry] = cx < st.n0 && cy < st.n1;
        bool in = true;
        if (cx >= st.n0) {
            if (st.per0)
                cx = wrap_index(cx, st.n0);
            else
                in = false;
        }
        if (cy >= st.n1) {
            if (st.per1)
                cy = wrap_index(cy, st.n1);
            else
                in = false;
        }
        coff[ry] = in ? cx + st.n0 * cy : -1;
    }
    int hoff[NH], hlds[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        const int h = tid + j * kThreads;
        hoff[j] = -1;
        hlds[j] = -1;
        if (h < kHalo) {
            int ly, lx;
            if (h < kHaloRows) {
                const int r = h / LX;
                lx = h - r * LX;
                ly = r < R ? r : r + TY;
            } else {
                const int t = h - kHaloRows;
                const int c = t % (2 * R);
                ly = R + t / (2 * R);
                lx = c < R ? c : c + kTX;
            }
            hlds[j] = ly * LX + lx;
            int cx = x0 + lx - R, cy = y0 + ly - R;
            bool in = true;
            if (cx < 0 || cx >= st.n0) {
                if (st.per0)
                    cx = wrap_index(cx, st.n0);
                else
                    in = false;
            }
            if (cy < 0 || cy >= st.n1) {
                if (st.per1)
                    cy = wrap_index(cy, st.n1);
                else
                    in = false;
            }
            hoff[j] = in ? cx + st.n0 * cy : -1;
        }
    }
    // plane index under the z boundary rule (-1: zero plane)
    auto zplane = [&](int z) -> int {
        if (z < 0 || z >= st.n2)
            return st.per2 ? wrap_index(z, st.n2) : -1;
        return z;
    };
    auto ld = [&](int off, int zp) -> T { return (off >= 0 && zp >= 0) ? xin[off + plane * zp] : T(0); };

    // z-queue: q[ry][d] = x at plane z + dir (d - R) of this thread's column
    T q[RY][2 * R + 1];
#pragma unroll
    for (int ry = 0; ry < RY; ++ry)
#pragma unroll
        for (int d = 0; d < 2 * R; ++d)
            q[ry][d] = ld(coff[ry], zplane(zs + dir * (d - R)));

    // Values of the planes ahead (queue front, halo, b, velocity), fetched
    // kDepth plane steps before they are used, in kDepth register buffers:
    // a workgroup keeps kDepth planes of loads in flight while it computes
    // (one buffer for the register-heavy FP64 4-row tile, which would
    // otherwise lose half its occupancy)
    constexpr int kDepth = sizeof(T) * RY >= 32 ? 1 : 2;
    T front[kDepth][RY], hv[kDepth][NH], bv[kDepth][RY], vv[kDepth][CONV ? 3 * RY : 1];
    // loads for plane step i: queue front (plane z + dir R), halo, b and
    // velocity of plane z
    auto fetch = [&](auto buf, int i) {
        constexpr int u = decltype(buf)::value;
        const int z = zs + dir * i;
        const int zf = zplane(z + dir * R);
#pragma unroll
        for (int ry = 0; ry < RY; ++ry)
            front[u][ry] = ld(coff[ry], zf);
#pragma unroll
        for (int j = 0; j < NH; ++j)
            hv[u][j] = ld(hoff[j], z);
        if constexpr (MODE != kApply) {
#pragma unroll
            for (int ry = 0; ry < RY; ++ry)
                bv[u][ry] = own[ry] && !recur ? a.b[coff[ry] + plane * z] : T(0);
        }
        if constexpr (CONV) {
#pragma unroll
            for (int ry = 0; ry < RY; ++ry)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    vv[u][3 * ry + c] = own[ry] ? st.vel[c * st.N + coff[ry] + plane * z] : T(0);
        }
    };

    double acc = 0.0;
    // plane step i (plane z = zs + dir i) from register buffer `buf`
    auto step = [&](auto buf, int i) {
        constexpr int u = decltype(buf)::value;
        const int z = zs + dir * i;
#pragma unroll
        for (int ry = 0; ry < RY; ++ry)
            q[ry][2 * R] = front[u][ry];
        // Plane i goes to LDS buffer i & 1.  Its last readers were the taps
        // of step i - 2, which every thread finished before the barrier of
        // step i - 1, so one barrier per step suffices.
        // (with two register sets, steps of set u have i & 1 == u)
        T(&sp)[LY][LX] = sh[kDepth == 2 ? u : (i & 1)];
#pragma unroll
        for (int ry = 0; ry < RY; ++ry)
            sp[R + ty + ry * kWY][R + tx] = q[ry][R];
#pragma unroll
        for (int j = 0; j < NH; ++j)
            if (hlds[j] >= 0)
                (&sp[0][0])[hlds[j]] = hv[u][j];
        __syncthreads();
        T bcur[RY], vcur[CONV ? 3 * RY : 1];
#pragma unroll
        for (int ry = 0; ry < RY; ++ry)
            bcur[ry] = bv[u][ry];
        if constexpr (CONV) {
#pragma unroll
            for (int c = 0; c < 3 * RY; ++c)
                vcur[c] = vv[u][c];
        }
        if (i + kDepth < nz)
            fetch(buf, i + kDepth);

#pragma unroll
        for (int ry = 0; ry < RY; ++ry) {
            const int lx = R + tx, ly = R + ty + ry * kWY;
            const T c = q[ry][R];
            T ax;
            if constexpr (kStd) {
                ax = st.diag * c;
#pragma unroll
                for (int s = 1; s <= R; ++s) {
                    ax += st.c0[s] * (sp[ly][lx + s] + sp[ly][lx - s]);
                    ax += st.c1[s] * (sp[ly + s][lx] + sp[ly - s][lx]);
                    ax += st.c2[s] * (q[ry][R + s] + q[ry][R - s]);
                }
            } else {
                ax = st.sigma * c;
#pragma unroll
                for (int s = 1; s <= R; ++s) {
                    ax += st.c0[s] * ((sp[ly][lx + s] - c) + (sp[ly][lx - s] - c));
                    ax += st.c1[s] * ((sp[ly + s][lx] - c) + (sp[ly - s][lx] - c));
                    ax += st.c2[s] * ((q[ry][R + s] - c) + (q[ry][R - s] - c));
                }
            }
            if (!own[ry])
                continue;
            const int64_t id = coff[ry] + plane * z;
            T dg = st.jdiag;
            if constexpr (CONV) {
                const T v0 = vcur[3 * ry], v1 = vcur[3 * ry + 1], v2 = vcur[3 * ry + 2];
                ax += v0 > T(0) ? -v0 * st.ih0 * (sp[ly][lx - 1] - c) : v0 * st.ih0 * (sp[ly][lx + 1] - c);
                ax += v1 > T(0) ? -v1 * st.ih1 * (sp[ly - 1][lx] - c) : v1 * st.ih1 * (sp[ly + 1][lx] - c);
                const T zm = dir > 0 ? q[ry][R - 1] : q[ry][R + 1];   // plane z - 1
                const T zp = dir > 0 ? q[ry][R + 1] : q[ry][R - 1];   // plane z + 1
                ax += v2 > T(0) ? -v2 * st.ih2 * (zm - c) : v2 * st.ih2 * (zp - c);
                dg += fabs(v0) * st.ih0 + fabs(v1) * st.ih1 + fabs(v2) * st.ih2;
            }
            if constexpr (MODE == kApply) {
                a.out[id] = ax;
            } else if constexpr (MODE == kResid) {
                const T res = bcur[ry] - ax;
                a.out[id] = res;
                acc += sqnorm(res);
            } else {
                T f, res;
                if (recur) {
                    // f_k = f_{k-1} - omega D^-1 A f_{k-1}; b - A x_k = D f_k
                    f = c - a.omega * (CONV ? ax / dg : ax * st.inv_diag);
                    res = dg * f;
                } else {
                    res = bcur[ry] - ax;
                    f = CONV ? res / dg : res * st.inv_diag;
                }
                Hist<H>::store(fout, id, f);
                if constexpr (MODE == kSweep) {
                    if (a.out)
                        a.out[id] = c + a.omega * f;
                } else {
                    if (a.fcur)
                        a.fcur[id] = f;
                    acc += sqnorm(res);
                }
            }
        }

#pragma unroll
        for (int ry = 0; ry < RY; ++ry)
#pragma unroll
            for (int d = 0; d < 2 * R; ++d)
                q[ry][d] = q[ry][d + 1];
    };

    using B0 = std::integral_constant<int, 0>;
    using B1 = std::integral_constant<int, kDepth - 1>;
    if (nz > 0)
        fetch(B0{}, 0);
    if constexpr (kDepth == 1) {
        for (int i = 0; i < nz; ++i)
            step(B0{}, i);
    } else {
        if (nz > 1)
            fetch(B1{}, 1);
        for (int i = 0; i < nz; i += 2) {
            step(B0{}, i);
            if (i + 1 < nz)
                step(B1{}, i + 1);
        }
    }

    if constexpr (MODE == kFk || MODE == kResid) {
        acc = wave_sum(acc);
        if (tx == 0)
            red[ty] = acc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < kWY; ++w)
                s += red[w];
            *partial_out = s;
        }
    }
}

template <typename T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };

// Paired layout of the Richardson sweep and the Anderson-step residual
// (MODE kSweep or kFk, no convection, even n0, 16-byte aligned vectors).
// The 64 NW threads (NW = 4, 8 or 16 waves) form 32 lanes along x by 2 NW
// lane rows; a thread owns the two x-adjacent points (gx, gx + 1) in RY
// contiguous rows, so the tile is 64 x 2 NW RY.  Global loads and stores move
// both points as one vector, and the
// taps read pairs from LDS: for x the 2R + 2 values around the pair, for y a
// column pair per row, shared by the RY rows.  This halves the LDS requests
// per point of the one-point layout.  The z taps come from a register queue
// per point, as there.
// GM > 0 (MODE kFk only): the pass also forms the Gram products of the
// extrapolation step (Eqs. 4-5) for history length GM at its own points:
// the GM preceding ring slots are read beside f_k, and per-workgroup partials
// of the GM(GM+1)/2 + GM entries go to a.gram_partial (entry-major), which
// the one-wave solve kernel sums.
template <typename T, typename H, int R, int MODE, int RY, int NW, int GM = 0>
__device__ __forceinline__ void stencil_tile2(const StencilArgs<T> &a, int lin, double *partial_out)
{
    using V = typename Pair<T>::type;
    constexpr int kThr = 64 * NW;            // NW waves: 2 NW lane rows of 32
    constexpr int TY = 2 * NW * RY;
    constexpr int RP = R + (R & 1);          // x halo width rounded to even (LDS pair alignment)
    constexpr int LX = kTX + 2 * RP;
    constexpr int LY = TY + 2 * R;
    constexpr int kHaloRows = 2 * R * (kTX + 2 * R);
    constexpr int kHalo = kHaloRows + TY * 2 * R;
    constexpr int NH = (kHalo + kThr - 1) / kThr;
    constexpr int Q = 2 * R + 1;
    // two plane buffers: step i writes buffer i & 1 (see the z loop)
    __shared__ __align__(16) T sh[2][LY][LX];
    __shared__ double red[NW];
    constexpr int GNE = GM > 0 ? GM * (GM + 1) / 2 + GM : 1;
    __shared__ double gred[GM > 0 ? NW : 1][GNE];

    const StencilDev<T> &st = a.st;
    const InstState *s = a.state;
    if (s->status != kRunning)
        return;
    const int64_t k = s->cycle * a.p + a.j;
    if (k >= s->max_iter)
        return;
    // fused Gram: ring slots of history positions 0 .. l-1 (f_k is position l)
    double gacc[GNE];
    const H *gslot[GM > 0 ? GM : 1];
    int gl = 0;
    if constexpr (GM > 0) {
        gl = (int)(k < GM ? k : GM);
#pragma unroll
        for (int e = 0; e < GNE; ++e)
            gacc[e] = 0.0;
#pragma unroll
        for (int t = 0; t < GM; ++t)
            gslot[t] = reinterpret_cast<const H *>(a.fring) +
                       (int64_t)((k - gl + t + a.nslots) % a.nslots) * a.slot_stride;
    }

    const int tid = threadIdx.x + kTX * threadIdx.y;
    const int lx2 = tid % 32, lr = tid / 32;
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
    const int dir = ((a.order & kOrderAltZ) && (bz & 1)) ? -1 : 1;
    const int zs = dir > 0 ? z0 : z1 - 1;
    const int nz = z1 - z0;
    const int64_t plane = (int64_t)st.n0 * st.n1;
    H *fout = reinterpret_cast<H *>(a.fring) + (int64_t)(k % a.nslots) * a.slot_stride;
    // the stencil's input: x, or f_{k-1} from the ring for the recursion
    bool recur = false;
    const T *xin = a.x;
    if constexpr (std::is_same<T, H>::value) {
        recur = a.recur != 0;
        if (recur)
            xin = reinterpret_cast<const T *>(a.fring) + (int64_t)((k - 1) % a.nslots) * a.slot_stride;
    }

    // offset of this thread's pair in each of its rows (-1: outside a
    // Dirichlet boundary).  n0 is even, so a pair is never split by the
    // grid edge or a periodic wrap.
    const int gx = x0 + 2 * lx2;
    int coff[RY];
    bool own[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        int cx = gx, cy = y0 + lr * RY + r;
        own[r] = cx < st.n0 && cy < st.n1;
        bool in = true;
        if (cx >= st.n0) {
            if (st.per0)
                cx = wrap_index(cx, st.n0);
            else
                in = false;
        }
        if (cy >= st.n1) {
            if (st.per1)
                cy = wrap_index(cy, st.n1);
            else
                in = false;
        }
        coff[r] = in ? cx + st.n0 * cy : -1;
    }
    // halo cells: rows above and below (full width with x halo), then the
    // x halo of the tile rows; LDS column = x - x0 + RP
    int hoff[NH], hlds[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        const int h = tid + j * kThr;
        hoff[j] = -1;
        hlds[j] = -1;
        if (h < kHalo) {
            int ly, lx;          // lx: 0 .. kTX + 2R - 1, the column relative to x0 - R
            if (h < kHaloRows) {
                const int r = h / (kTX + 2 * R);
                lx = h - r * (kTX + 2 * R);
                ly = r < R ? r : r + TY;
            } else {
                const int t = h - kHaloRows;
                const int c = t % (2 * R);
                ly = R + t / (2 * R);
                lx = c < R ? c : c + kTX;
            }
            hlds[j] = ly * LX + lx + (RP - R);
            int cx = x0 + lx - R, cy = y0 + ly - R;
            bool in = true;
            if (cx < 0 || cx >= st.n0) {
                if (st.per0)
                    cx = wrap_index(cx, st.n0);
                else
                    in = false;
            }
            if (cy < 0 || cy >= st.n1) {
                if (st.per1)
                    cy = wrap_index(cy, st.n1);
                else
                    in = false;
            }
            hoff[j] = in ? cx + st.n0 * cy : -1;
        }
    }
    auto zplane = [&](int z) -> int {
        if (z < 0 || z >= st.n2)
            return st.per2 ? wrap_index(z, st.n2) : -1;
        return z;
    };
    auto ld2 = [&](int off, int zp) -> V {
        if (off >= 0 && zp >= 0)
            return *reinterpret_cast<const V *>(xin + off + plane * zp);
        V v;
        v.x = T(0);
        v.y = T(0);
        return v;
    };

    // q[r][e][d]: point (gx + e, row r) at plane z + dir (d - R)
    T q[RY][2][Q];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int d = 0; d < 2 * R; ++d) {
            const V v = ld2(coff[r], zplane(zs + dir * (d - R)));
            q[r][0][d] = v.x;
            q[r][1][d] = v.y;
        }

    // Loads of plane i (front plane of the z queue, halo cells, b) are issued
    // ahead of its step, into register set i mod NB.  With an FP64 iterate and
    // ring NB = 2: they go two plane steps ahead, so each has two steps of taps
    // to arrive (the z loop is unrolled by two so that both sets keep fixed
    // registers).  So do the FP32 sweeps over an FP32 ring (the recursion
    // steps of the FP32-ring and mixed modes), whose registers leave room for
    // it; the other narrower passes, which rely on more resident workgroups
    // instead, go one step ahead into one set.
    constexpr int NB = (sizeof(T) == 8 && sizeof(H) == 8) ||
                               (sizeof(H) == 4 && GM == 0 && (MODE == kSweep || MODE == kFk))
                           ? 2
                           : 1;
    V front[NB][RY], bv[NB][RY];
    T hv[NB][NH];
    auto fetch = [&](int i, int u) {
        const int z = zs + dir * i;
        const int zf = zplane(z + dir * R);
#pragma unroll
        for (int r = 0; r < RY; ++r)
            front[u][r] = ld2(coff[r], zf);
#pragma unroll
        for (int j = 0; j < NH; ++j)
            hv[u][j] = hoff[j] >= 0 ? xin[hoff[j] + plane * z] : T(0);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (own[r] && !recur) {
                bv[u][r] = *reinterpret_cast<const V *>(a.b + coff[r] + plane * z);
            } else {
                bv[u][r].x = T(0);
                bv[u][r].y = T(0);
            }
        }
    };
#pragma unroll
    for (int u = 0; u < NB; ++u)
        if (u < nz)
            fetch(u, u);

    double acc = 0.0;
    for (int i0 = 0; i0 < nz; i0 += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int i = i0 + u;
        if (NB > 1 && i >= nz)
            break;
        const int z = zs + dir * i;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            q[r][0][2 * R] = front[u][r].x;
            q[r][1][2 * R] = front[u][r].y;
        }
        V bcur[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r)
            bcur[r] = bv[u][r];
        // Plane i goes to LDS buffer i & 1.  Its last readers were the taps
        // of step i - 2, which every thread finished before the barrier of
        // step i - 1, so one barrier per step suffices.
        // (with an even number of register sets, i & 1 == u & 1)
        const int bi = NB % 2 == 0 ? (u & 1) : (i & 1);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            V c;
            c.x = q[r][0][R];
            c.y = q[r][1][R];
            *reinterpret_cast<V *>(&sh[bi][R + lr * RY + r][RP + 2 * lx2]) = c;
        }
#pragma unroll
        for (int j = 0; j < NH; ++j)
            if (hlds[j] >= 0)
                (&sh[bi][0][0])[hlds[j]] = hv[u][j];
        __syncthreads();
        if (i + NB < nz)
            fetch(i + NB, u);   // set u's plane is in the queue, LDS and bcur now

        T ax[RY][2];
        // x taps: the 2 RP + 2 values from column 2 lx2 hold x - RP .. x + 1 + RP
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int ly = R + lr * RY + r;
            T v[2 * RP + 2];
#pragma unroll
            for (int t = 0; t <= RP; ++t) {
                const V w = *reinterpret_cast<const V *>(&sh[bi][ly][2 * lx2 + 2 * t]);
                v[2 * t] = w.x;
                v[2 * t + 1] = w.y;
            }
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const T c = q[r][e][R];
                T acc_x;
                if constexpr (sizeof(T) == 8) {
                    acc_x = st.diag * c;
#pragma unroll
                    for (int sft = 1; sft <= R; ++sft)
                        acc_x += st.c0[sft] * (v[RP + e + sft] + v[RP + e - sft]);
                } else {
                    acc_x = st.sigma * c;
#pragma unroll
                    for (int sft = 1; sft <= R; ++sft)
                        acc_x += st.c0[sft] * ((v[RP + e + sft] - c) + (v[RP + e - sft] - c));
                }
                ax[r][e] = acc_x;
            }
        }
        // y taps: column pairs of rows lr RY - R + R .. , own rows from the queue
        {
            V col[RY + 2 * R];
#pragma unroll
            for (int t = 0; t < RY + 2 * R; ++t) {
                if (t >= R && t < R + RY) {
                    col[t].x = q[t - R][0][R];
                    col[t].y = q[t - R][1][R];
                } else {
                    col[t] = *reinterpret_cast<const V *>(&sh[bi][lr * RY + t][RP + 2 * lx2]);
                }
            }
#pragma unroll
            for (int r = 0; r < RY; ++r)
#pragma unroll
                for (int sft = 1; sft <= R; ++sft) {
                    if constexpr (sizeof(T) == 8) {
                        ax[r][0] += st.c1[sft] * (col[R + r + sft].x + col[R + r - sft].x);
                        ax[r][1] += st.c1[sft] * (col[R + r + sft].y + col[R + r - sft].y);
                    } else {
                        const T c0 = q[r][0][R], c1 = q[r][1][R];
                        ax[r][0] += st.c1[sft] * ((col[R + r + sft].x - c0) + (col[R + r - sft].x - c0));
                        ax[r][1] += st.c1[sft] * ((col[R + r + sft].y - c1) + (col[R + r - sft].y - c1));
                    }
                }
        }
        // z taps and outputs
#pragma unroll
        for (int r = 0; r < RY; ++r) {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const T c = q[r][e][R];
#pragma unroll
                for (int sft = 1; sft <= R; ++sft) {
                    if constexpr (sizeof(T) == 8)
                        ax[r][e] += st.c2[sft] * (q[r][e][R + sft] + q[r][e][R - sft]);
                    else
                        ax[r][e] += st.c2[sft] * ((q[r][e][R + sft] - c) + (q[r][e][R - sft] - c));
                }
            }
            if (!own[r])
                continue;
            const int64_t id = coff[r] + plane * z;
            T r0, r1, f0, f1;
            if (recur) {
                // f_k = f_{k-1} - omega D^-1 A f_{k-1}; b - A x_k = D f_k
                f0 = q[r][0][R] - a.omega * (st.inv_diag * ax[r][0]);
                f1 = q[r][1][R] - a.omega * (st.inv_diag * ax[r][1]);
                r0 = st.jdiag * f0;
                r1 = st.jdiag * f1;
            } else {
                r0 = bcur[r].x - ax[r][0];
                r1 = bcur[r].y - ax[r][1];
                f0 = r0 * st.inv_diag;
                f1 = r1 * st.inv_diag;
            }
            Hist<H>::store2(fout, id, f0, f1);
            if constexpr (MODE == kSweep) {
                if (a.out) {
                    V o;
                    o.x = q[r][0][R] + a.omega * f0;
                    o.y = q[r][1][R] + a.omega * f1;
                    *reinterpret_cast<V *>(a.out + id) = o;
                }
            } else {
                if (a.fcur) {
                    V o;
                    o.x = f0;
                    o.y = f1;
                    *reinterpret_cast<V *>(a.fcur + id) = o;
                }
                acc += (double)r0 * (double)r0 + (double)r1 * (double)r1;
                if constexpr (GM > 0) {
                    // the Gram pass sees f_k as stored in the ring (history
                    // precision); positions t >= l hold f_k itself, so their
                    // differences are exactly zero and the products take the
                    // fixed layout of a full history
                    H hk[2];
                    Hist<H>::store(hk, 0, f0);
                    Hist<H>::store(hk, 1, f1);
                    Pack<H, 2> sv[GM];
#pragma unroll
                    for (int t = 0; t < GM; ++t)
                        if (t < gl)
                            sv[t] = *reinterpret_cast<const Pack<H, 2> *>(gslot[t] + id);
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const double fe = (double)Hist<H>::load(hk, e);
                        double col[GM + 1];
#pragma unroll
                        for (int t = 0; t < GM; ++t)
                            col[t] = t < gl ? (double)Hist<H>::load(sv[t].v, e) : fe;
                        col[GM] = fe;
                        gram_point<GM>(col, GM, gacc);
                    }
                }
            }
        }

#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int e = 0; e < 2; ++e)
#pragma unroll
                for (int d = 0; d < 2 * R; ++d)
                    q[r][e][d] = q[r][e][d + 1];
    }
    }

    if constexpr (MODE == kFk) {
        acc = wave_sum(acc);
        if ((tid & 63) == 0)
            red[tid >> 6] = acc;
        if constexpr (GM > 0)
            wave_sums_to<GNE>(gacc, gred[tid >> 6]);   // gred[w][e]: wave w's total of entry e
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < NW; ++w)
                sum += red[w];
            *partial_out = sum;
        }
        if constexpr (GM > 0) {
            for (int e = tid; e < GNE; e += kThr) {
                double v = 0.0;
                for (int w = 0; w < NW; ++w)
                    v += gred[w][e];
                a.gram_partial[(int64_t)e * gridDim.x + blockIdx.x] = v;
            }
        }
    }
}

template <typename T, typename H, int R, int MODE, int RY, int NW, int GM>
__global__ __launch_bounds__(64 * NW) void k_stencil2(const StencilArgs<T> a)
{
    stencil_tile2<T, H, R, MODE, RY, NW, GM>(a, xcd_tile(blockIdx.x, gridDim.x), a.partial + blockIdx.x);
}

template <typename T, typename H, int R, bool CONV, int MODE, int RY>
__global__ __launch_bounds__(kThreads) void k_stencil(const StencilArgs<T> a)
{
    stencil_tile<T, H, R, CONV, MODE, RY>(a, xcd_tile(blockIdx.x, gridDim.x), a.partial + blockIdx.x);
}

// Batched form: work item w = (system, tile) of the active list; the system's
// operator, vectors and run state come from its descriptor.  Blocks stride
// over the list (its length is read on the device).
template <typename T, typename H, int R, bool CONV, int MODE, int RY>
__global__ __launch_bounds__(kThreads) void k_stencil_batched(const BatchStencilArgs<T> ba)
{
    const int nitems = *ba.nitems;
    for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
        const int2 it = ba.items[w];
        const BatchDesc<T> &d = ba.desc[it.x];
        StencilArgs<T> a;
        a.st = d.st;
        a.x = ba.x + d.off;
        a.b = ba.b + d.off;
        a.out = ba.out ? ba.out + d.off : nullptr;
        a.fring = (void *)((H *)ba.fring + d.off);
        a.fcur = ba.fcur ? ba.fcur + d.off : nullptr;
        a.partial = nullptr;
        a.state = ba.state + it.x;
        a.slot_stride = ba.slot_stride;
        a.j = ba.j;
        a.p = ba.p;
        a.nslots = ba.nslots;
        a.cz = d.cz;
        a.tiles_x = d.tiles_x;
        a.tiles_y = d.tiles_y;
        a.tiles_z = d.tiles_z;
        a.order = 0;
        a.omega = ba.omega;
        a.gram_partial = nullptr;
        a.recur = ba.recur;
        if constexpr (MODE == kResid) {
            if (!ba.mask || ba.mask[it.x] == 0)
                continue;
        }
        stencil_tile<T, H, R, CONV, MODE, RY>(a, it.y, ba.partial ? ba.partial + w : nullptr);
        __syncthreads();   // LDS is reused by the next item
    }
}

template <typename T, typename H, int MODE>
static hipError_t launch_batched_radius(int radius, bool conv, int ry, const BatchStencilArgs<T> &a, int grid,
                                        hipStream_t s)
{
#define AAR_BATCH_RY(R, CONV)                                                                      \
    switch (ry) {                                                                                  \
    case 1:                                                                                        \
        hipLaunchKernelGGL((k_stencil_batched<T, H, R, CONV, MODE, 1>), dim3(grid), dim3(kTX, kWY), \
                           0, s, a);                                                               \
        return hipGetLastError();                                                                  \
    case 2:                                                                                        \
        hipLaunchKernelGGL((k_stencil_batched<T, H, R, CONV, MODE, 2>), dim3(grid), dim3(kTX, kWY), \
                           0, s, a);                                                               \
        return hipGetLastError();                                                                  \
    case 4:                                                                                        \
        hipLaunchKernelGGL((k_stencil_batched<T, H, R, CONV, MODE, 4>), dim3(grid), dim3(kTX, kWY), \
                           0, s, a);                                                               \
        return hipGetLastError();                                                                  \
    default:                                                                                       \
        return hipErrorInvalidValue;                                                               \
    }
    if (conv) {
        if (radius != 1)
            return hipErrorInvalidValue;
        AAR_BATCH_RY(1, true)
    }
    switch (radius) {
    case 1:
        AAR_BATCH_RY(1, false)
    case 2:
        AAR_BATCH_RY(2, false)
    case 3:
        AAR_BATCH_RY(3, false)
    case 4:
        AAR_BATCH_RY(4, false)
    case 5:
        AAR_BATCH_RY(5, false)
    case 6:
        AAR_BATCH_RY(6, false)
    default:
        return hipErrorInvalidValue;
    }
#undef AAR_BATCH_RY
}

template <typename T, typename H, int R, bool CONV, int MODE, int RY>
static hipError_t launch_one(StencilArgs<T> a, const TileShape &ts, int *blocks_out, hipStream_t s)
{
    int tx, ty, tz, blocks;
    stencil_grid(a.st.n0, a.st.n1, a.st.n2, ts, &tx, &ty, &tz, &blocks);
    a.tiles_x = tx;
    a.tiles_y = ty;
    a.tiles_z = tz;
    a.cz = ts.cz;
    a.order = ts.order;
    if (blocks_out)
        *blocks_out = blocks;
    hipLaunchKernelGGL((k_stencil<T, H, R, CONV, MODE, RY>), dim3(blocks), dim3(kTX, kWY), 0, s, a);
    return hipGetLastError();
}

template <typename T, typename H, int R, int MODE, int RY, int NW>
static hipError_t launch_one2(StencilArgs<T> a, const TileShape &ts, int *blocks_out, hipStream_t s)
{
    int tx, ty, tz, blocks;
    stencil_grid(a.st.n0, a.st.n1, a.st.n2, ts, &tx, &ty, &tz, &blocks, true);
    a.tiles_x = tx;
    a.tiles_y = ty;
    a.tiles_z = tz;
    a.cz = ts.cz;
    a.order = ts.order;
    if (blocks_out)
        *blocks_out = blocks;
    // the fused Gram variant: FP64 iterate, FP64 or FP32 history, up to 8
    // waves (16-wave workgroups would spill its accumulators; with a bfloat16
    // history or an FP32 iterate the separate Gram pass runs)
    constexpr int GM = (MODE == kFk && NW <= 8 && sizeof(T) == 8 && sizeof(H) >= 4) ? kFusedGramM : 0;
    if (a.gram_partial && GM == 0)
        return hipErrorInvalidValue;
    if (a.gram_partial)
        hipLaunchKernelGGL((k_stencil2<T, H, R, MODE, RY, NW, GM>), dim3(blocks), dim3(kTX, NW), 0, s, a);
    else
        hipLaunchKernelGGL((k_stencil2<T, H, R, MODE, RY, NW, 0>), dim3(blocks), dim3(kTX, NW), 0, s, a);
    return hipGetLastError();
}

template <typename T, typename H, int MODE>
static hipError_t launch_paired(int radius, StencilArgs<T> a, const TileShape &ts, int *blocks_out, hipStream_t s)
{
    if (!paired_shape_ok(ts, sizeof(T) == 8))
        return hipErrorInvalidValue;
#define AAR_PAIR_RY(R)                                                      \
    switch (ts.ry + 4 * ts.pair) {                                          \
    case 1 + 4:                                                             \
        return launch_one2<T, H, R, MODE, 1, 4>(a, ts, blocks_out, s);      \
    case 2 + 4:                                                             \
        return launch_one2<T, H, R, MODE, 2, 4>(a, ts, blocks_out, s);      \
    case 1 + 8:                                                             \
        return launch_one2<T, H, R, MODE, 1, 8>(a, ts, blocks_out, s);      \
    case 2 + 8:                                                             \
        if constexpr (sizeof(T) == 4)                                       \
            return launch_one2<T, H, R, MODE, 2, 8>(a, ts, blocks_out, s);  \
        return hipErrorInvalidValue;                                        \
    case 1 + 12:                                                            \
        if constexpr (sizeof(T) == 4)                                       \
            return launch_one2<T, H, R, MODE, 1, 16>(a, ts, blocks_out, s); \
        return hipErrorInvalidValue;                                        \
    default:                                                                \
        return hipErrorInvalidValue;                                        \
    }
    switch (radius) {
    case 1:
        AAR_PAIR_RY(1)
    case 2:
        AAR_PAIR_RY(2)
    case 3:
        AAR_PAIR_RY(3)
    case 4:
        AAR_PAIR_RY(4)
    case 5:
        AAR_PAIR_RY(5)
    case 6:
        AAR_PAIR_RY(6)
    default:
        return hipErrorInvalidValue;
    }
#undef AAR_PAIR_RY
}

template <typename T, typename H, int R, bool CONV, int MODE>
static hipError_t launch_ry(StencilArgs<T> a, const TileShape &ts, int *blocks_out, hipStream_t s)
{
    switch (ts.ry) {
    case 1:
        return launch_one<T, H, R, CONV, MODE, 1>(a, ts, blocks_out, s);
    case 2:
        return launch_one<T, H, R, CONV, MODE, 2>(a, ts, blocks_out, s);
    case 4:
        return launch_one<T, H, R, CONV, MODE, 4>(a, ts, blocks_out, s);
    default:
        return hipErrorInvalidValue;
    }
}

template <typename T, typename H, int MODE>
static hipError_t launch_radius(int radius, bool conv, StencilArgs<T> a, const TileShape &ts, int *blocks_out,
                                hipStream_t s)
{
    if (conv) {
        if (radius != 1)
            return hipErrorInvalidValue;
        return launch_ry<T, H, 1, true, MODE>(a, ts, blocks_out, s);
    }
    switch (radius) {
    case 1:
        return launch_ry<T, H, 1, false, MODE>(a, ts, blocks_out, s);
    case 2:
        return launch_ry<T, H, 2, false, MODE>(a, ts, blocks_out, s);
    case 3:
        return launch_ry<T, H, 3, false, MODE>(a, ts, blocks_out, s);
    case 4:
        return launch_ry<T, H, 4, false, MODE>(a, ts, blocks_out, s);
    case 5:
        return launch_ry<T, H, 5, false, MODE>(a, ts, blocks_out, s);
    case 6:
        return launch_ry<T, H, 6, false, MODE>(a, ts, blocks_out, s);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace aar
