// Host driver and C ABI of the AAR solver (include/aar.h).
//
// A solve runs whole AAR cycles on the GPU: p-1 fused Richardson sweeps,
// the Anderson-step residual pass, the Gram products, the one-workgroup
// least-squares solve and the streamed update (Sec. 2, Eqs. 2-6).  All
// control decisions (convergence, breakdown, iteration cap, inner-solve
// stagnation) are taken on the device by the least-squares kernel and kept
// in a small state record; every kernel of a cycle reads that record and
// returns at once when the system is done, so the host only replays a
// captured graph of several cycles and polls the status between replays,
// one graph behind.
//
// Mixed precision wraps the FP32 iteration in FP64 iterative refinement:
// r = b - A x (FP64), inner FP32 AAR on A d = r / ||r||, x += ||r|| d.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/aar.h"
#include "aar_device.h"

using namespace aar;

namespace {

thread_local std::string g_error;

aar_status fail(aar_status st, const std::string &msg)
{
    g_error = msg;
    return st;
}

#define AAR_HIP(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(e_ == hipErrorOutOfMemory ? AAR_ERR_OUT_OF_MEMORY : AAR_ERR_DEVICE,     \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                     \
    } while (0)

// Order-2r central second-difference weights, unit spacing: w_s for s = 1..r
// by the product form 2 (-1)^{s+1} / s^2 * prod_{t=1..s} (r-t+1)/(r+t) of the
// standard central formula; w_0 = -2 sum_s w_s makes the rule exact on
// constants.
void central_weights(int r, double *w)
{
    double sum = 0.0;
    for (int s = 1; s <= r; ++s) {
        double prod = 1.0;
        for (int t = 1; t <= s; ++t)
            prod *= (double)(r - t + 1) / (double)(r + t);
        const double v = 2.0 * prod / ((double)s * s);
        w[s] = (s & 1) ? v : -v;
        sum += w[s];
    }
    w[0] = -2.0 * sum;
}

struct Operator {
    aar_problem prob;
    int64_t N = 0;
    double c[3][kMaxRadius + 1] = {};
    double diag = 0.0;    // centre weight of the stencil, without convection
    double jdiag = 0.0;   // diag(A) without convection (the Jacobi preconditioner)
    double *vel64 = nullptr;
    float *vel32 = nullptr;
    TileShape ts[2];      // stencil tile for FP64 [0] and FP32 [1] passes
};

template <typename T> StencilDev<T> make_stencil(const Operator &op, const T *vel)
{
    StencilDev<T> st;
    std::memset(&st, 0, sizeof(st));
    st.n0 = op.prob.n[0];
    st.n1 = op.prob.n[1];
    st.n2 = op.prob.n[2];
    st.per0 = op.prob.bc[0] == AAR_BC_PERIODIC;
    st.per1 = op.prob.bc[1] == AAR_BC_PERIODIC;
    st.per2 = op.prob.bc[2] == AAR_BC_PERIODIC;
    for (int s = 0; s <= kMaxRadius; ++s) {
        st.c0[s] = (T)op.c[0][s];
        st.c1[s] = (T)op.c[1][s];
        st.c2[s] = (T)op.c[2][s];
    }
    st.sigma = (T)op.prob.shift;
    st.diag = (T)op.diag;
    st.jdiag = (T)op.jdiag;
    st.inv_diag = (T)(1.0 / op.jdiag);
    st.ih0 = (T)(1.0 / op.prob.h[0]);
    st.ih1 = (T)(1.0 / op.prob.h[1]);
    st.ih2 = (T)(1.0 / op.prob.h[2]);
    st.vel = vel;
    st.N = op.N;
    return st;
}

TileShape default_tile(int radius, bool fp64)
{
    TileShape ts;
    if (radius <= 2) {
        ts.ry = 4;
        ts.cz = 32;
    } else if (fp64) {
        ts.ry = 2;
        ts.cz = 16;
    } else {
        ts.ry = 4;
        ts.cz = 16;
    }
    return ts;
}

// Buffers and launch arguments of the AAR iteration in precision T.
template <typename T> struct Path {
    Prec hist = Prec::F64;
    T *xa = nullptr, *xb = nullptr, *b = nullptr, *fcur = nullptr;
    void *dx = nullptr;        // Anderson increments, DxOf<T, hist> elements
    void *fring = nullptr;
    int64_t N = 0, slot_stride = 0;
    TileShape ts{};
    StencilDev<T> st{};
    int radius = 1;
    bool conv = false;
    int rho_blocks = 0, gram_blocks = 0, upd_blocks = 0;
    int64_t dx_stride = 0;     // elements between dx slots
    bool gram_fused = false;   // the Anderson-residual pass forms the Gram products
    bool recur = false;        // sweeps after a cycle's first use the residual recursion
    // FP64 iterate with an FP32 ring: the recursion sweeps and the Anderson-
    // step residual run the FP32 stencil on the ring (tile ts32, FP32
    // coefficients st32, rho_blocks32 workgroups)
    bool recur32 = false;
    TileShape ts32{};
    StencilDev<float> st32{};
    int rho_blocks32 = 0;
};

size_t hist_bytes(Prec p)
{
    return p == Prec::F64 ? 8 : (p == Prec::F32 ? 4 : 2);
}

bool is_mixed(int precision)
{
    return precision == AAR_MIXED_FP32 || precision == AAR_MIXED_FP32_BF16HIST;
}

Prec hist_of(int precision)
{
    switch (precision) {
    case AAR_MIXED_FP32:
    case AAR_FP64_FP32HIST:
        return Prec::F32;
    case AAR_MIXED_FP32_BF16HIST:
    case AAR_FP64_BF16HIST:
        return Prec::F32_BF16;
    default:
        return Prec::F64;
    }
}

// Byte offset added between consecutive bulk vectors (multiple of 64).
size_t stagger_bytes()
{
    const char *env = getenv("AAR_STAGGER_BYTES");
    long v = env ? atol(env) : 0;
    if (v < 0)
        v = 0;
    return (size_t)((v + 63) / 64 * 64);
}

}  // namespace

struct aar_solver_t {
    aar_params params{};
    std::vector<Operator> ops;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    int device = 0;
    int q = 0;              // dx ring slots
    int ne = 0;             // Gram entries
    int64_t maxN = 0;
    bool mixed = false;
    Prec hist = Prec::F64;
    std::vector<void *> allocations;

    // device workspace (sized for the largest system)
    InstState *state = nullptr;
    double *part_rho = nullptr, *part_gram = nullptr, *part_norm = nullptr;
    double *gram_final = nullptr;
    int part_rho_cap = 0;      // entries of part_rho (stencil workgroups of one pass)
    double *scal = nullptr;       // [0] ||r|| of the refinement, [1] ||b|| (FP64)
    double *log = nullptr;
    int32_t *rank_log = nullptr;   // beside log: rank kept by each Anderson step's solve
    int64_t log_cap = 0;
    Path<double> p64;
    Path<float> p32;
    double *x64 = nullptr, *b64 = nullptr, *r64 = nullptr;   // refinement vectors (mixed)

    int64_t slot_stride[2] = {0, 0};   // ring slot spacing (elements) for the FP64 and FP32 paths
    int64_t dx_stride = 0;              // FP32 path: dx slot spacing (elements)
    int64_t dx_stride64 = 0;            // FP64 path: dx slot spacing (elements)

    // graphs (single system)
    hipGraphExec_t graph = nullptr;
    int graph_cycles = 0;
    int graph_instance = -1;

    // pinned status mailbox
    int32_t *host_status = nullptr;     // pinned: the run status written by the update kernels
    int32_t *status_dev = nullptr;      // its device address
    hipEvent_t poll_ev[2] = {nullptr, nullptr};

    // sweep timing
    bool timing = false;
    std::vector<hipEvent_t> tev;
    std::vector<int64_t> tcycle;
    std::vector<int> tcount;        // positions each timed group covers
    size_t tused = 0;
    double t_total_ms = 0.0;
    int64_t t_launches = 0;

    std::vector<int64_t> last_log_count;
    int last_instance = 0;

    // complex-valued system (aar_create_complex): A = A_r + i shift_im I,
    // complex omega and beta; vectors interleaved (re, im)
    bool cplx = false;
    double shift_im = 0.0, omega_im = 0.0, beta_im = 0.0;
    Path<zd> pz;

    // general sparse system (aar_create_csr): CSR arrays, block bounds,
    // level schedules and ILU(0) factors on the device; vectors in p64
    bool csr = false;
    CsrDev cd{};

    // batched engine (count > 1 with one stencil radius and convection kind)
    struct Batch {
        bool on = false;
        int count = 0, radius = 1, ry = 2, grid_s = 1, grid_c = 1;
        bool conv = false;
        int64_t total = 0, stride = 0;
        int sum_tiles = 0, sum_chunks = 0;
        std::vector<int64_t> offs, sizes;
        std::vector<int> ntiles, nchunks;
        BatchDesc<double> *desc64 = nullptr;
        BatchDesc<float> *desc32 = nullptr;
        int64_t *d_offs = nullptr, *d_sizes = nullptr, *d_uoffs = nullptr;
        int *d_ntiles = nullptr, *d_nchunks = nullptr;
        double *d_invshift = nullptr;
        BatchCtl *ctl = nullptr;
        InstState *state = nullptr;
        int *refine = nullptr, *remaining = nullptr;
        int2 *c_s = nullptr, *c_c = nullptr, *a_s = nullptr, *a_c = nullptr;
        int *c_n = nullptr, *a_n = nullptr;
        int *c_sb = nullptr, *c_cb = nullptr, *a_sb = nullptr, *a_cb = nullptr;
        double *p_rho = nullptr, *p_gram = nullptr, *p_s = nullptr, *p_c = nullptr;
        double *xa64 = nullptr, *xb64 = nullptr, *b64 = nullptr, *r64 = nullptr;
        void *dx64 = nullptr;   // FP64 iterate's increments (FP32 beside an FP32 ring)
        double *fcur64 = nullptr;   // FP64 f_k when an FP64 iteration keeps a narrow history
        float *xa32 = nullptr, *xb32 = nullptr, *rhs32 = nullptr, *fcur32 = nullptr, *dx32 = nullptr;
        void *fring = nullptr;
        double *log = nullptr;
        int32_t *rank_log = nullptr;
        hipGraphExec_t graph = nullptr;
        int *h_remaining = nullptr;
        bool recur = false;     // cycles use the residual recursion (ring of the iterate's type)
        bool recur32 = false;   // FP64 iterate, FP32 ring: the recursion passes run the FP32 stencil
    } B;

    template <typename T> T *alloc(size_t count, aar_status *st)
    {
        void *p = nullptr;
        if (count == 0)
            count = 1;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) {
            *st = fail(e == hipErrorOutOfMemory ? AAR_ERR_OUT_OF_MEMORY : AAR_ERR_DEVICE,
                       std::string("hipMalloc: ") + hipGetErrorString(e));
            return nullptr;
        }
        allocations.push_back(p);
        return static_cast<T *>(p);
    }

    ~aar_solver_t()
    {
        if (graph)
            (void)hipGraphExecDestroy(graph);
        if (B.graph)
            (void)hipGraphExecDestroy(B.graph);
        if (B.h_remaining)
            (void)hipHostFree(B.h_remaining);
        for (void *p : allocations)
            (void)hipFree(p);
        if (host_status)
            (void)hipHostFree(host_status);
        for (hipEvent_t e : poll_ev)
            if (e)
                (void)hipEventDestroy(e);
        for (hipEvent_t e : tev)
            (void)hipEventDestroy(e);
        if (capture_stream)
            (void)hipStreamDestroy(capture_stream);
    }
};

namespace {

aar_status validate_params(const aar_params *pa)
{
    if (!pa)
        return fail(AAR_ERR_INVALID_ARG, "params is NULL");
    if (pa->m < 1 || pa->m > kMaxM)
        return fail(AAR_ERR_INVALID_ARG, "m must be in 1..32");
    if (pa->p < 1)
        return fail(AAR_ERR_INVALID_ARG, "p must be >= 1");
    if (!(pa->tol > 0.0) || !std::isfinite(pa->tol))
        return fail(AAR_ERR_INVALID_ARG, "tol must be positive and finite");
    if (pa->max_iter < 1)
        return fail(AAR_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (!std::isfinite(pa->omega) || !std::isfinite(pa->beta))
        return fail(AAR_ERR_INVALID_ARG, "omega and beta must be finite");
    if (pa->precision < AAR_FP64 || pa->precision > AAR_FP64_BF16HIST)
        return fail(AAR_ERR_INVALID_ARG, "unknown precision");
    if (!(pa->inner_tol >= 0.0) || pa->inner_tol >= 1.0 || pa->max_outer < 0)
        return fail(AAR_ERR_INVALID_ARG, "inner_tol must be in [0, 1) and max_outer >= 0");
    return AAR_OK;
}

aar_status validate_problem(const aar_problem &pr, int idx)
{
    const std::string at = " (system " + std::to_string(idx) + ")";
    for (int a = 0; a < 3; ++a) {
        if (pr.n[a] < 1)
            return fail(AAR_ERR_INVALID_ARG, "n must be >= 1" + at);
        if (!(pr.h[a] > 0.0) || !std::isfinite(pr.h[a]))
            return fail(AAR_ERR_INVALID_ARG, "h must be positive and finite" + at);
        if (pr.bc[a] != AAR_BC_ZERO_DIRICHLET && pr.bc[a] != AAR_BC_PERIODIC)
            return fail(AAR_ERR_INVALID_ARG, "unknown boundary condition" + at);
    }
    if (pr.radius < 1 || pr.radius > kMaxRadius)
        return fail(AAR_ERR_INVALID_ARG, "radius must be in 1..6" + at);
    if (!(pr.diffusion > 0.0) || !std::isfinite(pr.diffusion))
        return fail(AAR_ERR_INVALID_ARG, "diffusion must be positive and finite" + at);
    if (!(pr.shift >= 0.0) || !std::isfinite(pr.shift))
        return fail(AAR_ERR_INVALID_ARG, "shift must be non-negative and finite" + at);
    if (pr.velocity && pr.radius != 1)
        return fail(AAR_ERR_UNSUPPORTED, "convection needs radius 1" + at);
    // a periodic axis shorter than the stencil wraps its taps modulo n and
    // they add up (a circulant); with convection a one-point periodic axis
    // would make the upwind difference vanish, which the kernels' Jacobi
    // diagonal does not model
    for (int a = 0; a < 3; ++a)
        if (pr.velocity && pr.bc[a] == AAR_BC_PERIODIC && pr.n[a] < 2)
            return fail(AAR_ERR_UNSUPPORTED, "convection on a periodic axis of one point" + at);
    const int64_t N = (int64_t)pr.n[0] * pr.n[1] * pr.n[2];
    if (N > ((int64_t)1 << 40) || (int64_t)pr.n[0] * pr.n[1] >= ((int64_t)1 << 31))
        return fail(AAR_ERR_UNSUPPORTED, "grid too large" + at);
    return AAR_OK;
}

Operator build_operator(const aar_problem &pr)
{
    Operator op;
    op.prob = pr;
    op.N = (int64_t)pr.n[0] * pr.n[1] * pr.n[2];
    double w[kMaxRadius + 1];
    central_weights(pr.radius, w);
    double sum = 0.0;
    for (int a = 0; a < 3; ++a) {
        for (int s = 1; s <= pr.radius; ++s) {
            op.c[a][s] = -pr.diffusion * w[s] / (pr.h[a] * pr.h[a]);
            sum += op.c[a][s];
        }
    }
    op.diag = pr.shift - 2.0 * sum;
    // taps +-s of a periodic axis land on the point itself when n divides s
    op.jdiag = op.diag;
    for (int a = 0; a < 3; ++a)
        if (pr.bc[a] == AAR_BC_PERIODIC)
            for (int s = 1; s <= pr.radius; ++s)
                if (s % pr.n[a] == 0)
                    op.jdiag += 2.0 * op.c[a][s];
    op.ts[0] = default_tile(pr.radius, true);
    op.ts[1] = default_tile(pr.radius, false);
    return op;
}

struct Sizes {
    int64_t maxN = 0;
    int max_stencil_blocks = 0;
    int gram_blocks = 0;
    int q = 0, ne = 0;
    size_t bytes = 0;
    int64_t log_cap = 0;
};

Sizes compute_sizes(const aar_problem *probs, int count, const aar_params *pa)
{
    Sizes z;
    const bool mixed = is_mixed(pa->precision);
    const Prec hist = hist_of(pa->precision);
    int64_t vel_total = 0;
    for (int i = 0; i < count; ++i) {
        const aar_problem &pr = probs[i];
        const int64_t N = (int64_t)pr.n[0] * pr.n[1] * pr.n[2];
        z.maxN = std::max(z.maxN, N);
        // partial sums are one per stencil workgroup: size them for the
        // largest grid any candidate tile shape (autotuner, tile file) gives
        for (int ry : {1, 2, 4}) {
            for (int cz : {1, 2, 4, 8, 16, 32, 64}) {
                TileShape ts{ry, cz};
                int tx, ty, tz, blocks;
                stencil_grid(pr.n[0], pr.n[1], pr.n[2], ts, &tx, &ty, &tz, &blocks);
                z.max_stencil_blocks = std::max(z.max_stencil_blocks, blocks);
            }
        }
        if (pr.velocity)
            vel_total += 3 * N;
    }
    z.gram_blocks = std::max(gram_blocks(z.maxN, 1), stream_blocks(z.maxN));
    z.q = pa->m / pa->p;
    z.ne = pa->m * (pa->m + 1) / 2 + pa->m;
    const int slots = pa->m + 1;
    const size_t stagger = stagger_bytes();
    auto vec_span = [&](size_t esize) { return (((size_t)z.maxN * esize + 4095) / 4096) * 4096 + stagger; };
    size_t b = 0;
    b += sizeof(InstState) * (size_t)count;
    b += sizeof(double) * ((size_t)z.max_stencil_blocks + (size_t)std::max(z.gram_blocks, z.max_stencil_blocks) * z.ne +
                           z.gram_blocks + z.ne + 8);
    if (!mixed) {
        b += vec_span(8) * 3 + vec_span(hist == Prec::F32 ? 4 : 8) * z.q + vec_span(hist_bytes(hist)) * slots +
             (hist == Prec::F32_BF16 ? vec_span(8) : 0);
        b += (sizeof(double) + (hist == Prec::F32 ? sizeof(float) : 0)) * (size_t)vel_total;
    } else {
        b += vec_span(4) * (3 + z.q) + vec_span(hist_bytes(hist)) * slots + vec_span(8) * 3;
        if (hist == Prec::F32_BF16)
            b += vec_span(4);
        b += (sizeof(double) + sizeof(float)) * (size_t)vel_total;
    }
    if (pa->flags & AAR_FLAG_RECORD_RESIDUALS) {
        z.log_cap = std::min<int64_t>(pa->max_iter / pa->p + 2, (int64_t)1 << 22);
        b += (sizeof(double) + sizeof(int32_t)) * (size_t)z.log_cap;
    }
    z.bytes = b;
    return z;
}

// ---------------------------------------------------------------------------
// Enqueue one AAR cycle in precision T on stream s.
// ---------------------------------------------------------------------------
template <typename T> struct Launch;
template <> struct Launch<double> {
    static hipError_t stencil(int mode, const Path<double> &P, StencilArgs<double> a, hipStream_t s)
    {
        return launch_stencil_f64(mode, P.hist, P.radius, P.conv, P.ts, a, nullptr, s);
    }
    static hipError_t stencil(int mode, const Path<double> &P, StencilArgs<double> a, hipStream_t s,
                              const TileShape &ts)
    {
        return launch_stencil_f64(mode, P.hist, P.radius, P.conv, ts, a, nullptr, s);
    }
};
template <> struct Launch<float> {
    static hipError_t stencil(int mode, const Path<float> &P, StencilArgs<float> a, hipStream_t s)
    {
        return launch_stencil_f32(mode, P.hist, P.radius, P.conv, P.ts, a, nullptr, s);
    }
    static hipError_t stencil(int mode, const Path<float> &P, StencilArgs<float> a, hipStream_t s,
                              const TileShape &ts)
    {
        return launch_stencil_f32(mode, P.hist, P.radius, P.conv, ts, a, nullptr, s);
    }
};

template <typename T> hipError_t launch_tblock(const Path<T> &P, const StencilArgs<T> &a, int j0, int nt, bool last_fk,
                                               hipStream_t s, const TileShape &ts)
{
    if constexpr (std::is_same<T, double>::value)
        return launch_tblock_f64(P.radius, P.conv, ts, a, j0, nt, last_fk, s);
    else
        return launch_tblock_f32(P.radius, P.conv, ts, a, j0, nt, last_fk, s);
}

// Whether a cycle's positions 1 .. p-1 run as temporal blocks for this path:
// the residual recursion with a ring of the iterate's type, a one-point tile
// with a block depth of 2 or more, radius <= 2, and blocks whose LDS fits.
template <typename T> bool tblock_active(const Path<T> &P, int p, const TileShape &ts)
{
    return P.recur && !P.recur32 && p >= 2 && ts.tb >= 2 && ts.pair == 0 &&
           tblock_fits(P.radius, P.conv, ts, std::min(ts.tb, p - 1), std::is_same<T, double>::value);
}

// Arguments of an FP32 recursion pass over an FP32 ring (Path::recur32).
// The recursion reads neither x nor b; both point at the ring so that every
// pointer the kernel holds is a valid FP32 vector.
template <typename T> StencilArgs<float> ring_args32(aar_solver_t *S, const Path<T> &P, int j)
{
    const aar_params &pa = S->params;
    StencilArgs<float> a;
    std::memset(&a, 0, sizeof(a));
    a.st = P.st32;
    a.x = static_cast<const float *>(P.fring);
    a.b = static_cast<const float *>(P.fring);
    a.out = nullptr;
    a.fring = P.fring;
    a.state = S->state;
    a.slot_stride = P.slot_stride;
    a.j = j;
    a.p = pa.p;
    a.nslots = pa.m + 1;
    a.omega = (float)pa.omega;
    a.recur = 1;
    return a;
}

template <typename T>
hipError_t enqueue_cycle(aar_solver_t *S, const Path<T> &P, bool inner, hipStream_t s, int64_t cycle_tag)
{
    const aar_params &pa = S->params;
    StencilArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.st = P.st;
    a.b = P.b;
    a.fring = P.fring;
    a.state = S->state;
    a.slot_stride = P.slot_stride;
    a.p = pa.p;
    a.nslots = pa.m + 1;
    a.omega = (T)pa.omega;
    hipError_t e;
    const bool rec = P.recur || P.recur32;
    // temporal blocks: the first sweep alone, then blocks over positions
    // 1 .. p-1 (the last one ending with the Anderson-step residual)
    const bool tb = tblock_active(P, pa.p, P.ts);
    const int jend = tb ? 1 : pa.p - 1;
    for (int j = 0; j < jend; ++j) {
        a.j = j;
        if (rec) {
            // x stays the cycle's first iterate; the first sweep reads it and
            // b, the others continue from the previous f
            a.recur = j > 0 ? 1 : 0;
            a.x = P.xa;
            a.out = nullptr;
        } else {
            a.x = (j & 1) ? P.xb : P.xa;
            a.out = (j & 1) ? P.xa : P.xb;
        }
        // timing: one event pair around the cycle's p - 1 back-to-back sweeps
        if (S->timing && j == 0) {
            if (S->tused + 2 > S->tev.size()) {
                for (int t = 0; t < 64; ++t) {
                    hipEvent_t ev;
                    if ((e = hipEventCreate(&ev)) != hipSuccess)
                        return e;
                    S->tev.push_back(ev);
                }
            }
            if ((e = hipEventRecord(S->tev[S->tused], s)) != hipSuccess)
                return e;
        }
        if (P.recur32 && j > 0)
            e = launch_stencil_f32(kSweep, Prec::F32, P.radius, P.conv, P.ts32, ring_args32(S, P, j), nullptr, s);
        else
            e = Launch<T>::stencil(kSweep, P, a, s);
        if (e != hipSuccess)
            return e;
        if (S->timing && !tb && j == pa.p - 2) {
            if ((e = hipEventRecord(S->tev[S->tused + 1], s)) != hipSuccess)
                return e;
            S->tcycle.push_back(cycle_tag * pa.p + j);   // the group's last sweep
            S->tcount.push_back(pa.p - 1);
            S->tused += 2;
        }
    }
    const int jk = pa.p - 1;
    if (tb) {
        a.recur = 1;
        a.x = P.xa;
        a.out = nullptr;
        a.partial = S->part_rho;
        a.gram_partial = nullptr;
        for (int j = 1; j <= jk;) {
            const int nt = std::min(P.ts.tb, pa.p - j);
            if ((e = launch_tblock<T>(P, a, j, nt, j + nt - 1 == jk, s, P.ts)) != hipSuccess)
                return e;
            j += nt;
        }
        if (S->timing) {
            // the timed group covers every position of the cycle (the blocks
            // include the Anderson-step residual)
            if ((e = hipEventRecord(S->tev[S->tused + 1], s)) != hipSuccess)
                return e;
            S->tcycle.push_back(cycle_tag * pa.p + jk);
            S->tcount.push_back(pa.p);
            S->tused += 2;
        }
    }
    T *xk = rec ? P.xa : (jk & 1) ? P.xb : P.xa;
    a.j = jk;
    a.x = xk;
    a.recur = P.recur && jk > 0 ? 1 : 0;
    a.out = nullptr;
    a.fcur = P.fcur;
    a.partial = S->part_rho;
    a.gram_partial = P.gram_fused ? S->part_gram : nullptr;
    if (tb) {
        e = hipSuccess;   // the last block formed the Anderson-step residual
    } else if (P.recur32) {   // jk >= 1: p >= 2
        StencilArgs<float> a32 = ring_args32(S, P, jk);
        a32.partial = S->part_rho;
        e = launch_stencil_f32(kFk, Prec::F32, P.radius, P.conv, P.ts32, a32, nullptr, s);
    } else {
        e = Launch<T>::stencil(kFk, P, a, s);
    }
    if (e != hipSuccess)
        return e;

    GramArgs g;
    g.fring = P.fring;
    g.partial = S->part_gram;
    g.state = S->state;
    g.N = P.N;
    g.slot_stride = P.slot_stride;
    g.m = pa.m;
    g.p = pa.p;
    g.nslots = pa.m + 1;
    g.ne = S->ne;
    if (!P.gram_fused && (e = launch_gram(P.hist, g, P.gram_blocks, s)) != hipSuccess)
        return e;
    if (!P.gram_fused && (e = launch_gram_finish(S->part_gram, P.gram_blocks, S->gram_final, S->ne, S->state, pa.p,
                                                 s)) != hipSuccess)
        return e;

    LsqArgs l;
    l.state = S->state;
    l.rho_partial = S->part_rho;
    l.rho_blocks = P.recur32 ? P.rho_blocks32 : P.rho_blocks;
    l.gram_final = S->gram_final;
    l.ne = S->ne;
    // the fused pass leaves one partial per workgroup and entry; the solve
    // kernel sums them itself
    l.gram_partial = P.gram_fused ? S->part_gram : nullptr;
    l.gram_blocks = P.gram_fused ? P.rho_blocks : 0;
    l.m = pa.m;
    l.p = pa.p;
    l.nslots = pa.m + 1;
    l.q = S->q;
    l.omega = pa.omega;
    l.beta = pa.beta;
    l.rcond = std::ldexp(1.0, -52);
    l.stagnation_window = inner ? 8 : 0;
    l.stagnation_factor = 0.9;
    l.log = S->log;
    l.rank_log = S->rank_log;
    l.log_cap = S->log_cap;
    l.force_pinv = (pa.flags & AAR_FLAG_FORCE_PINV) ? 1 : 0;
    if ((e = launch_lsq(l, s)) != hipSuccess)
        return e;

    UpdateArgs<T> u;
    u.xin = xk;
    u.xout = P.xa;
    u.fring = P.fring;
    u.fcur = P.fcur;
    u.dxring = P.dx;
    u.state = S->state;
    u.N = P.N;
    u.slot_stride = P.slot_stride;
    u.dx_stride = P.dx_stride;
    u.status_out = S->status_dev;
    if (rec) {
        // xk is the cycle's first iterate: the update applies the cycle's
        // Richardson steps before the extrapolation
        u.omega_rich = (T)pa.omega;
        u.p_rich = pa.p;
    }
    if constexpr (std::is_same<T, double>::value)
        return launch_update(P.hist, &u, nullptr, P.upd_blocks, s);
    else
        return launch_update(P.hist, nullptr, &u, P.upd_blocks, s);
}

// One AAR cycle of a complex-valued system (complex.hip kernels): p - 1
// sweeps from x and b with x ping-ponged, the Anderson-step residual, the
// Hermitian Gram products, the one-wave solve and the update.
hipError_t enqueue_cycle_complex(aar_solver_t *S, const Path<zd> &P, hipStream_t s)
{
    const aar_params &pa = S->params;
    StencilArgs<zd> a;
    std::memset(&a, 0, sizeof(a));
    a.st = P.st;
    a.b = P.b;
    a.fring = P.fring;
    a.state = S->state;
    a.slot_stride = P.slot_stride;
    a.p = pa.p;
    a.nslots = pa.m + 1;
    a.omega = zd(pa.omega, S->omega_im);
    hipError_t e;
    for (int j = 0; j < pa.p - 1; ++j) {
        a.j = j;
        a.x = (j & 1) ? P.xb : P.xa;
        a.out = (j & 1) ? P.xa : P.xb;
        if ((e = launch_stencil_complex(kSweep, P.radius, P.ts, a, nullptr, s)) != hipSuccess)
            return e;
    }
    const int jk = pa.p - 1;
    zd *xk = (jk & 1) ? P.xb : P.xa;
    a.j = jk;
    a.x = xk;
    a.out = nullptr;
    a.partial = S->part_rho;
    if ((e = launch_stencil_complex(kFk, P.radius, P.ts, a, nullptr, s)) != hipSuccess)
        return e;
    GramArgs g;
    g.fring = P.fring;
    g.partial = S->part_gram;
    g.state = S->state;
    g.N = P.N;
    g.slot_stride = P.slot_stride;
    g.m = pa.m;
    g.p = pa.p;
    g.nslots = pa.m + 1;
    g.ne = S->ne;
    // real and imaginary parts in one pass: two entry-major partial tables
    // back to back, which one finishing launch over 2 ne entries sums into
    // [Re G, Re c | Im G, Im c]
    if ((e = launch_cgram(g, P.gram_blocks, s)) != hipSuccess)
        return e;
    if ((e = launch_gram_finish(S->part_gram, P.gram_blocks, S->gram_final, 2 * S->ne, S->state, pa.p, s)) !=
        hipSuccess)
        return e;
    LsqArgs l;
    l.state = S->state;
    l.rho_partial = S->part_rho;
    l.rho_blocks = P.rho_blocks;
    l.gram_final = S->gram_final;
    l.ne = S->ne;
    l.m = pa.m;
    l.p = pa.p;
    l.nslots = pa.m + 1;
    l.q = S->q;
    l.omega = pa.omega;
    l.beta = pa.beta;
    l.rcond = std::ldexp(1.0, -52);
    l.stagnation_window = 0;
    l.stagnation_factor = 0.9;
    l.log = S->log;
    l.rank_log = S->rank_log;
    l.log_cap = S->log_cap;
    l.force_pinv = (pa.flags & AAR_FLAG_FORCE_PINV) ? 1 : 0;
    if ((e = launch_clsq(l, S->omega_im, S->beta_im, s)) != hipSuccess)
        return e;
    UpdateArgs<zd> u;
    u.xin = xk;
    u.xout = P.xa;
    u.fring = P.fring;
    u.fcur = nullptr;
    u.dxring = P.dx;
    u.state = S->state;
    u.N = P.N;
    u.slot_stride = P.slot_stride;
    u.dx_stride = P.dx_stride;
    u.status_out = S->status_dev;
    return launch_cupdate(u, P.upd_blocks, s);
}

// One AAR cycle of a general sparse system (sparse.hip kernels): p - 1
// sweeps from x and b with x ping-ponged (every row reads x anywhere), the
// Anderson-step residual with its norm partials, the Gram products, the
// one-wave solve and the update.
hipError_t enqueue_cycle_csr(aar_solver_t *S, const Path<double> &P, hipStream_t s, int64_t cycle_tag)
{
    const aar_params &pa = S->params;
    CsrArgs a;
    std::memset(&a, 0, sizeof(a));
    a.c = S->cd;
    a.b = P.b;
    a.fring = P.fring;
    a.state = S->state;
    a.slot_stride = P.slot_stride;
    a.p = pa.p;
    a.nslots = pa.m + 1;
    a.omega = pa.omega;
    hipError_t e;
    for (int j = 0; j < pa.p - 1; ++j) {
        a.j = j;
        a.x = (j & 1) ? P.xb : P.xa;
        a.xout = (j & 1) ? P.xa : P.xb;
        // timing: one event pair around the cycle's p - 1 back-to-back sweeps
        if (S->timing && j == 0) {
            if (S->tused + 2 > S->tev.size()) {
                for (int t = 0; t < 64; ++t) {
                    hipEvent_t ev;
                    if ((e = hipEventCreate(&ev)) != hipSuccess)
                        return e;
                    S->tev.push_back(ev);
                }
            }
            if ((e = hipEventRecord(S->tev[S->tused], s)) != hipSuccess)
                return e;
        }
        if ((e = launch_csr(kSweep, a, s)) != hipSuccess)
            return e;
        if (S->timing && j == pa.p - 2) {
            if ((e = hipEventRecord(S->tev[S->tused + 1], s)) != hipSuccess)
                return e;
            S->tcycle.push_back(cycle_tag * pa.p + j);
            S->tcount.push_back(pa.p - 1);
            S->tused += 2;
        }
    }
    const int jk = pa.p - 1;
    double *xk = (jk & 1) ? P.xb : P.xa;
    a.j = jk;
    a.x = xk;
    a.xout = nullptr;
    a.partial = S->part_rho;
    if ((e = launch_csr(kFk, a, s)) != hipSuccess)
        return e;
    GramArgs g;
    g.fring = P.fring;
    g.partial = S->part_gram;
    g.state = S->state;
    g.N = P.N;
    g.slot_stride = P.slot_stride;
    g.m = pa.m;
    g.p = pa.p;
    g.nslots = pa.m + 1;
    g.ne = S->ne;
    if ((e = launch_gram(Prec::F64, g, P.gram_blocks, s)) != hipSuccess)
        return e;
    if ((e = launch_gram_finish(S->part_gram, P.gram_blocks, S->gram_final, S->ne, S->state, pa.p, s)) !=
        hipSuccess)
        return e;
    LsqArgs l;
    std::memset(&l, 0, sizeof(l));
    l.state = S->state;
    l.rho_partial = S->part_rho;
    l.rho_blocks = P.rho_blocks;
    l.gram_final = S->gram_final;
    l.ne = S->ne;
    l.gram_partial = nullptr;
    l.gram_blocks = 0;
    l.m = pa.m;
    l.p = pa.p;
    l.nslots = pa.m + 1;
    l.q = S->q;
    l.omega = pa.omega;
    l.beta = pa.beta;
    l.rcond = std::ldexp(1.0, -52);
    l.stagnation_window = 0;
    l.stagnation_factor = 0.9;
    l.log = S->log;
    l.rank_log = S->rank_log;
    l.log_cap = S->log_cap;
    l.force_pinv = (pa.flags & AAR_FLAG_FORCE_PINV) ? 1 : 0;
    if ((e = launch_lsq(l, s)) != hipSuccess)
        return e;
    UpdateArgs<double> u;
    u.xin = xk;
    u.xout = P.xa;
    u.fring = P.fring;
    u.fcur = nullptr;
    u.dxring = P.dx;
    u.state = S->state;
    u.N = P.N;
    u.slot_stride = P.slot_stride;
    u.dx_stride = P.dx_stride;
    u.status_out = S->status_dev;
    return launch_update(Prec::F64, &u, nullptr, P.upd_blocks, s);
}

template <typename T>
hipError_t enqueue_any(aar_solver_t *S, const Path<T> &P, bool inner, hipStream_t s, int64_t cycle_tag)
{
    if constexpr (std::is_same<T, zd>::value) {
        return enqueue_cycle_complex(S, P, s);
    } else {
        if constexpr (std::is_same<T, double>::value) {
            if (S->csr)
                return enqueue_cycle_csr(S, P, s, cycle_tag);
        }
        return enqueue_cycle<T>(S, P, inner, s, cycle_tag);
    }
}

constexpr int kGraphCycles = 4;

// Run cycles until the device state leaves kRunning (or every cycle up to
// max_iter has been issued).  The final state is copied to *out.
template <typename T>
aar_status run_cycles(aar_solver_t *S, const Path<T> &P, int64_t max_iter, bool inner, bool use_graph,
                      InstState *out)
{
    const int p = S->params.p;
    const int64_t needed = (max_iter + p - 1) / p;
    hipStream_t s = S->stream;
    if (use_graph && S->graph == nullptr) {
        AAR_HIP(hipStreamBeginCapture(S->capture_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int c = 0; c < kGraphCycles && e == hipSuccess; ++c)
            e = enqueue_any<T>(S, P, inner, S->capture_stream, 0);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(S->capture_stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g)
                (void)hipGraphDestroy(g);
            return fail(AAR_ERR_DEVICE, std::string("graph capture: ") +
                                            hipGetErrorString(e != hipSuccess ? e : e2));
        }
        hipError_t e3 = hipGraphInstantiate(&S->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        AAR_HIP(e3);
        S->graph_cycles = kGraphCycles;
    }
    int64_t issued = 0;
    int inflight = 0, slot = 0;
    if (S->host_status == nullptr) {
        // no pinned status word (the allocation-free entry point): read the
        // run state after every group of cycles
        while (issued < needed) {
            for (int c = 0; c < kGraphCycles && issued < needed; ++c, ++issued) {
                hipError_t e = enqueue_any<T>(S, P, inner, s, issued);
                if (e != hipSuccess)
                    return fail(AAR_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e));
            }
            AAR_HIP(hipMemcpyAsync(out, S->state, sizeof(InstState), hipMemcpyDeviceToHost, s));
            AAR_HIP(hipStreamSynchronize(s));
            if (out->status != kRunning)
                break;
        }
        AAR_HIP(hipMemcpyAsync(out, S->state, sizeof(InstState), hipMemcpyDeviceToHost, s));
        AAR_HIP(hipStreamSynchronize(s));
        return AAR_OK;
    }
    while (issued < needed) {
        if (use_graph) {
            AAR_HIP(hipGraphLaunch(S->graph, s));
            issued += S->graph_cycles;
        } else {
            for (int c = 0; c < kGraphCycles && issued < needed; ++c, ++issued) {
                hipError_t e = enqueue_any<T>(S, P, inner, s, issued);
                if (e != hipSuccess)
                    return fail(AAR_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e));
            }
        }
        // every update kernel stores the run status into pinned host memory
        // (the latest one to run wins; a status that left kRunning stays so)
        AAR_HIP(hipEventRecord(S->poll_ev[slot], s));
        slot ^= 1;
        ++inflight;
        if (inflight == 2) {
            AAR_HIP(hipEventSynchronize(S->poll_ev[slot]));
            --inflight;
            if (*reinterpret_cast<volatile int32_t *>(S->host_status) != kRunning)
                break;
        }
    }
    AAR_HIP(hipStreamSynchronize(s));
    AAR_HIP(hipMemcpy(out, S->state, sizeof(InstState), hipMemcpyDeviceToHost));
    if (S->timing) {
        // count only sweeps that did work: cycles up to the last one that ran
        const int64_t last_k = out->status == kMaxIter || out->status == kRunning
                                   ? max_iter - 1
                                   : out->iters - 1;
        for (size_t t = 0; t < S->tcycle.size(); ++t) {
            if (S->tcycle[t] > last_k)
                continue;      // a group that stopped early (or never ran)
            float ms = 0.0f;
            AAR_HIP(hipEventElapsedTime(&ms, S->tev[2 * t], S->tev[2 * t + 1]));
            S->t_total_ms += ms;
            S->t_launches += S->tcount[t];
        }
        S->tcycle.clear();
        S->tcount.clear();
        S->tused = 0;
    }
    return AAR_OK;
}

aar_status status_of(const InstState &st)
{
    switch (st.status) {
    case kConverged:
        return AAR_OK;
    case kBreakdown:
        return AAR_BREAKDOWN;
    default:
        return AAR_NOT_CONVERGED;
    }
}

// Whether the Anderson-residual pass of this tile shape also forms the Gram
// products (the paired layout's fused variant: FP64 iterate, FP64 or FP32
// history, up to 8 waves, history length kFusedGramM); otherwise the separate
// Gram pass runs.
bool gram_fusable(const TileShape &ts, bool paired_fk, int m, bool f64, Prec hist)
{
    return paired_fk && m == kFusedGramM && ts.pair <= 2 && f64 && hist != Prec::F32_BF16;
}

// Point Path<T> at the workspace for system `idx`.
template <typename T> void bind_path_op(aar_solver_t *S, Path<T> &P, const Operator &op, bool f64)
{
    P.N = op.N;
    P.radius = op.prob.radius;
    P.conv = op.prob.velocity != nullptr;
    P.ts = op.ts[f64 ? 0 : 1];
    int tx, ty, tz, blocks;
    const bool paired_fk = paired_layout(P.ts, op.prob.n[0], P.conv, kFk);
    stencil_grid(op.prob.n[0], op.prob.n[1], op.prob.n[2], P.ts, &tx, &ty, &tz, &blocks, paired_fk);
    P.rho_blocks = blocks;
    P.gram_fused = gram_fusable(P.ts, paired_fk, S->params.m, f64, P.hist);
    // Residual recursion (iterate and ring of one type: FP64, or FP32 in the
    // inner solves of the mixed mode): within a cycle,
    // f_{j+1} = f_j - omega D^-1 A f_j from the ring, no x or b traffic; the
    // ring must hold the cycle's p f's, so m + 1 >= p
    P.recur = (f64 ? !S->mixed && P.hist == Prec::F64 : S->mixed && P.hist == Prec::F32) && S->params.p >= 2 &&
              S->params.m + 1 >= S->params.p;
    // FP64 iterate, FP32 ring: the same recursion, computed in FP32 on the
    // ring.  Its rounding (u32 |f| per step) restarts from the FP64 residual
    // of x and b at every cycle, so the convergence test on |D f_k| keeps its
    // FP64 meaning to ~1e-6 relative
    P.recur32 = f64 && !S->mixed && P.hist == Prec::F32 && S->params.p >= 2 && S->params.m + 1 >= S->params.p;
    if (P.recur32) {
        P.ts32 = op.ts[1];
        P.st32 = make_stencil<float>(op, op.vel32);
        int tx2, ty2, tz2, blocks2;
        stencil_grid(op.prob.n[0], op.prob.n[1], op.prob.n[2], P.ts32, &tx2, &ty2, &tz2, &blocks2,
                     paired_layout(P.ts32, op.prob.n[0], P.conv, kFk));
        P.rho_blocks32 = blocks2;
        P.gram_fused = false;   // the FP32 pass forms no Gram products
    }
    P.gram_blocks = gram_blocks(op.N, S->params.m);
    P.upd_blocks = stream_blocks(op.N);
    P.slot_stride = S->slot_stride[f64 ? 0 : 1];
    P.dx_stride = f64 ? S->dx_stride64 : S->dx_stride;
    if constexpr (std::is_same<T, double>::value)
        P.st = make_stencil<double>(op, op.vel64);
    else
        P.st = make_stencil<float>(op, op.vel32);
}

template <typename T> void bind_path(aar_solver_t *S, Path<T> &P, int idx, bool f64)
{
    bind_path_op(S, P, S->ops[idx], f64);
}

// Tile autotuner: time the Richardson sweep for each candidate tile height
// (rows per thread) and z depth on this grid, keep the fastest.  Results are
// cached per (precision, radius, convection, grid) for the process.  The
// cache is seeded from a tile file (AAR_TUNE_CACHE, else tuned_tiles.txt next
// to this library: lines "prec radius conv n0 n1 n2 rows_per_thread z_depth
// [order [pair]]", prec 0 = FP64, 1 = FP32, order the kOrder* bits, pair 1,
// 2, 3 for the paired layout with 256, 512, 1024 threads per workgroup, both
// default 0), so tuned shapes are reproducible;
// with
// AAR_TUNE_CACHE_WRITE set, new results are appended to that file.
std::mutex g_tune_mutex;
std::map<std::tuple<int, int, int, int, int, int>, TileShape> g_tune_cache;
bool g_tune_loaded = false;
std::string g_tune_path;

// Read the tile file once per path: a new AAR_TUNE_CACHE value is read when
// it is first seen, its lines overriding cached shapes of the same key.
void load_tune_file()
{
    std::string path;
    if (const char *env = getenv("AAR_TUNE_CACHE")) {
        path = env;
    } else {
        Dl_info info;
        if (dladdr((void *)&load_tune_file, &info) && info.dli_fname) {
            std::string lib = info.dli_fname;
            const size_t slash = lib.rfind('/');
            path = (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/tuned_tiles.txt";
        }
    }
    if (g_tune_loaded && path == g_tune_path)
        return;
    g_tune_loaded = true;
    g_tune_path = path;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#')
            continue;
        std::istringstream in(line);
        int prec, radius, conv, n0, n1, n2, ry, cz, order = 0, pair = 0, tb = 0;
        if (!(in >> prec >> radius >> conv >> n0 >> n1 >> n2 >> ry >> cz))
            continue;
        if (!(in >> order))
            order = 0;
        if (!(in >> pair))
            pair = 0;
        if (!(in >> tb))
            tb = 0;
        if ((ry != 1 && ry != 2 && ry != 4) || cz < 1 || order < 0 || order > 3 || tb < 0 ||
            tb > kTbMaxDepth || (tb >= 2 && pair != 0) || !paired_shape_ok(TileShape{ry, cz, order, pair}, prec == 0))
            continue;
        g_tune_cache[std::make_tuple(prec, radius, conv, n0, n1, n2)] = TileShape{ry, cz, order, pair, tb};
    }
}

void append_tune_file(const std::tuple<int, int, int, int, int, int> &key, const TileShape &ts)
{
    const char *path = getenv("AAR_TUNE_CACHE_WRITE");
    if (!path)
        return;
    std::ofstream f(path, std::ios::app);
    f << std::get<0>(key) << ' ' << std::get<1>(key) << ' ' << std::get<2>(key) << ' ' << std::get<3>(key) << ' '
      << std::get<4>(key) << ' ' << std::get<5>(key) << ' ' << ts.ry << ' ' << ts.cz << ' ' << ts.order << ' '
      << ts.pair << ' ' << ts.tb << '\n';
}

// Tile of the FP32 passes from the tile file, without timing candidates
// (the FP32 recursion passes of an FP64 iteration over an FP32 ring, whose
// solver holds no FP32 vectors to time them on).  A grid the file does not
// list takes the FP64 shape timed for it (every FP64 shape is a valid FP32
// one; temporal blocks are not used for these passes), which fills the chip
// as the fixed default shape may not on a small grid.
void cached_tile32(Operator &op)
{
    const auto key = std::make_tuple(1, op.prob.radius, op.prob.velocity != nullptr ? 1 : 0, op.prob.n[0],
                                     op.prob.n[1], op.prob.n[2]);
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    load_tune_file();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
        op.ts[1] = it->second;
    } else if (paired_shape_ok(op.ts[0], false)) {
        op.ts[1] = op.ts[0];
        op.ts[1].tb = 0;
    }
}

// Tile of the FP64 passes of a mixed-precision solver (the refinement
// residual, the operator apply): the tile file's FP64 line for the grid, else
// the FP32 shape timed for it, with the paired flag dropped where FP64 has no
// such tile.  The fixed default shape may leave most of the chip idle on a
// small grid.
void cached_tile64(Operator &op)
{
    const auto key = std::make_tuple(0, op.prob.radius, op.prob.velocity != nullptr ? 1 : 0, op.prob.n[0],
                                     op.prob.n[1], op.prob.n[2]);
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    load_tune_file();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
        op.ts[0] = it->second;
    } else {
        op.ts[0] = op.ts[1];
        op.ts[0].tb = 0;
        if (!paired_shape_ok(op.ts[0], true))
            op.ts[0].pair = 0;
    }
}

template <typename T> aar_status autotune(aar_solver_t *S, int idx)
{
    const bool f64 = std::is_same<T, double>::value;
    Operator &op = S->ops[idx];
    const auto key = std::make_tuple(f64 ? 0 : 1, op.prob.radius, op.prob.velocity != nullptr ? 1 : 0,
                                     op.prob.n[0], op.prob.n[1], op.prob.n[2]);
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        load_tune_file();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            op.ts[f64 ? 0 : 1] = it->second;
            return AAR_OK;
        }
    }
    Path<T> P;
    if constexpr (std::is_same<T, double>::value)
        P = S->p64;
    else
        P = S->p32;
    bind_path(S, P, idx, f64);
    hipStream_t s = S->stream;
    const int64_t N = op.N;
    if constexpr (std::is_same<T, double>::value) {
        AAR_HIP(launch_fill_pattern_f64(P.xa, N, s));
        AAR_HIP(launch_fill_pattern_f64(P.b, N, s));
    } else {
        AAR_HIP(launch_fill_pattern_f32(P.xa, N, s));
        AAR_HIP(launch_fill_pattern_f32(P.b, N, s));
    }
    const int nb_blocks = stream_blocks(N);
    AAR_HIP(launch_norm_partial(f64, P.b, N, S->part_norm, nb_blocks, s));
    AAR_HIP(launch_init_state(S->state, S->part_norm, nb_blocks, (int64_t)1 << 40, 1.0, s));
    hipEvent_t e0, e1;
    AAR_HIP(hipEventCreate(&e0));
    AAR_HIP(hipEventCreate(&e1));
    StencilArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.st = P.st;
    a.b = P.b;
    a.fring = P.fring;
    a.state = S->state;
    a.slot_stride = P.slot_stride;
    a.p = S->params.p;
    a.nslots = S->params.m + 1;
    a.omega = (T)S->params.omega;
    a.j = 0;
    a.x = P.xa;
    a.out = P.xb;
    float best_ms = 1e30f;
    TileShape best = P.ts;
    // candidates: rows per thread x z depth (skipping depths that give the
    // same grid as a smaller one) x order bits (none when there is one chunk)
    std::vector<TileShape> cands;
    for (int ry : {1, 2, 4}) {
        int prev_tz = -1;
        for (int cz : {2, 4, 6, 8, 12, 16, 20, 24, 28, 32, 40, 48, 64}) {
            int tx, ty, tz, blocks;
            stencil_grid(op.prob.n[0], op.prob.n[1], op.prob.n[2], TileShape{ry, cz, 0}, &tx, &ty, &tz, &blocks);
            if (tz == prev_tz)
                continue;
            prev_tz = tz;
            for (int order = 0; order < (tz > 1 ? 4 : 1); ++order) {
                const bool conv = op.prob.velocity != nullptr;
                for (int pair = 0; pair <= 3; ++pair) {
                    const TileShape ts{ry, cz, order, pair};
                    if (paired_shape_ok(ts, f64) && (pair == 0 || paired_layout(ts, op.prob.n[0], conv, kSweep)))
                        cands.push_back(ts);
                }
            }
        }
    }
    aar_status result = AAR_OK;
    for (const TileShape &ts : cands) {
        hipError_t e = hipSuccess;
        for (int w = 0; w < 3 && e == hipSuccess; ++w)
            e = Launch<T>::stencil(kSweep, P, a, s, ts);
        if (e == hipSuccess)
            e = hipEventRecord(e0, s);
        for (int w = 0; w < 10 && e == hipSuccess; ++w)
            e = Launch<T>::stencil(kSweep, P, a, s, ts);
        if (e == hipSuccess)
            e = hipEventRecord(e1, s);
        if (e == hipSuccess)
            e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            result = fail(AAR_ERR_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = ts;
        }
    }
    // Temporal block depth (one-point tiles of radius <= 2 with the residual
    // recursion): time a cycle's positions 1 .. p-1 (its later Richardson
    // steps and the Anderson-step residual) as one pass per step and as
    // blocks of 2 .. kTbMaxDepth steps; keep the fastest.
    P.ts = best;
    if (result == AAR_OK && best.pair == 0 && P.recur && !P.recur32 && S->params.p >= 3 && op.prob.radius <= 2) {
        const int p = S->params.p;
        a.partial = S->part_rho;
        a.j = 0;
        a.recur = 0;
        a.x = P.xa;
        a.out = nullptr;
        hipError_t e = Launch<T>::stencil(kSweep, P, a, s, best);   // ring slot 0 <- f_0
        auto group = [&](int depth) -> hipError_t {
            hipError_t ge = hipSuccess;
            StencilArgs<T> g = a;
            g.recur = 1;
            if (depth < 2) {
                for (int j = 1; j < p && ge == hipSuccess; ++j) {
                    g.j = j;
                    ge = Launch<T>::stencil(j < p - 1 ? kSweep : kFk, P, g, s, best);
                }
                return ge;
            }
            TileShape ts = best;
            ts.tb = depth;
            for (int j = 1; j < p && ge == hipSuccess;) {
                const int nt = std::min(depth, p - j);
                ge = launch_tblock<T>(P, g, j, nt, j + nt - 1 == p - 1, s, ts);
                j += nt;
            }
            return ge;
        };
        float best_group = 1e30f;
        for (int depth = 0; depth <= kTbMaxDepth && e == hipSuccess; ++depth) {
            if (depth == 1)
                continue;
            TileShape ts = best;
            ts.tb = depth;
            if (depth >= 2 && !tblock_fits(op.prob.radius, op.prob.velocity != nullptr, ts, std::min(depth, p - 1), f64))
                continue;
            for (int w = 0; w < 2 && e == hipSuccess; ++w)
                e = group(depth);
            if (e == hipSuccess)
                e = hipEventRecord(e0, s);
            for (int w = 0; w < 5 && e == hipSuccess; ++w)
                e = group(depth);
            if (e == hipSuccess)
                e = hipEventRecord(e1, s);
            if (e == hipSuccess)
                e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess)
                e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && ms < best_group) {
                best_group = ms;
                best.tb = depth;
            }
        }
        if (e != hipSuccess)
            result = fail(AAR_ERR_DEVICE, std::string("autotune (temporal blocks): ") + hipGetErrorString(e));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != AAR_OK)
        return result;
    op.ts[f64 ? 0 : 1] = best;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache[key] = best;
    append_tune_file(key, best);
    return AAR_OK;
}

// The FP64 iteration (also with an FP32 or bfloat16 history ring) of one
// system: x (FP64 device) holds x0 on entry and the answer on exit.
aar_status solve_fp64(aar_solver_t *S, const Operator &op, const double *b, double *x, aar_result *res,
                      bool use_graph, int32_t *log_count)
{
    const aar_params &pa = S->params;
    const int64_t N = op.N;
    hipStream_t s = S->stream;
    aar_result r{};
    InstState st{};
    Path<double> &P = S->p64;
    bind_path_op(S, P, op, true);
    if (P.rho_blocks > S->part_rho_cap || P.rho_blocks32 > S->part_rho_cap)
        return fail(AAR_ERR_DEVICE, "stencil grid exceeds the partial-sum workspace");
    AAR_HIP(hipMemcpyAsync(P.b, b, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    AAR_HIP(hipMemcpyAsync(P.xa, x, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    const int nb_blocks = stream_blocks(N);
    if (pa.flags & AAR_FLAG_DEFLATE_CONSTANT) {
        // x_0 += mean(b - A x_0) / sigma; the first history slot is scratch here
        double *r = static_cast<double *>(P.fring);
        StencilArgs<double> ra;
        std::memset(&ra, 0, sizeof(ra));
        ra.st = P.st;
        ra.x = P.xa;
        ra.b = P.b;
        ra.out = r;
        ra.partial = S->part_rho;
        AAR_HIP(launch_stencil_f64(kResid, Prec::F64, P.radius, P.conv, P.ts, ra, nullptr, s));
        AAR_HIP(launch_deflate(P.xa, r, N, 1.0 / op.prob.shift, S->part_norm, nb_blocks, S->scal, s));
    }
    AAR_HIP(launch_norm_partial(true, P.b, N, S->part_norm, nb_blocks, s));
    AAR_HIP(launch_init_state(S->state, S->part_norm, nb_blocks, pa.max_iter, pa.tol, s));
    AAR_HIP(hipMemcpyAsync(&st, S->state, sizeof(InstState), hipMemcpyDeviceToHost, s));
    AAR_HIP(hipStreamSynchronize(s));
    if (st.nb == 0.0) {
        AAR_HIP(launch_zero_f64(x, N, s));
        AAR_HIP(hipStreamSynchronize(s));
        r.status = AAR_OK;
        if (res)
            *res = r;
        *log_count = 0;
        return AAR_OK;
    }
    aar_status e = run_cycles<double>(S, P, pa.max_iter, false, use_graph, &st);
    if (e != AAR_OK)
        return e;
    if (P.recur || P.recur32) {
        // the sweeps wrote no x: add the unfinished cycle's Richardson steps
        AAR_HIP(launch_finalize_f64(P.hist, P.xa, P.fring, S->state, pa.p, pa.m + 1, P.slot_stride, pa.omega, N,
                                    s));
        AAR_HIP(hipMemcpyAsync(x, P.xa, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        AAR_HIP(hipStreamSynchronize(s));
        r.status = status_of(st);
        r.iterations = (st.status == kMaxIter || st.status == kRunning) ? pa.max_iter : st.iters;
        r.rel_residual = st.last_r;
        r.outer_steps = 0;
        *log_count = st.log_count;
        if (res)
            *res = r;
        return (aar_status)r.status;
    }
    // where x ended: after j sweeps of a cycle it is in xb when j is odd
    const int64_t done = (st.status == kMaxIter || st.status == kRunning) ? pa.max_iter : st.iters;
    const int64_t j = (done - 1) % pa.p;     // last iteration's position in its cycle
    const bool anderson_last = (st.status == kMaxIter || st.status == kRunning) && j == pa.p - 1;
    const double *xf;
    if (st.status == kConverged || st.status == kBreakdown)
        xf = ((pa.p - 1) & 1) ? P.xb : P.xa;     // x_k of the Anderson step
    else if (anderson_last)
        xf = P.xa;                              // the last iteration was an update
    else
        xf = ((j + 1) & 1) ? P.xb : P.xa;       // after j+1 sweeps of the cycle
    AAR_HIP(hipMemcpyAsync(x, xf, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    AAR_HIP(hipStreamSynchronize(s));
    r.status = status_of(st);
    r.iterations = (st.status == kMaxIter || st.status == kRunning) ? pa.max_iter : st.iters;
    r.rel_residual = st.last_r;
    r.outer_steps = 0;
    *log_count = st.log_count;
    if (res)
        *res = r;
    return (aar_status)r.status;
}

// Complex system: x (2N doubles, interleaved) holds x0 on entry and the answer on exit.
aar_status solve_complex(aar_solver_t *S, const double *b, double *x, aar_result *res)
{
    const aar_params &pa = S->params;
    Path<zd> &P = S->pz;
    const int64_t N = P.N;
    hipStream_t s = S->stream;
    const bool use_graph = !(pa.flags & AAR_FLAG_NO_GRAPH) && !S->timing;
    aar_result r{};
    InstState st{};
    AAR_HIP(hipMemcpyAsync(P.b, b, sizeof(zd) * N, hipMemcpyDeviceToDevice, s));
    AAR_HIP(hipMemcpyAsync(P.xa, x, sizeof(zd) * N, hipMemcpyDeviceToDevice, s));
    const int nb_blocks = stream_blocks(N);
    AAR_HIP(launch_cnorm_partial(P.b, N, S->part_norm, nb_blocks, s));
    AAR_HIP(launch_init_state(S->state, S->part_norm, nb_blocks, pa.max_iter, pa.tol, s));
    AAR_HIP(hipMemcpyAsync(&st, S->state, sizeof(InstState), hipMemcpyDeviceToHost, s));
    AAR_HIP(hipStreamSynchronize(s));
    if (st.nb == 0.0) {
        AAR_HIP(launch_zero_f64(x, 2 * N, s));
        AAR_HIP(hipStreamSynchronize(s));
        r.status = AAR_OK;
        if (res)
            *res = r;
        S->last_log_count[0] = 0;
        return AAR_OK;
    }
    aar_status e = run_cycles<zd>(S, P, pa.max_iter, false, use_graph, &st);
    if (e != AAR_OK)
        return e;
    const int64_t done = (st.status == kMaxIter || st.status == kRunning) ? pa.max_iter : st.iters;
    const int64_t j = (done - 1) % pa.p;
    const bool anderson_last = (st.status == kMaxIter || st.status == kRunning) && j == pa.p - 1;
    const zd *xf;
    if (st.status == kConverged || st.status == kBreakdown)
        xf = ((pa.p - 1) & 1) ? P.xb : P.xa;
    else if (anderson_last)
        xf = P.xa;
    else
        xf = ((j + 1) & 1) ? P.xb : P.xa;
    AAR_HIP(hipMemcpyAsync(x, xf, sizeof(zd) * N, hipMemcpyDeviceToDevice, s));
    AAR_HIP(hipStreamSynchronize(s));
    r.status = status_of(st);
    r.iterations = done;
    r.rel_residual = st.last_r;
    r.outer_steps = 0;
    S->last_log_count[0] = st.log_count;
    if (res)
        *res = r;
    return (aar_status)r.status;
}

// General sparse system: x holds x0 on entry and the answer on exit.
aar_status solve_csr(aar_solver_t *S, const double *b, double *x, aar_result *res)
{
    const aar_params &pa = S->params;
    Path<double> &P = S->p64;
    const int64_t N = P.N;
    hipStream_t s = S->stream;
    const bool use_graph = !(pa.flags & AAR_FLAG_NO_GRAPH) && !S->timing;
    aar_result r{};
    InstState st{};
    AAR_HIP(hipMemcpyAsync(P.b, b, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    AAR_HIP(hipMemcpyAsync(P.xa, x, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    const int nb_blocks = stream_blocks(N);
    AAR_HIP(launch_norm_partial(true, P.b, N, S->part_norm, nb_blocks, s));
    AAR_HIP(launch_init_state(S->state, S->part_norm, nb_blocks, pa.max_iter, pa.tol, s));
    AAR_HIP(hipMemcpyAsync(&st, S->state, sizeof(InstState), hipMemcpyDeviceToHost, s));
    AAR_HIP(hipStreamSynchronize(s));
    if (st.nb == 0.0) {
        AAR_HIP(launch_zero_f64(x, N, s));
        AAR_HIP(hipStreamSynchronize(s));
        r.status = AAR_OK;
        if (res)
            *res = r;
        S->last_log_count[0] = 0;
        return AAR_OK;
    }
    aar_status e = run_cycles<double>(S, P, pa.max_iter, false, use_graph, &st);
    if (e != AAR_OK)
        return e;
    const int64_t done = (st.status == kMaxIter || st.status == kRunning) ? pa.max_iter : st.iters;
    const int64_t j = (done - 1) % pa.p;
    const bool anderson_last = (st.status == kMaxIter || st.status == kRunning) && j == pa.p - 1;
    const double *xf;
    if (st.status == kConverged || st.status == kBreakdown)
        xf = ((pa.p - 1) & 1) ? P.xb : P.xa;     // x_k of the Anderson step
    else if (anderson_last)
        xf = P.xa;                              // the last iteration was an update
    else
        xf = ((j + 1) & 1) ? P.xb : P.xa;       // after j+1 sweeps of the cycle
    AAR_HIP(hipMemcpyAsync(x, xf, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    AAR_HIP(hipStreamSynchronize(s));
    r.status = status_of(st);
    r.iterations = done;
    r.rel_residual = st.last_r;
    r.outer_steps = 0;
    S->last_log_count[0] = st.log_count;
    if (res)
        *res = r;
    return (aar_status)r.status;
}

// Block bounds and level schedules of a sparse matrix (host, at creation).
// Rows of a block are grouped by the level of their forward substitution
// (0 when no earlier row of the block enters the row; else one more than the
// deepest such row) and, separately, of the backward substitution (the same
// with later rows).  Rows of one level never depend on each other.
struct CsrPlan {
    std::vector<int64_t> dpos, bstart;
    std::vector<int32_t> lrows, urows, lptr, uptr, blev_l, blev_u;
    int max_block_rows = 0;
    // packed substitution records (kp slots per row; kp = 0: none): block-
    // local rows and columns, and the CSR entry of each slot (-1: padding)
    int kp = 0;
    std::vector<int16_t> frow, fcol, brow, bcol;
    std::vector<int32_t> fe, be;
};

// Packed records of the substitutions, in the order of lrows and urows:
// each row's in-block entries below (above) the diagonal in increasing
// column order.  Left empty (kp = 0) when a row has more than kCsrMaxPack
// such entries or the entry indices exceed 32 bits.
void pack_csr(int64_t n, const int64_t *rowptr, const int32_t *col, CsrPlan *pl)
{
    pl->kp = 0;
    const int nblocks = (int)pl->bstart.size() - 1;
    if (rowptr[n] > INT32_MAX)
        return;
    std::vector<int64_t> blk_lo(n);
    for (int t = 0; t < nblocks; ++t)
        for (int64_t i = pl->bstart[t]; i < pl->bstart[t + 1]; ++i)
            blk_lo[i] = t;
    int kl = 0, ku = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t lo = pl->bstart[blk_lo[i]], hi = pl->bstart[blk_lo[i] + 1];
        int cl = 0, cu = 0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            cl += col[e] >= lo && col[e] < i;
            cu += col[e] > i && col[e] < hi;
        }
        kl = std::max(kl, cl);
        ku = std::max(ku, cu);
    }
    const int k = std::max(kl, ku);
    if (k > kCsrMaxPack)
        return;
    pl->kp = k <= 4 ? 4 : 8;
    const int kp = pl->kp;
    auto fill = [&](const std::vector<int32_t> &rows, bool upper, std::vector<int16_t> &prow,
                    std::vector<int16_t> &pcol, std::vector<int32_t> &pe) {
        prow.assign(n, -1);
        pcol.assign((size_t)n * kp, -1);
        pe.assign((size_t)n * kp, -1);
        for (int64_t q = 0; q < n; ++q) {
            const int64_t i = rows[q];
            const int64_t lo = pl->bstart[blk_lo[i]], hi = pl->bstart[blk_lo[i] + 1];
            prow[q] = (int16_t)(i - lo);
            int sl = 0;
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                const bool in = upper ? (col[e] > i && col[e] < hi) : (col[e] >= lo && col[e] < i);
                if (!in)
                    continue;
                pcol[q * kp + sl] = (int16_t)(col[e] - lo);
                pe[q * kp + sl] = (int32_t)e;
                ++sl;
            }
        }
    };
    fill(pl->lrows, false, pl->frow, pl->fcol, pl->fe);
    fill(pl->urows, true, pl->brow, pl->bcol, pl->be);
}

void plan_csr(int64_t n, const int64_t *rowptr, const int32_t *col, int nblocks, bool levels, CsrPlan *pl)
{
    pl->dpos.assign(n, -1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (col[e] == i)
                pl->dpos[i] = e;
    pl->bstart.resize(nblocks + 1);
    for (int t = 0; t <= nblocks; ++t)
        pl->bstart[t] = (int64_t)t * n / nblocks;
    pl->max_block_rows = 0;
    for (int t = 0; t < nblocks; ++t)
        pl->max_block_rows = std::max<int64_t>(pl->max_block_rows, pl->bstart[t + 1] - pl->bstart[t]);
    pl->lrows.clear();
    pl->urows.clear();
    pl->lptr.assign(1, 0);
    pl->uptr.assign(1, 0);
    pl->blev_l.assign(1, 0);
    pl->blev_u.assign(1, 0);
    if (!levels)
        return;
    pl->lrows.reserve(n);
    pl->urows.reserve(n);
    std::vector<int32_t> lev(n);
    auto group = [&](int64_t lo, int64_t hi, int32_t top, std::vector<int32_t> &rows, std::vector<int32_t> &ptr,
                     std::vector<int32_t> &blev) {
        std::vector<int32_t> cnt(top + 1, 0);
        for (int64_t i = lo; i < hi; ++i)
            ++cnt[lev[i]];
        const int32_t base = (int32_t)rows.size();
        std::vector<int32_t> pos(top + 1);
        int32_t run = base;
        for (int32_t v = 0; v <= top; ++v) {
            pos[v] = run;
            run += cnt[v];
            ptr.push_back(run);
        }
        rows.resize(run);
        for (int64_t i = lo; i < hi; ++i)
            rows[pos[lev[i]]++] = (int32_t)i;
        blev.push_back((int32_t)ptr.size() - 1);
    };
    for (int t = 0; t < nblocks; ++t) {
        const int64_t lo = pl->bstart[t], hi = pl->bstart[t + 1];
        int32_t top = 0;
        for (int64_t i = lo; i < hi; ++i) {
            int32_t v = 0;
            for (int64_t e = rowptr[i]; e < pl->dpos[i]; ++e)
                if (col[e] >= lo)
                    v = std::max(v, lev[col[e]] + 1);
            lev[i] = v;
            top = std::max(top, v);
        }
        group(lo, hi, top, pl->lrows, pl->lptr, pl->blev_l);
        top = 0;
        for (int64_t i = hi - 1; i >= lo; --i) {
            int32_t v = 0;
            for (int64_t e = pl->dpos[i] + 1; e < rowptr[i + 1] && col[e] < hi; ++e)
                v = std::max(v, lev[col[e]] + 1);
            lev[i] = v;
            top = std::max(top, v);
        }
        group(lo, hi, top, pl->urows, pl->uptr, pl->blev_u);
    }
}

// x (length N, FP64 device) on entry x0, on exit the answer of system idx.
aar_status solve_one(aar_solver_t *S, int idx, const double *b, double *x, aar_result *res)
{
    const aar_params &pa = S->params;
    const Operator &op = S->ops[idx];
    const int64_t N = op.N;
    hipStream_t s = S->stream;
    const bool use_graph = !(pa.flags & AAR_FLAG_NO_GRAPH) && !S->timing && S->ops.size() == 1;
    if (S->graph && S->graph_instance != idx) {
        (void)hipGraphExecDestroy(S->graph);
        S->graph = nullptr;
    }
    S->graph_instance = idx;
    S->last_instance = idx;
    aar_result r{};
    InstState st{};

    if (!S->mixed) {
        int32_t lc = 0;
        const aar_status e = solve_fp64(S, op, b, x, res, use_graph, &lc);
        S->last_log_count[idx] = lc;
        return e;
    }

    // ---- mixed precision: FP64 refinement around FP32 AAR ----
    Path<float> &P = S->p32;
    bind_path(S, P, idx, false);
    Path<double> R64;
    bind_path(S, R64, idx, true);
    if (P.rho_blocks > S->part_rho_cap || R64.rho_blocks > S->part_rho_cap)
        return fail(AAR_ERR_DEVICE, "stencil grid exceeds the partial-sum workspace");
    AAR_HIP(hipMemcpyAsync(S->b64, b, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    AAR_HIP(hipMemcpyAsync(S->x64, x, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    const int nb_blocks = stream_blocks(N);
    AAR_HIP(launch_norm_partial(true, S->b64, N, S->part_norm, nb_blocks, s));
    AAR_HIP(launch_finish_norm(S->scal + 1, S->part_norm, nb_blocks, s));
    double host_scal[2];
    AAR_HIP(hipMemcpyAsync(host_scal, S->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    AAR_HIP(hipStreamSynchronize(s));
    const double nb = host_scal[1];
    if (nb == 0.0) {
        AAR_HIP(launch_zero_f64(x, N, s));
        AAR_HIP(hipStreamSynchronize(s));
        r.status = AAR_OK;
        if (res)
            *res = r;
        S->last_log_count[idx] = 0;
        return AAR_OK;
    }
    const int max_outer = pa.max_outer > 0 ? pa.max_outer : 30;
    const bool recycle = (pa.flags & AAR_FLAG_RECYCLE_HISTORY) != 0;
    int64_t used = 0;
    int outer = 0;
    aar_status final = AAR_NOT_CONVERGED;
    double rel = 0.0;
    for (;;) {
        // r = b - A x in FP64 and its norm
        StencilArgs<double> ra;
        std::memset(&ra, 0, sizeof(ra));
        ra.st = R64.st;
        ra.x = S->x64;
        ra.b = S->b64;
        ra.out = S->r64;
        ra.partial = S->part_rho;
        // one partial per workgroup of this launch: the residual pass always
        // runs the one-point layout, whose grid differs from the paired one
        // that R64.rho_blocks counts when the tile has the paired flag
        int rtx, rty, rtz, resid_blocks = 0;
        stencil_grid(op.prob.n[0], op.prob.n[1], op.prob.n[2], R64.ts, &rtx, &rty, &rtz, &resid_blocks);
        if (resid_blocks > S->part_rho_cap)
            return fail(AAR_ERR_DEVICE, "residual grid exceeds the partial-sum workspace");
        AAR_HIP(launch_stencil_f64(kResid, Prec::F64, R64.radius, R64.conv, R64.ts, ra, &resid_blocks, s));
        if (pa.flags & AAR_FLAG_DEFLATE_CONSTANT) {
            AAR_HIP(launch_deflate(S->x64, S->r64, N, 1.0 / op.prob.shift, S->part_norm, nb_blocks, S->scal, s));
            AAR_HIP(launch_finish_norm(S->scal, S->part_norm, nb_blocks, s));
        } else {
            AAR_HIP(launch_finish_norm(S->scal, S->part_rho, resid_blocks, s));
        }
        AAR_HIP(hipMemcpyAsync(host_scal, S->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        AAR_HIP(hipStreamSynchronize(s));
        rel = host_scal[0] / nb;
        if (!std::isfinite(rel)) {
            final = AAR_BREAKDOWN;
            break;
        }
        if (rel < pa.tol) {
            final = AAR_OK;
            break;
        }
        if (outer >= max_outer || used >= pa.max_iter) {
            final = AAR_NOT_CONVERGED;
            break;
        }
        // inner FP32 AAR on A d = r / ||r||, d_0 = 0
        const double inner_tol = inner_tolerance(pa.inner_tol, pa.tol, rel);
        AAR_HIP(launch_cast_f64_to_f32(S->r64, P.b, N, S->scal, s));
        AAR_HIP(launch_zero_f32(P.xa, N, s));
        AAR_HIP(launch_norm_partial(false, P.b, N, S->part_norm, nb_blocks, s));
        const int64_t budget = pa.max_iter - used;
        // with AAR_FLAG_RECYCLE_HISTORY the inner runs after the first keep the
        // history of the previous one: its difference pairs satisfy
        // dF = -D^-1 A dX whatever the right-hand side, so they remain valid
        // extrapolation directions for the next correction equation
        const bool keep = recycle && outer > 0;
        const int64_t start = keep ? (st.cycle + 1) * pa.p : 0;   // the run's first position
        if (keep)
            AAR_HIP(launch_init_state_keep(S->state, S->part_norm, nb_blocks, budget, inner_tol, pa.p, s));
        else
            AAR_HIP(launch_init_state(S->state, S->part_norm, nb_blocks, budget, inner_tol, s));
        aar_status e = run_cycles<float>(S, P, start + budget, true, use_graph, &st);
        if (e != AAR_OK)
            return e;
        if (st.status == kBreakdown) {
            final = AAR_BREAKDOWN;
            used += st.iters - start;
            break;
        }
        const int64_t done = (st.status == kMaxIter || st.status == kRunning) ? budget : st.iters - start;
        used += done;
        const int64_t j = (done - 1) % pa.p;
        const bool anderson_last = (st.status == kMaxIter || st.status == kRunning) && j == pa.p - 1;
        const float *df;
        if (P.recur) {
            // the sweeps wrote no x: add the unfinished cycle's Richardson steps
            AAR_HIP(launch_finalize_f32(P.xa, P.fring, S->state, pa.p, pa.m + 1, P.slot_stride, (float)pa.omega, N,
                                        s));
            df = P.xa;
        } else if (st.status == kConverged || st.status == kStagnated)
            df = ((pa.p - 1) & 1) ? P.xb : P.xa;
        else if (anderson_last)
            df = P.xa;
        else
            df = ((j + 1) & 1) ? P.xb : P.xa;
        AAR_HIP(launch_correct(S->x64, df, S->scal, N, s));
        ++outer;
    }
    AAR_HIP(hipMemcpyAsync(x, S->x64, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    AAR_HIP(hipStreamSynchronize(s));
    r.status = final;
    r.iterations = used;
    r.outer_steps = outer;
    r.rel_residual = rel;
    S->last_log_count[idx] = st.log_count;
    if (res)
        *res = r;
    return final;
}


// ---------------------------------------------------------------------------
// Batched engine
// ---------------------------------------------------------------------------
constexpr int kBatchGraphCycles = 8;
constexpr int kBatchGrid = 8192;

// The batched engine needs one stencil radius and convection kind for all
// systems and a history the register Gram kernels hold (m <= 12); other
// batches are solved one system after another.
bool batch_eligible(const aar_problem *probs, int count, const aar_params *pa)
{
    if (count < 2 || pa->m > kFastGramM)
        return false;
    for (int i = 1; i < count; ++i) {
        if (probs[i].radius != probs[0].radius || (probs[i].velocity != nullptr) != (probs[0].velocity != nullptr))
            return false;
    }
    return true;
}

// Tile of the batched stencil passes (one-point layout): the tile file's
// batch line (grid fields 0 0 0) for this precision, radius and convection,
// else z depth 32 with 2 rows per thread (FP64 iterate) or 4 (FP32 iterate),
// the fastest of rows {1, 2, 4} x depth {4, 8, 16, 32} on the 512-system
// Helmholtz batch.
TileShape batch_tile(const aar_params *pa, int radius, bool conv)
{
    const bool mixed = is_mixed(pa->precision);
    TileShape ts{mixed ? 4 : 2, 32, 0, 0};
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    load_tune_file();
    const auto it = g_tune_cache.find(std::make_tuple(mixed ? 1 : 0, radius, conv ? 1 : 0, 0, 0, 0));
    if (it != g_tune_cache.end()) {
        ts.ry = it->second.ry;
        ts.cz = it->second.cz;
    }
    return ts;
}

template <typename T> BatchDesc<T> batch_desc(const Operator &op, int64_t off, const TileShape &bt, const T *vel)
{
    BatchDesc<T> d;
    std::memset(&d, 0, sizeof(d));
    d.st = make_stencil<T>(op, vel);
    d.off = off;
    TileShape ts{bt.ry, std::min(bt.cz, op.prob.n[2])};
    int tx, ty, tz, blocks;
    stencil_grid(op.prob.n[0], op.prob.n[1], op.prob.n[2], ts, &tx, &ty, &tz, &blocks);
    d.tiles_x = tx;
    d.tiles_y = ty;
    d.tiles_z = tz;
    d.cz = ts.cz;
    d.ntiles = blocks;
    d.nchunks = (int)((op.N + kChunk - 1) / kChunk);
    return d;
}

size_t batch_bytes(const aar_problem *probs, int count, const aar_params *pa)
{
    int64_t total = 0;
    int64_t tiles = 0, chunks = 0;
    const TileShape bt = batch_tile(pa, probs[0].radius, probs[0].velocity != nullptr);
    for (int i = 0; i < count; ++i) {
        const int64_t N = (int64_t)probs[i].n[0] * probs[i].n[1] * probs[i].n[2];
        total += (N + 15) / 16 * 16;
        int tx, ty, tz, blocks;
        stencil_grid(probs[i].n[0], probs[i].n[1], probs[i].n[2], TileShape{bt.ry, std::min(bt.cz, probs[i].n[2])},
                     &tx, &ty, &tz, &blocks);
        tiles += blocks;
        chunks += (N + kChunk - 1) / kChunk;
    }
    const int slots = pa->m + 1, q = pa->m / pa->p, ne = pa->m * (pa->m + 1) / 2 + pa->m;
    size_t b = 0;
    if (!is_mixed(pa->precision)) {
        const Prec h = hist_of(pa->precision);
        b += (size_t)total * (8 * 3 + (h == Prec::F32 ? 4 : 8) * q + hist_bytes(h) * slots + (h == Prec::F32_BF16 ? 8 : 0));
    } else
        b += (size_t)total * (4 * (3 + q) + hist_bytes(pa->precision == AAR_MIXED_FP32 ? Prec::F32 : Prec::F32_BF16) * slots +
                              8 * 3 + (pa->precision == AAR_MIXED_FP32_BF16HIST ? 4 : 0));
    b += sizeof(double) * (size_t)(2 * tiles + chunks * (ne + 1));
    b += (sizeof(int2) * 2 + sizeof(int) * 4) * (size_t)(tiles + chunks + count);
    b += (sizeof(InstState) + sizeof(BatchCtl) + sizeof(BatchDesc<double>) + sizeof(BatchDesc<float>) + 64) * count;
    if (pa->flags & AAR_FLAG_RECORD_RESIDUALS)
        b += (sizeof(double) + sizeof(int32_t)) * (size_t)std::min<int64_t>(pa->max_iter / pa->p + 2, (int64_t)1 << 16) *
             count;
    return b;
}

aar_status batch_setup(aar_solver_t *S)
{
    auto &B = S->B;
    const aar_params &pa = S->params;
    const int count = (int)S->ops.size();
    aar_status st = AAR_OK;
    B.on = true;
    B.count = count;
    B.radius = S->ops[0].prob.radius;
    B.conv = S->ops[0].prob.velocity != nullptr;
    const TileShape bt = batch_tile(&pa, B.radius, B.conv);
    B.ry = bt.ry;
    B.offs.resize(count);
    B.sizes.resize(count);
    B.ntiles.resize(count);
    B.nchunks.resize(count);
    std::vector<BatchDesc<double>> d64(count);
    std::vector<BatchDesc<float>> d32(count);
    std::vector<double> invshift(count);
    int64_t total = 0;
    for (int i = 0; i < count; ++i) {
        const Operator &op = S->ops[i];
        B.offs[i] = total;
        B.sizes[i] = op.N;
        total += (op.N + 15) / 16 * 16;
        d64[i] = batch_desc<double>(op, B.offs[i], bt, op.vel64);
        d32[i] = batch_desc<float>(op, B.offs[i], bt, op.vel32);
        B.ntiles[i] = d64[i].ntiles;
        B.nchunks[i] = d64[i].nchunks;
        B.sum_tiles += B.ntiles[i];
        B.sum_chunks += B.nchunks[i];
        invshift[i] = op.prob.shift > 0.0 ? 1.0 / op.prob.shift : 0.0;
    }
    B.total = total;
    B.stride = total;
    B.grid_s = std::min(B.sum_tiles, kBatchGrid);
    B.grid_c = std::min(B.sum_chunks, kBatchGrid);
    const int slots = pa.m + 1;
    const int ne = S->ne;
    B.desc64 = S->alloc<BatchDesc<double>>(count, &st);
    B.desc32 = S->alloc<BatchDesc<float>>(count, &st);
    B.d_offs = S->alloc<int64_t>(count, &st);
    B.d_sizes = S->alloc<int64_t>(count, &st);
    B.d_uoffs = S->alloc<int64_t>(count, &st);
    B.d_ntiles = S->alloc<int>(count, &st);
    B.d_nchunks = S->alloc<int>(count, &st);
    B.d_invshift = S->alloc<double>(count, &st);
    B.ctl = S->alloc<BatchCtl>(count, &st);
    B.state = S->alloc<InstState>(count, &st);
    B.refine = S->alloc<int>(count, &st);
    B.remaining = S->alloc<int>(1, &st);
    B.c_s = S->alloc<int2>(B.sum_tiles, &st);
    B.a_s = S->alloc<int2>(B.sum_tiles, &st);
    B.c_c = S->alloc<int2>(B.sum_chunks, &st);
    B.a_c = S->alloc<int2>(B.sum_chunks, &st);
    B.c_n = S->alloc<int>(2, &st);
    B.a_n = S->alloc<int>(2, &st);
    B.c_sb = S->alloc<int>(count, &st);
    B.c_cb = S->alloc<int>(count, &st);
    B.a_sb = S->alloc<int>(count, &st);
    B.a_cb = S->alloc<int>(count, &st);
    B.p_rho = S->alloc<double>(B.sum_tiles, &st);
    B.p_s = S->alloc<double>(B.sum_tiles, &st);
    B.p_gram = S->alloc<double>((size_t)B.sum_chunks * ne, &st);
    B.p_c = S->alloc<double>(B.sum_chunks, &st);
    if (st != AAR_OK)
        return st;
    // as for one system: the recursion needs a ring of the iterate's type
    // (FP64, or FP32 for mixed inner solves) that holds a cycle's p f's
    B.recur = (S->mixed ? S->hist == Prec::F32 : S->hist == Prec::F64) && S->params.p >= 2 &&
              S->params.m + 1 >= S->params.p;
    B.recur32 = !S->mixed && S->hist == Prec::F32 && S->params.p >= 2 && S->params.m + 1 >= S->params.p;
    if (!S->mixed) {
        B.xa64 = S->alloc<double>(total, &st);
        B.xb64 = S->alloc<double>(total, &st);
        B.b64 = S->alloc<double>(total, &st);
        if (S->hist == Prec::F64) {
            B.fring = S->alloc<double>((size_t)total * slots, &st);
        } else {
            B.fring = S->hist == Prec::F32 ? (void *)S->alloc<float>((size_t)total * slots, &st)
                                           : (void *)S->alloc<bf16_t>((size_t)total * slots, &st);
            if (S->hist == Prec::F32_BF16)
                B.fcur64 = S->alloc<double>(total, &st);
        }
        if (S->q > 0)
            B.dx64 = S->hist == Prec::F32 ? (void *)S->alloc<float>((size_t)total * S->q, &st)
                                          : (void *)S->alloc<double>((size_t)total * S->q, &st);
    } else {
        B.xa64 = S->alloc<double>(total, &st);      // x in FP64 (refinement)
        B.b64 = S->alloc<double>(total, &st);
        B.r64 = S->alloc<double>(total, &st);
        B.xa32 = S->alloc<float>(total, &st);
        B.xb32 = S->alloc<float>(total, &st);
        B.rhs32 = S->alloc<float>(total, &st);
        if (S->hist == Prec::F32_BF16) {
            B.fring = S->alloc<bf16_t>((size_t)total * slots, &st);
            B.fcur32 = S->alloc<float>(total, &st);
        } else {
            B.fring = S->alloc<float>((size_t)total * slots, &st);
        }
        B.dx32 = S->q > 0 ? S->alloc<float>((size_t)total * S->q, &st) : nullptr;
    }
    if (pa.flags & AAR_FLAG_RECORD_RESIDUALS) {
        S->log_cap = std::min<int64_t>(pa.max_iter / pa.p + 2, (int64_t)1 << 16);
        B.log = S->alloc<double>((size_t)S->log_cap * count, &st);
        B.rank_log = S->alloc<int32_t>((size_t)S->log_cap * count, &st);
    }
    if (st != AAR_OK)
        return st;
    hipStream_t s = S->stream;
    AAR_HIP(hipMemcpyAsync(B.desc64, d64.data(), sizeof(BatchDesc<double>) * count, hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemcpyAsync(B.desc32, d32.data(), sizeof(BatchDesc<float>) * count, hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemcpyAsync(B.d_offs, B.offs.data(), sizeof(int64_t) * count, hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemcpyAsync(B.d_sizes, B.sizes.data(), sizeof(int64_t) * count, hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemcpyAsync(B.d_ntiles, B.ntiles.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemcpyAsync(B.d_nchunks, B.nchunks.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemcpyAsync(B.d_invshift, invshift.data(), sizeof(double) * count, hipMemcpyHostToDevice, s));
    AAR_HIP(hipHostMalloc((void **)&B.h_remaining, 2 * sizeof(int), hipHostMallocDefault));
    AAR_HIP(hipStreamSynchronize(s));
    return AAR_OK;
}

CompactArgs batch_compact_args(aar_solver_t *S, int mode, bool cycle_lists)
{
    auto &B = S->B;
    CompactArgs c;
    c.mode = mode;
    c.count = B.count;
    c.ctl = B.ctl;
    c.state = B.state;
    c.refine = B.refine;
    c.ntiles = B.d_ntiles;
    c.nchunks = B.d_nchunks;
    c.sitems = cycle_lists ? B.c_s : B.a_s;
    c.citems = cycle_lists ? B.c_c : B.a_c;
    c.nsitems = cycle_lists ? B.c_n : B.a_n;
    c.ncitems = cycle_lists ? B.c_n + 1 : B.a_n + 1;
    c.sbase = cycle_lists ? B.c_sb : B.a_sb;
    c.cbase = cycle_lists ? B.c_cb : B.a_cb;
    return c;
}

BatchStreamArgs batch_stream(aar_solver_t *S, int op, const int *mask, int mask_min)
{
    auto &B = S->B;
    BatchStreamArgs a;
    std::memset(&a, 0, sizeof(a));
    a.items = B.a_c;
    a.nitems = B.a_n + 1;
    a.op = op;
    a.mask = mask;
    a.mask_min = mask_min;
    a.ctl = B.ctl;
    a.offs = B.d_offs;
    a.sizes = B.d_sizes;
    a.uoffs = B.d_uoffs;
    a.inv_shift = B.d_invshift;
    return a;
}

BatchCtlArgs batch_ctl(aar_solver_t *S, int step, const double *partial, bool deflate)
{
    auto &B = S->B;
    const aar_params &pa = S->params;
    BatchCtlArgs c;
    std::memset(&c, 0, sizeof(c));
    c.step = step;
    c.p = pa.p;
    c.mixed = S->mixed ? 1 : 0;
    c.deflate = deflate ? 1 : 0;
    c.max_outer = pa.max_outer > 0 ? pa.max_outer : 30;
    c.max_iter = pa.max_iter;
    c.tol = pa.tol;
    c.inner_tol = pa.inner_tol;   // 0: the per-step rule of inner_tolerance
    c.ctl = B.ctl;
    c.state = B.state;
    c.refine = B.refine;
    c.remaining = B.remaining;
    c.partial = partial;
    c.sbase = B.a_sb;
    c.cbase = B.a_cb;
    c.ntiles = B.d_ntiles;
    c.nchunks = B.d_nchunks;
    c.sizes = B.d_sizes;
    return c;
}

// One batched AAR cycle over the running systems' work lists.
template <typename T> hipError_t batch_enqueue_cycle(aar_solver_t *S, hipStream_t s)
{
    auto &B = S->B;
    const aar_params &pa = S->params;
    const bool f64 = std::is_same<T, double>::value;
    T *xa, *xb, *b;
    void *dx;
    T *fcur = nullptr;
    if constexpr (std::is_same<T, double>::value) {
        xa = B.xa64;
        xb = B.xb64;
        b = B.b64;
        dx = B.dx64;
        fcur = B.fcur64;
    } else {
        xa = B.xa32;
        xb = B.xb32;
        b = B.rhs32;
        dx = B.dx32;
        fcur = B.fcur32;
    }
    BatchStencilArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    if constexpr (std::is_same<T, double>::value)
        a.desc = B.desc64;
    else
        a.desc = B.desc32;
    a.items = B.c_s;
    a.nitems = B.c_n;
    a.b = b;
    a.fring = B.fring;
    a.state = B.state;
    a.slot_stride = B.stride;
    a.p = pa.p;
    a.nslots = pa.m + 1;
    a.omega = (T)pa.omega;
    hipError_t e;
    const Prec hist = S->hist;   // history storage of this path (F64 for the plain FP64 solve)
    // residual recursion: the first sweep forms f from x and b and leaves x
    // alone; later sweeps and the Anderson-step residual follow
    // f_{j+1} = f_j - omega D^-1 A f_j from the ring; x stays in xa and the
    // update adds the cycle's Richardson steps
    const bool recur32 = f64 && B.recur32;
    const bool recur = B.recur || recur32;
    // FP32 recursion passes over the FP32 ring of an FP64 iteration: the same
    // (system, tile) items, FP32 coefficients; x and b are not read and point
    // at the ring so that every pointer is a valid FP32 vector
    BatchStencilArgs<float> a32;
    std::memset(&a32, 0, sizeof(a32));
    a32.desc = B.desc32;
    a32.items = B.c_s;
    a32.nitems = B.c_n;
    a32.x = static_cast<const float *>(B.fring);
    a32.b = static_cast<const float *>(B.fring);
    a32.fring = B.fring;
    a32.state = B.state;
    a32.slot_stride = B.stride;
    a32.p = pa.p;
    a32.nslots = pa.m + 1;
    a32.omega = (float)pa.omega;
    a32.recur = 1;
    for (int j = 0; j < pa.p - 1; ++j) {
        a.j = j;
        a.x = (j & 1) ? xb : xa;
        a.out = (j & 1) ? xa : xb;
        if (recur) {
            a.x = xa;
            a.out = nullptr;
            a.recur = j > 0;
        }
        if (recur32 && j > 0) {
            a32.j = j;
            e = launch_stencil_batched_f32(kSweep, Prec::F32, B.radius, B.conv, B.ry, a32, B.grid_s, s);
        } else if constexpr (std::is_same<T, double>::value) {
            e = launch_stencil_batched_f64(kSweep, hist, B.radius, B.conv, B.ry, a, B.grid_s, s);
        } else {
            e = launch_stencil_batched_f32(kSweep, hist, B.radius, B.conv, B.ry, a, B.grid_s, s);
        }
        if (e != hipSuccess)
            return e;
    }
    const int jk = pa.p - 1;
    T *xk = recur ? xa : (jk & 1) ? xb : xa;
    a.recur = recur && jk > 0;
    a.j = jk;
    a.x = xk;
    a.out = nullptr;
    a.fcur = fcur;
    a.partial = B.p_rho;
    if (recur32) {   // jk >= 1: p >= 2
        a32.j = jk;
        a32.partial = B.p_rho;
        e = launch_stencil_batched_f32(kFk, Prec::F32, B.radius, B.conv, B.ry, a32, B.grid_s, s);
    } else if constexpr (std::is_same<T, double>::value) {
        e = launch_stencil_batched_f64(kFk, hist, B.radius, B.conv, B.ry, a, B.grid_s, s);
    } else {
        e = launch_stencil_batched_f32(kFk, hist, B.radius, B.conv, B.ry, a, B.grid_s, s);
    }
    if (e != hipSuccess)
        return e;

    BatchGramArgs g;
    g.items = B.c_c;
    g.nitems = B.c_n + 1;
    g.state = B.state;
    g.fring = B.fring;
    g.offs = B.d_offs;
    g.sizes = B.d_sizes;
    g.partial = B.p_gram;
    g.slot_stride = B.stride;
    g.m = pa.m;
    g.p = pa.p;
    g.nslots = pa.m + 1;
    if ((e = launch_gram_batched(hist, g, B.grid_c, s)) != hipSuccess)
        return e;

    LsqArgs l;
    std::memset(&l, 0, sizeof(l));
    l.ne = S->ne;
    l.m = pa.m;
    l.p = pa.p;
    l.nslots = pa.m + 1;
    l.q = S->q;
    l.omega = pa.omega;
    l.beta = pa.beta;
    l.rcond = std::ldexp(1.0, -52);
    l.stagnation_window = S->mixed ? 8 : 0;
    l.stagnation_factor = 0.9;
    l.log = B.log;
    l.rank_log = B.rank_log;
    l.log_cap = S->log_cap;
    l.force_pinv = (pa.flags & AAR_FLAG_FORCE_PINV) ? 1 : 0;
    BatchLsqArgs bl;
    bl.state = B.state;
    bl.sbase = B.c_sb;
    bl.cbase = B.c_cb;
    bl.ntiles = B.d_ntiles;
    bl.nchunks = B.d_nchunks;
    bl.rho_partial = B.p_rho;
    bl.gram_partial = B.p_gram;
    if ((e = launch_lsq_batched(l, bl, B.count, s)) != hipSuccess)
        return e;

    BatchUpdateArgs<T> u;
    u.items = B.c_c;
    u.nitems = B.c_n + 1;
    u.state = B.state;
    u.offs = B.d_offs;
    u.sizes = B.d_sizes;
    u.xin = xk;
    u.xout = xa;
    u.fring = B.fring;
    u.fcur = fcur;
    u.dxring = dx;
    u.slot_stride = B.stride;
    u.dx_stride = B.stride;
    u.omega_rich = recur ? (T)pa.omega : T(0);
    u.p_rich = recur ? pa.p : 0;
    if constexpr (std::is_same<T, double>::value)
        return launch_update_batched(hist, &u, nullptr, B.grid_c, s);
    else
        return launch_update_batched(hist, nullptr, &u, B.grid_c, s);
}

#define AAR_HIPE(expr)                                                                          \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(AAR_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

// FP64 residual r = b - A x of the systems marked for refinement, with
// per-stencil-item partial norms in p_s.
aar_status batch_residual(aar_solver_t *S, double *x, const double *b, double *r)
{
    auto &B = S->B;
    BatchStencilArgs<double> a;
    std::memset(&a, 0, sizeof(a));
    a.desc = B.desc64;
    a.items = B.a_s;
    a.nitems = B.a_n;
    a.x = x;
    a.b = b;
    a.out = r;
    a.partial = B.p_s;
    a.mask = B.refine;
    a.slot_stride = B.stride;
    AAR_HIPE(launch_stencil_batched_f64(kResid, Prec::F64, B.radius, B.conv, B.ry, a, B.grid_s, S->stream));
    return AAR_OK;
}

aar_status batch_solve(aar_solver_t *S, const double *b, double *x, const int64_t *offsets, aar_result *results)
{
    auto &B = S->B;
    const aar_params &pa = S->params;
    hipStream_t s = S->stream;
    const bool deflate = (pa.flags & AAR_FLAG_DEFLATE_CONSTANT) != 0;
    const bool use_graph = !(pa.flags & AAR_FLAG_NO_GRAPH);
    const int count = B.count;
    AAR_HIP(hipMemcpyAsync(B.d_uoffs, offsets, sizeof(int64_t) * count, hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemsetAsync(B.ctl, 0, sizeof(BatchCtl) * count, s));
    AAR_HIP(hipMemsetAsync(B.refine, 0, sizeof(int) * count, s));
    double *x64 = B.xa64;          // FP64 iterate (FP64 mode: the cycles' xa)
    // gather b and x0 into the packed layout
    AAR_HIPE(launch_compact(batch_compact_args(S, 2, false), s));
    {
        BatchStreamArgs g = batch_stream(S, kOpGather, nullptr, 0);
        g.user = const_cast<double *>(b);
        g.v64 = B.b64;
        AAR_HIPE(launch_stream_batched(g, B.grid_c, s));
        g.user = x;
        g.v64 = x64;
        AAR_HIPE(launch_stream_batched(g, B.grid_c, s));
    }
    auto select = [&]() -> aar_status {
        AAR_HIP(hipMemsetAsync(B.remaining, 0, sizeof(int), s));
        AAR_HIPE(launch_ctl_batched(batch_ctl(S, kCtlSelect, nullptr, deflate), count, s));
        AAR_HIPE(launch_compact(batch_compact_args(S, 1, false), s));
        return AAR_OK;
    };
    // refinement step of the selected systems (mixed), or the start of FP64 runs
    auto refine_body = [&](bool first) -> aar_status {
        aar_status e;
        if (S->mixed) {
            if (first) {
                BatchStreamArgs nb = batch_stream(S, kOpNorm, B.refine, 1);
                nb.v64 = B.b64;
                nb.partial = B.p_c;
                AAR_HIPE(launch_stream_batched(nb, B.grid_c, s));
                AAR_HIPE(launch_ctl_batched(batch_ctl(S, kCtlNormB, B.p_c, deflate), count, s));
            } else {
                BatchStreamArgs c = batch_stream(S, kOpCorrect, B.refine, 1);
                c.v64 = x64;
                c.xa32 = B.xa32;
                c.xb32 = B.xb32;
                c.recur = B.recur ? 1 : 0;
                c.state = B.state;
                c.fring = B.fring;
                c.slot_stride = B.stride;
                c.p = pa.p;
                c.nslots = pa.m + 1;
                c.omega = pa.omega;
                AAR_HIPE(launch_stream_batched(c, B.grid_c, s));
            }
            if ((e = batch_residual(S, x64, B.b64, B.r64)) != AAR_OK)
                return e;
            if (deflate) {
                BatchStreamArgs sm = batch_stream(S, kOpSum, B.refine, 1);
                sm.v64 = B.r64;
                sm.partial = B.p_c;
                AAR_HIPE(launch_stream_batched(sm, B.grid_c, s));
                AAR_HIPE(launch_ctl_batched(batch_ctl(S, kCtlMean, B.p_c, deflate), count, s));
                BatchStreamArgs df = batch_stream(S, kOpDeflate, B.refine, 1);
                df.v64 = B.r64;
                df.x64 = x64;
                df.partial = B.p_c;
                AAR_HIPE(launch_stream_batched(df, B.grid_c, s));
                AAR_HIPE(launch_ctl_batched(batch_ctl(S, kCtlDecide, B.p_c, true), count, s));
            } else {
                AAR_HIPE(launch_ctl_batched(batch_ctl(S, kCtlDecide, B.p_s, false), count, s));
            }
            BatchStreamArgs pr = batch_stream(S, kOpPrepare, B.refine, 2);
            pr.v64 = B.r64;
            pr.rhs32 = B.rhs32;
            pr.xa32 = B.xa32;
            pr.partial = B.p_c;
            AAR_HIPE(launch_stream_batched(pr, B.grid_c, s));
            AAR_HIPE(launch_ctl_batched(batch_ctl(S, kCtlStart, B.p_c, deflate), count, s));
        } else {
            if (deflate) {
                double *r = static_cast<double *>(B.fring);   // slot 0 is scratch before the run
                if ((e = batch_residual(S, x64, B.b64, r)) != AAR_OK)
                    return e;
                BatchStreamArgs sm = batch_stream(S, kOpSum, B.refine, 1);
                sm.v64 = r;
                sm.partial = B.p_c;
                AAR_HIPE(launch_stream_batched(sm, B.grid_c, s));
                AAR_HIPE(launch_ctl_batched(batch_ctl(S, kCtlMean, B.p_c, deflate), count, s));
                BatchStreamArgs df = batch_stream(S, kOpDeflate, B.refine, 1);
                df.v64 = r;
                df.x64 = x64;
                AAR_HIPE(launch_stream_batched(df, B.grid_c, s));
            }
            AAR_HIPE(launch_ctl_batched(batch_ctl(S, kCtlDecide, nullptr, deflate), count, s));
            BatchStreamArgs nb = batch_stream(S, kOpNorm, B.refine, 2);
            nb.v64 = B.b64;
            nb.partial = B.p_c;
            AAR_HIPE(launch_stream_batched(nb, B.grid_c, s));
            AAR_HIPE(launch_ctl_batched(batch_ctl(S, kCtlStart, B.p_c, deflate), count, s));
        }
        return AAR_OK;
    };
    aar_status e;
    if ((e = select()) != AAR_OK)
        return e;
    if ((e = refine_body(true)) != AAR_OK)
        return e;
    if (use_graph && B.graph == nullptr) {
        AAR_HIP(hipStreamBeginCapture(S->capture_stream, hipStreamCaptureModeThreadLocal));
        hipError_t ce = hipSuccess;
        for (int c = 0; c < kBatchGraphCycles && ce == hipSuccess; ++c)
            ce = S->mixed ? batch_enqueue_cycle<float>(S, S->capture_stream)
                          : batch_enqueue_cycle<double>(S, S->capture_stream);
        hipGraph_t g = nullptr;
        hipError_t ce2 = hipStreamEndCapture(S->capture_stream, &g);
        if (ce != hipSuccess || ce2 != hipSuccess) {
            if (g)
                (void)hipGraphDestroy(g);
            return fail(AAR_ERR_DEVICE, std::string("batched graph capture: ") +
                                            hipGetErrorString(ce != hipSuccess ? ce : ce2));
        }
        hipError_t ce3 = hipGraphInstantiate(&B.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        AAR_HIP(ce3);
    }
    // Each replay: the active systems' cycles (one graph launch), then the
    // selection that counts the systems still running.  The count of replay
    // i is read only after replay i + 1 has been queued behind it (two pinned
    // slots, one event each), so the stream never drains between replays.
    // Work of a finished system is skipped by every kernel, so the one replay
    // queued after the last system finished changes nothing.
    int slot = 0;
    bool pending = false;
    for (;;) {
        AAR_HIPE(launch_compact(batch_compact_args(S, 0, true), s));
        if (use_graph) {
            AAR_HIP(hipGraphLaunch(B.graph, s));
        } else {
            for (int c = 0; c < kBatchGraphCycles; ++c)
                AAR_HIPE(S->mixed ? batch_enqueue_cycle<float>(S, s) : batch_enqueue_cycle<double>(S, s));
        }
        if ((e = select()) != AAR_OK)
            return e;
        AAR_HIP(hipMemcpyAsync(B.h_remaining + slot, B.remaining, sizeof(int), hipMemcpyDeviceToHost, s));
        AAR_HIP(hipEventRecord(S->poll_ev[slot], s));
        if (pending) {
            AAR_HIP(hipEventSynchronize(S->poll_ev[slot ^ 1]));
            if (B.h_remaining[slot ^ 1] == 0)
                break;   // every system had finished before this replay
        }
        pending = true;
        if (S->mixed && (e = refine_body(false)) != AAR_OK)
            return e;
        slot ^= 1;
    }
    // write the answers back in the caller's layout
    AAR_HIPE(launch_compact(batch_compact_args(S, 2, false), s));
    BatchStreamArgs sc = batch_stream(
        S, S->mixed ? kOpScatter : (B.recur || B.recur32) ? kOpScatterRecur : kOpScatterSel, nullptr, 0);
    sc.ring_f32 = B.recur32 ? 1 : 0;
    sc.user = x;
    sc.v64 = x64;
    sc.x64 = B.xb64;
    sc.state = B.state;
    sc.fring = B.fring;
    sc.slot_stride = B.stride;
    sc.p = pa.p;
    sc.nslots = pa.m + 1;
    sc.omega = pa.omega;
    AAR_HIPE(launch_stream_batched(sc, B.grid_c, s));
    std::vector<BatchCtl> ctl(count);
    std::vector<InstState> sts(count);
    AAR_HIP(hipMemcpyAsync(ctl.data(), B.ctl, sizeof(BatchCtl) * count, hipMemcpyDeviceToHost, s));
    AAR_HIP(hipMemcpyAsync(sts.data(), B.state, sizeof(InstState) * count, hipMemcpyDeviceToHost, s));
    AAR_HIP(hipStreamSynchronize(s));
    aar_status worst = AAR_OK;
    for (int i = 0; i < count; ++i) {
        aar_result r{};
        r.status = ctl[i].status;
        r.iterations = ctl[i].used;
        r.outer_steps = S->mixed ? ctl[i].outer : 0;
        r.rel_residual = ctl[i].rel;
        results[i] = r;
        S->last_log_count[i] = sts[i].log_count;
        if (r.status > worst)
            worst = (aar_status)r.status;
    }
    return worst;
}
// ---------------------------------------------------------------------------
// Allocation-free solve (aar_solve_noalloc): the workspace of one FP64 solve
// is carved from a fixed device array instead of device allocations.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)32 << 20;

// Each GPU the library runs on holds its own copy of this array until the
// process ends.  In host code `scratch` names a host-side stand-in; the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with it current).
aar_status scratch_address(int device, unsigned char **out)
{
    if (device < 0 || device >= kMaxScratchDevices)
        return fail(AAR_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(AAR_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[device]);
    return AAR_OK;
}

// Byte layout of the scratch workspace of one FP64 solve: run state, the
// partial sums of the stencil, Gram and norm passes, then x (two copies), b,
// the m + 1 history slots and the floor(m/p) increment slots, each vector on a
// 4 KiB boundary (slots stay 8-element aligned).
struct NoAllocLayout {
    size_t state, rho, gram, norm, gfinal, scal, xa, xb, b, ring, dx, total;
    int64_t slot_stride;       // elements between ring slots (and between dx slots)
    int rho_cap;
};

NoAllocLayout noalloc_layout(const aar_problem &pr, const aar_params &pa)
{
    const Sizes z = compute_sizes(&pr, 1, &pa);
    NoAllocLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const int64_t Np = (z.maxN + 7) / 8 * 8;
    const size_t span = ((size_t)Np * sizeof(double) + 4095) / 4096 * 4096;
    L.state = take(sizeof(InstState));
    L.rho = take(sizeof(double) * (size_t)z.max_stencil_blocks);
    L.gram = take(sizeof(double) * (size_t)std::max(z.gram_blocks, z.max_stencil_blocks) * z.ne);
    L.norm = take(sizeof(double) * (size_t)z.gram_blocks);
    L.gfinal = take(sizeof(double) * (size_t)z.ne);
    L.scal = take(sizeof(double) * 8);
    off = (off + 4095) / 4096 * 4096;
    L.xa = take(span);
    L.xb = take(span);
    L.b = take(span);
    L.ring = take(span * (size_t)(pa.m + 1));
    L.dx = take(span * (size_t)z.q);
    L.total = off;
    L.slot_stride = (int64_t)(span / sizeof(double));
    L.rho_cap = z.max_stencil_blocks;
    return L;
}

aar_status solve_noalloc(const aar_problem *problem, const aar_params *params, const double *b, double *x,
                         aar_result *res, void *hip_stream)
{
    if (!problem || !params || !b || !x)
        return fail(AAR_ERR_INVALID_ARG, "problem, params, b or x is NULL");
    aar_status st = validate_params(params);
    if (st != AAR_OK)
        return st;
    if ((st = validate_problem(*problem, 0)) != AAR_OK)
        return st;
    if (params->precision != AAR_FP64)
        return fail(AAR_ERR_UNSUPPORTED, "aar_solve_noalloc runs the FP64 iteration only");
    if (params->flags & AAR_FLAG_RECORD_RESIDUALS)
        return fail(AAR_ERR_UNSUPPORTED, "aar_solve_noalloc keeps no residual log");
    if (params->flags & AAR_FLAG_DEFLATE_CONSTANT) {
        const aar_problem &pr = *problem;
        if (!(pr.bc[0] == AAR_BC_PERIODIC && pr.bc[1] == AAR_BC_PERIODIC && pr.bc[2] == AAR_BC_PERIODIC &&
              pr.shift > 0.0))
            return fail(AAR_ERR_UNSUPPORTED, "AAR_FLAG_DEFLATE_CONSTANT needs periodic axes and shift > 0");
    }
    const NoAllocLayout L = noalloc_layout(*problem, *params);
    if (L.total > kScratchBytes)
        return fail(AAR_ERR_UNSUPPORTED, "system needs " + std::to_string(L.total) +
                                             " bytes of scratch; aar_solve_noalloc holds " +
                                             std::to_string(kScratchBytes));
    int device = 0;
    AAR_HIP(hipGetDevice(&device));
    unsigned char *base = nullptr;
    if ((st = scratch_address(device, &base)) != AAR_OK)
        return st;

    // the operator: tile shapes are the defaults (no timing, no tile file);
    // the caller's velocity array is read in place
    Operator op = build_operator(*problem);
    op.vel64 = const_cast<double *>(problem->velocity);
    aar_solver_t S;
    S.params = *params;
    S.stream = (hipStream_t)hip_stream;
    S.device = device;
    S.mixed = false;
    S.hist = Prec::F64;
    S.maxN = op.N;
    S.q = params->m / params->p;
    S.ne = params->m * (params->m + 1) / 2 + params->m;
    S.state = reinterpret_cast<InstState *>(base + L.state);
    S.part_rho = reinterpret_cast<double *>(base + L.rho);
    S.part_rho_cap = L.rho_cap;
    S.part_gram = reinterpret_cast<double *>(base + L.gram);
    S.part_norm = reinterpret_cast<double *>(base + L.norm);
    S.gram_final = reinterpret_cast<double *>(base + L.gfinal);
    S.scal = reinterpret_cast<double *>(base + L.scal);
    Path<double> &P = S.p64;
    P.hist = Prec::F64;
    P.xa = reinterpret_cast<double *>(base + L.xa);
    P.xb = reinterpret_cast<double *>(base + L.xb);
    P.b = reinterpret_cast<double *>(base + L.b);
    P.fring = base + L.ring;
    P.dx = S.q > 0 ? (void *)(base + L.dx) : nullptr;
    S.slot_stride[0] = L.slot_stride;
    S.dx_stride64 = L.slot_stride;
    int32_t lc = 0;
    return solve_fp64(&S, op, b, x, res, false, &lc);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *aar_last_error(void)
{
    return g_error.c_str();
}

aar_status aar_workspace_bytes(const aar_problem *problems, int32_t count, const aar_params *params,
                               size_t *bytes)
{
    if (!problems || count < 1 || !bytes)
        return fail(AAR_ERR_INVALID_ARG, "problems, count or bytes invalid");
    aar_status st = validate_params(params);
    if (st != AAR_OK)
        return st;
    for (int i = 0; i < count; ++i)
        if ((st = validate_problem(problems[i], i)) != AAR_OK)
            return st;
    *bytes = batch_eligible(problems, count, params) ? batch_bytes(problems, count, params)
                                             : compute_sizes(problems, count, params).bytes;
    return AAR_OK;
}

aar_status aar_create(aar_solver *out, const aar_problem *problems, int32_t count, const aar_params *params,
                      void *hip_stream)
{
    g_error.clear();
    if (!out)
        return fail(AAR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!problems || count < 1)
        return fail(AAR_ERR_INVALID_ARG, "problems is NULL or count < 1");
    aar_status st = validate_params(params);
    if (st != AAR_OK)
        return st;
    for (int i = 0; i < count; ++i)
        if ((st = validate_problem(problems[i], i)) != AAR_OK)
            return st;
    if (params->flags & AAR_FLAG_DEFLATE_CONSTANT) {
        for (int i = 0; i < count; ++i) {
            const aar_problem &pr = problems[i];
            const bool ok = pr.bc[0] == AAR_BC_PERIODIC && pr.bc[1] == AAR_BC_PERIODIC &&
                            pr.bc[2] == AAR_BC_PERIODIC && pr.shift > 0.0;
            if (!ok)
                return fail(AAR_ERR_UNSUPPORTED, "AAR_FLAG_DEFLATE_CONSTANT needs periodic axes and shift > 0 "
                                                 "(system " + std::to_string(i) + ")");
        }
    }

    if ((params->flags & AAR_FLAG_RECYCLE_HISTORY) &&
        (!is_mixed(params->precision) || batch_eligible(problems, count, params)))
        return fail(AAR_ERR_UNSUPPORTED, "AAR_FLAG_RECYCLE_HISTORY needs a mixed precision mode and single solves");

    std::unique_ptr<aar_solver_t> S(new aar_solver_t());
    S->params = *params;
    S->stream = (hipStream_t)hip_stream;
    S->mixed = is_mixed(params->precision);
    S->hist = hist_of(params->precision);
    AAR_HIP(hipGetDevice(&S->device));
    AAR_HIP(hipStreamCreateWithFlags(&S->capture_stream, hipStreamNonBlocking));
    // coherent pinned memory: the update kernels' stores reach the host without caching
    AAR_HIP(hipHostMalloc((void **)&S->host_status, 2 * sizeof(int32_t),
                          hipHostMallocMapped | hipHostMallocCoherent));
    S->host_status[0] = S->host_status[1] = kRunning;
    AAR_HIP(hipHostGetDevicePointer((void **)&S->status_dev, S->host_status, 0));
    for (auto &e : S->poll_ev)
        AAR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));

    const Sizes z = compute_sizes(problems, count, params);
    const bool batched = batch_eligible(problems, count, params);
    S->maxN = z.maxN;
    S->q = z.q;
    S->ne = z.ne;
    S->last_log_count.assign(count, 0);
    const int64_t N = (z.maxN + 7) / 8 * 8;    // vectors padded: ring slots stay 8-element aligned
    const int slots = params->m + 1;

    st = AAR_OK;
    S->state = S->alloc<InstState>(1, &st);
    S->part_rho = S->alloc<double>(z.max_stencil_blocks, &st);
    S->part_rho_cap = z.max_stencil_blocks;
    // Gram partials: one column per Gram-pass workgroup, or per stencil
    // workgroup when the Anderson-residual pass forms the products
    S->part_gram = S->alloc<double>((size_t)std::max(z.gram_blocks, z.max_stencil_blocks) * z.ne, &st);
    S->part_norm = S->alloc<double>(z.gram_blocks, &st);
    S->gram_final = S->alloc<double>(z.ne, &st);
    S->scal = S->alloc<double>(8, &st);
    if (st != AAR_OK)
        return st;
    if (z.log_cap > 0) {
        S->log_cap = z.log_cap;
        S->log = S->alloc<double>(z.log_cap, &st);
        S->rank_log = S->alloc<int32_t>(z.log_cap, &st);
    }
    if (!batched) {
        // Bulk vectors and ring slots come from one arena, each starting on a
        // 4 KiB boundary plus an optional stagger (AAR_STAGGER_BYTES; measured
        // to make no difference on MI355X, so 0 by default).
        const size_t stagger = stagger_bytes();
        auto vec_span = [&](size_t esize) { return (((size_t)N * esize + 4095) / 4096) * 4096 + stagger; };
        size_t arena = 0;
        // Anderson increments of an FP64 iteration: FP32 beside an FP32 ring
        const size_t dx_bytes = S->hist == Prec::F32 ? 4 : 8;
        if (!S->mixed) {
            arena = vec_span(8) * 3 + vec_span(dx_bytes) * S->q + vec_span(hist_bytes(S->hist)) * slots +
                    (S->hist == Prec::F32_BF16 ? vec_span(8) : 0);
        } else {
            arena = vec_span(4) * (3 + S->q) + vec_span(hist_bytes(S->hist)) * slots + vec_span(8) * 3 +
                    (S->hist == Prec::F32_BF16 ? vec_span(4) : 0);
        }
        char *base = S->alloc<char>(arena, &st);
        if (st != AAR_OK)
            return st;
        size_t off = 0;
        auto carve = [&](size_t esize, int count_vec) -> void * {
            void *p = base + off;
            off += vec_span(esize) * count_vec;
            return p;
        };
        if (!S->mixed) {
            Path<double> &P = S->p64;
            P.hist = S->hist;
            P.xa = (double *)carve(8, 1);
            P.xb = (double *)carve(8, 1);
            P.b = (double *)carve(8, 1);
            P.fring = carve(hist_bytes(S->hist), slots);
            if (S->hist == Prec::F32_BF16)
                P.fcur = (double *)carve(8, 1);      // f_k of the update in FP64
            P.dx = S->q > 0 ? carve(dx_bytes, S->q) : nullptr;
            S->slot_stride[0] = vec_span(hist_bytes(S->hist)) / hist_bytes(S->hist);
            S->dx_stride64 = vec_span(dx_bytes) / dx_bytes;
        } else {
            Path<float> &P = S->p32;
            P.hist = S->hist;
            P.xa = (float *)carve(4, 1);
            P.xb = (float *)carve(4, 1);
            P.b = (float *)carve(4, 1);
            P.fring = carve(hist_bytes(S->hist), slots);
            if (S->hist == Prec::F32_BF16)
                P.fcur = (float *)carve(4, 1);
            P.dx = S->q > 0 ? carve(4, S->q) : nullptr;
            S->x64 = (double *)carve(8, 1);
            S->b64 = (double *)carve(8, 1);
            S->r64 = (double *)carve(8, 1);
            S->slot_stride[1] = vec_span(hist_bytes(S->hist)) / hist_bytes(S->hist);
            S->dx_stride = vec_span(4) / 4;
        }
        if (st != AAR_OK)
            return st;
    }

    for (int i = 0; i < count; ++i) {
        Operator op = build_operator(problems[i]);
        if (problems[i].velocity) {
            op.vel64 = S->alloc<double>(3 * op.N, &st);
            if (st != AAR_OK)
                return st;
            AAR_HIP(hipMemcpyAsync(op.vel64, problems[i].velocity, sizeof(double) * 3 * op.N,
                                   hipMemcpyDeviceToDevice, S->stream));
            if (S->mixed || S->hist == Prec::F32) {   // FP32 passes: mixed inner solves, FP32-ring recursion
                op.vel32 = S->alloc<float>(3 * op.N, &st);
                if (st != AAR_OK)
                    return st;
                AAR_HIP(launch_cast_f64_f32_plain(op.vel64, op.vel32, 3 * op.N, S->stream));
            }
        }
        S->ops.push_back(op);
    }
    AAR_HIP(hipStreamSynchronize(S->stream));
    if (batched && (st = batch_setup(S.get())) != AAR_OK)
        return st;
    if (!(params->flags & AAR_FLAG_NO_AUTOTUNE) && count == 1) {
        st = S->mixed ? autotune<float>(S.get(), 0) : autotune<double>(S.get(), 0);
        if (st != AAR_OK)
            return st;
        if (!S->mixed && S->hist == Prec::F32)
            cached_tile32(S->ops[0]);
        if (S->mixed)
            cached_tile64(S->ops[0]);
        AAR_HIP(hipStreamSynchronize(S->stream));
    }
    *out = S.release();
    return AAR_OK;
}

aar_status aar_solve_noalloc(const aar_problem *problem, const aar_params *params, const double *b, double *x,
                             aar_result *r, void *hip_stream)
{
    g_error.clear();
    return solve_noalloc(problem, params, b, x, r, hip_stream);
}

// Tile of the complex sweep (one-point layout, at most 2 rows per thread):
// the tile file's line for the grid with precision field 2, else the fastest
// candidate (rows per thread 1 or 2, z depths 2 .. 32, every tile order)
// timed on the solver's own buffers, which every solve overwrites.  A small
// grid needs short z chunks to fill the chip.  The choice is kept per grid
// for the process.
aar_status tune_complex_tile(aar_solver_t *S, const aar_problem &pr, Path<zd> &P)
{
    const auto key = std::make_tuple(2, pr.radius, 0, pr.n[0], pr.n[1], pr.n[2]);
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        load_tune_file();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end() && it->second.pair == 0 && it->second.tb == 0) {
            P.ts = it->second;
            P.ts.ry = std::min(P.ts.ry, 2);
            return AAR_OK;
        }
    }
    hipStream_t s = S->stream;
    const int64_t N = P.N;
    AAR_HIP(launch_fill_pattern_f64(reinterpret_cast<double *>(P.xa), 2 * N, s));
    AAR_HIP(launch_fill_pattern_f64(reinterpret_cast<double *>(P.b), 2 * N, s));
    const int nb_blocks = stream_blocks(N);
    AAR_HIP(launch_cnorm_partial(P.b, N, S->part_norm, nb_blocks, s));
    AAR_HIP(launch_init_state(S->state, S->part_norm, nb_blocks, (int64_t)1 << 40, 1.0, s));
    StencilArgs<zd> a;
    std::memset(&a, 0, sizeof(a));
    a.st = P.st;
    a.b = P.b;
    a.fring = P.fring;
    a.state = S->state;
    a.slot_stride = P.slot_stride;
    a.p = S->params.p;
    a.nslots = S->params.m + 1;
    a.omega = zd(S->params.omega, S->omega_im);
    a.j = 0;
    a.x = P.xa;
    a.out = P.xb;
    std::vector<TileShape> cands;
    for (int ry : {1, 2}) {
        int prev_tz = -1;
        for (int cz : {2, 4, 6, 8, 12, 16, 24, 32}) {
            int tx, ty, tz, blocks;
            stencil_grid(pr.n[0], pr.n[1], pr.n[2], TileShape{ry, cz, 0}, &tx, &ty, &tz, &blocks);
            if (tz == prev_tz || blocks > S->part_rho_cap)
                continue;
            prev_tz = tz;
            for (int order = 0; order < (tz > 1 ? 4 : 1); ++order)
                cands.push_back(TileShape{ry, cz, order, 0});
        }
    }
    hipEvent_t e0, e1;
    AAR_HIP(hipEventCreate(&e0));
    AAR_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    TileShape best = P.ts;
    hipError_t e = hipSuccess;
    for (const TileShape &ts : cands) {
        for (int w = 0; w < 3 && e == hipSuccess; ++w)
            e = launch_stencil_complex(kSweep, P.radius, ts, a, nullptr, s);
        if (e == hipSuccess)
            e = hipEventRecord(e0, s);
        for (int w = 0; w < 10 && e == hipSuccess; ++w)
            e = launch_stencil_complex(kSweep, P.radius, ts, a, nullptr, s);
        if (e == hipSuccess)
            e = hipEventRecord(e1, s);
        if (e == hipSuccess)
            e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess)
            break;
        if (ms < best_ms) {
            best_ms = ms;
            best = ts;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess)
        return fail(AAR_ERR_DEVICE, std::string("complex tile timing: ") + hipGetErrorString(e));
    P.ts = best;
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        g_tune_cache[key] = best;
    }
    append_tune_file(key, best);
    return AAR_OK;
}

aar_status aar_create_complex(aar_solver *out, const aar_problem *problem, const aar_params *params,
                              double shift_imag, double omega_imag, double beta_imag, void *hip_stream)
{
    g_error.clear();
    if (!out)
        return fail(AAR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!problem)
        return fail(AAR_ERR_INVALID_ARG, "problem is NULL");
    aar_status st = validate_params(params);
    if (st != AAR_OK)
        return st;
    // the real part of a complex shift may be negative (Eq. 7: Re Q < 0)
    aar_problem pr = *problem;
    if (!std::isfinite(pr.shift))
        return fail(AAR_ERR_INVALID_ARG, "shift must be finite");
    pr.shift = std::fabs(pr.shift);
    if ((st = validate_problem(pr, 0)) != AAR_OK)
        return st;
    if (!std::isfinite(shift_imag) || !std::isfinite(omega_imag) || !std::isfinite(beta_imag))
        return fail(AAR_ERR_INVALID_ARG, "imaginary parts must be finite");
    if (params->precision != AAR_FP64)
        return fail(AAR_ERR_UNSUPPORTED, "complex systems run the FP64 iteration only");
    if (params->m > 8)
        return fail(AAR_ERR_UNSUPPORTED, "complex systems need m <= 8");
    if (problem->velocity)
        return fail(AAR_ERR_UNSUPPORTED, "complex systems take no convection");
    if (params->flags & AAR_FLAG_DEFLATE_CONSTANT)
        return fail(AAR_ERR_UNSUPPORTED, "AAR_FLAG_DEFLATE_CONSTANT is for real systems");
    std::unique_ptr<aar_solver_t> S(new aar_solver_t());
    S->params = *params;
    S->stream = (hipStream_t)hip_stream;
    S->cplx = true;
    S->shift_im = shift_imag;
    S->omega_im = omega_imag;
    S->beta_im = beta_imag;
    AAR_HIP(hipGetDevice(&S->device));
    AAR_HIP(hipStreamCreateWithFlags(&S->capture_stream, hipStreamNonBlocking));
    AAR_HIP(hipHostMalloc((void **)&S->host_status, 2 * sizeof(int32_t),
                          hipHostMallocMapped | hipHostMallocCoherent));
    S->host_status[0] = S->host_status[1] = kRunning;
    AAR_HIP(hipHostGetDevicePointer((void **)&S->status_dev, S->host_status, 0));
    for (auto &e : S->poll_ev)
        AAR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const Sizes z = compute_sizes(problem, 1, params);
    S->maxN = z.maxN;
    S->q = z.q;
    S->ne = z.ne;
    S->last_log_count.assign(1, 0);
    Operator op = build_operator(*problem);
    op.ts[0] = default_tile(problem->radius, true);
    op.ts[0].ry = std::min(op.ts[0].ry, 2);   // complex tiles hold at most 2 rows per thread
    S->ops.push_back(op);
    const int64_t N = (z.maxN + 7) / 8 * 8;
    const int slots = params->m + 1;
    st = AAR_OK;
    S->state = S->alloc<InstState>(1, &st);
    S->part_rho = S->alloc<double>(z.max_stencil_blocks, &st);
    S->part_rho_cap = z.max_stencil_blocks;
    // Gram partials: the real-part table, then the imaginary-part table
    S->part_gram = S->alloc<double>(
        std::max(2 * (size_t)gram_blocks(z.maxN, params->m), (size_t)z.max_stencil_blocks) * z.ne, &st);
    S->part_norm = S->alloc<double>(z.gram_blocks, &st);
    S->gram_final = S->alloc<double>(2 * z.ne, &st);
    S->scal = S->alloc<double>(8, &st);
    if (z.log_cap > 0) {
        S->log_cap = z.log_cap;
        S->log = S->alloc<double>(z.log_cap, &st);
        S->rank_log = S->alloc<int32_t>(z.log_cap, &st);
    }
    Path<zd> &P = S->pz;
    P.xa = S->alloc<zd>(N, &st);
    P.xb = S->alloc<zd>(N, &st);
    P.b = S->alloc<zd>(N, &st);
    P.fring = S->alloc<zd>((size_t)N * slots, &st);
    P.dx = S->q > 0 ? (void *)S->alloc<zd>((size_t)N * S->q, &st) : nullptr;
    if (st != AAR_OK)
        return st;
    P.hist = Prec::F64;
    P.N = op.N;
    P.radius = problem->radius;
    P.conv = false;
    P.ts = op.ts[0];
    P.gram_blocks = gram_blocks(op.N, params->m);
    P.upd_blocks = stream_blocks(op.N);
    P.slot_stride = N;
    P.dx_stride = N;
    P.st = make_stencil<zd>(op, (const zd *)nullptr);
    // the imaginary shift enters the centre weight, sigma and the Jacobi diagonal
    P.st.sigma = zd(problem->shift, shift_imag);
    P.st.diag = zd(op.diag, shift_imag);
    P.st.jdiag = zd(op.jdiag, shift_imag);
    P.st.inv_diag = zd(1.0) / P.st.jdiag;
    if ((st = tune_complex_tile(S.get(), *problem, P)) != AAR_OK)
        return st;
    S->ops[0].ts[0] = P.ts;
    int tx, ty, tz, blocks;
    stencil_grid(problem->n[0], problem->n[1], problem->n[2], P.ts, &tx, &ty, &tz, &blocks);
    P.rho_blocks = blocks;
    if (P.rho_blocks > S->part_rho_cap)
        return fail(AAR_ERR_DEVICE, "stencil grid exceeds the partial-sum workspace");
    *out = S.release();
    return AAR_OK;
}

aar_status aar_create_csr(aar_solver *out, int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                          int32_t preconditioner, int32_t nblocks, const aar_params *params, void *hip_stream)
{
    g_error.clear();
    if (!out)
        return fail(AAR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!rowptr || !col || !val)
        return fail(AAR_ERR_INVALID_ARG, "rowptr, col or val is NULL");
    aar_status st = validate_params(params);
    if (st != AAR_OK)
        return st;
    if (n < 1 || n > INT32_MAX)
        return fail(AAR_ERR_INVALID_ARG, "n must be in 1 .. 2^31 - 1");
    if (preconditioner != AAR_PRECOND_JACOBI && preconditioner != AAR_PRECOND_ILU0)
        return fail(AAR_ERR_INVALID_ARG, "unknown preconditioner");
    if (rowptr[0] != 0)
        return fail(AAR_ERR_INVALID_ARG, "rowptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i) {
        if (rowptr[i + 1] < rowptr[i])
            return fail(AAR_ERR_INVALID_ARG, "rowptr decreases at row " + std::to_string(i));
        bool diag = false;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if (col[e] < 0 || col[e] >= n)
                return fail(AAR_ERR_INVALID_ARG, "column out of range in row " + std::to_string(i));
            if (e > rowptr[i] && col[e] <= col[e - 1])
                return fail(AAR_ERR_INVALID_ARG, "columns not strictly increasing in row " + std::to_string(i));
            if (!std::isfinite(val[e]))
                return fail(AAR_ERR_INVALID_ARG, "non-finite value in row " + std::to_string(i));
            diag = diag || col[e] == i;
        }
        if (!diag)
            return fail(AAR_ERR_INVALID_ARG, "row " + std::to_string(i) + " has no diagonal entry");
    }
    const bool ilu = preconditioner == AAR_PRECOND_ILU0;
    if (ilu && (nblocks < 1 || nblocks > n))
        return fail(AAR_ERR_INVALID_ARG, "nblocks must be in 1 .. n for block ILU(0)");
    // Jacobi: plain row chunks, one workgroup each
    const int nb = ilu ? nblocks : (int)std::max<int64_t>(1, (n + 2047) / 2048);
    if (ilu && (n + nb - 1) / nb > kCsrMaxBlockRows)
        return fail(AAR_ERR_UNSUPPORTED, "block ILU(0) blocks hold at most " + std::to_string(kCsrMaxBlockRows) +
                                             " rows: raise nblocks");
    if (params->precision != AAR_FP64)
        return fail(AAR_ERR_UNSUPPORTED, "sparse systems run the FP64 iteration only");
    if (params->flags & (AAR_FLAG_DEFLATE_CONSTANT | AAR_FLAG_RECYCLE_HISTORY))
        return fail(AAR_ERR_UNSUPPORTED, "deflation and recycling are for stencil systems");
    std::unique_ptr<aar_solver_t> S(new aar_solver_t());
    S->params = *params;
    S->stream = (hipStream_t)hip_stream;
    S->csr = true;
    AAR_HIP(hipGetDevice(&S->device));
    AAR_HIP(hipStreamCreateWithFlags(&S->capture_stream, hipStreamNonBlocking));
    AAR_HIP(hipHostMalloc((void **)&S->host_status, 2 * sizeof(int32_t),
                          hipHostMallocMapped | hipHostMallocCoherent));
    S->host_status[0] = S->host_status[1] = kRunning;
    AAR_HIP(hipHostGetDevicePointer((void **)&S->status_dev, S->host_status, 0));
    for (auto &e : S->poll_ev)
        AAR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    S->q = params->m / params->p;
    S->ne = params->m * (params->m + 1) / 2 + params->m;
    S->maxN = n;
    S->last_log_count.assign(1, 0);
    Operator op;
    std::memset(&op.prob, 0, sizeof(op.prob));
    op.N = n;
    S->ops.push_back(op);

    CsrPlan pl;
    plan_csr(n, rowptr, col, nb, ilu, &pl);
    if (ilu)
        pack_csr(n, rowptr, col, &pl);
    const int64_t nnz = rowptr[n];
    st = AAR_OK;
    int64_t *d_rowptr = S->alloc<int64_t>(n + 1, &st);
    int32_t *d_col = S->alloc<int32_t>(nnz, &st);
    double *d_val = S->alloc<double>(nnz, &st);
    double *d_lu = ilu ? S->alloc<double>(nnz, &st) : nullptr;
    int64_t *d_dpos = S->alloc<int64_t>(n, &st);
    int64_t *d_bstart = S->alloc<int64_t>(nb + 1, &st);
    int32_t *d_lrows = S->alloc<int32_t>(pl.lrows.size(), &st);
    int32_t *d_urows = S->alloc<int32_t>(pl.urows.size(), &st);
    int32_t *d_lptr = S->alloc<int32_t>(pl.lptr.size(), &st);
    int32_t *d_uptr = S->alloc<int32_t>(pl.uptr.size(), &st);
    int32_t *d_blevl = S->alloc<int32_t>(pl.blev_l.size(), &st);
    int32_t *d_blevu = S->alloc<int32_t>(pl.blev_u.size(), &st);
    int *d_bad = S->alloc<int>(1, &st);
    const size_t pk = (size_t)n * pl.kp;
    int16_t *d_frow = pl.kp ? S->alloc<int16_t>(n, &st) : nullptr;
    int16_t *d_brow = pl.kp ? S->alloc<int16_t>(n, &st) : nullptr;
    int16_t *d_fcol = pl.kp ? S->alloc<int16_t>(pk, &st) : nullptr;
    int16_t *d_bcol = pl.kp ? S->alloc<int16_t>(pk, &st) : nullptr;
    int32_t *d_fe = pl.kp ? S->alloc<int32_t>(pk, &st) : nullptr;
    int32_t *d_be = pl.kp ? S->alloc<int32_t>(pk, &st) : nullptr;
    double *d_fval = pl.kp ? S->alloc<double>(pk, &st) : nullptr;
    double *d_bval = pl.kp ? S->alloc<double>(pk, &st) : nullptr;
    double *d_bdiag = pl.kp ? S->alloc<double>(n, &st) : nullptr;
    const int64_t N = (n + 7) / 8 * 8;
    const int slots = params->m + 1;
    const int gblocks = gram_blocks(n, params->m);
    S->state = S->alloc<InstState>(1, &st);
    S->part_rho = S->alloc<double>(nb, &st);
    S->part_rho_cap = nb;
    S->part_gram = S->alloc<double>((size_t)gblocks * S->ne, &st);
    S->part_norm = S->alloc<double>(stream_blocks(n), &st);
    S->gram_final = S->alloc<double>(S->ne, &st);
    S->scal = S->alloc<double>(8, &st);
    if (params->flags & AAR_FLAG_RECORD_RESIDUALS) {
        S->log_cap = std::min<int64_t>(params->max_iter / params->p + 2, (int64_t)1 << 22);
        S->log = S->alloc<double>(S->log_cap, &st);
        S->rank_log = S->alloc<int32_t>(S->log_cap, &st);
    }
    Path<double> &P = S->p64;
    P.xa = S->alloc<double>(N, &st);
    P.xb = S->alloc<double>(N, &st);
    P.b = S->alloc<double>(N, &st);
    P.fring = S->alloc<double>((size_t)N * slots, &st);
    P.dx = S->q > 0 ? (void *)S->alloc<double>((size_t)N * S->q, &st) : nullptr;
    if (st != AAR_OK)
        return st;
    hipStream_t s = S->stream;
    AAR_HIP(hipMemcpyAsync(d_rowptr, rowptr, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemcpyAsync(d_col, col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemcpyAsync(d_val, val, sizeof(double) * nnz, hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemcpyAsync(d_dpos, pl.dpos.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemcpyAsync(d_bstart, pl.bstart.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice, s));
    if (ilu) {
        AAR_HIP(hipMemcpyAsync(d_lu, val, sizeof(double) * nnz, hipMemcpyHostToDevice, s));
        AAR_HIP(hipMemcpyAsync(d_lrows, pl.lrows.data(), sizeof(int32_t) * pl.lrows.size(), hipMemcpyHostToDevice, s));
        AAR_HIP(hipMemcpyAsync(d_urows, pl.urows.data(), sizeof(int32_t) * pl.urows.size(), hipMemcpyHostToDevice, s));
    }
    AAR_HIP(hipMemcpyAsync(d_lptr, pl.lptr.data(), sizeof(int32_t) * pl.lptr.size(), hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemcpyAsync(d_uptr, pl.uptr.data(), sizeof(int32_t) * pl.uptr.size(), hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemcpyAsync(d_blevl, pl.blev_l.data(), sizeof(int32_t) * pl.blev_l.size(), hipMemcpyHostToDevice, s));
    AAR_HIP(hipMemcpyAsync(d_blevu, pl.blev_u.data(), sizeof(int32_t) * pl.blev_u.size(), hipMemcpyHostToDevice, s));
    CsrDev &c = S->cd;
    c.n = n;
    c.rowptr = d_rowptr;
    c.col = d_col;
    c.val = d_val;
    c.lu = d_lu;
    c.dpos = d_dpos;
    c.bstart = d_bstart;
    c.lrows = d_lrows;
    c.urows = d_urows;
    c.lptr = d_lptr;
    c.uptr = d_uptr;
    c.blev_l = d_blevl;
    c.blev_u = d_blevu;
    c.nblocks = nb;
    c.max_block_rows = pl.max_block_rows;
    c.ilu = ilu ? 1 : 0;
    c.kp = pl.kp;
    c.depth = 1;
    c.lev_lds = 0;
    if (pl.kp) {
        // the level bounds of the deepest block beside its values, if they fit
        int most = 0;
        for (int t = 0; t < nb; ++t)
            most = std::max(most, (pl.blev_l[t + 1] - pl.blev_l[t]) + (pl.blev_u[t + 1] - pl.blev_u[t]) + 2);
        if ((size_t)pl.max_block_rows * sizeof(double) + (size_t)most * sizeof(int32_t) <= kCsrMaxLds)
            c.lev_lds = most;
    }
    c.frow = d_frow;
    c.fcol = d_fcol;
    c.brow = d_brow;
    c.bcol = d_bcol;
    c.fval = d_fval;
    c.bval = d_bval;
    c.bdiag = d_bdiag;
    if (pl.kp) {
        AAR_HIP(hipMemcpyAsync(d_frow, pl.frow.data(), sizeof(int16_t) * n, hipMemcpyHostToDevice, s));
        AAR_HIP(hipMemcpyAsync(d_brow, pl.brow.data(), sizeof(int16_t) * n, hipMemcpyHostToDevice, s));
        AAR_HIP(hipMemcpyAsync(d_fcol, pl.fcol.data(), sizeof(int16_t) * pk, hipMemcpyHostToDevice, s));
        AAR_HIP(hipMemcpyAsync(d_bcol, pl.bcol.data(), sizeof(int16_t) * pk, hipMemcpyHostToDevice, s));
        AAR_HIP(hipMemcpyAsync(d_fe, pl.fe.data(), sizeof(int32_t) * pk, hipMemcpyHostToDevice, s));
        AAR_HIP(hipMemcpyAsync(d_be, pl.be.data(), sizeof(int32_t) * pk, hipMemcpyHostToDevice, s));
    }
    if (ilu) {
        AAR_HIP(prepare_csr_kernels());
        // the factors: once, on the device
        int bad = 0;
        AAR_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), s));
        AAR_HIP(launch_ilu0(c, d_bad, s));
        AAR_HIP(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
        AAR_HIP(hipStreamSynchronize(s));
        if (bad)
            return fail(AAR_ERR_UNSUPPORTED, "ILU(0) meets a zero or non-finite pivot");
        if (pl.kp) {
            AAR_HIP(launch_pack_factors(c, d_fe, d_be, d_fval, d_bval, d_bdiag, s));
            // prefetch depth of the packed substitutions: the fastest of three
            // preconditioner passes each (the iterate buffers serve as input
            // and output; their contents do not matter)
            AAR_HIP(launch_fill_pattern_f64(P.xa, n, s));
            hipEvent_t e0, e1;
            AAR_HIP(hipEventCreate(&e0));
            AAR_HIP(hipEventCreate(&e1));
            float best = 0.0f;
            int best_depth = 1;
            bool timed = false;
            // AAR_CSR_DEPTH fixes the depth instead (a tuning override, as the
            // tile file is for stencils)
            const char *fixed = std::getenv("AAR_CSR_DEPTH");
            const int want = fixed ? std::atoi(fixed) : 0;
            for (int d : {1, 2, 4}) {
                if ((d == 4 && pl.kp != 4) || (want && d != want))
                    continue;
                c.depth = d;
                CsrArgs a;
                std::memset(&a, 0, sizeof(a));
                a.c = c;
                a.x = P.xa;
                a.out = P.xb;
                AAR_HIP(launch_csr(kPrecond, a, s));   // warm-up
                AAR_HIP(hipEventRecord(e0, s));
                for (int r = 0; r < 3; ++r)
                    AAR_HIP(launch_csr(kPrecond, a, s));
                AAR_HIP(hipEventRecord(e1, s));
                AAR_HIP(hipEventSynchronize(e1));
                float ms = 0.0f;
                AAR_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (!timed || ms < best) {
                    best = ms;
                    best_depth = d;
                    timed = true;
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            c.depth = best_depth;
        }
    }
    AAR_HIP(hipStreamSynchronize(s));
    P.hist = Prec::F64;
    P.N = n;
    P.rho_blocks = nb;
    P.gram_blocks = gblocks;
    P.upd_blocks = stream_blocks(n);
    P.slot_stride = N;
    P.dx_stride = N;
    *out = S.release();
    return AAR_OK;
}

aar_status aar_precondition(aar_solver s, const double *r, double *z)
{
    g_error.clear();
    if (!s || !r || !z)
        return fail(AAR_ERR_INVALID_ARG, "solver, r or z is NULL");
    if (!s->csr)
        return fail(AAR_ERR_UNSUPPORTED, "aar_precondition is for solvers from aar_create_csr");
    CsrArgs a;
    std::memset(&a, 0, sizeof(a));
    a.c = s->cd;
    a.x = r;
    a.out = z;
    AAR_HIP(launch_csr(kPrecond, a, s->stream));
    AAR_HIP(hipStreamSynchronize(s->stream));
    return AAR_OK;
}

aar_status aar_select_parameters(const aar_problem *problem, const aar_params *params, const double *b,
                                 const double *betas, int32_t nbeta, const int32_t *ps, int32_t np,
                                 int64_t trial_iterations, void *hip_stream, double *beta_out, int32_t *p_out,
                                 double *scores)
{
    g_error.clear();
    if (!problem || !params || !b || !betas || !ps || nbeta < 1 || np < 1 || !beta_out || !p_out)
        return fail(AAR_ERR_INVALID_ARG, "problem, params, b, candidates or outputs invalid");
    if (trial_iterations < 1)
        return fail(AAR_ERR_INVALID_ARG, "trial_iterations must be >= 1");
    aar_status st = validate_params(params);
    if (st != AAR_OK)
        return st;
    if ((st = validate_problem(*problem, 0)) != AAR_OK)
        return st;
    for (int i = 0; i < nbeta; ++i)
        if (!std::isfinite(betas[i]))
            return fail(AAR_ERR_INVALID_ARG, "beta candidates must be finite");
    for (int i = 0; i < np; ++i)
        if (ps[i] < 1)
            return fail(AAR_ERR_INVALID_ARG, "p candidates must be >= 1");
    const int64_t N = (int64_t)problem->n[0] * problem->n[1] * problem->n[2];
    hipStream_t s = (hipStream_t)hip_stream;
    double *x = nullptr;
    hipError_t he = hipMalloc(&x, sizeof(double) * N);
    if (he != hipSuccess)
        return fail(he == hipErrorOutOfMemory ? AAR_ERR_OUT_OF_MEMORY : AAR_ERR_DEVICE,
                    std::string("hipMalloc: ") + hipGetErrorString(he));
    double best = -1.0;
    aar_status result = AAR_OK;
    for (int ip = 0; ip < np && result == AAR_OK; ++ip) {
        for (int ib = 0; ib < nbeta && result == AAR_OK; ++ib) {
            aar_params pa = *params;
            pa.beta = betas[ib];
            pa.p = ps[ip];
            // a common budget: the trial's iterations rounded up to a multiple of p
            pa.max_iter = (trial_iterations + pa.p - 1) / pa.p * pa.p;
            pa.flags &= ~(uint32_t)AAR_FLAG_RECORD_RESIDUALS;
            aar_solver h = nullptr;
            if ((result = aar_create(&h, problem, 1, &pa, hip_stream)) != AAR_OK)
                break;
            double score = 0.0;
            aar_result r{};
            for (int rep = 0; rep < 2 && result == AAR_OK; ++rep) {   // the first run warms up
                if (hipMemsetAsync(x, 0, sizeof(double) * N, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess) {
                    result = fail(AAR_ERR_DEVICE, "aar_select_parameters: clearing x failed");
                    break;
                }
                const auto t0 = std::chrono::steady_clock::now();
                const aar_status e = aar_solve(h, b, x, &r);
                const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                if (e < 0) {
                    result = e;
                    break;
                }
                // decimal digits of residual reduction per second (0 for a
                // trial that broke down or grew the residual)
                const double digits = (e == AAR_BREAKDOWN || !(r.rel_residual > 0.0)) ? 0.0
                                      : -std::log10(r.rel_residual);
                score = std::max(0.0, digits) / std::max(dt, 1e-9);
            }
            (void)aar_destroy(h);
            if (result != AAR_OK)
                break;
            if (scores)
                scores[ip * nbeta + ib] = score;
            if (score > best) {
                best = score;
                *beta_out = pa.beta;
                *p_out = pa.p;
            }
        }
    }
    (void)hipFree(x);
    return result;
}

aar_status aar_destroy(aar_solver s)
{
    if (!s)
        return AAR_OK;
    (void)hipStreamSynchronize(s->stream);
    delete s;
    return AAR_OK;
}

aar_status aar_solve(aar_solver s, const double *b, double *x, aar_result *r)
{
    g_error.clear();
    if (!s || !b || !x)
        return fail(AAR_ERR_INVALID_ARG, "solver, b or x is NULL");
    if (s->ops.size() != 1)
        return fail(AAR_ERR_INVALID_ARG, "aar_solve needs a solver created with count == 1");
    if (s->cplx)
        return solve_complex(s, b, x, r);
    if (s->csr)
        return solve_csr(s, b, x, r);
    return solve_one(s, 0, b, x, r);
}

aar_status aar_solve_batched(aar_solver s, const double *b, double *x, const int64_t *offsets,
                             aar_result *results)
{
    g_error.clear();
    if (!s || !b || !x || !offsets || !results)
        return fail(AAR_ERR_INVALID_ARG, "solver, b, x, offsets or results is NULL");
    const int count = (int)s->ops.size();
    for (int i = 0; i < count; ++i) {
        if (offsets[i] < 0 || offsets[i + 1] - offsets[i] != s->ops[i].N)
            return fail(AAR_ERR_INVALID_ARG, "offsets do not match the system sizes (system " +
                                                 std::to_string(i) + ")");
    }
    if (s->cplx || s->csr)
        return fail(AAR_ERR_UNSUPPORTED, "complex and sparse systems are solved one by one (aar_solve)");
    if (s->B.on)
        return batch_solve(s, b, x, offsets, results);
    aar_status worst = AAR_OK;
    for (int i = 0; i < count; ++i) {
        aar_status st = solve_one(s, i, b + offsets[i], x + offsets[i], &results[i]);
        if (st < 0)
            return st;
        if (st > worst)
            worst = st;
    }
    return worst;
}

aar_status aar_apply(aar_solver s, int32_t instance, const double *x, double *y)
{
    g_error.clear();
    if (!s || !x || !y)
        return fail(AAR_ERR_INVALID_ARG, "solver, x or y is NULL");
    if (instance < 0 || instance >= (int)s->ops.size())
        return fail(AAR_ERR_INVALID_ARG, "instance out of range");
    if (s->csr) {
        CsrArgs a;
        std::memset(&a, 0, sizeof(a));
        a.c = s->cd;
        a.x = x;
        a.out = y;
        AAR_HIP(launch_csr(kApply, a, s->stream));
        AAR_HIP(hipStreamSynchronize(s->stream));
        return AAR_OK;
    }
    if (s->cplx) {
        StencilArgs<zd> a;
        std::memset(&a, 0, sizeof(a));
        a.st = s->pz.st;
        a.x = reinterpret_cast<const zd *>(x);
        a.out = reinterpret_cast<zd *>(y);
        AAR_HIP(launch_stencil_complex(kApply, s->pz.radius, s->pz.ts, a, nullptr, s->stream));
        AAR_HIP(hipStreamSynchronize(s->stream));
        return AAR_OK;
    }
    Path<double> P;
    bind_path(s, P, instance, true);
    StencilArgs<double> a;
    std::memset(&a, 0, sizeof(a));
    a.st = P.st;
    a.x = x;
    a.out = y;
    AAR_HIP(launch_stencil_f64(kApply, Prec::F64, P.radius, P.conv, P.ts, a, nullptr, s->stream));
    AAR_HIP(hipStreamSynchronize(s->stream));
    return AAR_OK;
}

aar_status aar_residual_log(aar_solver s, int32_t instance, double *out, int64_t cap, int64_t *count)
{
    g_error.clear();
    if (!s || !count || (cap > 0 && !out))
        return fail(AAR_ERR_INVALID_ARG, "solver, out or count invalid");
    if (instance < 0 || instance >= (int)s->ops.size())
        return fail(AAR_ERR_INVALID_ARG, "instance out of range");
    const double *log = s->B.on ? s->B.log : s->log;
    if (!log)
        return fail(AAR_ERR_INVALID_ARG, "solver created without AAR_FLAG_RECORD_RESIDUALS");
    if (!s->B.on && instance != s->last_instance && s->ops.size() > 1)
        return fail(AAR_ERR_UNSUPPORTED, "only the last solved system's log is kept");
    const int64_t have = std::min<int64_t>(s->last_log_count[instance], s->log_cap);
    *count = have;
    const int64_t n = std::min(have, cap);
    if (n > 0)
        AAR_HIP(hipMemcpy(out, log + (s->B.on ? (int64_t)instance * s->log_cap : 0), sizeof(double) * n,
                          hipMemcpyDeviceToHost));
    return AAR_OK;
}

aar_status aar_rank_log(aar_solver s, int32_t instance, int32_t *out, int64_t cap, int64_t *count)
{
    g_error.clear();
    if (!s || !count || (cap > 0 && !out))
        return fail(AAR_ERR_INVALID_ARG, "solver, out or count invalid");
    if (instance < 0 || instance >= (int)s->ops.size())
        return fail(AAR_ERR_INVALID_ARG, "instance out of range");
    const int32_t *log = s->B.on ? s->B.rank_log : s->rank_log;
    if (!log)
        return fail(AAR_ERR_INVALID_ARG, "solver created without AAR_FLAG_RECORD_RESIDUALS");
    if (!s->B.on && instance != s->last_instance && s->ops.size() > 1)
        return fail(AAR_ERR_UNSUPPORTED, "only the last solved system's log is kept");
    const int64_t have = std::min<int64_t>(s->last_log_count[instance], s->log_cap);
    *count = have;
    const int64_t n = std::min(have, cap);
    if (n > 0)
        AAR_HIP(hipMemcpy(out, log + (s->B.on ? (int64_t)instance * s->log_cap : 0), sizeof(int32_t) * n,
                          hipMemcpyDeviceToHost));
    return AAR_OK;
}

aar_status aar_set_timing(aar_solver s, int32_t enable)
{
    if (!s)
        return fail(AAR_ERR_INVALID_ARG, "solver is NULL");
    s->timing = enable != 0;
    s->t_total_ms = 0.0;
    s->t_launches = 0;
    s->tcycle.clear();
    s->tcount.clear();
    s->tused = 0;
    return AAR_OK;
}

aar_status aar_sweep_time(aar_solver s, double *total_ms, int64_t *launches)
{
    if (!s || !total_ms || !launches)
        return fail(AAR_ERR_INVALID_ARG, "argument is NULL");
    *total_ms = s->t_total_ms;
    *launches = s->t_launches;
    return AAR_OK;
}

}  // extern "C"
