// Internal device-side definitions shared by the solver's HIP sources.
//
// Data layout in HBM (per system):
//   x        two ping-pong copies (Richardson sweeps read one, write the other)
//   b        right-hand side
//   fring    m+1 slots of f_j = D^{-1}(b - A x_j); slot j mod (m+1) holds f_j
//   dxring   q = floor(m/p) slots of the Anderson increments x_{k+1} - x_k
//            (ring slots are N rounded up to 8 elements apart, so vector
//            accesses stay aligned)
//   fcur     f_k of the Anderson step in the bulk precision (bf16 history only)
// All vectors are x-fastest, one value per grid point: i + n0*(j + n1*k).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aar {

constexpr int kTX = 64;        // tile width along x: one wave64 row
constexpr int kWY = 4;         // waves per workgroup, stacked along y
constexpr int kThreads = kTX * kWY;
constexpr int kMaxRadius = 6;
constexpr int kMaxM = 32;      // history columns
constexpr int kMaxSlots = kMaxM + 1;
constexpr int kFastGramM = 12; // per-thread Gram accumulators up to this m
constexpr int kXcds = 8;       // MI355X: workgroups are dealt round-robin to 8 XCDs

enum class Prec : int { F64 = 0, F32 = 1, F32_BF16 = 2 };

// Per-system run state, written only by single-workgroup kernels.
enum : int32_t {
    kRunning = 0,
    kConverged = 1,
    kBreakdown = 2,
    kStagnated = 3,
    kMaxIter = 4,
};

struct alignas(64) InstState {
    int64_t cycle;          // completed Anderson cycles (p iterations each)
    int64_t iters;          // iterations at termination
    int64_t max_iter;       // iteration cap of this run
    double tol;             // tolerance of this run
    int32_t status;
    int32_t rank;           // rank kept by the last pseudoinverse
    double nb;              // ||b||_2
    double last_r;          // last measured ||b - A x_k|| / ||b||
    double best_r;          // stagnation tracking (inner solves)
    int32_t since_best;
    int32_t log_count;
    // update plan of the current Anderson step, x_{k+1} = x_k + sum alpha_t f_t + sum delta_a dx_a
    // first history position of the current run when the history is carried
    // over from a previous run (0: none); the difference column that spans it
    // pairs residuals of two right-hand sides and is left out (a null column)
    int64_t restart_pos;
    int32_t nf;             // number of f slots used (l + 1); the last one is f_k
    int32_t nd;             // number of dx slots used
    int32_t wslot;          // dx slot receiving x_{k+1} - x_k (-1: none kept)
    int32_t pad0;
    int32_t fslot[kMaxSlots];
    int32_t dslot[kMaxM];
    double alpha[kMaxSlots];
    double delta[kMaxM];
    // imaginary parts of the plan's coefficients (complex-valued systems)
    double alpha_im[kMaxSlots];
    double delta_im[kMaxM];
};

// bfloat16 storage: the upper half of an IEEE float, rounded to nearest even.
struct bf16_t {
    uint16_t bits;
};

// Complex FP64 value (the complex-valued systems of Eq. 1; the periodic
// Helmholtz problem of Eq. 7): stored interleaved (re, im), 16 bytes.
struct zd {
    double re, im;
    zd() = default;   // trivial (LDS arrays); zd() value-initializes to 0
    __host__ __device__ zd(double r) : re(r), im(0.0) {}
    __host__ __device__ zd(double r, double i) : re(r), im(i) {}
    __host__ __device__ zd &operator+=(const zd &o)
    {
        re += o.re;
        im += o.im;
        return *this;
    }
};
__host__ __device__ inline zd operator+(const zd &a, const zd &b) { return zd(a.re + b.re, a.im + b.im); }
__host__ __device__ inline zd operator-(const zd &a, const zd &b) { return zd(a.re - b.re, a.im - b.im); }
__host__ __device__ inline zd operator*(const zd &a, const zd &b)
{
    return zd(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__host__ __device__ inline zd operator/(const zd &a, const zd &b)
{
    const double d = b.re * b.re + b.im * b.im;
    return zd((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
__host__ __device__ inline zd conj(const zd &a) { return zd(a.re, -a.im); }

// |v|^2 in FP64 (the residual norms of the convergence test)
__host__ __device__ inline double sqnorm(double v) { return v * v; }
__host__ __device__ inline double sqnorm(float v) { return (double)v * (double)v; }
__host__ __device__ inline double sqnorm(const zd &v) { return v.re * v.re + v.im * v.im; }

template <typename H> struct Hist;
// store2: elements i and i + 1 (i even, p 16-byte aligned) in one store.
template <> struct Hist<double> {
    __device__ static inline double load(const double *p, int64_t i) { return p[i]; }
    __device__ static inline void store(double *p, int64_t i, double v) { p[i] = v; }
    __device__ static inline void store2(double *p, int64_t i, double v0, double v1)
    {
        *reinterpret_cast<double2 *>(p + i) = make_double2(v0, v1);
    }
};
template <> struct Hist<float> {
    __device__ static inline float load(const float *p, int64_t i) { return p[i]; }
    __device__ static inline void store(float *p, int64_t i, float v) { p[i] = v; }
    __device__ static inline void store(float *p, int64_t i, double v) { p[i] = (float)v; }
    template <typename V> __device__ static inline void store2(float *p, int64_t i, V v0, V v1)
    {
        *reinterpret_cast<float2 *>(p + i) = make_float2((float)v0, (float)v1);
    }
};
template <> struct Hist<zd> {
    __device__ static inline zd load(const zd *p, int64_t i) { return p[i]; }
    __device__ static inline void store(zd *p, int64_t i, const zd &v) { p[i] = v; }
};
template <> struct Hist<bf16_t> {
    __device__ static inline float load(const bf16_t *p, int64_t i)
    {
        return __uint_as_float(((uint32_t)p[i].bits) << 16);
    }
    __device__ static inline void store(bf16_t *p, int64_t i, float v)
    {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) {           // NaN stays a (quiet) NaN
            p[i].bits = (uint16_t)((u >> 16) | 0x40u);
            return;
        }
        u += 0x7fffu + ((u >> 16) & 1u);                 // round to nearest, ties to even
        p[i].bits = (uint16_t)(u >> 16);
    }
    __device__ static inline void store(bf16_t *p, int64_t i, double v) { store(p, i, (float)v); }
    template <typename V> __device__ static inline void store2(bf16_t *p, int64_t i, V v0, V v1)
    {
        bf16_t t[2];
        store(t, 0, (float)v0);
        store(t, 1, (float)v1);
        *reinterpret_cast<uint32_t *>(p + i) = (uint32_t)t[0].bits | ((uint32_t)t[1].bits << 16);
    }
};

// Operator description passed by value to the stencil kernels.
template <typename T> struct StencilDev {
    int32_t n0, n1, n2;
    int32_t per0, per1, per2;   // 1: periodic axis, 0: zero Dirichlet
    T c0[kMaxRadius + 1];       // -a w_s / h_0^2, s = 1..r (index 0 unused)
    T c1[kMaxRadius + 1];
    T c2[kMaxRadius + 1];
    T sigma;
    T diag;                     // centre weight of the stencil: sigma - 2 sum_axes sum_s c[s]
    // Jacobi preconditioner D = diag(A) without convection: the centre weight
    // plus the taps that a periodic axis shorter than the stencil wraps back
    // onto the point itself (equal to diag when every periodic n >= 2r + 1)
    T jdiag;
    T inv_diag;                 // 1 / jdiag
    T ih0, ih1, ih2;            // 1/h per axis (upwind convection)
    const T *vel;               // planar [vx|vy|vz] or nullptr
    int64_t N;
};

enum StencilMode : int {
    kSweep = 0,   // f = D^-1 (b - A x); out = x + omega f; ring <- f
    kFk = 1,      // f_k = D^-1 (b - A x); ring <- f_k; partial += ||b - A x||^2
    kResid = 2,   // out = b - A x; partial += ||b - A x||^2
    kApply = 3,   // out = A x
    kPrecond = 4, // sparse A only: out = M^-1 x
};

template <typename T> struct StencilArgs {
    StencilDev<T> st;
    const T *x;
    const T *b;
    T *out;
    void *fring;            // H-typed ring base
    T *fcur;                // kFk: f_k copy in T when the ring is bf16
    double *partial;        // one double per workgroup
    const InstState *state; // kSweep / kFk: run state for early exit and slot index
    int64_t slot_stride;    // elements per ring slot
    int32_t j;              // position within the cycle (0..p-1)
    int32_t p;
    int32_t nslots;         // m + 1
    int32_t cz;             // z planes per workgroup
    int32_t tiles_x, tiles_y, tiles_z;
    int32_t order;          // kOrder* bits: tile numbering and z direction
    T omega;
    double *gram_partial;   // kFk, paired layout, m = kFusedGramM: [ne][blocks] Gram partials, else null
    // kSweep / kFk, ring type T (either layout): the residual recursion of
    // Richardson steps.  The input is ring slot k - 1 (f_{k-1}) instead of x,
    // b is not read, f_k = f_{k-1} - omega D^-1 A f_{k-1}, and kFk's norm is
    // that of D f_k (= b - A x_k); kSweep then writes no x (out may be null).
    int32_t recur;
};

// History length whose Gram products the paired Anderson-residual pass forms
// itself (the evaluation workloads' m) when the iterate is FP64 and the
// history FP64 or FP32; other lengths and precisions use the separate Gram pass.
constexpr int kFusedGramM = 7;
constexpr int kFusedGramNE = kFusedGramM * (kFusedGramM + 1) / 2 + kFusedGramM;

// Batched systems: one descriptor per system; packed vectors hold system i
// at element offset `off` (64-byte aligned) in every array.
template <typename T> struct BatchDesc {
    StencilDev<T> st;
    int64_t off;
    int32_t tiles_x, tiles_y, tiles_z, cz;
    int32_t ntiles;          // stencil tiles
    int32_t nchunks;         // streaming chunks of kChunk points
};

constexpr int kChunk = 8192;   // points per streaming work item of the batched passes

template <typename T> struct BatchStencilArgs {
    const BatchDesc<T> *desc;
    const int2 *items;       // (system, tile)
    const int *nitems;
    const T *x;
    const T *b;
    T *out;
    void *fring;             // H-typed, slot stride slot_stride
    T *fcur;
    double *partial;         // one per work item (kFk, kResid)
    const InstState *state;  // per system
    const int *mask;         // kResid: systems to process (nonzero)
    int64_t slot_stride;
    int32_t j, p, nslots;
    T omega;
    int32_t recur;           // kSweep / kFk: the residual recursion (see StencilArgs)
};

// ---- batched driver ----
enum : int32_t { kPhaseStart = 0, kPhaseInner = 1, kPhaseDone = 2 };

// Inner FP32 tolerance of one refinement step when none is given: each step
// reduces the FP64 residual by at least kInnerTolDefault (three steps reach
// 1e-10), and the last one only by what remains, half of tol / rel, where rel
// is the FP64 relative residual the step starts from.  A deeper inner target
// runs the FP32 solve into its accuracy floor, kappa(A) u_32, where its
// iterations stop paying.
constexpr double kInnerTolDefault = 3e-4;
__host__ __device__ inline double inner_tolerance(double given, double tol, double rel)
{
    if (given > 0.0)
        return given;
    const double need = 0.5 * tol / rel;
    const double eta = need > kInnerTolDefault ? need : kInnerTolDefault;
    return eta < 0.5 ? eta : 0.5;
}

struct BatchCtl {            // per-system control of a batched solve
    int32_t phase;
    int32_t status;          // final aar status of the system
    int32_t outer;           // refinement steps taken
    int32_t dsel;            // buffer holding the last run's answer (0: xa, 1: xb)
    int32_t zero;            // b == 0: the answer is x = 0
    int32_t pad;
    int64_t used;            // iterations used so far
    int64_t iters_last;      // iterations of the last run
    double rnorm;            // ||r|| of the current refinement step
    double nb64;             // ||b|| (FP64)
    double rel;              // last FP64 relative residual
    double mean;             // deflation: mean of r
};

struct CompactArgs {
    int32_t mode;            // 0: running inner systems, 1: refine != 0, 2: all systems
    int32_t count;
    const BatchCtl *ctl;
    const InstState *state;
    const int *refine;
    const int *ntiles;
    const int *nchunks;
    int2 *sitems;
    int2 *citems;
    int *nsitems;
    int *ncitems;
    int *sbase;
    int *cbase;
};

struct BatchGramArgs {
    const int2 *items;
    const int *nitems;
    const InstState *state;
    const void *fring;
    const int64_t *offs;
    const int64_t *sizes;
    double *partial;         // [item][ne]
    int64_t slot_stride;
    int32_t m, p, nslots;
};

struct BatchLsqArgs {
    InstState *state;
    const int *sbase;
    const int *cbase;
    const int *ntiles;
    const int *nchunks;
    const double *rho_partial;   // per stencil item
    const double *gram_partial;  // per chunk item, ne entries each
};

template <typename T> struct BatchUpdateArgs {
    const int2 *items;
    const int *nitems;
    const InstState *state;
    const int64_t *offs;
    const int64_t *sizes;
    const T *xin;
    T *xout;
    const void *fring;
    const T *fcur;
    void *dxring;           // DxOf<T, H> elements
    int64_t slot_stride;
    int64_t dx_stride;
    T omega_rich = 0;       // residual recursion: as in UpdateArgs
    int32_t p_rich = 0;
};

enum : int32_t {
    kOpGather = 0, kOpScatter = 1, kOpNorm = 2, kOpSum = 3, kOpCorrect = 4, kOpDeflate = 5, kOpPrepare = 6,
    kOpZero64 = 7, kOpScatterSel = 8, kOpScatterRecur = 9,
};

struct BatchStreamArgs {
    const int2 *items;
    const int *nitems;
    int32_t op;
    int32_t mask_min;        // process systems with mask >= mask_min (mask may be null)
    const int *mask;
    const BatchCtl *ctl;
    const int64_t *offs;
    const int64_t *sizes;
    const int64_t *uoffs;    // caller's offsets (gather / scatter)
    double *user;
    double *v64;
    double *x64;
    float *xa32;             // kOpCorrect reads, kOpPrepare zeroes xa32
    const float *xb32;
    float *rhs32;
    const double *inv_shift;
    double *partial;         // per item, or null
    // runs that used the residual recursion: their answer is the cycle-start
    // iterate plus omega times the Richardson f of the unfinished cycle
    // (kOpScatterRecur: FP64 v64, FP64 ring or FP32 ring when ring_f32 is
    // set; kOpCorrect with recur set: FP32 xa32 and ring)
    const InstState *state;
    const void *fring;
    int64_t slot_stride;
    int32_t p, nslots;
    double omega;
    int32_t recur;
    int32_t ring_f32;
};

enum : int32_t { kCtlSelect = 0, kCtlNormB = 1, kCtlMean = 2, kCtlDecide = 3, kCtlStart = 4 };

struct BatchCtlArgs {
    int32_t step;
    int32_t p;
    int32_t mixed;
    int32_t deflate;
    int32_t max_outer;
    int32_t pad;
    int64_t max_iter;
    double tol, inner_tol;
    BatchCtl *ctl;
    InstState *state;
    int *refine;
    int *remaining;
    const double *partial;
    const int *sbase;
    const int *cbase;
    const int *ntiles;
    const int *nchunks;
    const int64_t *sizes;
};

hipError_t launch_compact(const CompactArgs &a, hipStream_t s);
hipError_t launch_gram_batched(Prec prec, const BatchGramArgs &a, int grid, hipStream_t s);
hipError_t launch_update_batched(Prec prec, const BatchUpdateArgs<double> *a64, const BatchUpdateArgs<float> *a32,
                                 int grid, hipStream_t s);
hipError_t launch_stream_batched(const BatchStreamArgs &a, int grid, hipStream_t s);
hipError_t launch_ctl_batched(const BatchCtlArgs &a, int count, hipStream_t s);

struct GramArgs {
    const void *fring;
    double *partial;        // [ne][gridDim.x] (entry-major)
    const InstState *state;
    int64_t N;
    int64_t slot_stride;
    int32_t m, p, nslots;
    int32_t ne;             // m(m+1)/2 + m
};

struct LsqArgs {
    InstState *state;
    const double *rho_partial;   // from the kFk stencil pass
    int32_t rho_blocks;
    const double *gram_final;    // G (upper triangle) and c, summed by k_gram_finish
    int32_t ne;
    // non-null: the per-workgroup partials of the fused Gram pass (entry-major,
    // gram_blocks per entry, kFusedGramNE entries), summed by the solve kernel
    // itself in place of gram_final
    const double *gram_partial = nullptr;
    int32_t gram_blocks = 0;
    int32_t m, p, nslots, q;     // q: dx ring slots (0: none kept)
    double omega, beta;
    double rcond;                // pseudoinverse threshold factor (times l * lambda_max)
    int32_t stagnation_window;   // 0: off
    double stagnation_factor;    // best_r must fall below factor * best_r within the window
    double *log;                 // residual log or nullptr
    int64_t log_cap;
    // beside the residual log (same index): the rank kept by that Anderson
    // step's pseudoinverse solve, -1 for the step whose test stopped the run
    int32_t *rank_log = nullptr;
    // nonzero: skip the Cholesky shortcut, so every solve takes the
    // eigendecomposition (a check of that branch on well-posed data)
    int32_t force_pinv = 0;
};

// Element type of the ring of Anderson increments x_{k+1} - x_k (the X_k
// columns of Anderson steps, Eq. 4): the iterate's type, except FP32 beside an
// FP32 history ring of an FP64 iteration, where like the f_j it is only an
// extrapolation direction.
template <typename T, typename H> struct DxOf {
    using type = T;
};
template <> struct DxOf<double, float> {
    using type = float;
};

template <typename T> struct UpdateArgs {
    const T *xin;
    T *xout;
    const void *fring;
    const T *fcur;          // non-null: use instead of the ring slot for f_k
    void *dxring;           // DxOf<T, H> elements, slots dx_stride elements apart
    const InstState *state;
    int64_t N;
    int64_t slot_stride;    // elements between f slots, a multiple of 8
    int64_t dx_stride;      // elements between dx slots, a multiple of 8
    // non-null: pinned host word that workgroup 0 sets to the run status on
    // entry, so the host polls it without a copy on the stream
    int32_t *status_out = nullptr;
    // p_rich > 0 (residual recursion): xin is the cycle's first iterate x_c,
    // and the p_rich - 1 Richardson steps of the cycle are applied first,
    // x_k = x_c + omega_rich sum f_j over history positions nf - p_rich ..
    // nf - 2; the increment kept is then x_{k+1} - x_k
    T omega_rich = 0;
    int32_t p_rich = 0;
};

// Workgroup index -> logical tile index so that each XCD (and its L2) gets a
// contiguous range of tiles: neighbouring tiles share halos through L2.
__device__ inline int xcd_tile(int b, int nb)
{
    int xcd = b % kXcds, idx = b / kXcds;
    int per = nb / kXcds, rem = nb % kXcds;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// ---------------------------------------------------------------------------
// Host-side launch helpers (implemented in the .hip sources)
// ---------------------------------------------------------------------------

// Tile order bits.  kOrderAltZ: odd z chunks march downwards, so two
// z-neighbouring chunks read the planes they share at the same moment (both
// at their start or both at their end) and the second read hits L2.
// kOrderZFast: consecutive tile numbers (one XCD's share) run along z first,
// so z-neighbours sit on the same XCD; otherwise along x, then y.
constexpr int kOrderAltZ = 1;
constexpr int kOrderZFast = 2;

constexpr int kTbMaxDepth = 5;   // deepest temporal block of recursion steps

struct TileShape {
    int ry;      // y rows per thread (tile height = kWY * ry; 2 kWY * ry paired)
    int cz;      // z planes per workgroup
    int order = 0;   // kOrder* bits
    int pair = 0;    // paired layout for the sweep and residual passes: 1, 2, 3 = 4, 8, 16 waves
    int tb = 0;      // temporal block depth of the recursion steps (0, 1: one pass per step)
};

// The paired layout (each thread owns two x-adjacent points, loaded and
// stored as one vector) serves the Richardson sweep and the Anderson-step
// residual of grids with an even x extent and no convection.
inline bool paired_layout(const TileShape &ts, int n0, bool conv, int mode)
{
    return ts.pair != 0 && (n0 % 2) == 0 && !conv && (mode == kSweep || mode == kFk);
}

// Paired shapes that are compiled: pair p uses 4 << (p - 1) waves per
// workgroup; FP64 keeps at most 8 waves and 2 rows per thread (its register
// queue would not fit more), FP32 also has 8 waves x 2 rows and 16 waves.
inline bool paired_shape_ok(const TileShape &ts, bool f64)
{
    switch (ts.pair) {
    case 0:
        return true;
    case 1:
        return ts.ry == 1 || ts.ry == 2;
    case 2:
        return ts.ry == 1 || (!f64 && ts.ry == 2);
    case 3:
        return !f64 && ts.ry == 1;
    default:
        return false;
    }
}

// Stencil pass; T is double for Prec::F64 and float otherwise; history type
// follows prec.  Returns hipSuccess or the launch error.
hipError_t launch_stencil_f64(int mode, Prec hist, int radius, bool conv, const TileShape &ts,
                              StencilArgs<double> a, int *blocks_out, hipStream_t s);
hipError_t launch_stencil_f32(int mode, Prec hist, int radius, bool conv, const TileShape &ts,
                              StencilArgs<float> a, int *blocks_out, hipStream_t s);
// FP64 iterate with an FP32 or bfloat16 history (kSweep, kFk)
hipError_t launch_stencil_f64_narrow(int mode, Prec hist, int radius, bool conv, const TileShape &ts,
                                     StencilArgs<double> a, int *blocks_out, hipStream_t s);
void stencil_grid(int n0, int n1, int n2, const TileShape &ts, int *tx, int *ty, int *tz, int *blocks,
                  bool paired = false);
hipError_t launch_stencil_batched_f64(int mode, Prec hist, int radius, bool conv, int ry,
                                      const BatchStencilArgs<double> &a, int grid, hipStream_t s);
hipError_t launch_stencil_batched_f64_narrow(int mode, Prec hist, int radius, bool conv, int ry,
                                             const BatchStencilArgs<double> &a, int grid, hipStream_t s);
hipError_t launch_stencil_batched_f32(int mode, Prec hist, int radius, bool conv, int ry,
                                      const BatchStencilArgs<float> &a, int grid, hipStream_t s);

// Temporal block of nt recursion steps at cycle positions j0 .. j0+nt-1
// (j0 >= 1; one-point tiles, radius <= 2, ring of the iterate's type); the
// last stage is the Anderson-step residual with its norm partial when
// last_fk.  tblock_fits: whether that block's LDS rings fit a workgroup.
bool tblock_fits(int radius, bool conv, const TileShape &ts, int nt, bool f64);
hipError_t launch_tblock_f64(int radius, bool conv, const TileShape &ts, StencilArgs<double> a, int j0, int nt,
                             bool last_fk, hipStream_t s);
hipError_t launch_tblock_f32(int radius, bool conv, const TileShape &ts, StencilArgs<float> a, int j0, int nt,
                             bool last_fk, hipStream_t s);

hipError_t launch_gram(Prec prec, const GramArgs &a, int blocks, hipStream_t s);
hipError_t launch_lsq(const LsqArgs &a, hipStream_t s);
hipError_t launch_lsq_batched(const LsqArgs &base, const BatchLsqArgs &b, int count, hipStream_t s);

hipError_t launch_gram_finish(const double *partial, int blocks, double *out, int ne, const InstState *state,
                              int p, hipStream_t s);
hipError_t launch_update(Prec prec, const UpdateArgs<double> *a64, const UpdateArgs<float> *a32, int blocks,
                         hipStream_t s);
// Residual recursion: x += omega * (the Richardson f_j of the unfinished cycle)
// once a run has stopped (FP64 iterate with an FP64 or FP32 ring; FP32
// iterate and ring for the inner solves of the mixed mode).
hipError_t launch_finalize_f64(Prec hist, double *x, const void *fring, const InstState *state, int p, int nslots,
                               int64_t slot_stride, double omega, int64_t N, hipStream_t s);
hipError_t launch_finalize_f32(float *x, const void *fring, const InstState *state, int p, int nslots,
                               int64_t slot_stride, float omega, int64_t N, hipStream_t s);
hipError_t launch_norm_partial(bool f64, const void *v, int64_t N, double *partial, int blocks, hipStream_t s);
hipError_t launch_init_state(InstState *st, const double *partial, int blocks, int64_t max_iter, double tol,
                             hipStream_t s);
// Start a run that keeps the history of the previous one (which ended at an
// Anderson step): the positions continue after it, budget iterations from there.
hipError_t launch_init_state_keep(InstState *st, const double *partial, int blocks, int64_t budget, double tol,
                                  int p, hipStream_t s);
hipError_t launch_finish_norm(double *out, const double *partial, int blocks, hipStream_t s);
hipError_t launch_cast_f64_to_f32(const double *in, float *out, int64_t N, const double *scale_inv_of,
                                  hipStream_t s);
hipError_t launch_zero_f32(float *v, int64_t N, hipStream_t s);
hipError_t launch_correct(double *x, const float *d, const double *scale, int64_t N, hipStream_t s);
hipError_t launch_copy_f64(const double *in, double *out, int64_t N, hipStream_t s);
hipError_t launch_cast_f64_f32_plain(const double *in, float *out, int64_t N, hipStream_t s);
hipError_t launch_zero_f64(double *v, int64_t N, hipStream_t s);
hipError_t launch_fill_pattern_f64(double *v, int64_t N, hipStream_t s);
hipError_t launch_fill_pattern_f32(float *v, int64_t N, hipStream_t s);
// constant-mode deflation: mean of r -> scal[2]; x += mean * inv_sigma; r -= mean; partial ||r||^2
hipError_t launch_deflate(double *x, double *r, int64_t N, double inv_sigma, double *partial, int blocks,
                          double *scal, hipStream_t s);

// Complex-valued systems (complex.hip)
hipError_t launch_stencil_complex(int mode, int radius, const TileShape &ts, StencilArgs<zd> a, int *blocks_out,
                                  hipStream_t s);
// Imaginary parts of the Hermitian Gram products (the real parts come from
// launch_gram over the interleaved vectors).
hipError_t launch_cgram(const GramArgs &a, int blocks, hipStream_t s);
hipError_t launch_clsq(const LsqArgs &a, double omega_im, double beta_im, hipStream_t s);
hipError_t launch_cupdate(const UpdateArgs<zd> &a, int blocks, hipStream_t s);
hipError_t launch_cnorm_partial(const zd *v, int64_t N, double *partial, int blocks, hipStream_t s);

int stream_blocks(int64_t N);
int gram_blocks(int64_t N, int m);

// ---------------------------------------------------------------------------
// General sparse A (compressed sparse rows) with the Jacobi or block-Jacobi
// ILU(0) preconditioner (sparse.hip).
// ---------------------------------------------------------------------------

// Largest LDS a sparse block may hold: its rows' values during the
// substitutions (FP64).
constexpr size_t kCsrMaxLds = 128 * 1024;
constexpr int kCsrMaxBlockRows = (int)(kCsrMaxLds / sizeof(double));

struct CsrDev {
    int64_t n;
    const int64_t *rowptr;   // n + 1
    const int32_t *col;      // strictly increasing per row, diagonal present
    const double *val;
    double *lu;              // ILU(0) factors in A's pattern (entries inside each block), or null
    const int64_t *dpos;     // position of each row's diagonal entry
    const int64_t *bstart;   // nblocks + 1 row bounds of the blocks
    // level schedules of each block: rows grouped by level of the forward
    // (lrows, lptr) and backward (urows, uptr) substitution; block t owns
    // levels blev_l[t] .. blev_l[t+1] - 1 (and likewise blev_u)
    const int32_t *lrows, *urows;
    const int32_t *lptr, *uptr;
    const int32_t *blev_l, *blev_u;
    int nblocks;
    int max_block_rows;
    int ilu;                 // 1: block ILU(0); 0: Jacobi (blocks are plain row chunks)
    // packed substitution records (kp > 0): for position q of lrows (urows),
    // the block-local row frow[q] (brow[q]) and kp slots of (block-local
    // column, factor value) in increasing column order, padded with column
    // -1; bdiag[q] = u_ii.  kp = 0: the substitutions walk the CSR arrays.
    int kp;
    const int16_t *frow, *fcol, *brow, *bcol;
    const double *fval, *bval, *bdiag;
    // > 0: the packed substitutions stage each block's level bounds in LDS
    // after its values; lev_lds = the most levels of a block (forward plus
    // backward) + 2
    int lev_lds;
    // levels the packed records are loaded ahead: 1, 2 or 4 (4 with kp = 4
    // only)
    int depth;
};

// Dynamic LDS of a block-ILU(0) pass: the block's values, then (packed
// substitutions) its level bounds.
inline size_t csr_lds_bytes(const CsrDev &c)
{
    return (size_t)c.max_block_rows * sizeof(double) + (size_t)c.lev_lds * sizeof(int32_t);
}

// Largest number of in-block entries per triangular row the packed records
// hold.
constexpr int kCsrMaxPack = 8;

struct CsrArgs {
    CsrDev c;
    const double *x;         // kSweep / kFk / kApply: the iterate (any row is read); kPrecond: the input
    const double *b;
    double *xout;            // kSweep: x + omega f
    double *out;             // kApply: A x; kPrecond: M^-1 x
    void *fring;             // kSweep / kFk: history ring (FP64)
    const InstState *state;
    int64_t slot_stride;
    int j, p, nslots;
    double omega;
    double *partial;         // kFk: one ||b - A x||^2 partial per block
};

// Allow the block-ILU(0) passes the LDS of the largest block (call once per
// device before the first launch, outside any stream capture).
hipError_t prepare_csr_kernels();
hipError_t launch_csr(int mode, const CsrArgs &a, hipStream_t s);
hipError_t launch_ilu0(const CsrDev &c, int *bad, hipStream_t s);
// Fill the packed records' values from the factors (after launch_ilu0):
// fval/bval slot s of record q takes lu[fe/be[q kp + s]] (0 for padding),
// bdiag[q] = lu[dpos[urows[q]]].
hipError_t launch_pack_factors(const CsrDev &c, const int32_t *fe, const int32_t *be, double *fval, double *bval,
                               double *bdiag, hipStream_t s);

}  // namespace aar
