// ppmlr_lib.hip -- host side of the C ABI declared in include/ppmlr.h:
// context and grid tables, kernel launches for sweeps and split steps, the
// CFL reduction, deterministic totals, counters and the device-resident
// time-step loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ppmlr.h"
#include "ppmlr_iono.hpp"
#include "ppmlr_sweep.hpp"

using ppmlr::kG;
using ppmlr::kSlotsA;
using ppmlr::kSlotsB;
using ppmlr::kStatWords;
using ppmlr::kStatSlots;

struct AxisTables {
    // FP64 and FP32 copies: extended widths [M], centres [M], faces [M+1];
    // interior widths and centres [n]
    double *dx64 = nullptr, *xc64 = nullptr, *xf64 = nullptr, *dxi64 = nullptr, *xci64 = nullptr;
    float *dx32 = nullptr, *xc32 = nullptr, *xf32 = nullptr, *dxi32 = nullptr, *xci32 = nullptr;
};

struct ppmlr_ctx {
    int n[3];
    int bc_lo[3], bc_hi[3];
    double r_inner = 0.0;
    double gamma = 5.0 / 3.0;
    ppmlr_options opt;
    std::vector<double> faces[3];
    std::vector<double> ext_dx[3], ext_xc[3], ext_xf[3];
    AxisTables tab[3];
    double dip_m = 0.0, dir[3] = {0.0, 0.0, -1.0}, bext[3] = {0.0, 0.0, 0.0};
    double inflow[8] = {1, 0, 0, 0, 0, 0, 0, 1};
    double inner_rho = 1.0, inner_p = 1.0;
    unsigned long long *d_stats = nullptr;   // kStatSlots x kStatWords
    unsigned long long *d_cflmax = nullptr;  // signal-speed max (double bits), kCflSlots slots
    double *d_dt = nullptr;                  // device-resident dt
    double *d_time = nullptr;                // accumulated simulated time
    double *d_series = nullptr;              // inflow time series: rows (t, prim[8])
    int series_n = 0, series_cap = 0;
    double *d_inflow = nullptr;              // the current step's inflow from the series (8 values)
    double *d_partials = nullptr;            // totals partial sums
    int partial_blocks = 0;
    long long step = 0;
    int tile[3] = {0, 0, 0};
    int seg[3] = {0, 0, 0};                  // segments per pencil (0: automatic)
    int seg_order[3] = {0, 0, 0};            // tile order of segments (0: automatic, 1: adjacent, 2: bands)
    void *d_pong = nullptr;                  // second state for segmented sweeps
    size_t pong_bytes = 0;
    int device = 0;
    std::string err;
    // profiling: event pairs around sweep launches
    bool profiling = false;
    struct Mark { hipEvent_t start, stop; int axis; };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> event_pool;
    // learned Riemann guess
    int guess = PPMLR_GUESS_PLAIN;
    unsigned short *d_mlp_frag = nullptr;    // packed BF16 weight fragments
    float *d_mlp_theta = nullptr;            // FP32 parameters
    double gate_p = 0.1, gate_u = 0.1;
    float *harvest = nullptr;                // caller-owned interface records
    long long harvest_cap = 0;
    unsigned long long *harvest_count = nullptr;
    // ionosphere coupling: shell buffers (j_r, Phi, pole values) and the
    // drift of the reset zones over an index box
    double *d_iono = nullptr;
    size_t iono_bytes = 0;
    double *d_inner_v = nullptr;
    size_t inner_v_bytes = 0;
    int inner_box[6] = {0, 0, 0, 0, 0, 0};
    bool inner_drift = false;
};

struct ppmlr_mlp {
    int device = 0;
    int max_batch = 0;
    unsigned short *d_frag = nullptr;        // packed fragments of the current parameters
    float *d_partials = nullptr;             // [max_batch / 64][kNPar + 1]
    std::string err;
};

namespace {

constexpr int kTotBlocks = 1024;  // fixed block count of the totals reduction

ppmlr_status fail(ppmlr_ctx *c, ppmlr_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

ppmlr_status hip_check(ppmlr_ctx *c, hipError_t e, const char *what)
{
    if (e == hipSuccess) return PPMLR_OK;
    return fail(c, e == hipErrorOutOfMemory ? PPMLR_ENOMEM : PPMLR_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
ppmlr_status upload(ppmlr_ctx *c, T **dst, const std::vector<double> &src)
{
    std::vector<T> tmp(src.begin(), src.end());
    ppmlr_status s = hip_check(c, hipMalloc((void **)dst, sizeof(T) * std::max<size_t>(tmp.size(), 1)), "hipMalloc");
    if (s) return s;
    return hip_check(c, hipMemcpy(*dst, tmp.data(), sizeof(T) * tmp.size(), hipMemcpyHostToDevice), "hipMemcpy");
}

// Extended geometry of one axis: ghost widths wrap on periodic axes and are
// mirrored otherwise; ghost faces continue from the domain faces.
void extend_axis(ppmlr_ctx *c, int a)
{
    const int N = c->n[a], M = N + 2 * kG;
    const std::vector<double> &f = c->faces[a];
    std::vector<double> &dx = c->ext_dx[a], &xc = c->ext_xc[a], &xf = c->ext_xf[a];
    dx.assign(M, 0.0);
    xc.assign(M, 0.0);
    xf.assign(M + 1, 0.0);
    auto width = [&](int k) { return f[k + 1] - f[k]; };
    for (int i = 0; i < M; ++i) {
        int gi = i - kG;
        if (gi >= 0 && gi < N) {
            dx[i] = width(gi);
        } else if (gi < 0) {
            if (c->bc_lo[a] == PPMLR_PERIODIC) dx[i] = width(((gi % N) + N) % N);
            else dx[i] = width(std::min(-gi - 1, N - 1));
        } else {
            if (c->bc_hi[a] == PPMLR_PERIODIC) dx[i] = width(gi % N);
            else dx[i] = width(std::max(2 * N - 1 - gi, 0));
        }
    }
    for (int k = 0; k <= N; ++k) xf[kG + k] = f[k];
    for (int i = kG + N; i < M; ++i) xf[i + 1] = xf[i] + dx[i];
    for (int i = kG - 1; i >= 0; --i) xf[i] = xf[i + 1] - dx[i];
    for (int i = 0; i < M; ++i) xc[i] = 0.5 * (xf[i] + xf[i + 1]);
}

void free_tables(ppmlr_ctx *c)
{
    for (int a = 0; a < 3; ++a) {
        AxisTables &t = c->tab[a];
        void *ptrs[] = {t.dx64, t.xc64, t.xf64, t.dxi64, t.xci64, t.dx32, t.xc32, t.xf32, t.dxi32, t.xci32};
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
        t = AxisTables();
    }
    void *more[] = {c->d_stats, c->d_cflmax, c->d_dt, c->d_time, c->d_partials};
    for (void *p : more)
        if (p) (void)hipFree(p);
    c->d_stats = nullptr;
    c->d_cflmax = nullptr;
    c->d_dt = nullptr;
    c->d_time = nullptr;
    c->d_partials = nullptr;
}

bool has_background(const ppmlr_ctx *c)
{
    return c->dip_m != 0.0 || c->bext[0] != 0.0 || c->bext[1] != 0.0 || c->bext[2] != 0.0;
}

// Threads needed for a tile of P pencils, rounded to whole waves.
int block_threads(int P, int M) { return ((P * M + 63) / 64) * 64; }

// Segments of a pencil of N zones cut into `nseg`: interior length of all but
// the last (which is shorter or equal, and not empty); 0 if nseg is invalid.
int seg_len(int N, int nseg)
{
    if (nseg < 1 || nseg > N) return 0;
    const int L = (N + nseg - 1) / nseg;
    return (nseg - 1) * L < N ? L : 0;
}

constexpr int kMaxSegments = 8;           // autotuner's search range

int stride_for(int threads, int elem);

// Segments per pencil: the context's setting, or (0 = automatic) the fewest
// whose tile of one pencil segment fits a workgroup and the LDS (one for
// any FP32 pencil up to 1010 zones).
int seg_count(const ppmlr_ctx *c, int axis, int elem)
{
    if (c->seg[axis] > 0) return c->seg[axis];
    const int N = c->n[axis];
    for (int k = 1; k <= N; ++k) {
        const int L = seg_len(N, k);
        if (L == 0) continue;
        const int thr = block_threads(1, L + 2 * kG);
        if (thr <= 1024 && stride_for(thr, elem) >= 0) return k;
    }
    return 1;
}

// Whether the segments of a pencil group are adjacent in the tile order (1)
// or the grid is dealt out one segment band after another (0).  Automatic:
// adjacent for x, bands for y and z (measured on the 256x192x192 sweeps:
// bands take the z sweep from 0.42 to 0.36 ms, cost x 10 %).
int seg_fast_for(const ppmlr_ctx *c, int axis)
{
    if (c->seg_order[axis] == 1) return 1;
    if (c->seg_order[axis] == 2) return 0;
    return axis == 0 ? 1 : 0;
}

// Zones of one tile's pencil segment (interior + ghosts).
int tile_M(const ppmlr_ctx *c, int axis, int elem) { return seg_len(c->n[axis], seg_count(c, axis, elem)) + 2 * kG; }

// LDS stride of a sweep launch with `threads` lanes: the smallest of the
// compile-time strides 256, 384, ..., 1024 (steps of 128) that holds them and
// whose two buffers fit the 160 KB LDS; 0 = the exact runtime stride (an
// FP64 tile of 832 lanes, whose rounded stride would not fit); -1 = does not
// fit.  A stride close to the workgroup size leaves LDS for more resident
// workgroups per CU.
int stride_for(int threads, int elem)
{
    if (threads > 1024) return -1;
    const int sm = threads <= 256 ? 256 : (threads + 127) / 128 * 128;
    if (ppmlr::lds_bytes(kSlotsA + kSlotsB, sm, elem) <= 160 * 1024) return sm;
    if (ppmlr::lds_bytes(kSlotsA + kSlotsB, threads, elem) <= 160 * 1024 && elem == 8) return 0;
    return -1;
}

// Automatic tile: the number of pencil segments per workgroup that wastes the
// fewest lanes (padding to whole waves plus ghost zones), within the thread
// budget.
int auto_tile(const ppmlr_ctx *c, int axis, int elem)
{
    const int L = seg_len(c->n[axis], seg_count(c, axis, elem)), M = L + 2 * kG;
    const int cap = (elem == 8) ? 512 : 1024;
    const int nq = (axis == 0) ? c->n[1] : c->n[0];
    int best = 1;
    double best_cost = 1e30;
    for (int P = 1; P <= 16; ++P) {
        int thr = block_threads(P, M);
        if (thr > cap && P > 1) break;
        if (stride_for(block_threads(P, M), elem) < 0) break;
        int tiles_q = (nq + P - 1) / P;
        double cost = (double)thr * tiles_q / ((double)L * nq);  // lanes per useful zone
        if (cost < best_cost - 1e-9) { best_cost = cost; best = P; }
    }
    return best;
}

int pick_tile(const ppmlr_ctx *c, int axis, int elem)
{
    return c->tile[axis] > 0 ? c->tile[axis] : auto_tile(c, axis, elem);
}

template <typename T>
void fill_args(const ppmlr_ctx *c, ppmlr::SweepArgs<T> &a, const T *in, T *u, int axis, double dt,
               const double *dt_dev, int P, int nseg)
{
    const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
    const int N = c->n[axis], L = seg_len(N, nseg), M = L + 2 * kG;
    const bool f64 = sizeof(T) == 8;
    auto tabs = [&](int ax, const T *&dx, const T *&xc, const T *&xf, const T *&dxi, const T *&xci) {
        const AxisTables &t = c->tab[ax];
        if (f64) {
            dx = (const T *)t.dx64; xc = (const T *)t.xc64; xf = (const T *)t.xf64;
            dxi = (const T *)t.dxi64; xci = (const T *)t.xci64;
        } else {
            dx = (const T *)t.dx32; xc = (const T *)t.xc32; xf = (const T *)t.xf32;
            dxi = (const T *)t.dxi32; xci = (const T *)t.xci32;
        }
    };
    std::memset(&a, 0, sizeof(a));
    a.u = u;
    a.vol = (long long)nx * ny * nz;
    for (int k = 0; k < 8; ++k) {
        a.vin[k] = in + (size_t)k * a.vol;
        a.var[k] = u + (size_t)k * a.vol;
    }
    a.N = N;
    a.M = M;
    a.L = L;
    a.nseg = nseg;
    a.Mext = N + 2 * kG;
    a.seg_fast = seg_fast_for(c, axis);
    a.P = P;
    a.S = P * M;
    int qax, rax;
    if (axis == 0) { a.stride_n = 1; a.stride_q = nx; a.stride_r = (long long)nx * ny; qax = 1; rax = 2; }
    else if (axis == 1) { a.stride_n = nx; a.stride_q = 1; a.stride_r = (long long)nx * ny; qax = 0; rax = 2; }
    else { a.stride_n = (long long)nx * ny; a.stride_q = 1; a.stride_r = nx; qax = 0; rax = 1; }
    a.nq = c->n[qax];
    a.nr = c->n[rax];
    a.tiles_q = (a.nq + P - 1) / P;
    a.inv_div = 1.0f / (float)(axis == 0 ? M : P);
    a.ntiles = a.tiles_q * a.nr;
    const T *dummy;
    tabs(axis, a.dx, a.xc, a.xf, dummy, dummy);
    const T *t0, *t1, *t2;
    tabs(qax, t0, t1, t2, a.dx_q, a.xc_q);
    tabs(rax, t0, t1, t2, a.dx_r, a.xc_r);
    a.bc_lo = c->bc_lo[axis];
    a.bc_hi = c->bc_hi[axis];
    a.gamma = (T)c->gamma;
    a.dt = (T)dt;
    a.dt_dev = dt_dev;
    a.has_bd = has_background(c) ? 1 : 0;
    a.dip_m = (T)c->dip_m;
    a.dir_x = (T)c->dir[0]; a.dir_y = (T)c->dir[1]; a.dir_z = (T)c->dir[2];
    a.bext_x = (T)c->bext[0]; a.bext_y = (T)c->bext[1]; a.bext_z = (T)c->bext[2];
    a.in_rho = (T)c->inflow[0];
    a.in_vx = (T)c->inflow[1]; a.in_vy = (T)c->inflow[2]; a.in_vz = (T)c->inflow[3];
    a.in_bx = (T)c->inflow[4]; a.in_by = (T)c->inflow[5]; a.in_bz = (T)c->inflow[6];
    a.in_p = (T)c->inflow[7];
    a.in_dev = c->series_n > 0 ? c->d_inflow : nullptr;
    a.has_inner = c->r_inner > 0.0 ? 1 : 0;
    a.r_inner2 = (T)(c->r_inner * c->r_inner);
    a.inner_rho = (T)c->inner_rho;
    a.inner_E = (T)(c->inner_p / (c->gamma - 1.0));
    if (c->inner_drift) {
        a.inner_v = c->d_inner_v;
        for (int q = 0; q < 6; ++q) a.ib[q] = c->inner_box[q];
    }
    a.flatten = c->opt.flatten;
    a.janhunen = c->opt.janhunen;
    a.max_iter = c->opt.max_iter;
    a.tol = (T)(f64 ? c->opt.tol_f64 : c->opt.tol_f32);
    a.p_floor = (T)c->opt.p_floor;
    a.stats = c->opt.collect_stats ? c->d_stats : nullptr;
    a.cfl_max = c->d_cflmax;
    if (f64) {
        a.dxw_x = (const T *)c->tab[0].dxi64; a.dxw_y = (const T *)c->tab[1].dxi64; a.dxw_z = (const T *)c->tab[2].dxi64;
    } else {
        a.dxw_x = (const T *)c->tab[0].dxi32; a.dxw_y = (const T *)c->tab[1].dxi32; a.dxw_z = (const T *)c->tab[2].dxi32;
    }
    // plain tile order along q then r (grouping q tiles that share cache
    // lines before stepping r was measured on the z sweep and raised its
    // fetched bytes)
    a.nslots = a.tiles_q * a.nr;
    a.tiles_per_xcd = (a.nslots * nseg + 7) / 8;
    a.mlp_frag = c->d_mlp_frag;
    a.mlp_theta = c->d_mlp_theta;
    a.gate_p = (T)c->gate_p;
    a.gate_u = (T)c->gate_u;
    a.harvest = c->harvest;
    a.harvest_cap = c->harvest_cap;
    a.harvest_count = c->harvest_count;
}

template <int AX, typename T, bool STATS, bool FUSE, int SM, int GUESS = 0, bool TRACE = false>
ppmlr_status launch_one(ppmlr_ctx *c, const ppmlr::SweepArgs<T> &a, hipStream_t st)
{
    const int threads = block_threads(a.P, a.M);
    const int slots = (GUESS == ppmlr::kGuessPlain ? kSlotsA : ppmlr::kSlotsAGuess) + kSlotsB;
    const size_t lds = ppmlr::lds_bytes(slots, SM > 0 ? SM : a.S, (int)sizeof(T));
    const int blocks = 8 * a.tiles_per_xcd;
    auto kern = ppmlr::sweep_kernel<AX, T, STATS, FUSE, SM, GUESS, TRACE>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_check(c, e, "hipFuncSetAttribute");
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, st, a);
    return hip_check(c, hipGetLastError(), "sweep launch");
}

template <int AX, typename T, bool STATS, bool FUSE, bool TRACE = false>
ppmlr_status launch_sm(ppmlr_ctx *c, const ppmlr::SweepArgs<T> &a, hipStream_t st)
{
    switch (stride_for(block_threads(a.P, a.M), (int)sizeof(T))) {
    case 256: return launch_one<AX, T, STATS, FUSE, 256, 0, TRACE>(c, a, st);
    case 384: return launch_one<AX, T, STATS, FUSE, 384, 0, TRACE>(c, a, st);
    case 512: return launch_one<AX, T, STATS, FUSE, 512, 0, TRACE>(c, a, st);
    case 640: return launch_one<AX, T, STATS, FUSE, 640, 0, TRACE>(c, a, st);
    case 768: return launch_one<AX, T, STATS, FUSE, 768, 0, TRACE>(c, a, st);
    case 896: return launch_one<AX, T, STATS, FUSE, 896, 0, TRACE>(c, a, st);
    case 1024:
        if constexpr (sizeof(T) == 4) return launch_one<AX, T, STATS, FUSE, 1024, 0, TRACE>(c, a, st);
        else return fail(c, PPMLR_EINVAL, "tile does not fit the LDS");
    case 0:
        if constexpr (sizeof(T) == 8) return launch_one<AX, T, STATS, FUSE, 0, 0, TRACE>(c, a, st);
        else return fail(c, PPMLR_EINVAL, "tile does not fit the LDS");
    default: return fail(c, PPMLR_EINVAL, "tile does not fit the LDS");
    }
}

// Learned / harvest sweeps: FP32, counters on, compile-time stride.
template <int AX, bool FUSE, int GUESS>
ppmlr_status launch_guess(ppmlr_ctx *c, const ppmlr::SweepArgs<float> &a, hipStream_t st)
{
    const int thr = block_threads(a.P, a.M);
    switch (thr <= 256 ? 256 : (thr <= 512 ? 512 : (thr <= 1024 ? 1024 : -1))) {
    case 256: return launch_one<AX, float, true, FUSE, 256, GUESS>(c, a, st);
    case 512: return launch_one<AX, float, true, FUSE, 512, GUESS>(c, a, st);
    case 1024: return launch_one<AX, float, true, FUSE, 1024, GUESS>(c, a, st);
    default: return fail(c, PPMLR_EINVAL, "tile does not fit the LDS");
    }
}

template <int AX, typename T>
ppmlr_status launch_axis(ppmlr_ctx *c, const ppmlr::SweepArgs<T> &a, hipStream_t st, bool stats, bool fuse)
{
    if (c->opt.tracing == PPMLR_TRACE_CHARACTERISTIC) {
        // counters always collected in the kernel (not stored without a buffer)
        if (c->guess != PPMLR_GUESS_PLAIN)
            return fail(c, PPMLR_EINVAL, "the characteristic mode takes the plain interface solve");
        return fuse ? launch_sm<AX, T, true, true, true>(c, a, st) : launch_sm<AX, T, true, false, true>(c, a, st);
    }
    if constexpr (sizeof(T) == 4) {
        if (c->guess == PPMLR_GUESS_LEARNED)
            return fuse ? launch_guess<AX, true, ppmlr::kGuessLearned>(c, a, st)
                        : launch_guess<AX, false, ppmlr::kGuessLearned>(c, a, st);
        if (c->guess == PPMLR_GUESS_HARVEST)
            return fuse ? launch_guess<AX, true, ppmlr::kGuessHarvest>(c, a, st)
                        : launch_guess<AX, false, ppmlr::kGuessHarvest>(c, a, st);
    }
    if (stats) return fuse ? launch_sm<AX, T, true, true>(c, a, st) : launch_sm<AX, T, true, false>(c, a, st);
    return fuse ? launch_sm<AX, T, false, true>(c, a, st) : launch_sm<AX, T, false, false>(c, a, st);
}

template <typename T>
ppmlr_status sweep_typed(ppmlr_ctx *c, const T *in, T *u, hipStream_t st, double dt, const double *dt_dev, int axis,
                         bool fuse)
{
    const int P = pick_tile(c, axis, (int)sizeof(T));
    const int M = tile_M(c, axis, (int)sizeof(T));
    if (block_threads(P, M) > 1024 || ppmlr::lds_bytes(kSlotsA + kSlotsB, P * M, (int)sizeof(T)) > 160 * 1024)
        return fail(c, PPMLR_EINVAL, "tile does not fit one workgroup");
    ppmlr::SweepArgs<T> a;
    fill_args(c, a, in, u, axis, dt, dt_dev, P, seg_count(c, axis, (int)sizeof(T)));
    const bool stats = c->opt.collect_stats != 0;
    if (axis == 0) return launch_axis<0, T>(c, a, st, stats, fuse);
    if (axis == 1) return launch_axis<1, T>(c, a, st, stats, fuse);
    return launch_axis<2, T>(c, a, st, stats, fuse);
}

ppmlr_status check_state(ppmlr_ctx *c, const ppmlr_state *s)
{
    if (!c) return PPMLR_EINVAL;
    if (!s || !s->u) return fail(c, PPMLR_EINVAL, "null state");
    if (s->dtype != PPMLR_F32 && s->dtype != PPMLR_F64) return fail(c, PPMLR_EINVAL, "bad dtype");
    // the sweeps address each variable with 32-bit byte offsets
    const unsigned long long vbytes = (unsigned long long)c->n[0] * c->n[1] * c->n[2] * (s->dtype == PPMLR_F64 ? 8 : 4);
    if (vbytes >= (1ull << 32)) return fail(c, PPMLR_EINVAL, "one variable of the state exceeds 4 GiB");
    return PPMLR_OK;
}

hipEvent_t pooled_event(ppmlr_ctx *c)
{
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Where the state of a sequence of sweeps is: the caller's buffer (home) or
// the context's second state.  Whole-pencil sweeps update in place (each
// workgroup reads and writes its own pencils only).  A segmented sweep reads
// its ghost zones from neighbouring segments that other workgroups update,
// so it writes the other buffer; a whole-pencil sweep that reads the second
// state writes home, so the pair of adjacent segmented sweeps of a split
// step pair ends at home.
struct Flow {
    void *home, *cur;
};

size_t state_bytes(const ppmlr_ctx *c, const ppmlr_state *s)
{
    return (size_t)8 * c->n[0] * c->n[1] * c->n[2] * (s->dtype == PPMLR_F64 ? 8 : 4);
}

ppmlr_status ensure_pong(ppmlr_ctx *c, size_t bytes)
{
    if (c->pong_bytes >= bytes) return PPMLR_OK;
    if (c->d_pong) {
        ppmlr_status e = hip_check(c, hipDeviceSynchronize(), "hipDeviceSynchronize");
        if (e) return e;
        (void)hipFree(c->d_pong);
        c->d_pong = nullptr;
        c->pong_bytes = 0;
    }
    ppmlr_status e = hip_check(c, hipMalloc(&c->d_pong, bytes), "hipMalloc");
    if (!e) c->pong_bytes = bytes;
    return e;
}

// Bring the state home after a sequence of sweeps.
ppmlr_status finish_flow(ppmlr_ctx *c, const ppmlr_state *s, Flow &f)
{
    if (f.cur == f.home) return PPMLR_OK;
    ppmlr_status e = hip_check(c, hipMemcpyAsync(f.home, f.cur, state_bytes(c, s), hipMemcpyDeviceToDevice,
                                                 (hipStream_t)s->stream), "hipMemcpyAsync");
    f.cur = f.home;
    return e;
}

ppmlr_status do_sweep(ppmlr_ctx *c, const ppmlr_state *s, double dt, const double *dt_dev, int axis, bool fuse,
                      Flow &f)
{
    hipStream_t st = (hipStream_t)s->stream;
    void *out = f.home;
    if (seg_count(c, axis, s->dtype == PPMLR_F64 ? 8 : 4) > 1) {
        ppmlr_status e = ensure_pong(c, state_bytes(c, s));
        if (e) return e;
        out = (f.cur == f.home) ? c->d_pong : f.home;
    }
    ppmlr_ctx::Mark mk{nullptr, nullptr, axis};
    if (c->profiling) {
        mk.start = pooled_event(c);
        mk.stop = pooled_event(c);
        if (!mk.start || !mk.stop) return fail(c, PPMLR_EDEVICE, "hipEventCreate failed");
        ppmlr_status e = hip_check(c, hipEventRecord(mk.start, st), "hipEventRecord");
        if (e) return e;
    }
    ppmlr_status r = (s->dtype == PPMLR_F64)
                         ? sweep_typed<double>(c, (const double *)f.cur, (double *)out, st, dt, dt_dev, axis, fuse)
                         : sweep_typed<float>(c, (const float *)f.cur, (float *)out, st, dt, dt_dev, axis, fuse);
    if (!r) f.cur = out;
    if (c->profiling) {
        ppmlr_status e = hip_check(c, hipEventRecord(mk.stop, st), "hipEventRecord");
        if (e) return e;
        c->marks.push_back(mk);
    }
    return r;
}

// ---------------------------------------------------------------- CFL

template <typename T>
struct CflArgs {
    const T *u;
    int nx, ny, nz;
    long long vol;
    const double *dx, *dy, *dz, *xc, *yc, *zc;
    double gamma, p_floor, r_inner2;
    int has_inner;
    double dip_m, dir[3], bext[3];
    unsigned long long *out;
};

__device__ inline void bg64(double dip_m, const double *dir, const double *bext, double x, double y, double z,
                            double &bx, double &by, double &bz)
{
    bx = bext[0];
    by = bext[1];
    bz = bext[2];
    if (dip_m != 0.0) {
        double r2 = x * x + y * y + z * z;
        double ir = 1.0 / __builtin_sqrt(r2);
        double ir3 = ir * ir * ir;
        double ir5 = ir3 * ir * ir;
        double mr = dir[0] * x + dir[1] * y + dir[2] * z;
        double cc = 3.0 * mr * ir5;
        bx += dip_m * (cc * x - dir[0] * ir3);
        by += dip_m * (cc * y - dir[1] * ir3);
        bz += dip_m * (cc * z - dir[2] * ir3);
    }
}

// Signal speed of zone z outside the inner boundary (0 inside): max_a
// (|v_a| + c_f,a) / dx_a in FP64.
template <typename T>
__device__ inline double cfl_zone(const CflArgs<T> &a, long long z)
{
    int i = (int)(z % a.nx);
    int j = (int)((z / a.nx) % a.ny);
    int k = (int)(z / ((long long)a.nx * a.ny));
    double x = a.xc[i], y = a.yc[j], zz = a.zc[k];
    if (a.has_inner && x * x + y * y + zz * zz < a.r_inner2) return 0.0;
    double r = (double)a.u[z];
    double vx = (double)a.u[a.vol + z] / r, vy = (double)a.u[2 * a.vol + z] / r, vz = (double)a.u[3 * a.vol + z] / r;
    double px = (double)a.u[4 * a.vol + z], py = (double)a.u[5 * a.vol + z], pz = (double)a.u[6 * a.vol + z];
    double p = (a.gamma - 1.0) * ((double)a.u[7 * a.vol + z] - 0.5 * r * (vx * vx + vy * vy + vz * vz) -
                                  0.5 * (px * px + py * py + pz * pz));
    if (p < a.p_floor) p = a.p_floor;
    double bx, by, bz;
    bg64(a.dip_m, a.dir, a.bext, x, y, zz, bx, by, bz);
    bx += px; by += py; bz += pz;
    double a2 = a.gamma * p / r;
    double b2 = (bx * bx + by * by + bz * bz) / r;
    double w[3] = {a.dx[i], a.dy[j], a.dz[k]};
    double v[3] = {vx, vy, vz};
    double B[3] = {bx, by, bz};
    double smax = 0.0;
    for (int c = 0; c < 3; ++c) {
        double ba2 = B[c] * B[c] / r;
        double disc = (a2 + b2) * (a2 + b2) - 4.0 * a2 * ba2;
        disc = disc > 0.0 ? disc : 0.0;
        double cf = __builtin_sqrt(0.5 * (a2 + b2 + __builtin_sqrt(disc)));
        double s = (__builtin_fabs(v[c]) + cf) / w[c];
        smax = s > smax ? s : smax;
    }
    return smax;
}

// Signal-speed maximum over all zones outside the inner boundary: per zone
// cfl_zone; wave shuffles, then one atomic per workgroup on the bits of the
// (non-negative) double.
template <typename T>
__global__ void __launch_bounds__(256) cfl_kernel(const CflArgs<T> a)
{
    __shared__ double red[4];
    double smax = 0.0;
    for (long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x; z < a.vol;
         z += (long long)gridDim.x * blockDim.x) {
        const double s = cfl_zone(a, z);
        smax = s > smax ? s : smax;
    }
    for (int off = 32; off > 0; off >>= 1) {
        double o = __shfl_xor(smax, off);
        smax = o > smax ? o : smax;
    }
    if (__lane_id() == 0) red[threadIdx.x >> 6] = smax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < 4; ++w) m = red[w] > m ? red[w] : m;
        atomicMax(a.out + (blockIdx.x % ppmlr::kCflSlots) * ppmlr::kCflStride,
                  (unsigned long long)__double_as_longlong(m));
    }
}

// Maximum of the signal-speed slots (one wave; the bits of non-negative
// doubles order as unsigned integers, as for the atomics that filled them).
__device__ inline unsigned long long slot_max(const unsigned long long *slots)
{
    unsigned long long v = slots[threadIdx.x * ppmlr::kCflStride];
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// Fold the slots into slot 0 (one wave of kCflSlots threads).
__global__ void fold_slots(unsigned long long *slots)
{
    const unsigned long long v = slot_max(slots);
    slots[threadIdx.x * ppmlr::kCflStride] = threadIdx.x == 0 ? v : 0ull;
}

__global__ void clear_slots(unsigned long long *slots)
{
    slots[threadIdx.x * ppmlr::kCflStride] = 0ull;
}

// dt for the next step from the fused signal-speed maximum; accumulates the
// simulated time and clears the maximum for the next reduction.
// Inflow state of a time series at time t: linear between the knots
// (rows t_k, prim_k[8], t increasing), held at the first / last knot outside.
__device__ inline void series_at(const double *series, int n, double t, double *out)
{
    int k;
    double w;
    if (t <= series[0]) { k = 0; w = 0.0; }
    else if (t >= series[(size_t)(n - 1) * 9]) { k = n - 1; w = 0.0; }
    else {
        int lo = 0, hi = n - 1;                  // series[lo].t <= t < series[hi].t
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (series[(size_t)mid * 9] <= t) lo = mid; else hi = mid;
        }
        k = lo;
        const double t0 = series[(size_t)lo * 9], t1 = series[(size_t)hi * 9];
        w = (t - t0) / (t1 - t0);
    }
    const double *a = series + (size_t)k * 9 + 1;
    for (int q = 0; q < 8; ++q)
        out[q] = w == 0.0 ? a[q] : a[q] + w * (a[9 + q] - a[q]);
}

// (one wave of kCflSlots threads)  A step of length d starting at t takes
// the inflow of the time series (if any) at its mid-time t + d/2.
__global__ void dt_kernel(unsigned long long *smax_bits, double *dt, double *t, double cfl, const double *series,
                          int series_n, double *inflow)
{
    const unsigned long long bits = slot_max(smax_bits);
    smax_bits[threadIdx.x * ppmlr::kCflStride] = 0ull;
    if (threadIdx.x != 0) return;
    double smax = __longlong_as_double((long long)bits);
    double d = smax > 0.0 ? cfl / smax : 0.0;
    *dt = d;
    if (series_n > 0) series_at(series, series_n, *t + 0.5 * d, inflow);
    *t += d;
}

// Host-given dt: the time series' inflow at t + dt/2; advance: t += dt.
__global__ void step_time_kernel(double *t, double dt, int advance, const double *series, int series_n,
                                 double *inflow)
{
    if (series_n > 0) series_at(series, series_n, *t + 0.5 * dt, inflow);
    if (advance) *t += dt;
}

__global__ void clear_u64(unsigned long long *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}
__global__ void clear_f64(double *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

// ---------------------------------------------------------------- totals

// Volume integrals in a fixed order: block b sums the contiguous chunk b of
// the zones (each thread a fixed strided subset, then a fixed tree), then a
// single block sums the partials in index order.
template <typename T>
__global__ void __launch_bounds__(256) totals_partial(const T *u, long long vol, int nx, int ny, const double *dx,
                                                      const double *dy, const double *dz, double *partials)
{
    __shared__ double red[8][256];
    const long long chunk = (vol + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < vol ? lo + chunk : vol;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (long long z = lo + threadIdx.x; z < hi; z += blockDim.x) {
        int i = (int)(z % nx);
        int j = (int)((z / nx) % ny);
        int k = (int)(z / ((long long)nx * ny));
        double dv = dx[i] * dy[j] * dz[k];
        for (int v = 0; v < 8; ++v) acc[v] += (double)u[v * vol + z] * dv;
    }
    for (int v = 0; v < 8; ++v) red[v][threadIdx.x] = acc[v];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int v = 0; v < 8; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 8) partials[blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void totals_final(const double *partials, int nblocks, double *out)
{
    if (threadIdx.x < 8) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partials[b * 8 + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

template <typename T>
CflArgs<T> cfl_args(const ppmlr_ctx *c, const T *u)
{
    CflArgs<T> a;
    a.u = u;
    a.nx = c->n[0]; a.ny = c->n[1]; a.nz = c->n[2];
    a.vol = (long long)a.nx * a.ny * a.nz;
    a.dx = c->tab[0].dxi64; a.dy = c->tab[1].dxi64; a.dz = c->tab[2].dxi64;
    a.xc = c->tab[0].xci64; a.yc = c->tab[1].xci64; a.zc = c->tab[2].xci64;
    a.gamma = c->gamma;
    a.p_floor = c->opt.p_floor;
    a.r_inner2 = c->r_inner * c->r_inner;
    a.has_inner = c->r_inner > 0.0;
    a.dip_m = c->dip_m;
    for (int k = 0; k < 3; ++k) { a.dir[k] = c->dir[k]; a.bext[k] = c->bext[k]; }
    a.out = c->d_cflmax;
    return a;
}

template <typename T>
ppmlr_status cfl_typed(ppmlr_ctx *c, const T *u, hipStream_t st)
{
    const CflArgs<T> a = cfl_args(c, u);
    long long blocks = (a.vol + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(cfl_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hip_check(c, hipGetLastError(), "cfl launch");
}

ppmlr_status cfl_launch(ppmlr_ctx *c, const ppmlr_state *s)
{
    hipStream_t st = (hipStream_t)s->stream;
    hipLaunchKernelGGL(clear_slots, dim3(1), dim3(ppmlr::kCflSlots), 0, st, c->d_cflmax);
    if (s->dtype == PPMLR_F64) return cfl_typed<double>(c, (const double *)s->u, st);
    return cfl_typed<float>(c, (const float *)s->u, st);
}

}  // namespace

// ================================================================ C ABI

extern "C" {

void ppmlr_default_options(ppmlr_options *o)
{
    if (!o) return;
    o->flatten = 1;
    o->janhunen = 1;
    o->max_iter = 20;
    o->tol_f64 = 1e-12;
    o->tol_f32 = 1e-6;
    o->p_floor = 1e-8;
    o->collect_stats = 1;
    o->debug_cfl = 0;
    o->tracing = PPMLR_TRACE_TWO_FAMILY;
}

ppmlr_status ppmlr_create(const ppmlr_grid *grid, double gamma, const ppmlr_coords *coords,
                          const ppmlr_options *opt, ppmlr_ctx **out)
{
    if (!out) return PPMLR_EINVAL;
    *out = nullptr;
    if (!grid || !coords || !(gamma > 1.0)) return PPMLR_EINVAL;
    for (int a = 0; a < 3; ++a) {
        if (grid->n[a] < 1 || !coords->faces[a]) return PPMLR_EINVAL;
        int lo = grid->bc_lo[a], hi = grid->bc_hi[a];
        if (lo < 0 || lo > 2 || hi < 0 || hi > 2) return PPMLR_EINVAL;
        if ((lo == PPMLR_PERIODIC) != (hi == PPMLR_PERIODIC)) return PPMLR_EINVAL;
        if (lo != PPMLR_PERIODIC && grid->n[a] < kG) return PPMLR_EINVAL;
        if (grid->n[a] > (1 << 24)) return PPMLR_EINVAL;     // 32-bit zone indexing with margin
        for (int i = 0; i < grid->n[a]; ++i)
            if (!(coords->faces[a][i + 1] > coords->faces[a][i]) || !std::isfinite(coords->faces[a][i + 1]))
                return PPMLR_EINVAL;
    }
    ppmlr_ctx *c = new ppmlr_ctx();
    for (int a = 0; a < 3; ++a) {
        c->n[a] = grid->n[a];
        c->bc_lo[a] = grid->bc_lo[a];
        c->bc_hi[a] = grid->bc_hi[a];
        c->faces[a].assign(coords->faces[a], coords->faces[a] + grid->n[a] + 1);
    }
    c->r_inner = grid->r_inner;
    c->gamma = gamma;
    if (opt) c->opt = *opt;
    else ppmlr_default_options(&c->opt);
    if (c->opt.max_iter < 0 || !(c->opt.tol_f64 > 0) || !(c->opt.tol_f32 > 0) ||
        (c->opt.tracing != PPMLR_TRACE_TWO_FAMILY && c->opt.tracing != PPMLR_TRACE_CHARACTERISTIC)) {
        delete c;
        return PPMLR_EINVAL;
    }
    ppmlr_status s = hip_check(c, hipGetDevice(&c->device), "hipGetDevice");
    for (int a = 0; a < 3 && !s; ++a) {
        extend_axis(c, a);
        AxisTables &t = c->tab[a];
        std::vector<double> dxi(c->n[a]), xci(c->n[a]);
        for (int i = 0; i < c->n[a]; ++i) {
            dxi[i] = c->faces[a][i + 1] - c->faces[a][i];
            xci[i] = 0.5 * (c->faces[a][i] + c->faces[a][i + 1]);
        }
        if (!s) s = upload(c, &t.dx64, c->ext_dx[a]);
        if (!s) s = upload(c, &t.xc64, c->ext_xc[a]);
        if (!s) s = upload(c, &t.xf64, c->ext_xf[a]);
        if (!s) s = upload(c, &t.dxi64, dxi);
        if (!s) s = upload(c, &t.xci64, xci);
        if (!s) s = upload(c, &t.dx32, c->ext_dx[a]);
        if (!s) s = upload(c, &t.xc32, c->ext_xc[a]);
        if (!s) s = upload(c, &t.xf32, c->ext_xf[a]);
        if (!s) s = upload(c, &t.dxi32, dxi);
        if (!s) s = upload(c, &t.xci32, xci);
    }
    c->partial_blocks = kTotBlocks;
    if (!s) s = hip_check(c, hipMalloc((void **)&c->d_stats, sizeof(unsigned long long) * kStatWords * kStatSlots),
                          "hipMalloc");
    if (!s)
        s = hip_check(c, hipMalloc((void **)&c->d_cflmax, sizeof(unsigned long long) * ppmlr::kCflSlots * ppmlr::kCflStride),
                      "hipMalloc");
    if (!s) s = hip_check(c, hipMalloc((void **)&c->d_dt, sizeof(double)), "hipMalloc");
    if (!s) s = hip_check(c, hipMalloc((void **)&c->d_time, sizeof(double)), "hipMalloc");
    if (!s) s = hip_check(c, hipMalloc((void **)&c->d_partials, sizeof(double) * (8 * kTotBlocks + 8)), "hipMalloc");
    if (!s) {
        hipLaunchKernelGGL(clear_u64, dim3(1), dim3(256), 0, (hipStream_t)0, c->d_stats, kStatWords * kStatSlots);
        hipLaunchKernelGGL(clear_slots, dim3(1), dim3(ppmlr::kCflSlots), 0, (hipStream_t)0, c->d_cflmax);
        hipLaunchKernelGGL(clear_f64, dim3(1), dim3(64), 0, (hipStream_t)0, c->d_dt, 1);
        hipLaunchKernelGGL(clear_f64, dim3(1), dim3(64), 0, (hipStream_t)0, c->d_time, 1);
        s = hip_check(c, hipDeviceSynchronize(), "init");
    }
    if (s) {
        free_tables(c);
        delete c;
        return s;
    }
    *out = c;
    return PPMLR_OK;
}

void ppmlr_destroy(ppmlr_ctx *c)
{
    if (!c) return;
    (void)hipDeviceSynchronize();
    for (auto &m : c->marks) {
        (void)hipEventDestroy(m.start);
        (void)hipEventDestroy(m.stop);
    }
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    if (c->d_mlp_frag) (void)hipFree(c->d_mlp_frag);
    if (c->d_pong) (void)hipFree(c->d_pong);
    if (c->d_mlp_theta) (void)hipFree(c->d_mlp_theta);
    if (c->d_series) (void)hipFree(c->d_series);
    if (c->d_inflow) (void)hipFree(c->d_inflow);
    if (c->d_iono) (void)hipFree(c->d_iono);
    if (c->d_inner_v) (void)hipFree(c->d_inner_v);
    free_tables(c);
    delete c;
}

ppmlr_status ppmlr_set_profiling(ppmlr_ctx *c, int enable)
{
    if (!c) return PPMLR_EINVAL;
    c->profiling = enable != 0;
    return PPMLR_OK;
}

ppmlr_status ppmlr_kernel_times(ppmlr_ctx *c, double ms[3], long long launches[3])
{
    if (!c || !ms || !launches) return PPMLR_EINVAL;
    for (int a = 0; a < 3; ++a) { ms[a] = 0.0; launches[a] = 0; }
    ppmlr_status e = PPMLR_OK;
    for (auto &m : c->marks) {
        if (!e) e = hip_check(c, hipEventSynchronize(m.stop), "hipEventSynchronize");
        float t = 0.0f;
        if (!e) e = hip_check(c, hipEventElapsedTime(&t, m.start, m.stop), "hipEventElapsedTime");
        if (!e) { ms[m.axis] += (double)t; launches[m.axis] += 1; }
        c->event_pool.push_back(m.start);
        c->event_pool.push_back(m.stop);
    }
    c->marks.clear();
    return e;
}

const char *ppmlr_last_error(const ppmlr_ctx *c)
{
    return c ? c->err.c_str() : "null context";
}

ppmlr_status ppmlr_set_dipole(ppmlr_ctx *c, double moment, const double dir[3])
{
    if (!c) return PPMLR_EINVAL;
    if (!std::isfinite(moment)) return fail(c, PPMLR_EINVAL, "bad moment");
    if (moment != 0.0) {
        if (!dir) return fail(c, PPMLR_EINVAL, "null direction");
        double n2 = dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2];
        if (!(n2 > 0.0) || !std::isfinite(n2)) return fail(c, PPMLR_EINVAL, "bad direction");
        for (int k = 0; k < 3; ++k) c->dir[k] = dir[k] / std::sqrt(n2);
    }
    c->dip_m = moment;
    return PPMLR_OK;
}

ppmlr_status ppmlr_set_background(ppmlr_ctx *c, const double b[3])
{
    if (!c || !b) return PPMLR_EINVAL;
    for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(b[k])) return fail(c, PPMLR_EINVAL, "bad field");
        c->bext[k] = b[k];
    }
    return PPMLR_OK;
}

ppmlr_status ppmlr_set_inflow(ppmlr_ctx *c, const double prim[8])
{
    if (!c || !prim) return PPMLR_EINVAL;
    for (int k = 0; k < 8; ++k)
        if (!std::isfinite(prim[k])) return fail(c, PPMLR_EINVAL, "non-finite inflow");
    if (!(prim[0] > 0.0) || !(prim[7] > 0.0)) return fail(c, PPMLR_EINVAL, "inflow needs rho > 0, p > 0");
    std::memcpy(c->inflow, prim, sizeof(double) * 8);
    return PPMLR_OK;
}

ppmlr_status ppmlr_set_inner(ppmlr_ctx *c, double rho, double p)
{
    if (!c) return PPMLR_EINVAL;
    if (!(rho > 0.0) || !(p > 0.0) || !std::isfinite(rho) || !std::isfinite(p))
        return fail(c, PPMLR_EINVAL, "inner state needs rho > 0, p > 0");
    c->inner_rho = rho;
    c->inner_p = p;
    return PPMLR_OK;
}

void ppmlr_iono_default_params(ppmlr_iono_params *p)
{
    if (!p) return;
    p->n_theta = 32;
    p->n_phi = 64;
    p->r_shell = 1.017;
    p->r_fac = 3.5;
    p->sigma = 5.0 * 4.0e-7 * M_PI * 21.81e3;   // 5 S in code units (mu_0 v_0 per siemens)
}

ppmlr_status ppmlr_ionosphere_detach(ppmlr_ctx *c)
{
    if (!c) return PPMLR_EINVAL;
    c->inner_drift = false;
    return PPMLR_OK;
}

ppmlr_status ppmlr_ionosphere_couple(ppmlr_ctx *c, const ppmlr_state *s, const ppmlr_iono_params *prm, double *jr,
                                     double *phi)
{
    ppmlr_status e = check_state(c, s);
    if (e) return e;
    if (!prm) return fail(c, PPMLR_EINVAL, "null parameters");
    if (c->dip_m == 0.0) return fail(c, PPMLR_EINVAL, "the ionosphere coupling needs a dipole");
    if (!(c->r_inner > 0.0)) return fail(c, PPMLR_EINVAL, "the ionosphere coupling needs an inner boundary");
    const int nt = prm->n_theta, nph = prm->n_phi;
    if (nt < 2 || nph < 4 || (long long)nt * nph > ppmlr::kIonoMaxCells)
        return fail(c, PPMLR_EINVAL, "shell cells: n_theta >= 2, n_phi >= 4, n_theta * n_phi <= 4096");
    const long long N = (long long)nt * nph;
    const size_t lds = sizeof(double) * (size_t)(4 * N + 3 * nt + 2 * nph);
    if (lds > 160 * 1024) return fail(c, PPMLR_EINVAL, "shell arrays do not fit the LDS");
    if (!(prm->r_fac > prm->r_shell) || !(prm->r_shell > 0.0) || !(prm->sigma > 0.0) ||
        !std::isfinite(prm->r_fac) || !std::isfinite(prm->sigma))
        return fail(c, PPMLR_EINVAL, "shell parameters: r_fac > r_shell > 0, sigma > 0");
    // the sphere r_fac with the central differences' neighbours inside the grid
    for (int a = 0; a < 3; ++a) {
        const std::vector<double> &f = c->faces[a];
        const int n = c->n[a];
        if (n < 4) return fail(c, PPMLR_EINVAL, "the ionosphere coupling needs 4 or more zones per axis");
        const double c1 = 0.5 * (f[1] + f[2]), cn2 = 0.5 * (f[n - 2] + f[n - 1]);
        if (!(c1 < -prm->r_fac) || !(prm->r_fac < cn2))
            return fail(c, PPMLR_EINVAL, "the sphere r_fac does not fit inside the zone centres");
    }
    hipStream_t st = (hipStream_t)s->stream;
    // magnetic frame: z_m opposite to the dipole moment
    double m[3] = {c->dir[0], c->dir[1], c->dir[2]};
    const double mn = std::sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    ppmlr::IonoArgs a;
    std::memset(&a, 0, sizeof(a));
    for (int d = 0; d < 3; ++d) {
        a.mdir[d] = m[d] / mn;
        a.zm[d] = -a.mdir[d];
    }
    {
        double x[3] = {1.0, 0.0, 0.0};
        double dz = a.zm[0];
        double xm[3] = {x[0] - dz * a.zm[0], x[1] - dz * a.zm[1], x[2] - dz * a.zm[2]};
        double nx_ = std::sqrt(xm[0] * xm[0] + xm[1] * xm[1] + xm[2] * xm[2]);
        if (nx_ < 1e-6) {
            double y[3] = {0.0, 1.0, 0.0};
            dz = a.zm[1];
            for (int d = 0; d < 3; ++d) xm[d] = y[d] - dz * a.zm[d];
            nx_ = std::sqrt(xm[0] * xm[0] + xm[1] * xm[1] + xm[2] * xm[2]);
        }
        for (int d = 0; d < 3; ++d) a.xm[d] = xm[d] / nx_;
        a.ym[0] = a.zm[1] * a.xm[2] - a.zm[2] * a.xm[1];
        a.ym[1] = a.zm[2] * a.xm[0] - a.zm[0] * a.xm[2];
        a.ym[2] = a.zm[0] * a.xm[1] - a.zm[1] * a.xm[0];
    }
    a.u = s->u;
    a.nx = c->n[0]; a.ny = c->n[1]; a.nz = c->n[2];
    a.vol = (long long)a.nx * a.ny * a.nz;
    a.xc = c->tab[0].xci64; a.yc = c->tab[1].xci64; a.zc = c->tab[2].xci64;
    a.M = c->dip_m;
    a.nt = nt; a.nph = nph;
    a.r_shell = prm->r_shell; a.r_fac = prm->r_fac;
    a.theta_c = std::asin(std::sqrt(prm->r_shell / prm->r_fac));
    a.dth = a.theta_c / nt;
    a.dph = 2.0 * M_PI / nph;
    a.sigma = prm->sigma;
    a.r_inner2 = c->r_inner * c->r_inner;
    // index box of the zones inside r_inner
    bool have_box = true;
    for (int d = 0; d < 3; ++d) {
        const std::vector<double> &f = c->faces[d];
        int lo = -1, hi = -1;
        for (int i = 0; i < c->n[d]; ++i) {
            const double x = 0.5 * (f[i] + f[i + 1]);
            if (x * x < a.r_inner2) { if (lo < 0) lo = i; hi = i + 1; }
        }
        if (lo < 0) { have_box = false; break; }
        a.box[2 * d] = lo;
        a.box[2 * d + 1] = hi;
    }
    const long long nb = have_box ? (long long)(a.box[1] - a.box[0]) * (a.box[3] - a.box[2]) * (a.box[5] - a.box[4]) : 0;
    // work buffers
    const size_t need = sizeof(double) * (size_t)(4 * N + 2);
    if (c->iono_bytes < need) {
        if (c->d_iono) { (void)hipStreamSynchronize(st); (void)hipFree(c->d_iono); c->d_iono = nullptr; c->iono_bytes = 0; }
        e = hip_check(c, hipMalloc((void **)&c->d_iono, need), "hipMalloc");
        if (e) return e;
        c->iono_bytes = need;
    }
    const size_t vneed = sizeof(double) * (size_t)std::max<long long>(3 * nb, 1);
    if (c->inner_v_bytes < vneed) {
        c->inner_drift = false;
        if (c->d_inner_v) { (void)hipStreamSynchronize(st); (void)hipFree(c->d_inner_v); c->d_inner_v = nullptr; c->inner_v_bytes = 0; }
        e = hip_check(c, hipMalloc((void **)&c->d_inner_v, vneed), "hipMalloc");
        if (e) return e;
        c->inner_v_bytes = vneed;
    }
    a.jr = c->d_iono;
    a.phi = c->d_iono + 2 * N;
    a.pole = c->d_iono + 4 * N;
    a.v = c->d_inner_v;
    const unsigned fac_blocks = (unsigned)((2 * N + 255) / 256);
    if (s->dtype == PPMLR_F64)
        hipLaunchKernelGGL(ppmlr::iono_fac_kernel<double>, dim3(fac_blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(ppmlr::iono_fac_kernel<float>, dim3(fac_blocks), dim3(256), 0, st, a);
    e = hip_check(c, hipGetLastError(), "ionosphere current launch");
    if (e) return e;
    if (lds > 64 * 1024) {
        e = hip_check(c, hipFuncSetAttribute((const void *)ppmlr::iono_solve_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                      "hipFuncSetAttribute");
        if (e) return e;
    }
    hipLaunchKernelGGL(ppmlr::iono_solve_kernel, dim3(2), dim3(ppmlr::kIonoThreads), lds, st, a);
    e = hip_check(c, hipGetLastError(), "ionosphere potential launch");
    if (e) return e;
    if (nb > 0) {
        hipLaunchKernelGGL(ppmlr::iono_drift_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, a);
        e = hip_check(c, hipGetLastError(), "ionosphere drift launch");
        if (e) return e;
    }
    if (jr) e = hip_check(c, hipMemcpyAsync(jr, a.jr, sizeof(double) * 2 * N, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
    if (!e && phi)
        e = hip_check(c, hipMemcpyAsync(phi, a.phi, sizeof(double) * 2 * N, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
    if (!e) e = hip_check(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    if (e) return e;
    for (int q = 0; q < 6; ++q) c->inner_box[q] = a.box[q];
    c->inner_drift = nb > 0;
    return PPMLR_OK;
}

ppmlr_status ppmlr_set_inflow_series(ppmlr_ctx *c, int n, const double *t, const double *prim)
{
    if (!c || n < 0 || n > (1 << 20)) return PPMLR_EINVAL;
    if (n == 0) {
        c->series_n = 0;
        return PPMLR_OK;
    }
    if (!t || !prim) return fail(c, PPMLR_EINVAL, "null series");
    std::vector<double> rows((size_t)n * 9);
    for (int k = 0; k < n; ++k) {
        if (!std::isfinite(t[k]) || (k > 0 && !(t[k] > t[k - 1])))
            return fail(c, PPMLR_EINVAL, "series times must be finite and increasing");
        for (int q = 0; q < 8; ++q)
            if (!std::isfinite(prim[(size_t)k * 8 + q])) return fail(c, PPMLR_EINVAL, "series values must be finite");
        if (!(prim[(size_t)k * 8] > 0.0) || !(prim[(size_t)k * 8 + 7] > 0.0))
            return fail(c, PPMLR_EINVAL, "series density and pressure must be positive");
        rows[(size_t)k * 9] = t[k];
        for (int q = 0; q < 8; ++q) rows[(size_t)k * 9 + 1 + q] = prim[(size_t)k * 8 + q];
    }
    // the buffers may be in use by queued work: wait before replacing them
    ppmlr_status e = hip_check(c, hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (!e && n > c->series_cap) {
        if (c->d_series) (void)hipFree(c->d_series);
        c->d_series = nullptr;
        c->series_cap = 0;
        e = hip_check(c, hipMalloc((void **)&c->d_series, rows.size() * sizeof(double)), "hipMalloc");
        if (!e) c->series_cap = n;
    }
    if (!e && !c->d_inflow) e = hip_check(c, hipMalloc((void **)&c->d_inflow, 8 * sizeof(double)), "hipMalloc");
    if (!e) e = hip_check(c, hipMemcpy(c->d_series, rows.data(), rows.size() * sizeof(double), hipMemcpyHostToDevice),
                          "hipMemcpy");
    if (e) {
        c->series_n = 0;
        return e;
    }
    c->series_n = n;
    // the inflow at the current time until the next step sets it
    hipLaunchKernelGGL(step_time_kernel, dim3(1), dim3(1), 0, (hipStream_t)0, c->d_time, 0.0, 0, c->d_series,
                       c->series_n, c->d_inflow);
    return hip_check(c, hipDeviceSynchronize(), "hipDeviceSynchronize");
}

ppmlr_status ppmlr_sweep(ppmlr_ctx *c, const ppmlr_state *s, double dt, int axis)
{
    ppmlr_status e = check_state(c, s);
    if (e) return e;
    if (axis < 0 || axis > 2) return fail(c, PPMLR_EINVAL, "axis must be 0, 1 or 2");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, PPMLR_EINVAL, "dt must be positive and finite");
    if (c->series_n > 0)
        hipLaunchKernelGGL(step_time_kernel, dim3(1), dim3(1), 0, (hipStream_t)s->stream, c->d_time, dt, 0,
                           c->d_series, c->series_n, c->d_inflow);
    Flow f{s->u, s->u};
    e = do_sweep(c, s, dt, nullptr, axis, false, f);
    if (e) return e;
    return finish_flow(c, s, f);
}

ppmlr_status ppmlr_step(ppmlr_ctx *c, const ppmlr_state *s, double dt)
{
    ppmlr_status e = check_state(c, s);
    if (e) return e;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, PPMLR_EINVAL, "dt must be positive and finite");
    if (c->opt.debug_cfl) {
        double lim = 0.0;
        e = ppmlr_cfl_dt(c, s, 1.0, &lim);
        if (e) return e;
        if (dt > 1.0001 * lim) return fail(c, PPMLR_ECFL, "dt above the CFL limit");
    }
    static const int even[3] = {0, 1, 2}, odd[3] = {2, 1, 0};
    const int *ord = (c->step % 2 == 0) ? even : odd;
    hipLaunchKernelGGL(step_time_kernel, dim3(1), dim3(1), 0, (hipStream_t)s->stream, c->d_time, dt, 1, c->d_series,
                       c->series_n, c->d_inflow);
    Flow f{s->u, s->u};
    for (int k = 0; k < 3; ++k) {
        e = do_sweep(c, s, dt, nullptr, ord[k], false, f);
        if (e) return e;
    }
    c->step++;
    return finish_flow(c, s, f);
}

ppmlr_status ppmlr_set_step_index(ppmlr_ctx *c, long long step)
{
    if (!c || step < 0) return PPMLR_EINVAL;
    c->step = step;
    return PPMLR_OK;
}

ppmlr_status ppmlr_get_step_index(const ppmlr_ctx *c, long long *step)
{
    if (!c || !step) return PPMLR_EINVAL;
    *step = c->step;
    return PPMLR_OK;
}

ppmlr_status ppmlr_cfl_dt(ppmlr_ctx *c, const ppmlr_state *s, double cfl, double *dt_out)
{
    ppmlr_status e = check_state(c, s);
    if (e) return e;
    if (!dt_out || !(cfl > 0.0)) return fail(c, PPMLR_EINVAL, "cfl must be positive");
    e = cfl_launch(c, s);
    if (e) return e;
    unsigned long long bits = 0;
    hipStream_t st = (hipStream_t)s->stream;
    hipLaunchKernelGGL(fold_slots, dim3(1), dim3(ppmlr::kCflSlots), 0, st, c->d_cflmax);
    e = hip_check(c, hipMemcpyAsync(&bits, c->d_cflmax, sizeof(bits), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    if (!e) e = hip_check(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    if (e) return e;
    double smax;
    std::memcpy(&smax, &bits, sizeof(smax));
    if (!(smax > 0.0) || !std::isfinite(smax)) return fail(c, PPMLR_ENONPHYS, "no finite signal speed");
    *dt_out = cfl / smax;
    return PPMLR_OK;
}

ppmlr_status ppmlr_advance(ppmlr_ctx *c, const ppmlr_state *s, int nsteps, double cfl)
{
    ppmlr_status e = check_state(c, s);
    if (e) return e;
    if (nsteps < 0 || !(cfl > 0.0)) return fail(c, PPMLR_EINVAL, "nsteps >= 0 and cfl > 0 required");
    if (nsteps == 0) return PPMLR_OK;
    hipStream_t st = (hipStream_t)s->stream;
    e = cfl_launch(c, s);   // signal-speed maximum of the current state
    if (e) return e;
    static const int even[3] = {0, 1, 2}, odd[3] = {2, 1, 0};
    Flow f{s->u, s->u};
    for (int n = 0; n < nsteps; ++n) {
        hipLaunchKernelGGL(dt_kernel, dim3(1), dim3(ppmlr::kCflSlots), 0, st, c->d_cflmax, c->d_dt, c->d_time, cfl,
                           c->d_series, c->series_n, c->d_inflow);
        const int *ord = (c->step % 2 == 0) ? even : odd;
        for (int k = 0; k < 3; ++k) {
            e = do_sweep(c, s, 0.0, c->d_dt, ord[k], k == 2, f);
            if (e) return e;
        }
        c->step++;
    }
    e = finish_flow(c, s, f);
    if (e) return e;
    return hip_check(c, hipGetLastError(), "advance");
}

ppmlr_status ppmlr_time(ppmlr_ctx *c, const ppmlr_state *s, double *t_out)
{
    if (!c || !t_out) return PPMLR_EINVAL;
    hipStream_t st = s ? (hipStream_t)s->stream : (hipStream_t)0;
    ppmlr_status e = hip_check(c, hipMemcpyAsync(t_out, c->d_time, sizeof(double), hipMemcpyDeviceToHost, st),
                               "hipMemcpyAsync");
    if (!e) e = hip_check(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    return e;
}

ppmlr_status ppmlr_totals(ppmlr_ctx *c, const ppmlr_state *s, double out[8])
{
    ppmlr_status e = check_state(c, s);
    if (e) return e;
    if (!out) return fail(c, PPMLR_EINVAL, "null output");
    hipStream_t st = (hipStream_t)s->stream;
    const long long vol = (long long)c->n[0] * c->n[1] * c->n[2];
    if (s->dtype == PPMLR_F64)
        hipLaunchKernelGGL(totals_partial<double>, dim3(kTotBlocks), dim3(256), 0, st, (const double *)s->u, vol,
                           c->n[0], c->n[1], c->tab[0].dxi64, c->tab[1].dxi64, c->tab[2].dxi64, c->d_partials);
    else
        hipLaunchKernelGGL(totals_partial<float>, dim3(kTotBlocks), dim3(256), 0, st, (const float *)s->u, vol,
                           c->n[0], c->n[1], c->tab[0].dxi64, c->tab[1].dxi64, c->tab[2].dxi64, c->d_partials);
    hipLaunchKernelGGL(totals_final, dim3(1), dim3(64), 0, st, c->d_partials, kTotBlocks, c->d_partials + 8 * kTotBlocks);
    e = hip_check(c, hipGetLastError(), "totals launch");
    if (!e) e = hip_check(c, hipMemcpyAsync(out, c->d_partials + 8 * kTotBlocks, sizeof(double) * 8,
                                            hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    if (!e) e = hip_check(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    return e;
}

ppmlr_status ppmlr_stats(ppmlr_ctx *c, void *stream, ppmlr_stats_t *out)
{
    if (!c || !out) return PPMLR_EINVAL;
    std::vector<unsigned long long> raw((size_t)kStatWords * kStatSlots);
    hipStream_t st = (hipStream_t)stream;
    ppmlr_status e = hip_check(c, hipMemcpyAsync(raw.data(), c->d_stats, sizeof(unsigned long long) * raw.size(),
                                                 hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    if (!e) e = hip_check(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    if (e) return e;
    unsigned long long h[kStatWords] = {0};
    for (int sl = 0; sl < kStatSlots; ++sl)
        for (int k = 0; k < kStatWords; ++k) h[k] += raw[(size_t)sl * kStatWords + k];
    for (int b = 0; b < 32; ++b) out->iters_hist[b] = (long long)h[b];
    out->floor_hits = (long long)h[32];
    out->nonconverged = (long long)h[33];
    out->nonphys = (long long)h[34];
    out->guess_faces = (long long)h[35];
    out->guess_fallbacks = (long long)h[36];
    return PPMLR_OK;
}

ppmlr_status ppmlr_reset_stats(ppmlr_ctx *c, void *stream)
{
    if (!c) return PPMLR_EINVAL;
    hipLaunchKernelGGL(clear_u64, dim3(1), dim3(256), 0, (hipStream_t)stream, c->d_stats, kStatWords * kStatSlots);
    return hip_check(c, hipGetLastError(), "reset stats");
}

ppmlr_status ppmlr_status_check(ppmlr_ctx *c, void *stream)
{
    ppmlr_stats_t s;
    ppmlr_status e = ppmlr_stats(c, stream, &s);
    if (e) return e;
    if (s.nonphys > 0) return fail(c, PPMLR_ENONPHYS, "non-physical zones entered a sweep");
    if (s.nonconverged > 0) return fail(c, PPMLR_ERIEMANN, "Riemann iteration limit reached");
    return PPMLR_OK;
}

ppmlr_status ppmlr_set_tile(ppmlr_ctx *c, int axis, int pencils)
{
    if (!c || axis < 0 || axis > 2 || pencils < 0) return PPMLR_EINVAL;
    if (pencils > 0) {
        int M = tile_M(c, axis, 4);
        if (block_threads(pencils, M) > 1024) return fail(c, PPMLR_EINVAL, "tile exceeds 1024 threads");
        if (ppmlr::lds_bytes(kSlotsA + kSlotsB, pencils * M, 4) > 160 * 1024)
            return fail(c, PPMLR_EINVAL, "tile exceeds the LDS budget");
    }
    c->tile[axis] = pencils;
    return PPMLR_OK;
}

ppmlr_status ppmlr_set_segments(ppmlr_ctx *c, int axis, int segments)
{
    if (!c || axis < 0 || axis > 2 || segments < 0) return PPMLR_EINVAL;
    const int old = c->seg[axis];
    c->seg[axis] = segments;
    const int k = seg_count(c, axis, 4);
    const int L = seg_len(c->n[axis], k);
    const char *why = nullptr;
    if (L == 0) why = "segment count leaves a segment empty";
    else if (k > 1 && L < kG) why = "segments shorter than the ghost width";
    else if (c->tile[axis] > 0 && block_threads(c->tile[axis], L + 2 * kG) > 1024) why = "tile exceeds 1024 threads";
    if (why) {
        c->seg[axis] = old;
        return fail(c, PPMLR_EINVAL, why);
    }
    return PPMLR_OK;
}

ppmlr_status ppmlr_set_segment_order(ppmlr_ctx *c, int axis, int order)
{
    if (!c || axis < 0 || axis > 2 || order < 0 || order > 2) return PPMLR_EINVAL;
    c->seg_order[axis] = order;
    return PPMLR_OK;
}

ppmlr_status ppmlr_get_segment_order(const ppmlr_ctx *c, int axis, int *order)
{
    if (!c || axis < 0 || axis > 2 || !order) return PPMLR_EINVAL;
    *order = seg_fast_for(c, axis) ? 1 : 2;
    return PPMLR_OK;
}

ppmlr_status ppmlr_get_segments(const ppmlr_ctx *c, int axis, int dtype, int *segments)
{
    if (!c || axis < 0 || axis > 2 || !segments) return PPMLR_EINVAL;
    *segments = seg_count(c, axis, dtype == PPMLR_F64 ? 8 : 4);
    return PPMLR_OK;
}

ppmlr_status ppmlr_autotune(ppmlr_ctx *c, const ppmlr_state *s, int reps, int tiles[3])
{
    ppmlr_status e = check_state(c, s);
    if (e) return e;
    if (reps < 1) return fail(c, PPMLR_EINVAL, "reps must be >= 1");
    const size_t elem = s->dtype == PPMLR_F64 ? 8 : 4;
    const size_t bytes = (size_t)8 * c->n[0] * c->n[1] * c->n[2] * elem;
    hipStream_t st = (hipStream_t)s->stream;
    double dt = 0.0;
    e = ppmlr_cfl_dt(c, s, 0.2, &dt);
    if (e) return e;
    void *scratch = nullptr;
    e = hip_check(c, hipMalloc(&scratch, bytes), "hipMalloc");
    if (e) return e;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (!e) e = hip_check(c, hipEventCreate(&t0), "hipEventCreate");
    if (!e) e = hip_check(c, hipEventCreate(&t1), "hipEventCreate");
    const bool prof = c->profiling;
    c->profiling = false;
    const int guess = c->guess;             // the scratch copy is never harvested
    if (guess == PPMLR_GUESS_HARVEST) c->guess = PPMLR_GUESS_PLAIN;
    ppmlr_state tmp = *s;
    tmp.u = scratch;
    // time `r` sweeps of the current shape on a fresh copy of the state
    auto time_shape = [&](int axis, int r, float &ms) -> ppmlr_status {
        ppmlr_status e2 = hip_check(c, hipMemcpyAsync(scratch, s->u, bytes, hipMemcpyDeviceToDevice, st),
                                    "hipMemcpyAsync");
        Flow f{scratch, scratch};
        if (!e2) e2 = do_sweep(c, &tmp, dt, nullptr, axis, false, f);   // warm-up
        if (!e2) e2 = hip_check(c, hipEventRecord(t0, st), "hipEventRecord");
        for (int k = 0; k < r && !e2; ++k) e2 = do_sweep(c, &tmp, dt, nullptr, axis, false, f);
        if (!e2) e2 = hip_check(c, hipEventRecord(t1, st), "hipEventRecord");
        if (!e2) e2 = hip_check(c, hipEventSynchronize(t1), "hipEventSynchronize");
        if (!e2) e2 = hip_check(c, hipEventElapsedTime(&ms, t0, t1), "hipEventElapsedTime");
        ms /= (float)r;
        return e2;
    };
    struct Shape { float ms; int P, nseg, order; };
    for (int axis = 0; axis < 3 && !e; ++axis) {
        std::vector<Shape> shapes;
        for (int cand = 0; cand < 2 * kMaxSegments && !e; ++cand) {
            const int nseg = 1 + cand / 2, order = 1 + cand % 2;
            if (nseg == 1 && order == 2) continue;         // one segment: no order
            const int L = seg_len(c->n[axis], nseg);
            if (L == 0) continue;
            if (L < kG) break;
            const int M = L + 2 * kG;
            c->seg[axis] = nseg;
            c->seg_order[axis] = nseg == 1 ? 0 : order;
            for (int P = 1; P <= 32 && !e; ++P) {
                const int thr = block_threads(P, M);
                if (thr > 1024) break;
                if (stride_for(thr, (int)elem) < 0) continue;
                c->tile[axis] = P;
                float ms = 0.0f;
                e = time_shape(axis, reps, ms);
                if (!e) shapes.push_back({ms, P, nseg, c->seg_order[axis]});
            }
        }
        // the three fastest again, with three times the repetitions
        std::sort(shapes.begin(), shapes.end(), [](const Shape &x, const Shape &y) { return x.ms < y.ms; });
        Shape best = shapes.empty() ? Shape{0.0f, 1, 1, 0} : shapes[0];
        float best_ms = 1e30f;
        for (size_t k = 0; k < shapes.size() && k < 3 && !e; ++k) {
            c->seg[axis] = shapes[k].nseg;
            c->seg_order[axis] = shapes[k].order;
            c->tile[axis] = shapes[k].P;
            float ms = 0.0f;
            e = time_shape(axis, 3 * reps, ms);
            if (!e && ms < best_ms) { best_ms = ms; best = shapes[k]; }
        }
        c->tile[axis] = best.P;
        c->seg[axis] = best.nseg;
        c->seg_order[axis] = best.order;
        if (tiles) tiles[axis] = best.P;
    }
    c->profiling = prof;
    c->guess = guess;
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(scratch);
    return e;
}

}  // extern "C"

namespace {

// Polls of a barrier wait before it gives up, by default (each poll is an
// agent-scope load plus a short sleep, well above a microsecond: seconds in
// all, against milliseconds for the longest sweep of an ensemble).
constexpr long long kBarSpinLimit = 1ll << 22;
int g_ensemble_block = 0;   // set by ppmlr_ensemble_autotune
int g_ensemble_launch = PPMLR_ENSEMBLE_PER_SWEEP;    // set by ppmlr_set_ensemble_launch
long long g_ensemble_barrier_polls = kBarSpinLimit;  // set by ppmlr_set_ensemble_barrier_limit

// dt of every member from its signal-speed maximum, exactly as dt_kernel
// (one wave of kCflSlots threads per member)
__global__ void ens_dt_kernel(unsigned long long *const *smax_bits, double *const *dt, double *const *t, int members,
                              double cfl)
{
    const int m = blockIdx.x;
    if (m >= members) return;
    const unsigned long long bits = slot_max(smax_bits[m]);
    smax_bits[m][threadIdx.x * ppmlr::kCflStride] = 0ull;
    if (threadIdx.x != 0) return;
    double smax = __longlong_as_double((long long)bits);
    double d = smax > 0.0 ? cfl / smax : 0.0;
    *dt[m] = d;
    *t[m] += d;
}

// Device work tables of one ensemble call: the sweep descriptors (3 axes x 2
// buffer parities x members), the tile offsets (3 axes x (members + 1)), the
// per-member signal-speed / dt / time pointers (3 x members), the members'
// signal-speed arguments and the barrier words of the persistent launch,
// each part starting on a 256-byte boundary.
// ---------------------------------------------------------------- persistent ensemble

// Barrier words of one persistent launch, each on its own 256-byte line:
// arrival count, generation, status (0 = running, 1 = a barrier wait gave
// up); then the tile counters of the sweeps, two sets (sweeps alternate
// between them) of one counter per XCD, 256 bytes apart.
constexpr int kBarCount = 0, kBarGen = 64, kBarStatus = 128, kBarTiles = 192, kBarWords = kBarTiles + 2 * 8 * 64;

// Grid-wide barrier of a co-resident grid (cooperative launch).  Every
// workgroup's writes before the barrier are visible to every workgroup after
// it: the workgroup barrier orders the workgroup's writes before thread 0's
// agent-scope release (which on a multi-XCD device writes dirty L2 lines
// back), and thread 0's agent-scope acquire after the wait invalidates the
// stale lines of its CU and XCD before any thread reads.  A wait that sees
// the status set, or polls `limit` times, gives up: it sets the status
// and returns false, and so does every later barrier, so all workgroups
// leave the kernel.  gen: this workgroup's count of barriers passed; s_ok:
// one LDS word of the workgroup.
__device__ bool grid_barrier(unsigned int *bar, unsigned int nblocks, unsigned int &gen, unsigned int *s_ok,
                             long long limit)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned int target = gen + 1;
        __threadfence();
        const unsigned int prev =
            __hip_atomic_fetch_add(&bar[kBarCount], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == nblocks - 1) {
            // last to arrive: reset the count, then open the next generation
            __hip_atomic_store(&bar[kBarCount], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar[kBarGen], target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long long polls = 0;
            while (__hip_atomic_load(&bar[kBarGen], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != target) {
                if (__hip_atomic_load(&bar[kBarStatus], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                    ++polls > limit) {
                    __hip_atomic_store(&bar[kBarStatus], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        if (ok && __hip_atomic_load(&bar[kBarStatus], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) ok = 0;
        __threadfence();
        gen = target;
        *s_ok = (unsigned int)ok;
    }
    __syncthreads();
    return *s_ok != 0u;
}

template <typename T>
struct PersistArgs {
    const ppmlr::SweepArgs<T> *desc;   // [3 axes][2 buffer parities][members]
    const int *mo;                     // [3][members + 1] tile offsets
    const CflArgs<T> *cfla;            // [members]: the start-of-call signal-speed maximum
    unsigned long long *const *smax;   // [members] signal-speed slots
    double *const *dt;                 // [members] device dt
    double *const *t;                  // [members] simulated time
    unsigned int *bar;                 // barrier words (kBarWords, zero at launch)
    long long barrier_polls;           // polls of a barrier wait before it gives up
    int members, steps;
    int odd0;                          // the first step runs z, y, x
    double cfl;
};

// One persistent launch for a whole ensemble call.  Phases, separated by
// grid barriers: clear the members' signal-speed slots; the start-of-call
// maximum of every member (the arithmetic of cfl_kernel); then per step the
// members' dt (the arithmetic of dt_kernel) and the step's three sweeps over
// the tiles of all members (sweep_tile, exactly as in ensemble_sweep_kernel;
// the last sweep of a step also collects the next maximum).  The tiles of a
// sweep are cut into 8 consecutive shares in the order of the
// one-launch-per-sweep kernel, share x for the workgroups of XCD x (b mod 8;
// G is a multiple of 8), so that neighbouring tiles meet in one L2; within
// its share a workgroup claims the next tile from the XCD's counter, which
// balances tiles of unequal cost.  The grid must be co-resident: it is
// launched cooperatively.
template <typename T, bool STATS, int SM>
__global__ void __launch_bounds__(SM) ensemble_persistent_kernel(const PersistArgs<T> p)
{
    // all LDS is the dynamic allocation (tile buffers at address 0, then the
    // workgroup's scalars: per-wave maxima, counters, the barrier flag)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    unsigned char *tail = smem_raw + ppmlr::lds_tile_bytes(kSlotsA + kSlotsB, SM, (int)sizeof(T));
    double *s_red = reinterpret_cast<double *>(tail);
    unsigned int *s_stat = reinterpret_cast<unsigned int *>(tail + 16 * sizeof(double));
    unsigned int *s_ok = s_stat + ppmlr::kStatWords;
    double *cred = s_red;
    const int b = blockIdx.x;
    const unsigned int G = gridDim.x;
    unsigned int gen = 0;
    const int n = p.members;
    // slots cleared
    for (int m = b; m < n; m += (int)G)
        if (threadIdx.x < ppmlr::kCflSlots) p.smax[m][threadIdx.x * ppmlr::kCflStride] = 0ull;
    if (!grid_barrier(p.bar, G, gen, s_ok, p.barrier_polls)) return;
    // start-of-call signal-speed maximum of every member
    for (int m = 0; m < n; ++m) {
        const CflArgs<T> &ca = p.cfla[m];
        double smax = 0.0;
        for (long long z = (long long)b * SM + threadIdx.x; z < ca.vol; z += (long long)G * SM) {
            const double s = cfl_zone(ca, z);
            smax = s > smax ? s : smax;
        }
        for (int off = 32; off > 0; off >>= 1) {
            double o = __shfl_xor(smax, off);
            smax = o > smax ? o : smax;
        }
        if (__lane_id() == 0) cred[threadIdx.x >> 6] = smax;
        __syncthreads();
        if (threadIdx.x == 0) {
            double mx = cred[0];
            for (int w = 1; w < SM / 64; ++w) mx = cred[w] > mx ? cred[w] : mx;
            atomicMax(p.smax[m] + (b % ppmlr::kCflSlots) * ppmlr::kCflStride,
                      (unsigned long long)__double_as_longlong(mx));
        }
        __syncthreads();
    }
    if (!grid_barrier(p.bar, G, gen, s_ok, p.barrier_polls)) return;
    static const int even[3] = {0, 1, 2}, odd[3] = {2, 1, 0};
    long long j = 0;                                   // sweeps done in this call
    for (int s = 0; s < p.steps; ++s) {
        // dt of every member from its maximum; the slots are cleared for the next one
        for (int m = b; m < n; m += (int)G) {
            if (threadIdx.x < 64) {
                const unsigned long long bits = slot_max(p.smax[m]);
                p.smax[m][threadIdx.x * ppmlr::kCflStride] = 0ull;
                if (threadIdx.x == 0) {
                    const double smx = __longlong_as_double((long long)bits);
                    const double d = smx > 0.0 ? p.cfl / smx : 0.0;
                    *p.dt[m] = d;
                    *p.t[m] += d;
                }
            }
        }
        if (!grid_barrier(p.bar, G, gen, s_ok, p.barrier_polls)) return;
        const int *ord = ((p.odd0 + s) % 2 == 0) ? even : odd;
        for (int k = 0; k < 3; ++k, ++j) {
            const int ax = ord[k];
            const ppmlr::SweepArgs<T> *desc = p.desc + ((size_t)ax * 2 + (size_t)(j & 1)) * n;
            const int *mo = p.mo + (size_t)ax * (n + 1);
            const int total = mo[n];
            const int per_xcd = (total + 7) / 8;
            const int xcd = b & 7;
            unsigned int *ctr = p.bar + kBarTiles + ((j & 1) * 8 + xcd) * 64;
            // the other set is free (its sweep ended before the last barrier)
            // and is cleared for the next sweep, before the barrier after this one
            if (b < 8 && threadIdx.x == 0)
                __hip_atomic_store(p.bar + kBarTiles + (((j + 1) & 1) * 8 + b) * 64, 0u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            const int lo_t = xcd * per_xcd, hi_t = min(total, lo_t + per_xcd);
            for (;;) {
                if (threadIdx.x == 0)
                    s_ok[1] = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __syncthreads();
                const int jt = lo_t + (int)s_ok[1];
                __syncthreads();                      // the claim word is reused by the next claim
                if (jt >= hi_t) break;
                int lo = 0, hi = n - 1;               // largest m with mo[m] <= jt
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (mo[mid] <= jt) lo = mid; else hi = mid - 1;
                }
                const ppmlr::SweepArgs<T> &a = desc[lo];
                const int t = jt - mo[lo];
                int seg, tt;
                if (a.seg_fast) { seg = t % a.nseg; tt = t / a.nseg; }
                else { seg = t / a.ntiles; tt = t - seg * a.ntiles; }
                const int tq = tt % a.tiles_q;
                const int r = tt / a.tiles_q;
                const T dtm = T(*a.dt_dev);
                unsigned long long *cm =
                    (k == 2 && a.cfl_max) ? a.cfl_max + (b % ppmlr::kCflSlots) * ppmlr::kCflStride : nullptr;
                if (ax == 0)
                    ppmlr::sweep_tile<0, T, STATS, true, SM>(a, tq, r, seg, dtm, cm, b % kStatSlots, smem_raw, s_red,
                                                             s_stat);
                else if (ax == 1)
                    ppmlr::sweep_tile<1, T, STATS, true, SM>(a, tq, r, seg, dtm, cm, b % kStatSlots, smem_raw, s_red,
                                                             s_stat);
                else
                    ppmlr::sweep_tile<2, T, STATS, true, SM>(a, tq, r, seg, dtm, cm, b % kStatSlots, smem_raw, s_red,
                                                             s_stat);
                __syncthreads();                      // the tile buffers are reused by the next tile
            }
            if (!grid_barrier(p.bar, G, gen, s_ok, p.barrier_polls)) return;
        }
    }
}

template <typename T>
struct EnsTables {
    static constexpr size_t up256(size_t b) { return (b + 255) / 256 * 256; }
    static constexpr size_t desc_bytes(int n) { return up256(sizeof(ppmlr::SweepArgs<T>) * 6 * (size_t)n); }
    static constexpr size_t mo_bytes(int n) { return up256(sizeof(int) * 3 * ((size_t)n + 1)); }
    static constexpr size_t ptr_bytes(int n) { return up256(sizeof(void *) * 3 * (size_t)n); }
    static constexpr size_t cfl_bytes(int n) { return up256(sizeof(CflArgs<T>) * (size_t)n); }
    static constexpr size_t bar_bytes() { return up256(sizeof(unsigned int) * kBarWords); }
    static constexpr size_t bytes(int n)
    {
        return desc_bytes(n) + mo_bytes(n) + ptr_bytes(n) + cfl_bytes(n) + bar_bytes();
    }
};

// One ensemble call.  tables: device memory of EnsTables<T>::bytes(n) for
// the work tables, or nullptr to allocate them for this call (and free them
// at its end).  With tables given, nothing is allocated: a member whose
// pencils are cut into segments must then already have its context's second
// state.
template <typename T>
ppmlr_status ensemble_typed(ppmlr_ctx *const *ctxs, const ppmlr_state *const *states, int n, int steps, double cfl,
                            int block, unsigned char *tables = nullptr, bool persistent = true)
{
    ppmlr_ctx *c0 = ctxs[0];
    hipStream_t st = (hipStream_t)states[0]->stream;
    // Members whose pencils are cut into segments (their contexts' setting)
    // alternate every sweep between their state and their context's second
    // state: sweep j of this call reads the first when j is even.  The other
    // members sweep in place.
    std::vector<char> pp(n, 0);
    for (int m = 0; m < n; ++m) {
        for (int ax = 0; ax < 3; ++ax)
            if (seg_count(ctxs[m], ax, (int)sizeof(T)) > 1) pp[m] = 1;
        if (pp[m] && tables) {
            if (ctxs[m]->pong_bytes < state_bytes(ctxs[m], states[m]))
                return fail(c0, PPMLR_EINVAL,
                            "member " + std::to_string(m) + " is cut into pencil segments but its context has no "
                            "second state yet (run it once through ppmlr_ensemble_run or sweep it, or use whole "
                            "pencils)");
        } else if (pp[m]) {
            ppmlr_status e = ensure_pong(ctxs[m], state_bytes(ctxs[m], states[m]));
            if (e) return e;
        }
    }
    // per axis, sweep parity and member: pencils per workgroup = as many as
    // fit the block; dt from the member's device dt, signal speeds into its
    // own slot
    std::vector<ppmlr::SweepArgs<T>> desc((size_t)6 * n);
    std::vector<int> mo((size_t)3 * (n + 1));
    bool stats = false;
    for (int ax = 0; ax < 3; ++ax) {
        long long off = 0;
        for (int m = 0; m < n; ++m) {
            ppmlr_ctx *c = ctxs[m];
            if (c->opt.collect_stats) stats = true;
            const int nseg = seg_count(c, ax, (int)sizeof(T));
            const int M = tile_M(c, ax, (int)sizeof(T));
            const int nq = (ax == 0) ? c->n[1] : c->n[0];
            const int P = std::max(1, std::min(block / M, nq));
            T *home = (T *)states[m]->u, *pong = (T *)c->d_pong;
            for (int par = 0; par < 2; ++par) {
                const T *in = (pp[m] && par) ? pong : home;
                T *out = pp[m] ? (par ? home : pong) : home;
                fill_args(c, desc[((size_t)ax * 2 + par) * n + m], in, out, ax, 0.0, c->d_dt, P, nseg);
            }
            mo[(size_t)ax * (n + 1) + m] = (int)off;
            off += (long long)desc[(size_t)ax * 2 * n + m].ntiles * nseg;
        }
        if (off > (long long)INT_MAX / 2) return fail(c0, PPMLR_EINVAL, "ensemble too large for one launch");
        mo[(size_t)ax * (n + 1) + n] = (int)off;
    }
    ppmlr_status err = PPMLR_OK;
    unsigned char *owned = nullptr;
    if (!tables) {
        err = hip_check(c0, hipMalloc((void **)&owned, EnsTables<T>::bytes(n)), "hipMalloc");
        tables = owned;
    }
    auto up = [&](void *dst, const void *src, size_t bytes) {
        if (!err) err = hip_check(c0, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    };
    auto *d_desc = (ppmlr::SweepArgs<T> *)tables;
    auto *d_mo = (int *)(tables + EnsTables<T>::desc_bytes(n));
    auto *d_ptr = (void **)(tables + EnsTables<T>::desc_bytes(n) + EnsTables<T>::mo_bytes(n));
    auto *d_cfl = (CflArgs<T> *)(tables + EnsTables<T>::desc_bytes(n) + EnsTables<T>::mo_bytes(n) +
                                  EnsTables<T>::ptr_bytes(n));
    auto *d_bar = (unsigned int *)((unsigned char *)d_cfl + EnsTables<T>::cfl_bytes(n));
    std::vector<CflArgs<T>> cfla((size_t)n);
    std::vector<unsigned int> bar0(kBarWords, 0u);
    if (!err) {
        std::vector<void *> ptr((size_t)3 * n);
        for (int m = 0; m < n; ++m) {
            ptr[m] = ctxs[m]->d_cflmax;
            ptr[(size_t)n + m] = ctxs[m]->d_dt;
            ptr[(size_t)2 * n + m] = ctxs[m]->d_time;
        }
        up(d_desc, desc.data(), sizeof(ppmlr::SweepArgs<T>) * desc.size());
        up(d_mo, mo.data(), sizeof(int) * mo.size());
        up(d_ptr, ptr.data(), sizeof(void *) * ptr.size());
        if (persistent) {
            for (int m = 0; m < n; ++m) cfla[m] = cfl_args(ctxs[m], (const T *)states[m]->u);
            up(d_cfl, cfla.data(), sizeof(CflArgs<T>) * cfla.size());
            up(d_bar, bar0.data(), sizeof(unsigned int) * bar0.size());
        }
        // the host tables must stay alive until the copies have been made
        if (!err) err = hip_check(c0, hipStreamSynchronize(st), "hipStreamSynchronize");
    }
    const size_t lds = ppmlr::lds_bytes(kSlotsA + kSlotsB, block, (int)sizeof(T));
    long long j = 0;                                       // sweeps enqueued by this call
    if (persistent && !err) {
        // one cooperative launch of as many workgroups as the device holds at
        // once (the runtime refuses a grid that cannot be co-resident)
        PersistArgs<T> pa;
        pa.desc = d_desc;
        pa.mo = d_mo;
        pa.cfla = d_cfl;
        pa.smax = (unsigned long long *const *)d_ptr;
        pa.dt = (double *const *)(d_ptr + n);
        pa.t = (double *const *)(d_ptr + 2 * (size_t)n);
        pa.bar = d_bar;
        pa.barrier_polls = g_ensemble_barrier_polls;
        pa.members = n;
        pa.steps = steps;
        pa.odd0 = (int)(c0->step % 2);
        pa.cfl = cfl;
        int maxtiles = 8;
        for (int ax = 0; ax < 3; ++ax) maxtiles = std::max(maxtiles, mo[(size_t)ax * (n + 1) + n]);
        auto launch = [&](auto kern) {
            if (lds > 64 * 1024) {
                hipError_t he =
                    hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                if (he != hipSuccess) { err = hip_check(c0, he, "hipFuncSetAttribute"); return; }
            }
            int per_cu = 0, cus = 0, coop = 0;
            err = hip_check(c0, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, block, lds),
                            "hipOccupancyMaxActiveBlocksPerMultiprocessor");
            if (!err) err = hip_check(c0, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c0->device),
                                      "hipDeviceGetAttribute");
            if (!err) err = hip_check(c0, hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c0->device),
                                      "hipDeviceGetAttribute");
            if (err) return;
            if (!coop || per_cu < 1) { err = fail(c0, PPMLR_EDEVICE, "no cooperative launch for the ensemble kernel"); return; }
            // a multiple of 8 (the XCD-aware tile order keeps each workgroup on its XCD's share)
            long long G = (long long)per_cu * cus;
            G = std::min<long long>(G, ((long long)maxtiles + 7) / 8 * 8);
            G = std::max<long long>(8, G / 8 * 8);
            void *args[] = {(void *)&pa};
            err = hip_check(c0, hipLaunchCooperativeKernel((const void *)kern, dim3((unsigned)G), dim3(block), args,
                                                           (unsigned)lds, st), "hipLaunchCooperativeKernel");
        };
#define PPMLR_PERS(B_)                                                                   \
        if (stats) launch(ensemble_persistent_kernel<T, true, B_>);                       \
        else launch(ensemble_persistent_kernel<T, false, B_>);
        if (block == 256) { PPMLR_PERS(256) }
        else if (block == 512) { PPMLR_PERS(512) }
        else {
            if constexpr (sizeof(T) == 4) { PPMLR_PERS(1024) }
            else err = fail(c0, PPMLR_EINVAL, "FP64 ensembles use block 256 or 512");
        }
#undef PPMLR_PERS
        unsigned int status = 0;
        if (!err) err = hip_check(c0, hipMemcpyAsync(&status, d_bar + kBarStatus, sizeof(status),
                                                     hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
        if (!err) err = hip_check(c0, hipStreamSynchronize(st), "hipStreamSynchronize");
        if (!err && status != 0u)
            err = fail(c0, PPMLR_EDEVICE, "ensemble kernel: a grid barrier wait gave up (workgroups not co-resident?)");
        j = 3LL * steps;
    }
    // one launch per sweep: the start-of-call maximum, then per step the dt
    // kernel and three sweep kernels
    if (!persistent)
        for (int m = 0; m < n && !err; ++m) err = cfl_launch(ctxs[m], states[m]);
    static const int even[3] = {0, 1, 2}, odd[3] = {2, 1, 0};
    for (int s = 0; s < steps && !err && !persistent; ++s) {
        hipLaunchKernelGGL(ens_dt_kernel, dim3(n), dim3(ppmlr::kCflSlots), 0, st, (unsigned long long *const *)d_ptr,
                           (double *const *)(d_ptr + n), (double *const *)(d_ptr + 2 * (size_t)n), n, cfl);
        const int *ord = ((c0->step + s) % 2 == 0) ? even : odd;
        for (int k = 0; k < 3 && !err; ++k) {
            const int ax = ord[k];
            ppmlr::EnsembleSweepArgs<T> e;
            e.desc = d_desc + ((size_t)ax * 2 + (size_t)(j & 1)) * n;
            e.mo = d_mo + (size_t)ax * (n + 1);
            e.members = n;
            e.total = mo[(size_t)ax * (n + 1) + n];
            e.per_xcd = (e.total + 7) / 8;
            const dim3 grid(8 * e.per_xcd);
            auto launch = [&](auto kern) {
                if (lds > 64 * 1024) {
                    hipError_t he = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                        (int)lds);
                    if (he != hipSuccess) { err = hip_check(c0, he, "hipFuncSetAttribute"); return; }
                }
                hipLaunchKernelGGL(kern, grid, dim3(block), lds, st, e);
            };
#define PPMLR_ENS3(AX_, B_)                                                                              \
            if (stats) { if (k == 2) launch(ppmlr::ensemble_sweep_kernel<AX_, T, true, true, B_>);         \
                         else launch(ppmlr::ensemble_sweep_kernel<AX_, T, true, false, B_>); }             \
            else { if (k == 2) launch(ppmlr::ensemble_sweep_kernel<AX_, T, false, true, B_>);              \
                   else launch(ppmlr::ensemble_sweep_kernel<AX_, T, false, false, B_>); }
#define PPMLR_ENS(B_)                                                                                    \
            if (ax == 0) { PPMLR_ENS3(0, B_) } else if (ax == 1) { PPMLR_ENS3(1, B_) } else { PPMLR_ENS3(2, B_) }
            if (block == 256) { PPMLR_ENS(256) }
            else if (block == 512) { PPMLR_ENS(512) }
            else {
                if constexpr (sizeof(T) == 4) { PPMLR_ENS(1024) }
                else err = fail(c0, PPMLR_EINVAL, "FP64 ensembles use block 256 or 512");
            }
#undef PPMLR_ENS
#undef PPMLR_ENS3
            if (!err) err = hip_check(c0, hipGetLastError(), "ensemble sweep launch");
            ++j;
        }
    }
    // after an odd number of sweeps the alternating members are in their
    // second state
    for (int m = 0; m < n && !err && (j & 1); ++m)
        if (pp[m])
            err = hip_check(c0, hipMemcpyAsync(states[m]->u, ctxs[m]->d_pong, state_bytes(ctxs[m], states[m]),
                                               hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
    // tables allocated here are freed once the launches that read them are done
    if (owned) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(owned);
    }
    return err;
}

ppmlr_status ensemble_check(ppmlr_ctx *const *ctxs, const ppmlr_state *const *states, int n, int steps, double cfl,
                            int block)
{
    if (!ctxs || !states || n < 1 || steps < 0 || !(cfl > 0.0)) return PPMLR_EINVAL;
    for (int m = 0; m < n; ++m) {
        if (!ctxs[m] || !states[m]) return PPMLR_EINVAL;
        ppmlr_status e = check_state(ctxs[m], states[m]);
        if (e) return e;
        if (states[m]->dtype != states[0]->dtype) return fail(ctxs[0], PPMLR_EINVAL, "members differ in dtype");
        if (states[m]->stream != states[0]->stream) return fail(ctxs[0], PPMLR_EINVAL, "members differ in stream");
        if ((ctxs[m]->step & 1) != (ctxs[0]->step & 1)) return fail(ctxs[0], PPMLR_EINVAL, "step parity differs");
        if (ctxs[m]->series_n > 0) return fail(ctxs[0], PPMLR_EINVAL, "inflow time series are not supported in ensembles");
        if (ctxs[m]->opt.tracing != PPMLR_TRACE_TWO_FAMILY)
            return fail(ctxs[0], PPMLR_EINVAL, "ensembles use the two-family tracing");
        const int elem = states[m]->dtype == PPMLR_F64 ? 8 : 4;
        for (int a = 0; a < 3; ++a)
            if (tile_M(ctxs[m], a, elem) > block)
                return fail(ctxs[0], PPMLR_EINVAL, "a pencil segment does not fit the block");
    }
    if (block != 256 && block != 512 && block != 1024) return fail(ctxs[0], PPMLR_EINVAL, "block must be 256, 512 or 1024");
    if (block == 1024 && states[0]->dtype == PPMLR_F64) return fail(ctxs[0], PPMLR_EINVAL, "FP64 block <= 512");
    return PPMLR_OK;
}

// Most members of one ppmlr_ensemble_run_noalloc call, and the bytes of its
// work tables at that count (FP64 descriptors are the larger).
constexpr int kNoallocMaxMembers = 64;
constexpr size_t kNoallocBytes = EnsTables<double>::bytes(kNoallocMaxMembers);
static_assert(EnsTables<float>::bytes(kNoallocMaxMembers) <= kNoallocBytes, "FP32 tables fit");

}  // namespace

// Work tables of ppmlr_ensemble_run_noalloc: a fixed array in device memory,
// one copy per GPU that the library runs on, held until the process ends.
// Host code never uses this name as a device address: each device's address
// comes from hipGetSymbolAddress (noalloc_tables below).
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on device dev, looked up once per device with that
// device current (and the caller's current device restored).
ppmlr_status noalloc_tables(ppmlr_ctx *c, int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(c, PPMLR_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        ppmlr_status e = hip_check(c, hipGetDevice(&cur), "hipGetDevice");
        if (!e && cur != dev) e = hip_check(c, hipSetDevice(dev), "hipSetDevice");
        if (e) return e;
        void *ptr = nullptr;
        e = hip_check(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
        if (cur != dev) {
            ppmlr_status e2 = hip_check(c, hipSetDevice(cur), "hipSetDevice");
            if (!e) e = e2;
        }
        if (e) return e;
        if (!ptr) return fail(c, PPMLR_EDEVICE, "hipGetSymbolAddress returned no address");
        g_scratch_ptr[dev] = (unsigned char *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return PPMLR_OK;
}

}  // namespace

extern "C" {

ppmlr_status ppmlr_ensemble_run_noalloc(ppmlr_ctx *const *ctxs, const ppmlr_state *const *states, int n, int steps,
                                        double cfl, int block, ppmlr_status *per_member)
{
    if (block == 0) block = g_ensemble_block ? g_ensemble_block : 512;
    ppmlr_status e = ensemble_check(ctxs, states, n, steps, cfl, block);
    if (e) return e;
    if (n > kNoallocMaxMembers)
        return fail(ctxs[0], PPMLR_EINVAL, "ppmlr_ensemble_run_noalloc takes at most " +
                                               std::to_string(kNoallocMaxMembers) + " members, got " +
                                               std::to_string(n));
    for (int m = 1; m < n; ++m)
        if (ctxs[m]->device != ctxs[0]->device)
            return fail(ctxs[0], PPMLR_EINVAL, "members are on different devices");
    if (steps > 0) {
        unsigned char *tables = nullptr;
        e = noalloc_tables(ctxs[0], ctxs[0]->device, &tables);
        if (!e)
            e = states[0]->dtype == PPMLR_F64
                    ? ensemble_typed<double>(ctxs, states, n, steps, cfl, block, tables,
                                             g_ensemble_launch == PPMLR_ENSEMBLE_PERSISTENT)
                    : ensemble_typed<float>(ctxs, states, n, steps, cfl, block, tables,
                                            g_ensemble_launch == PPMLR_ENSEMBLE_PERSISTENT);
        if (!e)
            for (int m = 0; m < n; ++m) ctxs[m]->step += steps;
    }
    if (per_member)
        for (int m = 0; m < n; ++m) per_member[m] = e ? e : ppmlr_status_check(ctxs[m], states[m]->stream);
    return e;
}

ppmlr_status ppmlr_ensemble_run(ppmlr_ctx *const *ctxs, const ppmlr_state *const *states, int n, int steps,
                                double cfl, int block, ppmlr_status *per_member)
{
    if (block == 0) block = g_ensemble_block ? g_ensemble_block : 512;
    ppmlr_status e = ensemble_check(ctxs, states, n, steps, cfl, block);
    if (e) return e;
    if (steps > 0) {
        e = states[0]->dtype == PPMLR_F64
                ? ensemble_typed<double>(ctxs, states, n, steps, cfl, block, nullptr,
                                         g_ensemble_launch == PPMLR_ENSEMBLE_PERSISTENT)
                : ensemble_typed<float>(ctxs, states, n, steps, cfl, block, nullptr,
                                        g_ensemble_launch == PPMLR_ENSEMBLE_PERSISTENT);
        if (!e)
            for (int m = 0; m < n; ++m) ctxs[m]->step += steps;
    }
    if (per_member)
        for (int m = 0; m < n; ++m) per_member[m] = e ? e : ppmlr_status_check(ctxs[m], states[m]->stream);
    return e;
}

ppmlr_status ppmlr_set_ensemble_launch(int mode)
{
    if (mode != PPMLR_ENSEMBLE_PERSISTENT && mode != PPMLR_ENSEMBLE_PER_SWEEP) return PPMLR_EINVAL;
    g_ensemble_launch = mode;
    return PPMLR_OK;
}

ppmlr_status ppmlr_set_ensemble_barrier_limit(long long polls)
{
    if (polls < 0) return PPMLR_EINVAL;
    g_ensemble_barrier_polls = polls;
    return PPMLR_OK;
}

ppmlr_status ppmlr_ensemble_autotune(ppmlr_ctx *const *ctxs, const ppmlr_state *const *states, int n, int reps,
                                     double cfl, int *block)
{
    if (!ctxs || !states || n < 1 || reps < 1) return PPMLR_EINVAL;
    hipStream_t st = (hipStream_t)states[0]->stream;
    std::vector<void *> scratch(n, nullptr);
    std::vector<ppmlr_state> tmp(n);
    std::vector<const ppmlr_state *> tptr(n);
    std::vector<long long> step0(n);
    std::vector<double> time0(n);
    std::vector<int> stat0(n);
    ppmlr_status e = PPMLR_OK;
    for (int m = 0; m < n && !e; ++m) {
        e = check_state(ctxs[m], states[m]);
        if (e) break;
        const size_t bytes = (size_t)8 * ctxs[m]->n[0] * ctxs[m]->n[1] * ctxs[m]->n[2] *
                             (states[m]->dtype == PPMLR_F64 ? 8 : 4);
        e = hip_check(ctxs[m], hipMalloc(&scratch[m], bytes), "hipMalloc");
        if (!e) e = hip_check(ctxs[m], hipMemcpyAsync(scratch[m], states[m]->u, bytes, hipMemcpyDeviceToDevice, st),
                              "hipMemcpyAsync");
        tmp[m] = *states[m];
        tmp[m].u = scratch[m];
        tptr[m] = &tmp[m];
        step0[m] = ctxs[m]->step;
        stat0[m] = ctxs[m]->opt.collect_stats;
        ctxs[m]->opt.collect_stats = 0;
        if (!e) e = hip_check(ctxs[m], hipMemcpy(&time0[m], ctxs[m]->d_time, sizeof(double), hipMemcpyDeviceToHost),
                              "hipMemcpy");
    }
    int best = 0, best_len = 0;
    float best_ms = 1e30f;
    const int cands[3] = {256, 512, 1024};
    // target interior zones per segment (0: whole pencils)
    const int lens[5] = {0, 96, 64, 48, 32};
    auto set_lengths = [&](int len) {
        for (int m = 0; m < n; ++m)
            for (int ax = 0; ax < 3; ++ax) {
                const int N = ctxs[m]->n[ax];
                int k = len > 0 ? (N + len - 1) / len : 0;   // 0: whole pencils where they fit
                while (k > 1 && (seg_len(N, k) == 0 || seg_len(N, k) < kG)) --k;
                ctxs[m]->seg[ax] = k;
            }
    };
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (!e) e = hip_check(ctxs[0], hipEventCreate(&t0), "hipEventCreate");
    if (!e) e = hip_check(ctxs[0], hipEventCreate(&t1), "hipEventCreate");
    for (int cand = 0; cand < 15 && !e; ++cand) {
        const int B = cands[cand / 5], len = lens[cand % 5];
        set_lengths(len);
        if (ensemble_check(ctxs, tptr.data(), n, reps, cfl, B) != PPMLR_OK) continue;
        e = hip_check(ctxs[0], hipEventRecord(t0, st), "hipEventRecord");
        if (!e) e = ppmlr_ensemble_run(ctxs, tptr.data(), n, reps, cfl, B, nullptr);
        if (!e) e = hip_check(ctxs[0], hipEventRecord(t1, st), "hipEventRecord");
        if (!e) e = hip_check(ctxs[0], hipEventSynchronize(t1), "hipEventSynchronize");
        float ms = 0.0f;
        if (!e) e = hip_check(ctxs[0], hipEventElapsedTime(&ms, t0, t1), "hipEventElapsedTime");
        if (!e && ms < best_ms) { best_ms = ms; best = B; best_len = len; }
        for (int m = 0; m < n; ++m) ctxs[m]->step = step0[m];
    }
    set_lengths(best_len);
    // then each axis's segment length on its own, at the chosen block size
    // (the axes favour different lengths: x longer, y and z shorter), timed
    // over at least 5 steps
    if (!e && best) {
        auto set_axis = [&](int ax, int len) {
            for (int m = 0; m < n; ++m) {
                const int N = ctxs[m]->n[ax];
                int k = len > 0 ? (N + len - 1) / len : 0;
                while (k > 1 && (seg_len(N, k) == 0 || seg_len(N, k) < kG)) --k;
                ctxs[m]->seg[ax] = k;
            }
        };
        const int rr = std::max(reps, 5);
        auto timed = [&](float &ms) -> ppmlr_status {
            ppmlr_status er = hip_check(ctxs[0], hipEventRecord(t0, st), "hipEventRecord");
            if (!er) er = ppmlr_ensemble_run(ctxs, tptr.data(), n, rr, cfl, best, nullptr);
            if (!er) er = hip_check(ctxs[0], hipEventRecord(t1, st), "hipEventRecord");
            if (!er) er = hip_check(ctxs[0], hipEventSynchronize(t1), "hipEventSynchronize");
            if (!er) er = hip_check(ctxs[0], hipEventElapsedTime(&ms, t0, t1), "hipEventElapsedTime");
            for (int m = 0; m < n; ++m) ctxs[m]->step = step0[m];
            return er;
        };
        float base_ms = 0.0f;
        e = timed(base_ms);
        for (int ax = 0; ax < 3 && !e; ++ax) {
            int keep = best_len;
            for (int q = 0; q < 5 && !e; ++q) {
                if (lens[q] == keep) continue;
                set_axis(ax, lens[q]);
                float ms = 0.0f;
                if (ensemble_check(ctxs, tptr.data(), n, rr, cfl, best) == PPMLR_OK) {
                    e = timed(ms);
                    if (!e && ms < base_ms) { base_ms = ms; keep = lens[q]; }
                }
                set_axis(ax, keep);
            }
        }
    }
    for (int m = 0; m < n; ++m) {
        ctxs[m]->step = step0[m];
        ctxs[m]->opt.collect_stats = stat0[m];
        (void)hipMemcpy(ctxs[m]->d_time, &time0[m], sizeof(double), hipMemcpyHostToDevice);
        if (scratch[m]) (void)hipFree(scratch[m]);
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (!e && best) {
        g_ensemble_block = best;
        if (block) *block = best;
    } else if (!e) {
        e = fail(ctxs[0], PPMLR_EINVAL, "no feasible ensemble block size");
    }
    return e;
}

ppmlr_status ppmlr_get_tile(const ppmlr_ctx *c, int axis, int dtype, int *pencils)
{
    if (!c || axis < 0 || axis > 2 || !pencils) return PPMLR_EINVAL;
    *pencils = pick_tile(c, axis, dtype == PPMLR_F64 ? 8 : 4);
    return PPMLR_OK;
}


// ---------------------------------------------------------------- learned guess

ppmlr_status ppmlr_set_guess(ppmlr_ctx *c, int mode, const float *theta, void *stream)
{
    if (!c) return PPMLR_EINVAL;
    if (mode != PPMLR_GUESS_PLAIN && mode != PPMLR_GUESS_LEARNED && mode != PPMLR_GUESS_HARVEST)
        return fail(c, PPMLR_EINVAL, "unknown guess mode");
    if (mode == PPMLR_GUESS_LEARNED) {
        if (!theta) return fail(c, PPMLR_EINVAL, "the learned guess needs parameters");
        hipStream_t st = (hipStream_t)stream;
        ppmlr_status e = PPMLR_OK;
        if (!c->d_mlp_frag)
            e = hip_check(c, hipMalloc((void **)&c->d_mlp_frag, sizeof(unsigned short) * 256 * ppmlr::mlp::kTiles),
                          "hipMalloc");
        if (!e && !c->d_mlp_theta)
            e = hip_check(c, hipMalloc((void **)&c->d_mlp_theta, sizeof(float) * ppmlr::mlp::kNPar), "hipMalloc");
        if (!e) e = hip_check(c, hipMemcpyAsync(c->d_mlp_theta, theta, sizeof(float) * ppmlr::mlp::kNPar,
                                                hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
        if (e) return e;
        const int n = 256 * ppmlr::mlp::kTiles;
        hipLaunchKernelGGL(ppmlr::mlp::pack_kernel, dim3((n + 255) / 256), dim3(256), 0, st, c->d_mlp_theta,
                           c->d_mlp_frag, ppmlr::mlp::kTiles);
        e = hip_check(c, hipGetLastError(), "pack launch");
        if (!e) e = hip_check(c, hipStreamSynchronize(st), "hipStreamSynchronize");
        if (e) return e;
    }
    if (mode == PPMLR_GUESS_HARVEST && !c->harvest) return fail(c, PPMLR_EINVAL, "no harvest buffer set");
    c->guess = mode;
    return PPMLR_OK;
}

ppmlr_status ppmlr_set_gate(ppmlr_ctx *c, double rel_p, double rel_u)
{
    if (!c) return PPMLR_EINVAL;
    if (!(rel_p >= 0.0) || !(rel_u >= 0.0)) return fail(c, PPMLR_EINVAL, "gate thresholds must be >= 0");
    c->gate_p = rel_p;
    c->gate_u = rel_u;
    return PPMLR_OK;
}

ppmlr_status ppmlr_set_harvest(ppmlr_ctx *c, float *records, long long capacity, unsigned long long *count)
{
    if (!c) return PPMLR_EINVAL;
    if (records && (capacity < 0 || !count)) return fail(c, PPMLR_EINVAL, "harvest buffer needs a capacity and a counter");
    c->harvest = records;
    c->harvest_cap = records ? capacity : 0;
    c->harvest_count = records ? count : nullptr;
    if (!records && c->guess == PPMLR_GUESS_HARVEST) c->guess = PPMLR_GUESS_PLAIN;
    return PPMLR_OK;
}

// ---------------------------------------------------------------- MLP workspace

static ppmlr_status mlp_fail(ppmlr_mlp *w, ppmlr_status s, const std::string &msg)
{
    if (w) w->err = msg;
    return s;
}

static ppmlr_status mlp_check(ppmlr_mlp *w, hipError_t e, const char *what)
{
    if (e == hipSuccess) return PPMLR_OK;
    return mlp_fail(w, e == hipErrorOutOfMemory ? PPMLR_ENOMEM : PPMLR_EDEVICE,
                    std::string(what) + ": " + hipGetErrorString(e));
}

ppmlr_status ppmlr_mlp_create(int max_batch, ppmlr_mlp **out)
{
    if (!out || max_batch < 1) return PPMLR_EINVAL;
    *out = nullptr;
    ppmlr_mlp *w = new ppmlr_mlp();
    w->max_batch = max_batch;
    ppmlr_status e = mlp_check(w, hipGetDevice(&w->device), "hipGetDevice");
    const size_t blocks = (size_t)(max_batch + 63) / 64;
    if (!e) e = mlp_check(w, hipMalloc((void **)&w->d_frag, sizeof(unsigned short) * 256 * ppmlr::mlp::kTiles), "hipMalloc");
    if (!e) e = mlp_check(w, hipMalloc((void **)&w->d_partials, sizeof(float) * blocks * (ppmlr::mlp::kNPar + 1)),
                          "hipMalloc");
    if (e) {
        ppmlr_mlp_destroy(w);
        return e;
    }
    *out = w;
    return PPMLR_OK;
}

void ppmlr_mlp_destroy(ppmlr_mlp *w)
{
    if (!w) return;
    (void)hipDeviceSynchronize();
    if (w->d_frag) (void)hipFree(w->d_frag);
    if (w->d_partials) (void)hipFree(w->d_partials);
    delete w;
}

const char *ppmlr_mlp_last_error(const ppmlr_mlp *w) { return w ? w->err.c_str() : "null workspace"; }

static ppmlr_status mlp_pack(ppmlr_mlp *w, const float *theta, hipStream_t st)
{
    const int n = 256 * ppmlr::mlp::kTiles;
    hipLaunchKernelGGL(ppmlr::mlp::pack_kernel, dim3((n + 255) / 256), dim3(256), 0, st, theta, w->d_frag,
                       ppmlr::mlp::kTiles);
    return mlp_check(w, hipGetLastError(), "pack launch");
}

ppmlr_status ppmlr_mlp_forward(ppmlr_mlp *w, const float *theta, const float *X, int ldx, int n, float *Y, int ldy,
                               void *stream)
{
    if (!w) return PPMLR_EINVAL;
    if (n < 0) return mlp_fail(w, PPMLR_EINVAL, "negative sample count");
    if (n == 0) return PPMLR_OK;
    if (!theta || !X || !Y || ldx < ppmlr::mlp::kIn || ldy < ppmlr::mlp::kOut)
        return mlp_fail(w, PPMLR_EINVAL, "bad forward arguments");
    hipStream_t st = (hipStream_t)stream;
    ppmlr_status e = mlp_pack(w, theta, st);
    if (e) return e;
    hipLaunchKernelGGL(ppmlr::mlp::forward_kernel, dim3((n + 63) / 64), dim3(64), 0, st, X, ldx, n,
                       (const unsigned short *)w->d_frag, theta, Y, ldy);
    return mlp_check(w, hipGetLastError(), "forward launch");
}

static ppmlr_status mlp_grad_launch(ppmlr_mlp *w, const float *theta, const float *X, int ldx, const float *Y,
                                    int ldy, int n, hipStream_t st)
{
    if (!theta || !X || !Y || n < 1 || n > w->max_batch || ldx < ppmlr::mlp::kIn || ldy < ppmlr::mlp::kOut)
        return mlp_fail(w, PPMLR_EINVAL, "bad batch arguments (1 <= n <= max_batch)");
    ppmlr_status e = mlp_pack(w, theta, st);
    if (e) return e;
    hipLaunchKernelGGL(ppmlr::mlp::grad_kernel, dim3((n + 63) / 64), dim3(64), 0, st, X, ldx, Y, ldy, n,
                       (const unsigned short *)w->d_frag, theta, w->d_partials);
    return mlp_check(w, hipGetLastError(), "grad launch");
}

ppmlr_status ppmlr_mlp_grad(ppmlr_mlp *w, const float *theta, const float *X, int ldx, const float *Y, int ldy, int n,
                            float *grad, float *loss, void *stream)
{
    if (!w) return PPMLR_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    ppmlr_status e = mlp_grad_launch(w, theta, X, ldx, Y, ldy, n, st);
    if (e) return e;
    const int np = ppmlr::mlp::kNPar + 1;
    hipLaunchKernelGGL(ppmlr::mlp::reduce_adam_kernel, dim3((np + 255) / 256), dim3(256), 0, st, w->d_partials,
                       (n + 63) / 64, grad, loss, (float *)nullptr, (float *)nullptr, (float *)nullptr, 0, 0, 0.0f,
                       0.0f, 0.0f, 0.0f);
    return mlp_check(w, hipGetLastError(), "reduce launch");
}

ppmlr_status ppmlr_mlp_train_step(ppmlr_mlp *w, float *theta, float *m, float *v, const float *X, int ldx,
                                  const float *Y, int ldy, int n, int t, float lr, float beta1, float beta2,
                                  float eps, float *loss, void *stream)
{
    if (!w) return PPMLR_EINVAL;
    if (!m || !v || t < 1) return mlp_fail(w, PPMLR_EINVAL, "Adam needs moments and a step number >= 1");
    hipStream_t st = (hipStream_t)stream;
    ppmlr_status e = mlp_grad_launch(w, theta, X, ldx, Y, ldy, n, st);
    if (e) return e;
    const int np = ppmlr::mlp::kNPar + 1;
    hipLaunchKernelGGL(ppmlr::mlp::reduce_adam_kernel, dim3((np + 255) / 256), dim3(256), 0, st, w->d_partials,
                       (n + 63) / 64, (float *)nullptr, loss, theta, m, v, 1, t, lr, beta1, beta2, eps);
    return mlp_check(w, hipGetLastError(), "adam launch");
}

}  // extern "C"
