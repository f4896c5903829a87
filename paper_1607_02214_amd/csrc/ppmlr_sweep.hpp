// ppmlr_sweep.hpp -- gfx950 device code of one dimensionally split PPMLR-MHD
// sweep (paper, Section II: zone-centred averages, parabolic distribution in
// each zone, characteristic edge values, Lagrangian update with an interface
// Riemann solve, remap onto the Eulerian grid; Section III-A: one independent
// 1D problem per pencil).
//
// Execution model: one thread per zone, a workgroup owns one tile of P
// pencil segments (L interior zones + 7 ghosts per side each; one segment =
// the whole pencil), and every stencil is served from LDS.  Successive stages
// exchange only what a neighbour needs, through two LDS buffers (A, B) with
// one barrier per exchange:
//   R1 load + primitives                                  -> A
//   R2 limited slopes (mass coordinate), shock test   A -> B
//      edge values                                   A, B -> A (slots 9..15)
//   R3 parabolas, tracing, interface states       A, B -> A
//   R4 Riemann solves, Lagrangian fluxes              A -> B
//   R5 Lagrangian zone contents                       B -> A
//   R6 limited slopes (volume coordinate)             A -> B
//      remap edge values                           A, B -> A (slots 8..14)
//   R7 remap parabolas, donor-cell fluxes             A -> A
//   R8 conservative update, sources, store            A
// The pencil axis is a template parameter so that all component indexing is
// static (no private arrays with dynamic indices).
#pragma once
#include "ppmlr_char.hpp"
#include "ppmlr_mlp.hpp"
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppmlr {

constexpr int kG = 7;           // ghost zones per side
constexpr int kSlotsA = 16;     // values per zone in LDS buffer A
constexpr int kSlotsAGuess = 19;  // buffer A of the learned / harvest sweeps (3 more face values)
constexpr int kSlotsB = 8;       // values per zone in LDS buffer B
// The signal-speed maximum is accumulated in kCflSlots words kCflStride
// words apart (workgroup b uses slot b mod kCflSlots), so that the
// workgroups' atomics do not all queue on one address; readers take the
// maximum of the slots.
constexpr int kCflSlots = 64;
constexpr int kCflStride = 32;
constexpr int kStatWords = 37;  // iteration histogram [32], floors, nonconverged, nonphys,
                                // learned-guess faces, learned-guess fallbacks
constexpr int kStatSlots = 64;  // copies of the counters (workgroup b adds to copy b % 64)

// Dynamic LDS of a sweep workgroup: the tile buffers A and B (slots values
// per zone, stride S) from address 0, then the workgroup's scalars: 16
// doubles of per-wave signal-speed maxima, the kStatWords counters, the
// learned guess's face count (or a persistent launch's barrier flag) and a
// persistent launch's tile claim.  With the buffers at address 0 a zone's LDS
// address is its lane offset, with the slot in the instruction's offset
// field; behind static shared arrays every address needed their size added.
constexpr int kLdsTail = 16 * 8 + (kStatWords + 2) * 4;
__host__ __device__ constexpr size_t lds_tile_bytes(int slots, int S, int elem)
{
    return ((size_t)slots * (size_t)S * (size_t)elem + 15) / 16 * 16;
}
__host__ __device__ constexpr size_t lds_bytes(int slots, int S, int elem)
{
    return lds_tile_bytes(slots, S, elem) + kLdsTail;
}

enum { kPeriodic = 0, kOutflow = 1, kInflow = 2 };

// Arithmetic helpers: FP64 uses Newton-refined reciprocals and reciprocal
// square roots and the IEEE square root, FP32 the hardware reciprocal /
// square-root approximations (1 ulp).
template <typename T> struct Ar;
// FP64: the hardware reciprocal and reciprocal square root refined by two
// Newton steps each (quadratic convergence: faithfully rounded results for
// the positive, finite arguments of the sweep), in place of the
// correctly rounded division sequence (~10 instructions each).
__device__ inline double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ inline double rsqrt64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double t = __builtin_fma(-h * y, y, 0.5);
    y = __builtin_fma(y, t, y);
    t = __builtin_fma(-h * y, y, 0.5);
    return __builtin_fma(y, t, y);
}
template <> struct Ar<double> {
    __device__ static inline double rcp(double x) { return rcp64(x); }
    __device__ static inline double div(double a, double b) { return a * rcp64(b); }
    __device__ static inline double sqrt_(double x) { return __builtin_sqrt(x); }
    __device__ static inline double rsqrt(double x) { return rsqrt64(x); }
};
template <> struct Ar<float> {
    __device__ static inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static inline float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    __device__ static inline float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    __device__ static inline float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
};

template <typename T> __device__ inline T tmin(T a, T b) { return a < b ? a : b; }
template <typename T> __device__ inline T tmax(T a, T b) { return a > b ? a : b; }
template <typename T> __device__ inline T tabs(T a) { return a < T(0) ? -a : a; }
// Element i of an array at a uniform base address, addressed by a 32-bit byte
// offset (every array the sweep reads is below 4 GiB), so that the load or
// store takes the scalar-base + vector-offset form.
template <typename T> __device__ inline T &elem(T *base, unsigned int i)
{
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + i * (unsigned int)sizeof(T));
}
template <typename T> __device__ inline const T &elem(const T *base, unsigned int i)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + i * (unsigned int)sizeof(T));
}
// IEEE min / |x| / copysign in the type's own precision (the unsuffixed
// builtins are the double versions and would convert FP32 operands)
__device__ inline float fmin_(float a, float b) { return __builtin_fminf(a, b); }
__device__ inline double fmin_(double a, double b) { return __builtin_fmin(a, b); }
__device__ inline float fmax_(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ inline double fmax_(double a, double b) { return __builtin_fmax(a, b); }
__device__ inline float fabs_(float a) { return __builtin_fabsf(a); }
__device__ inline double fabs_(double a) { return __builtin_fabs(a); }
__device__ inline float copysign_(float a, float b) { return __builtin_copysignf(a, b); }
__device__ inline double copysign_(double a, double b) { return __builtin_copysign(a, b); }
template <typename T> __device__ inline T tsgn(T a) { return a > T(0) ? T(1) : (a < T(0) ? T(-1) : T(0)); }

template <typename T>
struct SweepArgs {
    T *u;                       // state, SoA [8][nz][ny][nx]
    long long vol;              // zones per variable
    int N, M;                   // zones along the pencil; zones of one tile's segment, L + 2G
    int L, nseg;                // interior zones per segment (the last may be shorter), segments per pencil
    int Mext;                   // N + 2G: extent of the geometry tables along the pencil
    int P;                      // pencils per workgroup
    int S;                      // LDS slots = P * M
    long long stride_n, stride_q, stride_r;   // element strides
    float inv_div;              // 1 / M (x sweep) or 1 / P (y, z): lane -> (pencil, zone)
    const T *vin[8];            // base of each conserved variable of the input state
    T *var[8];                  // ... and of the output state (the same when whole pencils are swept in place)
    int nq, nr;                 // pencils along q (memory-fastest transverse) and r
    int tiles_q, ntiles, tiles_per_xcd;   // ntiles: tiles of one segment band (tiles_q * nr)
    int nslots;                 // tiles of one segment band: tiles_q * nr
    int seg_fast;               // 1: consecutive tiles are the segments of one pencil group; 0: bands in turn
    const T *dx, *xc, *xf;      // sweep axis: extended widths [Mext], centres [Mext], faces [Mext+1]
    const T *xc_q, *xc_r;       // transverse centres (interior zones)
    const T *dx_q, *dx_r;       // transverse widths (interior zones)
    int bc_lo, bc_hi;
    T gamma;
    T dt;                       // used when dt_dev == nullptr
    const double *dt_dev;       // device-resident dt (advance loop)
    int has_bd;                 // background field present
    T dip_m, dir_x, dir_y, dir_z, bext_x, bext_y, bext_z;
    T in_rho, in_vx, in_vy, in_vz, in_bx, in_by, in_bz, in_p;   // inflow (total B)
    const double *in_dev;       // inflow of this step on the device (time series) or nullptr
    T r_inner2, inner_rho, inner_E;
    int has_inner;
    const double *inner_v;      // drift of the reset zones [3][box] (ionosphere coupling) or nullptr: at rest
    int ib[6];                  // its index box i0, i1, j0, j1, k0, k1 (half-open)
    int flatten, janhunen, max_iter;
    T tol, p_floor;
    unsigned long long *stats;  // kStatSlots x kStatWords counters or nullptr
    unsigned long long *cfl_max;// fused signal-speed max (double bits, kCflSlots slots) or nullptr
    const T *dxw_x, *dxw_y, *dxw_z;       // interior widths of all axes (fused CFL)
    // learned Riemann guess (FP32 single-run sweeps)
    const unsigned short *mlp_frag;       // packed BF16 weight fragments
    const float *mlp_theta;               // FP32 parameters (biases)
    T gate_p, gate_u;                     // relative pressure / velocity jump that selects a face
    float *harvest;                       // [harvest_cap][28] interface records or nullptr
    long long harvest_cap;
    unsigned long long *harvest_count;    // records offered (may exceed the capacity)
};

// Riemann initial-guess modes of the sweep body
enum { kGuessPlain = 0, kGuessLearned = 1, kGuessHarvest = 2 };

// Background field B_d = M [3 (m.r) r / r^5 - m / r^3] + b_ext at (x, y, z).
template <typename T>
__device__ inline void background(const SweepArgs<T> &a, T x, T y, T z, T &bx, T &by, T &bz)
{
    bx = a.bext_x;
    by = a.bext_y;
    bz = a.bext_z;
    if (a.dip_m != T(0)) {
        T r2 = x * x + y * y + z * z;
        T ir = Ar<T>::rsqrt(r2);
        T ir2 = ir * ir;
        T ir3 = ir2 * ir;
        T ir5 = ir3 * ir2;
        T mr = a.dir_x * x + a.dir_y * y + a.dir_z * z;
        T c = T(3) * mr * ir5;
        bx += a.dip_m * (c * x - a.dir_x * ir3);
        by += a.dip_m * (c * y - a.dir_y * ir3);
        bz += a.dip_m * (c * z - a.dir_z * ir3);
    }
}

// Map pencil-frame coordinates (n, t1, t2) of axis AX to (x, y, z) and the
// field back; t1, t2 are the cyclic successors of the sweep axis.
template <int AX, typename T>
__device__ inline void to_xyz(T n, T t1, T t2, T &x, T &y, T &z)
{
    if (AX == 0) { x = n; y = t1; z = t2; }
    else if (AX == 1) { y = n; z = t1; x = t2; }
    else { z = n; x = t1; y = t2; }
}
template <int AX, typename T>
__device__ inline void to_pencil(T bx, T by, T bz, T &bn, T &b1, T &b2)
{
    if (AX == 0) { bn = bx; b1 = by; b2 = bz; }
    else if (AX == 1) { bn = by; b1 = bz; b2 = bx; }
    else { bn = bz; b1 = bx; b2 = by; }
}
template <int AX, typename T>
__device__ inline void field_at(const SweepArgs<T> &a, T n, T c1, T c2, T &bn, T &b1, T &b2)
{
    T x, y, z, bx, by, bz;
    to_xyz<AX>(n, c1, c2, x, y, z);
    background(a, x, y, z, bx, by, bz);
    to_pencil<AX>(bx, by, bz, bn, b1, b2);
}

// Edge value a_{j+1/2} on nonuniform widths w0..w3 = w_{j-1..j+2}
// (Colella & Woodward 1984, Eq. 1.6) from the (limited) slopes of zones j
// and j+1.  The width weights are shared by all variables of a face and
// folded into three coefficients: a_j + E0 (a_{j+1} - a_j) + E2 da_{j+1} + E3 da_j.
template <typename T>
struct EdgeW {
    T E0, E2, E3;
    __device__ inline void init(T w0, T w1, T w2, T w3)
    {
        T i12 = Ar<T>::rcp(w1 + w2);
        T id1 = Ar<T>::rcp(T(2) * w1 + w2);
        T id2 = Ar<T>::rcp(w1 + T(2) * w2);
        T inv4 = Ar<T>::rcp(w0 + w1 + w2 + w3);
        T t1 = T(2) * w2 * w1 * i12 * ((w0 + w1) * id1 - (w3 + w2) * id2);
        E0 = w1 * i12 + t1 * inv4;
        E2 = -w1 * (w0 + w1) * id1 * inv4;
        E3 = w2 * (w2 + w3) * id2 * inv4;
    }
    __device__ inline T edge(T aj, T ajp, T daj, T dajp) const
    {
        return aj + E0 * (ajp - aj) + E2 * dajp + E3 * daj;
    }
};

// Median of three.
__device__ inline float med3_(float x, float y, float z) { return __builtin_amdgcn_fmed3f(x, y, z); }
__device__ inline double med3_(double x, double y, double z)
{
    return fmax_(fmin_(x, y), fmin_(fmax_(x, y), z));
}

// Eq. 1.8 limiter: sgn(da) min(|da|, 2|dm|, 2|dp|) where dm and dp share a
// sign, else zero.  When they share a sign da shares it too (the weights of
// Eq. 1.7 are positive).  In single precision this is two medians: med(dm,
// dp, 0) is the one-sided difference nearer zero when the signs agree and
// zero otherwise, and med(da, 2 med(dm, dp, 0), 0) clips da to it.
__device__ inline float limit_slope(float da, float dm, float dp)
{
    const float mm = med3_(dm, dp, 0.0f);
    return med3_(da, mm + mm, 0.0f);
}
__device__ inline double limit_slope(double da, double dm, double dp)
{
    double m = fmin_(fmin_(fabs_(0.5 * da), fabs_(dm)), fabs_(dp));
    double r = copysign_(m + m, dp);
    return (dp * dm > 0.0) ? r : 0.0;
}

// Average slope times width in zone j on widths wm, w0, wp (CW84 Eq. 1.7),
// da = A (a_{j+1} - a_j) + B (a_j - a_{j-1}), limited by Eq. 1.8.
template <typename T>
struct SlopeW {
    T A, B;
    __device__ inline void init(T wm, T w0, T wp)
    {
        T cs = w0 * Ar<T>::rcp(wm + w0 + wp);
        A = cs * (T(2) * wm + w0) * Ar<T>::rcp(wp + w0);
        B = cs * (w0 + T(2) * wp) * Ar<T>::rcp(wm + w0);
    }
    __device__ inline T slope(T am, T a0, T ap) const
    {
        T dp = ap - a0;
        T dm = a0 - am;
        return limit_slope(A * dp + B * dm, dm, dp);
    }
};

// Domain-of-dependence fraction y with its two shared coefficients.
template <typename T>
struct Frac {
    T h, c;   // y/2 and 1 - 2y/3
    __device__ inline explicit Frac(T y) : h(T(0.5) * y), c(T(1) - (T(2) / T(3)) * y) {}
};

// Flattening toward the zone average, then CW84 Eq. 1.10 monotonicity.  At a
// local extremum both edges take the zone average; otherwise the edge on the
// far side of an overshooting parabola is moved to 3a - 2a_other.  Both rules
// are one median each: for a monotone profile (say a_L < a < a_R) the
// overshoot test a6 > dA reads a_L < 3a - 2a_R, so the new left edge is
// max(a_L, 3a - 2a_R) = med(a_L, 3a - 2a_R, a) (a is the largest of the
// three); at an extremum 3a - 2a_R lies beyond a on the far side from a_L, so
// the median is a.  Likewise on the right with a_L and a_R exchanged.
template <typename T>
__device__ inline void parabola(T a, T aL, T aR, T f, T &oL, T &oD, T &o6)
{
    aL = aL + f * (a - aL);
    aR = aR + f * (a - aR);
    const T a3 = T(3) * a;
    const T nL = med3_(aL, a3 - T(2) * aR, a);
    const T nR = med3_(aR, a3 - T(2) * aL, a);
    oL = nL;
    oD = nR - nL;
    o6 = T(6) * (a - T(0.5) * (nL + nR));
}

// Averages of a zone parabola over the fraction y next to its right edge
// (avgR) or left edge (avgL) (CW84 Eq. 1.12).
template <typename T>
__device__ inline T avgR(T aL, T dA, T a6, const Frac<T> &f)
{
    return (aL + dA) - f.h * (dA - f.c * a6);
}
template <typename T>
__device__ inline T avgL(T aL, T dA, T a6, const Frac<T> &f)
{
    return aL + f.h * (dA + f.c * a6);
}

// Counter update aggregated per wave: the lowest active lane of each group of
// lanes with the same bin adds the group's population to the workgroup's LDS
// counters (flushed to global memory once per workgroup).
__device__ inline void wave_add(unsigned int *s_ctr, bool pred)
{
    unsigned long long m = __ballot(pred);
    if (m != 0ull && __lane_id() == __ffsll((long long)m) - 1) atomicAdd(s_ctr, (unsigned int)__popcll(m));
}
__device__ inline void wave_hist(unsigned int *s_hist, bool counted, int bin)
{
    // bin 0 (a face whose linear guess already meets the tolerance) is by far
    // the most common: one ballot for it, then a loop over the other bins
    const unsigned long long zero = __ballot(counted && bin == 0);
    if (zero != 0ull && __lane_id() == __ffsll((long long)zero) - 1)
        atomicAdd(&s_hist[0], (unsigned int)__popcll(zero));
    unsigned long long active = __ballot(counted && bin != 0);
    while (active) {
        int leader = __ffsll((long long)active) - 1;
        int lb = __shfl(bin, leader);
        unsigned long long same = __ballot(counted && bin == lb);
        if (__lane_id() == leader) atomicAdd(&s_hist[lb], (unsigned int)__popcll(same));
        active &= ~same;
    }
}

// Inputs of the learned guess for one face (see the Riemann block of
// sweep_tile): sides s = (rho, u, v_t1, v_t2, B_t1, B_t2, P), normalised by
// the pair means.  Returns whether the face is selected (strong pressure or
// velocity jump); Pbar and cbar are the mean pressure and sqrt(P/rho).
template <typename T>
__device__ inline bool guess_features(const T *L, const T *R, T gate_p, T gate_u, T *feat, T &Pbar, T &cbar)
{
    const T rbar = T(0.5) * (L[0] + R[0]);
    Pbar = T(0.5) * (L[6] + R[6]);
    const T irb = Ar<T>::rcp(rbar), iPb = Ar<T>::rcp(Pbar);
    cbar = Ar<T>::sqrt_(Pbar * irb);
    const T icb = Ar<T>::rcp(cbar), ibs = Ar<T>::rsqrt(Pbar);
    const T ub = T(0.5) * (L[1] + R[1]), v1b = T(0.5) * (L[2] + R[2]), v2b = T(0.5) * (L[3] + R[3]);
    const T *side[2] = {L, R};
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
        const T *x = side[sd];
        T *f = feat + 7 * sd;
        f[0] = x[0] * irb;
        f[1] = (x[1] - ub) * icb;
        f[2] = (x[2] - v1b) * icb;
        f[3] = (x[3] - v2b) * icb;
        f[4] = x[4] * ibs;
        f[5] = x[5] * ibs;
        f[6] = x[6] * iPb;
    }
    return tabs(R[6] - L[6]) > gate_p * tmin(L[6], R[6]) || tabs(R[1] - L[1]) > gate_u * cbar;
}

// One tile of a sweep, executed by one workgroup: P pencils, each cut to
// segment `seg` (interior zones seg*L .. seg*L + L - 1 with G zones on either
// side; one segment = the whole pencil).  A zone's result depends on the
// zones within G of it only, so segments give the whole-pencil result
// bit for bit; neighbour reads are clamped at the ends of the pencil's
// extended range, as for a whole pencil.  tq, r: tile position (q tiles of P
// pencils, r the slow transverse index).  The state is read through a.vin
// and written through a.var: the same buffer for whole pencils, different
// buffers for segments (a segment's ghost zones are other segments' interior
// zones).  dt: the time step; cfl_max: target
// of the fused signal-speed maximum (FUSE_CFL); stat_slot: which copy of the
// counters this workgroup adds to.
// SM: LDS stride per stored value (a power of two >= P*M, so that every LDS
// access uses an immediate offset), or 0 for a runtime stride P*M.
// GUESS: initial guess of the normal-pair Newton iteration: the plain linear
// guess, the learned (MLP) guess on selected faces, or the plain guess with
// the selected faces' states and solutions recorded for training.  s_guess:
// one LDS counter (learned mode).
// Margin of the shock detector's compression test, in sound speeds
// sqrt(P / rho): no shock compresses by less, and a strict u_{j-1} > u_{j+1}
// at a pressure jump at rest would let rounding noise decide flattening.
constexpr double kCompMin = 1e-5;

template <int AX, typename T, bool STATS, bool FUSE_CFL, int SM, int GUESS = kGuessPlain, bool TRACE = false>
__device__ __forceinline__ void sweep_tile(const SweepArgs<T> &a, const int tq, const int r, const int seg, const T dt,
                                           unsigned long long *cfl_max, const int stat_slot,
                                           unsigned char *smem_raw, double *s_red, unsigned int *s_stat,
                                           unsigned int *s_guess = nullptr)
{
    static_assert(GUESS == kGuessPlain || (SM > 0 && sizeof(T) == 4 && STATS),
                  "learned / harvest modes are FP32 sweeps with a compile-time stride and counters");
    static_assert(!TRACE || GUESS == kGuessPlain, "the characteristic mode takes the plain interface solve");
    const int S = SM > 0 ? SM : a.S;                      // LDS stride
    T *sA = reinterpret_cast<T *>(smem_raw);
    T *sB = sA + (GUESS == kGuessPlain ? kSlotsA : kSlotsAGuess) * S;
    const int q0 = tq * a.P;

    const int tid = threadIdx.x;
    if (STATS && tid < kStatWords) s_stat[tid] = 0u;   // ordered by the first barrier
    if (GUESS == kGuessLearned && tid == 0) s_guess[0] = 0u;
    const int Suse = a.S, M = a.M, N = a.N, P = a.P;
    const bool slot_ok = tid < Suse;
    int p, i;
    // tid / divisor as floor((tid + 1/2) * (1/divisor)): exact for tid < 2^12
    // and divisors up to 2^11 (the distance to the next integer, >= 1/(2 div),
    // exceeds the rounding error, < tid * 2^-23 / div)
    const int qd = (int)(((float)tid + 0.5f) * a.inv_div);
    if (AX == 0) { p = qd; i = tid - p * M; }             // zones of a pencil adjacent
    else { i = qd; p = tid - i * P; }                     // pencils adjacent (coalesced)
    const int d = (AX == 0) ? 1 : P;                      // slot offset of zone i+1
    const int q = q0 + p;
    const int g0 = seg * a.L;                             // first interior zone of the segment
    const int ie = g0 + i;                                // index into the extended tables
    const int Mext = a.Mext;
    const bool pen = slot_ok && q < a.nq && ie < Mext;
    const int g = ie - kG;                                // zone index along the pencil
    const int gend = min(g0 + a.L, N);                    // end of the segment's interior
    const bool interior = pen && g >= g0 && g < gend;
    const int tsafe = slot_ok ? tid : Suse - 1;           // padding lanes read a valid slot
    auto nb = [&](int k) -> int {                         // slot of zone i+k (clamped)
        int ii = i + k;
        return (ii >= 0 && ii < M && ie + k >= 0 && ie + k < Mext && slot_ok) ? tid + k * d : tsafe;
    };
    // faces owned by this segment (counted and recorded once per pencil):
    // -1/2 .. N-1/2 over all segments
    const int own_lo = seg == 0 ? -1 : g0;
    const T gam = a.gamma;

    // transverse coordinates of the pencil
    const int qq = q < a.nq ? q : a.nq - 1;
    int j1, j2;
    T c1, c2;
    // q is t1 for the x and z sweeps, t2 for the y sweep
    if (AX == 1) { j1 = r; j2 = qq; c1 = elem(a.xc_r, r); c2 = elem(a.xc_q, qq); }
    else { j1 = qq; j2 = r; c1 = elem(a.xc_q, qq); c2 = elem(a.xc_r, r); }
    (void)j1; (void)j2;
    // 32-bit element offsets within one variable (the host keeps a variable
    // below 4 GiB); each variable's base pointer is uniform
    const unsigned int base = (unsigned int)(qq * (int)a.stride_q + r * (int)a.stride_r);

    // ------------------------------------------------------------ R1
    const int ic = ie < Mext ? ie : Mext - 1;
    const T dxi = elem(a.dx, ic);
    const T xci = elem(a.xc, ic);
    const T xfr = elem(a.xf, ic + 1);
    int src = g;
    bool inflow_zone = false;
    if (g < 0) {
        if (a.bc_lo == kPeriodic) { src = g % N; if (src < 0) src += N; }
        else if (a.bc_lo == kOutflow) src = 0;
        else inflow_zone = true;
    } else if (g >= N) {
        if (a.bc_hi == kPeriodic) src = g % N;
        else if (a.bc_hi == kOutflow) src = N - 1;
        else inflow_zone = true;
    }
    // centre and right-face background field (pencil frame)
    T bdn = 0, bd1 = 0, bd2 = 0, bfn = 0, bf1 = 0, bf2 = 0;
    if (a.has_bd) {
        field_at<AX>(a, xci, c1, c2, bdn, bd1, bd2);
        field_at<AX>(a, xfr, c1, c2, bfn, bf1, bf2);
    }
    // conserved state in pencil frame: rho, mn, m1, m2, bn, b1, b2, E
    T Q[8];
    constexpr int kn = AX, k1 = (AX + 1) % 3, k2 = (AX + 2) % 3;
    if (pen && !inflow_zone) {
        const unsigned int o = base + (unsigned int)(src * (int)a.stride_n);
        Q[0] = elem(a.vin[0], o);
        Q[1] = elem(a.vin[1 + kn], o);
        Q[2] = elem(a.vin[1 + k1], o);
        Q[3] = elem(a.vin[1 + k2], o);
        Q[4] = elem(a.vin[4 + kn], o);
        Q[5] = elem(a.vin[4 + k1], o);
        Q[6] = elem(a.vin[4 + k2], o);
        Q[7] = elem(a.vin[7], o);
    } else if (pen) {
        // inflow ghost: primitive inflow state with B' = B_in - B_d(centre)
        // (a time series of inflow states puts this step's in a.in_dev)
        T in[8] = {a.in_rho, a.in_vx, a.in_vy, a.in_vz, a.in_bx, a.in_by, a.in_bz, a.in_p};
        if (a.in_dev) {
#pragma unroll
            for (int k = 0; k < 8; ++k) in[k] = (T)a.in_dev[k];
        }
        T vn, v1, v2, Bn, B1, B2;
        to_pencil<AX>(in[1], in[2], in[3], vn, v1, v2);
        to_pencil<AX>(in[4], in[5], in[6], Bn, B1, B2);
        T pbn = Bn - bdn, pb1 = B1 - bd1, pb2 = B2 - bd2;
        Q[0] = in[0];
        Q[1] = in[0] * vn;
        Q[2] = in[0] * v1;
        Q[3] = in[0] * v2;
        Q[4] = pbn;
        Q[5] = pb1;
        Q[6] = pb2;
        Q[7] = in[7] / (gam - T(1)) + T(0.5) * in[0] * (vn * vn + v1 * v1 + v2 * v2) +
               T(0.5) * (pbn * pbn + pb1 * pb1 + pb2 * pb2);
    } else {
        Q[0] = T(1); Q[1] = Q[2] = Q[3] = T(0); Q[4] = Q[5] = Q[6] = T(0); Q[7] = T(1);
    }
    const T rho = Q[0];
    const T irho = Ar<T>::rcp(rho);
    const T un = Q[1] * irho, v1 = Q[2] * irho, v2 = Q[3] * irho;
    const T bn = Q[4], b1 = Q[5], b2 = Q[6];
    T pth = (gam - T(1)) * (Q[7] - T(0.5) * rho * (un * un + v1 * v1 + v2 * v2) -
                            T(0.5) * (bn * bn + b1 * b1 + b2 * b2));
    const bool floored = pth < a.p_floor;
    if (floored) pth = a.p_floor;
    const T dm = rho * dxi;
    const T Pt = pth + bd1 * b1 + bd2 * b2 + T(0.5) * (b1 * b1 + b2 * b2);
    const T Pa = Pt + T(0.5) * (bd1 * bd1 + bd2 * bd2);
    const bool cnt_floor = interior && floored;
    const bool cnt_bad = interior && (!(rho > T(0)) || !__builtin_isfinite(rho) || !__builtin_isfinite(Q[7]));
    // primitive set used for reconstruction: rho, u, v1, v2, b1, b2, p
    const T W[7] = {rho, un, v1, v2, b1, b2, pth};
    if (slot_ok) {
#pragma unroll
        for (int k = 0; k < 7; ++k) sA[k * S + tid] = W[k];
        sA[7 * S + tid] = dm;
        sA[8 * S + tid] = bn;
        sA[9 * S + tid] = Pt;
        sA[10 * S + tid] = Pa;
        sA[11 * S + tid] = bfn;
        sA[12 * S + tid] = bf1;
        sA[13 * S + tid] = bf2;
    }
    __syncthreads();

    // ------------------------------------------------------------ R2
    const int sm1 = nb(-1), sp1 = nb(1), sp2 = nb(2), sm2 = nb(-2);
    const T dmm = sA[7 * S + sm1], dmp = sA[7 * S + sp1], dmp2 = sA[7 * S + sp2];
    const T bnm = sA[8 * S + sm1], bnp = sA[8 * S + sp1];
    const T bln = sA[11 * S + sm1], bl1 = sA[12 * S + sm1], bl2 = sA[13 * S + sm1];  // left face
    const T Ptm = sA[9 * S + sm1], Ptp = sA[9 * S + sp1];
    // Each zone limits its own slopes (CW84 Eq. 1.7-1.8) and hands them to
    // the zone on its left through buffer B; the right-edge value then needs
    // the neighbour's slope only.  The edges go to buffer A, slots 9..15
    // (the face values of R1 there have been read by then).
    T edgeR[7];
    T ftil = T(0);
    {
        SlopeW<T> s0;
        s0.init(dmm, dm, dmp);
        EdgeW<T> ew;
        ew.init(dmm, dm, dmp, dmp2);
        T da0[7], apv[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const T am = sA[k * S + sm1];
            apv[k] = sA[k * S + sp1];
            da0[k] = s0.slope(am, W[k], apv[k]);
        }
        if (a.flatten) {
            T Ptm2 = sA[9 * S + sm2], Ptp2 = sA[9 * S + sp2];
            T Pam = sA[10 * S + sm1], Pap = sA[10 * S + sp1];
            T um = sA[1 * S + sm1], up = sA[1 * S + sp1];
            T d1 = Ptp - Ptm, d2 = Ptp2 - Ptm2;
            // compression with a margin of kCompMin sound speeds
            // sqrt(P_min / rho), so that equal velocities (a pressure jump at
            // rest) and rounding noise about them never flatten
            const T pmin = tmin(Pap, Pam), du = um - up;
            if (tabs(d1) > T(0.33) * pmin && du > T(0) && du * du * rho > T(kCompMin * kCompMin) * pmin) {
                if (d2 != T(0)) ftil = tmax(T(0), tmin(T(1), T(10) * (Ar<T>::div(d1, d2) - T(0.75))));
                else ftil = T(1);
            }
        }
        if (slot_ok) {
#pragma unroll
            for (int k = 0; k < 7; ++k) sB[k * S + tid] = da0[k];
            sB[7 * S + tid] = ftil;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 7; ++k) edgeR[k] = ew.edge(W[k], apv[k], da0[k], sB[k * S + sp1]);
    }
    if (slot_ok) {
#pragma unroll
        for (int k = 0; k < 7; ++k) sA[(9 + k) * S + tid] = edgeR[k];
    }
    __syncthreads();

    // ------------------------------------------------------------ R3
    T fl = T(0);
    if (a.flatten) {
        T fm = sB[7 * S + sm1], fp = sB[7 * S + sp1];
        fl = tmax(ftil, (Ptp - Ptm < T(0)) ? fp : fm);
    }
    T pLc[7], pDc[7], p6c[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        T aL = sA[(9 + k) * S + sm1];
        parabola(W[k], aL, edgeR[k], fl, pLc[k], pDc[k], p6c[k]);
    }
    // tracing speeds (Lagrangian): normal pair C_n, Alfven pair C_A
    const T Bt1c = bd1 + b1, Bt2c = bd2 + b2, Bnc = bdn + bn;
    const T Cn = Ar<T>::sqrt_(rho * (gam * pth + Bt1c * Bt1c + Bt2c * Bt2c));
    const T CA = Ar<T>::sqrt_(rho) * tabs(Bnc);
    const T idm = Ar<T>::rcp(dm);
    const Frac<T> yn(tmin(T(1), Cn * dt * idm));
    const Frac<T> yA(tmin(T(1), CA * dt * idm));
    // time-centring of the couplings left out of the two decoupled Riemann
    // problems: oblique-field terms and the variation of B_n along the pencil
    const T hdt = T(0.5) * dt;
    const T dbn = (bnp - bnm) * Ar<T>::rcp(T(0.5) * dmm + dm + T(0.5) * dmp);
    const T ddn = (bfn - bln) * idm, dd1 = (bf1 - bl1) * idm, dd2 = (bf2 - bl2) * idm;
    const T dBn = ddn + dbn;
    // (the oblique-field terms are in the eigenvectors of the characteristic mode)
    T corrP = TRACE ? T(0) : hdt * rho * Bnc * (Bt1c * pDc[2] + Bt2c * pDc[3]) * idm;
    T corrB1 = TRACE ? T(0) : -hdt * rho * Bt1c * pDc[1] * idm;
    T corrB2 = TRACE ? T(0) : -hdt * rho * Bt2c * pDc[1] * idm;
    const T corrU = hdt * (Bnc * dbn + bn * ddn);
    const T corrV1 = hdt * (b1 * dBn + bd1 * dbn + bn * dd1);
    const T corrV2 = hdt * (b2 * dBn + bd2 * dbn + bn * dd2);
    corrB1 += hdt * rho * (v1 * dBn - un * dd1);
    corrB2 += hdt * rho * (v2 * dBn - un * dd2);
    corrP += hdt * rho * ((Bt1c * v1 + Bt2c * v2) * dBn - un * (Bt1c * dd1 + Bt2c * dd2));

    // Characteristic mode: the face states traced wave by wave.  The
    // reference is the zone's parabola averaged over the fast wave's domain
    // of dependence; the Alfven and slow waves moving into the face get their
    // own averages (difference projected on the left eigenvector, taken out
    // along the right one).  A traced state without positive density and
    // pressure falls back to the zone average.  The split multi-D terms are
    // added to u, v_t and B_t; the thermal pressure takes none (its
    // Lagrangian equation has no term in dB_n/dm: corrP is the magnetic-
    // pressure change B_t . corrB, which the corrected field carries into
    // the interface total pressure).  The right-face state stays in
    // registers, the left-face state goes to the zone on the left through
    // LDS (slots 0..6).
    T WLc[7];
    if constexpr (TRACE) {
        Waves7<T> wz;
        wz.template init<Ar<T>>(rho, pth, gam, Bnc, Bt1c, Bt2c);
        const T sp = rho * dt * idm;
        const Frac<T> yf(tmin(T(1), wz.cf * sp)), ya(tmin(T(1), wz.ca * sp)), ys(tmin(T(1), wz.cs * sp));
        const T corr[7] = {T(0), corrU, corrV1, corrV2, corrB1, corrB2, T(0)};
        T WRc[7];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const T dir = side == 0 ? T(1) : T(-1);
            T ref[7], DA[7], DS[7];
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                if (side == 0) {
                    ref[k] = avgR(pLc[k], pDc[k], p6c[k], yf);
                    DA[k] = ref[k] - avgR(pLc[k], pDc[k], p6c[k], ya);
                    DS[k] = ref[k] - avgR(pLc[k], pDc[k], p6c[k], ys);
                } else {
                    ref[k] = avgL(pLc[k], pDc[k], p6c[k], yf);
                    DA[k] = ref[k] - avgL(pLc[k], pDc[k], p6c[k], ya);
                    DS[k] = ref[k] - avgL(pLc[k], pDc[k], p6c[k], ys);
                }
            }
            T bfa, baa, bsa, bfs, bas, bss;
            wz.project(DA, dir, bfa, baa, bsa);
            wz.project(DS, dir, bfs, bas, bss);
            wz.add(ref, dir, T(0), wz.moves(wz.ca) ? -baa : T(0), wz.moves(wz.cs) ? -bss : T(0));
            const bool phys = ref[0] > T(0) && ref[6] > T(0);
            T *dst = side == 0 ? WLc : WRc;
#pragma unroll
            for (int k = 0; k < 7; ++k) dst[k] = (phys ? ref[k] : W[k]) + corr[k];
        }
        if (slot_ok) {
#pragma unroll
            for (int k = 0; k < 7; ++k) sA[k * S + tid] = WRc[k];
        }
    }

    // interface states of this zone: L at its right face (i+1/2), R at its
    // left face (i-1/2); normal pair traced with y_n, Alfven pair with y_A
    // right-face (L) state, kept in registers
    T LPt, Lu, LC, Lk, Lr, Lv1, Lv2, Lb1, Lb2;
    T LrN, LT1, LT2;      // normal-pair density and total transverse field (guess features)
    {
        T r_ = avgR(pLc[0], pDc[0], p6c[0], yn);
        T u_ = avgR(pLc[1], pDc[1], p6c[1], yn);
        T p_ = avgR(pLc[6], pDc[6], p6c[6], yn);
        T c1_ = avgR(pLc[4], pDc[4], p6c[4], yn);
        T c2_ = avgR(pLc[5], pDc[5], p6c[5], yn);
        T T1 = bf1 + c1_, T2 = bf2 + c2_;
        const T C2 = r_ * (gam * p_ + T1 * T1 + T2 * T2);
        T C = Ar<T>::sqrt_(C2);
        T P0 = p_ + T(0.5) * (T1 * T1 + T2 * T2);
        T Pd = T(0.5) * (bf1 * bf1 + bf2 * bf2);
        T Pt_ = p_ + bf1 * c1_ + bf2 * c2_ + T(0.5) * (c1_ * c1_ + c2_ * c2_) + corrP;
        if (Pt_ + Pd < T(0.5) * P0) Pt_ = T(0.5) * P0 - Pd;
        // k = (ge + 1) / (2 ge) with ge = C^2 / (rho P): 1/2 + rho P / (2 C^2)
        const T kh = T(0.5) * r_ * (Pt_ + Pd) * Ar<T>::rcp(C2) + T(0.5);
        LPt = Pt_;
        LrN = r_;
        LT1 = T1;
        LT2 = T2;
        Lu = u_ + corrU;
        LC = C;
        Lk = kh;
        Lr = Ar<T>::sqrt_(avgR(pLc[0], pDc[0], p6c[0], yA));
        Lv1 = avgR(pLc[2], pDc[2], p6c[2], yA) + corrV1;
        Lv2 = avgR(pLc[3], pDc[3], p6c[3], yA) + corrV2;
        Lb1 = avgR(pLc[4], pDc[4], p6c[4], yA) + corrB1;
        Lb2 = avgR(pLc[5], pDc[5], p6c[5], yA) + corrB2;
    }
    // left-face (R) state, handed to the zone on the left through LDS
    {
        T r_ = avgL(pLc[0], pDc[0], p6c[0], yn);
        T u_ = avgL(pLc[1], pDc[1], p6c[1], yn);
        T p_ = avgL(pLc[6], pDc[6], p6c[6], yn);
        T c1_ = avgL(pLc[4], pDc[4], p6c[4], yn);
        T c2_ = avgL(pLc[5], pDc[5], p6c[5], yn);
        T T1 = bl1 + c1_, T2 = bl2 + c2_;
        const T C2 = r_ * (gam * p_ + T1 * T1 + T2 * T2);
        T C = Ar<T>::sqrt_(C2);
        T P0 = p_ + T(0.5) * (T1 * T1 + T2 * T2);
        T Pd = T(0.5) * (bl1 * bl1 + bl2 * bl2);
        T Pt_ = p_ + bl1 * c1_ + bl2 * c2_ + T(0.5) * (c1_ * c1_ + c2_ * c2_) + corrP;
        if (Pt_ + Pd < T(0.5) * P0) Pt_ = T(0.5) * P0 - Pd;
        // k = (ge + 1) / (2 ge) with ge = C^2 / (rho P): 1/2 + rho P / (2 C^2)
        const T kh = T(0.5) * r_ * (Pt_ + Pd) * Ar<T>::rcp(C2) + T(0.5);
        if (!TRACE && slot_ok) {
            sA[0 * S + tid] = Pt_;
            sA[1 * S + tid] = u_ + corrU;
            sA[2 * S + tid] = C;
            sA[3 * S + tid] = kh;
            sA[4 * S + tid] = Ar<T>::sqrt_(avgL(pLc[0], pDc[0], p6c[0], yA));
            sA[5 * S + tid] = avgL(pLc[2], pDc[2], p6c[2], yA) + corrV1;
            sA[6 * S + tid] = avgL(pLc[3], pDc[3], p6c[3], yA) + corrV2;
            sA[7 * S + tid] = avgL(pLc[4], pDc[4], p6c[4], yA) + corrB1;
            sA[8 * S + tid] = avgL(pLc[5], pDc[5], p6c[5], yA) + corrB2;
            if (GUESS != kGuessPlain) {
                sA[16 * S + tid] = r_;
                sA[17 * S + tid] = T1;
                sA[18 * S + tid] = T2;
            }
        }
    }
    __syncthreads();

    // ------------------------------------------------------------ R4
    // face i+1/2 between this zone (L) and zone i+1 (R)
    const bool face_ok = pen && i >= 3 && i <= M - 5;
    // Learned guess: faces with a strong jump are compacted per workgroup into
    // buffer B (free until the fluxes are written) and run through the network
    // 64 at a time on the matrix cores.  This pass comes before the solver's
    // right states are loaded, so that they do not occupy registers next to
    // the network's; they are read again from LDS below.
    bool lg_gate = false, lg_have = false;   // selected; network output available
    T lg_y = T(0), lg_Pbar = T(1);
    if constexpr (GUESS == kGuessLearned) {
        constexpr int kCap = ((8 * SM * (int)sizeof(T)) / 40) / 64 * 64;
        const int lane = tid & 63;
        unsigned short *F = reinterpret_cast<unsigned short *>(sB);
        float *Yo = reinterpret_cast<float *>(F + kCap * 16);
        int slot = 0;
        {
            const T Pd_ = T(0.5) * (bf1 * bf1 + bf2 * bf2);
            const T Ls[7] = {LrN, Lu, Lv1, Lv2, LT1, LT2, LPt + Pd_};
            T Rs[7];
            if (face_ok) {
                Rs[0] = sA[16 * S + sp1]; Rs[1] = sA[1 * S + sp1]; Rs[2] = sA[5 * S + sp1];
                Rs[3] = sA[6 * S + sp1]; Rs[4] = sA[17 * S + sp1]; Rs[5] = sA[18 * S + sp1];
                Rs[6] = sA[0 * S + sp1] + Pd_;
            } else {
#pragma unroll
                for (int k = 0; k < 7; ++k) Rs[k] = Ls[k];
            }
            T feat[14], cbar_;
            lg_gate = face_ok && guess_features(Ls, Rs, a.gate_p, a.gate_u, feat, lg_Pbar, cbar_);
            const unsigned long long bal = __ballot(lg_gate);
            int base = 0;
            if (lane == 0 && bal) base = (int)atomicAdd(&s_guess[0], (unsigned int)__popcll(bal));
            base = __shfl(base, 0);
            slot = base + __popcll(bal & ((1ull << lane) - 1ull));
            if (lg_gate && slot < kCap) {
                unsigned int w[8];
#pragma unroll
                for (int k = 0; k < 7; ++k)
                    w[k] = (unsigned int)mlp::f2bf((float)feat[2 * k]) |
                           ((unsigned int)mlp::f2bf((float)feat[2 * k + 1]) << 16);
                w[7] = 0u;
                uint4 *dst = reinterpret_cast<uint4 *>(F + slot * 16);
                dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
                dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
            }
        }
        if (STATS) wave_add(&s_stat[35], lg_gate && g >= own_lo && g < gend);
        __syncthreads();
        const int nf = min((int)s_guess[0], kCap);
        for (int b0 = (tid >> 6) * 64; b0 < nf; b0 += (int)(blockDim.x >> 6) * 64)
            mlp::forward_wave(F + b0 * 16, a.mlp_frag, a.mlp_theta, Yo + b0 * 2, 2);
        __syncthreads();
        lg_have = lg_gate && slot < kCap;
        if (lg_have) lg_y = (T)Yo[slot * 2];
        __syncthreads();   // buffer B is written with the fluxes next
    }
    T RPt = sA[0 * S + sp1], Ru = sA[1 * S + sp1], RC = sA[2 * S + sp1], Rk = sA[3 * S + sp1];
    T Rr = sA[4 * S + sp1], Rv1 = sA[5 * S + sp1], Rv2 = sA[6 * S + sp1];
    T Rb1 = sA[7 * S + sp1], Rb2 = sA[8 * S + sp1];
    T RrN = LrN, RT1 = LT1, RT2 = LT2;
    if (GUESS == kGuessHarvest && face_ok) {
        RrN = sA[16 * S + sp1];
        RT1 = sA[17 * S + sp1];
        RT2 = sA[18 * S + sp1];
    }
    if (!face_ok) {  // keep unused lanes trivial (no Newton iterations)
        RPt = LPt; Ru = Lu; RC = LC; Rk = Lk; Rr = Lr; Rv1 = Lv1; Rv2 = Lv2; Rb1 = Lb1; Rb2 = Lb2;
    }
    T Pst, ust, v1s, b1s, v2s, b2s;
    const T bns = T(0.5) * (bn + bnp);
    const T Bns = bfn + bns;
    if constexpr (TRACE) {
        // characteristic mode: the interface problem in its linearisation about
        // the mean of the two traced states; the face state is the left state
        // plus the waves of negative Lagrangian speed
        T WRc[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) WRc[k] = face_ok ? sA[k * S + sp1] : WLc[k];
        Waves7<T> wf;
        wf.template init<Ar<T>>(T(0.5) * (WLc[0] + WRc[0]), T(0.5) * (WLc[6] + WRc[6]), gam, Bns,
                                bf1 + T(0.5) * (WLc[4] + WRc[4]), bf2 + T(0.5) * (WLc[5] + WRc[5]));
        T D[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) D[k] = WRc[k] - WLc[k];
        T cfw, caw, csw;
        wf.project(D, T(-1), cfw, caw, csw);
        T Ws[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) Ws[k] = WLc[k];
        wf.add(Ws, T(-1), wf.cf > T(0) ? cfw : T(0), wf.moves(wf.ca) ? caw : T(0), wf.moves(wf.cs) ? csw : T(0));
        ust = Ws[1];
        v1s = Ws[2];
        v2s = Ws[3];
        b1s = Ws[4];
        b2s = Ws[5];
        Pst = Ws[6] + bf1 * b1s + bf2 * b2s + T(0.5) * (b1s * b1s + b2s * b2s);
        if (STATS) {
            const bool counted = face_ok && g >= own_lo && g < gend;
            wave_add(&s_stat[0], counted);          // no iteration
            wave_add(&s_stat[32], cnt_floor);
            wave_add(&s_stat[34], cnt_bad);
        }
    } else {
    {
        const T Pd = T(0.5) * (bf1 * bf1 + bf2 * bf2);
        const T PL = LPt + Pd, PR = RPt + Pd;
        const T iPL = Ar<T>::rcp(PL), iPR = Ar<T>::rcp(PR);
        const T Pfloor = T(1e-6) * tmin(PL, PR) - Pd;
        const T tol = a.tol;
        T P = LPt + LC * ((RPt - LPt) + RC * (Lu - Ru)) * Ar<T>::rcp(LC + RC);
        P = tmax(P, Pfloor);
        const T P0 = P;
        // Faces with a strong jump are selected for the learned guess.  Its
        // 14 inputs: both sides' (rho, u, v_t1, v_t2, B_t1, B_t2, P) of the
        // normal-pair problem, normalised by the pair means (velocities
        // relative to the mean, scaled by c = sqrt(P/rho); fields by
        // sqrt(P)).  Outputs: (P* - P0) / P and (u* - u0) / c.
        bool gate = false;
        T feat[14], Pbar = T(1), cbar = T(1);
        if (GUESS == kGuessHarvest) {
            const T Ls[7] = {LrN, Lu, Lv1, Lv2, LT1, LT2, PL};
            const T Rs[7] = {RrN, Ru, Rv1, Rv2, RT1, RT2, PR};
            gate = face_ok && g >= own_lo && g < gend && guess_features(Ls, Rs, a.gate_p, a.gate_u, feat, Pbar, cbar);
            if (STATS) wave_add(&s_stat[35], gate);
        }
        if (GUESS == kGuessLearned) {
            bool used = false;
            if (lg_have) {
                const T Pg = P + lg_Pbar * lg_y;
                if (__builtin_isfinite(Pg) && Pg > Pfloor) {
                    P = Pg;
                    used = true;
                }
            }
            if (STATS) wave_add(&s_stat[36], lg_gate && !used && g >= own_lo && g < gend);
        }
        int it = 0;
        bool conv = true;
        // The velocity mismatch u*_R - u*_L is formed from differences
        // ((u_R - u_L) + jumps / W) rather than as the difference of the two
        // star velocities, so that a large bulk velocity does not bury it in
        // rounding (same quantity; matters in single precision at high Mach).
        const T duRL = Ru - Lu;
        // Shock impedances W_s = C_s sqrt(q_s), q_s = 1 + k_s (P - P_s) / P_s,
        // and Z_s = 2 W_s^3 / (W_s^2 + C_s^2), carried as 1/sqrt(q_s) and
        // 1/Z_s = (q_s + 1) / (2 C_s q_s^{3/2}): two reciprocal square roots
        // and one reciprocal per iteration.  Then dP = -mis Z_L Z_R / (Z_L + Z_R)
        // = -mis / (1/Z_L + 1/Z_R).
        const T kL = Lk * iPL, kR = Rk * iPR;
        const T iCL = Ar<T>::rcp(LC), iCR = Ar<T>::rcp(RC);
        T jL, gL, ig, dP, mis;
        for (;;) {
            const T qL = T(1) + kL * (P - LPt), qR = T(1) + kR * (P - RPt);
            const T sL = Ar<T>::rsqrt(qL), sR = Ar<T>::rsqrt(qR);
            jL = (P - LPt) * sL * iCL;
            mis = duRL + (P - RPt) * sR * iCR + jL;
            gL = T(0.5) * (qL + T(1)) * (sL * sL) * (sL * iCL);
            const T gR = T(0.5) * (qR + T(1)) * (sR * sR) * (sR * iCR);
            ig = Ar<T>::rcp(gL + gR);
            dP = -mis * ig;
            if (tabs(dP) <= tol * (P + Pd)) break;
            if (it >= a.max_iter) { conv = false; break; }
            P = tmax(P + dP, Pfloor);
            ++it;
        }
        Pst = tmax(P + dP, Pfloor);
        ust = (Lu - jL) + mis * gL * ig;
        if constexpr (GUESS == kGuessHarvest) {
            // record the selected faces: inputs, targets and the solver's own
            // scalars (for checks against an independent solver)
            const int lane = tid & 63;
            const unsigned long long bal = __ballot(gate);
            if (bal && a.harvest) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(a.harvest_count, (unsigned long long)__popcll(bal));
                base = __shfl(base, 0);
                const unsigned long long slot = base + (unsigned long long)__popcll(bal & ((1ull << lane) - 1ull));
                if (gate && slot < (unsigned long long)a.harvest_cap) {
                    float *rec = a.harvest + slot * mlp::kRecord;
                    const T u0 = (LC * Lu + RC * Ru - (RPt - LPt)) * Ar<T>::rcp(LC + RC);
#pragma unroll
                    for (int k = 0; k < 14; ++k) rec[k] = (float)feat[k];
                    rec[14] = (float)((Pst - P0) * Ar<T>::rcp(Pbar));
                    rec[15] = (float)((ust - u0) * Ar<T>::rcp(cbar));
                    rec[16] = (float)LPt; rec[17] = (float)RPt; rec[18] = (float)Pd;
                    rec[19] = (float)Lu;  rec[20] = (float)Ru;
                    rec[21] = (float)LC;  rec[22] = (float)RC;
                    rec[23] = (float)Lk;  rec[24] = (float)Rk;
                    rec[25] = (float)P0;  rec[26] = (float)Pst; rec[27] = (float)ust;
                }
            }
        }
        if (STATS) {
            // owned faces: iteration histogram and non-converged count; zone
            // counters of R1 (after the first barrier)
            const bool counted = face_ok && g >= own_lo && g < gend;
            wave_hist(s_stat, counted, it < 31 ? it : 31);
            wave_add(&s_stat[33], counted && !conv);
            wave_add(&s_stat[32], cnt_floor);
            wave_add(&s_stat[34], cnt_bad);
        }
    }
    // transverse pair: linear Alfven problem, increment form from the left
    const T sig = tsgn(Bns);
    const T irs = Ar<T>::rcp(Lr + Rr);
    v1s = Lv1 + (Rr * (Rv1 - Lv1) + sig * (Rb1 - Lb1)) * irs;
    b1s = Lb1 + (Lr * (Rb1 - Lb1) + sig * Lr * Rr * (Rv1 - Lv1)) * irs;
    v2s = Lv2 + (Rr * (Rv2 - Lv2) + sig * (Rb2 - Lb2)) * irs;
    b2s = Lb2 + (Lr * (Rb2 - Lb2) + sig * Lr * Rr * (Rv2 - Lv2)) * irs;
    }
    // Lagrangian fluxes in dipole + deviation flux form
    const T nn = bns * (bfn + T(0.5) * bns);
    const T Fpi = Pst - nn;
    const T Fv1 = -(Bns * b1s + bns * bf1);
    const T Fv2 = -(Bns * b2s + bns * bf2);
    const T Fb1 = ust * bf1 - Bns * v1s;
    const T Fb2 = ust * bf2 - Bns * v2s;
    const T Fe = ust * (Pst + nn) - Bns * (ust * bns + v1s * b1s + v2s * b2s);
    const T delR = ust * dt;
    if (slot_ok) {
        sB[0 * S + tid] = Fpi;
        sB[1 * S + tid] = Fv1;
        sB[2 * S + tid] = Fv2;
        sB[3 * S + tid] = Fb1;
        sB[4 * S + tid] = Fb2;
        sB[5 * S + tid] = Fe;
        sB[6 * S + tid] = delR;
    }
    __syncthreads();

    // ------------------------------------------------------------ R5
    // Lagrangian update of the zone contents (faces i-1/2, i+1/2)
    const T delL = sB[6 * S + sm1];
    T dC[7];
    dC[0] = T(0);
    dC[1] = -dt * (Fpi - sB[0 * S + sm1]);
    dC[2] = -dt * (Fv1 - sB[1 * S + sm1]);
    dC[3] = -dt * (Fv2 - sB[2 * S + sm1]);
    dC[4] = -dt * (Fb1 - sB[3 * S + sm1]);
    dC[5] = -dt * (Fb2 - sB[4 * S + sm1]);
    dC[6] = -dt * (Fe - sB[5 * S + sm1]);
    // remapped quantities per volume: rho, mn, m1, m2, b1, b2, E
    const T Qr[7] = {Q[0], Q[1], Q[2], Q[3], Q[5], Q[6], Q[7]};
    const T dd = delR - delL;
    const T dVL = dxi + dd;
    const T idVL = Ar<T>::rcp(dVL);
    T QL[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) QL[k] = Qr[k] + (dC[k] - Qr[k] * dd) * idVL;
    if (slot_ok) {
#pragma unroll
        for (int k = 0; k < 7; ++k) sA[k * S + tid] = QL[k];
        sA[7 * S + tid] = dVL;
    }
    __syncthreads();

    // ------------------------------------------------------------ R6
    // slopes shared through buffer B as in R2; edges to buffer A, slots 8..14
    T redgeR[7];
    {
        const T vm = sA[7 * S + sm1], vp = sA[7 * S + sp1], vp2 = sA[7 * S + sp2];
        SlopeW<T> s0;
        s0.init(vm, dVL, vp);
        EdgeW<T> ew;
        ew.init(vm, dVL, vp, vp2);
        T da0[7], apv[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const T am = sA[k * S + sm1];
            apv[k] = sA[k * S + sp1];
            da0[k] = s0.slope(am, QL[k], apv[k]);
        }
        if (slot_ok) {
#pragma unroll
            for (int k = 0; k < 7; ++k) sB[k * S + tid] = da0[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 7; ++k) redgeR[k] = ew.edge(QL[k], apv[k], da0[k], sB[k * S + sp1]);
    }
    if (slot_ok) {
#pragma unroll
        for (int k = 0; k < 7; ++k) sA[(8 + k) * S + tid] = redgeR[k];
    }
    __syncthreads();

    // ------------------------------------------------------------ R7
    // donor-cell remap fluxes: this zone gives its right part across face
    // i+1/2 when delta > 0 and its left part across i-1/2 when delta < 0
    {
        const bool zone_ok = pen && i >= 6 && i <= M - 7;
        const bool wr = zone_ok && delR >= T(0);
        const bool wl = zone_ok && delL < T(0) && i >= 1;
        const Frac<T> yR(delR * idVL), yL(-delL * idVL);
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            T aL = sA[(8 + k) * S + sm1];
            T cL, cD, c6;
            parabola(QL[k], aL, redgeR[k], fl, cL, cD, c6);
            if (wr) sA[k * S + tid] = delR * avgR(cL, cD, c6, yR);
            if (wl) sA[k * S + tid - d] = delL * avgL(cL, cD, c6, yL);
        }
    }
    __syncthreads();

    // ------------------------------------------------------------ R8
    // signal-speed maximum in the sweep's precision: a maximum selects one
    // value, so reducing in FP32 and converting the result gives the FP64
    // maximum of the converted values exactly
    T smax = T(0);
    if (interior) {
        T out[8];
        const T idx = Ar<T>::rcp(dxi);
        T nw[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) nw[k] = Qr[k] + (dC[k] + sA[k * S + sm1] - sA[k * S + tid]) * idx;
        T nbn = bn, nb1 = nw[4], nb2 = nw[5];
        if (a.janhunen) {
            // -v div B' source, split: n-derivative of B'_n, pre-sweep velocity
            const T xm = elem(a.xc, ie - 1), xp = elem(a.xc, ie + 1);
            const T divn = (bnp - bnm) * Ar<T>::rcp(xp - xm);
            nbn -= dt * un * divn;
            nb1 -= dt * v1 * divn;
            nb2 -= dt * v2 * divn;
        }
        out[0] = nw[0];
        out[1 + kn] = nw[1];
        out[1 + k1] = nw[2];
        out[1 + k2] = nw[3];
        out[4 + kn] = nbn;
        out[4 + k1] = nb1;
        out[4 + k2] = nb2;
        out[7] = nw[6];
        bool masked = false;
        if (a.has_inner) {
            T x, y, z;
            to_xyz<AX>(xci, c1, c2, x, y, z);
            if (x * x + y * y + z * z < a.r_inner2) {
                masked = true;
                // the inner state: rest, or the drift the ionosphere coupling set
                T vx = T(0), vy = T(0), vz = T(0);
                if (a.inner_v) {
                    int ix, iy, iz;
                    if (AX == 0) { ix = g; iy = j1; iz = j2; }
                    else if (AX == 1) { iy = g; iz = j1; ix = j2; }
                    else { iz = g; ix = j1; iy = j2; }
                    if (ix >= a.ib[0] && ix < a.ib[1] && iy >= a.ib[2] && iy < a.ib[3] && iz >= a.ib[4] &&
                        iz < a.ib[5]) {
                        const long long bi = a.ib[1] - a.ib[0], bj = a.ib[3] - a.ib[2];
                        const long long nb = bi * bj * (a.ib[5] - a.ib[4]);
                        const long long o = ((long long)(iz - a.ib[4]) * bj + (iy - a.ib[2])) * bi + (ix - a.ib[0]);
                        vx = (T)a.inner_v[o];
                        vy = (T)a.inner_v[nb + o];
                        vz = (T)a.inner_v[2 * nb + o];
                    }
                }
                out[0] = a.inner_rho;
                out[1] = a.inner_rho * vx;
                out[2] = a.inner_rho * vy;
                out[3] = a.inner_rho * vz;
                out[4] = out[5] = out[6] = T(0);
                out[7] = a.inner_E + T(0.5) * a.inner_rho * (vx * vx + vy * vy + vz * vz);
            }
        }
        const unsigned int o = base + (unsigned int)(g * (int)a.stride_n);
#pragma unroll
        for (int v = 0; v < 8; ++v) elem(a.var[v], o) = out[v];
        if (FUSE_CFL && cfl_max && !masked) {
            // signal speed of the updated zone, for the next step's dt (the
            // maximum is reduced in FP64)
            int ix, iy, iz;
            if (AX == 0) { ix = g; iy = j1; iz = j2; }
            else if (AX == 1) { iy = g; iz = j1; ix = j2; }
            else { iz = g; ix = j1; iy = j2; }
            const T r_ = out[0];
            const T ir = Ar<T>::rcp(r_);
            const T vx = out[1] * ir, vy = out[2] * ir, vz = out[3] * ir;
            const T px = out[4], py = out[5], pz = out[6];
            T p_ = (gam - T(1)) * (out[7] - T(0.5) * r_ * (vx * vx + vy * vy + vz * vz) -
                                   T(0.5) * (px * px + py * py + pz * pz));
            // fmax / fabs where they agree with the selects for every input
            // (a NaN p or discriminant gives the floor / zero either way);
            // the running maximum keeps its select, which passes a NaN on
            p_ = fmax_(p_, a.p_floor);
            T Bx = px, By = py, Bz = pz;
            if (a.has_bd) {
                // the zone-centre background field of R1, back from the pencil frame
                T bx, by, bz;
                to_xyz<AX>(bdn, bd1, bd2, bx, by, bz);
                Bx += bx; By += by; Bz += bz;
            }
            const T a2 = gam * p_ * ir;
            const T b2 = (Bx * Bx + By * By + Bz * Bz) * ir;
            const T s2 = a2 + b2;
            const T q4 = T(4) * a2 * ir;
            const T wx = elem(a.dxw_x, ix), wy = elem(a.dxw_y, iy), wz = elem(a.dxw_z, iz);
            T sp = T(0);
            {
                T disc = fmax_(s2 * s2 - q4 * Bx * Bx, T(0));
                T cf = Ar<T>::sqrt_(T(0.5) * (s2 + Ar<T>::sqrt_(disc)));
                sp = tmax(sp, (fabs_(vx) + cf) * Ar<T>::rcp(wx));
            }
            {
                T disc = fmax_(s2 * s2 - q4 * By * By, T(0));
                T cf = Ar<T>::sqrt_(T(0.5) * (s2 + Ar<T>::sqrt_(disc)));
                sp = tmax(sp, (fabs_(vy) + cf) * Ar<T>::rcp(wy));
            }
            {
                T disc = fmax_(s2 * s2 - q4 * Bz * Bz, T(0));
                T cf = Ar<T>::sqrt_(T(0.5) * (s2 + Ar<T>::sqrt_(disc)));
                sp = tmax(sp, (fabs_(vz) + cf) * Ar<T>::rcp(wz));
            }
            smax = sp;
        }
    }
    if (STATS) {
        __syncthreads();
        if (tid < kStatWords && s_stat[tid] != 0u && a.stats)
            atomicAdd(&a.stats[stat_slot * kStatWords + tid], (unsigned long long)s_stat[tid]);
    }
    if (FUSE_CFL && cfl_max) {
        // wave max (all lanes active), workgroup max, one atomic per workgroup
        // (no target: a sweep that is not the last of its step in a launch
        // that runs several)
        for (int off = 32; off > 0; off >>= 1) {
            T o = __shfl_xor(smax, off);
            smax = o > smax ? o : smax;
        }
        if (__lane_id() == 0) s_red[tid >> 6] = (double)smax;
        __syncthreads();
        if (tid == 0) {
            double m = 0.0;
            const int nw = (blockDim.x + 63) >> 6;
            for (int w = 0; w < nw; ++w) m = s_red[w] > m ? s_red[w] : m;
            atomicMax(cfl_max, (unsigned long long)__double_as_longlong(m));
        }
    }
}

// Standalone sweep: one workgroup per tile.  The learned-guess form holds
// the network pass next to the sweep's registers (~132 VGPRs, 3 waves per
// SIMD); a budget of 4 waves per SIMD (128 registers, a few bytes spilled
// in the fused form) makes it ~20 % faster (measured).
template <int AX, typename T, bool STATS, bool FUSE_CFL, int SM, int GUESS = kGuessPlain, bool TRACE = false>
__global__ void __launch_bounds__(SM > 0 ? SM : 1024)
    __attribute__((amdgpu_waves_per_eu(GUESS == kGuessLearned ? 4 : 1))) sweep_kernel(const SweepArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int kSlots = (GUESS == kGuessPlain ? kSlotsA : kSlotsAGuess) + kSlotsB;
    unsigned char *tail = smem_raw + lds_tile_bytes(kSlots, SM > 0 ? SM : a.S, (int)sizeof(T));
    double *s_red = reinterpret_cast<double *>(tail);
    unsigned int *s_stat = reinterpret_cast<unsigned int *>(tail + 16 * sizeof(double));
    unsigned int *s_guess = s_stat + kStatWords;
    // XCD-aware tile order: consecutive workgroups go to different XCDs
    // round-robin, so workgroups b, b+8, b+16, ... (one XCD) take consecutive
    // tiles (q fastest, then r) and share L2 lines of neighbouring pencils.
    // The segments of a pencil group are either consecutive in this order
    // (seg_fast) or the grid is dealt out one segment band after another.
    const int b = blockIdx.x;
    const int slot = (b & 7) * a.tiles_per_xcd + (b >> 3);
    if (slot >= a.nslots * a.nseg) return;
    int seg, tile;
    if (a.seg_fast) { seg = slot % a.nseg; tile = slot / a.nseg; }
    else { seg = slot / a.nslots; tile = slot - seg * a.nslots; }
    const int r = tile / a.tiles_q;
    const int tq = tile - r * a.tiles_q;
    const T dt = a.dt_dev ? T(*a.dt_dev) : a.dt;
    unsigned long long *cm = a.cfl_max ? a.cfl_max + (b % kCflSlots) * kCflStride : nullptr;
    sweep_tile<AX, T, STATS, FUSE_CFL, SM, GUESS, TRACE>(a, tq, r, seg, dt, cm, b % kStatSlots, smem_raw, s_red, s_stat,
                                                  s_guess);
}

// ---------------------------------------------------------------------------
// Batched ensemble sweep: one launch performs the same sweep (one axis) of
// every member of an ensemble of independent runs (different sizes, inflows
// and dt).  The tiles of all members are concatenated in member order
// (mo[m] = first tile of member m, mo[members] = total) and dealt out with the
// same XCD-aware order as the single-run kernel.  Each member's geometry, dt
// pointer, signal-speed slot and counters are in its own descriptor, so a
// member's arithmetic is exactly that of a single-run sweep with the same
// tiles (and segments: a segmented member reads one state and writes the
// other, as a single run does).  Successive sweeps are ordered by the launch boundaries: no
// workgroup waits on another.
template <typename T>
struct EnsembleSweepArgs {
    const SweepArgs<T> *desc;      // [members]: this axis's descriptor of each member
    const int *mo;                 // [members + 1]: tile offsets
    int members, total, per_xcd;
};

template <int AX, typename T, bool STATS, bool FUSE_CFL, int SM>
__global__ void __launch_bounds__(SM) ensemble_sweep_kernel(const EnsembleSweepArgs<T> e)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int b = blockIdx.x;
    const int j = (b & 7) * e.per_xcd + (b >> 3);
    if (j >= e.total) return;
    int lo = 0, hi = e.members - 1;               // largest m with mo[m] <= j
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (e.mo[mid] <= j) lo = mid; else hi = mid - 1;
    }
    const SweepArgs<T> &a = e.desc[lo];
    unsigned char *tail = smem_raw + lds_tile_bytes(kSlotsA + kSlotsB, SM, (int)sizeof(T));
    double *s_red = reinterpret_cast<double *>(tail);
    unsigned int *s_stat = reinterpret_cast<unsigned int *>(tail + 16 * sizeof(double));
    const int t = j - e.mo[lo];
    int seg, tt;                                  // as in the single-run order
    if (a.seg_fast) { seg = t % a.nseg; tt = t / a.nseg; }
    else { seg = t / a.ntiles; tt = t - seg * a.ntiles; }
    const int tq = tt % a.tiles_q;
    const int r = tt / a.tiles_q;
    const T dt = a.dt_dev ? T(*a.dt_dev) : a.dt;
    unsigned long long *cm = a.cfl_max ? a.cfl_max + (b % kCflSlots) * kCflStride : nullptr;
    sweep_tile<AX, T, STATS, FUSE_CFL, SM>(a, tq, r, seg, dt, cm, b % kStatSlots, smem_raw, s_red, s_stat);
}

}  // namespace ppmlr
