// ppmlr_char.hpp -- device helpers of the characteristic mode of the sweep:
// the seven waves of 1D ideal MHD in the mass coordinate, used to trace
// zone-edge values wave by wave and to solve the interface problem in its
// linearisation (paper, Section II: edge values by a characteristic method,
// a Lagrangian update with an interface Riemann solve).
//
// Primitive variables of a pencil: W = (rho, u, v_t1, v_t2, B_t1, B_t2, p).
// In the mass coordinate the system is dW/dt + A dW/dm = 0 with A = rho times
// the Eulerian primitive matrix without advection, so the waves are the
// Eulerian ones with Lagrangian speeds rho c: -fast, -Alfven, -slow,
// entropy (0), +slow, +Alfven, +fast.  The right eigenvectors take the
// normalisation of Roe & Balsara (1996): alpha_f, alpha_s weights, the unit
// vector beta along the transverse field and s = sgn(B_n) (sgn 0 = 1), which
// keeps them complete at every degeneracy.  The left eigenvectors are their
// closed-form inverse, written in the frame of beta (parallel component
// along beta, perpendicular along beta_perp = (-beta_2, beta_1)):
//   fast +-:   u +- af cf / 2Q,  v_par -+ s as cs / 2Q,  B_par as / (2 sqrt(rho) a),  p af / (2 rho a^2)
//   slow +-:   u +- as cs / 2Q,  v_par +- s af cf / 2Q,  B_par -af / (2 sqrt(rho) a), p as / (2 rho a^2)
//   Alfven +-: v_perp 1/2,       B_perp -+ s / (2 sqrt(rho))
// with Q = af^2 cf^2 + as^2 cs^2 (rho and the entropy direction do not enter).
#pragma once
#include <hip/hip_runtime.h>

namespace ppmlr {

// Where the normal field vanishes the Alfven and slow waves stop, and the
// traced face state jumps between the reference value (wave at rest) and the
// edge value (wave of speed 0+), with the Alfven family's eigenvector set by
// sgn(B_n).  A normal field that is zero in exact arithmetic (a background
// field cancelled by the deviation field) is rounding noise, so a wave slower
// than kWaveMin times the fast wave counts as at rest, in the tracing and in
// the interface problem: its domain of dependence is then below 1e-4 of the
// fast wave's, and no decision rests on the sign of noise.
constexpr double kWaveMin = 1e-4;

// The wave structure at one state (total field Bn, Bt1, Bt2).
template <typename T>
struct Waves7 {
    T cf, cs, ca;       // Eulerian fast, slow, Alfven speeds (Lagrangian speed = rho c)
    T af, as;           // Roe-Balsara weights
    T b1, b2;           // unit vector along the transverse field
    T sg;               // sgn(B_n), 1 for B_n = 0
    T sr, a, ra2;       // sqrt(rho), sound speed, rho a^2
    T iQ2;              // 1 / (2 Q)
    T ira, ira2;        // 1 / (2 sqrt(rho) a), 1 / (2 rho a^2)
    T isr2;             // 1 / (2 sqrt(rho))
    T rho;

    template <typename AR>
    __device__ __forceinline__ void init(T rho_, T p, T gam, T Bn, T Bt1, T Bt2)
    {
        rho = rho_;
        const T irho = AR::rcp(rho);
        const T a2 = gam * p * irho;
        const T bn2 = Bn * Bn * irho;
        const T btt = Bt1 * Bt1 + Bt2 * Bt2;
        const T bt2 = btt * irho;
        const T b2_ = bn2 + bt2;
        // c_f^2 - c_s^2 without cancellation (exact where bt = 0)
        const T dab = a2 - b2_;
        const T disc = AR::sqrt_(dab * dab + T(4) * a2 * bt2);
        const T cf2 = T(0.5) * (a2 + b2_ + disc);
        const T cs2 = cf2 > T(0) ? a2 * bn2 * AR::rcp(cf2) : T(0);    // c_f^2 c_s^2 = a^2 c_A^2
        cf = AR::sqrt_(cf2);
        cs = AR::sqrt_(cs2);
        ca = AR::sqrt_(bn2);
        a = AR::sqrt_(a2);
        if (disc > T(0)) {
            // the smaller weight as 2 a^2 bt^2 / (disc (disc + |a^2 - b^2|))
            T small = T(2) * a2 * bt2 * AR::rcp(disc * (disc + (dab < T(0) ? -dab : dab)));
            small = small < T(1) ? small : T(1);
            const T big = T(1) - small > T(0) ? T(1) - small : T(0);
            if (dab >= T(0)) { as = AR::sqrt_(small); af = AR::sqrt_(big); }
            else { af = AR::sqrt_(small); as = AR::sqrt_(big); }
        } else {
            af = T(1);
            as = T(0);
        }
        const T bt = AR::sqrt_(btt);
        if (bt > T(1e-12) * AR::sqrt_(rho * (a2 + b2_))) {
            const T ibt = AR::rcp(bt);
            b1 = Bt1 * ibt;
            b2 = Bt2 * ibt;
        } else {
            b1 = b2 = T(0.70710678118654752440);
        }
        sg = Bn < T(0) ? T(-1) : T(1);
        sr = AR::sqrt_(rho);
        ra2 = rho * a2;
        const T Q = af * af * cf2 + as * as * cs2;
        iQ2 = AR::rcp(T(2) * Q);
        ira = AR::rcp(T(2) * sr * a);
        ira2 = AR::rcp(T(2) * ra2);
        isr2 = AR::rcp(T(2) * sr);
    }
    // Whether a wave of Eulerian speed c (Alfven or slow) moves, in the sense
    // of kWaveMin.
    __device__ __forceinline__ bool moves(T c) const { return c > T(kWaveMin) * cf; }
    // Projections of a primitive difference D on the left eigenvectors of the
    // waves moving in direction dir (+1 or -1): fast, Alfven, slow.
    __device__ __forceinline__ void project(const T D[7], T dir, T &bf, T &ba, T &bs) const
    {
        const T vpar = b1 * D[2] + b2 * D[3], vper = -b2 * D[2] + b1 * D[3];
        const T Bpar = b1 * D[4] + b2 * D[5], Bper = -b2 * D[4] + b1 * D[5];
        bf = dir * (af * cf * D[1] - sg * as * cs * vpar) * iQ2 + as * ira * Bpar + af * ira2 * D[6];
        bs = dir * (as * cs * D[1] + sg * af * cf * vpar) * iQ2 - af * ira * Bpar + as * ira2 * D[6];
        ba = T(0.5) * vper - dir * sg * isr2 * Bper;
    }
    // W += c_f r_fast + c_a r_alfven + c_s r_slow of the waves moving in direction dir.
    __device__ __forceinline__ void add(T W[7], T dir, T c_f, T c_a, T c_s) const
    {
        const T mf = c_f * rho * af + c_s * rho * as;
        const T mu = dir * (c_f * af * cf + c_s * as * cs);
        const T mv = dir * sg * (-c_f * as * cs + c_s * af * cf);      // along beta
        const T mb = sr * a * (c_f * as - c_s * af);                    // along beta
        const T ma = dir * sg * sr * c_a;                               // B along -beta_perp per unit v_perp
        W[0] += mf;
        W[1] += mu;
        W[2] += mv * b1 - c_a * b2;
        W[3] += mv * b2 + c_a * b1;
        W[4] += mb * b1 + ma * b2;
        W[5] += mb * b2 - ma * b1;
        W[6] += ra2 * (c_f * af + c_s * as);
    }
};

}  // namespace ppmlr
