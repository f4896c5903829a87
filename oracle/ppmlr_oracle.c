/*
 * ppmlr_oracle.c -- TEST INFRASTRUCTURE ONLY (the oracle).
 *
 * A plain, slow, FP64 CPU implementation of one dimensionally split
 * PPMLR-MHD sweep and of the split step built from three of them.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load this library.  It shares no code, header, table or helper with the GPU
 * library; the two are written independently from the same reading of the
 * method.
 *
 * What is computed (paper, Section II "The PPMLR-MHD Method", and the
 * dimensional splitting of Section III-A):
 *   - the 3D ideal-MHD equations with the dipole split B = B_d + B' (the
 *     equation block of Section II: evolved variables rho, rho v, B', E with
 *     E = p/(gamma-1) + rho v^2/2 + B'^2/2, mu0 = 1 in code units);
 *   - all variables are zone-centred volume averages;
 *   - a piecewise-parabolic distribution in each zone (Colella & Woodward
 *     1984, "CW84" below: Eqs. 1.6-1.8 for edge values, 1.10 for monotonicity,
 *     1.12 for domain-of-dependence averages, appendix for flattening);
 *   - edge values from characteristic tracing, a Lagrangian update with an
 *     interface Riemann solve, and a conservative remap back to the fixed
 *     Eulerian grid;
 *   - three independent 1D problems per zone, one per axis.
 *
 * Conserved state per zone, SoA [8][nz][ny][nx] (x fastest):
 *   U = (rho, m_x, m_y, m_z, B'_x, B'_y, B'_z, E').
 *
 * The readings the paper leaves open (Riemann solver form, tracing, flux form
 * of the dipole terms, floors, boundary ghosts, the div B source in a split
 * scheme) are listed with their justification in the design notes; every
 * function below names the one it follows.
 *
 * What pins this oracle (tests/test_oracle_*.py): exact edge values for cubic
 * profiles on random nonuniform grids; the uniform-grid 7/12, -1/12 stencil;
 * no new extrema; monotone, average-preserving parabolas; domain-of-
 * dependence averages against Gauss quadrature; the exact gas-dynamic star
 * state for two-shock problems (independent bisection); linear acoustics for
 * small jumps; the Alfven pair against an eigen-decomposition; bitwise
 * preservation of uniform and static-dipole states; conservation of mass,
 * momentum and energy on periodic boxes; axis permutation and mirror
 * symmetry; second-order convergence of fast, Alfven and slow eigenmodes
 * (along an axis, oblique, on a moving background, with the background field
 * carried as B_d); Sod and colliding-stream problems against the exact
 * solution; convergence of the dipole split form to the plain form; the
 * -v div B' source; inflow ghosts and the inner-boundary reset; the CFL dt
 * against the largest eigenvalue of the MHD Jacobian per axis (total field,
 * stretched grids, inner mask); the totals against closed-form volume
 * integrals of linear fields; the Alfven pair with unequal densities against
 * the two-medium jump conditions; the factor 2 of the Eq. 1.8 limiter (a
 * clipped linear profile reaches the neighbouring average); the
 * time-centring terms B'_n dB_d/dm of the split step (a plasma at rest on a
 * pencil through the dipole against the exact second-order Taylor expansion
 * of its transverse field, both tracing modes); the flattening constants
 * (measured from outside with compressive steps against the published
 * CW84 values); the P >= P0/2 bound on the coupled traced pressure (active
 * in a low-beta shear, which stays positive and converged only with it).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#define NV 8
#define NG 7            /* ghost zones per side (flattening needs 7) */

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_INFLOW = 2 };

typedef struct {
    int n[3];                 /* nx, ny, nz */
    const double *faces[3];   /* n[a]+1 increasing face coordinates per axis */
    int bc_lo[3], bc_hi[3];
    double gamma;
    double dip_moment;        /* B_d = M [3 (m.r) r / r^5 - m / r^3]; 0 = none */
    double dip_dir[3];        /* unit vector m */
    double bext[3];           /* uniform external field added to B_d */
    double inflow[8];         /* rho, vx, vy, vz, Bx, By, Bz (total field), p */
    double r_inner;           /* zones with centre radius < r_inner are reset */
    double inner_rho, inner_p;
    const double *inner_v;    /* optional velocity of the reset zones (the
                                 ionosphere's E x B drift): [3][box] over the
                                 index box inner_box = (i0, i1, j0, j1, k0, k1),
                                 x fastest; NULL (or a zone outside the box):
                                 at rest */
    int inner_box[6];
    int flatten;              /* CW84 appendix shock flattening on/off */
    int janhunen;             /* -v div B' induction source on/off */
    int max_iter;
    double tol;               /* Newton stop: |dP| <= tol * P */
    double p_floor;           /* thermal-pressure floor (absolute) */
    int tracing;              /* 0: two-family tracing (fast pair, Alfven pair)
                                 with the oblique coupling terms and the
                                 two-shock / linear Alfven solvers; 1:
                                 characteristic mode: tracing of the seven
                                 waves and the linearised seven-wave
                                 Riemann problem */
} oracle_problem;

typedef struct {
    long long iters_hist[32];
    long long floor_hits;
    long long nonconverged;
    long long nonphys;
} oracle_stats;

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }
static double dsgn(double a) { return (a > 0.0) ? 1.0 : ((a < 0.0) ? -1.0 : 0.0); }

/* Static curl-free background field B_d at a point: the Earth dipole (point
 * dipole of moment M along the unit vector m, evaluated analytically wherever
 * it is needed) plus an optional uniform field. */
static void dipole_field(const oracle_problem *pr, const double r[3], double B[3])
{
    for (int k = 0; k < 3; ++k) B[k] = pr->bext[k];
    if (pr->dip_moment == 0.0) return;
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double rr = sqrt(r2);
    double r3 = r2 * rr;
    double r5 = r3 * r2;
    double mr = pr->dip_dir[0] * r[0] + pr->dip_dir[1] * r[1] + pr->dip_dir[2] * r[2];
    for (int k = 0; k < 3; ++k)
        B[k] += pr->dip_moment * (3.0 * mr * r[k] / r5 - pr->dip_dir[k] / r3);
}

/* ------------------------------------------------------------------ */
/* CW84 piecewise-parabolic reconstruction on a nonuniform coordinate  */
/* ------------------------------------------------------------------ */

/* CW84 Eq. 1.7: average slope in zone j times its width, on nonuniform
 * widths w.  Then Eq. 1.8: limited so that the edge values stay between
 * neighbouring averages; zero at a local extremum. */
static double cw84_slope(const double *a, const double *w, int j, int limit)
{
    double wm = w[j - 1], w0 = w[j], wp = w[j + 1];
    double dp = a[j + 1] - a[j];
    double dm = a[j] - a[j - 1];
    double da = w0 / (wm + w0 + wp) *
                ((2.0 * wm + w0) / (wp + w0) * dp + (w0 + 2.0 * wp) / (wm + w0) * dm);
    if (!limit) return da;
    if (dp * dm > 0.0) {
        double m = dmin(fabs(da), dmin(2.0 * fabs(dm), 2.0 * fabs(dp)));
        return dsgn(da) * m;
    }
    return 0.0;
}

/* CW84 Eq. 1.6: value at the edge j+1/2 from the averages a_{j-1..j+2},
 * the widths w_{j-1..j+2} and the (limited) slopes of zones j and j+1. */
static double cw84_edge(const double *a, const double *w, const double *dma, int j)
{
    double w0 = w[j - 1], w1 = w[j], w2 = w[j + 1], w3 = w[j + 2];
    double d = a[j + 1] - a[j];
    double sum4 = w0 + w1 + w2 + w3;
    double t1 = 2.0 * w2 * w1 / (w1 + w2) *
                ((w0 + w1) / (2.0 * w1 + w2) - (w3 + w2) / (2.0 * w2 + w1)) * d;
    double t2 = -w1 * (w0 + w1) / (2.0 * w1 + w2) * dma[j + 1];
    double t3 = w2 * (w2 + w3) / (w1 + 2.0 * w2) * dma[j];
    return a[j] + w1 / (w1 + w2) * d + (t1 + t2 + t3) / sum4;
}

/* Edge values a_{j+1/2} (stored at index j) for j in [1, M-3], from
 * unlimited (limit=0) or limited (limit=1) slopes. */
static void ppm_edges(int M, const double *a, const double *w, int limit,
                      double *slope, double *edge)
{
    for (int j = 0; j < M; ++j) { slope[j] = 0.0; edge[j] = 0.0; }
    for (int j = 1; j <= M - 2; ++j) slope[j] = cw84_slope(a, w, j, limit);
    for (int j = 1; j <= M - 3; ++j) edge[j] = cw84_edge(a, w, slope, j);
}

/* Zone parabola from its edge values: optional flattening toward the zone
 * average (CW84 appendix, weight f), then the CW84 Eq. 1.10 monotonicity
 * constraints, then the coefficients (a_L, Delta a, a_6). */
static void ppm_parabola(double a, double aL, double aR, double f, int monot,
                         double *outL, double *outD, double *out6)
{
    aL = aL + f * (a - aL);
    aR = aR + f * (a - aR);
    if (monot) {
        if ((aR - a) * (a - aL) <= 0.0) {
            aL = a;
            aR = a;
        } else {
            double dA = aR - aL;
            double a6 = 6.0 * (a - 0.5 * (aL + aR));
            if (dA * a6 > dA * dA) aL = 3.0 * a - 2.0 * aR;
            else if (-dA * dA > dA * a6) aR = 3.0 * a - 2.0 * aL;
        }
    }
    *outL = aL;
    *outD = aR - aL;
    *out6 = 6.0 * (a - 0.5 * (aL + aR));
}

/* CW84 Eq. 1.12: exact averages of the zone parabola over the fraction y of
 * the zone adjacent to its right edge (fL) and to its left edge (fR). */
static double par_avg_right_part(double aL, double dA, double a6, double y)
{
    double aR = aL + dA;
    return aR - 0.5 * y * (dA - (1.0 - (2.0 / 3.0) * y) * a6);
}
static double par_avg_left_part(double aL, double dA, double a6, double y)
{
    return aL + 0.5 * y * (dA + (1.0 - (2.0 / 3.0) * y) * a6);
}

/* ------------------------------------------------------------------ */
/* Full characteristic tracing: the seven waves of Lagrangian 1D MHD    */
/* ------------------------------------------------------------------ */

/* Eigen-structure of the 1D ideal-MHD equations in the mass coordinate m,
 * in the primitive variables W = (rho, u, v_t1, v_t2, B_t1, B_t2, p) of a
 * pencil: dW/dt + A dW/dm = 0, where A is rho times the Eulerian primitive
 * matrix without the advection term (the material derivative takes the flow
 * along), so the eigenvectors are the Eulerian ones and the eigenvalues are
 * rho times the wave speeds relative to the flow.  Order of the waves:
 * 0 -fast, 1 -Alfven, 2 -slow, 3 entropy, 4 +slow, 5 +Alfven, 6 +fast.
 * Right eigenvectors (columns of R) in the normalisation of Roe & Balsara
 * (1996): weights alpha_f^2 = (a^2 - c_s^2)/(c_f^2 - c_s^2) and alpha_s^2 =
 * (c_f^2 - a^2)/(c_f^2 - c_s^2) (1 and 0 where c_f = c_s), the unit vector
 * beta along the transverse field (a fixed diagonal direction where the
 * transverse field vanishes) and sgn(B_n) with sgn(0) = 1, so that the set
 * stays complete at every degeneracy.  Bn, Bt1, Bt2: the total field. */
static void mhd7_eigen(double rho, double p, double g, double Bn, double Bt1, double Bt2,
                       double lam[7], double R[7][7])
{
    double a2 = g * p / rho;
    double bn2 = Bn * Bn / rho;
    double bt2 = (Bt1 * Bt1 + Bt2 * Bt2) / rho;
    double bt = sqrt(Bt1 * Bt1 + Bt2 * Bt2);
    double b2 = bn2 + bt2;
    /* c_f^2 - c_s^2, written without cancellation: exact where bt = 0 */
    double disc = sqrt((a2 - b2) * (a2 - b2) + 4.0 * a2 * bt2);
    double cf2 = 0.5 * (a2 + b2 + disc);
    double cs2 = cf2 > 0.0 ? a2 * bn2 / cf2 : 0.0;   /* c_f^2 c_s^2 = a^2 c_A^2 */
    double cf = sqrt(cf2), cs = sqrt(cs2), ca = sqrt(bn2), a = sqrt(a2);
    /* alpha_f^2 = (a^2 - c_s^2) / (c_f^2 - c_s^2) = (1 + (a^2 - b^2) / disc) / 2
     * and alpha_s^2 = 1 - alpha_f^2; the smaller of the two is written as
     * 2 a^2 bt^2 / (disc (disc + |a^2 - b^2|)), exact for small bt */
    double af, as;
    if (disc > 0.0) {
        double small = 2.0 * a2 * bt2 / (disc * (disc + fabs(a2 - b2)));
        if (a2 >= b2) { as = sqrt(dmin(1.0, small)); af = sqrt(dmax(0.0, 1.0 - small)); }
        else { af = sqrt(dmin(1.0, small)); as = sqrt(dmax(0.0, 1.0 - small)); }
    } else {                                          /* a = c_A, no transverse field */
        af = 1.0;
        as = 0.0;
    }
    double be1, be2;
    if (bt > 1e-12 * sqrt(rho * (a2 + b2))) { be1 = Bt1 / bt; be2 = Bt2 / bt; }
    else { be1 = be2 = sqrt(0.5); }
    double sg = Bn < 0.0 ? -1.0 : 1.0;
    double sr = sqrt(rho);
    for (int i = 0; i < 7; ++i)
        for (int k = 0; k < 7; ++k) R[i][k] = 0.0;
    for (int side = 0; side < 2; ++side) {
        double s = side == 0 ? -1.0 : 1.0;          /* direction of the wave */
        int kf = side == 0 ? 0 : 6, ka = side == 0 ? 1 : 5, ks = side == 0 ? 2 : 4;
        lam[kf] = s * rho * cf;
        lam[ka] = s * rho * ca;
        lam[ks] = s * rho * cs;
        /* fast */
        R[0][kf] = rho * af;
        R[1][kf] = s * af * cf;
        R[2][kf] = -s * as * cs * sg * be1;
        R[3][kf] = -s * as * cs * sg * be2;
        R[4][kf] = as * sr * a * be1;
        R[5][kf] = as * sr * a * be2;
        R[6][kf] = af * rho * a2;
        /* slow */
        R[0][ks] = rho * as;
        R[1][ks] = s * as * cs;
        R[2][ks] = s * af * cf * sg * be1;
        R[3][ks] = s * af * cf * sg * be2;
        R[4][ks] = -af * sr * a * be1;
        R[5][ks] = -af * sr * a * be2;
        R[6][ks] = as * rho * a2;
        /* Alfven: the velocity and field across beta, dB = -s sgn(Bn) sqrt(rho) dv */
        R[2][ka] = -be2;
        R[3][ka] = be1;
        R[4][ka] = s * sg * sr * be2;
        R[5][ka] = -s * sg * sr * be1;
    }
    lam[3] = 0.0;
    R[0][3] = 1.0;                                   /* entropy: density only */
}

/* Waves of zero Lagrangian speed: where the normal field vanishes the Alfven
 * and slow waves stop, and the traced face state jumps between the reference
 * value (wave at rest) and the edge value (wave of speed 0+), with the
 * Alfven family's eigenvector set by sgn(B_n).  A normal field that is zero
 * in exact arithmetic (a background field cancelled by the deviation field)
 * is rounding noise in any implementation, so the characteristic mode
 * takes a wave slower than WAVE_MIN times the fast wave as at rest, in the
 * tracing and in the interface problem: its domain of dependence is then
 * below 1e-4 of the fast wave's, and the decision no longer rests on the
 * sign of noise. */
#define WAVE_MIN 1e-4

/* Inverse of a 7 x 7 matrix by Gauss-Jordan elimination with partial
 * pivoting (the left eigenvectors are the rows of the inverse of R). */
static int invert7(double A[7][7], double X[7][7])
{
    double M[7][14];
    for (int i = 0; i < 7; ++i)
        for (int j = 0; j < 14; ++j) M[i][j] = j < 7 ? A[i][j] : (j - 7 == i ? 1.0 : 0.0);
    for (int c = 0; c < 7; ++c) {
        int piv = c;
        for (int i = c + 1; i < 7; ++i)
            if (fabs(M[i][c]) > fabs(M[piv][c])) piv = i;
        if (M[piv][c] == 0.0) return -1;
        if (piv != c)
            for (int j = 0; j < 14; ++j) { double t = M[c][j]; M[c][j] = M[piv][j]; M[piv][j] = t; }
        double d = M[c][c];
        for (int j = 0; j < 14; ++j) M[c][j] /= d;
        for (int i = 0; i < 7; ++i) {
            if (i == c || M[i][c] == 0.0) continue;
            double f = M[i][c];
            for (int j = 0; j < 14; ++j) M[i][j] -= f * M[c][j];
        }
    }
    for (int i = 0; i < 7; ++i)
        for (int j = 0; j < 7; ++j) X[i][j] = M[i][j + 7];
    return 0;
}

/* Interface states of one zone by full characteristic tracing (CW84's
 * tracing with one reference state, for the seven Lagrangian MHD waves):
 * at the right face the waves with positive speed arrive within dt, at the
 * left face those with negative speed.  The reference state is the average
 * of the zone's parabolas (aL, dA, a6 per primitive) over the domain of
 * dependence of the fast wave, y = |lambda| dt / dm (at most 1); every
 * slower wave that arrives is given the average over its own domain: the
 * difference of the two averages is projected on that wave's left
 * eigenvector and taken out along its right eigenvector.  WL: the state at
 * the right face, WR: at the left face. */
static void trace7(const double aL[7], const double dA[7], const double a6[7], const double lam[7],
                   double R[7][7], double Li[7][7], double dt, double dm, double WL[7], double WR[7])
{
    for (int side = 0; side < 2; ++side) {
        int kref = side == 0 ? 6 : 0;                 /* fast wave into this face */
        int slower[2] = {side == 0 ? 5 : 1, side == 0 ? 4 : 2};
        double *out = side == 0 ? WL : WR;
        double yref = dmin(1.0, fabs(lam[kref]) * dt / dm);
        double ref[7];
        for (int v = 0; v < 7; ++v)
            ref[v] = side == 0 ? par_avg_right_part(aL[v], dA[v], a6[v], yref)
                               : par_avg_left_part(aL[v], dA[v], a6[v], yref);
        for (int v = 0; v < 7; ++v) out[v] = ref[v];
        for (int q = 0; q < 2; ++q) {
            int k = slower[q];
            /* a wave slower than WAVE_MIN times the fast wave counts as not
             * reaching the face (see WAVE_MIN) */
            if (!(fabs(lam[k]) > WAVE_MIN * fabs(lam[kref]))) continue;
            double y = dmin(1.0, fabs(lam[k]) * dt / dm);
            double beta = 0.0;
            for (int v = 0; v < 7; ++v) {
                double avg = side == 0 ? par_avg_right_part(aL[v], dA[v], a6[v], y)
                                       : par_avg_left_part(aL[v], dA[v], a6[v], y);
                beta += Li[k][v] * (ref[v] - avg);
            }
            for (int v = 0; v < 7; ++v) out[v] -= beta * R[v][k];
        }
    }
}

/* The Riemann problem at a face in the mass coordinate, linearised about the
 * mean of the two states: the face is at rest, so its state is the left
 * state plus the jumps of the waves with negative speed, W* = W_L +
 * sum_{lambda_k < 0} (l_k . (W_R - W_L)) r_k (the pairs of the two-family
 * mode are solved separately; here all seven waves are one system).  W_L,
 * W_R: primitives with B'_t; Bn: total normal field at the face; Bd1, Bd2:
 * the background transverse field at the face. */
static int riemann7(const double WL[7], const double WR[7], double g, double Bn, double Bd1, double Bd2,
                    double Ws[7])
{
    double lam[7], R[7][7], Li[7][7];
    mhd7_eigen(0.5 * (WL[0] + WR[0]), 0.5 * (WL[6] + WR[6]), g, Bn, Bd1 + 0.5 * (WL[4] + WR[4]),
               Bd2 + 0.5 * (WL[5] + WR[5]), lam, R);
    if (invert7(R, Li) != 0) return -1;
    for (int v = 0; v < 7; ++v) Ws[v] = WL[v];
    for (int k = 0; k < 7; ++k) {
        /* waves of negative speed cross to the left; one slower than
         * WAVE_MIN times the fast wave counts as at rest (see WAVE_MIN) */
        if (!(lam[k] < -WAVE_MIN * fabs(lam[6]))) continue;
        double beta = 0.0;
        for (int v = 0; v < 7; ++v) beta += Li[k][v] * (WR[v] - WL[v]);
        for (int v = 0; v < 7; ++v) Ws[v] += beta * R[v][k];
    }
    return 0;
}

/* CW84 appendix shock detection / flattening coefficients on the transverse
 * total pressure.  Pt: perturbation pressure differences are taken on it;
 * Pa: absolute (positive) pressure for the relative-jump test; un: normal
 * velocity; rho: density.  Constants eps = 0.33, omega1 = 0.75, omega2 = 10.
 * The compression test u_{j-1} > u_{j+1} is taken with a margin of COMP_MIN
 * times the speed sqrt(P_min / rho_j) of the jump test's pressure: at a
 * pressure jump at rest the two velocities are equal, and a strict
 * comparison would let rounding noise (which two implementations produce
 * differently) switch full flattening on or off; no shock compresses at
 * 1e-5 of a sound speed. */
#define COMP_MIN 1e-5
static void flattening(int M, const double *Pt, const double *Pa, const double *un, const double *rho,
                       double *ftil, double *f)
{
    const double eps = 0.33, om1 = 0.75, om2 = 10.0;
    for (int j = 0; j < M; ++j) { ftil[j] = 0.0; f[j] = 0.0; }
    for (int j = 2; j <= M - 3; ++j) {
        double d1 = Pt[j + 1] - Pt[j - 1];
        double d2 = Pt[j + 2] - Pt[j - 2];
        double pmin = dmin(Pa[j + 1], Pa[j - 1]);
        double ft = 0.0;
        if (fabs(d1) > eps * pmin && un[j - 1] - un[j + 1] > COMP_MIN * sqrt(pmin / rho[j])) {
            if (d2 != 0.0) ft = dmax(0.0, dmin(1.0, om2 * (d1 / d2 - om1)));
            else ft = 1.0;
        }
        ftil[j] = ft;
    }
    for (int j = 3; j <= M - 4; ++j) {
        int s = (Pt[j + 1] - Pt[j - 1] < 0.0) ? 1 : -1;
        f[j] = dmax(ftil[j], ftil[j + s]);
    }
}

/* ------------------------------------------------------------------ */
/* Interface Riemann problems                                          */
/* ------------------------------------------------------------------ */

/* Normal pair (total pressure, normal velocity).  Two-shock Newton iteration
 * of CW84 Section 2 on the total transverse pressure, with a per-side
 * effective adiabatic index gamma_e = C^2 / (rho P) (gamma_e = gamma when
 * B = 0).  Pressures are carried as perturbations Pt = P - Pd with Pd the
 * common dipole part, so that only differences of Pt enter the jumps.
 * Returns the iteration count (number of applied updates); the final Newton
 * correction is applied on exit and u* is its linearised value. */
static int riemann_normal(double PtL, double PtR, double Pd, double uL, double uR,
                          double CL, double CR, double gL, double gR,
                          double tol, int max_iter, double *Pstar, double *ustar,
                          int *converged)
{
    double PL = PtL + Pd, PR = PtR + Pd;
    double kL = (gL + 1.0) / (2.0 * gL);
    double kR = (gR + 1.0) / (2.0 * gR);
    double Pfloor = 1e-6 * dmin(PL, PR) - Pd;
    /* linear acoustic guess, increment form */
    double P = PtL + CL * ((PtR - PtL) + CR * (uL - uR)) / (CL + CR);
    P = dmax(P, Pfloor);
    int iters = 0;
    double WL, WR, usL, usR, ZL, ZR, dP;
    *converged = 1;
    for (;;) {
        WL = CL * sqrt(1.0 + kL * (P - PtL) / PL);
        WR = CR * sqrt(1.0 + kR * (P - PtR) / PR);
        usL = uL - (P - PtL) / WL;
        usR = uR + (P - PtR) / WR;
        ZL = 2.0 * WL * WL * WL / (WL * WL + CL * CL);
        ZR = 2.0 * WR * WR * WR / (WR * WR + CR * CR);
        dP = -ZL * ZR * (usR - usL) / (ZL + ZR);
        if (fabs(dP) <= tol * (P + Pd)) break;
        if (iters >= max_iter) { *converged = 0; break; }
        P = dmax(P + dP, Pfloor);
        iters++;
    }
    *Pstar = dmax(P + dP, Pfloor);
    *ustar = usL + ZR * (usR - usL) / (ZL + ZR);
    return iters;
}

/* Transverse pair: linear Alfven Riemann problem in closed form.  Riemann
 * invariants v -+ sigma B / sqrt(rho) carried at -+ sqrt(rho)|B_n| in the
 * mass coordinate; written in increment form from the left state. */
static void riemann_alfven(double rL, double rR, double sigma,
                           double vL, double vR, double bL, double bR,
                           double *vstar, double *bstar)
{
    double s = rL + rR;
    *vstar = vL + (rR * (vR - vL) + sigma * (bR - bL)) / s;
    *bstar = bL + (rL * (bR - bL) + sigma * rL * rR * (vR - vL)) / s;
}

/* ------------------------------------------------------------------ */
/* One pencil                                                          */
/* ------------------------------------------------------------------ */

/* Work arrays for one pencil of M = N + 2*NG zones. */
typedef struct {
    int M;
    double *buf;
} pencil_work;

/* Sweep one pencil.  Inputs (length M, ghosts already filled):
 *   U[8][M]   conserved, dx[M] widths, xc[M] centres, xf[M+1] faces
 *   (xf[i] is the left face of zone i), c1, c2: the pencil's transverse
 *   centre coordinates (axes t1, t2).
 * Output: Uout[8][N] interior zones. */
static void sweep_pencil(const oracle_problem *pr, int axis, int N, int j1, int j2,
                         double *const U[NV], const double *dx, const double *xc,
                         const double *xf, double c1, double c2, double dt,
                         double *const Uout[NV], oracle_stats *st, double *face_states)
{
    const int M = N + 2 * NG;
    const int n = axis, t1 = (axis + 1) % 3, t2 = (axis + 2) % 3;
    const double g = pr->gamma;

    /* allocate work arrays */
    enum { W_RHO = 0, W_U, W_V1, W_V2, W_B1, W_B2, W_P, NW };
    double *mem = (double *)calloc((size_t)M * 130 + 64, sizeof(double));
    double *p_ = mem;
#define TAKE(ptr) double *ptr = p_; p_ += M + 1;
#define TAKEN(arr, cnt) double *arr[cnt]; for (int q_ = 0; q_ < (cnt); ++q_) { arr[q_] = p_; p_ += M + 1; }
    TAKEN(W, NW)
    TAKE(bn)            /* B'_n at centres */
    TAKE(dm)            /* zone masses */
    TAKEN(Bdc, 3)       /* dipole at centres, pencil frame (n,t1,t2) */
    TAKEN(Bdf, 3)       /* dipole at face i+1/2 (index i), pencil frame */
    TAKE(Pt) TAKE(Pa)   /* flattening pressures */
    TAKE(ftil) TAKE(fl)
    TAKE(slope) TAKE(edge)
    TAKEN(pL, NW) TAKEN(pD, NW) TAKEN(p6, NW)  /* Lagrangian parabolas */
    /* traced states: L at face i+1/2 from zone i, R at face i-1/2 from zone i */
    TAKE(Ln_rho) TAKE(Ln_u) TAKE(Ln_p) TAKE(Ln_b1) TAKE(Ln_b2)
    TAKE(Rn_rho) TAKE(Rn_u) TAKE(Rn_p) TAKE(Rn_b1) TAKE(Rn_b2)
    TAKE(LA_rho) TAKE(LA_v1) TAKE(LA_v2) TAKE(LA_b1) TAKE(LA_b2)
    TAKE(RA_rho) TAKE(RA_v1) TAKE(RA_v2) TAKE(RA_b1) TAKE(RA_b2)
    TAKE(corrP) TAKE(corrB1) TAKE(corrB2)
    TAKE(corrU) TAKE(corrV1) TAKE(corrV2)
    /* face quantities (index i = face i+1/2) */
    TAKE(F_pi) TAKE(F_v1) TAKE(F_v2) TAKE(F_b1) TAKE(F_b2) TAKE(F_e) TAKE(delta)
    /* Lagrangian zone results */
    TAKE(dVL)
    TAKEN(dC, 7)
    TAKEN(QL, 7)
    TAKEN(rL, 7) TAKEN(rD, 7) TAKEN(r6, 7)
    TAKEN(FR, 7)
#undef TAKE
#undef TAKEN

    /* conserved index of each remapped quantity, in pencil frame */
    const int qidx[7] = {0, 1 + n, 1 + t1, 1 + t2, 4 + t1, 4 + t2, 7};

    /* ---- step a2: primitives, masses, dipole values ---- */
    for (int i = 0; i < M; ++i) {
        double rho = U[0][i];
        int interior = (i >= NG && i < NG + N);
        if (!(rho > 0.0) || !isfinite(rho) || !isfinite(U[7][i])) {
            if (interior) st->nonphys++;
        }
        double u = U[1 + n][i] / rho, v1 = U[1 + t1][i] / rho, v2 = U[1 + t2][i] / rho;
        double b0 = U[4 + n][i], b1 = U[4 + t1][i], b2 = U[4 + t2][i];
        double ke = 0.5 * rho * (u * u + v1 * v1 + v2 * v2);
        double me = 0.5 * (b0 * b0 + b1 * b1 + b2 * b2);
        double p = (g - 1.0) * (U[7][i] - ke - me);
        if (p < pr->p_floor) {
            p = pr->p_floor;
            if (interior) st->floor_hits++;
        }
        W[W_RHO][i] = rho; W[W_U][i] = u; W[W_V1][i] = v1; W[W_V2][i] = v2;
        W[W_B1][i] = b1; W[W_B2][i] = b2; W[W_P][i] = p;
        bn[i] = b0;
        dm[i] = rho * dx[i];

        double pos[3], B[3];
        pos[n] = xc[i]; pos[t1] = c1; pos[t2] = c2;
        dipole_field(pr, pos, B);
        Bdc[0][i] = B[n]; Bdc[1][i] = B[t1]; Bdc[2][i] = B[t2];
        pos[n] = xf[i + 1];
        dipole_field(pr, pos, B);
        Bdf[0][i] = B[n]; Bdf[1][i] = B[t1]; Bdf[2][i] = B[t2];

        Pt[i] = p + Bdc[1][i] * b1 + Bdc[2][i] * b2 + 0.5 * (b1 * b1 + b2 * b2);
        Pa[i] = Pt[i] + 0.5 * (Bdc[1][i] * Bdc[1][i] + Bdc[2][i] * Bdc[2][i]);
    }

    /* ---- step a3: parabolas in the mass coordinate ---- */
    if (pr->flatten) flattening(M, Pt, Pa, W[W_U], W[W_RHO], ftil, fl);
    else for (int i = 0; i < M; ++i) fl[i] = 0.0;
    for (int k = 0; k < NW; ++k) {
        ppm_edges(M, W[k], dm, 1, slope, edge);
        for (int i = 2; i <= M - 3; ++i)
            ppm_parabola(W[k][i], edge[i - 1], edge[i], fl[i], 1, &pL[k][i], &pD[k][i], &p6[k][i]);
    }

    /* ---- step a4: characteristic tracing ---- */
    for (int i = 2; i <= M - 3; ++i) {
        double rho = W[W_RHO][i], p = W[W_P][i];
        double Bt1 = Bdc[1][i] + W[W_B1][i], Bt2 = Bdc[2][i] + W[W_B2][i];
        double Bn = Bdc[0][i] + bn[i];
        double Cn = sqrt(rho * (g * p + Bt1 * Bt1 + Bt2 * Bt2));
        double CA = sqrt(rho) * fabs(Bn);
        double yn = dmin(1.0, Cn * dt / dm[i]);
        double yA = dmin(1.0, CA * dt / dm[i]);
        if (pr->tracing == 1) {
            /* one traced state per face for both Riemann problems; the
             * couplings between the pairs are in the eigenvectors */
            double lam[7], R[7][7], Li[7][7], aL[7], dA[7], a6[7], WL[7], WR[7];
            mhd7_eigen(rho, p, g, Bn, Bt1, Bt2, lam, R);
            if (invert7(R, Li) != 0) abort();
            for (int v = 0; v < 7; ++v) { aL[v] = pL[v][i]; dA[v] = pD[v][i]; a6[v] = p6[v][i]; }
            trace7(aL, dA, a6, lam, R, Li, dt, dm[i], WL, WR);
            /* a traced state without positive density and pressure (no
             * eigen-structure at the face) falls back to the zone average */
            if (!(WL[W_RHO] > 0.0) || !(WL[W_P] > 0.0))
                for (int v = 0; v < 7; ++v) WL[v] = W[v][i];
            if (!(WR[W_RHO] > 0.0) || !(WR[W_P] > 0.0))
                for (int v = 0; v < 7; ++v) WR[v] = W[v][i];
            Ln_rho[i] = LA_rho[i] = WL[W_RHO]; Rn_rho[i] = RA_rho[i] = WR[W_RHO];
            Ln_u[i] = WL[W_U]; Rn_u[i] = WR[W_U];
            Ln_p[i] = WL[W_P]; Rn_p[i] = WR[W_P];
            Ln_b1[i] = LA_b1[i] = WL[W_B1]; Rn_b1[i] = RA_b1[i] = WR[W_B1];
            Ln_b2[i] = LA_b2[i] = WL[W_B2]; Rn_b2[i] = RA_b2[i] = WR[W_B2];
            LA_v1[i] = WL[W_V1]; RA_v1[i] = WR[W_V1];
            LA_v2[i] = WL[W_V2]; RA_v2[i] = WR[W_V2];
            corrP[i] = corrB1[i] = corrB2[i] = 0.0;
        } else {
#define TR(k, y, Ldst, Rdst) \
        Ldst[i] = par_avg_right_part(pL[k][i], pD[k][i], p6[k][i], y); \
        Rdst[i] = par_avg_left_part(pL[k][i], pD[k][i], p6[k][i], y);
        TR(W_RHO, yn, Ln_rho, Rn_rho)
        TR(W_U, yn, Ln_u, Rn_u)
        TR(W_P, yn, Ln_p, Rn_p)
        TR(W_B1, yn, Ln_b1, Rn_b1)
        TR(W_B2, yn, Ln_b2, Rn_b2)
        TR(W_RHO, yA, LA_rho, RA_rho)
        TR(W_V1, yA, LA_v1, RA_v1)
        TR(W_V2, yA, LA_v2, RA_v2)
        TR(W_B1, yA, LA_b1, RA_b1)
        TR(W_B2, yA, LA_b2, RA_b2)
#undef TR
        /* time-centring of the oblique-field couplings (linearised
         * Lagrangian equations: dP/dt gains rho B_n B_t . dv_t/dm and
         * dB_t/dt gains -rho B_t du/dm); same value for both edges */
        corrP[i] = 0.5 * dt * rho * Bn * (Bt1 * pD[W_V1][i] + Bt2 * pD[W_V2][i]) / dm[i];
        corrB1[i] = -0.5 * dt * rho * Bt1 * pD[W_U][i] / dm[i];
        corrB2[i] = -0.5 * dt * rho * Bt2 * pD[W_U][i] / dm[i];
        }
        /* terms from the variation of the normal field along the pencil
         * (zero in 1D, nonzero in a split multi-D step): mass-coordinate
         * derivatives of B'_n (centred) and of the dipole (face values) */
        double dbn = (bn[i + 1] - bn[i - 1]) / (0.5 * dm[i - 1] + dm[i] + 0.5 * dm[i + 1]);
        double ddn = (Bdf[0][i] - Bdf[0][i - 1]) / dm[i];
        double dd1 = (Bdf[1][i] - Bdf[1][i - 1]) / dm[i];
        double dd2 = (Bdf[2][i] - Bdf[2][i - 1]) / dm[i];
        double dBn = ddn + dbn;
        double u = W[W_U][i], v1 = W[W_V1][i], v2 = W[W_V2][i];
        double bp1 = W[W_B1][i], bp2 = W[W_B2][i];
        corrU[i] = 0.5 * dt * (Bn * dbn + bn[i] * ddn);
        corrV1[i] = 0.5 * dt * (bp1 * dBn + Bdc[1][i] * dbn + bn[i] * dd1);
        corrV2[i] = 0.5 * dt * (bp2 * dBn + Bdc[2][i] * dbn + bn[i] * dd2);
        corrB1[i] += 0.5 * dt * rho * (v1 * dBn - u * dd1);
        corrB2[i] += 0.5 * dt * rho * (v2 * dBn - u * dd2);
        corrP[i] += 0.5 * dt * rho * ((Bt1 * v1 + Bt2 * v2) * dBn - u * (Bt1 * dd1 + Bt2 * dd2));
    }

    /* ---- step a5 + a6: Riemann problems and Lagrangian fluxes ---- */
    for (int i = 3; i <= M - 5; ++i) {   /* face i+1/2 between zones i, i+1 */
        double Bdn = Bdf[0][i], Bd1 = Bdf[1][i], Bd2 = Bdf[2][i];
        double Pd = 0.5 * (Bd1 * Bd1 + Bd2 * Bd2);
        if (pr->tracing == 1) {
            /* characteristic mode: the interface problem in its
             * linearisation about the mean of the two traced states, with
             * the time-centring terms of the split multi-D step on u, v_t
             * and B_t.  The thermal pressure takes none: its Lagrangian
             * equation has no term in the variation of B_n, and corrP is
             * the magnetic-pressure change B_t . corrB that the corrected
             * field already carries into the total pressure. */
            double WLs[7] = {Ln_rho[i], Ln_u[i] + corrU[i], LA_v1[i] + corrV1[i], LA_v2[i] + corrV2[i],
                             Ln_b1[i] + corrB1[i], Ln_b2[i] + corrB2[i], Ln_p[i]};
            double WRs[7] = {Rn_rho[i + 1], Rn_u[i + 1] + corrU[i + 1], RA_v1[i + 1] + corrV1[i + 1],
                             RA_v2[i + 1] + corrV2[i + 1], Rn_b1[i + 1] + corrB1[i + 1],
                             Rn_b2[i + 1] + corrB2[i + 1], Rn_p[i + 1]};
            double bns = 0.5 * (bn[i] + bn[i + 1]);
            double Bns = Bdn + bns;
            double Ws[7];
            if (face_states)    /* test hook: the two states of the solve */
                for (int v = 0; v < 7; ++v) {
                    face_states[i * 14 + v] = WLs[v];
                    face_states[i * 14 + 7 + v] = WRs[v];
                }
            if (riemann7(WLs, WRs, g, Bns, Bd1, Bd2, Ws) != 0) abort();
            double ust = Ws[1], v1s = Ws[2], v2s = Ws[3], b1s = Ws[4], b2s = Ws[5];
            double Pst = Ws[6] + Bd1 * b1s + Bd2 * b2s + 0.5 * (b1s * b1s + b2s * b2s);
            if (i >= NG - 1 && i <= NG + N - 1) st->iters_hist[0]++;   /* no iteration */
            double nn = bns * (Bdn + 0.5 * bns);
            F_pi[i] = Pst - nn;
            F_v1[i] = -(Bns * b1s + bns * Bd1);
            F_v2[i] = -(Bns * b2s + bns * Bd2);
            F_b1[i] = ust * Bd1 - Bns * v1s;
            F_b2[i] = ust * Bd2 - Bns * v2s;
            F_e[i] = ust * (Pst + nn) - Bns * (ust * bns + v1s * b1s + v2s * b2s);
            delta[i] = ust * dt;
            continue;
        }
        /* left state (zone i) */
        double rl = Ln_rho[i], ul = Ln_u[i] + corrU[i], pl = Ln_p[i], b1l = Ln_b1[i], b2l = Ln_b2[i];
        double T1l = Bd1 + b1l, T2l = Bd2 + b2l;
        double CL = sqrt(rl * (g * pl + T1l * T1l + T2l * T2l));
        double P0l = pl + 0.5 * (T1l * T1l + T2l * T2l);
        double PtL = pl + Bd1 * b1l + Bd2 * b2l + 0.5 * (b1l * b1l + b2l * b2l) + corrP[i];
        if (PtL + Pd < 0.5 * P0l) PtL = 0.5 * P0l - Pd;
        /* right state (zone i+1) */
        double rr = Rn_rho[i + 1], ur = Rn_u[i + 1] + corrU[i + 1], pr_ = Rn_p[i + 1];
        double b1r = Rn_b1[i + 1], b2r = Rn_b2[i + 1];
        double T1r = Bd1 + b1r, T2r = Bd2 + b2r;
        double CR = sqrt(rr * (g * pr_ + T1r * T1r + T2r * T2r));
        double P0r = pr_ + 0.5 * (T1r * T1r + T2r * T2r);
        double PtR = pr_ + Bd1 * b1r + Bd2 * b2r + 0.5 * (b1r * b1r + b2r * b2r) + corrP[i + 1];
        if (PtR + Pd < 0.5 * P0r) PtR = 0.5 * P0r - Pd;
        double gL = CL * CL / (rl * (PtL + Pd));
        double gR = CR * CR / (rr * (PtR + Pd));

        double Pst, ust;
        int conv;
        int it = riemann_normal(PtL, PtR, Pd, ul, ur, CL, CR, gL, gR,
                                pr->tol, pr->max_iter, &Pst, &ust, &conv);
        if (i >= NG - 1 && i <= NG + N - 1) {   /* faces -1/2 .. N-1/2 */
            st->iters_hist[it < 31 ? it : 31]++;
            if (!conv) st->nonconverged++;
        }

        /* transverse pair */
        double bns = 0.5 * (bn[i] + bn[i + 1]);
        double Bns = Bdn + bns;
        double sig = dsgn(Bns);
        double sl = sqrt(LA_rho[i]), sr = sqrt(RA_rho[i + 1]);
        double v1s, v2s, b1s, b2s;
        riemann_alfven(sl, sr, sig, LA_v1[i] + corrV1[i], RA_v1[i + 1] + corrV1[i + 1],
                       LA_b1[i] + corrB1[i], RA_b1[i + 1] + corrB1[i + 1], &v1s, &b1s);
        riemann_alfven(sl, sr, sig, LA_v2[i] + corrV2[i], RA_v2[i + 1] + corrV2[i + 1],
                       LA_b2[i] + corrB2[i], RA_b2[i + 1] + corrB2[i + 1], &v2s, &b2s);

        /* Lagrangian fluxes, B_0 + B_1 (dipole + deviation) flux form */
        double nn = bns * (Bdn + 0.5 * bns);
        F_pi[i] = Pst - nn;
        F_v1[i] = -(Bns * b1s + bns * Bd1);
        F_v2[i] = -(Bns * b2s + bns * Bd2);
        F_b1[i] = ust * Bd1 - Bns * v1s;
        F_b2[i] = ust * Bd2 - Bns * v2s;
        F_e[i] = ust * (Pst + nn) - Bns * (ust * bns + v1s * b1s + v2s * b2s);
        delta[i] = ust * dt;
    }

    /* ---- step a6: Lagrangian update of zone contents ---- */
    for (int i = 4; i <= M - 5; ++i) {
        double dd = delta[i] - delta[i - 1];
        dVL[i] = dx[i] + dd;
        dC[0][i] = 0.0;
        dC[1][i] = -dt * (F_pi[i] - F_pi[i - 1]);
        dC[2][i] = -dt * (F_v1[i] - F_v1[i - 1]);
        dC[3][i] = -dt * (F_v2[i] - F_v2[i - 1]);
        dC[4][i] = -dt * (F_b1[i] - F_b1[i - 1]);
        dC[5][i] = -dt * (F_b2[i] - F_b2[i - 1]);
        dC[6][i] = -dt * (F_e[i] - F_e[i - 1]);
        for (int q = 0; q < 7; ++q) {
            double Q = U[qidx[q]][i];
            QL[q][i] = Q + (dC[q][i] - Q * dd) / dVL[i];
        }
    }

    /* ---- step a7: remap in the Lagrangian volume coordinate ---- */
    {
        /* Only zones 4..M-5 hold valid Lagrangian data; fill the rest with
         * their nearest valid neighbour so the edge routine stays finite. */
        for (int q = 0; q < 7; ++q) {
            for (int i = 0; i < 4; ++i) QL[q][i] = QL[q][4];
            for (int i = M - 4; i < M; ++i) QL[q][i] = QL[q][M - 5];
        }
        for (int i = 0; i < 4; ++i) dVL[i] = dVL[4];
        for (int i = M - 4; i < M; ++i) dVL[i] = dVL[M - 5];
        for (int q = 0; q < 7; ++q) {
            ppm_edges(M, QL[q], dVL, 1, slope, edge);
            for (int i = 6; i <= M - 7; ++i)
                ppm_parabola(QL[q][i], edge[i - 1], edge[i], fl[i], 1, &rL[q][i], &rD[q][i], &r6[q][i]);
        }
        for (int i = 6; i <= M - 8; ++i) {    /* face i+1/2 */
            double d = delta[i];
            for (int q = 0; q < 7; ++q) {
                if (d > 0.0)
                    FR[q][i] = d * par_avg_right_part(rL[q][i], rD[q][i], r6[q][i], d / dVL[i]);
                else if (d < 0.0)
                    FR[q][i] = d * par_avg_left_part(rL[q][i + 1], rD[q][i + 1], r6[q][i + 1], -d / dVL[i + 1]);
                else
                    FR[q][i] = 0.0;
            }
        }
    }

    /* ---- conservative update, sources, inner boundary ---- */
    for (int i = NG; i < NG + N; ++i) {
        double out[NV];
        for (int q = 0; q < 7; ++q) {
            double Q = U[qidx[q]][i];
            out[qidx[q]] = Q + (dC[q][i] + FR[q][i - 1] - FR[q][i]) / dx[i];
        }
        out[4 + n] = U[4 + n][i];
        if (pr->janhunen) {
            /* -v div B' (paper's induction source), split: the n-derivative
             * of B'_n by central differences, pre-sweep velocity */
            double divn = (bn[i + 1] - bn[i - 1]) / (xc[i + 1] - xc[i - 1]);
            out[4 + n] -= dt * W[W_U][i] * divn;
            out[4 + t1] -= dt * W[W_V1][i] * divn;
            out[4 + t2] -= dt * W[W_V2][i] * divn;
        }
        if (pr->r_inner > 0.0) {
            double pos[3];
            pos[n] = xc[i]; pos[t1] = c1; pos[t2] = c2;
            double r = sqrt(pos[0] * pos[0] + pos[1] * pos[1] + pos[2] * pos[2]);
            if (r < pr->r_inner) {
                /* the inner state: rest, or the velocity the ionosphere
                 * coupling set for this zone */
                double v[3] = {0.0, 0.0, 0.0};
                if (pr->inner_v) {
                    int ijk[3];
                    ijk[n] = i - NG; ijk[t1] = j1; ijk[t2] = j2;
                    const int *bx = pr->inner_box;
                    if (ijk[0] >= bx[0] && ijk[0] < bx[1] && ijk[1] >= bx[2] && ijk[1] < bx[3] &&
                        ijk[2] >= bx[4] && ijk[2] < bx[5]) {
                        size_t nb = (size_t)(bx[1] - bx[0]) * (bx[3] - bx[2]) * (bx[5] - bx[4]);
                        size_t o = ((size_t)(ijk[2] - bx[4]) * (bx[3] - bx[2]) + (ijk[1] - bx[2])) *
                                       (bx[1] - bx[0]) + (ijk[0] - bx[0]);
                        for (int k = 0; k < 3; ++k) v[k] = pr->inner_v[k * nb + o];
                    }
                }
                out[0] = pr->inner_rho;
                out[1] = pr->inner_rho * v[0];
                out[2] = pr->inner_rho * v[1];
                out[3] = pr->inner_rho * v[2];
                out[4] = out[5] = out[6] = 0.0;
                out[7] = pr->inner_p / (g - 1.0) + 0.5 * pr->inner_rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            }
        }
        for (int v = 0; v < NV; ++v) Uout[v][i - NG] = out[v];
    }
    free(mem);
}

/* ------------------------------------------------------------------ */
/* Pencil extraction with boundary ghosts                              */
/* ------------------------------------------------------------------ */

static int wrap(int i, int N) { int r = i % N; return r < 0 ? r + N : r; }

/* Extended widths, centres and faces of axis a (length M, M, M+1). */
static void axis_geometry(const oracle_problem *pr, int a, double *dx, double *xc, double *xf)
{
    const int N = pr->n[a], M = N + 2 * NG;
    const double *f = pr->faces[a];
    for (int i = 0; i < M; ++i) {
        int gi = i - NG;
        double w;
        if (gi >= 0 && gi < N) w = f[gi + 1] - f[gi];
        else if (gi < 0) {
            if (pr->bc_lo[a] == BC_PERIODIC) { int s = wrap(gi, N); w = f[s + 1] - f[s]; }
            else { int s = -gi - 1; if (s > N - 1) s = N - 1; w = f[s + 1] - f[s]; }
        } else {
            if (pr->bc_hi[a] == BC_PERIODIC) { int s = wrap(gi, N); w = f[s + 1] - f[s]; }
            else { int s = 2 * N - 1 - gi; if (s < 0) s = 0; w = f[s + 1] - f[s]; }
        }
        dx[i] = w;
    }
    xf[NG] = f[0];
    for (int i = NG; i < M; ++i) xf[i + 1] = (i - NG < N) ? f[i - NG + 1] : xf[i] + dx[i];
    for (int i = NG - 1; i >= 0; --i) xf[i] = xf[i + 1] - dx[i];
    for (int i = 0; i < M; ++i) xc[i] = 0.5 * (xf[i] + xf[i + 1]);
}

static size_t lin(const int n[3], int i, int j, int k)
{
    return ((size_t)k * n[1] + j) * n[0] + i;
}

/* Index (i,j,k) of the zone at position s along axis a, transverse j1, j2. */
static void pencil_ijk(int a, int s, int j1, int j2, int ijk[3])
{
    ijk[a] = s;
    ijk[(a + 1) % 3] = j1;
    ijk[(a + 2) % 3] = j2;
}

static void inflow_conserved(const oracle_problem *pr, const double pos[3], double out[NV])
{
    double B[3];
    dipole_field(pr, pos, B);
    double rho = pr->inflow[0];
    double v[3] = {pr->inflow[1], pr->inflow[2], pr->inflow[3]};
    double bp[3] = {pr->inflow[4] - B[0], pr->inflow[5] - B[1], pr->inflow[6] - B[2]};
    double p = pr->inflow[7];
    out[0] = rho;
    for (int k = 0; k < 3; ++k) { out[1 + k] = rho * v[k]; out[4 + k] = bp[k]; }
    out[7] = p / (pr->gamma - 1.0) + 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) +
             0.5 * (bp[0] * bp[0] + bp[1] * bp[1] + bp[2] * bp[2]);
}

/* Fill the extended pencil (conserved values) from the 3D state. */
static void extract_pencil(const oracle_problem *pr, const double *U3, int a, int j1, int j2,
                           const double *xc_a, double c1, double c2, double *const P[NV])
{
    const int N = pr->n[a], M = N + 2 * NG;
    const size_t vol = (size_t)pr->n[0] * pr->n[1] * pr->n[2];
    for (int i = 0; i < M; ++i) {
        int gi = i - NG;
        int src = -1;
        int inflow = 0;
        if (gi >= 0 && gi < N) src = gi;
        else if (gi < 0) {
            if (pr->bc_lo[a] == BC_PERIODIC) src = wrap(gi, N);
            else if (pr->bc_lo[a] == BC_OUTFLOW) src = 0;
            else inflow = 1;
        } else {
            if (pr->bc_hi[a] == BC_PERIODIC) src = wrap(gi, N);
            else if (pr->bc_hi[a] == BC_OUTFLOW) src = N - 1;
            else inflow = 1;
        }
        if (inflow) {
            double pos[3], out[NV];
            pos[a] = xc_a[i]; pos[(a + 1) % 3] = c1; pos[(a + 2) % 3] = c2;
            inflow_conserved(pr, pos, out);
            for (int v = 0; v < NV; ++v) P[v][i] = out[v];
        } else {
            int ijk[3];
            pencil_ijk(a, src, j1, j2, ijk);
            size_t o = lin(pr->n, ijk[0], ijk[1], ijk[2]);
            for (int v = 0; v < NV; ++v) P[v][i] = U3[v * vol + o];
        }
    }
}

static int check_problem(const oracle_problem *pr, int axis)
{
    if (axis < 0 || axis > 2) return -1;
    for (int a = 0; a < 3; ++a) {
        if (pr->n[a] < 1) return -1;
        if ((pr->bc_lo[a] == BC_PERIODIC) != (pr->bc_hi[a] == BC_PERIODIC)) return -1;
        if (pr->bc_lo[a] != BC_PERIODIC && pr->n[a] < NG) return -1;
        for (int i = 0; i < pr->n[a]; ++i)
            if (!(pr->faces[a][i + 1] > pr->faces[a][i])) return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Public entry points                                                 */
/* ------------------------------------------------------------------ */

/* Sweep along `axis` over the whole grid, in place. Returns 0 or -1. */
int oracle_sweep(const oracle_problem *pr, double *U3, double dt, int axis, oracle_stats *st_out)
{
    if (check_problem(pr, axis) != 0 || !(dt > 0.0)) return -1;
    const int a = axis, t1 = (a + 1) % 3, t2 = (a + 2) % 3;
    const int N = pr->n[a], M = N + 2 * NG;
    const size_t vol = (size_t)pr->n[0] * pr->n[1] * pr->n[2];
    double *dx = malloc(sizeof(double) * (M + 1)), *xc = malloc(sizeof(double) * (M + 1));
    double *xf = malloc(sizeof(double) * (M + 2));
    axis_geometry(pr, a, dx, xc, xf);
    double *xc1 = malloc(sizeof(double) * pr->n[t1]), *xc2 = malloc(sizeof(double) * pr->n[t2]);
    for (int j = 0; j < pr->n[t1]; ++j) xc1[j] = 0.5 * (pr->faces[t1][j] + pr->faces[t1][j + 1]);
    for (int j = 0; j < pr->n[t2]; ++j) xc2[j] = 0.5 * (pr->faces[t2][j] + pr->faces[t2][j + 1]);
    double *src = malloc(sizeof(double) * NV * vol);
    memcpy(src, U3, sizeof(double) * NV * vol);
    const int npen = pr->n[t1] * pr->n[t2];
    oracle_stats tot;
    memset(&tot, 0, sizeof(tot));

#pragma omp parallel
    {
        oracle_stats loc;
        memset(&loc, 0, sizeof(loc));
        double *pbuf = malloc(sizeof(double) * NV * (M + 1));
        double *obuf = malloc(sizeof(double) * NV * (N + 1));
        double *P[NV], *O[NV];
        for (int v = 0; v < NV; ++v) { P[v] = pbuf + v * (M + 1); O[v] = obuf + v * (N + 1); }
#pragma omp for schedule(static)
        for (int pidx = 0; pidx < npen; ++pidx) {
            int j1 = pidx % pr->n[t1], j2 = pidx / pr->n[t1];
            extract_pencil(pr, src, a, j1, j2, xc, xc1[j1], xc2[j2], P);
            sweep_pencil(pr, a, N, j1, j2, P, dx, xc, xf, xc1[j1], xc2[j2], dt, O, &loc, NULL);
            for (int s = 0; s < N; ++s) {
                int ijk[3];
                pencil_ijk(a, s, j1, j2, ijk);
                size_t o = lin(pr->n, ijk[0], ijk[1], ijk[2]);
                for (int v = 0; v < NV; ++v) U3[v * vol + o] = O[v][s];
            }
        }
#pragma omp critical
        {
            for (int b = 0; b < 32; ++b) tot.iters_hist[b] += loc.iters_hist[b];
            tot.floor_hits += loc.floor_hits;
            tot.nonconverged += loc.nonconverged;
            tot.nonphys += loc.nonphys;
        }
        free(pbuf);
        free(obuf);
    }
    if (st_out) {
        for (int b = 0; b < 32; ++b) st_out->iters_hist[b] += tot.iters_hist[b];
        st_out->floor_hits += tot.floor_hits;
        st_out->nonconverged += tot.nonconverged;
        st_out->nonphys += tot.nonphys;
    }
    free(src); free(dx); free(xc); free(xf); free(xc1); free(xc2);
    return 0;
}

/* Sweep only the listed pencils (transverse indices j1[p], j2[p]) from the
 * state U3 (not modified); writes out[p][8][N]. */
int oracle_sweep_pencils(const oracle_problem *pr, const double *U3, double dt, int axis,
                         int npen, const int *j1s, const int *j2s, double *out, oracle_stats *st_out)
{
    if (check_problem(pr, axis) != 0 || !(dt > 0.0)) return -1;
    const int a = axis, t1 = (a + 1) % 3, t2 = (a + 2) % 3;
    const int N = pr->n[a], M = N + 2 * NG;
    double *dx = malloc(sizeof(double) * (M + 1)), *xc = malloc(sizeof(double) * (M + 1));
    double *xf = malloc(sizeof(double) * (M + 2));
    axis_geometry(pr, a, dx, xc, xf);
    oracle_stats tot;
    memset(&tot, 0, sizeof(tot));
    int bad = 0;
#pragma omp parallel
    {
        oracle_stats loc;
        memset(&loc, 0, sizeof(loc));
        double *pbuf = malloc(sizeof(double) * NV * (M + 1));
        double *P[NV], *O[NV];
        for (int v = 0; v < NV; ++v) P[v] = pbuf + v * (M + 1);
#pragma omp for schedule(static)
        for (int p = 0; p < npen; ++p) {
            int j1 = j1s[p], j2 = j2s[p];
            if (j1 < 0 || j1 >= pr->n[t1] || j2 < 0 || j2 >= pr->n[t2]) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            double c1 = 0.5 * (pr->faces[t1][j1] + pr->faces[t1][j1 + 1]);
            double c2 = 0.5 * (pr->faces[t2][j2] + pr->faces[t2][j2 + 1]);
            for (int v = 0; v < NV; ++v) O[v] = out + ((size_t)p * NV + v) * N;
            extract_pencil(pr, U3, a, j1, j2, xc, c1, c2, P);
            sweep_pencil(pr, a, N, j1, j2, P, dx, xc, xf, c1, c2, dt, O, &loc, NULL);
        }
#pragma omp critical
        {
            for (int b = 0; b < 32; ++b) tot.iters_hist[b] += loc.iters_hist[b];
            tot.floor_hits += loc.floor_hits;
            tot.nonconverged += loc.nonconverged;
            tot.nonphys += loc.nonphys;
        }
        free(pbuf);
    }
    if (st_out) {
        for (int b = 0; b < 32; ++b) st_out->iters_hist[b] += tot.iters_hist[b];
        st_out->floor_hits += tot.floor_hits;
        st_out->nonconverged += tot.nonconverged;
        st_out->nonphys += tot.nonphys;
    }
    free(dx); free(xc); free(xf);
    return bad ? -1 : 0;
}

/* Test hook (characteristic mode): sweep one pencil (j1, j2) of `axis` and
 * write the two primitive states (W_L, W_R, 7 values each, after the split
 * multi-D time-centring terms) of the linearised interface problem at every
 * face: out[14 * i ...] for the face between pencil zones i - NG and
 * i - NG + 1, i = 3 .. N + NG + 2; out holds 14 (N + 2 NG) values. */
int oracle_face_states(const oracle_problem *pr, const double *U3, double dt, int axis, int j1, int j2,
                       double *out)
{
    if (check_problem(pr, axis) != 0 || !(dt > 0.0) || pr->tracing != 1) return -1;
    const int a = axis, t1 = (a + 1) % 3, t2 = (a + 2) % 3;
    if (j1 < 0 || j1 >= pr->n[t1] || j2 < 0 || j2 >= pr->n[t2]) return -1;
    const int N = pr->n[a], M = N + 2 * NG;
    double *dx = malloc(sizeof(double) * (M + 1)), *xc = malloc(sizeof(double) * (M + 1));
    double *xf = malloc(sizeof(double) * (M + 2));
    double *pbuf = malloc(sizeof(double) * NV * (M + 1)), *obuf = malloc(sizeof(double) * NV * N);
    double *P[NV], *O[NV];
    for (int v = 0; v < NV; ++v) { P[v] = pbuf + v * (M + 1); O[v] = obuf + v * N; }
    axis_geometry(pr, a, dx, xc, xf);
    for (int i = 0; i < 14 * M; ++i) out[i] = 0.0;
    double c1 = 0.5 * (pr->faces[t1][j1] + pr->faces[t1][j1 + 1]);
    double c2 = 0.5 * (pr->faces[t2][j2] + pr->faces[t2][j2 + 1]);
    oracle_stats loc;
    memset(&loc, 0, sizeof(loc));
    extract_pencil(pr, U3, a, j1, j2, xc, c1, c2, P);
    sweep_pencil(pr, a, N, j1, j2, P, dx, xc, xf, c1, c2, dt, O, &loc, out);
    free(dx); free(xc); free(xf); free(pbuf); free(obuf);
    return 0;
}

/* One split step: x, y, z sweeps on even steps, z, y, x on odd steps, all
 * with the same dt (alternating order keeps the splitting error second
 * order for oblique waves). */
int oracle_step(const oracle_problem *pr, double *U3, double dt, long long step_index,
                oracle_stats *st)
{
    static const int even[3] = {0, 1, 2}, odd[3] = {2, 1, 0};
    const int *ord = (step_index % 2 == 0) ? even : odd;
    for (int s = 0; s < 3; ++s)
        if (oracle_sweep(pr, U3, dt, ord[s], st) != 0) return -1;
    return 0;
}

/* Largest stable dt: CFL / max over unmasked zones of
 * max_a (|v_a| + c_f,a) / dx_a, c_f,a the fast speed along axis a computed
 * with the total field. */
double oracle_cfl_dt(const oracle_problem *pr, const double *U3, double cfl)
{
    const size_t vol = (size_t)pr->n[0] * pr->n[1] * pr->n[2];
    const double g = pr->gamma;
    double smax = 0.0;
    for (int k = 0; k < pr->n[2]; ++k)
        for (int j = 0; j < pr->n[1]; ++j)
            for (int i = 0; i < pr->n[0]; ++i) {
                int id[3] = {i, j, k};
                double pos[3], w[3];
                for (int a = 0; a < 3; ++a) {
                    pos[a] = 0.5 * (pr->faces[a][id[a]] + pr->faces[a][id[a] + 1]);
                    w[a] = pr->faces[a][id[a] + 1] - pr->faces[a][id[a]];
                }
                if (pr->r_inner > 0.0 &&
                    sqrt(pos[0] * pos[0] + pos[1] * pos[1] + pos[2] * pos[2]) < pr->r_inner)
                    continue;
                size_t o = lin(pr->n, i, j, k);
                double rho = U3[o];
                double v[3], bp[3], B[3], Bd[3];
                for (int a = 0; a < 3; ++a) { v[a] = U3[(1 + a) * vol + o] / rho; bp[a] = U3[(4 + a) * vol + o]; }
                dipole_field(pr, pos, Bd);
                for (int a = 0; a < 3; ++a) B[a] = Bd[a] + bp[a];
                double p = (g - 1.0) * (U3[7 * vol + o] - 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) -
                                        0.5 * (bp[0] * bp[0] + bp[1] * bp[1] + bp[2] * bp[2]));
                if (p < pr->p_floor) p = pr->p_floor;
                double a2 = g * p / rho;
                double b2 = (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]) / rho;
                for (int a = 0; a < 3; ++a) {
                    double ba2 = B[a] * B[a] / rho;
                    double disc = (a2 + b2) * (a2 + b2) - 4.0 * a2 * ba2;
                    if (disc < 0.0) disc = 0.0;
                    double cf = sqrt(0.5 * (a2 + b2 + sqrt(disc)));
                    double s = (fabs(v[a]) + cf) / w[a];
                    if (s > smax) smax = s;
                }
            }
    return smax > 0.0 ? cfl / smax : 0.0;
}

/* Volume integrals of the 8 conserved variables (plain ordered sum). */
void oracle_totals(const oracle_problem *pr, const double *U3, double out[NV])
{
    const size_t vol = (size_t)pr->n[0] * pr->n[1] * pr->n[2];
    for (int v = 0; v < NV; ++v) out[v] = 0.0;
    for (int k = 0; k < pr->n[2]; ++k)
        for (int j = 0; j < pr->n[1]; ++j)
            for (int i = 0; i < pr->n[0]; ++i) {
                double dv = (pr->faces[0][i + 1] - pr->faces[0][i]) *
                            (pr->faces[1][j + 1] - pr->faces[1][j]) *
                            (pr->faces[2][k + 1] - pr->faces[2][k]);
                size_t o = lin(pr->n, i, j, k);
                for (int v = 0; v < NV; ++v) out[v] += U3[v * vol + o] * dv;
            }
}

/* ------------------------------------------------------------------ */
/* Unit-level entry points used by the pins                            */
/* ------------------------------------------------------------------ */

/* Edge values a_{j+1/2} (written to edge[j]) for j in [1, M-3]. */
void oracle_ppm_edges(int M, const double *a, const double *w, int limit, double *edge)
{
    double *slope = malloc(sizeof(double) * M);
    ppm_edges(M, a, w, limit, slope, edge);
    free(slope);
}

/* Limited slopes (CW84 1.7 + 1.8) for j in [1, M-2]. */
void oracle_ppm_slopes(int M, const double *a, const double *w, int limit, double *slope)
{
    for (int j = 0; j < M; ++j) slope[j] = 0.0;
    for (int j = 1; j <= M - 2; ++j) slope[j] = cw84_slope(a, w, j, limit);
}

/* Parabola coefficients for zones j in [2, M-3]; out is [3][M]. */
void oracle_ppm_parabolas(int M, const double *a, const double *w, const double *flat,
                          int limit, int monot, double *out)
{
    double *slope = malloc(sizeof(double) * M), *edge = malloc(sizeof(double) * M);
    ppm_edges(M, a, w, limit, slope, edge);
    for (int j = 0; j < 3 * M; ++j) out[j] = 0.0;
    for (int j = 2; j <= M - 3; ++j)
        ppm_parabola(a[j], edge[j - 1], edge[j], flat ? flat[j] : 0.0, monot,
                     &out[j], &out[M + j], &out[2 * M + j]);
    free(slope);
    free(edge);
}

/* Test hooks of the full characteristic tracing: the eigen-structure at a
 * state (lam[7], R row-major [7][7]) and the traced face states of one zone
 * from its parabolas (a[7][3] = aL, dA, a6 per primitive). */
void oracle_mhd7_eigen(double rho, double p, double g, double Bn, double Bt1, double Bt2, double *lam, double *Rflat)
{
    double R[7][7];
    mhd7_eigen(rho, p, g, Bn, Bt1, Bt2, lam, R);
    for (int i = 0; i < 7; ++i)
        for (int k = 0; k < 7; ++k) Rflat[i * 7 + k] = R[i][k];
}

int oracle_riemann7(const double *WL, const double *WR, double g, double Bn, double Bd1, double Bd2, double *Ws)
{
    return riemann7(WL, WR, g, Bn, Bd1, Bd2, Ws);
}

int oracle_trace7(double rho, double p, double g, double Bn, double Bt1, double Bt2, const double *par, double dt,
                  double dm, double *WL, double *WR)
{
    double lam[7], R[7][7], Li[7][7], aL[7], dA[7], a6[7];
    mhd7_eigen(rho, p, g, Bn, Bt1, Bt2, lam, R);
    if (invert7(R, Li) != 0) return -1;
    for (int v = 0; v < 7; ++v) { aL[v] = par[v * 3]; dA[v] = par[v * 3 + 1]; a6[v] = par[v * 3 + 2]; }
    trace7(aL, dA, a6, lam, R, Li, dt, dm, WL, WR);
    return 0;
}

double oracle_par_avg(double aL, double dA, double a6, double y, int right_part)
{
    return right_part ? par_avg_right_part(aL, dA, a6, y) : par_avg_left_part(aL, dA, a6, y);
}

void oracle_flattening(int M, const double *Pt, const double *Pa, const double *un, const double *rho, double *f)
{
    double *ft = malloc(sizeof(double) * M);
    flattening(M, Pt, Pa, un, rho, ft, f);
    free(ft);
}

int oracle_riemann_normal(double PtL, double PtR, double Pd, double uL, double uR,
                          double CL, double CR, double gL, double gR, double tol, int max_iter,
                          double *Pstar, double *ustar, int *converged)
{
    return riemann_normal(PtL, PtR, Pd, uL, uR, CL, CR, gL, gR, tol, max_iter, Pstar, ustar, converged);
}

void oracle_riemann_alfven(double rL, double rR, double sigma, double vL, double vR,
                           double bL, double bR, double *vstar, double *bstar)
{
    riemann_alfven(rL, rR, sigma, vL, vR, bL, bR, vstar, bstar);
}

void oracle_dipole(const oracle_problem *pr, const double r[3], double B[3])
{
    dipole_field(pr, r, B);
}

int oracle_ghosts(void) { return NG; }

/* Host threads of the pencil loops (timing only; results do not depend on
 * it: each pencil is computed by one thread). */
#ifdef _OPENMP
#include <omp.h>
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_get_threads(void) { return omp_get_max_threads(); }
#else
void oracle_set_threads(int n) { (void)n; }
int oracle_get_threads(void) { return 1; }
#endif
