// ppmlr_iono.hpp -- the ionosphere shell coupling on the device (paper,
// Section II: a thin shell at r = 1.017 R_E closes the field-aligned
// currents under the electrostatic assumption; the potential solved on it is
// carried along dipole field lines to the magnetospheric inner boundary,
// where it sets the flow).
//
// Three kernels, FP64 throughout (a few thousand shell cells and the zones
// inside the inner boundary: negligible next to a sweep):
//   iono_fac_kernel    one thread per shell cell: J = curl B' at the zone
//                      centres around the point where the cell's field line
//                      crosses r_fac (central differences, trilinear
//                      interpolation), its component along the dipole, and
//                      the radial current density that reaches the shell
//                      (J_par / |B| is constant along a flux tube);
//   iono_solve_kernel  one workgroup per hemisphere: finite volumes for
//                      div_h(Sigma grad_h Phi) = j_r on the polar cap whose
//                      field lines cross r_fac (Phi = 0 at its edge), solved
//                      directly in LDS (Fourier transform in longitude, one
//                      tridiagonal system per mode in colatitude);
//   iono_drift_kernel  one thread per zone of the index box around the
//                      inner boundary: the shell potential at the footpoint
//                      of the zone's field line and of its six neighbours,
//                      E = -grad Phi by central differences, v = E x B_d /
//                      |B_d|^2.
// The sweep's inner reset then gives the zones inside r_inner this drift.
#pragma once
#include <hip/hip_runtime.h>

namespace ppmlr {

constexpr int kIonoMaxCells = 4096;   // cells per cap (the solve's arrays in LDS)
constexpr int kIonoThreads = 1024;    // threads of the solve's workgroup

struct IonoArgs {
    const void *u;                     // state, SoA [8][nz][ny][nx] (T)
    long long vol;
    int nx, ny, nz;
    const double *xc, *yc, *zc;        // zone centres (FP64)
    double M, mdir[3];                 // dipole moment and unit direction
    double xm[3], ym[3], zm[3];        // magnetic frame (z_m opposite to the moment)
    int nt, nph;                       // cells per cap: colatitude rings, longitudes
    double r_shell, r_fac, theta_c, dth, dph, sigma;
    double *jr;                        // [2][nt][nph] radial current density at the shell
    double *phi;                       // [2][nt][nph] shell potential
    double *pole;                      // [2] mean of the first ring (value at the pole)
    double r_inner2;
    int box[6];                        // i0, i1, j0, j1, k0, k1 (half-open)
    double *v;                         // [3][box] drift of the reset zones
};

__device__ inline void iono_dipole(const IonoArgs &a, double x, double y, double z, double B[3])
{
    const double r2 = x * x + y * y + z * z;
    const double rr = sqrt(r2);
    const double r3 = r2 * rr, r5 = r3 * r2;
    const double mr = a.mdir[0] * x + a.mdir[1] * y + a.mdir[2] * z;
    B[0] = a.M * (3.0 * mr * x / r5 - a.mdir[0] / r3);
    B[1] = a.M * (3.0 * mr * y / r5 - a.mdir[1] / r3);
    B[2] = a.M * (3.0 * mr * z / r5 - a.mdir[2] / r3);
}

// Largest i with c[i] <= p, at most n - 2 (the caller keeps p inside the
// centres), and the weight of c[i + 1].
__device__ inline int iono_locate(const double *c, int n, double p, double &w)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (c[mid] <= p) lo = mid; else hi = mid - 1;
    }
    if (lo > n - 2) lo = n - 2;
    w = (p - c[lo]) / (c[lo + 1] - c[lo]);
    return lo;
}

template <typename T>
__device__ inline double iono_b(const IonoArgs &a, int v, int i, int j, int k)
{
    return (double)static_cast<const T *>(a.u)[(size_t)v * a.vol + ((size_t)k * a.ny + j) * a.nx + i];
}

// curl B' at zone (i, j, k) by central differences; zero in the outermost layer.
template <typename T>
__device__ inline void iono_curl(const IonoArgs &a, int i, int j, int k, double J[3])
{
    if (i < 1 || i > a.nx - 2 || j < 1 || j > a.ny - 2 || k < 1 || k > a.nz - 2) {
        J[0] = J[1] = J[2] = 0.0;
        return;
    }
    const double dx = a.xc[i + 1] - a.xc[i - 1], dy = a.yc[j + 1] - a.yc[j - 1], dz = a.zc[k + 1] - a.zc[k - 1];
    const double dBz_dy = (iono_b<T>(a, 6, i, j + 1, k) - iono_b<T>(a, 6, i, j - 1, k)) / dy;
    const double dBy_dz = (iono_b<T>(a, 5, i, j, k + 1) - iono_b<T>(a, 5, i, j, k - 1)) / dz;
    const double dBx_dz = (iono_b<T>(a, 4, i, j, k + 1) - iono_b<T>(a, 4, i, j, k - 1)) / dz;
    const double dBz_dx = (iono_b<T>(a, 6, i + 1, j, k) - iono_b<T>(a, 6, i - 1, j, k)) / dx;
    const double dBy_dx = (iono_b<T>(a, 5, i + 1, j, k) - iono_b<T>(a, 5, i - 1, j, k)) / dx;
    const double dBx_dy = (iono_b<T>(a, 4, i, j + 1, k) - iono_b<T>(a, 4, i, j - 1, k)) / dy;
    J[0] = dBz_dy - dBy_dz;
    J[1] = dBx_dz - dBz_dx;
    J[2] = dBy_dx - dBx_dy;
}

template <typename T>
__global__ void __launch_bounds__(256) iono_fac_kernel(IonoArgs a)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncell = a.nt * a.nph;
    if (t >= 2 * ncell) return;
    const int h = t / ncell, q = t - h * ncell, k = q / a.nph, j = q - k * a.nph;
    const double th = (k + 0.5) * a.dth, ph = (j + 0.5) * a.dph;
    const double sgn = h == 0 ? 1.0 : -1.0;
    const double st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
    double rs[3], P[3];
    const double sf = st * sqrt(a.r_fac / a.r_shell);
    const double cf = sqrt(fmax(0.0, 1.0 - sf * sf));
    for (int d = 0; d < 3; ++d) {
        rs[d] = st * cp * a.xm[d] + st * sp * a.ym[d] + sgn * ct * a.zm[d];
        P[d] = a.r_fac * (sf * cp * a.xm[d] + sf * sp * a.ym[d] + sgn * cf * a.zm[d]);
    }
    // trilinear interpolation of curl B' between the 8 zone centres around P
    double wx, wy, wz;
    const int i0 = iono_locate(a.xc, a.nx, P[0], wx);
    const int j0 = iono_locate(a.yc, a.ny, P[1], wy);
    const int k0 = iono_locate(a.zc, a.nz, P[2], wz);
    double JP[3] = {0.0, 0.0, 0.0};
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                const double wt = (di ? wx : 1.0 - wx) * (dj ? wy : 1.0 - wy) * (dk ? wz : 1.0 - wz);
                double J[3];
                iono_curl<T>(a, i0 + di, j0 + dj, k0 + dk, J);
                for (int d = 0; d < 3; ++d) JP[d] += wt * J[d];
            }
    double BP[3], Bs[3];
    iono_dipole(a, P[0], P[1], P[2], BP);
    iono_dipole(a, a.r_shell * rs[0], a.r_shell * rs[1], a.r_shell * rs[2], Bs);
    const double nP = sqrt(BP[0] * BP[0] + BP[1] * BP[1] + BP[2] * BP[2]);
    const double ns = sqrt(Bs[0] * Bs[0] + Bs[1] * Bs[1] + Bs[2] * Bs[2]);
    const double jpar = (JP[0] * BP[0] + JP[1] * BP[1] + JP[2] * BP[2]) / nP;
    a.jr[t] = jpar * (ns / nP) * (Bs[0] * rs[0] + Bs[1] * rs[1] + Bs[2] * rs[2]) / ns;
}

// One workgroup per hemisphere: the potential on the cap by a direct solve.
// With a uniform conductance the finite-volume operator separates: along
// longitude it is the circulant second difference b_k (P_{j+1} - 2 P_j +
// P_{j-1}), so a discrete Fourier transform in longitude turns it into
// b_k (2 cos(2 pi m / n_phi) - 2) for mode m, and what remains for each mode
// is a tridiagonal system in colatitude,
//   cN_k P_{k-1} + cS_k P_{k+1} - (cN_k + cS_k + 2 b_k (1 - cos(2 pi m / n_phi))) P_k = F_k
// (cN_0 = 0 at the pole; for the last ring cS is the edge term on the
// diagonal alone, Phi = 0 half a cell outside), solved by elimination; the
// inverse transform gives Phi.  LDS: the complex right-hand side / solution
// [n_theta][n_phi] (re, im), the Thomas factors [n_phi][n_theta], the
// per-ring coefficients and the twiddles.
__global__ void __launch_bounds__(kIonoThreads) iono_solve_kernel(IonoArgs a)
{
    extern __shared__ __align__(16) double sm[];
    const int h = blockIdx.x;
    const int nt = a.nt, nph = a.nph, N = nt * nph;
    double *re = sm, *im = sm + N;                     // [k][m]
    double *cp = sm + 2 * N;                           // Thomas factors [m][k]
    double *cS = cp + N, *cN = cS + nt, *cB = cN + nt;
    double *tc = cB + nt, *ts = tc + nph;              // cos, sin of 2 pi t / n_phi
    double *src = ts + nph;                            // right-hand side [k][j]
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int k = tid; k < nt; k += nthr) {
        cS[k] = k + 1 < nt ? sin((k + 1) * a.dth) * a.dph / a.dth : sin(a.theta_c) * a.dph / (0.5 * a.dth);
        cN[k] = k > 0 ? sin(k * a.dth) * a.dph / a.dth : 0.0;
        cB[k] = a.dth / (sin((k + 0.5) * a.dth) * a.dph);
    }
    for (int t = tid; t < nph; t += nthr) {
        tc[t] = cos(2.0 * M_PI * t / nph);
        ts[t] = sin(2.0 * M_PI * t / nph);
    }
    const double *jr = a.jr + (size_t)h * N;
    for (int q = tid; q < N; q += nthr) {
        const int k = q / nph;
        const double area = a.r_shell * a.r_shell * (cos(k * a.dth) - cos((k + 1) * a.dth)) * a.dph;
        src[q] = jr[q] * area / a.sigma;
    }
    __syncthreads();
    // forward transform along longitude: F[k][m] = sum_j src[k][j] e^{-2 pi i m j / n_phi}
    for (int q = tid; q < N; q += nthr) {
        const int k = q / nph, m = q - k * nph;
        double sr = 0.0, si = 0.0;
        for (int j = 0; j < nph; ++j) {
            const int t = (m * j) % nph;
            sr += src[k * nph + j] * tc[t];
            si -= src[k * nph + j] * ts[t];
        }
        re[q] = sr;
        im[q] = si;
    }
    __syncthreads();
    // one tridiagonal system per mode (the same real matrix for both parts)
    for (int m = tid; m < nph; m += nthr) {
        const double lam = 2.0 * (1.0 - tc[m]);
        double prev_c = 0.0, prev_r = 0.0, prev_i = 0.0;
        for (int k = 0; k < nt; ++k) {
            const double diag = -(cN[k] + cS[k] + cB[k] * lam);
            const double lower = cN[k];                       // coefficient of P_{k-1}
            const double upper = k + 1 < nt ? cS[k] : 0.0;    // of P_{k+1}
            const double den = diag - lower * prev_c;
            const double c = upper / den;
            const double r = (re[k * nph + m] - lower * prev_r) / den;
            const double i = (im[k * nph + m] - lower * prev_i) / den;
            cp[m * nt + k] = c;
            re[k * nph + m] = r;
            im[k * nph + m] = i;
            prev_c = c;
            prev_r = r;
            prev_i = i;
        }
        for (int k = nt - 2; k >= 0; --k) {
            const double c = cp[m * nt + k];
            re[k * nph + m] -= c * re[(k + 1) * nph + m];
            im[k * nph + m] -= c * im[(k + 1) * nph + m];
        }
    }
    __syncthreads();
    // inverse transform: Phi[k][j] = (1 / n_phi) Re sum_m P[k][m] e^{2 pi i m j / n_phi}
    double *out = a.phi + (size_t)h * N;
    for (int q = tid; q < N; q += nthr) {
        const int k = q / nph, j = q - k * nph;
        double s = 0.0;
        for (int m = 0; m < nph; ++m) {
            const int t = (m * j) % nph;
            s += re[k * nph + m] * tc[t] - im[k * nph + m] * ts[t];
        }
        src[q] = s / nph;
        out[q] = s / nph;
    }
    __syncthreads();
    if (tid == 0) {
        double ring0 = 0.0;
        for (int j = 0; j < nph; ++j) ring0 += src[j];
        a.pole[h] = ring0 / nph;
    }
}

// Shell potential carried along the dipole field line through (x, y, z);
// false inside the shell.
__device__ inline bool iono_phi_at(const IonoArgs &a, const double *pos, double &out)
{
    const double r = sqrt(pos[0] * pos[0] + pos[1] * pos[1] + pos[2] * pos[2]);
    if (r <= a.r_shell) return false;
    const double x = pos[0] * a.xm[0] + pos[1] * a.xm[1] + pos[2] * a.xm[2];
    const double y = pos[0] * a.ym[0] + pos[1] * a.ym[1] + pos[2] * a.ym[2];
    const double z = pos[0] * a.zm[0] + pos[1] * a.zm[1] + pos[2] * a.zm[2];
    const double s2 = (a.r_shell / r) * (x * x + y * y) / (r * r);
    const double sc = sin(a.theta_c);
    if (s2 > sc * sc) { out = 0.0; return true; }
    const double th = asin(sqrt(s2));
    double ph = atan2(y, x);
    if (ph < 0.0) ph += 2.0 * M_PI;
    const int h = z >= 0.0 ? 0 : 1;
    const double *f = a.phi + (size_t)h * a.nt * a.nph;
    const double sj = ph / a.dph - 0.5;
    const double fj = floor(sj);
    const double wj = sj - fj;
    int j0 = (int)fj % a.nph;
    if (j0 < 0) j0 += a.nph;
    const int j1 = j0 + 1 < a.nph ? j0 + 1 : 0;
    auto ring = [&](int k) { return (1.0 - wj) * f[k * a.nph + j0] + wj * f[k * a.nph + j1]; };
    const double t = th / a.dth - 0.5;
    if (t < 0.0) {
        const double w = (t + 0.5) / 0.5;
        out = (1.0 - w) * a.pole[h] + w * ring(0);
    } else if (t > a.nt - 1) {
        const double w = (t - (a.nt - 1)) / 0.5;
        out = (1.0 - w) * ring(a.nt - 1);
    } else {
        const int k = (int)floor(t);
        const double w = t - k;
        out = (1.0 - w) * ring(k) + w * ring(k + 1);
    }
    return true;
}

__global__ void __launch_bounds__(256) iono_drift_kernel(IonoArgs a)
{
    const int bi = a.box[1] - a.box[0], bj = a.box[3] - a.box[2], bk = a.box[5] - a.box[4];
    const long long nb = (long long)bi * bj * bk;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb) return;
    const int ii = (int)(t % bi), jj = (int)((t / bi) % bj), kk = (int)(t / ((long long)bi * bj));
    const int i = a.box[0] + ii, j = a.box[2] + jj, k = a.box[4] + kk;
    double v[3] = {0.0, 0.0, 0.0};
    const double pos[3] = {a.xc[i], a.yc[j], a.zc[k]};
    const int idx[3] = {i, j, k}, n[3] = {a.nx, a.ny, a.nz};
    const double *cs[3] = {a.xc, a.yc, a.zc};
    bool ok = pos[0] * pos[0] + pos[1] * pos[1] + pos[2] * pos[2] < a.r_inner2;
    double E[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < 3 && ok; ++d) {
        if (idx[d] == 0 || idx[d] == n[d] - 1) { ok = false; break; }
        double pp[3] = {pos[0], pos[1], pos[2]}, pm[3] = {pos[0], pos[1], pos[2]};
        pp[d] = cs[d][idx[d] + 1];
        pm[d] = cs[d][idx[d] - 1];
        double fp, fm, f0;
        if (!iono_phi_at(a, pp, fp) || !iono_phi_at(a, pm, fm) || !iono_phi_at(a, pos, f0)) { ok = false; break; }
        E[d] = -(fp - fm) / (pp[d] - pm[d]);
    }
    if (ok) {
        double B[3];
        iono_dipole(a, pos[0], pos[1], pos[2], B);
        const double b2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
        v[0] = (E[1] * B[2] - E[2] * B[1]) / b2;
        v[1] = (E[2] * B[0] - E[0] * B[2]) / b2;
        v[2] = (E[0] * B[1] - E[1] * B[0]) / b2;
    }
    a.v[t] = v[0];
    a.v[nb + t] = v[1];
    a.v[2 * nb + t] = v[2];
}

}  // namespace ppmlr
