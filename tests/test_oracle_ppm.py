"""Pins of the oracle's parabolic reconstruction against closed forms.

The paper (Section II) reconstructs each zone by a parabola continuous within
the zone; the oracle uses Colella & Woodward (1984) Eqs. 1.6-1.8, 1.10, 1.12.
None of these checks re-types the oracle's formulas: each compares against
exact integrals of polynomials, Gauss quadrature, or an invariant.
"""
import numpy as np
import pytest

from oracle import oracle as O


def _grid(rng, M, lo=0.3, hi=2.5):
    w = rng.uniform(lo, hi, M)
    xf = np.concatenate([[0.0], np.cumsum(w)])
    return w, xf


@pytest.mark.parametrize("seed", range(5))
def test_edges_exact_for_cubics_on_random_nonuniform_grids(seed):
    # The edge value is the derivative of the quartic interpolating the
    # cumulative integral, so it reproduces any cubic profile exactly.
    rng = np.random.default_rng(seed)
    M = 24
    w, xf = _grid(rng, M)
    c = rng.uniform(-1, 1, 4)
    F = lambda x: c[0] * x + c[1] * x ** 2 / 2 + c[2] * x ** 3 / 3 + c[3] * x ** 4 / 4
    f = lambda x: c[0] + c[1] * x + c[2] * x ** 2 + c[3] * x ** 3
    a = (F(xf[1:]) - F(xf[:-1])) / w
    e = O.ppm_edges(a, w, limit=False)
    j = np.arange(1, M - 2)
    scale = np.max(np.abs(f(xf)))
    assert np.max(np.abs(e[j] - f(xf[j + 1]))) <= 1e-13 * scale


def test_uniform_grid_reduces_to_fourth_order_stencil():
    rng = np.random.default_rng(7)
    a = rng.normal(size=30)
    w = np.full(30, 0.37)
    e = O.ppm_edges(a, w, limit=False)
    j = np.arange(1, 27)
    ref = 7.0 / 12.0 * (a[j] + a[j + 1]) - 1.0 / 12.0 * (a[j - 1] + a[j + 2])
    assert np.max(np.abs(e[j] - ref)) < 1e-14


@pytest.mark.parametrize("seed", range(3))
def test_unlimited_slope_is_edge_difference_for_quadratics(seed):
    rng = np.random.default_rng(100 + seed)
    M = 20
    w, xf = _grid(rng, M)
    c = rng.uniform(-1, 1, 3)
    F = lambda x: c[0] * x + c[1] * x ** 2 / 2 + c[2] * x ** 3 / 3
    f = lambda x: c[0] + c[1] * x + c[2] * x ** 2
    a = (F(xf[1:]) - F(xf[:-1])) / w
    s = O.ppm_slopes(a, w, limit=False)
    j = np.arange(1, M - 1)
    scale = np.max(np.abs(f(xf)))
    assert np.max(np.abs(s[j] - (f(xf[j + 1]) - f(xf[j])))) < 1e-13 * scale


@pytest.mark.parametrize("seed", range(10))
def test_limited_edges_create_no_new_extrema(seed):
    rng = np.random.default_rng(200 + seed)
    M = 40
    w, _ = _grid(rng, M)
    a = np.cumsum(rng.normal(size=M)) + 3 * (rng.uniform(size=M) < 0.2) * rng.normal(size=M)
    e = O.ppm_edges(a, w, limit=True)
    j = np.arange(1, M - 2)
    lo = np.minimum(a[j], a[j + 1])
    hi = np.maximum(a[j], a[j + 1])
    assert np.all(e[j] >= lo - 1e-12) and np.all(e[j] <= hi + 1e-12)


@pytest.mark.parametrize("seed", range(10))
def test_monotonised_parabolas_are_monotone_and_conservative(seed):
    rng = np.random.default_rng(300 + seed)
    M = 40
    w, _ = _grid(rng, M)
    a = rng.normal(size=M)
    par = O.ppm_parabolas(a, w)
    xg, wg = np.polynomial.legendre.leggauss(6)
    xg = 0.5 * (xg + 1.0)
    wg = 0.5 * wg
    for j in range(2, M - 2):
        aL, dA, a6 = par[:, j]
        prof = lambda x: aL + x * (dA + a6 * (1.0 - x))
        # zone average preserved
        assert abs(np.sum(wg * prof(xg)) - a[j]) < 1e-13 * (1 + abs(a[j]))
        # no interior extremum: derivative dA + a6 (1 - 2x) keeps one sign
        d0, d1 = dA + a6, dA - a6
        assert d0 * d1 >= -1e-12 * (1 + dA * dA + a6 * a6)
        # range of the parabola inside the neighbours' range
        lo = min(a[j - 1], a[j], a[j + 1]) - 1e-12
        hi = max(a[j - 1], a[j], a[j + 1]) + 1e-12
        xs = np.linspace(0, 1, 21)
        assert np.all(prof(xs) >= lo) and np.all(prof(xs) <= hi)


@pytest.mark.parametrize("y", [0.0, 0.05, 0.3, 0.77, 1.0])
def test_domain_of_dependence_averages_match_quadrature(y):
    rng = np.random.default_rng(11)
    xg, wg = np.polynomial.legendre.leggauss(8)
    for _ in range(20):
        aL, dA, a6 = rng.normal(size=3)
        prof = lambda x: aL + x * (dA + a6 * (1.0 - x))
        if y == 0.0:
            ref_r = aL + dA
            ref_l = aL
        else:
            # average over [1-y, 1] and over [0, y]
            xr = 1.0 - y + 0.5 * y * (xg + 1.0)
            xl = 0.5 * y * (xg + 1.0)
            ref_r = 0.5 * np.sum(wg * prof(xr))
            ref_l = 0.5 * np.sum(wg * prof(xl))
        assert abs(O.par_avg(aL, dA, a6, y, True) - ref_r) < 1e-14 * (1 + abs(ref_r))
        assert abs(O.par_avg(aL, dA, a6, y, False) - ref_l) < 1e-14 * (1 + abs(ref_l))


def test_uniform_data_gives_flat_parabolas_bitwise():
    rng = np.random.default_rng(3)
    w, _ = _grid(rng, 30)
    a = np.full(30, 0.123456789)
    par = O.ppm_parabolas(a, w)
    assert np.all(par[0, 2:28] == a[0])
    assert np.all(par[1, 2:28] == 0.0)
    assert np.all(par[2, 2:28] == 0.0)
    for y in (0.0, 0.3, 1.0):
        assert O.par_avg(a[0], 0.0, 0.0, y, True) == a[0]
        assert O.par_avg(a[0], 0.0, 0.0, y, False) == a[0]


def test_flattening_off_for_smooth_data_and_on_at_a_sharp_shock():
    M = 40
    x = np.arange(M)
    # smooth compression: small relative jumps -> no flattening
    Pt = 1.0 + 0.01 * np.sin(2 * np.pi * x / M)
    un = -0.01 * np.sin(2 * np.pi * x / M)
    f = O.flattening(Pt, Pt, un)
    assert np.all(f == 0.0)
    # strong compressive jump over one zone -> full flattening near it
    Pt = np.where(x < 20, 10.0, 1.0)
    un = np.where(x < 20, 1.0, 0.0)
    f = O.flattening(Pt, Pt, un)
    assert f[19] == 1.0 and f[20] == 1.0
    assert np.all(f[:15] == 0.0) and np.all(f[25:] == 0.0)
    # expansion (diverging flow) is never flattened
    f = O.flattening(Pt, Pt, -un)
    assert np.all(f == 0.0)


def test_flattening_compression_margin_at_a_jump_at_rest():
    # a strong pressure jump at rest: equal velocities, or velocities that
    # differ by rounding noise, never flatten; a compression well above the
    # margin (1e-5 of sqrt(P/rho)) does
    M = 40
    x = np.arange(M)
    Pt = np.where(x < 20, 20.0, 1.0)
    rho = np.where(x < 20, 2.0, 1.0)
    # (velocities falling along the pencil: a compression at noise level)
    for un in (np.zeros(M), 1e-18 * (M - x), 1e-9 * (M - x) / M):
        assert np.all(O.flattening(Pt, Pt, un, rho) == 0.0)
    un = np.where(x < 20, 1e-3, 0.0)
    f = O.flattening(Pt, Pt, un, rho)
    assert f[19] > 0.0 and f[20] > 0.0


def test_parabolas_with_full_flattening_are_constant():
    rng = np.random.default_rng(5)
    w, _ = _grid(rng, 20)
    a = rng.normal(size=20)
    par = O.ppm_parabolas(a, w, flat=np.ones(20))
    assert np.allclose(par[0, 2:18], a[2:18], rtol=0, atol=1e-15)
    assert np.allclose(par[1:, 2:18], 0.0, atol=1e-15)


def test_flattening_constants_measured_from_outside_match_cw84():
    # Colella & Woodward (1984), appendix, give the shock detector's constants
    # as epsilon = 0.33 (relative pressure jump that counts as a shock),
    # omega1 = 0.75 and omega2 = 10 (the coefficient rises from 0 to 1 as the
    # ratio of the 2-zone to the 4-zone pressure difference goes from omega1
    # to omega1 + 1/omega2).  The oracle is probed as a black box with
    # compressive steps, and the three numbers are measured from its output.
    M, j = 15, 7
    i = np.arange(M)
    un = np.where(i < j, 1.0, 0.0)

    def step(PL, D, w):
        return PL + D * 0.5 * (1.0 + np.tanh((i - j) / w))

    # epsilon: a sharp step (ratio ~1, full flattening once detected); the
    # jump at which the coefficient turns on, relative to the lower pressure
    PL, lo, hi = 2.0, 0.1, 1.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        Pt = step(PL, mid * PL, 0.05)
        if np.max(O.flattening(Pt, Pt, un)) > 0.0:
            hi = mid
        else:
            lo = mid
    assert abs(hi - 0.33) < 1e-12, hi
    # omega1, omega2: steps of growing width lower the central ratio
    # r = (P_{j+1} - P_{j-1}) / (P_{j+2} - P_{j-2}); the coefficient's peak
    # against r is a ramp whose zero and slope are the constants
    rs, fs = [], []
    for w in np.linspace(0.3, 1.2, 40):
        Pt = step(PL, 3.0 * PL, w)
        rs.append((Pt[j + 1] - Pt[j - 1]) / (Pt[j + 2] - Pt[j - 2]))
        fs.append(np.max(O.flattening(Pt, Pt, un)))
    rs, fs = np.array(rs), np.array(fs)
    ramp = (fs > 0.0) & (fs < 1.0)
    assert ramp.sum() >= 8
    k, c = np.polyfit(rs[ramp], fs[ramp], 1)
    assert abs(k - 10.0) < 1e-9 and abs(-c / k - 0.75) < 1e-12, (k, -c / k)
    assert np.all(fs[rs <= 0.75] == 0.0) and np.all(fs[rs >= 0.85] == 1.0)
    # the coefficient of the steepest zone spreads one zone to the side of
    # the higher pressure (CW84: f_j takes the larger of its own and its
    # lower-pressure neighbour's), and the mirror image mirrors it
    Pt = step(PL, 3.0 * PL, 0.95)
    f = O.flattening(Pt, Pt, un)
    assert 0.0 < f[j] < 1.0 and f[j + 1] == f[j] and f[j - 1] == 0.0
    fm = O.flattening(Pt[::-1].copy(), Pt[::-1].copy(), -un[::-1].copy())
    assert np.array_equal(fm, f[::-1])
