"""The seeded input recipe against the figures it is defined by: code units
with mu0 = 1 (R_E, 1 proton per cm^3, 1 nT), the solar-wind state and the
dipole moment in those units, the stretched 256 x 192 x 192 grid (widths
0.25 .. 2 R_E growing by 3 % outward from a 0.25 R_E core around the origin),
its split 512 x 384 x 384 form, and the ensemble sizes.  The reference
numbers are written out by hand from the physical constants, not computed
by the module."""

import numpy as np
import pytest

from paper_1607_02214_amd import inputs as I


def test_code_units():
    assert I.V0 / 1e3 == pytest.approx(21.81, abs=0.01)          # km/s
    assert I.P0 == pytest.approx(7.958e-13, rel=1e-3)              # Pa
    assert I.T0 == pytest.approx(292.1, abs=0.1)                    # s
    assert I.DIPOLE_MOMENT == pytest.approx(30936.0, rel=1e-4)      # nT R_E^3


def test_solar_wind_state_in_code_units():
    rho, vx, vy, vz, bx, by, bz, p = I.solar_wind(5.0, 400.0, 1e5, -5.0)
    assert rho == 5.0 and vy == 0.0 and vz == 0.0
    assert vx == pytest.approx(-18.34, abs=0.01)       # moving toward -x, away from the Sun
    assert p == pytest.approx(8.675, abs=0.001)        # n k_B T / p0
    assert (bx, by, bz) == (0.0, 0.0, -5.0)


def _widths(f):
    return np.diff(f)


def test_stretched_grid():
    fx, fy, fz = I.c2_faces()
    assert [len(f) - 1 for f in (fx, fy, fz)] == [256, 192, 192]
    for f in (fx, fy, fz):
        w = _widths(f)
        assert np.all(w > 0)
        assert w.min() == pytest.approx(0.25) and w.max() == pytest.approx(2.0)
        assert 0.0 in f                                   # a face at the origin
        # ratio of neighbouring widths: 1 in the core and at the cap, at most 1.03
        r = w[1:] / w[:-1]
        r = np.where(r < 1.0, 1.0 / r, r)
        assert np.all(r <= 1.03 + 1e-12)
        # the 16 cells on either side of the origin are the 0.25 core
        i0 = int(np.where(f == 0.0)[0][0])
        assert np.all(w[i0 - 16:i0 + 16] == 0.25)
    assert fx[0] == pytest.approx(-275.4, abs=0.05) and fx[-1] == pytest.approx(30.89, abs=0.005)
    for f in (fy, fz):
        assert f[0] == pytest.approx(-83.38, abs=0.005) and f[-1] == pytest.approx(83.38, abs=0.005)
        assert np.allclose(f, -f[::-1])                   # symmetric about the origin


def test_split_grid_keeps_the_domain_and_halves_every_cell():
    c2 = I.c2_faces()
    c3 = I.c3_faces()
    assert [len(f) - 1 for f in c3] == [512, 384, 384]
    for a, b in zip(c2, c3):
        assert np.array_equal(b[0::2], a)
        assert np.allclose(_widths(b)[0::2], 0.5 * _widths(a))
        assert np.allclose(_widths(b)[1::2], 0.5 * _widths(a))


def test_ensemble_members():
    m = I.ensemble_members()
    assert len(m) == 32
    sizes = [e["N"] for e in m]
    assert set(sizes) <= set(range(96, 161, 8))
    assert len(set(sizes)) >= 5                           # uneven sizes
    again = I.ensemble_members()                          # seeded: the same draw again
    assert all(a["N"] == b["N"] and np.array_equal(a["sw"], b["sw"]) for a, b in zip(m, again))
    for e in m:
        rho, vx, p = e["sw"][0], e["sw"][1], e["sw"][7]
        assert 1.0 <= rho <= 20.0
        assert -800e3 / I.V0 <= vx <= -300e3 / I.V0
        assert p == pytest.approx(rho * 1e6 * I.K_B * 1e5 / I.P0)
        f = I.member_faces(e["N"])
        assert [len(x) - 1 for x in f] == [e["N"]] * 3
