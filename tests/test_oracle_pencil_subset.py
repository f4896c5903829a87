"""The oracle's sweep of a list of pencils (the entry point that checks
full-size GPU runs pencil by pencil) against its sweep of the whole grid:
the listed pencils agree bitwise, on every axis of the inflow-dipole box
(stretched grid, inflow ghosts, dipole, inner boundary with a drift of the
reset zones), in both tracing modes."""
import numpy as np
import pytest

from oracle import ionosphere as IO

import gpu_cases as GC


@pytest.mark.parametrize("tracing", [0, 1])
def test_pencil_list_equals_whole_grid_sweep(tracing):
    case = GC.dipole_case(nx=32, ny=20, nz=18)
    case.tracing = tracing
    prob = case.oracle()
    box = IO.inner_box(case.faces, case.r_inner)
    assert box is not None
    rng = np.random.default_rng(3)
    v = 0.1 * rng.normal(size=(3, box[5] - box[4], box[3] - box[2], box[1] - box[0]))
    prob.set_inner_velocity(box, v)
    U = case.U
    dt = prob.cfl_dt(U, 0.4)
    n = [len(f) - 1 for f in case.faces]
    for axis in range(3):
        whole = prob.sweep(U, dt, axis)
        n1, n2 = n[(axis + 1) % 3], n[(axis + 2) % 3]
        # random pencils plus the ones through the middle (dipole, reset zones)
        j1 = np.concatenate([rng.integers(0, n1, 12), [n1 // 2, n1 // 2 - 1]])
        j2 = np.concatenate([rng.integers(0, n2, 12), [n2 // 2, n2 // 2]])
        listed = prob.sweep_pencils(U, dt, axis, j1, j2)
        for q in range(len(j1)):
            idx = [slice(None)] * 3
            idx[2 - (axis + 1) % 3] = j1[q]
            idx[2 - (axis + 2) % 3] = j2[q]
            assert np.array_equal(listed[q], whole[(slice(None),) + tuple(idx)]), (axis, j1[q], j2[q])
        # the middle pencils pass through the reset zones, whose drift shows
        assert not np.array_equal(whole, U)
