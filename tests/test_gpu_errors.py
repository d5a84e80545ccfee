"""Device-side error conditions reported through the C ABI.

A non-finite position or velocity (DEM_E_NONFINITE) and a cell holding more
particles than its slots inside a step's list build (DEM_E_CAPACITY) are
latched by the kernels, which carry on and exit normally, and every later
synchronising call reports them until dem_set_state replaces the state.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1607_02427_amd import inputs as I

pytestmark = pytest.mark.gpu


def _dem():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1607_02427_amd import dem
    return dem


def test_nonfinite_velocity_is_reported():
    dem = _dem()
    s = I.cubes_3d_contact(n_side=4)
    s.ensemble = "nve"
    s.v[5] = [math.inf, 0.0, 0.0]
    print(f"[errors] nonfinite n={s.n}", flush=True)
    with dem.DemSystem(s, "fp32") as g:
        g.sync()  # the initial forces do not read velocities
        blob = g.get_state()
        g.step(2)
        for call in (g.sync, g.energy):
            with pytest.raises(dem.DemError) as ei:
                call()
            assert ei.value.status == 6, ei.value
        clean = s.copy()
        clean.v[5] = [0.0, 0.0, 0.0]
        with dem.DemSystem(clean, "fp32") as h:
            good = h.get_state()
        g.set_state(good)  # a new state clears the latched condition
        g.step(2)
        g.sync()
        assert len(blob) == len(good)


def _converging_ring(n=70):
    """n tiny squares that start spread over the eight cells around the
    centre cell of a 3 x 3 cell box (at most 64 to a cell) and move straight
    at the centre: one step later they lie inside the centre cell, which
    raises the rebuild trigger, and the next step's list build finds n > 64
    particles in that cell.  The squares are far apart at every step, so no
    force acts and each moves by dt v per step."""
    shp = I.square(0.01, 0.005)
    skin, dt = 3.0, 1e-3
    s0 = I.System(dim=2, box=np.ones(3), shapes=[shp], shape_id=np.zeros(n, np.int32), x=np.zeros((n, 3)),
                  q=np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)), v=np.zeros((n, 3)), L=np.zeros((n, 3)),
                  image=np.zeros((n, 3), np.int32), skin=skin, dt=dt, ensemble="nve")
    rl = O.OracleSystem.of(s0).r_list(skin)
    box = 3.2 * rl
    w = box / 3
    c = np.array([1.5 * w, 1.5 * w, 0.0])
    a = 2 * np.pi * (np.arange(n) + 0.5) / n
    u = np.stack([np.cos(a), np.sin(a), np.zeros(n)], axis=1)
    D = 0.8 * w  # distance per step
    s0.box = np.array([box, box, 1.0])
    s0.x = c + 1.2 * w * u
    s0.v = -u * (D / dt)
    return s0, rl, w


def test_cell_overflow_in_a_step_is_reported():
    dem = _dem()
    s, rl, w = _converging_ring()
    # the construction, checked on the host: at most 64 per cell at the
    # start, all n in the centre cell after two steps, never a contact
    for k in range(3):
        xk = s.copy()
        xk.x = (s.x + k * s.dt * s.v) % s.box
        nc, cs, _ = O.cell_list(xk, rl)
        counts = np.diff(cs)
        d = xk.x[:, None, :2] - xk.x[None, :, :2]
        d -= s.box[:2] * np.rint(d / s.box[:2])
        dmin = np.sqrt((d ** 2).sum(-1) + np.eye(s.n) * 1e9).min()
        assert dmin > 2 * s.shapes[0].circumradius + 2 ** (1 / 6) * 2 * s.shapes[0].r
        if k == 0:
            assert tuple(nc[:2]) == (3, 3) and counts.max() <= 64
        else:
            assert counts[4] == s.n  # the centre cell
    print(f"[errors] cell overflow n={s.n} r_list={rl:.3f} cell={w:.3f}", flush=True)
    with dem.DemSystem(s, "fp64") as g:
        g.sync()
        g.step(2)
        for call in (g.sync, g.energy):
            with pytest.raises(dem.DemError) as ei:
                call()
            assert ei.value.status == 5 and "cell" in str(ei.value), ei.value
