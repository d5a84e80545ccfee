"""Short-term energy conservation of the NVE integrator with the pair
forces (Sec. IV.A): on a thermalized fluid of squares of edge 4.24 sigma,
the standard deviation of the total energy per particle over a short NVE
run grows as dt^2 for a second-order integrator, and at a timestep where
truncation dominates the FP32 pair geometry fluctuates as the FP64 path
does."""
import numpy as np
import pytest

from paper_1607_02427_amd import inputs as I

pytestmark = pytest.mark.gpu


def _sigma(dem, th, prec, dt_tau, tau, duration_tau=2.0, samples=200):
    t = th.copy()
    t.ensemble = "nve"
    t.dt = dt_tau * tau
    n = int(round(duration_tau / dt_tau))
    k = max(1, n // samples)
    E = []
    with dem.DemSystem(t, prec) as g:
        for _ in range(n // k):
            e = g.energy()
            E.append(e["U"] + e["K_trans"] + e["K_rot"])
            g.step(k)
    return float(np.std(np.asarray(E) / t.n))


def test_energy_fluctuations_scale_as_dt_squared():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1607_02427_amd import dem
    s = I.energy_fluid(2, n_side=16)
    tau = 2 * s.shapes[0].r
    print(f"[energy] {s.name} n={s.n}", flush=True)
    with dem.DemSystem(s, "fp64") as g:
        g.step(400)
        th = g.state()
    sig = {dt: _sigma(dem, th, "fp64", dt, tau) for dt in (0.0025, 0.005, 0.01)}
    s32 = _sigma(dem, th, "fp32", 0.01, tau)
    print("[energy] sigma(E/N)", sig, "fp32 at 0.01:", s32, flush=True)
    assert 3.0 < sig[0.005] / sig[0.0025] < 5.3
    assert 3.0 < sig[0.01] / sig[0.005] < 5.3
    assert 0.8 < s32 / sig[0.01] < 1.25
