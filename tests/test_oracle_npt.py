"""Pins for the oracle's isothermal-isobaric integrator (Sec. IV.C: the
assembly runs at fixed pressure, with a barostat driven by the pressure
from the virial tensor, after the measure-preserving integrator of
Tuckerman et al. 2006).

* Time reversibility of the whole step (particles, box, barostat and
  thermostat reversed together).
* The conserved quantity K + U + W v_eps^2 / 2 + P V + Q xi^2 / 2 + g' kT eta:
  its fluctuation shrinks four times when dt halves (second order).
* The ideal-gas limit of the isobaric ensemble: with the centre of mass at
  rest, p(V) ~ V^(N - 1) exp(-P V / kT), so <V> = N kT / P; a dilute gas of
  rounded cubes differs from it by its second virial coefficient, about
  0.4% here, far inside the tolerance, while a wrong pressure term (a
  factor in P or in d) would move <V> by tens of percent.
* Equipartition: <2 (K_trans + K_rot)> = g kT with g = 6N - 3, the
  thermostat's target less the barostat's one degree of freedom.
"""
import numpy as np

import oracle as O
from paper_1607_02427_amd import inputs as I


def _fluid():
    """64 rounded cubes from their lattice at volume fraction 0.4 (pressure
    about 0.2), compressed at P = 2: the box shrinks by a quarter within
    one tau while contacts form."""
    s = I.cubes_3d(n_side=4)
    s.ensemble = "npt"
    s.kT, s.tau_T, s.tau_P, s.P = 1.0, 0.5, 0.5, 2.0
    return s


def test_npt_time_reversible():
    s = _fluid()
    s.dt = 5e-4
    n = 400
    a, th, veps, lg, _ = O.run_npt(s, n)
    assert abs(veps) > 1e-3 and a.box[0] < 0.99 * s.box[0] and lg[:, 0].max() > 1.0
    b = a.copy()
    b.v = -a.v
    b.L = -a.L
    back, th2, veps2, _, _ = O.run_npt(b, n, thermo=(-th[0], th[1]), veps=-veps)
    assert np.allclose(back.box, s.box, rtol=0, atol=1e-10)
    d = back.x + back.image * back.box - (s.x + s.image * s.box)
    assert np.abs(d).max() < 1e-9
    assert np.abs(back.v + s.v).max() < 1e-9
    assert abs(veps2) < 1e-10 and abs(th2[0]) < 1e-10


def test_npt_conserved_quantity_is_second_order():
    s = _fluid()
    sig = []
    for dt in (1e-3, 5e-4):
        s.dt = dt
        _, _, _, lg, _ = O.run_npt(s, int(round(1.0 / dt)))
        assert lg[:, 6].min() < 0.8 * lg[0, 6]  # compressed, through contacts
        sig.append(lg[:, 5].std())
    ratio = sig[0] / sig[1]
    assert 3.5 < ratio < 4.5, (sig, ratio)


def test_npt_ideal_gas_volume_and_equipartition():
    shp = I.cube(1.0, 0.15)
    N, P = 64, 0.001
    L0 = (N / P) ** (1.0 / 3.0)
    s = I.lattice_system(shp, 4, 0.01, 5, orient="uniform", spacing=L0 / 4, name="dilute_cubes_64")
    s.box = np.array([L0, L0, L0])
    s.ensemble, s.P, s.tau_P, s.tau_T, s.dt, s.kT = "npt", P, 0.5, 0.5, 2e-3, 1.0
    th, veps, V, K2 = None, 0.0, [], []
    for _ in range(6):
        s, th, veps, lg, _ = O.run_npt(s, 100000, thermo=th, veps=veps, threads=2)
        V.append(lg[:, 6])
        K2.append(2.0 * (lg[:, 1] + lg[:, 2]))
    V = np.concatenate(V)[100000:]
    K2 = np.concatenate(K2)[100000:]
    ratio = V.mean() / (N * s.kT / P)
    assert abs(ratio - 1.0) < 0.12, ratio
    g = 6 * N - 3
    assert abs(K2.mean() / g - 1.0) < 0.02, K2.mean() / g
