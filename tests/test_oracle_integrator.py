"""Pins for the oracle's integrator (Sec. IV.A: a second-order integrator for
rigid bodies; Sec. IV.C: Nose-Hoover on translation and rotation).

Free particle and free rotors against exact motion, conservation of the
space-frame angular momentum, time reversibility, the dt^2 scaling of the
energy error (Sec. IV.A) and the Nose-Hoover conserved quantity."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1607_02427_amd import inputs as I

PIN = {p["id"]: p for p in json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_pins.json")))["pins"]}


def _rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _single(shape, L_body, v=(0.0, 0.0, 0.0), dim=3, box=50.0, q=(1.0, 0, 0, 0)):
    s = I.System(dim=dim, box=np.array([box, box, box if dim == 3 else 1.0]), shapes=[shape],
                 shape_id=np.zeros(1, np.int32), x=np.array([[box / 2, box / 2, box / 2 if dim == 3 else 0.0]]),
                 q=np.array([q], float), v=np.array([v], float), L=np.array([L_body], float),
                 image=np.zeros((1, 3), np.int32))
    return s


def test_free_particle_moves_in_a_straight_line():
    s = _single(I.cube(), [0, 0, 0], v=(3.1, -2.3, 1.7), box=10.0)
    dt, n = 0.01, 500
    s.dt = dt
    out, _, _, _ = O.run(s, n)
    unwrapped = out.x + out.image * s.box
    assert np.allclose(unwrapped, s.x + n * dt * s.v, rtol=0, atol=1e-10)


def test_free_symmetric_rotor():
    """Cube (isotropic inertia): the space-frame angular momentum is exactly
    conserved, K_rot is constant and the body turns about L at |L|/I."""
    c = I.cube()
    Lb = np.array([0.3, -0.7, 0.5])
    s = _single(c, Lb)
    dt, n = 1e-3, 2000
    s.dt = dt
    out, _, log, _ = O.run(s, n)
    Ls0 = _rot(s.q[0]) @ Lb
    Ls1 = _rot(out.q[0]) @ out.L[0]
    assert np.allclose(Ls1, Ls0, atol=1e-12)
    assert np.ptp(log[:, 2]) < 1e-13
    I0 = c.inertia[0]
    ang = np.linalg.norm(Ls0) / I0 * n * dt
    axis = Ls0 / np.linalg.norm(Ls0)
    qe = I.quat_from_axis_angle(axis, np.array(ang))
    Rexact = _rot(qe) @ _rot(s.q[0])
    assert np.abs(_rot(out.q[0]) - Rexact).max() < 1e-5


def test_free_asymmetric_rotor():
    """Concave L-prism (three distinct principal moments): the space-frame
    angular momentum is conserved to rounding and K_rot stays bounded."""
    lp = I.lprism(0.1, quad_h=0.05)
    assert len(set(np.round(lp.inertia, 6))) == 3
    Lb = np.array([0.4, 0.1, -0.6])
    s = _single(lp, Lb, q=I.uniform_quaternions(np.random.default_rng(1), 1)[0])
    s.dt = 2e-3
    out, _, log, _ = O.run(s, 3000)
    assert np.allclose(_rot(out.q[0]) @ out.L[0], _rot(s.q[0]) @ Lb, atol=1e-12)
    K0 = 0.5 * np.sum(Lb ** 2 / lp.inertia)
    assert np.abs(log[:, 2] - K0).max() < 1e-4 * K0


def test_planar_rotor():
    sq = I.square()
    s = _single(sq, [0, 0, 0.8], dim=2)
    s.dt = 1e-3
    out, _, _, _ = O.run(s, 1000)
    theta = 0.8 / sq.inertia[2] * 1.0
    assert np.allclose(out.q[0], [math.cos(theta / 2), 0, 0, math.sin(theta / 2)], atol=1e-12)


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_time_reversibility(which):
    if which == "2d":
        s = I.squares_2d_contact()
        s.dt, n = 1e-4, 100
    else:
        s = I.cubes_3d_contact(n_side=3)
        s.ensemble = "nve"
        s.dt, n = 5e-4, 60
    fwd, _, lg, _ = O.run(s, n)
    assert np.max(np.abs(O.forces(fwd)["F"])) > 1.0
    back = fwd.copy()
    back.v = -fwd.v
    back.L = -fwd.L
    ret, _, _, _ = O.run(back, n)
    unwrap0 = s.x + s.image * s.box
    unwrap1 = ret.x + ret.image * s.box
    assert np.abs(unwrap1 - unwrap0).max() < 1e-9
    assert np.abs(ret.v + s.v).max() < 1e-7
    qa, qb = ret.q, s.q
    sgn = np.sign(np.sum(qa * qb, axis=1))[:, None]
    assert np.abs(qa * sgn - qb).max() < 1e-9


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_energy_error_scales_as_dt_squared(which):
    """Sec. IV.A: for a second-order integrator the energy error at fixed
    simulated time scales as dt^2; halving dt divides it by ~4."""
    if which == "2d":
        s = I.squares_2d_contact()
        T, dts = 0.02, [4e-4, 2e-4]
    else:
        s = I.cubes_3d_contact(n_side=3)
        T, dts = 0.03, [1e-3, 5e-4]
    s.ensemble = "nve"
    errs = []
    for dt in dts:
        s.dt = dt
        n = int(round(T / dt))
        _, _, lg, f = O.run(s, n)
        E0 = O.forces(s)["U"].sum() + sum(O.kinetic(s))
        errs.append(np.max(np.abs(lg[:, 5] - E0)))
    ratio = errs[0] / errs[1]
    assert PIN["integrator_order"]["exponent"] == 2
    assert 3.0 < ratio < 5.0, (errs, ratio)


def test_nose_hoover_conserved_quantity():
    """The Nose-Hoover extended energy K + U + Q xi^2/2 + g kT eta is
    conserved as well as the plain energy is under NVE at the same dt, while
    the thermostat variable moves, and its error scales as dt^2."""
    ptp = {}
    for ens in ("nve", "nvt"):
        for dt in (5e-4, 2.5e-4):
            s = I.cubes_3d_contact(n_side=3, seed=21)
            s.ensemble = ens
            s.kT = 2.0
            s.dt = dt
            _, th, lg, _ = O.run(s, int(round(0.1 / dt)))
            ptp[ens, dt] = np.ptp(lg[:, 5])
            if ens == "nvt":
                assert np.abs(lg[:, 3]).max() > 0.1  # the thermostat acts
                assert np.ptp(lg[:, 1] + lg[:, 2] + lg[:, 0]) > 2 * ptp[ens, dt]
    for dt in (5e-4, 2.5e-4):
        assert ptp["nvt", dt] < 1.5 * ptp["nve", dt]
    assert 3.0 < ptp["nvt", 5e-4] / ptp["nvt", 2.5e-4] < 5.0


def _dof(dim, n):
    """Kinetic degrees of freedom of n rigid bodies with the total momentum
    held at zero: d n - d translational (the centre-of-mass momentum is
    conserved and zero) and d_rot n rotational (d_rot = 1 in 2D, 3 in 3D)."""
    drot = 1 if dim == 2 else 3
    return dim * n - dim, drot * n


@pytest.mark.parametrize("dim", [2, 3])
def test_nose_hoover_equipartition(dim):
    """Sec. IV.C thermostats translation and rotation with one variable: over
    a long NVT run of a small dense fluid the time averages of K_trans and
    K_rot each carry kT/2 per kinetic degree of freedom (equipartition), so
    <K_trans + K_rot> is (g/2) kT with g the degrees of freedom counted
    independently here.  A thermostat that targets another g (say one that
    forgets the conserved centre-of-mass momentum, or counts one rotational
    degree of freedom in 3D) fails the total; a wrong split between
    translation and rotation fails the two parts."""
    if dim == 2:
        s = I.lattice_system(I.square(1.0, 0.25), 2, 0.3, 3, orient="uniform", spacing=2.0)
        steps = 200000
    else:
        s = I.lattice_system(I.tetrahedron(1.0, 0.2), 2, 0.3, 5, orient="uniform", spacing=1.7)
        steps = 30000
    s.ensemble, s.kT, s.dt, s.tau_T = "nvt", 1.3, 2e-3, 0.5
    O.set_threads(1)
    try:
        _, _, lg, _ = O.run(s, steps, mode=0)
    finally:
        O.set_threads(os.cpu_count() or 1)
    tail = lg[steps // 10:]
    ft, fr = _dof(dim, s.n)
    busy = float((tail[:, 0] > 0).mean())  # some pair in contact: a fluid, not a free gas
    ktot = (tail[:, 1] + tail[:, 2]).mean() / (0.5 * (ft + fr) * s.kT)
    kt = tail[:, 1].mean() / (0.5 * ft * s.kT)
    kr = tail[:, 2].mean() / (0.5 * fr * s.kT)
    print(dim, s.n, busy, ktot, kt, kr)
    assert busy > 0.25, busy
    assert abs(ktot - 1.0) < 5e-3, ktot
    assert abs(kt - 1.0) < 0.08 and abs(kr - 1.0) < 0.08, (kt, kr)


@pytest.mark.parametrize("dim", [2, 3])
def test_nose_hoover_ideal_gas_oscillation(dim):
    """Bodies that never touch (a dilute box) under Nose-Hoover: with
    u = ln(K / K0), K0 = g kT / 2, the thermostat equations reduce to
    du/dt = -2 xi, Q dxi/dt = 2K - g kT, i.e. d2u/dt2 = -(2 g kT / Q)(e^u - 1),
    an oscillation of angular frequency sqrt(2 g kT / Q) = sqrt(2) / tau_T
    for Q = g kT tau_T^2 at small amplitude.  Its exact period at the
    run's amplitude (integrated here with scipy) must match the period of
    the oracle's xi, which pins the thermostat mass Q."""
    from scipy.integrate import solve_ivp
    shp = I.square(1.0, 0.25) if dim == 2 else I.cube(1.0, 0.15)
    s = I.lattice_system(shp, 2, 0.3, 6, orient="uniform", spacing=20.0)
    s.ensemble, s.kT, s.dt, s.tau_T = "nvt", 0.8, 1e-3, 0.5
    _, _, lg, _ = O.run(s, 12000, mode=0)
    assert not lg[:, 0].any()  # no contact, ever
    ft, fr = _dof(dim, s.n)
    g = ft + fr
    K0 = 0.5 * g * s.kT
    Kt, Kr = O.kinetic(s)
    u0 = math.log((Kt + Kr) / K0)
    w2 = 2.0 / s.tau_T ** 2  # 2 g kT / Q with Q = g kT tau_T^2
    ev = lambda t, y: y[1]
    ev.direction = -1.0  # du/dt crosses zero downwards: u at its maximum
    sol = solve_ivp(lambda t, y: [y[1], -w2 * math.expm1(y[0])], (0.0, 20.0), [u0, 0.0], rtol=1e-12, atol=1e-14,
                    events=ev)
    period = float(np.diff(sol.t_events[0]).mean())
    xi = lg[:, 3]
    t = (np.arange(len(xi)) + 1) * s.dt
    k = np.where((xi[:-1] < 0) & (xi[1:] >= 0))[0]  # xi crosses zero upwards once per period
    tz = t[k] - xi[k] * s.dt / (xi[k + 1] - xi[k])
    measured = float(np.diff(tz).mean())
    print(dim, u0, period, measured, 2 * math.pi * s.tau_T / math.sqrt(2))
    assert len(tz) >= 4
    assert abs(measured / period - 1.0) < 1e-3, (measured, period)
