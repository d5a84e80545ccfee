"""Pins for the oracle's pair energy (Eq. 1 in 3D, Eq. 2 in 2D), forces and
torques: feature-pair counts in aligned contacts (Sec. II overcounting
paragraph, Eq. 1-2), Newton's third law and angular momentum per pair, swap
symmetry, and F = -grad E, tau = -dE/dtheta by central differences."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1607_02427_amd import inputs as I

PIN = {p["id"]: p for p in json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_pins.json")))["pins"]}
ID = [1.0, 0.0, 0.0, 0.0]


def _osys(shape, dim=3, big=100.0):
    return O.OracleSystem(dim, [big, big, big if dim == 3 else 1.0], [shape])


def test_cubes_face_to_face_count():
    p = PIN["overcount_face_to_face_cubes"]
    c = I.cube(1.0, 0.15)
    os_ = _osys(c)
    for d in [0.25, 0.3, 0.32]:
        o = O.pair(os_, 0, 0, [0, 0, 0], ID, [0, 0, 1 + d], ID)
        u1 = O.wca(d, 0.3)[0]
        assert o.n_in == p["eq1_count"]
        assert o.U == pytest.approx(p["eq1_count"] * u1, rel=1e-12)
        assert o.Fi[2] == pytest.approx(-p["eq1_count"] * O.wca(d, 0.3)[1], rel=1e-12)
        assert abs(o.Fi[0]) < 1e-9 and abs(o.Fi[1]) < 1e-9
        assert np.max(np.abs(o.Ti)) < 1e-9 and np.max(np.abs(o.Tj)) < 1e-9
    assert p["paper_prose_count"] != p["eq1_count"]  # recorded discrepancy, Eq. 1 followed


def test_cubes_corner_to_corner_count():
    c = I.cube(1.0, 0.15)
    os_ = _osys(c)
    d = 0.28
    o = O.pair(os_, 0, 0, [0, 0, 0], ID, [1 + d / math.sqrt(3)] * 3, ID)
    assert o.n_in == PIN["cubes_corner_to_corner"]["count"]
    assert o.U == pytest.approx(15 * O.wca(d, 0.3)[0], rel=1e-12)


def test_squares_counts():
    p = PIN["feature_families_2d"]
    s = I.square(1.0, 0.25)
    os_ = _osys(s, dim=2)
    d = 0.52
    o = O.pair(os_, 0, 0, [0, 0, 0], ID, [1 + d, 0, 0], ID)
    assert o.n_in == p["squares_edge_to_edge"]
    assert o.U == pytest.approx(8 * O.wca(d, 0.5)[0], rel=1e-12)
    o = O.pair(os_, 0, 0, [0, 0, 0], ID, [1 + d / math.sqrt(2), 1 + d / math.sqrt(2), 0], ID)
    assert o.n_in == p["squares_corner_to_corner"]


def test_single_feature_pair_counts():
    """A vertex facing the centre of a big face, and two crossed perpendicular
    edges, each give exactly one feature pair inside the cutoff."""
    c = I.cube(1.0, 0.15)
    os_ = _osys(c)
    # rotate j so one of its vertices points along -z onto i's top face centre
    ax = np.array([1.0, -1.0, 0.0]) / math.sqrt(2)
    th = math.acos(1 / math.sqrt(3))   # body diagonal (1,1,1) -> +z ... of j pointing down: use -(1,1,1)
    qj = I.quat_from_axis_angle(ax, np.array(math.pi - th))
    Rj = _rot(qj)
    vdown = min((Rj @ v for v in c.vertices), key=lambda w: w[2])
    d = 0.29
    xj = np.array([0, 0, 0.5 + d]) - vdown
    o = O.pair(os_, 0, 0, [0, 0, 0], ID, xj, qj)
    assert o.n_in == 1
    assert o.U == pytest.approx(O.wca(d, 0.3)[0], rel=1e-10)
    # crossed edges: both cubes stand on an edge (45 deg about y for i, about
    # x for j), so i's top ridge runs along y and j's bottom ridge along x
    qi = I.quat_from_axis_angle(np.array([0, 1.0, 0]), np.array(math.pi / 4))
    qj = I.quat_from_axis_angle(np.array([1.0, 0, 0]), np.array(math.pi / 4))
    top = max((_rot(qi) @ v for v in c.vertices), key=lambda w: w[2])[2]
    low = min((_rot(qj) @ v for v in c.vertices), key=lambda w: w[2])[2]
    xj = np.array([0.0, 0.0, top + d - low])
    o = O.pair(os_, 0, 0, [0, 0, 0], qi, xj, qj)
    assert o.n_in == 1
    assert o.U == pytest.approx(O.wca(d, 0.3)[0], rel=1e-10)


def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _contact_pair(os_, shape, rng, dim=3, depth=0.15):
    """Random orientations and direction; approach along the line of centres
    until the first feature pair enters the cutoff, then go `depth` sigma
    further.  Rejects configurations that use the parallel-edge rule."""
    sigma = 2 * shape.r
    for _ in range(100):
        if dim == 3:
            qi, qj = I.uniform_quaternions(rng, 2)
            u = I.random_unit_vectors(rng, 1)[0]
        else:
            qi, qj = I.planar_quaternions(rng.uniform(0, 2 * np.pi, 2))
            a = rng.uniform(0, 2 * np.pi)
            u = np.array([math.cos(a), math.sin(a), 0.0])
        R = shape.circumradius
        dist = 2 * R + 1.2 * sigma
        while dist > 0:
            o = O.pair(os_, 0, 0, [0, 0, 0], qi, dist * u, qj)
            if o.n_in > 0:
                break
            dist -= 0.01 * sigma
        dist -= depth * sigma
        o = O.pair(os_, 0, 0, [0, 0, 0], qi, dist * u, qj)
        if o.n_par == 0 and o.n_in > 0:
            return qi, qj, dist * u
    raise RuntimeError("no contact found")


SHAPES3 = [("cube", {}), ("octahedron", {}), ("tetrahedron", {}), ("lprism", {"quad_h": 0.05})]


@pytest.mark.parametrize("name,kw", SHAPES3)
def test_pair_newton_and_angular_momentum(name, kw):
    shape = I.SHAPES[name](**kw)
    os_ = _osys(shape)
    rng = np.random.default_rng(sum(map(ord, name)))
    for _ in range(5):
        qi, qj, xj = _contact_pair(os_, shape, rng)
        o = O.pair(os_, 0, 0, [0, 0, 0], qi, xj, qj)
        s = O.pair(os_, 0, 0, xj, qj, [0, 0, 0], qi)   # same pair seen from j
        scale = np.linalg.norm(o.Fi) + 1.0
        assert s.U == pytest.approx(o.U, rel=1e-12)
        assert np.allclose(np.array(s.Fi), -np.array(o.Fi), atol=1e-11 * scale)
        assert np.allclose(np.array(s.Ti), np.array(o.Tj), atol=1e-11 * scale)
        assert np.allclose(np.array(s.Tj), np.array(o.Ti), atol=1e-11 * scale)
        # angular momentum: tau_i + tau_j + (x_i - x_j) x F_i = 0
        L = np.array(o.Ti) + np.array(o.Tj) + np.cross(-xj, np.array(o.Fi))
        assert np.max(np.abs(L)) < 1e-11 * scale
        # virial is the outer product of the pair vector and the force
        assert np.allclose(np.array(o.W).reshape(3, 3), np.outer(-xj, o.Fi), atol=1e-11 * scale)


def _energy(os_, xi, qi, xj, qj):
    return O.pair(os_, 0, 0, xi, qi, xj, qj).U


def _rotq(axis_k, h, q):
    ax = np.zeros(3)
    ax[axis_k] = 1.0
    return _qmul(I.quat_from_axis_angle(ax, np.array(h)), q)  # space-frame rotation


@pytest.mark.parametrize("name,kw,dim", [(n, k, 3) for n, k in SHAPES3] + [("square", {}, 2), ("pentagon", {}, 2)])
def test_force_and_torque_are_energy_gradients(name, kw, dim):
    """F_i = -dU/dx_i and tau_i = -dU/dtheta_i (rotation of i about its centre
    around each space axis) by central differences, h = 1e-6."""
    shape = I.SHAPES[name](**kw)
    os_ = _osys(shape, dim)
    rng = np.random.default_rng(len(name) * 31 + dim)
    h = 1e-6
    checked = 0
    for _ in range(6):
        qi, qj, xj = _contact_pair(os_, shape, rng, dim=dim)
        xi = np.zeros(3)
        o = O.pair(os_, 0, 0, xi, qi, xj, qj)
        F = np.array(o.Fi)
        T = np.array(o.Ti)
        scale = np.linalg.norm(F) + np.linalg.norm(T)
        axes = range(3) if dim == 3 else range(2)
        for k in axes:
            e = np.zeros(3)
            e[k] = h
            fd = -(_energy(os_, xi + e, qi, xj, qj) - _energy(os_, xi - e, qi, xj, qj)) / (2 * h)
            assert fd == pytest.approx(F[k], abs=2e-6 * scale)
        raxes = range(3) if dim == 3 else [2]
        for k in raxes:
            fd = -(_energy(os_, xi, _rotq(k, h, qi), xj, qj) - _energy(os_, xi, _rotq(k, -h, qi), xj, qj)) / (2 * h)
            assert fd == pytest.approx(T[k], abs=2e-6 * scale)
        checked += 1
    assert checked == 6


def test_pair_outside_bound_is_zero():
    c = I.cube(1.0, 0.15)
    os_ = _osys(c)
    rng = np.random.default_rng(5)
    R = c.circumradius
    rc = 1.122462048309373 * 0.3
    for _ in range(20):
        qi, qj = I.uniform_quaternions(rng, 2)
        u = I.random_unit_vectors(rng, 1)[0]
        o = O.pair(os_, 0, 0, [0, 0, 0], qi, (2 * R + rc) * 1.0000001 * u, qj)
        assert o.n_in == 0 and o.U == 0.0
