"""Spheres and disks (a point rounded by r; Sec. IV.B's baseline, "central
WCA"): pinned against the closed form of the WCA potential (Eq. 3/4) at the
centre distance, and, against a polytope, against Eq. 1/2 with the point as
one vertex (the face's projection, and the double term on an edge shared
by two faces)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1607_02427_amd import inputs as I

ID = [1.0, 0.0, 0.0, 0.0]


def _wca(r, sigma, eps=1.0):
    """Eq. 3/4 written out: 4 eps ((sigma/r)^12 - (sigma/r)^6) + eps inside
    2^(1/6) sigma; returns (U, -dU/dr)."""
    if r >= 2.0 ** (1.0 / 6.0) * sigma:
        return 0.0, 0.0
    s6 = (sigma / r) ** 6
    return 4 * eps * (s6 * s6 - s6) + eps, 24 * eps * (2 * s6 * s6 - s6) / r


@pytest.mark.parametrize("dim", [3, 2])
def test_sphere_pair_is_central_wca(dim):
    a, b = (I.sphere(0.5), I.sphere(0.3)) if dim == 3 else (I.disk(0.5), I.disk(0.3))
    os_ = O.OracleSystem(dim, [50.0, 50.0, 50.0 if dim == 3 else 1.0], [a, b])
    rng = np.random.default_rng(3)
    sigma = 0.8
    for d in (0.75, 0.8, 0.85, 0.89, 0.9):
        u = rng.normal(size=3)
        if dim == 2:
            u[2] = 0.0
        u /= np.linalg.norm(u)
        qi, qj = I.uniform_quaternions(rng, 2) if dim == 3 else (ID, ID)
        o = O.pair(os_, 0, 1, [0, 0, 0], qi, d * u, qj)
        U, f = _wca(d, sigma)
        assert o.U == pytest.approx(U, rel=1e-13, abs=1e-15)
        assert np.allclose(o.Fi, -f * u, rtol=1e-12, atol=1e-14)   # i pushed away from j
        assert np.max(np.abs(o.Ti)) == 0.0 and np.max(np.abs(o.Tj)) == 0.0
        assert o.n_in == (1 if U > 0.0 or d < 2 ** (1 / 6) * sigma else 0)
        terms = O.pair_terms(os_, 0, 1, [0, 0, 0], qi, d * u, qj)
        assert all(t["family"] == "ViVj" for t in terms)


def test_sphere_against_cube_face_and_edge():
    c, s = I.cube(1.0, 0.15), I.sphere(0.2)
    os_ = O.OracleSystem(3, [50.0, 50.0, 50.0], [c, s])
    sigma = 0.35
    # over the middle of the top face: one vertex-face term at the gap d
    for d in (0.3, 0.34, 0.38):
        o = O.pair(os_, 0, 1, [0, 0, 0], ID, [0.1, -0.2, 0.5 + d], ID)
        U, f = _wca(d, sigma)
        assert o.n_in == 1
        assert o.U == pytest.approx(U, rel=1e-13)
        assert o.Fi[2] == pytest.approx(-f, rel=1e-12)
    # beyond the edge where the top face meets the +x face, at distance d
    # from it along the bisector: the point's nearest point on both faces is
    # that edge point, so Eq. 1 counts the term twice
    d = 0.33
    p = np.array([0.5, 0.0, 0.5]) + d * np.array([1.0, 0.0, 1.0]) / math.sqrt(2.0)
    o = O.pair(os_, 0, 1, [0, 0, 0], ID, p, ID)
    U, f = _wca(d, sigma)
    assert o.n_in == 2
    assert o.U == pytest.approx(2 * U, rel=1e-13)
    terms = O.pair_terms(os_, 1, 0, p, ID, [0, 0, 0], ID)
    assert sorted(t["family"] for t in terms) == ["ViFj", "ViFj"]


def test_disk_against_square_edge():
    q, d0 = I.square(1.0, 0.25), I.disk(0.25)
    os_ = O.OracleSystem(2, [50.0, 50.0, 1.0], [q, d0])
    for d in (0.45, 0.5, 0.55):
        o = O.pair(os_, 0, 1, [0, 0, 0], ID, [0.5 + d, 0.1, 0.0], ID)
        U, f = _wca(d, 0.5)
        assert o.n_in == 1
        assert o.U == pytest.approx(U, rel=1e-13)
        assert o.Fi[0] == pytest.approx(-f, rel=1e-12)
