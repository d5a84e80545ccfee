"""Pins for the oracle's potential and nearest-point primitives.

WCA closed forms (Sec. II, Eq. 3-4) and the overcounting figures (Sec. II,
overcounting paragraph) come from tests/golden/paper_pins.json; the
nearest-point primitives (Sec. II: point-line, line-line, point-plane
formulae) are checked against closed forms and a dense brute-force
minimisation that shares nothing with the oracle's formulas.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_pins.json")))
PIN = {p["id"]: p for p in GOLD["pins"]}


# ------------------------------------------------------------------ WCA
@pytest.mark.parametrize("sigma", [0.2, 0.3, 0.5, 1.0])
def test_wca_closed_forms(sigma):
    rc = PIN["wca_cutoff"]["r_cut_over_sigma"] * sigma
    U, F, inside = O.wca(sigma, sigma)
    assert inside
    assert U == pytest.approx(PIN["wca_contact"]["U_at_sigma_over_eps"], rel=1e-14)
    assert F == pytest.approx(PIN["wca_contact"]["F_at_sigma_times_sigma_over_eps"] / sigma, rel=1e-14)
    # continuity at the cutoff: U and F -> 0 from below, exactly 0 at/after
    U, F, inside = O.wca(rc * (1 - 1e-9), sigma)
    assert inside and abs(U) < 1e-15 and abs(F) < 1e-6 / sigma
    U, F, inside = O.wca(rc, sigma)
    assert not inside and U == 0.0 and F == 0.0
    # the Lennard-Jones form itself (Eq. 3) shifted by +eps (Eq. 4), by hand at a few radii
    for r in np.linspace(0.8 * sigma, 0.999 * rc, 7):
        U, F, _ = O.wca(r, sigma)
        lj = 4 * ((sigma / r) ** 12 - (sigma / r) ** 6)
        dlj = -4 * (12 * sigma ** 12 / r ** 13 - 6 * sigma ** 6 / r ** 7)
        assert U == pytest.approx(lj + 1.0, rel=1e-12, abs=1e-14)
        assert F == pytest.approx(-dlj, rel=1e-12)
    # derivative consistency: F = -dU/dr by central differences
    for r in np.linspace(0.85 * sigma, 1.1 * sigma, 5):
        h = 1e-7 * sigma
        fd = -(O.wca(r + h, sigma)[0] - O.wca(r - h, sigma)[0]) / (2 * h)
        assert O.wca(r, sigma)[1] == pytest.approx(fd, rel=1e-6)


def test_overcount_isosurface_shift():
    """64 U(r) = U(sigma) = eps is solved by r = (16/9)^(1/6) sigma: the shift
    per particle is ~10% of the rounding radius (Sec. II), and no
    multiplicity can move the isosurface beyond 2^(1/6) sigma."""
    p = PIN["overcount_shift"]
    sigma = 0.3
    r64 = (16.0 / 9.0) ** (1.0 / 6.0) * sigma
    assert p["multiplicity"] * O.wca(r64, sigma)[0] == pytest.approx(1.0, rel=1e-12)
    shift_per_particle = 0.5 * (r64 - sigma)
    assert shift_per_particle / (0.5 * sigma) == pytest.approx(p["shift_fraction_of_r"], abs=p["shift_tolerance"])
    # bound: for any multiplicity m the m*U = eps isosurface stays inside r_cut
    for m in [1, 8, 64, 1e3, 1e6]:
        lo, hi = sigma, PIN["wca_cutoff"]["r_cut_over_sigma"] * sigma
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if m * O.wca(mid, sigma)[0] > 1.0:
                lo = mid
            else:
                hi = mid
        assert lo / sigma <= PIN["overcount_bound"]["bound"] + 0.003


# ------------------------------------------------------ brute-force references
def _bf_point_segment(p, a, b):
    t = np.linspace(0, 1, 20001)
    pts = a[None] + t[:, None] * (b - a)[None]
    d2 = np.sum((pts - p) ** 2, axis=1)
    k = int(np.argmin(d2))
    f = lambda s: float(np.sum((a + np.clip(s[0], 0, 1) * (b - a) - p) ** 2))
    res = minimize(f, [t[k]], bounds=[(0, 1)], method="L-BFGS-B", options=dict(ftol=1e-16, gtol=1e-14))
    return min(float(res.fun), float(d2[k]))


def _bf_segment_segment(a0, a1, b0, b1):
    s = np.linspace(0, 1, 401)
    A = a0[None] + s[:, None] * (a1 - a0)[None]
    B = b0[None] + s[:, None] * (b1 - b0)[None]
    d2 = np.sum((A[:, None, :] - B[None, :, :]) ** 2, axis=2)
    k = np.unravel_index(np.argmin(d2), d2.shape)
    f = lambda z: float(np.sum((a0 + z[0] * (a1 - a0) - b0 - z[1] * (b1 - b0)) ** 2))
    res = minimize(f, [s[k[0]], s[k[1]]], bounds=[(0, 1), (0, 1)], method="L-BFGS-B",
                   options=dict(ftol=1e-18, gtol=1e-14, maxiter=1000))
    return min(float(res.fun), float(d2[k]))


def _winding_inside(p2, poly2):
    """Inside test by the winding number (sum of signed angles), a different
    algorithm from the oracle's crossing-number test."""
    ang = 0.0
    n = len(poly2)
    for k in range(n):
        a = poly2[k] - p2
        b = poly2[(k + 1) % n] - p2
        ang += math.atan2(a[0] * b[1] - a[1] * b[0], a @ b)
    return abs(ang) > math.pi


def _bf_point_polygon(p, loop):
    """Squared distance from p to a closed planar polygon: brute force over a
    dense boundary sampling, plus the plane distance when the projection is
    inside by the winding number."""
    loop = np.asarray(loop, float)
    c = loop.mean(axis=0)
    n = np.cross(loop[1] - loop[0], loop[2] - loop[0])
    n /= np.linalg.norm(n)
    e1 = (loop[1] - loop[0]) / np.linalg.norm(loop[1] - loop[0])
    e2 = np.cross(n, e1)
    poly2 = np.stack([(loop - c) @ e1, (loop - c) @ e2], axis=1)
    p2 = np.array([(p - c) @ e1, (p - c) @ e2])
    s = (p - c) @ n
    best = min(_bf_point_segment(p, loop[k], loop[(k + 1) % len(loop)]) for k in range(len(loop)))
    if _winding_inside(p2, poly2):
        best = min(best, s * s)
    return best


# ------------------------------------------------------------ primitives
def test_point_segment_closed_forms():
    a, b = np.array([0.0, 0, 0]), np.array([2.0, 0, 0])
    assert np.allclose(O.point_segment([1, 3, 4], a, b), [1, 0, 0], atol=0)
    assert np.allclose(O.point_segment([-1, 1, 0], a, b), a, atol=0)   # beyond an end
    assert np.allclose(O.point_segment([5, -2, 1], a, b), b, atol=0)


def test_point_segment_brute_force():
    rng = np.random.default_rng(101)
    for _ in range(60):
        p, a, b = rng.normal(size=(3, 3))
        q = O.point_segment(p, a, b)
        assert np.sum((q - p) ** 2) == pytest.approx(_bf_point_segment(p, a, b), rel=1e-9, abs=1e-13)
        # q lies on the segment
        t = (q - a) @ (b - a) / ((b - a) @ (b - a))
        assert -1e-15 <= t <= 1 + 1e-15
        assert np.linalg.norm(a + t * (b - a) - q) < 1e-12


def test_segment_segment_closed_forms():
    # perpendicular skew segments crossing at their centres: distance h
    P, Q, par = O.segment_segment([-1, 0, 0], [1, 0, 0], [0, -1, 0.7], [0, 1, 0.7])
    assert not par and np.allclose(P, [0, 0, 0], atol=1e-15) and np.allclose(Q, [0, 0, 0.7], atol=1e-15)
    # general skew lines with interior closest points: |(b0-a0).(u x v)| / |u x v|
    rng = np.random.default_rng(7)
    for _ in range(30):
        a0, u, v = rng.normal(size=(3, 3))
        n = np.cross(u, v)
        n /= np.linalg.norm(n)
        h = rng.uniform(0.1, 1.0)
        s, t = rng.uniform(0.1, 0.9, 2)
        p = a0 + s * u
        b0 = p + h * n - t * v
        P, Q, par = O.segment_segment(a0, a0 + u, b0, b0 + v)
        assert not par
        assert np.linalg.norm(P - Q) == pytest.approx(abs((b0 - a0) @ np.cross(u, v)) / np.linalg.norm(np.cross(u, v)), rel=1e-10)
        assert np.allclose(P, p, atol=1e-10) and np.allclose(Q, p + h * n, atol=1e-10)


def test_segment_segment_brute_force():
    rng = np.random.default_rng(202)
    for _ in range(40):
        a0, a1, b0, b1 = rng.normal(size=(4, 3))
        P, Q, par = O.segment_segment(a0, a1, b0, b1)
        assert not par
        d2 = np.sum((P - Q) ** 2)
        assert d2 == pytest.approx(_bf_segment_segment(a0, a1, b0, b1), rel=1e-8, abs=1e-12)


def test_segment_segment_parallel_rule():
    """Nearly parallel edges interact at the midpoints of their overlap
    (Sec. II, paragraph on parallel edges)."""
    # exactly parallel, partial overlap [0.5, 1] on a, [0, 0.5] on b
    P, Q, par = O.segment_segment([0, 0, 0], [1, 0, 0], [0.5, 0.3, 0], [1.5, 0.3, 0])
    assert par and np.allclose(P, [0.75, 0, 0]) and np.allclose(Q, [0.75, 0.3, 0])
    # one contains the other's projection
    P, Q, par = O.segment_segment([0, 0, 0], [2, 0, 0], [1.5, 0, 0.4], [0.5, 0, 0.4])
    assert par and np.allclose(P, [1.0, 0, 0]) and np.allclose(Q, [1.0, 0, 0.4])
    # collinear, no overlap: facing endpoints
    P, Q, par = O.segment_segment([0, 0, 0], [0, 0, 1], [0, 0, 1.2], [0, 0, 2.2])
    assert par and np.allclose(P, [0, 0, 1]) and np.allclose(Q, [0, 0, 1.2])
    # just inside the threshold (sin^2 = 0.5e-6) uses the rule, just outside does not
    th = math.asin(math.sqrt(0.5e-6))
    P, Q, par = O.segment_segment([0, 0, 0], [1, 0, 0], [0, 0.3, 0], [math.cos(th), 0.3 + math.sin(th), 0])
    assert par
    th = math.asin(math.sqrt(2e-6))
    P, Q, par = O.segment_segment([0, 0, 0], [1, 0, 0], [0, 0.3, 0], [math.cos(th), 0.3 + math.sin(th), 0])
    assert not par
    # symmetric under swapping the two segments
    rng = np.random.default_rng(3)
    for _ in range(10):
        a0 = rng.normal(size=3)
        u = rng.normal(size=3)
        b0 = rng.normal(size=3)
        b1 = b0 + u * rng.uniform(0.5, 1.5) + 1e-5 * rng.normal(size=3)
        P, Q, par = O.segment_segment(a0, a0 + u, b0, b1)
        Q2, P2, par2 = O.segment_segment(b0, b1, a0, a0 + u)
        assert par and par2 and np.allclose(P, P2, atol=1e-13) and np.allclose(Q, Q2, atol=1e-13)


def _lshape_loop(z=0.0):
    return np.array([[0, 0, z], [2, 0, z], [2, 1, z], [1, 1, z], [1, 2, z], [0, 2, z]], float)


def test_point_polygon_closed_forms():
    sq = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], float)
    assert np.allclose(O.point_polygon([0.3, 0.6, 0.8], sq), [0.3, 0.6, 0])   # over the interior
    assert np.allclose(O.point_polygon([0.3, 0.6, -0.8], sq), [0.3, 0.6, 0])  # closed face: both sides
    assert np.allclose(O.point_polygon([1.5, 0.5, 0.2], sq), [1, 0.5, 0])     # beyond an edge
    assert np.allclose(O.point_polygon([1.5, 1.7, 0.2], sq), [1, 1, 0])       # beyond a corner
    # concave L: a point over the notch projects outside; nearest point on the notch edge
    L = _lshape_loop()
    assert np.allclose(O.point_polygon([1.2, 1.7, 0.3], L), [1, 1.7, 0])
    assert np.allclose(O.point_polygon([1.5, 1.5, -0.3], L), [1.5, 1, 0])  # tie: first edge in loop order
    assert np.allclose(O.point_polygon([0.5, 1.5, 0.3], L), [0.5, 1.5, 0])


@pytest.mark.parametrize("kind", ["triangle", "quad", "lshape", "pentagon"])
def test_point_polygon_brute_force(kind):
    rng = np.random.default_rng({"triangle": 1, "quad": 2, "lshape": 3, "pentagon": 4}[kind])
    if kind == "triangle":
        loop = np.array([[0, 0, 0], [1, 0, 0], [0.3, 0.8, 0]], float)
    elif kind == "quad":
        loop = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], float)
    elif kind == "lshape":
        loop = _lshape_loop()
    else:
        a = 2 * np.pi * np.arange(5) / 5
        loop = np.stack([np.cos(a), np.sin(a), np.zeros(5)], axis=1)
    # arbitrary rigid placement in space
    Rm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Rm) < 0:
        Rm[:, 0] *= -1
    t = rng.normal(size=3)
    loopw = loop @ Rm.T + t
    for _ in range(40):
        p = rng.uniform(-1.0, 2.5, 3) @ Rm.T + t
        q = O.point_polygon(p, loopw)
        assert np.sum((q - p) ** 2) == pytest.approx(_bf_point_polygon(p, loopw), rel=1e-9, abs=1e-13)
