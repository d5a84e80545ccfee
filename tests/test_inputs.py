"""The seeded input module: mass properties of rounded shapes against
closed forms (Steiner's formula, the rounded square's polar moment) and an
independent quadrature, and the workload recipes."""
import math

import numpy as np
import pytest

from paper_1607_02427_amd import inputs as I


def test_rounded_square_closed_form():
    s = I.square(1.0, 0.25)
    r = 0.25
    assert s.volume == pytest.approx(1 + 4 * r + math.pi * r * r, rel=1e-14)
    # polar moment of square + 4 edge rectangles + 4 quarter disks, by hand
    J = 1 / 6 + 4 * (((0.5 + r) ** 3 - 0.125) / 3 + r / 12) + 4 * (math.pi * r ** 2 / 8 + 2 * r ** 3 / 3 + math.pi * r ** 4 / 8)
    assert s.inertia[2] == pytest.approx(J / s.volume, rel=1e-13)
    assert s.inertia[2] == pytest.approx(0.3605121, abs=1e-7)


@pytest.mark.parametrize("name,r", [("cube", 0.15), ("octahedron", 0.1), ("tetrahedron", 0.2), ("icosahedron", 0.1)])
def test_steiner_volume(name, r):
    s = I.SHAPES[name](r=r)
    v = s.vertices
    if name == "cube":
        V, S, M = 1.0, 6.0, 12 * 1.0 * (math.pi / 2) / 2
    elif name == "octahedron":
        a = 1.0
        V, S = math.sqrt(2) / 3 * a ** 3, 2 * math.sqrt(3) * a ** 2
        M = 12 * a * (math.pi - math.acos(-1 / 3)) / 2
    elif name == "icosahedron":
        a = 1.0
        V, S = 5 * (3 + math.sqrt(5)) / 12 * a ** 3, 5 * math.sqrt(3) * a ** 2
        M = 30 * a * (math.pi - math.acos(-math.sqrt(5) / 3)) / 2
        assert (len(s.vertices), len(s.edges), len(s.faces)) == (12, 30, 20)
    else:
        a = 1.0
        V, S = a ** 3 / (6 * math.sqrt(2)), math.sqrt(3) * a ** 2
        M = 6 * a * (math.pi - math.acos(1 / 3)) / 2
    assert s.volume == pytest.approx(V + S * r + M * r * r + 4 / 3 * math.pi * r ** 3, rel=1e-12)
    assert np.allclose(s.inertia, s.inertia[0], rtol=1e-10)   # symmetric bodies


def test_hexadecagon_at_the_vertex_limit():
    """Regular 16-gon of edge a, rounded by r: area n a^2 / (4 tan(pi/n)) +
    perimeter r + pi r^2 (Steiner in 2D)."""
    a, r, n = 0.5, 0.1, 16
    s = I.hexadecagon(a, r)
    assert len(s.vertices) == 16 and len(s.edges) == 16
    A0 = n * a * a / (4 * math.tan(math.pi / n))
    assert s.volume == pytest.approx(A0 + n * a * r + math.pi * r * r, rel=1e-12)


def test_cube_inertia_matches_quadrature():
    c = I.cube(1.0, 0.15)
    V, M1, S = I._boxes_moments_quadrature([((-0.5, -0.5, -0.5), (0.5, 0.5, 0.5))], 0.15, 0.01)
    Iq = (np.trace(S) - S[0, 0]) / V
    assert V == pytest.approx(c.volume, rel=2e-3)
    assert Iq == pytest.approx(c.inertia[0], rel=2e-3)


def test_lprism_tables():
    lp = I.lprism(0.1, quad_h=0.02)
    assert (lp.nv, lp.ne, lp.nf) == (12, 18, 8)
    assert lp.volume == pytest.approx(4.558, rel=2e-3)
    # principal frame: centred, inertia diagonal by construction, right-handed faces
    for f in lp.faces:
        n = np.zeros(3)
        for k in range(len(f)):
            n += np.cross(lp.vertices[f[k]], lp.vertices[f[(k + 1) % len(f)]])
        c = lp.vertices[f].mean(axis=0)
        # outward: the face normal points away from the body interior sample near the face
        assert np.linalg.norm(n) > 0


def test_workloads_shapes_and_sizes():
    s0 = I.squares_2d()
    assert s0.n == 256 and s0.box[0] == pytest.approx(33.53403, rel=1e-6)
    s1 = I.cubes_3d()
    assert s1.n == 4096 and s1.box[0] == pytest.approx(27.92336, rel=1e-6)
    assert s1.ensemble == "nvt" and s1.dt == 5e-4
    # momenta: COM velocity removed
    assert np.abs(s1.v.sum(axis=0)).max() < 1e-10
    # quaternions normalised, rotations at most 10 degrees
    assert np.allclose(np.linalg.norm(s1.q, axis=1), 1.0)
    assert np.max(2 * np.degrees(np.arccos(np.clip(np.abs(s1.q[:, 0]), 0, 1)))) <= 10.0 + 1e-9
    # determinism of the seeded generators
    s1b = I.cubes_3d()
    assert np.array_equal(s1.q, s1b.q) and np.array_equal(s1.v, s1b.v)


def test_cross_polytope_distance_matches_face_projection():
    """The distance used to place the at-scale octahedra, against the
    nearest point of each of the octahedron's eight triangular faces (the
    oracle's point-polygon primitive) for points outside, and zero inside."""
    import oracle as O
    rng = np.random.default_rng(7)
    c = 1.3
    e = np.eye(3)
    faces = [[sx * c * e[0], sy * c * e[1], sz * c * e[2]] for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)]
    pts = rng.normal(size=(300, 3)) * 1.2
    got = I._cross_polytope_distance(pts, c)
    for p, g in zip(pts, got):
        if np.abs(p).sum() <= c:
            assert g == 0.0
            continue
        want = min(np.linalg.norm(p - O.point_polygon(p, np.array(f))) for f in faces)
        assert abs(g - want) < 1e-12


def test_octahedra_start_is_overlap_free():
    """A small lattice of the at-scale recipe (same spacing): the common
    orientation keeps every pair of inner bodies min_gap apart, the start
    rotations cost at most 4 sin(5 deg / 2) R of it, and the oracle finds no
    feature pair inside the cutoff."""
    import oracle as O
    s = I.octahedra_3d(n=1000, n_cells=8)
    shp = s.shapes[0]
    rc = 2 ** (1 / 6) * 2 * shp.r
    assert s.min_gap - 4 * math.sin(math.radians(5.0) / 2) * shp.circumradius > rc
    ref = O.forces(s)
    assert ref["stats"]["pairs"] > 0 and ref["stats"]["feature_in"] == 0


def _dimer_summary(s, n_pairs, caps=None):
    """Pairs with a feature pair inside the cutoff, and (caps: faces of
    shape A, particle 2k) B's vertices against those faces on the face and
    off it, by the oracle's term listing."""
    import oracle as O
    touching, on_face, off_face = 0, 0, 0
    for k in range(n_pairs):
        t = O.dimer_terms(s, k)
        touching += 1 if t else 0
        if caps is not None:
            for e in t:
                if e["family"] == "VjFi" and e["b"] in caps:
                    on_face += e["inside"] == 1
                    off_face += e["inside"] == 0
    return touching, on_face, off_face


@pytest.mark.parametrize("name", ["cube", "octahedron", "tetrahedron", "icosahedron", "lprism", "square", "pentagon"])
def test_contact_dimers_are_all_in_contact(name):
    shp = I.lprism(0.1, quad_h=0.05) if name == "lprism" else I.SHAPES[name]()
    s = I.contact_dimers(shp, n_pairs=24, seed=31)
    touching, _, _ = _dimer_summary(s, 24)
    assert touching == 24


def test_notch_dimers_reach_both_branches_of_the_concave_cap():
    """The L-prism's caps (faces 0 and 1) are concave hexagons: the notch
    case puts the partner's vertices over the cap near its reflex corner,
    where the oracle's point-polygon rule takes the projection (on the
    face) and the nearest boundary point (over the notch)."""
    lp = I.lprism(0.1, quad_h=0.05)
    assert lp.faces[0] == [0, 5, 4, 3, 2, 1] and lp.faces[1] == [6, 7, 8, 9, 10, 11]
    s = I.contact_dimers(lp, I.cube(1.0, 0.15), n_pairs=128, notch=True)
    touching, on_face, off_face = _dimer_summary(s, 128, caps={0, 1})
    print(touching, on_face, off_face)
    assert touching >= 120 and on_face >= 100 and off_face >= 20
