"""Seeded synthetic inputs for the rounded-polytope DEM path.

Shapes (body-frame feature tables plus the mass properties of the rounded
body) and initial states (positions, orientations, velocities, angular
momenta, box).  This module defines workloads only: it holds no part of the
pair potential, the nearest-feature geometry, the lists or the integrator, so
both the HIP library and the CPU oracle consume exactly these arrays.

Model (Sec. II, Fig. 1): a particle is an inner polygon or polyhedron,
convex or concave, Minkowski-rounded by a disk or sphere of radius r, with
the WCA length sigma_ij = r_i + r_j (Sec. II, Eq. 4 and the sentence before
Eq. 3).  The paper does not say how mass is distributed; here it is uniform
over the rounded body with m = 1, and the body frame is the principal frame
with its origin at the rounded body's centre of mass.

Every random draw uses numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import math
import os
from typing import List, Optional, Sequence

import numpy as np

TWO_PI = 2.0 * math.pi
# stored starting states (written by tests/golden/make_states.py), with the
# SHA-256 of each file in states.json
GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden")


# --------------------------------------------------------------------------
# Shapes
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Shape:
    """Feature tables of one rounded polytope in its body frame.

    vertices : (nv, 3) float64; 2D shapes have z = 0.
    edges    : (ne, 2) int32 vertex indices.  2D: edge k = (k, k+1 mod nv),
               counter-clockwise (Sec. III: the edge that begins at a vertex,
               travelling counter-clockwise).
    faces    : list of vertex loops, counter-clockwise seen from outside
               (3D only; may be concave).
    r        : rounding radius (half of sigma for like particles).
    mass     : particle mass.
    inertia  : (3,) principal moments; 2D uses inertia[2].
    name     : label.
    """
    dim: int
    vertices: np.ndarray
    edges: np.ndarray
    faces: List[List[int]]
    r: float
    mass: float
    inertia: np.ndarray
    name: str = ""
    volume: float = 0.0  # rounded area (2D) or volume (3D)
    # (com, U) of the construction frame: a point p given in the coordinates
    # the shape was built in sits at (p - com) @ U in the body frame
    frame: Optional[tuple] = None

    @property
    def nv(self) -> int:
        return int(self.vertices.shape[0])

    @property
    def ne(self) -> int:
        return int(self.edges.shape[0])

    @property
    def nf(self) -> int:
        return len(self.faces)

    @property
    def circumradius(self) -> float:
        return float(np.max(np.sqrt(np.sum(self.vertices ** 2, axis=1))))

    def face_offsets(self) -> np.ndarray:
        off = [0]
        for f in self.faces:
            off.append(off[-1] + len(f))
        return np.asarray(off, dtype=np.int32)

    def face_vertices(self) -> np.ndarray:
        if not self.faces:
            return np.zeros(0, dtype=np.int32)
        return np.asarray([v for f in self.faces for v in f], dtype=np.int32)


def _edges_from_faces(faces: Sequence[Sequence[int]]) -> np.ndarray:
    seen = []
    keys = set()
    for f in faces:
        for k in range(len(f)):
            a, b = f[k], f[(k + 1) % len(f)]
            key = (min(a, b), max(a, b))
            if key not in keys:
                keys.add(key)
                seen.append(key)
    return np.asarray(seen, dtype=np.int32)


def _order_convex_faces(verts: np.ndarray, tol: float = 1e-9) -> List[List[int]]:
    """Faces of a convex polytope given by its vertices (counter-clockwise
    from outside).  Brute force over vertex triples; fine for <= 20 vertices."""
    nv = verts.shape[0]
    c = verts.mean(axis=0)
    planes = []
    for a in range(nv):
        for b in range(a + 1, nv):
            for d in range(b + 1, nv):
                n = np.cross(verts[b] - verts[a], verts[d] - verts[a])
                nn = np.linalg.norm(n)
                if nn < 1e-12:
                    continue
                n = n / nn
                off = n @ verts[a]
                s = verts @ n - off
                if np.all(s <= tol):
                    pass
                elif np.all(s >= -tol):
                    n, off, s = -n, -off, -s
                else:
                    continue
                if any(np.allclose(n, p[0], atol=1e-9) for p in planes):
                    continue
                planes.append((n, off))
    faces = []
    for n, off in planes:
        idx = [k for k in range(nv) if abs(verts[k] @ n - off) < 1e-9]
        fc = verts[idx].mean(axis=0)
        e1 = verts[idx[0]] - fc
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(n, e1)
        ang = [math.atan2((verts[k] - fc) @ e2, (verts[k] - fc) @ e1) for k in idx]
        order = [idx[k] for k in np.argsort(ang)]
        faces.append(order)
    # deterministic face order: by normal direction
    faces.sort(key=lambda f: tuple(np.round(_newell(verts, f), 6)))
    return faces


def _newell(verts: np.ndarray, loop: Sequence[int]) -> np.ndarray:
    n = np.zeros(3)
    for k in range(len(loop)):
        p = verts[loop[k]]
        q = verts[loop[(k + 1) % len(loop)]]
        n += np.cross(p, q)
    return n / np.linalg.norm(n)


# ---- exact mass properties of rounded convex bodies ------------------------
def _rounded_polygon_moments(v2: np.ndarray, r: float):
    """Area, first moment and polar second moment of a convex polygon
    (counter-clockwise, (n,2)) Minkowski-summed with a disk of radius r.
    Decomposition: polygon + one rectangle per edge + one circular sector per
    vertex (exterior angle)."""
    n = v2.shape[0]
    A = 0.0
    M1 = np.zeros(2)
    J = 0.0
    o = v2[0]
    for k in range(1, n - 1):  # fan triangles
        a, b, c = o, v2[k], v2[k + 1]
        area = 0.5 * ((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]))
        A += area
        M1 += area * (a + b + c) / 3.0
        J += area / 6.0 * (a @ a + b @ b + c @ c + a @ b + b @ c + c @ a)
    normals = []
    for k in range(n):
        a, b = v2[k], v2[(k + 1) % n]
        e = b - a
        ell = np.linalg.norm(e)
        nrm = np.array([e[1], -e[0]]) / ell  # outward for CCW
        normals.append(nrm)
        A += ell * r
        M1 += ell * r * (a + b) / 2.0 + ell * r * r / 2.0 * nrm
        J += r * ell * (a @ a + a @ b + b @ b) / 3.0 + r * r * ell * (a @ nrm) + r ** 3 * ell / 3.0
    for k in range(n):
        v = v2[k]
        n1 = normals[k - 1]  # edge ending at v
        n2 = normals[k]      # edge starting at v
        alpha = math.atan2(n1[0] * n2[1] - n1[1] * n2[0], n1 @ n2)
        if alpha < 0:
            alpha += TWO_PI
        m = np.array([-n1[1], n1[0]])
        w1 = math.sin(alpha) * n1 + (1.0 - math.cos(alpha)) * m
        A += alpha * r * r / 2.0
        M1 += v * alpha * r * r / 2.0 + r ** 3 / 3.0 * w1
        J += (v @ v) * alpha * r * r / 2.0 + 2.0 * r ** 3 / 3.0 * (v @ w1) + alpha * r ** 4 / 4.0
    return A, M1, J


def _tri_second(a, b, c, area):
    s = a + b + c
    return area / 12.0 * (np.outer(a, a) + np.outer(b, b) + np.outer(c, c) + np.outer(s, s))


def _rounded_polyhedron_moments(verts: np.ndarray, faces, r: float):
    """Volume V, first moment M1 (3,) and second moment S = int p p^T of a
    convex polyhedron Minkowski-summed with a ball of radius r (exact).

    Decomposition: the polyhedron, a prism over every face, a cylindrical
    wedge along every edge and a spherical sector at every vertex.  Vertex
    sectors use the solid angle and the vector integral of the normal cone
    (int w dOmega = 1/2 sum_arcs theta_k m_k); their r^5 terms sum over the
    whole sphere to (4 pi / 3) I.
    """
    V = 0.0
    M1 = np.zeros(3)
    S = np.zeros((3, 3))
    ctr = verts.mean(axis=0)
    fnorm = []
    for f in faces:
        n = _newell(verts, f)
        fnorm.append(n)
        o = verts[f[0]]
        for k in range(1, len(f) - 1):
            a, b, c = o, verts[f[k]], verts[f[k + 1]]
            # tetrahedron (ctr, a, b, c)
            vol = np.dot(a - ctr, np.cross(b - ctr, c - ctr)) / 6.0
            pts = [ctr, a, b, c]
            s = ctr + a + b + c
            V += vol
            M1 += vol * s / 4.0
            S += vol / 20.0 * (sum(np.outer(p, p) for p in pts) + np.outer(s, s))
            # face prism over triangle (a, b, c)
            area = 0.5 * np.linalg.norm(np.cross(b - a, c - a))
            q1 = area * (a + b + c) / 3.0
            q2 = _tri_second(a, b, c, area)
            V += area * r
            M1 += r * q1 + r * r / 2.0 * area * n
            S += r * q2 + r * r / 2.0 * (np.outer(q1, n) + np.outer(n, q1)) + r ** 3 / 3.0 * area * np.outer(n, n)
    # edges: adjacent face normals
    edge_faces = {}
    for fi, f in enumerate(faces):
        for k in range(len(f)):
            a, b = f[k], f[(k + 1) % len(f)]
            edge_faces.setdefault((min(a, b), max(a, b)), []).append(fi)
    for (ia, ib), fl in edge_faces.items():
        assert len(fl) == 2, "every edge must border exactly two faces"
        a, b = verts[ia], verts[ib]
        n1, n2 = fnorm[fl[0]], fnorm[fl[1]]
        e = b - a
        ell = np.linalg.norm(e)
        cosA = float(np.clip(n1 @ n2, -1.0, 1.0))
        alpha = math.acos(cosA)
        if alpha < 1e-12:
            continue
        m = n2 - cosA * n1
        m /= np.linalg.norm(m)
        w1 = math.sin(alpha) * n1 + (1.0 - math.cos(alpha)) * m
        w2 = ((alpha / 2 + math.sin(2 * alpha) / 4) * np.outer(n1, n1)
              + (alpha / 2 - math.sin(2 * alpha) / 4) * np.outer(m, m)
              + (math.sin(alpha) ** 2 / 2) * (np.outer(n1, m) + np.outer(m, n1)))
        ce = ell * (a + b) / 2.0
        cc = ell * (np.outer(a, a) + 0.5 * (np.outer(a, b) + np.outer(b, a)) + np.outer(b, b)) / 3.0
        V += ell * alpha * r * r / 2.0
        M1 += alpha * r * r / 2.0 * ce + ell * r ** 3 / 3.0 * w1
        S += alpha * r * r / 2.0 * cc + r ** 3 / 3.0 * (np.outer(ce, w1) + np.outer(w1, ce)) + r ** 4 / 4.0 * ell * w2
    # vertices: normal cones
    for vi in range(verts.shape[0]):
        inc = [fi for fi, f in enumerate(faces) if vi in f]
        # order incident faces around the vertex: consecutive faces share an edge at vi
        loop = [inc[0]]
        while len(loop) < len(inc):
            cur = faces[loop[-1]]
            k = cur.index(vi)
            prev_v = cur[k - 1]  # edge (prev_v, vi) of the current face
            nxt = [fi for fi in inc if fi not in loop and prev_v in faces[fi]]
            assert len(nxt) == 1
            loop.append(nxt[0])
        ns = [fnorm[fi] for fi in loop]
        if np.dot(np.cross(ns[0], ns[1]), ns[2] if len(ns) > 2 else ns[0]) < 0:
            ns = ns[::-1]
        omega = 0.0
        for k in range(1, len(ns) - 1):
            a, b, c = ns[0], ns[k], ns[k + 1]
            num = abs(a @ np.cross(b, c))
            den = 1.0 + a @ b + b @ c + c @ a
            omega += 2.0 * math.atan2(num, den)
        centre = sum(ns)
        centre /= np.linalg.norm(centre)
        s1 = np.zeros(3)
        for k in range(len(ns)):
            a, b = ns[k], ns[(k + 1) % len(ns)]
            th = math.acos(float(np.clip(a @ b, -1.0, 1.0)))
            mk = np.cross(a, b)
            mk /= np.linalg.norm(mk)
            if mk @ centre < 0:
                mk = -mk
            s1 += 0.5 * th * mk
        v = verts[vi]
        V += omega * r ** 3 / 3.0
        M1 += omega * r ** 3 / 3.0 * v + r ** 4 / 4.0 * s1
        S += omega * r ** 3 / 3.0 * np.outer(v, v) + r ** 4 / 4.0 * (np.outer(v, s1) + np.outer(s1, v))
    S += r ** 5 / 5.0 * (4.0 * math.pi / 3.0) * np.eye(3)
    return V, M1, S


def _boxes_moments_quadrature(boxes, r: float, h: float):
    """Volume, first and second moments of a union of axis-aligned boxes
    rounded by r, by midpoint quadrature on a grid of spacing h (used for the
    concave L-prism, whose rounded body is the union of its rounded cubes)."""
    lo = np.min([b[0] for b in boxes], axis=0) - r
    hi = np.max([b[1] for b in boxes], axis=0) + r
    n = np.ceil((hi - lo) / h).astype(int)
    xs = [lo[k] + (np.arange(n[k]) + 0.5) * h for k in range(3)]
    V = 0.0
    M1 = np.zeros(3)
    S = np.zeros((3, 3))
    Y, Z = np.meshgrid(xs[1], xs[2], indexing="ij")
    for x in xs[0]:
        P = np.stack([np.full_like(Y, x), Y, Z], axis=-1).reshape(-1, 3)
        inside = np.zeros(P.shape[0], dtype=bool)
        for blo, bhi in boxes:
            c = 0.5 * (np.asarray(blo) + np.asarray(bhi))
            hw = 0.5 * (np.asarray(bhi) - np.asarray(blo))
            dd = np.maximum(np.abs(P - c) - hw, 0.0)
            inside |= np.sum(dd * dd, axis=1) <= r * r
        Q = P[inside]
        w = h ** 3
        V += w * Q.shape[0]
        M1 += w * Q.sum(axis=0)
        S += w * Q.T @ Q
    return V, M1, S


def _finish_3d(name, verts, faces, r, V, M1, S, mass=1.0):
    com = M1 / V
    Sc = S - V * np.outer(com, com)          # second moment about the COM
    I = (np.trace(Sc) * np.eye(3) - Sc) * (mass / V)
    w, U = np.linalg.eigh(I)
    if np.max(np.abs(I - np.diag(np.diag(I)))) < 1e-12 * np.max(np.abs(I)):
        U = np.eye(3)
        w = np.diag(I).copy()
    if np.linalg.det(U) < 0:
        U[:, 2] *= -1.0  # proper rotation, so face loops keep their orientation
    verts_b = (verts - com) @ U
    edges = _edges_from_faces(faces)
    return Shape(dim=3, vertices=np.ascontiguousarray(verts_b), edges=edges, faces=faces, r=float(r),
                 mass=float(mass), inertia=np.asarray(w, dtype=np.float64), name=name, volume=float(V),
                 frame=(com, U))


def polygon(verts2: np.ndarray, r: float, name: str = "polygon", mass: float = 1.0) -> Shape:
    """Rounded convex polygon from counter-clockwise vertices (n,2)."""
    v2 = np.asarray(verts2, dtype=np.float64)
    A, M1, J = _rounded_polygon_moments(v2, r)
    com = M1 / A
    Jc = J - A * (com @ com)
    v3 = np.zeros((v2.shape[0], 3))
    v3[:, :2] = v2 - com
    n = v2.shape[0]
    edges = np.asarray([(k, (k + 1) % n) for k in range(n)], dtype=np.int32)
    Iz = mass * Jc / A
    return Shape(dim=2, vertices=v3, edges=edges, faces=[], r=float(r), mass=float(mass),
                 inertia=np.array([0.0, 0.0, Iz]), name=name, volume=float(A))


def sphere(r: float = 0.5, mass: float = 1.0) -> Shape:
    """A sphere of radius r: a single point rounded by r, no edges or faces.
    Two spheres interact by the central WCA potential at the distance of
    their centres (sigma = r_i + r_j), the baseline of Table I; a sphere and
    a polytope through the sphere's point as a vertex of Eq. 1."""
    I = 0.4 * mass * r * r
    return Shape(dim=3, vertices=np.zeros((1, 3)), edges=np.zeros((0, 2), dtype=np.int32), faces=[], r=float(r),
                 mass=float(mass), inertia=np.array([I, I, I]), name="sphere",
                 volume=4.0 / 3.0 * math.pi * r ** 3)


def disk(r: float = 0.5, mass: float = 1.0) -> Shape:
    """A disk of radius r: the 2D counterpart of sphere()."""
    return Shape(dim=2, vertices=np.zeros((1, 3)), edges=np.zeros((0, 2), dtype=np.int32), faces=[], r=float(r),
                 mass=float(mass), inertia=np.array([0.0, 0.0, 0.5 * mass * r * r]), name="disk",
                 volume=math.pi * r * r)


def regular_polygon(n: int, edge: float = 1.0, r: float = 0.25, name: Optional[str] = None) -> Shape:
    R = edge / (2.0 * math.sin(math.pi / n))
    ang = -math.pi / 2 - math.pi / n + TWO_PI * np.arange(n) / n  # flat bottom edge
    v2 = np.stack([R * np.cos(ang), R * np.sin(ang)], axis=1)
    return polygon(v2, r, name or f"{n}-gon")


def square(edge: float = 1.0, r: float = 0.25) -> Shape:
    h = 0.5 * edge
    v2 = np.array([[-h, -h], [h, -h], [h, h], [-h, h]])
    return polygon(v2, r, "square")


def pentagon(edge: float = 1.0, r: float = 0.15) -> Shape:
    return regular_polygon(5, edge, r, "pentagon")


def convex_polyhedron(verts: np.ndarray, r: float, name: str) -> Shape:
    verts = np.asarray(verts, dtype=np.float64)
    faces = _order_convex_faces(verts)
    V, M1, S = _rounded_polyhedron_moments(verts, faces, r)
    return _finish_3d(name, verts, faces, r, V, M1, S)


def cube(edge: float = 1.0, r: float = 0.15) -> Shape:
    h = 0.5 * edge
    v = np.array([[x, y, z] for x in (-h, h) for y in (-h, h) for z in (-h, h)])
    return convex_polyhedron(v, r, "cube")


def octahedron(edge: float = 1.0, r: float = 0.1) -> Shape:
    a = edge / math.sqrt(2.0)
    v = np.array([[a, 0, 0], [-a, 0, 0], [0, a, 0], [0, -a, 0], [0, 0, a], [0, 0, -a]])
    return convex_polyhedron(v, r, "octahedron")


def tetrahedron(edge: float = 1.0, r: float = 0.1) -> Shape:
    s = edge / (2.0 * math.sqrt(2.0))
    v = s * np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    return convex_polyhedron(v, r, "tetrahedron")


def lprism(r: float = 0.1, quad_h: float = 0.01) -> Shape:
    """Concave L-prism: three unit cubes in an L (cross-section the hexagon
    (0,0),(2,0),(2,1),(1,1),(1,2),(0,2)) extruded by 1: 12 vertices, 18 edges,
    8 faces, two of them concave hexagons."""
    hexa = [(0, 0), (2, 0), (2, 1), (1, 1), (1, 2), (0, 2)]
    verts = np.array([[x, y, 0.0] for x, y in hexa] + [[x, y, 1.0] for x, y in hexa])
    bottom = [0, 5, 4, 3, 2, 1]          # seen from -z: clockwise in xy
    top = [6, 7, 8, 9, 10, 11]
    sides = [[k, (k + 1) % 6, (k + 1) % 6 + 6, k + 6] for k in range(6)]
    faces = [bottom, top] + sides
    boxes = [((0, 0, 0), (1, 1, 1)), ((1, 0, 0), (2, 1, 1)), ((0, 1, 0), (1, 2, 1))]
    V, M1, S = _boxes_moments_quadrature(boxes, r, quad_h)
    return _finish_3d("lprism", verts, faces, r, V, M1, S)


def icosahedron(edge: float = 1.0, r: float = 0.1) -> Shape:
    """Regular icosahedron (12 vertices, 30 edges, 20 triangular faces: the
    face limit of the shape tables), vertices at the cyclic permutations of
    (0, +-1, +-phi) scaled to the edge."""
    phi = 0.5 * (1.0 + math.sqrt(5.0))
    base = []
    for a in (-1.0, 1.0):
        for b in (-phi, phi):
            base += [[0.0, a, b], [a, b, 0.0], [b, 0.0, a]]
    return convex_polyhedron(0.5 * edge * np.array(base), r, "icosahedron")


def hexadecagon(edge: float = 0.5, r: float = 0.1) -> Shape:
    """Regular 16-gon: the vertex limit of the shape tables, in 2D."""
    return regular_polygon(16, edge, r, "hexadecagon")


SHAPES = {
    "square": square, "pentagon": pentagon, "cube": cube,
    "octahedron": octahedron, "tetrahedron": tetrahedron, "lprism": lprism,
    "icosahedron": icosahedron, "hexadecagon": hexadecagon,
}


# --------------------------------------------------------------------------
# Rotations (input sampling only)
# --------------------------------------------------------------------------
def quat_from_axis_angle(axis: np.ndarray, angle: np.ndarray) -> np.ndarray:
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis, axis=-1, keepdims=True)
    half = 0.5 * np.asarray(angle, dtype=np.float64)
    q = np.concatenate([np.cos(half)[..., None], np.sin(half)[..., None] * axis], axis=-1)
    return q


def random_unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def uniform_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    g = rng.standard_normal((n, 4))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def small_rotations(rng: np.random.Generator, n: int, max_deg: float) -> np.ndarray:
    axis = random_unit_vectors(rng, n)
    ang = np.deg2rad(rng.uniform(0.0, max_deg, n))
    return quat_from_axis_angle(axis, ang)


def planar_quaternions(theta: np.ndarray) -> np.ndarray:
    theta = np.asarray(theta, dtype=np.float64)
    q = np.zeros(theta.shape + (4,))
    q[..., 0] = np.cos(0.5 * theta)
    q[..., 3] = np.sin(0.5 * theta)
    return q


# --------------------------------------------------------------------------
# Systems
# --------------------------------------------------------------------------
@dataclasses.dataclass
class System:
    """One simulation input: box, shapes, per-particle state and run knobs.

    x (N,3) positions in [0, L); q (N,4) unit quaternions (w, x, y, z),
    body -> space; v (N,3); L (N,3) angular momentum in the body frame;
    shape_id (N,) int32; image (N,3) int32.
    """
    dim: int
    box: np.ndarray
    shapes: List[Shape]
    shape_id: np.ndarray
    x: np.ndarray
    q: np.ndarray
    v: np.ndarray
    L: np.ndarray
    image: np.ndarray
    epsilon: float = 1.0
    skin: float = 0.3
    rebuild_frac: float = 0.5
    dt: float = 1e-4
    ensemble: str = "nve"
    kT: float = 1.0
    tau_T: float = 0.5
    parallel_sin2: float = 1e-6
    name: str = ""
    thermo: Optional[tuple] = None  # Nose-Hoover (xi, eta) of a stored state; None: (0, 0)
    P: float = 0.0                  # target pressure of the 'npt' ensemble
    tau_P: float = 2.0              # its barostat time constant
    veps: float = 0.0               # barostat velocity of a stored state

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def copy(self) -> "System":
        return dataclasses.replace(
            self, box=self.box.copy(), shape_id=self.shape_id.copy(), x=self.x.copy(), q=self.q.copy(),
            v=self.v.copy(), L=self.L.copy(), image=self.image.copy())


def thermal_momenta(rng: np.random.Generator, shapes: List[Shape], shape_id: np.ndarray, dim: int, kT: float):
    """v ~ N(0, kT/m) with the centre-of-mass velocity removed (no rescale);
    body-frame L_k ~ N(0, I_k kT)."""
    n = shape_id.shape[0]
    m = np.array([shapes[s].mass for s in shape_id])
    I = np.array([shapes[s].inertia for s in shape_id])
    v = np.zeros((n, 3))
    v[:, :dim] = rng.standard_normal((n, dim)) * np.sqrt(kT / m)[:, None]
    vcm = (m[:, None] * v).sum(axis=0) / m.sum()
    v -= vcm
    L = np.zeros((n, 3))
    if dim == 2:
        L[:, 2] = rng.standard_normal(n) * np.sqrt(I[:, 2] * kT)
    else:
        L[:, :] = rng.standard_normal((n, 3)) * np.sqrt(I * kT)
    return v, L


def _grid_positions(ncell: int, dim: int, spacing: float) -> np.ndarray:
    idx = np.stack(np.meshgrid(*([np.arange(ncell)] * dim), indexing="ij"), axis=-1).reshape(-1, dim)
    x = np.zeros((idx.shape[0], 3))
    x[:, :dim] = (idx + 0.5) * spacing
    return x


def _bounding_overlap(x: np.ndarray, box: np.ndarray, reach: float, dim: int) -> bool:
    """True if any two bounding disks/spheres of radius `reach` overlap
    (a conservative stand-in for shape overlap, used only to reject inits)."""
    n = x.shape[0]
    for i in range(n):
        d = x[i + 1:, :dim] - x[i, :dim]
        d -= box[:dim] * np.rint(d / box[:dim])
        if np.any(np.sum(d * d, axis=1) < (2 * reach) ** 2):
            return True
    return False


def lattice_system(shape: Shape, n_side: int, fraction: float, seed: int, *, orient: str,
                   max_deg: float = 10.0, kT: float = 1.0, jitter: float = 0.0,
                   spacing: Optional[float] = None, name: str = "") -> System:
    """Square (2D) or simple-cubic (3D) lattice at an area/volume fraction of
    the rounded shape, or at an explicit spacing.

    orient: 'uniform' (2D angle ~ U[0, 2 pi) or uniform 3D rotation),
            'small' (3D axis uniform on S^2, angle ~ U[0, max_deg]; 2D angle ~
            U[-max_deg, max_deg]), or 'aligned'.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    dim = shape.dim
    n = n_side ** dim
    if spacing is None:
        L = (n * shape.volume / fraction) ** (1.0 / dim)
        spacing = L / n_side
    else:
        L = spacing * n_side
    box = np.array([L, L, L if dim == 3 else 1.0])
    x = _grid_positions(n_side, dim, spacing)
    if jitter > 0:
        x[:, :dim] += rng.uniform(-jitter, jitter, (n, dim))
        x[:, :dim] %= L
    if dim == 2:
        if orient == "uniform":
            th = rng.uniform(0.0, TWO_PI, n)
        elif orient == "small":
            th = np.deg2rad(rng.uniform(-max_deg, max_deg, n))
        else:
            th = np.zeros(n)
        q = planar_quaternions(th)
    else:
        if orient == "uniform":
            q = uniform_quaternions(rng, n)
        elif orient == "small":
            q = small_rotations(rng, n, max_deg)
        else:
            q = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    shape_id = np.zeros(n, dtype=np.int32)
    v, Lm = thermal_momenta(rng, [shape], shape_id, dim, kT)
    return System(dim=dim, box=box, shapes=[shape], shape_id=shape_id, x=x, q=q, v=v, L=Lm,
                  image=np.zeros((n, 3), dtype=np.int32), kT=kT, name=name)


def random_gas(shape: Shape, n: int, box_len: float, seed: int, *, min_sep: Optional[float] = None,
               kT: float = 1.0, name: str = "") -> System:
    """Random sequential placement with a minimum centre distance (default:
    twice the circumradius plus 0.8 sigma, so no two feature points come
    closer than 0.8 sigma) and uniform random orientations.  Pairs closer
    than 2R + 2^(1/6) sigma can touch."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dim = shape.dim
    if min_sep is None:
        min_sep = 2.0 * shape.circumradius + 0.8 * 2.0 * shape.r
    box = np.array([box_len, box_len, box_len if dim == 3 else 1.0])
    pts = []
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > 200 * n:
            raise RuntimeError("random_gas: density too high for sequential placement")
        p = rng.uniform(0.0, box_len, dim)
        ok = True
        for qpt in pts:
            d = p - qpt
            d -= box_len * np.rint(d / box_len)
            if d @ d < min_sep * min_sep:
                ok = False
                break
        if ok:
            pts.append(p)
    x = np.zeros((n, 3))
    x[:, :dim] = np.asarray(pts)
    q = planar_quaternions(rng.uniform(0, TWO_PI, n)) if dim == 2 else uniform_quaternions(rng, n)
    shape_id = np.zeros(n, dtype=np.int32)
    v, Lm = thermal_momenta(rng, [shape], shape_id, dim, kT)
    return System(dim=dim, box=box, shapes=[shape], shape_id=shape_id, x=x, q=q, v=v, L=Lm,
                  image=np.zeros((n, 3), dtype=np.int32), kT=kT, name=name)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------
def squares_2d(seed: int = 1) -> System:
    """256 rounded squares (edge 1, r = 0.25, so sigma = 0.5) on a 16 x 16
    lattice at rounded-area fraction 0.5, uniform random orientations, kT = 1,
    NVE, dt = 1e-4.  Orientations are resampled if bounding disks overlap (they
    never do at this spacing)."""
    shp = square(1.0, 0.25)
    s = lattice_system(shp, 16, 0.5, seed, orient="uniform", name="squares_2d_256")
    assert not _bounding_overlap(s.x, s.box, shp.circumradius + shp.r, 2)
    s.dt = 1e-4
    s.ensemble = "nve"
    return s


def squares_2d_contact(seed: int = 11) -> System:
    """Contact-rich 2D state: the same squares on a 16 x 16 lattice whose
    inner gap (1.1 sigma) lies inside the WCA range, angles ~ U[-3, 3] deg,
    positions jittered by U[-0.01, 0.01]."""
    shp = square(1.0, 0.25)
    s = lattice_system(shp, 16, 0.5, seed, orient="small", max_deg=3.0, jitter=0.01,
                       spacing=1.0 + 1.1 * 2 * shp.r, name="squares_2d_contact_256")
    s.dt = 1e-4
    s.ensemble = "nve"
    return s


def cubes_3d(seed: int = 2, n_side: int = 16) -> System:
    """4096 rounded cubes (edge 1, r = 0.15) at volume fraction 0.4 on a
    16^3 simple-cubic lattice, rotations up to 10 degrees about random axes,
    kT = 1, Nose-Hoover NVT, dt = 5e-4."""
    shp = cube(1.0, 0.15)
    s = lattice_system(shp, n_side, 0.4, seed, orient="small", max_deg=10.0, name=f"cubes_3d_{n_side ** 3}")
    s.dt = 5e-4
    s.ensemble = "nvt"
    return s


def cubes_3d_contact(seed: int = 12, n_side: int = 8) -> System:
    """Contact-rich cubes: simple-cubic spacing 1 + 1.08 sigma, rotations up
    to 2 degrees, positions jittered by U[-0.005, 0.005]."""
    shp = cube(1.0, 0.15)
    s = lattice_system(shp, n_side, 0.4, seed, orient="small", max_deg=2.0, jitter=0.005,
                       spacing=1.0 + 1.08 * 2 * shp.r, name=f"cubes_3d_contact_{n_side ** 3}")
    s.dt = 5e-4
    s.ensemble = "nvt"
    return s


def stored_state(name: str, template: System) -> System:
    """A stored state (positions, orientations, momenta, image counters and
    the thermostat variables `thermo` = (xi, eta)) on the template's box,
    shapes and parameters; the file's SHA-256 must match states.json."""
    entry = json.load(open(os.path.join(GOLDEN, "states.json")))[name]
    path = os.path.join(GOLDEN, entry["file"])
    with open(path, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    if digest != entry["sha256"]:
        raise RuntimeError(f"{path}: SHA-256 {digest} differs from states.json")
    z = np.load(path)
    s = template.copy()
    s.x, s.q, s.v, s.L = (np.ascontiguousarray(z[k], dtype=np.float64) for k in ("x", "q", "v", "L"))
    s.image = np.ascontiguousarray(z["image"], dtype=np.int32)
    if "box" in z.files:
        s.box = np.ascontiguousarray(z["box"], dtype=np.float64)
    s.thermo = tuple(float(t) for t in z["thermo"])
    s.step = int(z["step"])
    s.name = name
    return s


def cubes_3d_equilibrated() -> System:
    """The 4096-cube workload (cubes_3d) after 1000 steps of its own NVT run
    (0.5 tau), integrated by the oracle from the seeded lattice start: a
    fluid with contacts, for full-size parity and for timing."""
    return stored_state("cubes4096_nvt_step1000", cubes_3d())


def energy_fluid(dim: int, n_side: int = None, seed: int = 21) -> System:
    """The fluids of the energy-conservation study (Sec. IV.A): 2D rounded
    squares of edge 4.24 sigma (edge 1, r = 1 / 8.48) on a 32 x 32 lattice at
    area fraction 0.4 with uniform orientations, or 3D rounded tetrahedra of
    edge 8.49 sigma (edge 1, r = 1 / 16.98) on a 10^3 simple-cubic lattice at
    volume fraction 0.15, all aligned (the spacing, 1.17, exceeds the
    tetrahedron's extent plus 2r, 1.12, so no two touch).  kT = 1, unit mass;
    the study thermalizes them before its NVE runs.  The time unit is
    tau = sigma sqrt(m / eps) = 2 r."""
    if dim == 2:
        shp = square(1.0, 1.0 / (2 * 4.24))
        k = n_side or 32
        s = lattice_system(shp, k, 0.4, seed, orient="uniform", name=f"squares_4.24sigma_{k * k}")
        assert not _bounding_overlap(s.x, s.box, shp.circumradius + shp.r, 2)
    else:
        shp = tetrahedron(1.0, 1.0 / (2 * 8.49))
        k = n_side or 10
        s = lattice_system(shp, k, 0.15, seed, orient="aligned", name=f"tetrahedra_8.49sigma_{k ** 3}")
        assert s.box[0] / k > 1.0 + 2 * shp.r
    s.ensemble = "nvt"
    s.dt = 0.005 * 2 * shp.r
    return s


def _gas_box(shp: Shape, n: int, excl_fraction: float) -> float:
    sep = 2.0 * shp.circumradius + 0.8 * 2.0 * shp.r
    if shp.dim == 3:
        return (n * (math.pi / 6.0) * sep ** 3 / excl_fraction) ** (1.0 / 3.0)
    return (n * (math.pi / 4.0) * sep ** 2 / excl_fraction) ** 0.5


def gas_3d(shape_name: str = "cube", n: int = 512, excl_fraction: float = 0.3, seed: int = 13, **kw) -> System:
    """Random-orientation gas with exclusion spheres of diameter 2R + 0.8 sigma
    filling `excl_fraction` of the box (vertex, edge and face contacts at
    arbitrary angles)."""
    shp = SHAPES[shape_name](**kw)
    s = random_gas(shp, n, _gas_box(shp, n, excl_fraction), seed, name=f"gas_{shape_name}_{n}")
    s.dt = 5e-4
    s.ensemble = "nve"
    return s


def gas_2d(n: int = 256, excl_fraction: float = 0.45, seed: int = 14, shape_name: str = "square") -> System:
    shp = SHAPES[shape_name]()
    s = random_gas(shp, n, _gas_box(shp, n, excl_fraction), seed, name=f"gas2d_{shape_name}_{n}")
    s.dt = 1e-4
    s.ensemble = "nve"
    return s


def dimer_gas(shape_name: str = "cube", n_pairs: int = 128, seed: int = 15, gap=(0.85, 1.1),
              excl_fraction: float = 0.25, dim: int = 3, **kw) -> System:
    """Gas of close pairs at arbitrary angles.

    Each pair has uniform random orientations and a random direction u; the
    second centre sits at distance h_i(u) + h_j(-u) + g along u, where h is
    the support function of the inner shape (max over vertices of v.u), so
    the inner shapes' projections on u are exactly g apart (no overlap).
    g ~ U[gap] * sigma.  The inner bodies' distance is g or more (more when
    u is not a direction in which their nearest features face each other),
    so only part of the pairs are in contact: by the oracle's count 24 of
    128 cube pairs, 20 of 128 octahedron pairs and 8 of 128 tetrahedron
    pairs at the default seed.  contact_dimers places pairs that are all in
    contact.  Pairs are placed at random with exclusion spheres around each
    pair."""
    shp = SHAPES[shape_name](**kw)
    rng = np.random.Generator(np.random.PCG64(seed))
    sigma = 2.0 * shp.r
    R = shp.circumradius
    reach = 2.0 * R + gap[1] * sigma
    excl_r = 0.5 * reach + R + 1.2 * sigma
    if dim == 3:
        Lb = (n_pairs * (4.0 / 3.0) * math.pi * excl_r ** 3 / excl_fraction) ** (1.0 / 3.0)
    else:
        Lb = (n_pairs * math.pi * excl_r ** 2 / excl_fraction) ** 0.5
    box = np.array([Lb, Lb, Lb if dim == 3 else 1.0])
    n = 2 * n_pairs
    x = np.zeros((n, 3))
    q = np.zeros((n, 4))
    centres = []
    k = 0
    tries = 0
    while k < n_pairs:
        tries += 1
        if tries > 500 * n_pairs:
            raise RuntimeError("dimer_gas: cannot place pairs")
        c = rng.uniform(0.0, Lb, dim)
        ok = True
        for cc in centres:
            d = c - cc
            d -= Lb * np.rint(d / Lb)
            if d @ d < (2 * excl_r) ** 2:
                ok = False
                break
        if not ok:
            continue
        if dim == 3:
            qa, qb = uniform_quaternions(rng, 2)
            u = random_unit_vectors(rng, 1)[0]
        else:
            qa, qb = planar_quaternions(rng.uniform(0.0, TWO_PI, 2))
            a = rng.uniform(0.0, TWO_PI)
            u = np.array([math.cos(a), math.sin(a), 0.0])
        Ra, Rb = _qmat(qa), _qmat(qb)
        ha = np.max((shp.vertices @ Ra.T) @ u)
        hb = np.max((shp.vertices @ Rb.T) @ (-u))
        g = rng.uniform(gap[0], gap[1]) * sigma
        D = ha + hb + g
        p0 = np.zeros(3)
        p0[:dim] = c
        p0 -= 0.5 * D * u
        p1 = p0 + D * u
        x[2 * k], x[2 * k + 1] = p0, p1
        q[2 * k], q[2 * k + 1] = qa, qb
        centres.append(c)
        k += 1
    x[:, :dim] %= Lb
    shape_id = np.zeros(n, dtype=np.int32)
    v, Lm = thermal_momenta(rng, [shp], shape_id, dim, 1.0)
    s = System(dim=dim, box=box, shapes=[shp], shape_id=shape_id, x=x, q=q, v=v, L=Lm,
               image=np.zeros((n, 3), dtype=np.int32), name=f"dimers_{shape_name}_{n}")
    s.dt = 5e-4 if dim == 3 else 1e-4
    return s


def _unit(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v)


def _supporting_features(shp: Shape):
    """The features of an inner shape that can face another body across a
    separating plane, each with a direction u in which it is the shape's
    whole support set (every other vertex lies strictly lower along u):
    faces (2D: edges) whose plane has the whole body on one side, with their
    outward normal; edges (3D) and vertices where only such faces meet, with
    the normalised sum of those faces' normals.  Returns a list of
    (kind, vertex indices, u) with kind 'face', 'edge' or 'vertex'."""
    V = shp.vertices
    if shp.dim == 3:
        loops = [list(f) for f in shp.faces]
        normals = [_newell(V, f) for f in loops]
    else:
        loops = [[k, (k + 1) % shp.nv] for k in range(shp.nv)] if shp.nv > 1 else []  # (a disk has no edges)
        normals = [_unit(np.array([V[b, 1] - V[a, 1], V[a, 0] - V[b, 0], 0.0])) for a, b in loops]

    def strict(idx, u):
        top = min(float(V[k] @ u) for k in idx)
        rest = [float(V[k] @ u) for k in range(shp.nv) if k not in idx]
        return all(abs(float(V[k] @ u) - top) < 1e-9 for k in idx) and (not rest or max(rest) < top - 1e-6)

    out = []
    sup = []
    for f, nf in zip(loops, normals):
        if strict(f, nf):
            out.append(("face", list(f), nf))
            sup.append((set(f), nf))
    if shp.dim == 3:
        for a, b in shp.edges:
            adj = [nf for f, nf in zip(loops, normals) if a in f and b in f]
            if len(adj) == 2 and all(any(nf is n2 for _, n2 in sup) for nf in adj):
                u = _unit(adj[0] + adj[1])
                if strict([int(a), int(b)], u):
                    out.append(("edge", [int(a), int(b)], u))
    for k in range(shp.nv):
        adj = [nf for f, nf in zip(loops, normals) if k in f]
        if adj and all(any(nf is n2 for _, n2 in sup) for nf in adj):
            u = _unit(np.sum(adj, axis=0))
            if strict([k], u):
                out.append(("vertex", [k], u))
    return out


def _align(dim: int, n_body: np.ndarray, target: np.ndarray, spin: float) -> np.ndarray:
    """A quaternion that turns the body-frame unit vector n_body onto the
    space-frame unit vector target, then spins by `spin` about target (3D);
    in 2D the rotation about z that does the same."""
    if dim == 2:
        th = math.atan2(target[1], target[0]) - math.atan2(n_body[1], n_body[0])
        return planar_quaternions(np.array([th]))[0]
    c = float(np.clip(n_body @ target, -1.0, 1.0))
    ax = np.cross(n_body, target)
    if np.linalg.norm(ax) < 1e-12:  # parallel or antiparallel
        ax = np.cross(n_body, [1.0, 0.0, 0.0] if abs(n_body[0]) < 0.9 else [0.0, 1.0, 0.0])
    q0 = quat_from_axis_angle(_unit(ax), math.acos(c))
    qs = quat_from_axis_angle(target, spin)
    q = _quat_mul(qs, q0)
    return q / np.linalg.norm(q)


def contact_dimers(shape_a: Shape, shape_b: Optional[Shape] = None, n_pairs: int = 128, seed: int = 16,
                   gap=(0.85, 1.1), excl_fraction: float = 0.25, notch: bool = False, name: str = "") -> System:
    """Pairs that are all in contact, over every kind of facing features.

    For each pair, body A takes a uniform random orientation and one of its
    supporting features (a face, an edge or a vertex, see
    _supporting_features) with its direction u; the anchor point P is a
    random point of that feature (a random convex combination of a face's
    vertices, a point of an edge, the vertex).  A's inner body lies in the
    half space (x - P).u <= 0.  Body B then faces A with a vertex (uniform
    random orientation, its lowest vertex along u), an edge or a face (a
    supporting edge or face of B turned to face -u, random spin about u),
    whose point (the vertex, the edge's midpoint, the face's vertex
    centroid) is put at P + g u, g ~ U[gap] sigma_AB.  B's inner body lies in
    (x - P).u >= g, so the inner bodies are exactly g apart, inside the WCA
    cutoff 2^(1/6) sigma for gap[1] < 2^(1/6).

    notch=True: A is the concave L-prism and its anchor is a point of one of
    its two concave caps (the L-hexagon (0,0),(2,0),(2,1),(1,1),(1,2),(0,2)),
    drawn uniformly from the square [0.55, 1.45]^2 around the reflex corner
    (1,1): three quarters of these points lie on the cap, a quarter over
    the notch, where B's point hangs g above the cap plane but off the
    face, so its nearest point on A lies on the notch's edges (a contact
    when that distance is below the cutoff).  Pairs are placed at random
    with exclusion spheres around each pair; shape ids are 0 for A and 1 for
    B (when shape_b is given)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sb = shape_a if shape_b is None else shape_b
    dim = shape_a.dim
    shapes = [shape_a] if shape_b is None else [shape_a, shape_b]
    sigma = shape_a.r + sb.r
    feats_a = _supporting_features(shape_a)
    feats_b = [f for f in _supporting_features(sb) if f[0] != "vertex"]
    Ra, Rb = shape_a.circumradius, sb.circumradius
    reach = Ra + Rb + gap[1] * sigma
    excl_r = 0.5 * (Ra + Rb + reach) + 1.2 * sigma
    if dim == 3:
        Lb = (n_pairs * (4.0 / 3.0) * math.pi * excl_r ** 3 / excl_fraction) ** (1.0 / 3.0)
    else:
        Lb = (n_pairs * math.pi * excl_r ** 2 / excl_fraction) ** 0.5
    box = np.array([Lb, Lb, Lb if dim == 3 else 1.0])
    n = 2 * n_pairs
    x = np.zeros((n, 3))
    q = np.zeros((n, 4))
    centres = []
    k = 0
    tries = 0
    while k < n_pairs:
        tries += 1
        if tries > 500 * n_pairs:
            raise RuntimeError("contact_dimers: cannot place pairs")
        c = rng.uniform(0.0, Lb, dim)
        ok = True
        for cc in centres:
            d = c - cc
            d -= Lb * np.rint(d / Lb)
            if d @ d < (2 * excl_r) ** 2:
                ok = False
                break
        if not ok:
            continue
        qa = planar_quaternions(rng.uniform(0.0, TWO_PI, 1))[0] if dim == 2 else uniform_quaternions(rng, 1)[0]
        Ma = _qmat(qa)
        if notch:
            com, U = shape_a.frame
            top = rng.random() < 0.5
            xy = rng.uniform(0.55, 1.45, 2)
            p_body = (np.array([xy[0], xy[1], 1.0 if top else 0.0]) - com) @ U
            n_body = np.array([0.0, 0.0, 1.0 if top else -1.0]) @ U
        else:
            kind, idx, n_body = feats_a[int(rng.integers(len(feats_a)))]
            if kind == "face":
                wts = rng.dirichlet(np.ones(len(idx)))
                p_body = wts @ shape_a.vertices[idx]
            elif kind == "edge":
                t = rng.uniform(0.1, 0.9)
                p_body = (1 - t) * shape_a.vertices[idx[0]] + t * shape_a.vertices[idx[1]]
            else:
                p_body = shape_a.vertices[idx[0]].copy()
        u = Ma @ n_body
        mode = int(rng.integers(3)) if feats_b else 0
        if mode == 0:  # B faces A with a vertex
            qb = planar_quaternions(rng.uniform(0.0, TWO_PI, 1))[0] if dim == 2 else uniform_quaternions(rng, 1)[0]
            Mb = _qmat(qb)
            pb = sb.vertices[int(np.argmin((sb.vertices @ Mb.T) @ u))]
        else:  # with a supporting edge or face of its own
            kinds = ("edge", "face") if dim == 3 else ("face",)
            cand = [f for f in feats_b if f[0] == kinds[(mode - 1) % len(kinds)]] or feats_b
            kb, idb, nb = cand[int(rng.integers(len(cand)))]
            qb = _align(dim, nb, -u, rng.uniform(0.0, TWO_PI))
            Mb = _qmat(qb)
            pb = sb.vertices[idb].mean(axis=0)
        g = rng.uniform(gap[0], gap[1]) * sigma
        off = Ma @ p_body + g * u - Mb @ pb  # x_B - x_A
        p0 = np.zeros(3)
        p0[:dim] = c
        p0[:dim] -= 0.5 * off[:dim]
        x[2 * k] = p0
        x[2 * k + 1] = p0
        x[2 * k + 1, :dim] += off[:dim]
        q[2 * k], q[2 * k + 1] = qa, qb
        centres.append(c)
        k += 1
    x[:, :dim] %= Lb
    shape_id = np.zeros(n, dtype=np.int32)
    if shape_b is not None:
        shape_id[1::2] = 1
    v, Lm = thermal_momenta(rng, shapes, shape_id, dim, 1.0)
    s = System(dim=dim, box=box, shapes=shapes, shape_id=shape_id, x=x, q=q, v=v, L=Lm,
               image=np.zeros((n, 3), dtype=np.int32), name=name or f"contact_{shape_a.name}_{n}")
    s.dt = 5e-4 if dim == 3 else 1e-4
    return s


def _qmat(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


# --------------------------------------------------------------------------
# Octahedra at scale
# --------------------------------------------------------------------------
def _quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product a b (rotation b first, then a); rows (w, x, y, z)."""
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([aw * bw - ax * bx - ay * by - az * bz, aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx, aw * bz + ax * by - ay * bx + az * bw], axis=-1)


def _cross_polytope_distance(p: np.ndarray, c: float) -> np.ndarray:
    """Euclidean distance from points p (..., 3) to {x : |x|_1 <= c}, by the
    sorted-threshold projection onto the l1 ball."""
    ap = np.abs(p)
    u = -np.sort(-ap, axis=-1)
    cs = np.cumsum(u, axis=-1)
    k = np.arange(1, p.shape[-1] + 1)
    ok = u - (cs - c) / k > 0
    rho = p.shape[-1] - 1 - np.argmax(ok[..., ::-1], axis=-1)
    theta = (np.take_along_axis(cs, rho[..., None], -1)[..., 0] - c) / (rho + 1)
    w = np.sign(p) * np.maximum(ap - theta[..., None], 0.0)
    inside = ap.sum(-1) <= c
    return np.where(inside, 0.0, np.linalg.norm(p - w, axis=-1))


def octahedra_3d(seed: int = 3, n: int = 262144, fraction: float = 0.55, n_cells: int = 51,
                 max_deg: float = 5.0, jitter: float = 0.0, kT: float = 1.0, trials: int = 4000) -> System:
    """n rounded octahedra (edge 1, r = 0.1) at volume fraction `fraction` on
    a BCC lattice of n_cells^3 cubic cells (2 n_cells^3 sites, n of them
    drawn at random, the rest left empty), box L = (n V / fraction)^(1/3).

    All bodies share one orientation: of `trials` seeded uniform rotations,
    the one that maximises the smallest distance between the inner
    octahedra of two lattice sites (K - K = 2K for the centrally symmetric
    octahedron K, so that distance is the distance from the site offset,
    in the body frame, to 2K), recorded as `min_gap`.  Each body is then
    rotated by <= max_deg about a random axis, which brings no two inner
    bodies closer than min_gap - 4 sin(max_deg / 2) R, and moved by
    U[-jitter, jitter] per axis.  NVT, kT = 1, dt = 2e-4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shp = octahedron(1.0, 0.1)
    a = float(np.abs(shp.vertices).max())  # the inner octahedron is |x|_1 <= a
    L = (n * shp.volume / fraction) ** (1.0 / 3.0)
    cell = L / n_cells
    offs = []
    for i in range(-2, 3):
        for j in range(-2, 3):
            for k in range(-2, 3):
                for h in (0.0, 0.5):
                    d = np.array([i + h, j + h, k + h]) * cell
                    if 1e-9 < np.linalg.norm(d) < 2.0 * shp.circumradius + 2.5 * shp.r:
                        offs.append(d)
    offs = np.array(offs)
    qs = uniform_quaternions(rng, trials)
    gaps = np.array([_cross_polytope_distance(offs @ _qmat(q), 2.0 * a).min() for q in qs])
    best = int(np.argmax(gaps))
    q0 = qs[best]
    g = np.arange(n_cells)
    corner = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.float64)
    sites = np.concatenate([corner, corner + 0.5]) * cell
    pick = np.sort(rng.choice(sites.shape[0], size=n, replace=False))
    x = sites[pick]
    if jitter > 0:
        x = x + rng.uniform(-jitter, jitter, x.shape)
    x %= L
    q = _quat_mul(small_rotations(rng, n, max_deg), np.tile(q0, (n, 1)))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    shape_id = np.zeros(n, dtype=np.int32)
    v, Lm = thermal_momenta(rng, [shp], shape_id, 3, kT)
    s = System(dim=3, box=np.array([L, L, L]), shapes=[shp], shape_id=shape_id, x=x, q=q, v=v, L=Lm,
               image=np.zeros((n, 3), dtype=np.int32), kT=kT, dt=2e-4, ensemble="nvt",
               name=f"octahedra_bcc_{n}")
    s.min_gap = float(gaps[best])
    return s


def octahedra_bcc_dilute(seed: int = 3, n: int = 4096, n_cells: int = 13, fraction: float = 0.25,
                         kT: float = 1.0) -> System:
    """n rounded octahedra (edge 1, r 0.1) with uniform random orientations
    on a BCC lattice of n_cells^3 cubic cells (2 n_cells^3 sites, n of them
    drawn at random), box L = (n V / fraction)^(1/3).  At fraction 0.25 the
    BCC nearest-neighbour distance exceeds twice the rounded circumradius,
    so no two bodies touch whatever their orientations.  NVT, kT = 1,
    dt = 2e-4: the start the compressed at-scale state is made from."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shp = octahedron(1.0, 0.1)
    L = (n * shp.volume / fraction) ** (1.0 / 3.0)
    cell = L / n_cells
    assert 0.5 * math.sqrt(3.0) * cell > 2.0 * (shp.circumradius + shp.r)
    g = np.arange(n_cells)
    corner = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.float64)
    sites = np.concatenate([corner + 0.25, corner + 0.75]) * cell
    x = sites[np.sort(rng.choice(sites.shape[0], size=n, replace=False))]
    q = uniform_quaternions(rng, n)
    shape_id = np.zeros(n, dtype=np.int32)
    v, Lm = thermal_momenta(rng, [shp], shape_id, 3, kT)
    return System(dim=3, box=np.array([L, L, L]), shapes=[shp], shape_id=shape_id, x=x, q=q, v=v, L=Lm,
                  image=np.zeros((n, 3), dtype=np.int32), kT=kT, dt=2e-4, ensemble="nvt",
                  name=f"octahedra_bcc_dilute_{n}")


def tile(s: System, k: int) -> System:
    """The periodic system s repeated k times along every axis (a valid
    periodic state of the k^d times larger box); momenta and image counters
    are copied with each particle."""
    dim = s.dim
    shifts = np.stack(np.meshgrid(*([np.arange(k)] * dim), indexing="ij"), axis=-1).reshape(-1, dim)
    x = np.concatenate([s.x + np.pad(t * s.box[:dim], (0, 3 - dim)) for t in shifts])
    t = s.copy()
    t.box = s.box.copy()
    t.box[:dim] *= k
    t.x = np.ascontiguousarray(x)
    t.q = np.ascontiguousarray(np.tile(s.q, (len(shifts), 1)))
    t.v = np.ascontiguousarray(np.tile(s.v, (len(shifts), 1)))
    t.L = np.ascontiguousarray(np.tile(s.L, (len(shifts), 1)))
    t.image = np.zeros((x.shape[0], 3), dtype=np.int32)
    t.shape_id = np.tile(s.shape_id, len(shifts))
    return t


def octahedra_compressed() -> System:
    """The at-scale workload: 262,144 rounded octahedra (edge 1, r 0.1) at
    volume fraction 0.55, NVT kT = 1, dt = 2e-4: a 4096-body cell compressed
    by the oracle from random orientations on a dilute BCC lattice
    (octahedra_bcc_dilute, tests/golden/make_states.py), tiled 4 x 4 x 4."""
    cell = stored_state("octahedra4096_compressed", octahedra_bcc_dilute())
    s = tile(cell, 4)
    s.name = "octahedra262144_compressed"
    s.thermo = None  # the tiled system has 64 times the degrees of freedom: its thermostat starts afresh
    return s


# --------------------------------------------------------------------------
# Replicas for batched and served runs
# --------------------------------------------------------------------------
# Time steps per shape (2D 1e-4, cube and tetrahedron and L-prism 5e-4,
# octahedron 2e-4).
DT = {"square": 1e-4, "pentagon": 1e-4, "cube": 5e-4, "tetrahedron": 5e-4, "lprism": 5e-4, "octahedron": 2e-4}


def replica_system(shape: Shape, n: int, fraction: float, seed: int, *, kT: float = 1.0, max_deg: float = 10.0,
                   dt: float = 5e-4, ensemble: str = "nvt", name: str = "") -> System:
    """n particles on an orthorhombic (2D: rectangular) lattice, n of its
    sites drawn at random, rotations up to max_deg (3D: about random axes;
    2D: in [-max_deg, max_deg]).  The lattice cell is the shape's rounded
    bounding box widened by 4 sin(max_deg / 2) R on every axis (a rotation
    by at most max_deg moves no point of the body farther than
    2 sin(max_deg / 2) R), stretched by a common factor >= 1 to reach the
    requested area or volume fraction; where even the unstretched cell is
    too large, the lattice is that cell and `fraction_realized` says what it
    gives.  Neighbouring bodies can therefore not overlap."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dim = shape.dim
    ext = shape.vertices[:, :dim].max(axis=0) - shape.vertices[:, :dim].min(axis=0) + 2.0 * shape.r
    ext = ext + 4.0 * math.sin(math.radians(max_deg) / 2.0) * shape.circumradius
    c = (n * float(np.prod(ext))) ** (1.0 / dim)
    k = np.maximum(1, np.rint(c / ext)).astype(int)
    while int(np.prod(k)) < n:
        a = int(np.argmin(k * ext))
        k[a] += 1
    lam = (n * shape.volume / (fraction * float(np.prod(k * ext)))) ** (1.0 / dim)
    lam = max(lam, 1.0)
    spacing = lam * ext
    box = np.ones(3)
    box[:dim] = k * spacing
    sites = np.sort(rng.choice(int(np.prod(k)), size=n, replace=False))
    idx = np.stack(np.unravel_index(sites, tuple(k)), axis=1)
    x = np.zeros((n, 3))
    x[:, :dim] = (idx + 0.5) * spacing
    if dim == 2:
        q = planar_quaternions(np.deg2rad(rng.uniform(-max_deg, max_deg, n)))
    else:
        q = small_rotations(rng, n, max_deg)
    shape_id = np.zeros(n, dtype=np.int32)
    v, Lm = thermal_momenta(rng, [shape], shape_id, dim, kT)
    s = System(dim=dim, box=box, shapes=[shape], shape_id=shape_id, x=x, q=q, v=v, L=Lm,
               image=np.zeros((n, 3), dtype=np.int32), kT=kT, name=name)
    s.dt = dt
    s.ensemble = ensemble
    s.fraction_realized = n * shape.volume / float(np.prod(box[:dim]))
    return s


def batched_replicas(count: int = 96, seed: int = 4, n_range=(512, 32768), steps: int = 500) -> List[System]:
    """The batched workload: `count` independent NVT replicas (kT = 1), sizes
    log-uniform in n_range, shapes uniform over {rounded cube, rounded
    tetrahedron, concave L-prism}, rounding radius U[0.1, 0.2], packing
    fraction U[0.3, 0.5] (capped by the lattice, see replica_system),
    replica r drawn from seed 1000 * seed + r.  `steps` is recorded on each
    as `steps`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    names = ("cube", "tetrahedron", "lprism")
    out = []
    for r in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        name = names[int(rng.integers(0, 3))]
        rr = float(rng.uniform(0.1, 0.2))
        phi = float(rng.uniform(0.3, 0.5))
        shp = SHAPES[name](r=rr) if name != "lprism" else lprism(r=rr, quad_h=0.02)
        s = replica_system(shp, n, phi, 1000 * seed + r, dt=DT[name], name=f"replica{r}_{name}_{n}")
        s.steps = steps
        s.fraction_requested = phi
        out.append(s)
    return out


def contact_lattice(shape: Shape, n: int, seed: int, *, gap: float = 1.05, max_deg: float = 0.25, kT: float = 1.0,
                    dt: float = 5e-4, ensemble: str = "nvt", name: str = "") -> System:
    """n bodies on an orthorhombic lattice whose spacing on each axis is the
    inner body's extent on that axis plus gap * sigma (sigma = 2 r), n of its
    sites drawn at random, rotated by at most max_deg about random axes.
    Aligned neighbours face each other across exactly gap * sigma (faces of
    cubes and L-prisms, crossed edges of tetrahedra); a rotation by at most
    max_deg moves no point of a body by more than 2 sin(max_deg / 2) R, so
    every inner gap between lattice neighbours lies within
    gap * sigma +- 4 sin(max_deg / 2) R: inside the WCA cutoff 2^(1/6) sigma
    and above zero for the defaults and rounding radii of 0.1 and more."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dim = shape.dim
    ext = shape.vertices[:, :dim].max(axis=0) - shape.vertices[:, :dim].min(axis=0)
    spacing = ext + gap * 2.0 * shape.r
    c = (n * float(np.prod(spacing))) ** (1.0 / dim)
    k = np.maximum(1, np.rint(c / spacing)).astype(int)
    while int(np.prod(k)) < n:
        a = int(np.argmin(k * spacing))
        k[a] += 1
    box = np.ones(3)
    box[:dim] = k * spacing
    sites = np.sort(rng.choice(int(np.prod(k)), size=n, replace=False))
    idx = np.stack(np.unravel_index(sites, tuple(k)), axis=1)
    x = np.zeros((n, 3))
    x[:, :dim] = (idx + 0.5) * spacing
    if dim == 2:
        q = planar_quaternions(np.deg2rad(rng.uniform(-max_deg, max_deg, n)))
    else:
        q = small_rotations(rng, n, max_deg)
    shape_id = np.zeros(n, dtype=np.int32)
    v, Lm = thermal_momenta(rng, [shape], shape_id, dim, kT)
    s = System(dim=dim, box=box, shapes=[shape], shape_id=shape_id, x=x, q=q, v=v, L=Lm,
               image=np.zeros((n, 3), dtype=np.int32), kT=kT, name=name)
    s.dt = dt
    s.ensemble = ensemble
    return s


def batched_replicas_contact(count: int = 96, seed: int = 4, n_range=(512, 32768), steps: int = 500) -> List[System]:
    """The batched workload's replicas (the same sizes, shapes and rounding
    radii, drawn from the same seeds as batched_replicas) on contact
    lattices (contact_lattice): every lattice neighbour in contact, so a
    full-size batch exercises every replica's feature pairs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    names = ("cube", "tetrahedron", "lprism")
    out = []
    for r in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        name = names[int(rng.integers(0, 3))]
        rr = float(rng.uniform(0.1, 0.2))
        rng.uniform(0.3, 0.5)  # the packing fraction draw of batched_replicas, unused here
        shp = SHAPES[name](r=rr) if name != "lprism" else lprism(r=rr, quad_h=0.02)
        s = contact_lattice(shp, n, 1000 * seed + r, dt=DT[name], name=f"replica{r}_{name}_{n}_contact")
        s.steps = steps
        out.append(s)
    return out


def served_trace(count: int = 256, seed: int = 5, rate: float = 40.0, n_range=(256, 65536),
                 steps_range=(1000, 5000)) -> List[System]:
    """The served workload: `count` requests arriving as a Poisson process of
    `rate` per second (attribute `arrival`, seconds), each an NVT replica of
    size log-uniform in n_range, shape uniform over {2D rounded pentagon, 3D
    rounded cube, 3D rounded octahedron}, rounding U[0.1, 0.2], packing
    fraction U[0.3, 0.5] (capped by the lattice), kT U[0.5, 2.0] and
    U{steps_range} steps (attribute `steps`); request k drawn from seed
    1000 * seed + k."""
    rng = np.random.Generator(np.random.PCG64(seed))
    names = ("pentagon", "cube", "octahedron")
    t = 0.0
    out = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        name = names[int(rng.integers(0, 3))]
        rr = float(rng.uniform(0.1, 0.2))
        phi = float(rng.uniform(0.3, 0.5))
        kT = float(rng.uniform(0.5, 2.0))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        shp = SHAPES[name](r=rr)
        s = replica_system(shp, n, phi, 1000 * seed + k, kT=kT, dt=DT[name], name=f"request{k}_{name}_{n}")
        s.arrival = t
        s.steps = steps
        s.fraction_requested = phi
        out.append(s)
    return out
