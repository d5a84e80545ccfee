"""ctypes wrapper of the FP64 CPU oracle (dem_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this package; the HIP library never loads it.

Inputs are duck-typed: any object with the attributes of a system
(dim, box, shapes, shape_id, x, q, v, L, image, epsilon, parallel_sin2) and
shapes with (dim, vertices, edges, faces, r, mass, inertia).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _OrSys(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n_shapes", C.c_int),
        ("nv", _ip), ("ne", _ip), ("nf", _ip),
        ("v_off", _ip), ("e_off", _ip), ("f_off", _ip),
        ("verts", _dp), ("edges", _ip), ("fl_off", _ip), ("floops", _ip),
        ("rad", _dp), ("mass", _dp), ("inertia", _dp),
        ("box", C.c_double * 3), ("epsilon", C.c_double), ("par_s2", C.c_double),
    ]


class PairOut(C.Structure):
    _fields_ = [("U", C.c_double), ("Fi", C.c_double * 3), ("Ti", C.c_double * 3), ("Tj", C.c_double * 3),
                ("W", C.c_double * 9), ("Fabs", C.c_double), ("Tabs_i", C.c_double), ("Wabs", C.c_double),
                ("n_in", C.c_int), ("n_par", C.c_int), ("n_near_par", C.c_int)]


class Term(C.Structure):
    _fields_ = [("family", C.c_int), ("a", C.c_int), ("b", C.c_int), ("inside", C.c_int), ("par", C.c_int),
                ("r", C.c_double)]


TERM_FAMILIES = {0: "EiEj", 1: "ViFj", 2: "VjFi", 3: "ViEj", 4: "VjEi", 5: "ViVj"}


class Stats(C.Structure):
    _fields_ = [("n_pairs_bound", C.c_long), ("n_feature_in", C.c_long), ("n_par", C.c_long),
                ("n_near_par", C.c_long)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        L.or_wca.argtypes = [C.c_double, C.c_double, C.c_double, _dp, _dp]
        L.or_wca.restype = C.c_int
        L.or_point_segment.argtypes = [_dp, _dp, _dp, _dp]
        L.or_segment_segment.argtypes = [_dp, _dp, _dp, _dp, C.c_double, _dp, _dp]
        L.or_segment_segment.restype = C.c_int
        L.or_point_polygon.argtypes = [_dp, _dp, C.c_int, _dp]
        L.or_pair.argtypes = [C.POINTER(_OrSys), C.c_int, C.c_int, _dp, _dp, _dp, _dp, C.POINTER(PairOut)]
        L.or_pair_terms.argtypes = [C.POINTER(_OrSys), C.c_int, C.c_int, _dp, _dp, _dp, _dp, C.POINTER(Term), C.c_int]
        L.or_pair_terms.restype = C.c_int
        L.or_r_list.argtypes = [C.POINTER(_OrSys), C.c_double]
        L.or_r_list.restype = C.c_double
        L.or_cell_dims.argtypes = [C.POINTER(_OrSys), C.c_double, _ip]
        L.or_cell_list.argtypes = [C.POINTER(_OrSys), C.c_int, _dp, C.c_double, _ip, _ip]
        L.or_cell_list.restype = C.c_int
        L.or_nbr_list.argtypes = [C.POINTER(_OrSys), C.c_int, _dp, C.c_double, C.c_int, C.c_int, _ip, _ip]
        L.or_nbr_list.restype = C.c_int
        L.or_forces.argtypes = [C.POINTER(_OrSys), C.c_int, _dp, _dp, _ip, C.c_int, _dp, _dp, _dp, _dp,
                                C.POINTER(Stats), _dp]
        L.or_forces_subset.argtypes = [C.POINTER(_OrSys), C.c_int, _dp, _dp, _ip, C.c_int, _ip, C.c_int, _dp, _dp,
                                       _dp, _dp, C.POINTER(Stats), _dp]
        L.or_run.argtypes = [C.POINTER(_OrSys), C.c_int, _dp, _dp, _dp, _dp, _ip, _ip, C.c_int, C.c_double,
                             C.c_int, C.c_double, C.c_double, _dp, C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.or_run_npt.argtypes = [C.POINTER(_OrSys), C.c_int, _dp, _dp, _dp, _dp, _ip, _ip, C.c_int, C.c_double,
                                 C.c_double, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp, C.c_int, _dp, _dp,
                                 _dp, _dp, _dp]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _vec(x):
    a = np.zeros(3)
    x = np.asarray(x, dtype=np.float64).ravel()
    a[: x.size] = x
    return a


class OracleSystem:
    """Packs shapes and box into the oracle's flat tables (kept alive here)."""

    def __init__(self, dim, box, shapes, epsilon=1.0, parallel_sin2=1e-6):
        self.dim = int(dim)
        nv, ne, nf, v_off, e_off, f_off, fl_off = [], [], [], [0], [0], [0], [0]
        verts, edges, loops = [], [], []
        for s in shapes:
            nv.append(s.vertices.shape[0])
            ne.append(s.edges.shape[0])
            nf.append(len(s.faces))
            v_off.append(v_off[-1] + nv[-1])
            e_off.append(e_off[-1] + ne[-1])
            f_off.append(f_off[-1] + nf[-1])
            verts.append(np.asarray(s.vertices, dtype=np.float64).reshape(-1, 3))
            edges.append(np.asarray(s.edges, dtype=np.int32).reshape(-1, 2))
            for f in s.faces:
                loops.extend(int(v) for v in f)
                fl_off.append(fl_off[-1] + len(f))
        self._keep = dict(
            nv=np.asarray(nv, np.int32), ne=np.asarray(ne, np.int32), nf=np.asarray(nf, np.int32),
            v_off=np.asarray(v_off, np.int32), e_off=np.asarray(e_off, np.int32), f_off=np.asarray(f_off, np.int32),
            verts=np.ascontiguousarray(np.concatenate(verts), dtype=np.float64),
            edges=np.ascontiguousarray(np.concatenate(edges), dtype=np.int32),
            fl_off=np.asarray(fl_off, np.int32), floops=np.asarray(loops if loops else [0], np.int32),
            rad=np.asarray([s.r for s in shapes], np.float64), mass=np.asarray([s.mass for s in shapes], np.float64),
            inertia=np.ascontiguousarray(np.asarray([s.inertia for s in shapes], np.float64).reshape(-1)),
        )
        k = self._keep
        self.c = _OrSys()
        self.c.dim = self.dim
        self.c.n_shapes = len(shapes)
        for name in ("nv", "ne", "nf", "v_off", "e_off", "f_off", "edges", "fl_off", "floops"):
            setattr(self.c, name, _i(k[name]))
        for name in ("verts", "rad", "mass", "inertia"):
            setattr(self.c, name, _d(k[name]))
        b = np.asarray(box, dtype=np.float64).ravel()
        for a in range(3):
            self.c.box[a] = float(b[a]) if a < b.size else 1.0
        self.c.epsilon = float(epsilon)
        self.c.par_s2 = float(parallel_sin2)

    @classmethod
    def of(cls, sysobj) -> "OracleSystem":
        return cls(sysobj.dim, sysobj.box, sysobj.shapes, sysobj.epsilon, sysobj.parallel_sin2)

    def r_list(self, skin):
        return lib().or_r_list(C.byref(self.c), float(skin))

    def cell_dims(self, r_list):
        nc = np.zeros(3, np.int32)
        lib().or_cell_dims(C.byref(self.c), float(r_list), _i(nc))
        return nc


# ---------------------------------------------------------------- primitives
def wca(r, sigma, eps=1.0):
    U = C.c_double()
    fr = C.c_double()
    inside = lib().or_wca(float(r) * float(r), float(sigma), float(eps), C.byref(U), C.byref(fr))
    return U.value, fr.value * float(r), bool(inside)  # (U, force magnitude -dU/dr, inside)


def point_segment(p, a, b):
    q = np.zeros(3)
    lib().or_point_segment(_d(_vec(p)), _d(_vec(a)), _d(_vec(b)), _d(q))
    return q


def segment_segment(a0, a1, b0, b1, par_s2=1e-6):
    P = np.zeros(3)
    Q = np.zeros(3)
    par = lib().or_segment_segment(_d(_vec(a0)), _d(_vec(a1)), _d(_vec(b0)), _d(_vec(b1)), float(par_s2), _d(P), _d(Q))
    return P, Q, bool(par)


def point_polygon(p, loop):
    loop = np.ascontiguousarray(np.asarray(loop, dtype=np.float64).reshape(-1, 3))
    q = np.zeros(3)
    lib().or_point_polygon(_d(_vec(p)), _d(loop), int(loop.shape[0]), _d(q))
    return q


def pair(osys: OracleSystem, si, sj, xi, qi, xj, qj) -> PairOut:
    o = PairOut()
    lib().or_pair(C.byref(osys.c), int(si), int(sj), _d(_vec(xi)), _d(np.asarray(qi, np.float64).copy()),
                  _d(_vec(xj)), _d(np.asarray(qj, np.float64).copy()), C.byref(o))
    return o


def pair_terms(osys: OracleSystem, si, sj, xi, qi, xj, qj, cap=4096):
    """The feature pairs of one particle pair inside the cutoff: a list of
    dicts (family name, feature indices a and b, inside: 1 projection onto
    the face, 0 nearest point on the face's edges, -1 not a vertex-face pair;
    par: the parallel-edge rule; r)."""
    buf = (Term * cap)()
    n = lib().or_pair_terms(C.byref(osys.c), int(si), int(sj), _d(_vec(xi)), _d(np.asarray(qi, np.float64).copy()),
                            _d(_vec(xj)), _d(np.asarray(qj, np.float64).copy()), buf, cap)
    return [dict(family=TERM_FAMILIES[t.family], a=t.a, b=t.b, inside=t.inside, par=t.par, r=t.r)
            for t in buf[: min(n, cap)]]


def dimer_terms(sysobj, k):
    """pair_terms for particles 2k and 2k + 1 of a system built in pairs,
    with the second at its image nearest to the first."""
    osys = OracleSystem.of(sysobj)
    i, j = 2 * k, 2 * k + 1
    d = np.asarray(sysobj.x[j], float) - np.asarray(sysobj.x[i], float)
    for a in range(sysobj.dim):
        d[a] -= sysobj.box[a] * np.rint(d[a] / sysobj.box[a])
    return pair_terms(osys, sysobj.shape_id[i], sysobj.shape_id[j], sysobj.x[i], sysobj.q[i], sysobj.x[i] + d,
                      sysobj.q[j])


# ---------------------------------------------------------------- system-level
def cell_list(sysobj, r_list):
    osys = OracleSystem.of(sysobj)
    nc = osys.cell_dims(r_list)
    ncell = int(np.prod(nc))
    x = np.ascontiguousarray(sysobj.x, dtype=np.float64)
    cs = np.zeros(ncell + 1, np.int32)
    cp = np.zeros(max(sysobj.n, 1), np.int32)
    lib().or_cell_list(C.byref(osys.c), int(sysobj.n), _d(x), float(r_list), _i(cs), _i(cp))
    return nc, cs, cp[: sysobj.n]


def nbr_list(sysobj, r_list, cap, mode=1):
    osys = OracleSystem.of(sysobj)
    n = sysobj.n
    x = np.ascontiguousarray(sysobj.x, dtype=np.float64)
    nbr = np.full(cap * max(n, 1), -1, np.int32)
    n_nbr = np.zeros(max(n, 1), np.int32)
    maxrow = lib().or_nbr_list(C.byref(osys.c), int(n), _d(x), float(r_list), int(cap), int(mode), _i(nbr), _i(n_nbr))
    return nbr.reshape(cap, max(n, 1))[:, :n], n_nbr[:n], maxrow


def forces(sysobj, mode=1, threads: Optional[int] = None):
    """Per-particle F (n,3), torque (n,3), U_i (n,), W_i (n,9), stats, and the
    per-particle magnitude scales of the sums: scale[:,0] = sum |f|,
    scale[:,1] = sum |(P - x_i) x f|, scale[:,2] = 1/2 sum |r_ij||f| over the
    feature pairs that contribute to particle i."""
    if threads:
        lib().or_set_threads(int(threads))
    osys = OracleSystem.of(sysobj)
    n = sysobj.n
    x = np.ascontiguousarray(sysobj.x, dtype=np.float64)
    q = np.ascontiguousarray(sysobj.q, dtype=np.float64)
    sid = np.ascontiguousarray(sysobj.shape_id, dtype=np.int32)
    F = np.zeros((n, 3))
    T = np.zeros((n, 3))
    U = np.zeros(n)
    W = np.zeros((n, 9))
    st = Stats()
    sc = np.zeros((n, 3))
    lib().or_forces(C.byref(osys.c), int(n), _d(x), _d(q), _i(sid), int(mode), _d(F), _d(T), _d(U), _d(W),
                    C.byref(st), _d(sc))
    return dict(F=F, T=T, U=U, W=W, scale=sc, stats=dict(pairs=st.n_pairs_bound, feature_in=st.n_feature_in,
                                                           par=st.n_par, near_par=st.n_near_par))


def forces_subset(sysobj, pick, mode=1, threads: Optional[int] = None):
    """forces() for the particles pick (each against all others): row k of
    every output belongs to particle pick[k]; stats count their pairs only."""
    if threads:
        lib().or_set_threads(int(threads))
    osys = OracleSystem.of(sysobj)
    n = sysobj.n
    pick = np.ascontiguousarray(pick, dtype=np.int32)
    m = pick.size
    x = np.ascontiguousarray(sysobj.x, dtype=np.float64)
    q = np.ascontiguousarray(sysobj.q, dtype=np.float64)
    sid = np.ascontiguousarray(sysobj.shape_id, dtype=np.int32)
    F, T, U, W = np.zeros((m, 3)), np.zeros((m, 3)), np.zeros(m), np.zeros((m, 9))
    st = Stats()
    sc = np.zeros((m, 3))
    lib().or_forces_subset(C.byref(osys.c), int(n), _d(x), _d(q), _i(sid), int(mode), _i(pick), int(m), _d(F), _d(T),
                           _d(U), _d(W), C.byref(st), _d(sc))
    return dict(F=F, T=T, U=U, W=W, scale=sc, stats=dict(pairs=st.n_pairs_bound, feature_in=st.n_feature_in,
                                                           par=st.n_par, near_par=st.n_near_par))


def run(sysobj, n_steps, *, mode=1, thermo=None, log=True, threads: Optional[int] = None):
    """Integrates a copy of the system; returns (final system, thermo, log,
    forces dict at the final state).  log rows: U, K_trans, K_rot, xi, eta, H."""
    if threads:
        lib().or_set_threads(int(threads))
    s = sysobj.copy()
    osys = OracleSystem.of(s)
    n = s.n
    for name in ("x", "q", "v", "L"):
        setattr(s, name, np.ascontiguousarray(getattr(s, name), dtype=np.float64))
    s.image = np.ascontiguousarray(s.image, dtype=np.int32)
    sid = np.ascontiguousarray(s.shape_id, dtype=np.int32)
    th = np.zeros(2) if thermo is None else np.asarray(thermo, np.float64).copy()
    F = np.zeros((n, 3))
    T = np.zeros((n, 3))
    U = np.zeros(n)
    W = np.zeros((n, 9))
    lg = np.zeros((max(n_steps, 1), 6)) if log else None
    ens = 1 if s.ensemble == "nvt" else 0
    lib().or_run(C.byref(osys.c), int(n), _d(s.x), _d(s.q), _d(s.v), _d(s.L), _i(s.image), _i(sid), int(n_steps),
                 float(s.dt), ens, float(s.kT), float(s.tau_T), _d(th), int(mode), _d(F), _d(T), _d(U), _d(W),
                 _d(lg) if lg is not None else None)
    return s, th, (lg[:n_steps] if lg is not None else None), dict(F=F, T=T, U=U, W=W)


def run_npt(sysobj, n_steps, *, mode=1, thermo=None, veps=0.0, log=True, threads: Optional[int] = None):
    """Integrates a copy of the system at fixed pressure sysobj.P (barostat
    time constant sysobj.tau_P, Sec. IV.C); returns (final system with its
    box, thermo, v_eps, log, forces).  log rows: U, K_trans, K_rot, xi, eta,
    H, V, P_int, v_eps."""
    if threads:
        lib().or_set_threads(int(threads))
    s = sysobj.copy()
    osys = OracleSystem.of(s)
    n = s.n
    for name in ("x", "q", "v", "L"):
        setattr(s, name, np.ascontiguousarray(getattr(s, name), dtype=np.float64))
    s.image = np.ascontiguousarray(s.image, dtype=np.int32)
    sid = np.ascontiguousarray(s.shape_id, dtype=np.int32)
    th = np.zeros(2) if thermo is None else np.asarray(thermo, np.float64).copy()
    baro = np.array([float(veps)])
    box = np.ascontiguousarray(s.box, dtype=np.float64).copy()
    F = np.zeros((n, 3))
    T = np.zeros((n, 3))
    U = np.zeros(n)
    W = np.zeros((n, 9))
    lg = np.zeros((max(n_steps, 1), 9)) if log else None
    lib().or_run_npt(C.byref(osys.c), int(n), _d(s.x), _d(s.q), _d(s.v), _d(s.L), _i(s.image), _i(sid),
                     int(n_steps), float(s.dt), float(s.kT), float(s.tau_T), float(s.P), float(s.tau_P), _d(box),
                     _d(th), _d(baro), int(mode), _d(F), _d(T), _d(U), _d(W), _d(lg) if lg is not None else None)
    s.box = box
    return s, th, float(baro[0]), (lg[:n_steps] if lg is not None else None), dict(F=F, T=T, U=U, W=W)


def kinetic(sysobj):
    m = np.array([sysobj.shapes[k].mass for k in sysobj.shape_id])
    I = np.array([sysobj.shapes[k].inertia for k in sysobj.shape_id])
    Kt = 0.5 * np.sum(m[:, None] * sysobj.v ** 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        kr = np.where(I > 0, 0.5 * sysobj.L ** 2 / np.where(I > 0, I, 1.0), 0.0)
    return float(Kt), float(kr.sum())


def set_threads(n):
    lib().or_set_threads(int(n))


def get_threads():
    return lib().or_get_threads()
