"""Python binding of libdem (include/dem.h): argument marshalling only.

PyTorch supplies device memory (the caller-owned state and output arrays)
and the stream; every step of the method runs in libdem's HIP kernels.  If
libdem.so is missing this module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdem.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "dem.h")

DEM_FP64, DEM_FP32 = 0, 1
DEM_NVE, DEM_NVT, DEM_NPT = 0, 1, 2
ENSEMBLES = {"nve": DEM_NVE, "nvt": DEM_NVT, "npt": DEM_NPT}
STATUS = {0: "DEM_OK", 1: "DEM_E_ARG", 2: "DEM_E_SHAPE", 3: "DEM_E_OOM", 4: "DEM_E_HIP", 5: "DEM_E_CAPACITY",
          6: "DEM_E_NONFINITE", 7: "DEM_E_STATE"}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class ShapeDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_vertices", C.c_int32), ("vertices", _dp), ("n_edges", C.c_int32),
                ("edges", _ip), ("n_faces", C.c_int32), ("face_offsets", _ip), ("face_vertices", _ip),
                ("rounding_radius", C.c_double), ("mass", C.c_double), ("inertia", C.c_double * 3)]


class Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int64), ("box", C.c_double * 3), ("n_shapes", C.c_int32),
                ("shapes", C.POINTER(ShapeDesc)), ("epsilon", C.c_double), ("skin", C.c_double),
                ("rebuild_frac", C.c_double), ("dt", C.c_double), ("ensemble", C.c_int32), ("kT", C.c_double),
                ("tau_T", C.c_double), ("precision", C.c_int32), ("parallel_sin2", C.c_double),
                ("nbr_capacity", C.c_int32), ("list_mode", C.c_int32), ("pressure", C.c_double),
                ("tau_P", C.c_double)]


class StatePtrs(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "z", "qw", "qx", "qy", "qz", "vx", "vy", "vz", "Lx", "Ly", "Lz",
                                          "shape_id", "image")]


class OutPtrs(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("Fx", "Fy", "Fz", "Tx", "Ty", "Tz", "U", "W")]


class BatchParams(C.Structure):
    _fields_ = [("dim", C.c_int32), ("precision", C.c_int32), ("max_replicas", C.c_int32),
                ("max_particles", C.c_int64), ("max_cells", C.c_int64), ("max_shapes", C.c_int32),
                ("nbr_capacity", C.c_int32), ("hbm_budget_bytes", C.c_int64)]


class OutputView(C.Structure):
    _fields_ = [("Fx", C.c_void_p), ("Fy", C.c_void_p), ("Fz", C.c_void_p), ("Tx", C.c_void_p),
                ("Ty", C.c_void_p), ("Tz", C.c_void_p), ("U", C.c_void_p), ("W", C.c_void_p),
                ("w_stride", C.c_int64), ("nbr", C.c_void_p), ("n_nbr", C.c_void_p), ("nbr_stride", C.c_int64),
                ("capacity", C.c_int32)]


class EnergyOut(C.Structure):
    _fields_ = [("U", C.c_double), ("K_trans", C.c_double), ("K_rot", C.c_double), ("H", C.c_double),
                ("T", C.c_double), ("P", C.c_double), ("W", C.c_double * 9), ("xi", C.c_double),
                ("eta", C.c_double), ("step", C.c_int64), ("n_rebuilds", C.c_int64), ("V", C.c_double),
                ("box", C.c_double * 3), ("veps", C.c_double)]


class DemError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def declared_functions():
    """Names of the functions dem.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(dem_[a-z_0-9]+)\s*\(", text, re.M)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libdem.so is not built at {LIB_PATH}; run __graft_entry__.build() "
                               f"or python -m paper_1607_02427_amd.build")
        # torch first: the library then binds to the HIP runtime torch loads
        # (the same soname); loaded first, it would pull in the system's copy
        # and leave the process with a runtime torch cannot initialise on
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        st = C.c_int
        L.dem_create_system.argtypes = [C.POINTER(Params), C.POINTER(StatePtrs), C.POINTER(OutPtrs), C.c_void_p,
                                        C.POINTER(C.c_void_p)]
        L.dem_create_system.restype = st
        for name in ("dem_destroy_system", "dem_build_celllist", "dem_compute_forces", "dem_sync"):
            getattr(L, name).argtypes = [C.c_void_p]
            getattr(L, name).restype = st
        L.dem_step.argtypes = [C.c_void_p, C.c_int64]
        L.dem_step.restype = st
        L.dem_batch_step.argtypes = [C.c_void_p, C.c_int64]
        L.dem_batch_step.restype = st
        L.dem_get_outputs.argtypes = [C.c_void_p, C.POINTER(OutputView)]
        L.dem_get_outputs.restype = st
        L.dem_state_bytes.argtypes = [C.c_void_p]
        L.dem_state_bytes.restype = C.c_size_t
        L.dem_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.dem_get_state.restype = st
        L.dem_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.dem_set_state.restype = st
        L.dem_energy.argtypes = [C.c_void_p, C.POINTER(EnergyOut)]
        L.dem_energy.restype = st
        L.dem_set_thermostat.argtypes = [C.c_void_p, C.c_double, C.c_double]
        L.dem_set_thermostat.restype = st
        L.dem_set_barostat.argtypes = [C.c_void_p, C.c_double]
        L.dem_set_barostat.restype = st
        L.dem_copy_lists.argtypes = [C.c_void_p, _ip, _ip, _ip, _ip, _ip]
        L.dem_copy_lists.restype = st
        L.dem_list_info.argtypes = [C.c_void_p, _dp, _ip, _ip]
        L.dem_list_info.restype = st
        L.dem_force_stats.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.c_int32]
        L.dem_force_stats.restype = st
        L.dem_set_counting.argtypes = [C.c_void_p, C.c_int32]
        L.dem_set_counting.restype = st
        L.dem_time_forces.argtypes = [C.c_void_p, C.c_int32, _dp]
        L.dem_time_forces.restype = st
        L.dem_set_pair_shape.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        L.dem_set_pair_shape.restype = st
        L.dem_set_feature_cells.argtypes = [C.c_void_p, C.c_int32]
        L.dem_set_feature_cells.restype = st
        L.dem_tune_pairs.argtypes = [C.c_void_p, C.c_int32, _ip, _dp]
        L.dem_tune_pairs.restype = st
        L.dem_footprint_bytes.argtypes = [C.POINTER(Params)]
        L.dem_footprint_bytes.restype = C.c_size_t
        L.dem_batch_create.argtypes = [C.POINTER(BatchParams), C.c_void_p, C.POINTER(C.c_void_p)]
        L.dem_batch_create.restype = st
        L.dem_batch_add.argtypes = [C.c_void_p, C.POINTER(Params), C.POINTER(StatePtrs), C.c_int64,
                                    C.POINTER(C.c_int32)]
        L.dem_batch_add.restype = st
        L.dem_batch_remove.argtypes = [C.c_void_p, C.c_int32]
        L.dem_batch_remove.restype = st
        L.dem_batch_read.argtypes = [C.c_void_p, C.c_int32, C.POINTER(StatePtrs), C.POINTER(OutPtrs)]
        L.dem_batch_read.restype = st
        L.dem_batch_set_steps.argtypes = [C.c_void_p, C.c_int32, C.c_int64]
        L.dem_batch_set_steps.restype = st
        L.dem_batch_progress.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_int32]
        L.dem_batch_progress.restype = st
        L.dem_batch_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.dem_batch_info.restype = st
        L.dem_replica_energy.argtypes = [C.c_void_p, C.c_int32, C.POINTER(EnergyOut)]
        L.dem_replica_energy.restype = st
        L.dem_replica_energy_noalloc.argtypes = [C.c_void_p, C.c_int32, C.POINTER(EnergyOut)]
        L.dem_replica_energy_noalloc.restype = st
        L.dem_replica_lists.argtypes = [C.c_void_p, C.c_int32, _ip, _ip, _ip, _ip, _ip]
        L.dem_replica_lists.restype = st
        L.dem_status_string.argtypes = [C.c_int]
        L.dem_status_string.restype = C.c_char_p
        L.dem_last_error.argtypes = [C.c_void_p]
        L.dem_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _shape_desc(shape, keep):
    v = np.ascontiguousarray(shape.vertices, dtype=np.float64)
    e = np.ascontiguousarray(shape.edges, dtype=np.int32)
    fo = np.ascontiguousarray(shape.face_offsets(), dtype=np.int32)
    fv = np.ascontiguousarray(shape.face_vertices() if shape.faces else np.zeros(1, np.int32), dtype=np.int32)
    keep += [v, e, fo, fv]
    d = ShapeDesc()
    d.dim = shape.dim
    d.n_vertices = v.shape[0]
    d.vertices = v.ctypes.data_as(_dp)
    d.n_edges = e.shape[0]
    d.edges = e.ctypes.data_as(_ip)
    d.n_faces = len(shape.faces)
    d.face_offsets = fo.ctypes.data_as(_ip)
    d.face_vertices = fv.ctypes.data_as(_ip)
    d.rounding_radius = shape.r
    d.mass = shape.mass
    for a in range(3):
        d.inertia[a] = float(shape.inertia[a])
    return d


def make_params(system, precision: str = "fp64", nbr_capacity: int = 0, list_mode: str = "auto"):
    keep = []
    descs = (ShapeDesc * len(system.shapes))(*[_shape_desc(s, keep) for s in system.shapes])
    keep.append(descs)
    p = Params()
    p.dim = system.dim
    p.n = system.n
    for a in range(3):
        p.box[a] = float(system.box[a])
    p.n_shapes = len(system.shapes)
    p.shapes = C.cast(descs, C.POINTER(ShapeDesc))
    p.epsilon = system.epsilon
    p.skin = system.skin
    p.rebuild_frac = system.rebuild_frac
    p.dt = system.dt
    p.ensemble = ENSEMBLES[system.ensemble]
    p.kT = system.kT
    p.tau_T = system.tau_T
    p.pressure = float(getattr(system, "P", 0.0))
    p.tau_P = float(getattr(system, "tau_P", 0.0))
    p.precision = DEM_FP32 if precision == "fp32" else DEM_FP64
    p.parallel_sin2 = system.parallel_sin2
    p.nbr_capacity = nbr_capacity
    p.list_mode = 1 if list_mode == "multi" else 0
    return p, keep


def footprint_bytes(system, precision="fp64", nbr_capacity=0) -> int:
    p, keep = make_params(system, precision, nbr_capacity)
    return int(lib().dem_footprint_bytes(C.byref(p)))


STATE = ("x", "y", "z", "qw", "qx", "qy", "qz", "vx", "vy", "vz", "Lx", "Ly", "Lz")
OUT = ("Fx", "Fy", "Fz", "Tx", "Ty", "Tz", "U")


def _state_tensors(system, device):
    import torch
    cols = {"x": system.x[:, 0], "y": system.x[:, 1], "z": system.x[:, 2], "qw": system.q[:, 0],
            "qx": system.q[:, 1], "qy": system.q[:, 2], "qz": system.q[:, 3], "vx": system.v[:, 0],
            "vy": system.v[:, 1], "vz": system.v[:, 2], "Lx": system.L[:, 0], "Ly": system.L[:, 1],
            "Lz": system.L[:, 2]}
    t = {k: torch.tensor(np.ascontiguousarray(cols[k]), dtype=torch.float64, device=device) for k in STATE}
    t["shape_id"] = torch.tensor(np.ascontiguousarray(system.shape_id, dtype=np.int32), device=device)
    t["image"] = torch.tensor(np.ascontiguousarray(system.image, dtype=np.int32).reshape(-1), device=device)
    return t


def _output_tensors(n, device):
    import torch
    o = {k: torch.zeros(n, dtype=torch.float64, device=device) for k in OUT}
    o["W"] = torch.zeros(9 * n, dtype=torch.float64, device=device)
    return o


def _state_ptrs(t):
    return StatePtrs(**{k: t[k].data_ptr() for k in STATE + ("shape_id", "image")})


def _out_ptrs(o):
    return OutPtrs(**{k: o[k].data_ptr() for k in OUT + ("W",)})


def _outputs_np(o, n):
    o = {k: v.cpu().numpy() for k, v in o.items()}
    return dict(F=np.stack([o["Fx"], o["Fy"], o["Fz"]], axis=1), T=np.stack([o["Tx"], o["Ty"], o["Tz"]], axis=1),
                U=o["U"], W=o["W"].reshape(9, n).T.copy())


def _state_np(t, template):
    t = {k: v.cpu().numpy() for k, v in t.items()}
    s = template.copy()
    s.x = np.stack([t["x"], t["y"], t["z"]], axis=1)
    s.q = np.stack([t["qw"], t["qx"], t["qy"], t["qz"]], axis=1)
    s.v = np.stack([t["vx"], t["vy"], t["vz"]], axis=1)
    s.L = np.stack([t["Lx"], t["Ly"], t["Lz"]], axis=1)
    s.image = t["image"].reshape(-1, 3).copy()
    return s


def _energy_dict(e):
    return dict(U=e.U, K_trans=e.K_trans, K_rot=e.K_rot, H=e.H, T=e.T, P=e.P, W=np.array(e.W[:]), xi=e.xi,
                eta=e.eta, step=e.step, n_rebuilds=e.n_rebuilds, V=e.V, box=np.array(e.box[:]), veps=e.veps)


def _lists_np(call, n, ncell, cap):
    cs = np.zeros(ncell + 1, np.int32)
    cp = np.zeros(max(n, 1), np.int32)
    nb = np.zeros(max(cap * n, 1), np.int32)
    nn = np.zeros(max(n, 1), np.int32)
    dims = np.zeros(4, np.int32)
    call(cs.ctypes.data_as(_ip), cp.ctypes.data_as(_ip), nb.ctypes.data_as(_ip), nn.ctypes.data_as(_ip),
         dims.ctypes.data_as(_ip))
    return dict(dims=dims[:3].copy(), capacity=int(dims[3]), cell_start=cs, cell_particles=cp[:n],
                nbr=nb[: cap * n].reshape(cap, n) if n else nb[:0].reshape(cap, 0), n_nbr=nn[:n])


# the tuner's candidates (lanes per pair, grid factor, waves per SIMD, separation lanes, split), in
# dem_tune_pairs order
PAIR_SHAPES = ((16, 1, 2, 4, 0), (8, 1, 2, 4, 0), (16, 2, 2, 4, 0), (8, 2, 2, 4, 0), (16, 1, 3, 4, 0), (8, 1, 3, 4, 0),
               (16, 2, 3, 4, 0), (8, 2, 3, 4, 0), (16, 1, 2, 16, 0), (16, 2, 2, 16, 0), (16, 1, 3, 16, 0),
               (16, 2, 3, 16, 0), (16, 1, 2, 4, 1), (8, 1, 2, 4, 1), (16, 1, 3, 4, 1), (8, 1, 3, 4, 1))


def _tune_pairs(check, h, reps):
    shape = (C.c_int32 * 5)()
    ms = (C.c_double * len(PAIR_SHAPES))()
    check(lib().dem_tune_pairs(h, int(reps), shape, ms), "dem_tune_pairs")
    return dict(lanes=shape[0], grid=shape[1], waves=shape[2], sep=shape[3], split=shape[4],
                mean_ms={"x".join(map(str, sh)): ms[k] for k, sh in enumerate(PAIR_SHAPES)})


class DemSystem:
    """One libdem system whose state and outputs are torch tensors on `device`."""

    STATE = STATE
    OUT = OUT

    def __init__(self, system, precision: str = "fp64", nbr_capacity: int = 0, device: str = "cuda:0",
                 stream=None, list_mode: str = "auto"):
        import torch
        self.torch = torch
        self.system = system
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        n = system.n
        with torch.cuda.device(self.device):
            self.t = _state_tensors(system, self.device)
            self.o = _output_tensors(n, self.device)
        sp = _state_ptrs(self.t)
        op = _out_ptrs(self.o)
        self._params, self._keep = make_params(system, precision, nbr_capacity, list_mode)
        h = C.c_void_p()
        torch.cuda.synchronize(self.device)
        with torch.cuda.device(self.device):
            st = lib().dem_create_system(C.byref(self._params), C.byref(sp), C.byref(op),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != 0:
            raise DemError(st, "dem_create_system", lib().dem_last_error(None).decode())
        self.h = h
        thermo = getattr(system, "thermo", None)  # a stored state's Nose-Hoover (xi, eta)
        if thermo is not None:
            self.set_thermostat(*thermo)
        if system.ensemble == "npt" and getattr(system, "veps", 0.0):
            self._check(lib().dem_set_barostat(self.h, float(system.veps)), "dem_set_barostat")

    # ---------------------------------------------------------------- calls
    def _check(self, st, where):
        if st != 0:
            raise DemError(st, where, lib().dem_last_error(self.h).decode())

    def build_lists(self):
        self._check(lib().dem_build_celllist(self.h), "dem_build_celllist")

    def compute_forces(self):
        self._check(lib().dem_compute_forces(self.h), "dem_compute_forces")

    def step(self, n: int):
        self._check(lib().dem_step(self.h, int(n)), "dem_step")

    def sync(self):
        self._check(lib().dem_sync(self.h), "dem_sync")

    def set_thermostat(self, xi: float, eta: float):
        self._check(lib().dem_set_thermostat(self.h, float(xi), float(eta)), "dem_set_thermostat")

    def set_counting(self, on: bool):
        self._check(lib().dem_set_counting(self.h, 1 if on else 0), "dem_set_counting")

    def energy(self) -> Dict[str, float]:
        e = EnergyOut()
        self._check(lib().dem_energy(self.h, C.byref(e)), "dem_energy")
        return _energy_dict(e)

    def energy_noalloc(self) -> Dict[str, float]:
        """energy() through the allocation-free entry point."""
        e = EnergyOut()
        self._check(lib().dem_replica_energy_noalloc(self.h, 0, C.byref(e)), "dem_replica_energy_noalloc")
        return _energy_dict(e)

    def list_info(self):
        rl = C.c_double()
        nc = C.c_int32()
        cap = C.c_int32()
        self._check(lib().dem_list_info(self.h, C.byref(rl), C.byref(nc), C.byref(cap)), "dem_list_info")
        return rl.value, nc.value, cap.value

    def lists(self):
        rl, ncell, cap = self.list_info()
        out = _lists_np(lambda *a: self._check(lib().dem_copy_lists(self.h, *a), "dem_copy_lists"),
                        self.system.n, ncell, cap)
        out["r_list"] = rl
        return out

    def force_stats(self, reset: bool = False):
        out = (C.c_int64 * 9)()
        self._check(lib().dem_force_stats(self.h, out, 1 if reset else 0), "dem_force_stats")
        return dict(pairs=out[0], features=out[1], in_cutoff=out[2], launches=out[3], vf_near=out[4],
                    refined=out[5], ee_near=out[6], separated=out[7], plane_tests=out[8])

    def get_state(self) -> bytes:
        """Checkpoint of the whole state and thermostat (host bytes, dem_get_state)."""
        n = lib().dem_state_bytes(self.h)
        buf = C.create_string_buffer(n)
        self._check(lib().dem_get_state(self.h, buf, n), "dem_get_state")
        return buf.raw

    def set_state(self, blob: bytes):
        """Restores a checkpoint from get_state (lists rebuilt, forces recomputed)."""
        buf = C.create_string_buffer(blob, len(blob))
        self._check(lib().dem_set_state(self.h, buf, len(blob)), "dem_set_state")

    def output_view(self) -> dict:
        """Device addresses of the outputs and neighbour rows (dem_get_outputs)."""
        v = OutputView()
        self._check(lib().dem_get_outputs(self.h, C.byref(v)), "dem_get_outputs")
        return {name: getattr(v, name) for name, _ in OutputView._fields_}

    def set_pair_shape(self, lanes: int, grid: int = 1, waves: int = 2, sep: int = 4, split: int = 0):
        """Pair-kernel launch shape (8 or 16 lanes per pair, grid factor 1..4, 2 or 3 waves per SIMD, 4 or 16
        separation lanes, split 0 or 1: one kernel, or a search kernel and a force kernel); results do not
        change."""
        self._check(lib().dem_set_pair_shape(self.h, int(lanes), int(grid), int(waves), int(sep), int(split)),
                    "dem_set_pair_shape")

    def set_feature_cells(self, on: bool):
        """Feature search through the shape-local feature cells (True) or the supporting-plane prefilter."""
        self._check(lib().dem_set_feature_cells(self.h, 1 if on else 0), "dem_set_feature_cells")

    def tune_pairs(self, reps: int = 20) -> dict:
        """Times every pair-kernel shape on the current state and keeps the fastest."""
        return _tune_pairs(self._check, self.h, reps)

    def time_forces(self, reps: int = 100) -> float:
        """Mean duration (ms) of one force-kernel launch, HIP events on the system's stream."""
        ms = C.c_double()
        self._check(lib().dem_time_forces(self.h, int(reps), C.byref(ms)), "dem_time_forces")
        return ms.value

    def outputs(self) -> Dict[str, np.ndarray]:
        """Synchronises and returns F (n,3), T (n,3), U (n,), W (n,9)."""
        self.sync()
        return _outputs_np(self.o, self.system.n)

    def state(self):
        """Synchronises and returns a numpy copy of the system at its current state (under
        the barostat with its current box, barostat velocity and thermostat)."""
        self.sync()
        s = _state_np(self.t, self.system)
        if self.system.ensemble == "npt":
            e = self.energy()
            s.box, s.veps, s.thermo = e["box"].copy(), e["veps"], (e["xi"], e["eta"])
        return s

    def close(self):
        if getattr(self, "h", None):
            lib().dem_destroy_system(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class DemBatch:
    """A libdem batch: many independent replicas advanced together.  The
    batch keeps every replica's state in its own device arrays; add() copies
    a system in, read() copies a replica out."""

    def __init__(self, dim: int, precision: str = "fp32", max_replicas: int = 128, max_particles: int = 1 << 20,
                 max_cells: int = 0, max_shapes: int = 0, nbr_capacity: int = 0, device: str = "cuda:0",
                 stream=None, budget_bytes: int = 0):
        import torch
        self.torch = torch
        self.dim = dim
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.systems = {}
        bp = BatchParams(dim=dim, precision=DEM_FP32 if precision == "fp32" else DEM_FP64, max_replicas=max_replicas,
                         max_particles=max_particles, max_cells=max_cells, max_shapes=max_shapes,
                         nbr_capacity=nbr_capacity, hbm_budget_bytes=int(budget_bytes))
        h = C.c_void_p()
        torch.cuda.synchronize(self.device)
        with torch.cuda.device(self.device):
            st = lib().dem_batch_create(C.byref(bp), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != 0:
            raise DemError(st, "dem_batch_create", lib().dem_last_error(None).decode())
        self.h = h

    def _check(self, st, where):
        if st != 0:
            raise DemError(st, where, lib().dem_last_error(self.h).decode())

    def add(self, system, steps: int = 0) -> int:
        """Adds a replica (copied in) that advances `steps` steps (0: without limit); returns its id."""
        torch = self.torch
        with torch.cuda.device(self.device):
            t = _state_tensors(system, self.device)
        params, keep = make_params(system, self.precision)
        rid = C.c_int32(-1)
        torch.cuda.current_stream(self.device).synchronize()
        with torch.cuda.device(self.device):
            st = lib().dem_batch_add(self.h, C.byref(params), C.byref(_state_ptrs(t)), int(steps), C.byref(rid))
        self._check(st, "dem_batch_add")
        self.systems[rid.value] = system
        del t, keep
        return rid.value

    def remove(self, rid: int):
        self._check(lib().dem_batch_remove(self.h, int(rid)), "dem_batch_remove")
        self.systems.pop(rid, None)

    def step(self, n: int):
        self._check(lib().dem_batch_step(self.h, int(n)), "dem_batch_step")

    def compute_forces(self):
        self._check(lib().dem_compute_forces(self.h), "dem_compute_forces")

    def sync(self):
        self._check(lib().dem_sync(self.h), "dem_sync")

    def set_steps(self, rid: int, n: int):
        self._check(lib().dem_batch_set_steps(self.h, int(rid), int(n)), "dem_batch_set_steps")

    def progress(self, count: int):
        left = (C.c_int64 * max(count, 1))()
        done = (C.c_int64 * max(count, 1))()
        self._check(lib().dem_batch_progress(self.h, left, done, int(count)), "dem_batch_progress")
        return np.array(left[:count]), np.array(done[:count])

    def info(self):
        out = (C.c_int64 * 10)()
        self._check(lib().dem_batch_info(self.h, out), "dem_batch_info")
        keys = ("live", "slots", "free_particles", "largest_free_run", "free_cells", "free_shapes", "capacity",
                "particle_slots", "bytes_charged", "budget_bytes")
        return dict(zip(keys, out[:10]))

    def energy(self, rid: int):
        e = EnergyOut()
        self._check(lib().dem_replica_energy(self.h, int(rid), C.byref(e)), "dem_replica_energy")
        return _energy_dict(e)

    def energy_noalloc(self, rid: int):
        """energy(rid) through the allocation-free entry point."""
        e = EnergyOut()
        self._check(lib().dem_replica_energy_noalloc(self.h, int(rid), C.byref(e)), "dem_replica_energy_noalloc")
        return _energy_dict(e)

    def lists(self, rid: int):
        n = self.systems[rid].n
        info = self.info()
        dims_probe = np.zeros(4, np.int32)
        self._check(lib().dem_replica_lists(self.h, int(rid), None, None, None, None, dims_probe.ctypes.data_as(_ip)),
                    "dem_replica_lists")
        ncell = int(dims_probe[0] * dims_probe[1] * dims_probe[2])
        return _lists_np(lambda *a: self._check(lib().dem_replica_lists(self.h, int(rid), *a), "dem_replica_lists"),
                         n, ncell, int(info["capacity"]))

    def read(self, rid: int):
        """Synchronises and returns (state as a System, outputs dict) of one replica."""
        torch = self.torch
        system = self.systems[rid]
        n = system.n
        with torch.cuda.device(self.device):
            t = _state_tensors(system, self.device)
            o = _output_tensors(n, self.device)
        torch.cuda.current_stream(self.device).synchronize()  # the batch's stream may be another one
        self._check(lib().dem_batch_read(self.h, int(rid), C.byref(_state_ptrs(t)), C.byref(_out_ptrs(o))),
                    "dem_batch_read")
        self.sync()
        s = _state_np(t, system)
        if system.ensemble == "npt":
            e = self.energy(rid)
            s.box, s.veps, s.thermo = e["box"].copy(), e["veps"], (e["xi"], e["eta"])
        return s, _outputs_np(o, n)

    def force_stats(self, reset: bool = False):
        out = (C.c_int64 * 9)()
        self._check(lib().dem_force_stats(self.h, out, 1 if reset else 0), "dem_force_stats")
        return dict(pairs=out[0], features=out[1], in_cutoff=out[2], launches=out[3], vf_near=out[4],
                    refined=out[5], ee_near=out[6], separated=out[7], plane_tests=out[8])

    def set_counting(self, on: bool):
        self._check(lib().dem_set_counting(self.h, 1 if on else 0), "dem_set_counting")

    def set_pair_shape(self, lanes: int, grid: int = 1, waves: int = 2, sep: int = 4, split: int = 0):
        self._check(lib().dem_set_pair_shape(self.h, int(lanes), int(grid), int(waves), int(sep), int(split)),
                    "dem_set_pair_shape")

    def set_feature_cells(self, on: bool):
        self._check(lib().dem_set_feature_cells(self.h, 1 if on else 0), "dem_set_feature_cells")

    def tune_pairs(self, reps: int = 5) -> dict:
        return _tune_pairs(self._check, self.h, reps)

    def time_forces(self, reps: int = 100) -> float:
        ms = C.c_double()
        self._check(lib().dem_time_forces(self.h, int(reps), C.byref(ms)), "dem_time_forces")
        return ms.value

    def close(self):
        if getattr(self, "h", None):
            lib().dem_destroy_system(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
