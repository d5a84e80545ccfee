"""Error metrics of the GPU parity tests (test helpers only).

Each per-particle output X_i (force, torque, energy, virial) is a sum of
feature-pair terms.  Its relative error is measured against the magnitude
of what was summed, S_i = sum over contributing feature pairs of |term|
(reported by the oracle):

    e_i = |X_gpu,i - X_ref,i| / max(S_i, 1e-3 * RMS_k S_k).

When the terms do not cancel, S_i = |X_ref,i| and this is the plain relative
error; when they cancel (a particle squeezed from both sides), S_i is the
scale rounding acts on.  The floor at 1e-3 of the system's RMS scale covers
contacts right at the WCA cutoff, where U and F vanish (U ~ (r_c - r)^2,
F ~ r_c - r) so that any perturbation delta r of the geometry gives a relative
error ~ delta r / (r_c - r) without bound.  Particles with no contributing
term (S_i = 0) must come out zero to within zero_tol of the largest S.  The
bars are max_i e_i <= 1e-5 for the FP64 path and 2e-4 for the FP32 path.
"""
import numpy as np

TOL = {"fp64": 1e-5, "fp32": 2e-4}
ZERO_TOL = {"fp64": 0.0, "fp32": 1e-6}


def rel_err(gpu, ref, scale, zero_tol=0.0, floor_frac=1e-3):
    gpu = np.asarray(gpu, dtype=np.float64).reshape(len(scale), -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(len(scale), -1)
    scale = np.asarray(scale, dtype=np.float64)
    if scale.size == 0:
        return 0.0
    d = np.linalg.norm(gpu - ref, axis=1)
    live = scale > 0
    err = 0.0
    if np.any(live):
        floor = floor_frac * float(np.sqrt(np.mean(scale[live] ** 2)))
        err = float(np.max(d[live] / np.maximum(scale[live], floor)))
    dead = ~live
    if np.any(dead):
        z = float(np.max(np.linalg.norm(gpu[dead], axis=1)))
        if z > zero_tol * max(float(scale.max()), 1.0):
            err = max(err, np.inf)
    return err


def compare(gpu_out, ref_out, prec="fp64", keys=("F", "T", "U", "W"), floor_frac=1e-3):
    sc = ref_out["scale"]
    scales = {"F": sc[:, 0], "T": sc[:, 1], "U": np.abs(ref_out["U"]), "W": sc[:, 2]}
    return {k: rel_err(gpu_out[k], ref_out[k], scales[k], ZERO_TOL[prec], floor_frac) for k in keys}


def unfloored(gpu_out, ref_out, keys=("F", "T", "U", "W")):
    """The same error without the floor (reported, not gated)."""
    return compare(gpu_out, ref_out, "fp64", keys, floor_frac=0.0)
