"""Error metrics used by the GPU parity tests (test helpers only).

Per-particle relative error of a vector quantity X (force, torque, virial
rows, energy): e_i = |X_gpu,i - X_ref,i| / max(|X_ref,i|, floor), with the
floor 1e-3 times the RMS of |X_ref| over particles, so particles with tiny
net values (cancelling contacts) are judged against the system's scale
rather than against an arbitrarily small denominator.  The bar is
max_i e_i <= 1e-5 for the FP64 path and 2e-4 for the FP32 path.
"""
import numpy as np

TOL = {"fp64": 1e-5, "fp32": 2e-4}


def rel_err(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.ndim == 1:
        gpu = gpu[:, None]
        ref = ref[:, None]
    d = np.linalg.norm(gpu - ref, axis=1)
    m = np.linalg.norm(ref, axis=1)
    rms = np.sqrt(np.mean(m ** 2)) if m.size else 0.0
    floor = max(1e-3 * rms, 1e-300)
    return float(np.max(d / np.maximum(m, floor))) if m.size else 0.0


def compare(gpu_out, ref_out, keys=("F", "T", "U", "W")):
    return {k: rel_err(gpu_out[k], ref_out[k]) for k in keys}
