"""Error metrics of the GPU parity tests (test helpers only).

The gated metric is the plain per-particle relative error with a floor:

    e_i = |X_gpu,i - X_ref,i| / max(|X_ref,i|, 1e-3 * RMS_k |X_ref,k|)

for X = F, tau, U_i, W_i (vectors and tensors by their Euclidean norm), the
RMS running over every particle of the system.  The floor covers contacts
right at the WCA cutoff, where U and F vanish (U ~ (r_c - r)^2,
F ~ r_c - r), so that no perturbation of the geometry, however small, could
keep a plain relative error bounded.  Particles with no feature pair inside
the cutoff (the oracle's sum of |term| is zero) must come out exactly zero
on both paths.  Bars: max_i e_i <= 1e-5 on the FP64 path, 2e-4 on the FP32
path.

Printed beside it, not gated, is the same error measured against what was
summed, S_i = sum over the particle's feature-pair terms of |term| (the
oracle reports it):

    s_i = |X_gpu,i - X_ref,i| / max(S_i, 1e-3 * RMS_k S_k),

with the cancellation ratio S_i / |X_ref,i| of the particle where e_i is
largest: where terms cancel (a particle squeezed from several sides, or the
torques of a face-to-face contact about its centre) FP32 rounding acts on
S_i, not on |X_ref,i|.
"""
import numpy as np

TOL = {"fp64": 1e-5, "fp32": 2e-4}
KEYS = ("F", "T", "U", "W")


def _rows(a, n):
    return np.asarray(a, dtype=np.float64).reshape(n, -1)


def _scales(ref_out):
    sc = ref_out["scale"]
    return {"F": sc[:, 0], "T": sc[:, 1], "U": np.abs(ref_out["U"]), "W": sc[:, 2]}


def _live(ref_out):
    return ref_out["scale"][:, 0] > 0  # some feature pair of the particle lies inside the cutoff


def errors(gpu, ref, summed, live, floor_frac=1e-3):
    """(max e_i, max s_i, index of the max e_i, S_i / |X_ref,i| there,
    particles with no term that are not exactly zero).  live marks the
    particles with a feature pair inside the cutoff."""
    n = len(summed)
    if n == 0:
        return 0.0, 0.0, -1, 1.0, 0
    g, r = _rows(gpu, n), _rows(ref, n)
    d = np.linalg.norm(g - r, axis=1)
    mag = np.linalg.norm(r, axis=1)
    summed = np.asarray(summed, dtype=np.float64)
    nonzero_dead = int(np.count_nonzero(np.any(g[~live] != 0.0, axis=1)))
    if not np.any(live):
        return 0.0, 0.0, -1, 1.0, nonzero_dead
    floor_e = floor_frac * float(np.sqrt(np.mean(mag ** 2)))
    floor_s = floor_frac * float(np.sqrt(np.mean(summed ** 2)))
    e = np.where(live, d / np.maximum(np.maximum(mag, floor_e), 1e-300), 0.0)
    s = np.where(live, d / np.maximum(np.maximum(summed, floor_s), 1e-300), 0.0)
    k = int(np.argmax(e))
    ratio = float(summed[k] / mag[k]) if mag[k] > 0 else float("inf")
    return float(e.max()), float(s.max()), k, ratio, nonzero_dead


def compare(gpu_out, ref_out, prec="fp64", keys=KEYS, floor_frac=1e-3):
    """Gated metric per output: max_i e_i, or inf when a particle with no
    term inside the cutoff is not exactly zero."""
    sc, live = _scales(ref_out), _live(ref_out)
    out = {}
    for k in keys:
        e, _, _, _, bad = errors(gpu_out[k], ref_out[k], sc[k], live, floor_frac)
        out[k] = float("inf") if bad else e
    return out


def report(gpu_out, ref_out, keys=KEYS, floor_frac=1e-3):
    """Both metrics per output, for the test log: {key: (e, s, worst particle,
    its cancellation ratio, nonzero dead particles)}."""
    sc, live = _scales(ref_out), _live(ref_out)
    return {k: errors(gpu_out[k], ref_out[k], sc[k], live, floor_frac) for k in keys}


def fmt(rep):
    return " ".join(f"{k}: e={v[0]:.2e} s={v[1]:.2e} (i={v[2]}, S/|X|={v[3]:.1f}{', dead!=0: %d' % v[4] if v[4] else ''})"
                    for k, v in rep.items())


def check(name, prec, gpu_out, ref_out, keys=KEYS):
    """Prints both metrics for a case and asserts the gated one."""
    rep = report(gpu_out, ref_out, keys)
    print(f"[parity] {name} {prec} {fmt(rep)}", flush=True)
    for k, v in rep.items():
        assert v[4] == 0, (name, prec, k, "particles with no term inside the cutoff are not exactly zero", v[4])
        assert v[0] <= TOL[prec], (name, prec, k, v[0])
    return rep
