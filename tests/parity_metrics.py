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

Beside it, the same error against what was summed, S_i = sum over the
particle's feature-pair terms of |term| (the oracle reports it):

    s_i = |X_gpu,i - X_ref,i| / max(S_i, 1e-3 * RMS_k S_k).

Where the terms of a particle cancel (a particle squeezed from several
sides, the torques of a contact patch centred on the line of centres), FP32
rounding acts on S_i, not on |X_ref,i|: a relative error delta of the terms
becomes delta * S_i / |X_ref,i| in the net.  The FP32 kernel's delta reaches
5e-5 to 8e-5 on particles whose terms do not cancel (the pair offset rounded
to FP32, about 1e-7 of the centre distance, moves the contact distance, and
the WCA force changes 13 times faster than the distance near sigma), so a
net four times smaller than what was summed can exceed 2e-4 however the
terms are evaluated in FP32.  On the FP32 path, and only there, a particle
whose terms cancel by at least CANCEL = 4 (S_i >= 4 |X_ref,i|) is held to
s_i <= 2e-4 instead of e_i; every particle that needs it is counted and
printed with the case, with its cancellation ratio.  Cancellation inside a single
term (a force line through a centre: the term's own torque is small against
|lever| |f|) is not covered by this: S_i is then small too, and the FP32
kernel redoes such terms in FP64.
"""
import numpy as np

TOL = {"fp64": 1e-5, "fp32": 2e-4}
CANCEL = 4.0
KEYS = ("F", "T", "U", "W")


def _rows(a, n):
    return np.asarray(a, dtype=np.float64).reshape(n, -1)


def _scales(ref_out):
    sc = ref_out["scale"]
    return {"F": sc[:, 0], "T": sc[:, 1], "U": np.abs(ref_out["U"]), "W": sc[:, 2]}


def _live(ref_out):
    return ref_out["scale"][:, 0] > 0  # some feature pair of the particle lies inside the cutoff


def errors(gpu, ref, summed, live, prec="fp64", floor_frac=1e-3):
    """dict(e: max e_i, s: max s_i, i: index of the max e_i, ratio: S_i /
    |X_ref,i| there, dead: particles with no term that are not exactly zero,
    gated: the gated maximum (e_i, or s_i for the FP32 particles that cancel
    by CANCEL or more), exempt: particles over the bar by e_i that the
    cancellation clause holds to s_i instead, max_ratio: the largest
    cancellation ratio among them)."""
    n = len(summed)
    out = dict(e=0.0, s=0.0, i=-1, ratio=1.0, dead=0, gated=0.0, exempt=0, max_ratio=0.0)
    if n == 0:
        return out
    g, r = _rows(gpu, n), _rows(ref, n)
    d = np.linalg.norm(g - r, axis=1)
    mag = np.linalg.norm(r, axis=1)
    summed = np.asarray(summed, dtype=np.float64)
    out["dead"] = int(np.count_nonzero(np.any(g[~live] != 0.0, axis=1)))
    if not np.any(live):
        return out
    floor_e = floor_frac * float(np.sqrt(np.mean(mag ** 2)))
    floor_s = floor_frac * float(np.sqrt(np.mean(summed ** 2)))
    e = np.where(live, d / np.maximum(np.maximum(mag, floor_e), 1e-300), 0.0)
    s = np.where(live, d / np.maximum(np.maximum(summed, floor_s), 1e-300), 0.0)
    ratio = np.where(mag > 0, summed / np.maximum(mag, 1e-300), np.inf)
    cancel = live & (ratio >= CANCEL) if prec == "fp32" else np.zeros(n, dtype=bool)
    gated = np.where(cancel, s, e)
    over = cancel & (e > TOL[prec])
    k = int(np.argmax(e))
    out.update(e=float(e.max()), s=float(s.max()), i=k, ratio=float(ratio[k]), gated=float(gated.max()),
               exempt=int(np.count_nonzero(over)), max_ratio=float(ratio[over].max()) if np.any(over) else 0.0)
    return out


def compare(gpu_out, ref_out, prec="fp64", keys=KEYS, floor_frac=1e-3):
    """Gated metric per output, or inf when a particle with no term inside
    the cutoff is not exactly zero."""
    sc, live = _scales(ref_out), _live(ref_out)
    out = {}
    for k in keys:
        r = errors(gpu_out[k], ref_out[k], sc[k], live, prec, floor_frac)
        out[k] = float("inf") if r["dead"] else r["gated"]
    return out


def report(gpu_out, ref_out, keys=KEYS, prec="fp64", floor_frac=1e-3):
    """Both metrics per output, for the test log: {key: errors(...)}."""
    sc, live = _scales(ref_out), _live(ref_out)
    return {k: errors(gpu_out[k], ref_out[k], sc[k], live, prec, floor_frac) for k in keys}


def fmt(rep):
    parts = []
    for k, v in rep.items():
        extra = f", dead!=0: {v['dead']}" if v["dead"] else ""
        if v["exempt"]:
            extra += f", {v['exempt']} held to s (S/|X| up to {v['max_ratio']:.0f})"
        parts.append(f"{k}: e={v['e']:.2e} s={v['s']:.2e} (i={v['i']}, S/|X|={v['ratio']:.1f}{extra})")
    return " ".join(parts)


def check(name, prec, gpu_out, ref_out, keys=KEYS):
    """Prints both metrics for a case and asserts the gated one."""
    rep = report(gpu_out, ref_out, keys, prec)
    print(f"[parity] {name} {prec} {fmt(rep)}", flush=True)
    for k, v in rep.items():
        assert v["dead"] == 0, (name, prec, k, "particles with no term inside the cutoff are not exactly zero", v["dead"])
        assert v["gated"] <= TOL[prec], (name, prec, k, v["e"], v["s"], v["gated"])
    return rep
