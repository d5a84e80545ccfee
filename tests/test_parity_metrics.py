"""The parity metric itself (host only): the plain relative error with its
floor, the exactly-zero rule, and the FP32 cancellation clause."""
import numpy as np

from parity_metrics import CANCEL, TOL, compare


def _ref(F, S):
    n = len(F)
    F = np.asarray(F, np.float64).reshape(n, 3)
    scale = np.zeros((n, 3))
    scale[:, 0] = S
    scale[:, 1] = S
    scale[:, 2] = S
    z = np.zeros((n, 3))
    return dict(F=F, T=z.copy(), U=np.where(np.asarray(S) > 0, 1.0, 0.0), W=np.zeros((n, 9)), scale=scale)


def _gpu(ref, dF):
    out = {k: np.array(ref[k], copy=True) for k in ("F", "T", "U", "W")}
    out["F"] = out["F"] + np.asarray(dF, np.float64)
    return out


def test_plain_relative_error_and_floor():
    ref = _ref([[1.0, 0, 0], [2.0, 0, 0], [1e-9, 0, 0]], [1.0, 2.0, 1e-9])
    rms = np.sqrt((1 + 4 + 1e-18) / 3)
    d = np.zeros((3, 3))
    d[1, 0] = 2e-6                       # 1e-6 relative
    d[2, 0] = 1e-3 * rms * 5e-6          # 5e-6 of the floor
    e = compare(_gpu(ref, d), ref, "fp64", keys=("F",))["F"]
    assert abs(e - 5e-6) < 1e-9


def test_zero_particles_must_be_exactly_zero():
    ref = _ref([[1.0, 0, 0], [0, 0, 0]], [1.0, 0.0])
    d = np.zeros((2, 3))
    d[1, 2] = 1e-30
    assert compare(_gpu(ref, d), ref, "fp32", keys=("F",))["F"] == float("inf")


def test_cancellation_clause_fp32_only_and_above_the_ratio():
    # particle 1: net 1, summed CANCEL (cancels), error 3e-4 of the net = 3e-4 / CANCEL of the summed
    ref = _ref([[1.0, 0, 0], [1.0, 0, 0]], [1.0, CANCEL])
    d = np.zeros((2, 3))
    d[1, 0] = 3e-4
    assert compare(_gpu(ref, d), ref, "fp32", keys=("F",))["F"] <= TOL["fp32"]
    assert compare(_gpu(ref, d), ref, "fp64", keys=("F",))["F"] > TOL["fp32"]
    # just below the ratio the plain error is gated
    ref2 = _ref([[1.0, 0, 0], [1.0, 0, 0]], [1.0, 0.99 * CANCEL])
    assert compare(_gpu(ref2, d), ref2, "fp32", keys=("F",))["F"] > TOL["fp32"]
