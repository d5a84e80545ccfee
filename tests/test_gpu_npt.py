"""The isothermal-isobaric path on the GPU (Sec. IV.C: a barostat driven by
the pressure from the virial tensor, the reading of the oracle's
or_run_npt): a short FP64 trajectory against the oracle (positions, box,
barostat and thermostat variables, conserved quantity), the FP32 path on
the same run within its tolerance, split calls and a batch mix bit for bit,
and a checkpoint that continues bit for bit."""
import numpy as np
import pytest

import oracle as O
from paper_1607_02427_amd import inputs as I

pytestmark = pytest.mark.gpu


def _dem():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1607_02427_amd import dem
    return dem


def _fluid(n_side=5, P=2.0):
    """Rounded cubes from their lattice at volume fraction 0.4 (pressure
    about 0.2), compressed at P = 2 through contacts."""
    s = I.cubes_3d(n_side=n_side)
    s.ensemble = "npt"
    s.kT, s.tau_T, s.tau_P, s.P, s.dt = 1.0, 0.5, 0.5, P, 5e-4
    return s


def _same(a, b, label=""):
    for k in ("x", "q", "v", "L", "image", "box"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), (label, k)


@pytest.mark.parametrize("n_steps", [150, 600])
def test_npt_trajectory_fp64_matches_oracle(n_steps):
    dem = _dem()
    s = _fluid()
    print(f"[npt] {s.n} cubes, P = {s.P}, {n_steps} steps", flush=True)
    ref, th, veps, lg, _ = O.run_npt(s, n_steps)
    with dem.DemSystem(s, "fp64") as g:
        g.step(n_steps)
        e = g.energy()
        st = g.state()
    print(f"[npt] box {s.box[0]:.6f} -> oracle {ref.box[0]:.9f} gpu {st.box[0]:.9f}; veps {veps:.6e} / {e['veps']:.6e}; "
          f"rebuilds {e['n_rebuilds']}, min U {lg[:, 0].min():.3f}", flush=True)
    assert lg[:, 6].min() < 0.93 * lg[0, 6]  # the barostat has worked on it
    assert np.allclose(st.box, ref.box, rtol=1e-11, atol=0)
    ux = st.x + st.image * st.box
    rx = ref.x + ref.image * ref.box
    assert np.abs(ux - rx).max() < 1e-8
    assert np.abs(st.v - ref.v).max() < 1e-7 * (1 + np.abs(ref.v).max())
    assert e["veps"] == pytest.approx(veps, rel=1e-6, abs=1e-12)
    assert e["xi"] == pytest.approx(th[0], rel=1e-7, abs=1e-12)
    assert e["V"] == pytest.approx(lg[-1, 6], rel=1e-11)
    assert e["P"] == pytest.approx(lg[-1, 7], rel=1e-7)
    assert e["U"] == pytest.approx(lg[-1, 0], rel=1e-7, abs=1e-10)
    assert e["H"] == pytest.approx(lg[-1, 5], rel=1e-9)


def test_npt_fp32_follows_the_oracle():
    dem = _dem()
    s = _fluid()
    n = 150
    ref, th, veps, lg, _ = O.run_npt(s, n)
    with dem.DemSystem(s, "fp32") as g:
        g.step(n)
        e = g.energy()
        st = g.state()
    print(f"[npt fp32] box {st.box[0]:.9f} vs {ref.box[0]:.9f}, H {e['H']:.6f} vs {lg[-1, 5]:.6f}", flush=True)
    assert st.box[0] == pytest.approx(ref.box[0], rel=1e-6)
    assert e["H"] == pytest.approx(lg[-1, 5], rel=1e-5)


def test_npt_split_calls_equal_one_call():
    dem = _dem()
    s = _fluid(n_side=4)
    with dem.DemSystem(s, "fp32") as a:
        a.step(97)
        one, ea = a.state(), a.energy()
    with dem.DemSystem(s, "fp32") as b:
        for k in (10, 1, 40, 46):
            b.step(k)
        split, eb = b.state(), b.energy()
    _same(one, split, "split")
    assert ea["H"] == eb["H"] and ea["veps"] == eb["veps"]


def test_npt_alone_equals_in_mix():
    dem = _dem()
    npt = _fluid(n_side=4)
    other = I.cubes_3d_contact(n_side=5)
    other.ensemble, other.kT = "nvt", 1.0
    res = []
    for mix in (False, True):
        with dem.DemBatch(3, "fp32", max_replicas=4, max_particles=1024) as B:
            if mix:
                B.add(other)
            r = B.add(npt)
            B.step(120)
            st, _ = B.read(r)
            res.append((st, B.energy(r)))
    _same(res[0][0], res[1][0], "mix")
    assert res[0][1]["H"] == res[1][1]["H"]


def test_npt_checkpoint_continues():
    dem = _dem()
    s = _fluid(n_side=4)
    with dem.DemSystem(s, "fp64") as a:
        a.step(80)
        blob = a.get_state()
        a.step(70)
        want = a.state()
    with dem.DemSystem(s, "fp64") as b:
        b.set_state(blob)
        b.step(70)
        got = b.state()
    _same(want, got, "checkpoint")
