"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

Lists are compared bit for bit; forces, torques, per-particle energies and
virials within 1e-5 (FP64 path) or 2e-4 (FP32 path) by the metric of
parity_metrics.py; short FP64 trajectories against the oracle's integrator.
"""
import numpy as np
import pytest

import oracle as O
from paper_1607_02427_amd import inputs as I
from parity_metrics import check, report

pytestmark = pytest.mark.gpu


def _dem():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1607_02427_amd import dem
    return dem


def _cases():
    return {
        "squares_2d_256": lambda: I.squares_2d(),
        "squares_2d_contact_256": lambda: I.squares_2d_contact(),
        "cubes_contact_512": lambda: I.cubes_3d_contact(n_side=8),
        "cubes_3d_1000": lambda: I.cubes_3d(n_side=10),
        "dimers_cube_256": lambda: I.dimer_gas("cube", 128),
        "dimers_octa_256": lambda: I.dimer_gas("octahedron", 128),
        "dimers_tetra_256": lambda: I.dimer_gas("tetrahedron", 128),
        "dimers_lprism_128": lambda: I.dimer_gas("lprism", 64, quad_h=0.05),
        "dimers_pentagon_256": lambda: I.dimer_gas("pentagon", 128, dim=2),
        # the table limits: 20 faces and 30 edges (3D), 16 vertices (2D)
        "dimers_icosa_128": lambda: I.dimer_gas("icosahedron", 64),
        "dimers_16gon_128": lambda: I.dimer_gas("hexadecagon", 64, dim=2),
        # small cores with a large rounding radius: a hundred to several
        # hundred feature problems per pair in range, so solve rounds end
        # part-way through a pair and pairs of one wavefront end them at
        # different points
        "fat_dimers_16gon_128": lambda: I.dimer_gas("hexadecagon", 64, dim=2, edge=0.1, r=0.5),
        "fat_dimers_icosa_128": lambda: I.dimer_gas("icosahedron", 64, edge=0.3, r=0.5),
        "ragged_cubes_37": lambda: _drop_last(I.dimer_gas("cube", 19, seed=5)),
        # every pair in contact, across faces, edges and vertices of both bodies
        "contact_cube_128": lambda: I.contact_dimers(I.cube(), n_pairs=64),
        "contact_octa_128": lambda: I.contact_dimers(I.octahedron(), n_pairs=64),
        "contact_tetra_128": lambda: I.contact_dimers(I.tetrahedron(), n_pairs=64),
        "contact_icosa_128": lambda: I.contact_dimers(I.icosahedron(), n_pairs=64),
        "contact_lprism_128": lambda: I.contact_dimers(I.lprism(0.1, quad_h=0.05), n_pairs=64),
        "contact_square_128": lambda: I.contact_dimers(I.square(), n_pairs=64),
        "contact_pentagon_128": lambda: I.contact_dimers(I.pentagon(), n_pairs=64),
        # the concave caps of the L-prism around their reflex corner, on the
        # face and over the notch (the nearest point then on the notch's edges)
        "notch_lprism_cube_256": lambda: I.contact_dimers(I.lprism(0.1, quad_h=0.05), I.cube(1.0, 0.15),
                                                          n_pairs=128, notch=True),
        "notch_lprism_lprism_128": lambda: I.contact_dimers(I.lprism(0.1, quad_h=0.05), I.lprism(0.15, quad_h=0.05),
                                                            n_pairs=64, notch=True, seed=17),
    }


def _drop_last(s):
    s = s.copy()
    s.x, s.q, s.v, s.L = s.x[:-1], s.q[:-1], s.v[:-1], s.L[:-1]
    s.shape_id, s.image = s.shape_id[:-1], s.image[:-1]
    return s


CASES = _cases()


@pytest.mark.parametrize("mode", ["auto", "multi"])
@pytest.mark.parametrize("name", list(CASES))
def test_lists_bit_exact(name, mode):
    dem = _dem()
    s = CASES[name]()
    print(f"[lists] {name} n={s.n} {mode}", flush=True)
    _check_lists(dem, s, mode)


def test_lists_bit_exact_large():
    """74,088 cubes: above the single-workgroup limit, so the automatic mode
    takes the one-kernel-per-phase build."""
    dem = _dem()
    s = I.cubes_3d(n_side=42)
    print(f"[lists] cubes_74088 n={s.n}", flush=True)
    _check_lists(dem, s, "auto")


def _check_lists(dem, s, mode):
    with dem.DemSystem(s, "fp64", list_mode=mode) as g:
        L = g.lists()
        rl_oracle = O.OracleSystem.of(s).r_list(s.skin)
        assert L["r_list"] == rl_oracle  # same FP64 bits
        nc, cs, cp = O.cell_list(s, rl_oracle)
        assert np.array_equal(L["dims"], nc)
        assert np.array_equal(L["cell_start"], cs)
        assert np.array_equal(L["cell_particles"], cp)
        nb, nn, maxrow = O.nbr_list(s, rl_oracle, cap=L["capacity"], mode=1)
        assert maxrow <= L["capacity"]
        assert np.array_equal(L["n_nbr"], nn)
        for i in range(s.n):
            assert np.array_equal(L["nbr"][: nn[i], i], nb[: nn[i], i])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_forces_match_oracle(name, prec):
    dem = _dem()
    s = CASES[name]()
    print(f"[forces] {name} n={s.n} {prec}", flush=True)
    ref = O.forces(s)
    assert ref["stats"]["near_par"] == 0
    with dem.DemSystem(s, prec) as g:
        out = g.outputs()
        st = g.force_stats()
    print(name, prec, ref["stats"], st, flush=True)
    check(name, prec, out, ref)
    assert st["pairs"] == ref["stats"]["pairs"] // 2  # the GPU evaluates each unordered pair once


def test_cubes_4096_full_size_fp32():
    """The benchmark's particle count and launch configuration (4096 cubes,
    FP32 geometry) on a contact-rich lattice: every particle against the
    oracle."""
    dem = _dem()
    s = I.cubes_3d_contact(n_side=16)
    print(f"[full] cubes_contact_4096 n={s.n}", flush=True)
    ref = O.forces(s)
    with dem.DemSystem(s, "fp32") as g:
        out = g.outputs()
    print("full", ref["stats"], flush=True)
    check("cubes_contact_4096", "fp32", out, ref)


def test_octahedra_262144_full_size():
    """The at-scale configuration: 262,144 rounded octahedra on a BCC lattice
    at volume fraction 0.55, perturbed (positions by up to 0.05 per axis,
    rotations up to 8 degrees) so that about 8,000 particles are in contact,
    with the tuned pair shape: every particle against the oracle, FP32 and
    FP64."""
    dem = _dem()
    s = I.octahedra_3d(jitter=0.05, max_deg=8.0)
    print(f"[full] octahedra_bcc n={s.n}", flush=True)
    ref = O.forces(s)
    assert int((ref["scale"][:, 0] > 0).sum()) > 1000
    for prec in ("fp32", "fp64"):
        with dem.DemSystem(s, prec) as g:
            shape = g.tune_pairs(2)
            g.compute_forces()
            out = g.outputs()
        print("octahedra", prec, shape["lanes"], shape["grid"], ref["stats"], flush=True)
        check("octahedra_262144", prec, out, ref)


@pytest.mark.parametrize("which", ["2d", "3d_nvt"])
def test_short_trajectory_fp64(which):
    dem = _dem()
    if which == "2d":
        s = I.squares_2d_contact()
        n = 100
    else:
        s = I.cubes_3d_contact(n_side=6)
        s.ensemble = "nvt"
        s.kT = 1.5
        n = 60
    print(f"[traj] {which} n={s.n} steps={n}", flush=True)
    ref, th, lg, rf = O.run(s, n)
    with dem.DemSystem(s, "fp64") as g:
        g.step(n)
        e = g.energy()
        out = g.outputs()
        st = g.state()
    ux = st.x + st.image * s.box
    rx = ref.x + ref.image * s.box
    assert np.abs(ux - rx).max() < 1e-9
    assert np.abs(st.v - ref.v).max() < 1e-7 * (1 + np.abs(ref.v).max())
    sgn = np.sign(np.sum(st.q * ref.q, axis=1))[:, None]
    assert np.abs(st.q * sgn - ref.q).max() < 1e-9
    assert e["U"] == pytest.approx(lg[-1, 0], rel=1e-8, abs=1e-10)
    assert e["K_trans"] == pytest.approx(lg[-1, 1], rel=1e-9)
    assert e["K_rot"] == pytest.approx(lg[-1, 2], rel=1e-9)
    assert e["xi"] == pytest.approx(th[0], rel=1e-7, abs=1e-12)
    assert e["H"] == pytest.approx(lg[-1, 5], rel=1e-9)
    rf["scale"] = O.forces(ref)["scale"]
    # two states 1e-9 apart: the gated metric over the oracle's live particles
    # (a contact that sits exactly at the cutoff may be on in one and off in the other)
    assert report(out, rf, keys=("F",))["F"]["e"] < 1e-6


def test_fast_rotors_fp64():
    """Free rotors whose half-angle per turn lies on both sides of 1/16, so
    both ways the kernel takes the sine and cosine of a turn (series and
    library call) meet the oracle's integrator (Sec. IV.A)."""
    dem = _dem()
    cube, lp = I.cube(), I.lprism(0.1, quad_h=0.05)
    box = 40.0
    s = I.System(dim=3, box=np.array([box, box, box]), shapes=[cube, lp],
                 shape_id=np.array([0, 0, 1, 1], np.int32),
                 x=np.array([[5.0, 5.0, 5.0], [15.0, 15.0, 15.0], [25.0, 25.0, 25.0], [35.0, 5.0, 25.0]]),
                 q=I.uniform_quaternions(np.random.default_rng(11), 4),
                 v=np.array([[0.1, -0.2, 0.05], [0.0, 0.3, -0.1], [-0.2, 0.0, 0.1], [0.05, 0.05, 0.05]]),
                 L=np.array([[0.8, -0.5, 0.3], [9.0, 4.0, -6.0], [12.0, -3.0, 8.0], [0.2, 7.0, -25.0]]),
                 image=np.zeros((4, 3), np.int32), dt=0.01)
    inertia = np.array([cube.inertia, cube.inertia, lp.inertia, lp.inertia])
    half = np.abs(s.L) * s.dt / (2 * inertia)  # the x turn spans dt; y and z turns span dt/2
    half[:, 1:] *= 0.5
    assert (half > 1 / 16).any() and (half < 1 / 16).any()
    n = 50
    print(f"[rotors] n={s.n} steps={n} max half-angle {half.max():.3f}", flush=True)
    ref, _, _, _ = O.run(s, n)
    with dem.DemSystem(s, "fp64") as g:
        g.step(n)
        st = g.state()
    sgn = np.sign(np.sum(st.q * ref.q, axis=1))[:, None]
    assert np.abs(st.q * sgn - ref.q).max() < 1e-11
    assert np.abs(st.L - ref.L).max() < 1e-10
    assert np.abs((st.x + st.image * s.box) - (ref.x + ref.image * s.box)).max() < 1e-12


def test_energy_and_virial_totals():
    dem = _dem()
    s = I.cubes_3d_contact(n_side=8)
    ref = O.forces(s)
    with dem.DemSystem(s, "fp64") as g:
        e = g.energy()
    assert e["U"] == pytest.approx(ref["U"].sum(), rel=1e-10)
    Kt, Kr = O.kinetic(s)
    assert e["K_trans"] == pytest.approx(Kt, rel=1e-12)
    assert e["K_rot"] == pytest.approx(Kr, rel=1e-12)
    W = ref["W"].sum(axis=0)
    assert np.allclose(e["W"], W, rtol=1e-9, atol=1e-9 * np.abs(W).max())
    P = (2 * Kt + W[0] + W[4] + W[8]) / (3 * np.prod(s.box))
    assert e["P"] == pytest.approx(P, rel=1e-9)


def test_nve_energy_fp32_tracks_fp64():
    """Mixed precision (FP32 geometry, FP64 state) conserves energy as well
    as the FP64 path at the same time step: on a contact-rich 3D NVE run the
    band of the total energy is set by the time step, not by FP32."""
    dem = _dem()
    bands = {}
    for prec in ("fp64", "fp32"):
        s = I.cubes_3d_contact(n_side=8)
        s.ensemble = "nve"
        with dem.DemSystem(s, prec) as g:
            Hs = [g.energy()["H"]]
            for _ in range(10):
                g.step(50)
                Hs.append(g.energy()["H"])
        bands[prec] = (max(Hs) - min(Hs)) / s.n
    print("nve H band per particle", bands, flush=True)
    assert bands["fp32"] < 1.2 * bands["fp64"] + 1e-5


def test_long_rows_forces_match_oracle():
    """Rows longer than 32 slots (56 with a skin of 1.0): records in the
    second word of a particle's written-slot mask are gathered too."""
    dem = _dem()
    s = I.cubes_3d_contact(n_side=8)
    s.skin = 1.0
    ref = O.forces(s)
    for prec in ("fp32", "fp64"):
        with dem.DemSystem(s, prec) as g:
            L = g.lists()
            out = g.outputs()
        n_nbr, nbr = L["n_nbr"], L["nbr"]
        assert n_nbr.max() > 40
        bound = 2 * s.shapes[0].circumradius + 2 ** (1 / 6) * 2 * s.shapes[0].r
        far = [(i, nbr[k, i]) for i in range(s.n) for k in range(32, n_nbr[i])]
        d = np.array([s.x[j] - s.x[i] for i, j in far])
        d -= s.box * np.round(d / s.box)
        assert (np.sum(d * d, axis=1) < bound ** 2).any(), "no interacting pair beyond slot 31"
        print("long rows", prec, int(n_nbr.max()), flush=True)
        check("long_rows_512", prec, out, ref)


def test_capacity_overflow_is_reported():
    dem = _dem()
    s = I.cubes_3d_contact(n_side=6)
    with pytest.raises(dem.DemError) as ei:
        dem.DemSystem(s, "fp64", nbr_capacity=4)
    assert ei.value.status == 5


def test_auto_capacity_grows():
    dem = _dem()
    s = I.cubes_3d_contact(n_side=6)
    with dem.DemSystem(s, "fp64") as g:
        g.build_lists()
        rl, ncell, cap = g.list_info()
        L = g.lists()
        assert L["n_nbr"].max() <= cap


def test_empty_system():
    dem = _dem()
    s = I.cubes_3d_contact(n_side=4)
    s.x, s.q, s.v, s.L = s.x[:0], s.q[:0], s.v[:0], s.L[:0]
    s.shape_id, s.image = s.shape_id[:0], s.image[:0]
    with dem.DemSystem(s, "fp32") as g:
        g.step(5)
        e = g.energy()
        assert e["U"] == 0.0 and e["step"] == 5
