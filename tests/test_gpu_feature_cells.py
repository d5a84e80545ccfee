"""Shape-local feature cells (Sec. V: spatial structures for the contact
point search), dem_set_feature_cells: every shape carries a grid of cells
over its body frame listing the faces (2D: edges) and edges within reach of
any point in each cell; a vertex is paired only with the faces of its cell,
an edge only with the edges of its midpoint's cell.

Checked against the FP64 oracle at the parity bars of parity_metrics.py, on
the many-feature shapes the structure is for (icosahedra: 12 vertices, 30
edges, 20 faces; 16-gons) and on contact-rich, concave and 2D cases; the
feature pairs inside the cutoff must be exactly those the supporting-plane
prefilter finds (same count, FP64), with no more problems reaching the cull;
every pair shape gives the same bits; short FP64 trajectories follow the
oracle's integrator."""
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


CASES = {
    "dimers_icosa_128": lambda: I.dimer_gas("icosahedron", 64),
    "contact_icosa_128": lambda: I.contact_dimers(I.icosahedron(), n_pairs=64),
    "fat_dimers_icosa_128": lambda: I.dimer_gas("icosahedron", 64, edge=0.3, r=0.5),
    "lattice_icosa_512": lambda: I.contact_lattice(I.icosahedron(1.0, 0.1), 512, seed=41, max_deg=2.0),
    "cubes_contact_512": lambda: I.cubes_3d_contact(n_side=8),
    "contact_octa_128": lambda: I.contact_dimers(I.octahedron(), n_pairs=64),
    "contact_tetra_128": lambda: I.contact_dimers(I.tetrahedron(), n_pairs=64),
    "notch_lprism_cube_256": lambda: I.contact_dimers(I.lprism(0.1, quad_h=0.05), I.cube(1.0, 0.15),
                                                      n_pairs=128, notch=True),
    "notch_lprism_lprism_128": lambda: I.contact_dimers(I.lprism(0.1, quad_h=0.05), I.lprism(0.15, quad_h=0.05),
                                                        n_pairs=64, notch=True, seed=17),
    "squares_2d_contact_256": lambda: I.squares_2d_contact(),
    "dimers_16gon_128": lambda: I.dimer_gas("hexadecagon", 64, dim=2),
    "fat_dimers_16gon_128": lambda: I.dimer_gas("hexadecagon", 64, dim=2, edge=0.1, r=0.5),
    "contact_pentagon_128": lambda: I.contact_dimers(I.pentagon(), n_pairs=64),
}


def _run(dem, s, prec, cells, shape=None):
    with dem.DemSystem(s, prec) as g:
        g.set_feature_cells(cells)
        if shape is not None:
            g.set_pair_shape(*shape)
        g.set_counting(True)
        g.force_stats(reset=True)
        g.compute_forces()
        return g.outputs(), g.force_stats()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_feature_cells_match_oracle(name, prec):
    dem = _dem()
    s = CASES[name]()
    print(f"[cells] {name} n={s.n} {prec}", flush=True)
    ref = O.forces(s)
    assert ref["stats"]["near_par"] == 0
    out, st = _run(dem, s, prec, True)
    _, st0 = _run(dem, s, prec, False)
    print(name, prec, "cells", st, "planes", st0, flush=True)
    check(name + "/cells", prec, out, ref)
    assert st["pairs"] == st0["pairs"] and st["separated"] == st0["separated"]
    assert st["in_cutoff"] > 0
    if prec == "fp64":  # the same feature pairs inside the cutoff
        assert st["in_cutoff"] == st0["in_cutoff"]


@pytest.mark.parametrize("name", ["contact_icosa_128", "fat_dimers_icosa_128", "lattice_icosa_512",
                                  "squares_2d_contact_256", "fat_dimers_16gon_128"])
def test_feature_cells_shapes_identical(name):
    dem = _dem()
    from test_gpu_shapes import SHAPES
    s = CASES[name]()
    print(f"[cells] shapes {name} n={s.n}", flush=True)
    outs = [_run(dem, s, "fp32", True, shape)[0] for shape in SHAPES]
    for o in outs[1:]:
        for k in o:
            assert np.array_equal(o[k], outs[0][k]), k


@pytest.mark.parametrize("which", ["cubes_nvt", "icosa_nve"])
def test_feature_cells_trajectory_fp64(which):
    dem = _dem()
    if which == "cubes_nvt":
        s = I.cubes_3d_contact(n_side=6)
        s.ensemble = "nvt"
        s.kT = 1.5
        n = 60
    else:
        s = I.contact_lattice(I.icosahedron(1.0, 0.1), 216, seed=43, ensemble="nve", max_deg=2.0)
        n = 60
    print(f"[cells] trajectory {which} n={s.n} steps={n}", flush=True)
    ref, th, lg, rf = O.run(s, n)
    with dem.DemSystem(s, "fp64") as g:
        g.set_feature_cells(True)
        g.step(n)
        e = g.energy()
        st = g.state()
    ux = st.x + st.image * s.box
    rx = ref.x + ref.image * s.box
    assert np.abs(ux - rx).max() < 1e-9
    assert np.abs(st.v - ref.v).max() < 1e-7 * (1 + np.abs(ref.v).max())
    sgn = np.sign(np.sum(st.q * ref.q, axis=1))[:, None]
    assert np.abs(st.q * sgn - ref.q).max() < 1e-9
    assert e["U"] == pytest.approx(lg[-1, 0], rel=1e-8, abs=1e-10)
    assert e["H"] == pytest.approx(lg[-1, 5], rel=1e-9)
