"""Pair-kernel launch shapes (lanes per pair, grid factor, waves per SIMD, separation lanes, split): every
shape the tuner can choose gives the same forces and the same trajectories
bit for bit, and tuning leaves the state alone.  The per-pair sums are
formed in a canonical order (problem k of a solve round into partial sum
k mod 16, one fixed combining tree), and a pair's result does not depend on
which wavefront or kernel takes it, so the shape, the two-kernel split of
contact search and forces included, is a pure performance knob."""
import numpy as np
import pytest

from paper_1607_02427_amd import inputs as I

pytestmark = pytest.mark.gpu

SHAPES = [(16, 1, 2, 4, 0), (8, 1, 2, 4, 0), (16, 2, 2, 4, 0), (8, 2, 2, 4, 0), (16, 1, 3, 4, 0), (8, 1, 3, 4, 0),
          (16, 2, 3, 4, 0), (8, 2, 3, 4, 0), (16, 1, 2, 16, 0), (16, 2, 2, 16, 0), (16, 1, 3, 16, 0),
          (16, 2, 3, 16, 0), (16, 1, 2, 4, 1), (8, 1, 2, 4, 1), (16, 1, 3, 4, 1), (8, 1, 3, 4, 1)]

CASES = {
    "cubes_contact_512": lambda: I.cubes_3d_contact(n_side=8),
    "dimers_tetra_256": lambda: I.dimer_gas("tetrahedron", 128),
    "dimers_lprism_128": lambda: I.dimer_gas("lprism", 64, quad_h=0.05),
    "squares_2d_contact_256": lambda: I.squares_2d_contact(),
    "dimers_pentagon_256": lambda: I.dimer_gas("pentagon", 128, dim=2),
    "dimers_icosa_128": lambda: I.dimer_gas("icosahedron", 64),
    # hundreds of in-range problems per pair: solve rounds end part-way
    # through pairs, at different points for the pairs of one wavefront
    "fat_dimers_16gon_128": lambda: I.dimer_gas("hexadecagon", 64, dim=2, edge=0.1, r=0.5),
    "fat_dimers_icosa_128": lambda: I.dimer_gas("icosahedron", 64, edge=0.3, r=0.5),
}


def _dem():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1607_02427_amd import dem
    return dem


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("name", list(CASES))
def test_shapes_give_identical_forces(name, prec):
    dem = _dem()
    s = CASES[name]()
    print(f"[shapes] {name} n={s.n} {prec}", flush=True)
    outs = []
    for shape in SHAPES:
        with dem.DemSystem(s, prec) as g:
            g.set_pair_shape(*shape)
            g.compute_forces()
            outs.append(g.outputs())
    for o in outs[1:]:
        _same(o, outs[0])


def _state_arrays(s):
    return dict(x=s.x, q=s.q, v=s.v, L=s.L, image=s.image)


def test_shapes_give_identical_trajectories():
    dem = _dem()
    s = I.cubes_3d(n_side=10)
    print(f"[shapes] cubes_1000 NVT 300 steps", flush=True)
    ends = []
    for shape in [(16, 1, 2, 4, 0), (8, 2, 3, 4, 0), (16, 1, 3, 16, 0), (8, 1, 3, 4, 1), (16, 1, 2, 4, 1)]:
        with dem.DemSystem(s, "fp32") as g:
            g.set_pair_shape(*shape)
            g.step(300)
            ends.append((_state_arrays(g.state()), g.energy()))
    for e in ends[1:]:
        _same(ends[0][0], e[0])
        assert ends[0][1]["H"] == e[1]["H"]


def test_tuner_keeps_state_and_results():
    dem = _dem()
    s = I.cubes_3d(n_side=10)
    print(f"[shapes] tuner on cubes_1000", flush=True)
    with dem.DemSystem(s, "fp32") as ref:
        ref.step(100)
        want = _state_arrays(ref.state())
    with dem.DemSystem(s, "fp32") as g:
        g.step(50)
        before = _state_arrays(g.state())
        r = g.tune_pairs(3)
        print("tuned", r, flush=True)
        assert (r["lanes"], r["grid"], r["waves"], r["sep"], r["split"]) in SHAPES
        assert all(v > 0 for v in r["mean_ms"].values())
        _same(_state_arrays(g.state()), before)
        g.step(50)
        _same(_state_arrays(g.state()), want)


def test_tuned_batch_equals_untuned():
    dem = _dem()
    reps = I.batched_replicas(6, seed=9, n_range=(300, 1500), steps=60)
    print(f"[shapes] batch of {len(reps)} replicas", flush=True)
    results = []
    for tune in (False, True):
        with dem.DemBatch(3, "fp32", max_replicas=8, max_particles=sum(s.n for s in reps) + 64 * 8) as b:
            ids = [b.add(s, steps=s.steps) for s in reps]
            if tune:
                print("tuned", b.tune_pairs(2), flush=True)
            b.step(60)
            results.append([_state_arrays(b.read(r)[0]) for r in ids])
    for a, c in zip(results[0], results[1]):
        _same(a, c)


def test_split_batch_equals_fused():
    """The split form compacts each replica's pairs into its own range and
    walks them replica by replica: a mixed 2D batch and a 3D batch step
    the same with it as with the one-kernel form, list rebuilds included."""
    dem = _dem()
    for dim, reps in ((3, I.batched_replicas(6, seed=9, n_range=(300, 1500), steps=60)),
                      (2, [I.squares_2d_contact(), I.dimer_gas("pentagon", 90, seed=21, dim=2),
                           I.dimer_gas("square", 33, seed=22, dim=2)])):
        print(f"[shapes] split vs fused, {dim}D batch of {len(reps)} replicas", flush=True)
        results = []
        for shape in ((16, 1, 2, 4, 0), (8, 1, 3, 4, 1), (16, 1, 2, 4, 1)):
            with dem.DemBatch(dim, "fp32", max_replicas=8, max_particles=sum(-(-s.n // 64) * 64 for s in reps) + 512,
                              max_cells=16384) as b:
                ids = [b.add(s, steps=60) for s in reps]
                b.set_pair_shape(*shape)
                b.step(60)
                results.append([_state_arrays(b.read(r)[0]) for r in ids])
        for other in results[1:]:
            for a, c in zip(results[0], other):
                _same(a, c)
