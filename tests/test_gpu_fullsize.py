"""GPU parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times (tuned pair shape).

* 4096 rounded cubes at step 1000 of their NVT run (a fluid with contacts,
  integrated by the oracle from the seeded start): every particle, FP64 and
  FP32.
* The 96-replica batch (867,840 particles): its seeded start exactly as the
  benchmark steps it, and the same replicas on contact lattices (every
  lattice neighbour in contact), all 96 in one batch; per replica a seeded
  sample of particles (all of them for the small replicas, and always the
  first and the last, the ragged tail of a chunk) against the oracle's
  subset evaluation.
"""
import numpy as np
import pytest

import oracle as O
from paper_1607_02427_amd import inputs as I
from parity_metrics import check

pytestmark = pytest.mark.gpu


def _dem():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1607_02427_amd import dem
    return dem


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cubes_4096_equilibrated(prec):
    dem = _dem()
    s = I.cubes_3d_equilibrated()
    print(f"[full] {s.name} n={s.n} {prec}", flush=True)
    ref = O.forces(s)
    assert ref["stats"]["feature_in"] > 1000
    with dem.DemSystem(s, prec) as g:
        shape = g.tune_pairs(2)
        g.compute_forces()
        out = g.outputs()
        st = g.force_stats()
    print(prec, shape["lanes"], shape["grid"], shape["waves"], shape["sep"], shape["split"], ref["stats"], st, flush=True)
    check(f"{s.name}", prec, out, ref)


def _sample(n, rng, k=128):
    if n <= 1200:
        return np.arange(n)
    pick = rng.choice(n, size=k, replace=False)
    return np.unique(np.concatenate([pick, [0, n - 1]]))


def _batch_against_oracle(dem, reps, prec, label):
    total = sum(s.n for s in reps)
    rng = np.random.Generator(np.random.PCG64(77))
    with dem.DemBatch(3, prec, max_replicas=len(reps) + 8, max_particles=total + 64 * len(reps)) as B:
        rids = [B.add(s) for s in reps]
        shape = B.tune_pairs(2)
        B.compute_forces()
        print(f"[full] {label} {prec} {len(reps)} replicas {total} particles, pair shape "
              f"{shape['lanes']}x{shape['grid']}x{shape['waves']}x{shape['sep']}x{shape['split']}", flush=True)
        worst = {}
        for s, r in zip(reps, rids):
            _, out = B.read(r)
            pick = _sample(s.n, rng)
            ref = O.forces_subset(s, pick)
            sub = {k: out[k][pick] for k in ("F", "T", "U", "W")}
            rep = check(f"{label}/{s.name}[{len(pick)} of {s.n}]", prec, sub, ref)
            name = s.shapes[0].name
            worst[name] = max(worst.get(name, 0.0), max(v["e"] for v in rep.values()))
        print(f"[full] {label} {prec} worst e by shape {worst}", flush=True)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch96_contact_lattices(prec):
    dem = _dem()
    reps = I.batched_replicas_contact()
    _batch_against_oracle(dem, reps, prec, "batch96_contact")


def test_batch96_workload_start():
    dem = _dem()
    reps = I.batched_replicas()
    _batch_against_oracle(dem, reps, "fp32", "batch96")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_octahedra_262144_compressed(prec):
    """The at-scale workload as the benchmark times it: 262,144 rounded
    octahedra at volume fraction 0.55, random orientations compressed from a
    dilute BCC lattice (the stored 4096-body cell, tiled 4 x 4 x 4); a
    seeded sample of particles, the first and the last included."""
    dem = _dem()
    s = I.octahedra_compressed()
    rng = np.random.Generator(np.random.PCG64(78))
    pick = _sample(s.n, rng, k=512)
    print(f"[full] {s.name} n={s.n} {prec}, {len(pick)} sampled", flush=True)
    ref = O.forces_subset(s, pick)
    assert ref["stats"]["feature_in"] > 100
    with dem.DemSystem(s, prec) as g:
        shape = g.tune_pairs(2)
        g.compute_forces()
        out = g.outputs()
        st = g.force_stats()
    print(prec, shape["lanes"], shape["grid"], shape["waves"], shape["sep"], shape["split"], ref["stats"], st, flush=True)
    sub = {k: out[k][pick] for k in ("F", "T", "U", "W")}
    check(f"{s.name}[{len(pick)} of {s.n}]", prec, sub, ref)
