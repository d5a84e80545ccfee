"""The allocation-free energy entry point (dem_replica_energy_noalloc)
against dem_replica_energy, through the C ABI: the same results bit for bit
on two calls in a row, the second on a smaller replica, then on a single
system, and its rejection of replicas beyond the static scratch."""
import numpy as np
import pytest

from paper_1607_02427_amd import inputs as I

pytestmark = pytest.mark.gpu


def _dem():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1607_02427_amd import dem
    return dem


def _same(a, b, label):
    for k in a:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (label, k, a[k], b[k])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_energy_equals_energy(prec):
    dem = _dem()
    big = I.cubes_3d_contact(n_side=8)      # 512 cubes, every lattice neighbour in contact
    small = I.cubes_3d(n_side=5)            # 125 cubes
    with dem.DemBatch(3, prec, max_replicas=4, max_particles=1024) as B:
        rb, rs = B.add(big), B.add(small)
        B.step(30)
        for rid, label in ((rb, "512 cubes"), (rs, "125 cubes")):  # the second call on the smaller replica
            print(f"[noalloc] {prec} replica {rid} ({label})", flush=True)
            ref = B.energy(rid)
            got = B.energy_noalloc(rid)
            assert ref["U"] > 0.0 or label == "125 cubes"
            _same(ref, got, label)
        # once more on the big one after the small one
        _same(B.energy(rb), B.energy_noalloc(rb), "512 cubes again")
    s = I.squares_2d_contact()
    with dem.DemSystem(s, prec) as g:
        g.step(10)
        print(f"[noalloc] {prec} single system {s.name}", flush=True)
        _same(g.energy(), g.energy_noalloc(), s.name)


def test_noalloc_rejects_replicas_beyond_scratch():
    dem = _dem()
    s = I.lattice_system(I.cube(1.0, 0.15), 65, 0.1, 91, orient="small", name="cubes_274625")  # 4292 chunks
    print(f"[noalloc] {s.name} n={s.n}", flush=True)
    with dem.DemSystem(s, "fp32") as g:
        with pytest.raises(dem.DemError) as ex:
            g.energy_noalloc()
        assert ex.value.status == 5  # DEM_E_CAPACITY
        assert "262144" in str(ex.value)
        e = g.energy()  # the allocating call still works on it
        assert np.isfinite(e["H"])
