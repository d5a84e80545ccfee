"""GPU batches of independent replicas (many systems, one launch per kernel
per step), through the C ABI.

* Every replica of a mixed batch matches the FP64 oracle (forces to the
  tolerances of parity_metrics.py, lists bit for bit).
* A replica's results are the same bit for bit alone (a single system), in
  a mix, and in a mix assembled in another order, after steps that cross
  list rebuilds, NVE and NVT replicas together.
* Step budgets: a replica with a budget stops exactly there; removing and
  adding replicas mid-run leaves the others bit-identical to their solo runs.
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


def _drop_last(s):
    s = s.copy()
    s.x, s.q, s.v, s.L = s.x[:-1], s.q[:-1], s.v[:-1], s.L[:-1]
    s.shape_id, s.image = s.shape_id[:-1], s.image[:-1]
    return s


def _mix3d():
    a = I.cubes_3d_contact(n_side=8)                       # 512 cubes, every neighbour in contact
    b = I.dimer_gas("tetrahedron", 100, seed=11)           # 200 tetrahedra in contact pairs
    c = I.dimer_gas("lprism", 40, seed=12, quad_h=0.05)    # 80 concave L-prisms
    d = _drop_last(I.dimer_gas("cube", 19, seed=13))       # 37: a ragged chunk
    e = I.cubes_3d(n_side=6)                               # 216 cubes at volume fraction 0.4, NVT
    f = I.dimer_gas("octahedron", 70, seed=14)             # 140 octahedra
    g = I.contact_dimers(I.lprism(0.1, quad_h=0.05), I.cube(1.0, 0.15), n_pairs=40, notch=True, seed=15)
    b.ensemble = c.ensemble = "nve"                        # g: 80, L-prisms against cubes over the concave caps
    return [a, b, c, d, e, f, g]


def _mix2d():
    a = I.squares_2d_contact()
    b = I.dimer_gas("pentagon", 90, seed=21, dim=2)
    c = _drop_last(I.dimer_gas("square", 33, seed=22, dim=2))
    return [a, b, c]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dim", [3, 2])
def test_batch_matches_oracle(dim, prec):
    dem = _dem()
    systems = _mix3d() if dim == 3 else _mix2d()
    print(f"[batch-oracle] dim={dim} {prec} sizes={[s.n for s in systems]}", flush=True)
    with dem.DemBatch(dim, prec, max_replicas=16, max_particles=4096) as B:
        rids = [B.add(s) for s in systems]
        for s, r in zip(systems, rids):
            _, out = B.read(r)
            ref = O.forces(s)
            check(f"batch{dim}d_replica{r}_{s.name}", prec, out, ref)
            L = B.lists(r)
            rl = O.OracleSystem.of(s).r_list(s.skin)
            nc, cs, cp = O.cell_list(s, rl)
            assert np.array_equal(L["dims"], nc)
            assert np.array_equal(L["cell_start"], cs)
            assert np.array_equal(L["cell_particles"], cp)
            nb, nn, _ = O.nbr_list(s, rl, cap=L["capacity"], mode=1)
            assert np.array_equal(L["n_nbr"], nn)
            for i in range(s.n):
                assert np.array_equal(L["nbr"][: nn[i], i], nb[: nn[i], i])


def _solo(dem, s, prec, steps):
    with dem.DemSystem(s, prec) as g:
        b0 = g.energy()["n_rebuilds"]
        g.step(steps)
        st = g.state()
        out = g.outputs()
        e = g.energy()
        e["rebuilds_in_run"] = e["n_rebuilds"] - b0
    return st, out, e


def _same(a, b):
    sa, oa = a
    sb, ob = b
    for k in ("x", "q", "v", "L", "image"):
        assert np.array_equal(getattr(sa, k), getattr(sb, k)), k
    for k in ("F", "T", "U", "W"):
        assert np.array_equal(oa[k], ob[k]), k


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_alone_equals_in_mix(prec):
    dem = _dem()
    systems = _mix3d()
    steps = 300
    solo = [_solo(dem, s, prec, steps) for s in systems]
    for order in (list(range(len(systems))), list(reversed(range(len(systems))))):
        print(f"[mix] {prec} order={order}", flush=True)
        with dem.DemBatch(3, prec, max_replicas=16, max_particles=8192) as B:
            rids = {k: B.add(systems[k]) for k in order}
            b0 = {k: B.energy(r)["n_rebuilds"] for k, r in rids.items()}
            B.step(steps)
            for k, r in rids.items():
                st, out = B.read(r)
                _same((st, out), solo[k][:2])
                e = B.energy(r)
                assert e["step"] == steps
                assert e["H"] == solo[k][2]["H"]
                assert e["n_rebuilds"] - b0[k] == solo[k][2]["rebuilds_in_run"]
    assert max(x[2]["rebuilds_in_run"] for x in solo) > 0  # the run crossed list rebuilds


def test_budgets_add_remove():
    dem = _dem()
    a, b, c = I.cubes_3d(n_side=5), I.dimer_gas("tetrahedron", 60, seed=31), I.cubes_3d_contact(n_side=5)
    b.ensemble = "nve"
    print("[budget] sizes", a.n, b.n, c.n, flush=True)
    with dem.DemBatch(3, "fp32", max_replicas=4, max_particles=1024) as B:
        ra = B.add(a, steps=100)
        rb = B.add(b)
        B.step(150)
        left, done = B.progress(4)
        assert done[ra] == 100 and left[ra] == 0
        assert done[rb] == 150
        _same(B.read(ra), _solo(dem, a, "fp32", 100)[:2])
        B.remove(ra)
        rc = B.add(c, steps=40)
        B.step(50)
        left, done = B.progress(4)
        assert done[rb] == 200 and done[rc] == 40
        _same(B.read(rb), _solo(dem, b, "fp32", 200)[:2])
        _same(B.read(rc), _solo(dem, c, "fp32", 40)[:2])
        info = B.info()
        assert info["live"] == 2


def test_batch_full_is_reported():
    dem = _dem()
    with dem.DemBatch(3, "fp32", max_replicas=2, max_particles=576) as B:
        B.add(I.cubes_3d_contact(n_side=8))                 # 512 of 576 slots
        with pytest.raises(dem.DemError) as ei:
            B.add(I.cubes_3d(n_side=5))                      # 125 more (two chunks of 64) do not fit
        assert ei.value.status == 3
        with pytest.raises(dem.DemError):
            B.add(I.squares_2d())                            # wrong dimension


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_split_calls_equal_one_call(prec):
    """NVT steps split over several dem_step calls give the same numbers as
    one call (the thermostat's pending half steps carry across calls)."""
    dem = _dem()
    s = I.cubes_3d(n_side=6)
    one = _solo(dem, s, prec, 122)
    with dem.DemSystem(s, prec) as g:
        for n in (37, 37, 37, 11):
            g.step(n)
        _same((g.state(), g.outputs()), one[:2])
        e = g.energy()
    assert e["H"] == one[2]["H"] and e["xi"] == one[2]["xi"]


def test_served_requests_equal_solo():
    """Requests served with continuous batching (arrivals while others run,
    two dimensions, chunked steps, admission and retirement mid-run) return
    the same state and forces, bit for bit, as each request run alone."""
    dem = _dem()
    from paper_1607_02427_amd import serve
    reqs = [I.replica_system(I.cube(r=0.15), 300, 0.4, 41, dt=5e-4),
            I.replica_system(I.pentagon(r=0.12), 256, 0.45, 42, dt=1e-4, kT=1.5),
            I.replica_system(I.octahedron(r=0.2), 200, 0.3, 43, dt=2e-4, kT=0.7),
            I.replica_system(I.tetrahedron(r=0.1), 150, 0.3, 44, dt=5e-4),
            I.replica_system(I.pentagon(r=0.18), 333, 0.4, 45, dt=1e-4, ensemble="nve")]
    for k, (t, n) in enumerate([(0.0, 130), (0.0, 95), (0.05, 70), (0.1, 111), (0.12, 64)]):
        reqs[k].arrival = t
        reqs[k].steps = n
    srv = serve.Server(budget_bytes=1 << 30, precision="fp32", max_replicas=8,
                       max_particles={2: 4096, 3: 4096}, chunk=20, keep_results=True)
    try:
        recs = srv.run(reqs)
    finally:
        srv.close()
    for r, s in zip(recs, reqs):
        print(f"[serve] request {r.index} n={s.n} steps={s.steps} latency {r.latency:.3f} s", flush=True)
        st, out = r.result
        solo = _solo(dem, s, "fp32", s.steps)
        _same((st, out), solo[:2])


def test_batch_admission_budget():
    """dem_batch_add charges each replica its footprint (lists, cells,
    scratch, state and outputs) against the batch's admission budget and
    returns DEM_E_OOM, with nothing changed, when a replica does not fit;
    removing a replica returns its charge."""
    dem = _dem()
    from paper_1607_02427_amd import serve
    a, b = I.cubes_3d(n_side=5), I.cubes_3d_contact(n_side=6)
    ca, cb = serve.request_bytes(a, "fp32"), serve.request_bytes(b, "fp32")
    with dem.DemBatch(3, "fp32", max_replicas=4, max_particles=4096, budget_bytes=max(ca, cb) + min(ca, cb) // 2) as B:
        ra = B.add(a)
        assert B.info()["bytes_charged"] == ca
        with pytest.raises(dem.DemError) as ex:
            B.add(b)
        assert ex.value.status == 3 and "admission budget" in str(ex.value)
        assert B.info()["live"] == 1 and B.info()["bytes_charged"] == ca
        B.remove(ra)
        assert B.info()["bytes_charged"] == 0
        rb = B.add(b)
        assert B.info()["bytes_charged"] == cb
        B.step(10)
        _, out = B.read(rb)
        assert np.isfinite(out["F"]).all()


def test_served_requests_wait_on_memory():
    """A budget that holds the largest request and little more:
    later arrivals wait for memory (not for slots) until earlier requests
    retire, and every result is still the request's solo result bit for bit."""
    dem = _dem()
    from paper_1607_02427_amd import serve
    reqs = [I.replica_system(I.cube(r=0.15), 512, 0.4, 51, dt=5e-4),
            I.replica_system(I.octahedron(r=0.2), 400, 0.3, 52, dt=2e-4, kT=0.7),
            I.replica_system(I.tetrahedron(r=0.1), 450, 0.3, 53, dt=5e-4),
            I.replica_system(I.cube(r=0.2), 300, 0.35, 54, dt=5e-4, kT=1.3)]
    for k, (t, n) in enumerate([(0.0, 120), (0.0, 90), (0.01, 60), (0.02, 75)]):
        reqs[k].arrival = t
        reqs[k].steps = n
    budget = int(1.05 * max(serve.request_bytes(s, "fp32") for s in reqs))
    srv = serve.Server(budget_bytes=budget, precision="fp32", max_replicas=8, max_particles={3: 8192}, chunk=20,
                       keep_results=True)
    try:
        recs = srv.run(reqs)
    finally:
        srv.close()
    waited = [r for r in recs if r.waited_on_memory]
    print(f"[serve] budget {budget} bytes, peak {srv.peak_used}, {len(waited)} requests waited on memory", flush=True)
    assert waited and srv.peak_used <= budget
    assert all(r.admitted > r.arrival for r in waited)
    for r, s in zip(recs, reqs):
        st, out = r.result
        _same((st, out), _solo(dem, s, "fp32", s.steps)[:2])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_with_spheres_and_cells_matches_oracle(prec):
    """A batch holding sphere replicas (central WCA) beside polytope ones,
    evaluated once with the supporting-plane prefilter and once with the
    shape-local feature cells: every replica against the oracle, and in
    FP64 the cells change no bit of the sphere replicas (their pairs never
    reach the feature stage)."""
    dem = _dem()
    systems = [I.lattice_system(I.sphere(0.5), 8, 0.4, 7, orient="uniform", jitter=0.05),
               I.contact_dimers(I.cube(1.0, 0.15), I.sphere(0.2), n_pairs=40),
               I.contact_dimers(I.icosahedron(), n_pairs=32),
               I.cubes_3d_contact(n_side=6)]
    outs = {}
    for cells in (False, True):
        print(f"[batch-spheres] {prec} cells={cells} sizes={[s.n for s in systems]}", flush=True)
        with dem.DemBatch(3, prec, max_replicas=8, max_particles=4096, max_cells=16384) as B:
            B.set_feature_cells(cells)
            rids = [B.add(s) for s in systems]
            B.compute_forces()
            for s, r in zip(systems, rids):
                _, out = B.read(r)
                check(f"batch_spheres_cells{int(cells)}_replica{r}_{s.name}", prec, out, O.forces(s))
                outs[(cells, r)] = out
    if prec == "fp64":
        for k in ("F", "T", "U", "W"):
            assert np.array_equal(outs[(False, rids[0])][k], outs[(True, rids[0])][k]), k
