#!/usr/bin/env python
"""Benchmark of the rounded-polytope DEM step on one MI355X.

Workload: 4096 rounded cubes (edge 1, rounding radius 0.15, so sigma 0.3) at
volume fraction 0.4 in a periodic cube, Nose-Hoover NVT at kT = 1,
dt = 5e-4; FP32 pair geometry with FP64 positions, integration and
reductions.  The timed steps start from the workload's own state at step
1000 of its NVT run from the seeded 16^3 lattice (a fluid with contacts,
integrated by the oracle and stored with its SHA-256), after --warmup more
steps on the GPU.  One step is the whole path: thermostat, kick-drift,
displacement-triggered cell and neighbour lists, pair forces (Eq. 1 with
WCA), closing kick.

Prints one JSON line: particle-timesteps/s of the FP32 path (the value), the
plain FP64 single-system path on the same inputs, the force kernel's ALU
roofline (the method's work per launch at fixed per-problem flop weights /
mean launch time from HIP events on the launch stream), the work counters
at both ends of the timed window, and the CPU oracle timed on this host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-timesteps/s (3D cubes) FP32-batched vs plain; p50/p99 replica latency"

# FP32 flop weights of the pair kernel's formulas (add/mul/sub 1, FMA 2,
# divide or reciprocal 1), per unit of work its counters report.
FLOPS = {
    "pair": 60,        # relative rotation R_i^T R_j and offset R_i^T d (once per particle pair)
    "sep_vertex": 18,  # vertex carried into the other body's frame for the separation test (nv_i + nv_j per pair)
    "plane_test": 6,   # one vertex against one supporting plane
    "vertex": 23,      # vertex carried across again + reach test (nv_i + nv_j per pair not separated),
                       # plus one plane_test per supporting plane of the other body
    "edge": 12,        # edge reach test (ne_i + ne_j per pair)
    "face": 12,        # face reach test (nf_i + nf_j per pair)
    "cull": 17,        # per-problem test: plane + bounding circle, or segment bounding spheres
                       # (the line-distance test of edge pairs whose spheres meet is not counted)
    "vf_solve": 100,   # inside test, projection or boundary edges, offset back to i's frame
    "ee_solve": 65,    # segment-segment closest points and offset
    "ve_solve": 20,    # 2D point-segment nearest point and offset
    "wca": 56,         # WCA energy/force, accumulation of F, both torques and U
}
# Algorithmic work of Eq. 1 / Eq. 2 per unordered particle pair within
# R_i + R_j + r_cut: every feature-pair problem at a fixed flop weight
# (vertex-edge 15, edge-edge 45, vertex-triangle 45, vertex-quadrilateral 60;
# a face of k > 4 vertices 60 + 15 (k - 4), one more edge test per vertex),
# plus 40 per feature pair inside the cutoff (WCA and accumulation).
METHOD_FLOPS = {"ve": 15, "ee": 45, "vtri": 45, "vquad": 60, "wca": 40}


def method_flops_per_pair(si, sj, dim):
    """Flops of every feature-pair problem between shapes si and sj."""
    if dim == 2:
        return (si.nv * sj.ne + sj.nv * si.ne) * METHOD_FLOPS["ve"]
    w = lambda k: METHOD_FLOPS["vtri"] if k == 3 else METHOD_FLOPS["vquad"] + METHOD_FLOPS["ve"] * (k - 4)
    vf = si.nv * sum(w(len(f)) for f in sj.faces) + sj.nv * sum(w(len(f)) for f in si.faces)
    return vf + si.ne * sj.ne * METHOD_FLOPS["ee"]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_pairs_cubes4096.txt")
PAIR_SOURCES = [os.path.join(ROOT, "paper_1607_02427_amd", "csrc", f) for f in ("dem_force.hip", "dem_internal.h")]
PEAK_FP32 = 157.3e12   # MI355X FP32 vector, published (needs packed FP32)
PEAK_FP32_NONPACKED = 78.6e12  # one FP32 lane operation per cycle, the rate this build's code can reach
PEAK_HBM = 8.0e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def counters_now(g):
    """Work counters of one force evaluation on the current state."""
    g.force_stats(reset=True)
    g.compute_forces()
    return g.force_stats(reset=True)


# --pair-shape and --feature-cells: a fixed pair-kernel shape instead of the
# tuner's choice, and the shape-local feature cells, on every leg
FORCED_SHAPE = None
CELLS = False


def pick_shape(g, reps):
    """The tuner's shape, or the forced one (reported the same way)."""
    if FORCED_SHAPE is None:
        return g.tune_pairs(reps)
    g.set_pair_shape(*FORCED_SHAPE)
    return dict(zip(("lanes", "grid", "waves", "sep", "split"), FORCED_SHAPE), forced=True)


def run_path(system, precision, steps, warmup, counting=False, tune=True, cells=None):
    import torch
    from paper_1607_02427_amd import dem
    g = dem.DemSystem(system, precision)
    g.set_feature_cells(CELLS if cells is None else cells)
    stream = g.stream
    if counting:
        g.set_counting(True)
    g.step(warmup)
    g.sync()
    shape = pick_shape(g, 20) if tune else None
    start = counters_now(g)  # the state the timed window starts from (forces are recomputed, unchanged)
    if counting:
        g.force_stats(reset=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    g.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    en = g.energy()
    return g, dict(wall_s=wall, gpu_ms=gpu_ms, energy=en, pair_shape=shape, counters_start=start)


def pair_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for p in PAIR_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per k_pairs launch from the committed counter summary, if it
    was taken on the kernel as it is now (same source digest), else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != pair_sources_digest():
        return None
    try:
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(mb):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = int(mb) * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: 5 copies of {mb} MiB")


def force_roofline(g, system, reps=200):
    """Work counters of one force launch on the current state, and the mean
    launch duration of the force kernel alone (HIP events on its stream).

    achieved: the method's algorithmic work per launch (every feature-pair
    problem of Eq. 1 for every unordered pair within R_i + R_j + r_cut, at
    the METHOD_FLOPS weights, plus the WCA terms inside the cutoff) over the
    mean launch time.  executed: the work the kernel actually does after it
    proves problems empty (separation test, prefilter, cull), at the
    weights of its own formulas (FLOPS), in separate fields."""
    st = counters_now(g)
    mean_ms = g.time_forces(reps)
    assert len(system.shapes) == 1
    shp = system.shapes[0]
    per_pair = method_flops_per_pair(shp, shp, system.dim)
    algorithmic = st["pairs"] * per_pair + st["in_cutoff"] * METHOD_FLOPS["wca"]
    exec_per_pair = FLOPS["pair"] + 2 * shp.nv * FLOPS["sep_vertex"]
    planes = shp.nf if system.dim == 3 else shp.ne  # supporting planes of a convex body
    per_feature_pair = 2 * (shp.nv * (FLOPS["vertex"] + planes * FLOPS["plane_test"]) + shp.ne * FLOPS["edge"]
                            + shp.nf * FLOPS["face"])
    executed = (st["pairs"] * exec_per_pair + st["plane_tests"] * FLOPS["plane_test"]
                + (st["pairs"] - st["separated"]) * per_feature_pair + st["features"] * FLOPS["cull"]
                + st["vf_near"] * FLOPS["vf_solve"] + st["ee_near"] * FLOPS["ee_solve"] + st["in_cutoff"] * FLOPS["wca"])
    t = mean_ms * 1e-3
    return dict(bound="alu", achieved=algorithmic / t / 1e12, peak=PEAK_FP32 / 1e12, unit="TFLOP/s",
                frac=algorithmic / t / PEAK_FP32, traffic=measured_traffic(), kernel="k_pairs<float,3>",
                mean_launch_ms=mean_ms, flops_per_launch=algorithmic, flops_per_pair=per_pair,
                flops_per_pts=algorithmic / system.n,
                peak_fp32_nonpacked=PEAK_FP32_NONPACKED / 1e12,
                frac_nonpacked=algorithmic / t / PEAK_FP32_NONPACKED,
                executed={"tflops": executed / t / 1e12, "frac": executed / t / PEAK_FP32,
                          "flops_per_launch": executed,
                          "note": "work the kernel executes after its separation test, prefilter and cull, "
                                  "at its own formulas' weights"},
                counters=st)


def run_batched(replicas, steps, warmup, precision="fp32"):
    """All replicas in one batch: every step is one launch per kernel."""
    import torch
    from paper_1607_02427_amd import dem
    total = sum(s.n for s in replicas)
    b = dem.DemBatch(3, precision, max_replicas=len(replicas) + 8, max_particles=total + 64 * len(replicas))
    b.set_feature_cells(CELLS)
    for s in replicas:
        b.add(s)
    b.step(warmup)
    b.sync()
    shape = pick_shape(b, 3)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    b.sync()
    b.close()
    return dict(value=total * steps / (ms * 1e-3), ms_per_step=ms / steps, particles=total, pair_shape=shape)


def run_plain_sequential(replicas, steps, warmup):
    """The same replicas one after another, each a single FP64 system."""
    import torch
    from paper_1607_02427_amd import dem
    total_ms = 0.0
    for s in replicas:
        with dem.DemSystem(s, "fp64") as g:
            g.step(warmup)
            g.sync()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(g.stream)
            g.step(steps)
            e1.record(g.stream)
            torch.cuda.synchronize()
            total_ms += e0.elapsed_time(e1)
    work = sum(s.n for s in replicas) * steps
    return dict(value=work / (total_ms * 1e-3), seconds=total_ms * 1e-3)


def cpu_baseline(system, target_s):
    """The oracle's own NVT run of the workload on this host's cores: all of
    them (the reported value) and one thread (the paper's comparison), each
    over a bounded number of steps from the same state."""
    import oracle as O
    threads = len(os.sched_getaffinity(0))
    out = {}
    for label, nt in (("all", threads), ("one", 1)):
        O.set_threads(nt)
        s = system.copy()
        th = list(system.thermo) if system.thermo is not None else None
        t0 = time.perf_counter()
        O.run(s, 1, log=False, thermo=th)
        one = time.perf_counter() - t0
        steps = max(1, min(500, int(0.5 * target_s / max(one, 1e-6))))
        t0 = time.perf_counter()
        O.run(s, steps, log=False, thermo=th)
        dt = time.perf_counter() - t0
        out[label] = dict(value=system.n * steps / dt, steps=steps, seconds=dt, threads=O.get_threads())
    a, o = out["all"], out["one"]
    return dict(value=a["value"], unit="particle-timesteps/s", cores=a["threads"], kind="oracle",
                single_thread={"value": o["value"], "unit": "particle-timesteps/s", "cores": 1,
                               "sample": f"{o['steps']} NVT steps, {o['seconds']:.1f} s"},
                sample=f"{a['steps']} NVT steps of the same 4096-cube workload from its stored step-1000 state "
                       f"(FP64 brute force over every feature pair, own cell list) on {a['threads']} threads, "
                       f"{a['seconds']:.1f} s")


def energy_fluctuations(dts_tau=(0.000625, 0.00125, 0.0025, 0.005, 0.01), duration_tau=10.0, samples=1000,
                        thermal_tau=10.0, n_side=None):
    """The short-term energy conservation study of Sec. IV.A on this engine:
    each fluid (2D squares of edge 4.24 sigma, 3D tetrahedra of edge 8.49
    sigma) is thermalized at kT = 1 (Nose-Hoover, FP64, dt = 0.005 tau) and
    then run NVE for duration_tau at each timestep, in FP64 and FP32 pair
    geometry, recording E = U + K_trans + K_rot `samples` times; reported are
    sigma(E/N) and the drift (E(end) - E(0)) / (N duration), both in eps and
    tau units (tau = sigma sqrt(m / eps), sigma = 2 r)."""
    import numpy as np
    from paper_1607_02427_amd import dem, inputs as I
    out = {}
    for dim in (2, 3):
        s = I.energy_fluid(dim, n_side=n_side)
        tau = 2 * s.shapes[0].r
        with dem.DemSystem(s, "fp64") as g:
            g.step(int(round(thermal_tau / 0.005)))
            th = g.state()
        rows = []
        for prec in ("fp64", "fp32"):
            for dtt in dts_tau:
                t = th.copy()
                t.ensemble = "nve"
                t.dt = dtt * tau
                n = int(round(duration_tau / dtt))
                k = max(1, n // samples)
                E = []
                with dem.DemSystem(t, prec) as g:
                    for _ in range(n // k):
                        e = g.energy()
                        E.append(e["U"] + e["K_trans"] + e["K_rot"])
                        g.step(k)
                    e = g.energy()
                    E.append(e["U"] + e["K_trans"] + e["K_rot"])
                E = np.asarray(E) / t.n
                rows.append(dict(precision=prec, dt_tau=dtt, steps=n, sigma_E_per_N=float(E.std()),
                                 drift_per_N_per_tau=float((E[-1] - E[0]) / duration_tau)))
                log(f"[energy] {s.name} {prec} dt {dtt:g} tau: sigma(E/N) {E.std():.3e}, "
                    f"drift {(E[-1] - E[0]) / duration_tau:.2e} per tau")
        out[s.name] = dict(n=s.n, tau=tau, runs=rows)
    return out


def table1_workloads(steps=(2000, 1000, 300), warmup=200, sides=(6, 16, 40), modes=(False, True)):
    """The paper's Table I shapes and sizes on this engine: spheres (r = 0.5,
    the central WCA baseline), rounded cubes and rounded icosahedra (edge 1,
    r = 0.15 and 0.1) at N = 6^3, 16^3 and 40^3 (its 256, 4096 and 65536 on
    cubic lattices), volume fraction 0.4, NVT kT = 1 after `warmup` steps,
    FP32 pair geometry, tuned pair shape; the polytopes with the
    supporting-plane prefilter and with the shape-local feature cells
    (`modes`), with the work counters of one force evaluation at the start of
    the timed window.  The paper gives no densities; these are ours."""
    from paper_1607_02427_amd import inputs as I
    out = []
    for name, shp, orient in (("sphere", I.sphere(0.5), "uniform"), ("cube", I.cube(1.0, 0.15), "small"),
                              ("icosahedron", I.icosahedron(1.0, 0.1), "aligned")):
        for n_side, k in zip(sides, steps):
            for cells in (modes if name != "sphere" else (False,)):
                s = I.lattice_system(shp, n_side, 0.4, 31 + n_side, orient=orient, max_deg=10.0,
                                     name=f"{name}_{n_side ** 3}")
                s.ensemble = "nvt"
                s.dt = 5e-4
                g, r = run_path(s, "fp32", k, warmup, cells=cells)
                g.close()
                ptps = s.n * k / (r["gpu_ms"] * 1e-3)
                c = r["counters_start"]
                out.append(dict(shape=name, n=s.n, feature_search="cells" if cells else "planes", steps=k, value=ptps,
                                ms_per_step=r["gpu_ms"] / k,
                                pair_shape=[r["pair_shape"][a] for a in ("lanes", "grid", "waves", "sep", "split")],
                                pair_ms=min(r["pair_shape"].get("mean_ms", {"": float("nan")}).values()),
                                counters={a: c[a] for a in ("pairs", "separated", "features", "vf_near", "ee_near",
                                                            "in_cutoff")}))
                log(f"[table1] {name} N={s.n} {'cells' if cells else 'planes'}: {ptps:.3e} PTPS "
                    f"({r['gpu_ms'] / k * 1e3:.1f} us/step, pair kernel {out[-1]['pair_ms'] * 1e3:.1f} us, "
                    f"{c['features']} problems to the cull, {c['in_cutoff']} in the cutoff)")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 path")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--replicas", type=int, default=96, help="replicas of the batched workload")
    ap.add_argument("--batched-steps", type=int, default=500)
    ap.add_argument("--requests", type=int, default=256, help="requests of the served trace")
    ap.add_argument("--serve-budget-mb", type=int, default=512,
                    help="admission budget of the served leg (device MiB for the live requests)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-scale", action="store_true", help="skip the 262,144-octahedra run")
    ap.add_argument("--no-npt", action="store_true", help="skip the isothermal-isobaric cube run")
    ap.add_argument("--no-table1", action="store_true",
                    help="skip the Table I shapes at N = 4096 (spheres, cubes, icosahedra) in the default line")
    ap.add_argument("--npt-steps", type=int, default=2000)
    ap.add_argument("--scale-steps", type=int, default=300)
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="finish with device copies of this many MiB (scale for the HBM byte counters)")
    ap.add_argument("--pair-shape", default=None,
                    help="lanes,grid,waves,sep,split: this pair-kernel shape on every leg instead of the tuner's")
    ap.add_argument("--feature-cells", action="store_true",
                    help="the shape-local feature cells on every leg (the table1 runs take both)")
    ap.add_argument("--table1", action="store_true",
                    help="run only the cube and icosahedron workloads of the paper's Table I and print their JSON line")
    ap.add_argument("--energy-study", action="store_true",
                    help="run only the NVE energy-fluctuation study (Sec. IV.A) and print its JSON line")
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip the one-at-a-time plain FP64 runs of the batched and served workloads")
    args = ap.parse_args()
    global FORCED_SHAPE, CELLS
    if args.pair_shape:
        FORCED_SHAPE = tuple(int(v) for v in args.pair_shape.split(","))
        assert len(FORCED_SHAPE) == 5, "--pair-shape lanes,grid,waves,sep,split"
    CELLS = args.feature_cells
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is design-only.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1607_02427_amd import inputs as I
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.table1:
        print(json.dumps({"metric": "particle-timesteps/s, Table I shapes and sizes", "unit": "particle-timesteps/s",
                          "data": "synthetic", "dtype": "f32", "runs": table1_workloads()}), flush=True)
        return
    if args.energy_study:
        print(json.dumps({"metric": "sigma(E/N) of NVE runs against the timestep (Sec. IV.A)", "unit": "eps",
                          "data": "synthetic", "study": energy_fluctuations()}), flush=True)
        return
    system = I.cubes_3d_equilibrated()
    n = system.n
    log(f"[bench] fp32 path: {n} cubes from {system.name}, warmup {args.warmup}, steps {args.steps}")
    g, r32 = run_path(system, "fp32", args.steps, args.warmup)
    ptps = n * args.steps / (r32["gpu_ms"] * 1e-3)
    end = counters_now(g)
    log(f"[bench] fp32 {r32['gpu_ms'] / args.steps * 1e3:.2f} us/step, {ptps:.3e} PTPS, rebuilds "
        f"{r32['energy']['n_rebuilds']}, in-cutoff feature pairs {r32['counters_start']['in_cutoff']} -> "
        f"{end['in_cutoff']}")
    assert r32["counters_start"]["in_cutoff"] > 0 and end["in_cutoff"] > 0, "the timed window must hold contacts"
    roof = force_roofline(g, system)
    log(f"[bench] force kernel {roof['mean_launch_ms'] * 1e3:.2f} us, {roof['achieved']:.2f} TFLOP/s algorithmic, "
        f"{roof['executed']['tflops']:.2f} TFLOP/s executed")
    line = {
        "metric": METRIC, "value": ptps, "unit": "particle-timesteps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r32["gpu_ms"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"4096 rounded cubes, edge 1, r 0.15, volume fraction 0.4, NVT kT 1, dt 5e-4, "
                               f"FP32 pair geometry / FP64 integration, single system; timed from its state at "
                               f"step 1000 of its NVT run (stored, {system.name}) plus {args.warmup} steps",
                   "n": n, "box": float(system.box[0]), "dt": system.dt, "ensemble": "nvt",
                   "precision": "fp32 geometry, fp64 state"},
        "wall_s": r32["wall_s"],
        "rebuilds": r32["energy"]["n_rebuilds"],
        "pair_shape": r32["pair_shape"],
        "counters_window": {"start": r32["counters_start"], "end": end},
        "roofline": roof,
    }
    g.close()
    if not args.no_plain:
        log("[bench] plain fp64 path")
        g64, r64 = run_path(system, "fp64", args.steps, args.warmup)
        line["plain_fp64"] = {"value": n * args.steps / (r64["gpu_ms"] * 1e-3), "ms_per_step": r64["gpu_ms"] / args.steps}
        line["fp32_over_plain"] = ptps / line["plain_fp64"]["value"]
        g64.close()
    if not args.no_npt:
        # the same cubes at fixed pressure (Sec. IV.C): the target is the
        # state's own virial pressure, so the box breathes about its size
        g0 = __import__("paper_1607_02427_amd.dem", fromlist=["dem"]).DemSystem(system, "fp32")
        p0 = g0.energy()["P"]
        g0.close()
        snpt = system.copy()
        snpt.ensemble, snpt.P, snpt.tau_P = "npt", p0, 0.5
        log(f"[bench] npt: {n} cubes at P = {p0:.4f}, {args.npt_steps} steps")
        gn, rn = run_path(snpt, "fp32", args.npt_steps, 100)
        en = gn.energy()
        gn.close()
        line["npt"] = {"workload": f"{n} rounded cubes from the same stored state, NPT at P = {p0:.4f} (the state's "
                                   f"virial pressure), tau_P 0.5, kT 1, dt 5e-4, {args.npt_steps} steps after 100",
                       "value": n * args.npt_steps / (rn["gpu_ms"] * 1e-3), "unit": "particle-timesteps/s",
                       "ms_per_step": rn["gpu_ms"] / args.npt_steps, "dtype": "f32", "target_P": p0,
                       "final_P": en["P"], "final_V": en["V"], "start_V": float(np.prod(system.box)),
                       "rebuilds": en["n_rebuilds"]}
        log(f"[bench] npt {line['npt']['value']:.3e} PTPS, V {line['npt']['start_V']:.1f} -> {en['V']:.1f}")
    if not args.no_scale:
        big = I.octahedra_compressed()
        log(f"[bench] at scale: {big.n} octahedra, {args.scale_steps} steps")
        gs, rs = run_path(big, "fp32", args.scale_steps, 50)
        end = counters_now(gs)
        gs.close()
        line["at_scale"] = {
            "workload": f"{big.n} rounded octahedra (edge 1, r 0.1) at volume fraction 0.55, random orientations "
                        f"compressed from BCC at 0.25 (a 4096-body cell, tiled 4 x 4 x 4), NVT kT 1, dt 2e-4, "
                        f"{args.scale_steps} steps after 50 warm-up",
            "n": big.n, "value": big.n * args.scale_steps / (rs["gpu_ms"] * 1e-3), "unit": "particle-timesteps/s",
            "ms_per_step": rs["gpu_ms"] / args.scale_steps, "rebuilds": rs["energy"]["n_rebuilds"],
            "pair_shape": rs["pair_shape"], "dtype": "f32",
            "counters_window": {"start": rs["counters_start"], "end": end}}
        log(f"[bench] at scale {line['at_scale']['value']:.3e} PTPS, in-cutoff feature pairs "
            f"{rs['counters_start']['in_cutoff']} -> {end['in_cutoff']}")
    if not args.no_batched:
        reps = I.batched_replicas(args.replicas, steps=args.batched_steps)
        log(f"[bench] batched: {len(reps)} replicas, {sum(s.n for s in reps)} particles, "
            f"{args.batched_steps} steps")
        rb = run_batched(reps, args.batched_steps, 20)
        log(f"[bench] batched fp32 {rb['value']:.3e} PTPS")
        rb64 = run_batched(reps, args.batched_steps, 20, precision="fp64")
        log(f"[bench] batched fp64 {rb64['value']:.3e} PTPS")
        rp = None if args.no_sequential else run_plain_sequential(reps, args.batched_steps, 20)
        line["batched"] = {
            "workload": f"{len(reps)} NVT replicas (kT 1), sizes log-uniform 512-32768, shapes uniform over rounded "
                        f"cube / tetrahedron / concave L-prism, rounding U[0.1, 0.2], packing fraction U[0.3, 0.5] "
                        f"capped by an overlap-free lattice, {args.batched_steps} steps after 20 warm-up",
            "replicas": len(reps), "particles": rb["particles"], "steps": args.batched_steps,
            "value": rb["value"], "unit": "particle-timesteps/s", "ms_per_step": rb["ms_per_step"], "dtype": "f32",
            "pair_shape": rb["pair_shape"],
            "batched_fp64": {"value": rb64["value"], "ms_per_step": rb64["ms_per_step"]},
            "plain_fp64_sequential": rp["value"] if rp else None,
            "speedup_vs_plain": rb["value"] / rp["value"] if rp else None,
            "batching_speedup_fp64": rb64["value"] / rp["value"] if rp else None}
    if not args.no_served:
        from paper_1607_02427_amd import serve
        trace = I.served_trace(args.requests)
        work = sum(s.n * s.steps for s in trace)
        log(f"[bench] served: {len(trace)} requests, {work:.3e} particle-steps, arrivals over "
            f"{trace[-1].arrival:.2f} s")
        srv = serve.Server(budget_bytes=args.serve_budget_mb << 20, precision="fp32", max_replicas=len(trace) + 8,
                           max_particles={2: sum(s.n for s in trace if s.dim == 2) + 64 * len(trace),
                                          3: sum(s.n for s in trace if s.dim == 3) + 64 * len(trace)},
                           chunk=100)
        try:
            srs = serve.summarize(srv.run(trace))
        finally:
            srv.close()
        log(f"[bench] served p50 {srs['p50_latency_s']:.2f} s p99 {srs['p99_latency_s']:.2f} s, "
            f"{srs['value']:.3e} PTPS; sequential plain fp64")
        sqs = None if args.no_sequential else serve.summarize(serve.run_sequential(trace, "fp64"))
        line["served"] = {
            "workload": f"{len(trace)} requests, Poisson arrivals at 40/s, sizes log-uniform 256-65536, 2D rounded "
                        f"pentagons or 3D rounded cubes / octahedra, 1000-5000 NVT steps, kT U[0.5, 2]; "
                        f"{args.serve_budget_mb} MiB admission budget, continuous batching in chunks of 100 steps",
            "requests": len(trace), "p50_latency_s": srs["p50_latency_s"], "p99_latency_s": srs["p99_latency_s"],
            "budget_bytes": args.serve_budget_mb << 20, "peak_bytes": srv.peak_used,
            "waited_on_memory": srs["waited_on_memory"],
            "value": srs["value"], "unit": "particle-timesteps/s", "makespan_s": srs["makespan_s"],
            "offered_load": work / trace[-1].arrival, "dtype": "f32",
            "sequential_plain_fp64": None if sqs is None else {
                "p50_latency_s": sqs["p50_latency_s"], "p99_latency_s": sqs["p99_latency_s"], "value": sqs["value"],
                "makespan_s": sqs["makespan_s"]}}
    if not args.no_table1:
        log("[bench] Table I shapes at N = 4096")
        line["table1_4096"] = {
            "workload": "spheres (r 0.5, central WCA), rounded cubes (edge 1, r 0.15) and rounded icosahedra (edge 1, "
                        "r 0.1), 16^3 on a cubic lattice at volume fraction 0.4, NVT kT 1, 1000 steps after 200, FP32 "
                        "pair geometry, tuned pair shape",
            "paper_table1_gpu_m6000": {"sphere": 4.6e7, "cube": 3.8e5, "icosahedron": 8.0e4},
            "runs": table1_workloads(steps=(1000,), sides=(16,), modes=(False,))}
    if args.copy_mb > 0:
        copy_calibration(args.copy_mb)
    if not args.no_cpu:
        log("[bench] cpu oracle baseline")
        line["cpu_baseline"] = cpu_baseline(system, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
