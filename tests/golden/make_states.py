"""Writes the equilibrated starting states kept under tests/golden/.

Each state is the seeded synthetic workload integrated by the oracle's own
FP64 integrator (oracle/, nothing else): the parity tests compare the HIP
path with the oracle on it at full size, and the benchmark times the HIP
path from it, so that both see contacts rather than the contact-free start
of a lattice.  The states' SHA-256 digests go to states.json, which the
loader in paper_1607_02427_amd/inputs.py checks.

    python tests/golden/make_states.py [cubes]

cubes: the 4096 rounded cubes (edge 1, r 0.15) at volume fraction 0.4, NVT
kT = 1, dt = 5e-4, from their seeded 16^3 lattice start (inputs.cubes_3d),
1000 steps (0.5 tau), thermostat variables included.

octahedra: 4096 rounded octahedra (edge 1, r 0.1) with uniform random
orientations on a BCC lattice at volume fraction 0.25 (inputs.octahedra_bcc_dilute,
where no two can touch whatever their orientations), compressed to 0.55 by
affine rescaling of the box and the positions, by 0.25% in length after
every 50 NVT steps (kT = 1, dt = 2e-4, thermostat time constant 0.05 so that
the work of compression is drawn off as it is done), then 1000 NVT steps at
0.55 with the workload's time constant 0.5.  The
262,144-octahedra workload tiles this cell 4 x 4 x 4.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1607_02427_amd import inputs as I  # noqa: E402


def sha256(path):
    h = hashlib.sha256()
    with open(path, "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def save(name, s, thermo, step, log, meta):
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, x=s.x, q=s.q, v=s.v, L=s.L, image=s.image, box=np.asarray(s.box, np.float64),
                        thermo=np.asarray(thermo, np.float64), step=np.int64(step), log=np.asarray(log, np.float64))
    index_path = os.path.join(HERE, "states.json")
    index = json.load(open(index_path)) if os.path.exists(index_path) else {}
    index[name] = dict(file=name + ".npz", sha256=sha256(path), **meta)
    with open(index_path, "w") as f:
        json.dump(index, f, indent=1, sort_keys=True)
        f.write("\n")
    print(f"wrote {path} ({os.path.getsize(path)} bytes)", flush=True)


def cubes(steps=1000):
    O.set_threads(len(os.sched_getaffinity(0)))
    s = I.cubes_3d()
    t0 = time.perf_counter()
    end, thermo, log, _ = O.run(s, steps)
    el = time.perf_counter() - t0
    st = O.forces(end)["stats"]
    meta = dict(workload="4096 rounded cubes, volume fraction 0.4, NVT kT 1, dt 5e-4, seeded 16^3 lattice start",
                steps=steps, oracle_seconds=round(el, 1), pairs_within_bound=st["pairs"] // 2,
                feature_pairs_in_cutoff=st["feature_in"] // 2)
    print(meta, flush=True)
    save("cubes4096_nvt_step1000", end, thermo, steps, log[:, :6], meta)


def octahedra(target=0.55, every=50, factor=0.9975, settle=1000, tau_compress=0.05):
    O.set_threads(len(os.sched_getaffinity(0)))
    s = I.octahedra_bcc_dilute()
    tau_T = s.tau_T
    s.tau_T = tau_compress
    vol = s.shapes[0].volume * s.n
    thermo = np.zeros(2)
    t0 = time.perf_counter()
    steps = 0
    logs = []
    while True:
        phi = vol / float(np.prod(s.box))
        if phi >= target:
            break
        # one rescale: by `factor` in length, the last one exactly onto the target
        f = max(factor, (phi / target) ** (1.0 / 3.0))
        s.box = s.box * f
        s.x = s.x * f
        s, thermo, log, _ = O.run(s, every, thermo=thermo)
        steps += every
        logs.append(log[-1])
        if steps % 1000 == 0:
            print(f"step {steps} phi {vol / float(np.prod(s.box)):.4f} U {log[-1, 0]:.1f} "
                  f"K {log[-1, 1] + log[-1, 2]:.1f} {time.perf_counter() - t0:.0f} s", flush=True)
    s.tau_T = tau_T
    s, thermo, log, _ = O.run(s, settle, thermo=thermo)
    steps += settle
    logs.extend(log)
    el = time.perf_counter() - t0
    st = O.forces(s)["stats"]
    meta = dict(workload="4096 rounded octahedra, random orientations, BCC at volume fraction 0.25 compressed to "
                         "0.55 (0.25% in length per 50 NVT steps, kT 1, dt 2e-4, tau_T 0.05), then 1000 NVT steps "
                         "(tau_T 0.5)",
                steps=steps, volume_fraction=vol / float(np.prod(s.box)), oracle_seconds=round(el, 1),
                pairs_within_bound=st["pairs"] // 2, feature_pairs_in_cutoff=st["feature_in"] // 2)
    print(meta, flush=True)
    save("octahedra4096_compressed", s, thermo, steps, np.asarray(logs), meta)


if __name__ == "__main__":
    which = sys.argv[1:] or ["cubes", "octahedra"]
    for w in which:
        {"cubes": cubes, "octahedra": octahedra}[w]()
