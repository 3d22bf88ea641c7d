"""Write tests/golden/c1_oracle.json: the FP64 oracle's c1 run, sampled.

c1 is the 2D3V workload of 256x128 cells (0.05 wavelengths), electrons and
protons at 4 per cell each, 1 keV, linearly polarized a0=3 pulse, spins +y,
dt = 0.95 of the Courant limit, run for 200 steps.  This script calls only
``oracle`` and the seeded input generator ``synth``.  Stored per snapshot
(steps 100 and 200): polarization (all species and per species), energies,
256 particles per species (192 drawn at random plus the 64 with the largest
|u|, the ones most sensitive to rounding) and 256 random field values.  Also
stored: the polarization of all species after every step (P_t, N_t: Eq. 4
over the whole ensemble, steps 1 .. 200).  Also
stored, at step 100: the same particles from the oracle run with float32
particle storage (state rounded to float32 after every step), which bounds
what any float32 particle store must deviate from the float64 run.

    python tests/golden/make_c1_golden.py [--full-dump path.npz]
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth   # noqa: E402

SNAPSHOTS = (100, 200)


def main():
    full = None
    if "--full-dump" in sys.argv:
        full = sys.argv[sys.argv.index("--full-dump") + 1]
    spec = synth.preset("c1")
    state = synth.make_state(spec)
    sim = oracle.Sim(spec, state)
    rng = np.random.default_rng(2024)
    out = {"workload": "c1", "seed": spec["seed"], "script": "tests/golden/make_c1_golden.py",
           "snapshots": {}}
    dumps = {}
    step = 0
    P_t, N_t = [], []
    for target in SNAPSHOTS:
        while step < target:
            sim.step(1)
            step += 1
            P, N = sim.polarization()
            P_t.append([float(v) for v in P])
            N_t.append(int(N))
        snap = {"P_all": list(sim.polarization()[0]), "N_all": sim.polarization()[1],
                "P_species": [list(sim.polarization(k)[0]) for k in range(2)],
                "energy": list(sim.energy()), "particles": {}}
        for k in range(2):
            rows = sim.particles(k)
            umag = np.max(np.abs(rows[:, 4:7]), axis=1)
            fast = np.argsort(umag)[-64:]
            rest = np.setdiff1d(np.arange(rows.shape[0]), fast)
            ids = np.sort(np.concatenate([fast, rng.choice(rest, 192, replace=False)]))
            snap["particles"][str(k)] = {"ids": ids.tolist(), "rows": rows[ids].tolist()}
            dumps["p%d_%d" % (k, target)] = rows
        F = sim.fields()
        cells = np.stack([rng.integers(0, 9, 256), np.zeros(256, dtype=int),
                          rng.integers(0, F.shape[2], 256), rng.integers(0, F.shape[3], 256)], axis=1)
        snap["field_cells"] = cells.tolist()
        snap["field_values"] = [float(F[c, z, y, x]) for c, z, y, x in cells]
        dumps["F_%d" % target] = F
        out["snapshots"][str(target)] = snap
        print("step", target, "P", snap["P_all"], "energy", snap["energy"], flush=True)
    out["P_t"] = P_t
    out["N_t"] = N_t
    sim32 = oracle.Sim(spec, state, store_fp32=True)
    sim32.step(100)
    out["store_fp32"] = {"100": {}}
    for k in range(2):
        ids = out["snapshots"]["100"]["particles"][str(k)]["ids"]
        out["store_fp32"]["100"][str(k)] = sim32.particles(k)[ids].tolist()
    P32, _ = sim32.polarization()
    out["store_fp32"]["P_100"] = list(P32)
    print("store_fp32 step 100 P", list(P32), flush=True)
    with open(os.path.join(HERE, "c1_oracle.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
    if full:
        np.savez_compressed(full, **dumps)


if __name__ == "__main__":
    main()
