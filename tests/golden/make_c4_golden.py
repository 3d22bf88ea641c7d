"""Write tests/golden/c4_oracle.json: the FP64 oracle on a sample of the c4
beam (2^20 protons through the analytic wake, 4000 steps).

The sample is 256 particles drawn by index from the full seeded beam.  Stored
per sampled particle: its index, final x, u, s, and by complex step the
derivatives of c . s_i(final), c = (0, 0, 1), with respect to E0, kp and its
own initial x, u, s (the gradient of J = c . P over the whole beam is these
divided by the beam size); and the final states of the oracle run with
float32 state storage, the reference for float32 trajectories.  Calls only ``oracle`` and the input generator
``synth``.

    python tests/golden/make_c4_golden.py
"""

import json
import os
import sys
import warnings

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth   # noqa: E402

NSAMPLE = 256
C = (0.0, 0.0, 1.0)


def main():
    warnings.simplefilter("ignore")
    spec = synth.tracking_preset("c4")
    x, u, s = synth.make_beam(spec)
    idx = np.sort(np.random.default_rng(404).choice(spec["n"], NSAMPLE, replace=False))
    sp = spec["species"]
    args = (spec["E0"], spec["kp"], spec["dt"], spec["nsteps"], sp["Z"], sp["mu"], sp["a"])
    xf, uf, sf = oracle.tracking_forward(x[idx], u[idx], s[idx], *args)
    x32, u32, s32 = oracle.tracking_forward(x[idx], u[idx], s[idx], *args, store_fp32=True)
    dE0, dkp, dx, du, ds = oracle.per_particle_complex_step(x[idx], u[idx], s[idx], *args, C)
    out = {"workload": "c4", "seed": spec["seed"], "script": "tests/golden/make_c4_golden.py",
           "c": list(C), "n": spec["n"], "nsteps": spec["nsteps"], "index": idx.tolist(),
           "x": xf.tolist(), "u": uf.tolist(), "s": sf.tolist(),
           "d_dE0": dE0.tolist(), "d_dkp": dkp.tolist(),
           "d_dx0": dx.tolist(), "d_du0": du.tolist(), "d_ds0": ds.tolist(),
           "store_fp32": {"x": x32.tolist(), "u": u32.tolist(), "s": s32.tolist()}}
    with open(os.path.join(HERE, "c4_oracle.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("sample P_z", float(np.mean(sf[:, 2])), "d_dE0 mean", float(np.mean(dE0)))


if __name__ == "__main__":
    main()
