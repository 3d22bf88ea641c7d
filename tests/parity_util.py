"""Comparison helpers shared by the GPU parity tests (no GPU needed to import).

Particle rows are (id, x, y, z, ux, uy, uz, sx, sy, sz, w) sorted by id, as
returned by pic_particles and the oracle's Sim.particles.
"""

import numpy as np


def particle_errors(got, want, spec, u_floor):
    """Per-particle errors: position in cells (periodic), momentum relative to
    max(|u|, u_floor), spin absolute; each an (N,) array."""
    assert got.shape == want.shape, (got.shape, want.shape)
    np.testing.assert_array_equal(got[:, 0], want[:, 0])
    ndim = spec["ndim"]
    pos = np.zeros(got.shape[0])
    for a in range(ndim):
        L = spec["n"][a] * spec["d"][a]
        dx = np.abs(got[:, 1 + a] - want[:, 1 + a])
        dx = np.minimum(dx, L - dx) / spec["d"][a]
        pos = np.maximum(pos, dx)
    umag = np.max(np.abs(want[:, 4:7]), axis=1)
    mom = np.max(np.abs(got[:, 4:7] - want[:, 4:7]), axis=1) / np.maximum(umag, u_floor)
    spin = np.max(np.abs(got[:, 7:10] - want[:, 7:10]), axis=1)
    return pos, mom, spin


def max_particle_error(got, want, spec, u_floor):
    pos, mom, spin = particle_errors(got, want, spec, u_floor)
    return max(pos.max(initial=0.0), mom.max(initial=0.0), spin.max(initial=0.0))


def field_error(got, want):
    """Max |got - want| over the array divided by max |want| (or 1 if that is 0)."""
    scale = np.max(np.abs(want))
    return np.max(np.abs(got - want)) / (scale if scale > 0 else 1.0)


def thermal_floor(spec, k):
    """Momentum floor for relative errors: the species' thermal spread."""
    T = spec.get("plasma", {}).get("T_keV", 1.0)
    return np.sqrt(T / (spec["species"][k]["mu"] * 510.99895))


def fp32_rounded_state(spec, state):
    """The initial state as the FP32 path stores it: in-cell offsets, momenta,
    spins and weights rounded to float32 (fields unchanged)."""
    parts = []
    for p in state["particles"]:
        q = np.array(p, dtype=np.float64, copy=True)
        for a in range(spec["ndim"]):
            xi = q[:, a] / spec["d"][a]
            fl = np.floor(xi)
            off = (xi - fl).astype(np.float32).astype(np.float64)
            q[:, a] = (fl + off) * spec["d"][a]
        q[:, 3:10] = q[:, 3:10].astype(np.float32).astype(np.float64)
        parts.append(q)
    return {"particles": parts, "fields": state["fields"]}


def per_particle_error(got, want, spec, k):
    pos, mom, spin = particle_errors(got, want, spec, thermal_floor(spec, k))
    return np.maximum(np.maximum(pos, mom), spin)


def storage_bounded(e32, e_ref, bound=1e-5, factor=3.0, quantiles=(50, 99, 100)):
    """FP32 per-particle errors are acceptable at each quantile if they are
    within the bound, or within factor times the error of the exact method
    with float32 particle storage (the oracle with store_fp32), i.e. close to
    what storing particles in float32 costs by itself.  Returns (ok, report)."""
    ok = True
    rep = []
    for q in quantiles:
        a = float(np.percentile(e32, q)) if e32.size else 0.0
        c = float(np.percentile(e_ref, q)) if e_ref.size else 0.0
        lim = max(bound, factor * c)
        ok = ok and a <= lim
        rep.append("q%d fp32 %.2e fp32-storage %.2e limit %.2e" % (q, a, c, lim))
    return ok, "; ".join(rep)
