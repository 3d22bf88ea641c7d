"""Workload recipes: plasma loading and the laser initial condition.

Units are normalized laser units: time in 1/omega0, length in c/omega0 (one
wavelength is 2*pi), momentum u = gamma*beta of each species, fields in
m_e*c*omega0/e and densities in the critical density n_c.  The paper's runs
(section 2: a circularly polarized pulse into a near-critical gas, all
protons spin-aligned along y, two macro-particles per species per cell) are
not reproducible here, so these seeded synthetic plasmas of the same
structure stand in for them:

* ``c1``: 2D 256x128 cells of 0.05 wavelengths, uniform e/p plasma at
  0.01 n_c, 4 per cell per species, 1 keV, linearly polarized a0=3 pulse with
  a 4-wavelength waist and 10-wavelength duration, spins +y, FP64.
* ``c2``: 2D 4096x1024, 8 per cell per species, density ramp 0 -> 0.02 n_c over
  50 wavelengths then flat, a0=10, waist 8, duration 15, spins +y.
* ``c3``: 3D 512x256x256 cells of 0.1 wavelengths, 2 per cell per species,
  0.005 n_c with a 1 % per-cell density noise, circular a0=20, waist 6,
  duration 10, spins +x.

Every random draw comes from a numpy PCG64 stream seeded by the recipe.
"""

import math

import numpy as np

LAMBDA = 2.0 * math.pi          # one laser wavelength in c/omega0
ME_C2_MEV = 0.51099895          # electron rest energy
ME_C2_KEV = ME_C2_MEV * 1e3
MP_OVER_ME = 1836.15267343      # proton/electron mass ratio
A_E = 0.00116                   # electron anomaly used by the workloads
A_P = 1.793                     # proton anomaly used by the workloads

PARTICLE_COLUMNS = ("x", "y", "z", "ux", "uy", "uz", "sx", "sy", "sz", "w")


def electron():
    return {"name": "e", "Z": -1.0, "mu": 1.0, "a": A_E}


def proton():
    return {"name": "p", "Z": 1.0, "mu": MP_OVER_ME, "a": A_P}


def courant_dt(d, ndim, courant=0.95):
    """Time step as a fraction of the Yee stability limit (c = 1)."""
    return courant / math.sqrt(sum(1.0 / (d[i] * d[i]) for i in range(ndim)))


def grid_shape(spec):
    """Array shape of one field component, (nz, ny, nx); nz = 1 in 2D."""
    nx, ny, nz = spec["n"]
    return (nz, ny, nx)


def _base(name, ndim, n, d_lambda, steps, seed, precision, tile):
    d = tuple(float(v) * LAMBDA for v in d_lambda)
    n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
    d = d + (d[0],) * (3 - len(d))
    return {
        "name": name, "ndim": ndim, "n": n, "d": d,
        "dt": courant_dt(d, ndim), "steps": steps, "seed": seed,
        "precision": precision, "tile": tile,
        "species": [electron(), proton()],
    }


def _c1(**kw):
    s = _base("c1", 2, (256, 128), (0.05, 0.05), 200, 1, "fp64", (16, 16, 1))
    s["plasma"] = {"ppc": 4, "profile": "uniform", "n0": 0.01, "ramp_len": 0.0,
                   "noise": 0.0, "T_keV": 1.0, "s0": (0.0, 1.0, 0.0)}
    s["laser"] = {"a0": 3.0, "waist": 4 * LAMBDA, "duration": 10 * LAMBDA,
                  "x_center": 0.5 * 256 * s["d"][0], "pol": "lp"}
    s.update(kw)
    return s


def _c2(**kw):
    s = _base("c2", 2, (4096, 1024), (0.05, 0.05), 1000, 2, "fp32", (16, 16, 1))
    s["plasma"] = {"ppc": 8, "profile": "ramp", "n0": 0.02, "ramp_len": 50 * LAMBDA,
                   "noise": 0.0, "T_keV": 1.0, "s0": (0.0, 1.0, 0.0)}
    s["laser"] = {"a0": 10.0, "waist": 8 * LAMBDA, "duration": 15 * LAMBDA,
                  "x_center": 15 * LAMBDA, "pol": "lp"}
    s.update(kw)
    return s


def _c3(**kw):
    s = _base("c3", 3, (512, 256, 256), (0.1, 0.1, 0.1), 500, 3, "fp32", (0, 0, 0))
    s["plasma"] = {"ppc": 2, "profile": "uniform", "n0": 0.005, "ramp_len": 0.0,
                   "noise": 0.01, "T_keV": 1.0, "s0": (1.0, 0.0, 0.0)}
    s["laser"] = {"a0": 20.0, "waist": 6 * LAMBDA, "duration": 10 * LAMBDA,
                  "x_center": 10 * LAMBDA, "pol": "cp"}
    s.update(kw)
    return s


def _small2d(**kw):
    """A c1-like plasma on a 72x40 grid: several 16x16 tiles and ragged last tiles."""
    s = _base("small2d", 2, (72, 40), (0.05, 0.05), 40, 11, "fp64", (16, 16, 1))
    s["plasma"] = {"ppc": 3, "profile": "ramp", "n0": 0.05, "ramp_len": 2 * LAMBDA,
                   "noise": 0.02, "T_keV": 5.0, "s0": (0.0, 1.0, 0.0)}
    s["laser"] = {"a0": 3.0, "waist": 1.0 * LAMBDA, "duration": 1.5 * LAMBDA,
                  "x_center": 1.8 * LAMBDA, "pol": "lp"}
    s.update(kw)
    return s


def _small3d(**kw):
    s = _base("small3d", 3, (20, 12, 10), (0.1, 0.1, 0.1), 20, 12, "fp64", (0, 0, 0))
    s["plasma"] = {"ppc": 2, "profile": "uniform", "n0": 0.05, "ramp_len": 0.0,
                   "noise": 0.02, "T_keV": 5.0, "s0": (1.0, 0.0, 0.0)}
    s["laser"] = {"a0": 3.0, "waist": 0.4 * LAMBDA, "duration": 0.8 * LAMBDA,
                  "x_center": 1.0 * LAMBDA, "pol": "cp"}
    s.update(kw)
    return s


PRESETS = {"c1": _c1, "c2": _c2, "c3": _c3, "small2d": _small2d, "small3d": _small3d}


def preset(name, **overrides):
    """A workload recipe by name; keyword arguments replace top-level keys."""
    return PRESETS[name](**overrides)


def _density_weight(spec, x_first):
    p = spec["plasma"]
    ppc = p["ppc"]
    if p["profile"] == "uniform":
        return np.full(x_first.shape, p["n0"] / ppc)
    if p["profile"] == "ramp":
        ramp = np.minimum(x_first / p["ramp_len"], 1.0) if p["ramp_len"] > 0 else 1.0
        return p["n0"] * ramp / ppc
    raise ValueError("unknown density profile %r" % p["profile"])


def make_particles(spec, seed=None):
    """Plasma particles, one float64 array of shape (N, 10) per species.

    Columns are x, y, z, ux, uy, uz, sx, sy, sz, w.  Every cell holds ``ppc``
    particles of each species at uniform random positions inside the cell;
    electrons and protons share positions and weights, so the initial charge
    density is exactly zero.  Momenta are drawn from a non-relativistic
    Maxwellian of temperature T_keV; spins all equal s0; the weight is the
    local density over ppc, times a per-cell noise factor when requested.
    In 2D the z column is 0.
    """
    rng = np.random.Generator(np.random.PCG64(spec["seed"] if seed is None else seed))
    ndim = spec["ndim"]
    nx, ny, nz = spec["n"]
    dx, dy, dz = spec["d"]
    p = spec["plasma"]
    ppc = p["ppc"]
    ncell = nx * ny * (nz if ndim == 3 else 1)
    npart = ncell * ppc
    cell = np.repeat(np.arange(ncell, dtype=np.int64), ppc)
    pos = np.empty((npart, 3))
    pos[:, 0] = (cell % nx + rng.random(npart)) * dx
    pos[:, 1] = ((cell // nx) % ny + rng.random(npart)) * dy
    if ndim == 3:
        pos[:, 2] = (cell // (nx * ny) + rng.random(npart)) * dz
    else:
        pos[:, 2] = 0.0
    w = _density_weight(spec, pos[:, 0])
    if p["noise"] > 0:
        factor = 1.0 + p["noise"] * rng.standard_normal(ncell)
        w = w * factor[cell]
    del cell
    out = []
    for sp in spec["species"]:
        arr = np.empty((npart, 10))
        arr[:, 0:3] = pos
        sigma = math.sqrt(p["T_keV"] / (sp["mu"] * ME_C2_KEV))
        arr[:, 3:6] = sigma * rng.standard_normal((npart, 3))
        arr[:, 6:9] = np.asarray(p["s0"], dtype=np.float64)
        arr[:, 9] = w
        out.append(arr)
    return out


def _envelope(spec, x, y, z):
    las = spec["laser"]
    ndim = spec["ndim"]
    nx, ny, nz = spec["n"]
    dx, dy, dz = spec["d"]
    xi = x - las["x_center"]
    r2 = (y - 0.5 * ny * dy) ** 2
    if ndim == 3:
        r2 = r2 + (z - 0.5 * nz * dz) ** 2
    length = las["duration"]
    g = np.exp(-2.0 * math.log(2.0) * xi * xi / (length * length))
    f = np.exp(-r2 / (las["waist"] ** 2))
    return las["a0"] * g * f, xi


def make_laser_fields(spec):
    """Initial E and B of the pulse, shape (6, nz, ny, nx): Ex Ey Ez Bx By Bz.

    The pulse travels along +x, focused, without wavefront curvature or a
    longitudinal field.  Its transverse field is a0*g*f*cos(x - xc) along y
    (plus a0*g*f*sin(x - xc) along z when circular), with g a Gaussian of
    intensity FWHM equal to the duration and f = exp(-r^2/waist^2); B is x-hat
    cross E.  Each component is evaluated at its own staggered Yee position.
    """
    ndim = spec["ndim"]
    nx, ny, nz = spec["n"]
    dx, dy, dz = spec["d"]
    shape = grid_shape(spec)
    F = np.zeros((6,) + shape)
    las = spec.get("laser")
    if not las or las["a0"] == 0.0:
        return F
    k = np.arange(shape[0], dtype=np.float64)[:, None, None]
    j = np.arange(ny, dtype=np.float64)[None, :, None]
    i = np.arange(nx, dtype=np.float64)[None, None, :]
    def at(sx, sy, sz):
        return (i + sx) * dx, (j + sy) * dy, (k + (sz if ndim == 3 else 0.0)) * dz

    cp = las["pol"] == "cp"
    # E_y at (i, j+1/2, k); B_z at (i+1/2, j+1/2, k)
    amp, xi = _envelope(spec, *at(0.0, 0.5, 0.0))
    F[1] = amp * np.cos(xi)
    amp, xi = _envelope(spec, *at(0.5, 0.5, 0.0))
    F[5] = amp * np.cos(xi)
    if cp:
        # E_z at (i, j, k+1/2); B_y at (i+1/2, j, k+1/2)
        amp, xi = _envelope(spec, *at(0.0, 0.0, 0.5))
        F[2] = amp * np.sin(xi)
        amp, xi = _envelope(spec, *at(0.5, 0.0, 0.5))
        F[4] = -amp * np.sin(xi)
    return F


def make_static_fields(spec, uniform_amp, smooth_amp, kmax=1, nmodes=6, seed=0):
    """Static E and B for test-particle runs, shape (6, nz, ny, nx).

    Each component is a random constant, uniform in [-uniform_amp,
    uniform_amp], plus a smooth random part: nmodes plane waves with random
    amplitude and phase whose wave numbers are whole multiples (at most
    kmax) of the box's fundamental along each axis, scaled so that the part's
    largest value on the grid is smooth_amp.  Either amplitude may be a pair
    (for E, for B).  The values are taken at the grid indices (the field is
    smooth, so the staggering does not matter)."""
    def pair(v):
        return (float(v[0]), float(v[1])) if isinstance(v, (tuple, list)) else (float(v), float(v))
    uni, smo = pair(uniform_amp), pair(smooth_amp)
    rng = np.random.default_rng(seed)
    shape = grid_shape(spec)
    nx, ny, nz = spec["n"]
    dx, dy, dz = spec["d"]
    x = (np.arange(nx) * dx)[None, None, :]
    y = (np.arange(ny) * dy)[None, :, None]
    z = (np.arange(shape[0]) * dz)[:, None, None]
    L = (nx * dx, ny * dy, shape[0] * dz)
    F = np.zeros((6,) + shape)
    for c in range(6):
        part = np.zeros(shape)
        for _ in range(nmodes):
            kv = [2.0 * math.pi / L[a] * rng.integers(-kmax, kmax + 1) for a in range(3)]
            if spec["ndim"] == 2:
                kv[2] = 0.0
            phase = rng.uniform(0.0, 2.0 * math.pi)
            part = part + rng.normal() * np.cos(kv[0] * x + kv[1] * y + kv[2] * z + phase)
        peak = np.max(np.abs(part))
        if smo[c // 3] > 0.0 and peak > 0.0:
            F[c] += part * (smo[c // 3] / peak)
        F[c] += uni[c // 3] * rng.uniform(-1.0, 1.0)
    return F


def make_state(spec, with_particles=True):
    """Everything the simulation starts from: particles per species and fields."""
    return {
        "particles": make_particles(spec) if with_particles else [
            np.zeros((0, 10)) for _ in spec["species"]],
        "fields": make_laser_fields(spec),
    }


# ---------------------------------------------------------------- test-particle beams

MICRON = LAMBDA / 0.8   # one micrometre in c/omega0 for a 0.8 um laser wavelength


def tracking_preset(name="c4", **overrides):
    """Beam and wake of the differentiable tracking workloads.

    ``c4``: 2^20 protons through a linear wake with E0 = 0.1 m_e c omega0 / e and
    kp = 0.1 omega0 / c (n = 0.01 n_c), dt = 0.5 / omega0, 4000 steps, states kept
    every 100 steps.  gamma ~ N(20, 2) along z, x and y ~ N(0, 1 um), z uniform
    over one plasma wavelength, spins +z.  ``track_small``: 64 of them for 300
    steps, kept every 40 (so the last segment is short)."""
    s = {"name": "c4", "n": 1 << 20, "seed": 4, "E0": 0.1, "kp": 0.1, "dt": 0.5, "nsteps": 4000,
         "checkpoint": 100, "gamma_mean": 20.0, "gamma_std": 2.0, "sigma_r": MICRON,
         "species": proton(), "s0": (0.0, 0.0, 1.0), "precision": "fp32"}
    if name == "track_small":
        s.update({"name": "track_small", "n": 64, "seed": 44, "nsteps": 300, "checkpoint": 40,
                  "precision": "fp64"})
    elif name != "c4":
        raise KeyError(name)
    s.update(overrides)
    return s


def make_beam(spec):
    """x0, u0, s0, each (n, 3), of a tracking workload."""
    rng = np.random.default_rng(spec["seed"])
    n = int(spec["n"])
    x = np.empty((n, 3))
    x[:, 0] = rng.normal(0.0, spec["sigma_r"], n)
    x[:, 1] = rng.normal(0.0, spec["sigma_r"], n)
    x[:, 2] = rng.uniform(0.0, 2.0 * math.pi / spec["kp"], n)
    gamma = np.maximum(rng.normal(spec["gamma_mean"], spec["gamma_std"], n), 1.01)
    u = np.zeros((n, 3))
    u[:, 2] = np.sqrt(gamma * gamma - 1.0)
    s = np.tile(np.asarray(spec["s0"], dtype=np.float64), (n, 1))
    return x, u, s


# ---------------------------------------------------------------- batches of runs

def batch_specs(name="c5", **overrides):
    """Recipes of a batch of independent 2D runs.

    ``c5``: 64 runs, grids drawn uniformly from 128-1024 x 64-256 cells of
    0.05 wavelengths, density log-uniform in 0.001-0.05 n_c (uniform in each
    run), 2-8 particles per cell per species, linearly polarized a0 uniform in
    1-10 with a waist of a quarter of the box height and a 10-wavelength
    duration, centred a quarter into the box; 1 keV, spins +y, FP32, 300 steps.
    ``batch_small``: five small runs of uneven size for parity tests (FP64)."""
    seed = overrides.pop("seed", 5 if name == "c5" else 55)
    rng = np.random.default_rng(seed)
    specs = []
    if name == "c5":
        nrun = overrides.pop("nrun", 64)
        for r in range(nrun):
            nx = int(rng.integers(128, 1025))
            ny = int(rng.integers(64, 257))
            n0 = float(np.exp(rng.uniform(np.log(0.001), np.log(0.05))))
            ppc = int(rng.integers(2, 9))
            a0 = float(rng.uniform(1.0, 10.0))
            specs.append(_batch_run("c5_%02d" % r, nx, ny, n0, ppc, a0, 1000 + r, "fp32"))
    elif name == "batch_small":
        shapes = [(48, 32, 2), (80, 40, 3), (64, 24, 1), (96, 48, 2), (32, 32, 4)]
        for r, (nx, ny, ppc) in enumerate(shapes):
            specs.append(_batch_run("small_%d" % r, nx, ny, 0.05, ppc, 2.0 + r, 2000 + r, "fp64",
                                    T_keV=5.0, steps=20))
    else:
        raise KeyError(name)
    for s in specs:
        s.update(overrides)
    return specs


def _batch_run(name, nx, ny, n0, ppc, a0, seed, precision, T_keV=1.0, steps=300):
    s = _base(name, 2, (nx, ny), (0.05, 0.05), steps, seed, precision, (0, 0, 1))
    s["plasma"] = {"ppc": ppc, "profile": "uniform", "n0": n0, "ramp_len": 0.0,
                   "noise": 0.0, "T_keV": T_keV, "s0": (0.0, 1.0, 0.0)}
    Ly = ny * s["d"][1]
    Lx = nx * s["d"][0]
    s["laser"] = {"a0": a0, "waist": 0.25 * Ly, "duration": 10 * LAMBDA,
                  "x_center": 0.25 * Lx, "pol": "lp"}
    return s
