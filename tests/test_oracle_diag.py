"""Pins of the oracle's move, polarization (section 2 Eq. 4) and energies,
and of the seeded workload generator's statistics (T15)."""

import math

import numpy as np
import pytest

import oracle
import synth
from oracle import pic as O


def test_free_streaming_moves_by_u_over_gamma_and_wraps():
    """With zero fields a particle moves dt*u/gamma per step, periodically."""
    n, d, dt = (10, 6, 1), (0.5, 0.25, 1.0), 0.1
    spec = {"ndim": 2, "n": n, "d": d, "dt": dt,
            "species": [{"Z": -1.0, "mu": 1.0, "a": 0.0}]}
    p = np.zeros((3, 10))
    p[:, 0] = [0.1, 4.9, 2.5]
    p[:, 1] = [0.2, 1.4, 0.01]
    p[:, 3] = [3.0, -0.5, 0.0]
    p[:, 4] = [4.0, 0.0, -20.0]
    p[:, 7] = 1.0
    p[:, 9] = 0.1
    sim = oracle.Sim(spec, {"particles": [p], "fields": np.zeros((6, 1, 6, 10))},
                     test_particle=True)
    sim.step(25)
    gamma = np.sqrt(1 + np.sum(p[:, 3:6] ** 2, axis=1))
    L = np.array([n[0] * d[0], n[1] * d[1]])
    want = np.mod(p[:, 0:2] + 25 * dt * p[:, 3:5] / gamma[:, None], L)
    got = sim.particles(0)[:, 1:3]
    np.testing.assert_allclose(got, want, atol=1e-12)


def _brute_polarization(s_list, u_list, mus, species, emin, emax):
    tot = [0.0, 0.0, 0.0]
    count = 0
    for k, (s, u) in enumerate(zip(s_list, u_list)):
        if species not in (-1, k):
            continue
        for i in range(s.shape[0]):
            gamma = math.sqrt(1.0 + u[i, 0] ** 2 + u[i, 1] ** 2 + u[i, 2] ** 2)
            ek = mus[k] * (gamma - 1.0) * 0.51099895
            if emin <= ek < emax:
                count += 1
                for c in range(3):
                    tot[c] += s[i, c]
    if count == 0:
        return np.zeros(3), 0
    return np.array(tot) / count, count


@pytest.mark.parametrize("species,emin,emax", [
    (-1, -np.inf, np.inf), (0, -np.inf, np.inf), (1, -np.inf, np.inf),
    (0, 0.05, 0.5), (-1, 0.0, 0.2), (1, 0.2, 1.0), (1, 1e9, 2e9)])
def test_polarization_eq4_against_loops(species, emin, emax):
    spec = synth.preset("small2d", n=(24, 16, 1))
    state = synth.make_state(spec)
    sim = oracle.Sim(spec, state)
    sim.step(3)
    rng = np.random.default_rng(0)
    for k in range(2):
        sim.s[k] = rng.normal(0, 1, sim.s[k].shape)
        sim.u[k] = rng.normal(0, 1.0 / (1 + 40 * k), sim.u[k].shape)
    P, N = sim.polarization(species, emin, emax)
    if np.isfinite(emax) and emax < 1e3:
        assert 0 < N < sum(s.shape[0] for s in sim.s)
    Pb, Nb = _brute_polarization(sim.s, sim.u, [1.0, synth.MP_OVER_ME], species, emin, emax)
    assert N == Nb
    np.testing.assert_allclose(P, Pb, rtol=1e-12, atol=1e-15)


def test_polarization_at_start_equals_s0():
    spec = synth.preset("small2d")
    sim = oracle.Sim(spec, synth.make_state(spec))
    P, N = sim.polarization()
    assert N == sum(p.shape[0] for p in sim.xi)
    np.testing.assert_array_equal(P, np.array(spec["plasma"]["s0"], dtype=float))


def test_energy_field_sum_and_kinetic_by_hand():
    spec = {"ndim": 2, "n": (4, 3, 1), "d": (0.5, 0.25, 1.0), "dt": 0.1,
            "species": [{"Z": -1.0, "mu": 1.0, "a": 0.0}, {"Z": 1.0, "mu": 4.0, "a": 0.0}]}
    F = np.zeros((6, 1, 3, 4))
    F[1, 0, 1, 2] = 2.0
    F[5, 0, 0, 0] = -1.0
    p = np.zeros((1, 10))
    p[0, 3:6] = [0.0, 0.75, 0.0]   # gamma = 1.25
    p[0, 9] = 0.5
    sim = oracle.Sim(spec, {"particles": [p, p.copy()], "fields": F})
    e = sim.energy()
    V = 0.5 * 0.25
    assert e[0] == pytest.approx(1.0 * 0.25 * 0.5 * V, rel=1e-14)
    assert e[1] == pytest.approx(4.0 * 0.25 * 0.5 * V, rel=1e-14)
    assert e[2] == pytest.approx(0.5 * (4.0 + 1.0) * V, rel=1e-14)
    assert e[3] == 0.0


@pytest.mark.parametrize("name", ["small2d", "small3d"])
def test_T15_loader_statistics(name):
    spec = synth.preset(name)
    parts = synth.make_particles(spec)
    nx, ny, nz = spec["n"]
    ndim = spec["ndim"]
    ppc = spec["plasma"]["ppc"]
    ncell = nx * ny * (nz if ndim == 3 else 1)
    e, p = parts
    # exact ppc per cell, co-located species, exact spins
    cell = np.floor(e[:, 0] / spec["d"][0]).astype(int) + nx * np.floor(e[:, 1] / spec["d"][1]).astype(int)
    if ndim == 3:
        cell += nx * ny * np.floor(e[:, 2] / spec["d"][2]).astype(int)
    assert np.all(np.bincount(cell, minlength=ncell) == ppc)
    np.testing.assert_array_equal(e[:, 0:3], p[:, 0:3])
    np.testing.assert_array_equal(e[:, 9], p[:, 9])
    for arr in parts:
        np.testing.assert_array_equal(arr[:, 6:9], np.broadcast_to(spec["plasma"]["s0"], (arr.shape[0], 3)))
    # Maxwellian moments within 5 sigma of their sampling error
    for arr, sp in zip(parts, spec["species"]):
        sigma = math.sqrt(spec["plasma"]["T_keV"] / (sp["mu"] * synth.ME_C2_MEV * 1e3))
        n = arr.shape[0]
        for c in range(3):
            u = arr[:, 3 + c]
            assert abs(u.mean()) < 5 * sigma / math.sqrt(n)
            assert abs(u.var() / sigma ** 2 - 1) < 5 * math.sqrt(2.0 / n)
    # zero initial charge density on the grid
    sim = oracle.Sim(spec, {"particles": parts, "fields": synth.make_laser_fields(spec)})
    assert np.max(np.abs(sim.rho())) < 1e-15


def test_T15_c2_ramp_weights():
    spec = synth.preset("c2", n=(512, 8, 1))
    e, _ = synth.make_particles(spec)
    ramp = spec["plasma"]["ramp_len"]
    want = 0.02 * np.minimum(e[:, 0] / ramp, 1.0) / 8
    np.testing.assert_allclose(e[:, 9], want, rtol=1e-15)


def test_laser_peak_and_polarization():
    spec = synth.preset("c1")
    F = synth.make_laser_fields(spec)
    assert np.max(np.abs(F[1])) == pytest.approx(3.0, rel=1e-3)
    assert np.max(np.abs(F[2])) == 0.0
    spec3 = synth.preset("small3d")
    F3 = synth.make_laser_fields(spec3)
    amp = np.sqrt(F3[1] ** 2 + F3[2] ** 2)
    assert np.max(amp) <= 3.0 + 1e-12
    assert np.max(np.abs(F3[4])) > 0.5


def test_store_fp32_rounds_the_stored_state_only():
    """With store_fp32 the stored offsets, momenta and spins are float32 values
    after every step; with it off, the same run keeps float64 values."""
    spec = synth.preset("small2d", n=(24, 16, 1))
    state = synth.make_state(spec)
    a = oracle.Sim(spec, state, store_fp32=True)
    b = oracle.Sim(spec, state)
    a.step(2)
    b.step(2)
    for k in range(2):
        for arr in (a.u[k], a.s[k], a.w[k], a.xi[k][:, :2] - np.floor(a.xi[k][:, :2])):
            np.testing.assert_array_equal(arr, arr.astype(np.float32).astype(np.float64))
        assert np.any(b.u[k] != b.u[k].astype(np.float32).astype(np.float64))
        # the rounding is a perturbation at float32 resolution, not a change of method
        assert np.max(np.abs(a.u[k] - b.u[k])) < 1e-5


def test_store_fp32_cell_edge_tie_rule():
    """The cell-edge reading for float32 offsets: cell = floor(x / dx) with the
    offset in [0, 1); an offset that rounds up to 1 in float32 moves the
    particle to the next cell (wrapping at the box edge) with offset 0.
    Expected cells and offsets below are worked out by hand from the float32
    neighbours of 1 (1 - 2^-24 and 1) and of 0."""
    n = (32, 8, 1)
    d = (0.3, 0.3, 1.0)
    dt = 0.2
    spec = {"ndim": 2, "n": n, "d": d, "dt": dt, "species": [{"Z": -1.0, "mu": 1.0, "a": 0.0}]}
    ulp = 2.0 ** -24            # spacing of float32 values just below 1
    top = 1.0 - ulp             # largest float32 offset below 1
    # (start cell, start offset, displacement in cells) -> (end cell, end offset)
    cases = [
        (31, top, 0.75 * ulp, 0, 0.0),        # rounds up to 1 at the last cell: wraps to cell 0
        (31, top, 0.25 * ulp, 31, top),       # rounds back to the top offset
        (15, top, 0.75 * ulp, 16, 0.0),       # next cell (another 16-cell tile)
        (0, 0.0, -0.25 * ulp, 0, 0.0),        # 1 - ulp/4 rounds to 1: stays at the edge of cell 0
        (0, 0.0, -0.75 * ulp, 31, top),       # 1 - 3 ulp/4 rounds to 1 - ulp: previous cell (wrapped)
        (16, 0.0, -0.75 * ulp, 15, top),
        (7, top, 0.0, 7, top),                # at rest
    ]
    rows = []
    for c, o, disp, _, _ in cases:
        v = disp * d[0] / dt
        u = v / np.sqrt(1.0 - v * v)
        rows.append([(c + o) * d[0], 2.5 * d[1], 0.0, u, 0.0, 0.0, 0.0, 1.0, 0.0, 0.01])
    state = {"particles": [np.array(rows)], "fields": np.zeros((6, 1, n[1], n[0]))}
    sim = oracle.Sim(spec, state, test_particle=True, store_fp32=True)
    sim.step(1)
    xi = sim.xi[0][:, 0]
    for q, (_, _, _, c1, o1) in enumerate(cases):
        assert xi[q] == c1 + o1, (q, xi[q], c1 + o1)
        assert 0.0 <= xi[q] < n[0]
