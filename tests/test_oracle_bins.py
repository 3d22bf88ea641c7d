"""Pins of the oracle's binned diagnostics: brute-force loops over every
particle, conservation of counts and weights, and the per-bin polarization
of section 2 Eq. 4 against the oracle's windowed polarization (a separate
code path: the Eq. 4 mean over particles selected by a kinetic-energy
window)."""

import math

import numpy as np

import oracle
import synth


def _rand_particles(rng, n, umax=3.0):
    u = rng.normal(0.0, umax / 3.0, (n, 3))
    s = rng.normal(0.0, 1.0, (n, 3))
    s /= np.linalg.norm(s, axis=1)[:, None]
    w = rng.uniform(0.5, 2.0, n)
    return u, s, w


def test_spectrum_against_loops():
    rng = np.random.default_rng(11)
    u, s, w = _rand_particles(rng, 400)
    mu, emin, emax, nb = 1.0, 0.05, 0.9, 7
    count, weight, spin = oracle.spectrum(u, s, w, mu, emin, emax, nb)
    c2 = np.zeros(nb)
    w2 = np.zeros(nb)
    s2 = np.zeros((nb, 3))
    width = (emax - emin) / nb
    for i in range(u.shape[0]):
        g = math.sqrt(1.0 + float(u[i] @ u[i]))
        e = mu * (g - 1.0) * 0.51099895
        if not (emin <= e < emax):
            continue
        b = min(int((e - emin) // width), nb - 1)
        c2[b] += 1
        w2[b] += w[i]
        s2[b] += s[i]
    np.testing.assert_array_equal(count, c2)
    np.testing.assert_allclose(weight, w2, rtol=1e-13)
    np.testing.assert_allclose(spin, s2, rtol=1e-12, atol=1e-13)


def test_spectrum_conserves_count_and_weight():
    rng = np.random.default_rng(12)
    u, s, w = _rand_particles(rng, 1000)
    e = oracle.kinetic_energy_binned(u, 1.0)
    lo, hi = float(e.min()), float(e.max()) * 1.0001
    count, weight, spin = oracle.spectrum(u, s, w, 1.0, lo, hi, 33)
    assert count.sum() == 1000
    assert weight.sum() == np.float64(w.sum()) or abs(weight.sum() - w.sum()) < 1e-10
    np.testing.assert_allclose(spin.sum(axis=0), s.sum(axis=0), atol=1e-10)


def test_per_bin_polarization_equals_windowed_eq4():
    spec = synth.preset("small2d")
    state = synth.make_state(spec)
    sim = oracle.Sim(spec, state)
    sim.step(6)
    emin, emax, nb = 0.0, 0.02, 5
    count, weight, spin = sim.spectrum(0, emin, emax, nb)
    edges = np.linspace(emin, emax, nb + 1)
    for b in range(nb):
        # interior of the bin, away from the edges where rounding could differ
        lo = edges[b] + 1e-12
        hi = edges[b + 1] - 1e-12
        P, N = sim.polarization(0, lo, hi)
        if N == 0:
            continue
        assert abs(N - count[b]) <= 2
        if N == count[b]:
            np.testing.assert_allclose(spin[b] / count[b], P, rtol=1e-12, atol=1e-14)
        else:
            np.testing.assert_allclose(spin[b] / count[b], P, atol=4.0 / N)


def test_phase_space_against_loops_and_total_weight():
    rng = np.random.default_rng(13)
    n = 300
    x = rng.uniform(-1.0, 11.0, n)
    p = rng.normal(0.0, 2.0, n)
    w = rng.uniform(0.1, 1.0, n)
    H = oracle.phase_space(x, p, w, 0.0, 10.0, 5, -3.0, 3.0, 4)
    H2 = np.zeros((5, 4))
    for i in range(n):
        if 0.0 <= x[i] < 10.0 and -3.0 <= p[i] < 3.0:
            H2[min(int(x[i] // 2.0), 4), min(int((p[i] + 3.0) // 1.5), 3)] += w[i]
    np.testing.assert_allclose(H, H2, rtol=1e-13)
    inside = (x >= 0) & (x < 10) & (p >= -3) & (p < 3)
    assert abs(H.sum() - w[inside].sum()) < 1e-12


def test_bin_index_edges():
    v = np.array([0.0, 0.25, 0.5, 0.999999999, 1.0, -1e-300])
    np.testing.assert_array_equal(oracle.bin_index(v, 0.0, 1.0, 4), [0, 1, 2, 3, -1, -1])


def test_density_sums_to_total_weight_per_cell_volume():
    spec = synth.preset("small2d")
    state = synth.make_state(spec)
    sim = oracle.Sim(spec, state)
    for k in range(2):
        n = sim.density(k)
        assert abs(n.sum() - sim.w[k].sum()) < 1e-9 * sim.w[k].sum()
        # electrons and protons are loaded at the same positions and weights
    np.testing.assert_allclose(sim.density(0), sim.density(1), rtol=1e-12, atol=1e-15)
