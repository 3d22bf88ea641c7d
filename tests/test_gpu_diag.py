"""Binned diagnostics on the GPU against the oracle's histograms of the same
particles: the GPU state is read back (pic_particles) and binned by the
oracle's functions.  Bin decisions are made in FP64 from the same values
with the same formula on both sides, so bin counts must agree exactly;
weight, spin and density sums to 1e-12 (summation order only)."""

import numpy as np
import pytest

import oracle
import synth
from paper_2002_02211_amd import spinpic as S

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rows_state(sim, spec):
    """u, s, w, x per species from the GPU's particle rows."""
    out = []
    for k in range(len(spec["species"])):
        r = sim.particles(k)
        out.append({"x": r[:, 1:4], "u": r[:, 4:7], "s": r[:, 7:10], "w": r[:, 10]})
    return out


def _check_spectrum(sim, spec, rows, species, emin, emax, nbins):
    c, w, sp = sim.spectrum(species, emin, emax, nbins)
    c2, w2, s2 = np.zeros(nbins), np.zeros(nbins), np.zeros((nbins, 3))
    for k, sp_k in enumerate(spec["species"]):
        if species not in (-1, k):
            continue
        a, b, d = oracle.spectrum(rows[k]["u"], rows[k]["s"], rows[k]["w"], sp_k["mu"], emin, emax, nbins)
        c2 += a
        w2 += b
        s2 += d
    np.testing.assert_array_equal(c, c2)
    np.testing.assert_allclose(w, w2, rtol=1e-12, atol=0)
    scale = max(1.0, float(np.max(np.abs(s2))))
    assert np.max(np.abs(sp - s2)) <= 1e-12 * scale
    return c


@pytest.mark.parametrize("name,precision", [("small2d", "fp64"), ("small2d", "fp32"), ("small3d", "fp32")])
def test_binned_diagnostics_match_oracle(name, precision):
    spec = synth.preset(name)
    _say(name, precision, "binned diagnostics")
    state = synth.make_state(spec)
    sim = S.Simulation(S.config_from_spec(spec, precision=precision), state["particles"], state["fields"])
    sim.step(12)
    rows = _rows_state(sim, spec)
    for species in (-1, 0, 1):
        mu_max = max(sp["mu"] for sp in spec["species"])
        c = _check_spectrum(sim, spec, rows, species, 0.0, 0.05 if species != 1 else 0.05, 64)
        assert c.sum() > 0
    # all particles: the total count equals the particle count when the range covers them
    ek = [oracle.kinetic_energy_binned(r["u"], sp["mu"]) for r, sp in zip(rows, spec["species"])]
    hi = float(max(e.max() for e in ek)) * 1.01 + 1e-9
    c = _check_spectrum(sim, spec, rows, -1, 0.0, hi, 1024)
    assert c.sum() == sum(r["w"].shape[0] for r in rows)
    # phase space along every axis and momentum component
    L = [spec["n"][a] * spec["d"][a] for a in range(3)]
    for k, sp_k in enumerate(spec["species"]):
        for axis in range(spec["ndim"]):
            for comp in range(3):
                pm = float(np.max(np.abs(sp_k["mu"] * rows[k]["u"][:, comp]))) * 1.01 + 1e-12
                H = sim.phase_space(k, axis, 0.0, L[axis], 37, comp, -pm, pm, 29)
                H2 = oracle.phase_space(rows[k]["x"][:, axis], sp_k["mu"] * rows[k]["u"][:, comp],
                                        rows[k]["w"], 0.0, L[axis], 37, -pm, pm, 29)
                np.testing.assert_allclose(H, H2, rtol=1e-12, atol=1e-300)
                assert abs(H.sum() - rows[k]["w"].sum()) <= 1e-12 * rows[k]["w"].sum()
    # number density per species from the same particles
    grid = oracle.Grid(spec["ndim"], spec["n"], spec["d"], spec["dt"])
    for k in range(len(spec["species"])):
        xi = np.zeros((rows[k]["x"].shape[0], 3))
        for a in range(spec["ndim"]):
            xi[:, a] = rows[k]["x"][:, a] / spec["d"][a]
        n_gpu = sim.density(k)
        n_ref = oracle.charge_density(xi, rows[k]["w"], grid)
        assert np.max(np.abs(n_gpu - n_ref)) <= 1e-12 * np.max(np.abs(n_ref))
    sim.close()


def test_per_bin_polarization_and_windowed_eq4_agree():
    spec = synth.preset("small2d")
    _say("per-bin Eq. 4 vs windowed Eq. 4")
    state = synth.make_state(spec)
    sim = S.Simulation(S.config_from_spec(spec, precision="fp64"), state["particles"], state["fields"])
    sim.step(10)
    emin, emax, nb = 0.0, 0.04, 8
    c, w, sp = sim.spectrum(0, emin, emax, nb)
    edges = np.linspace(emin, emax, nb + 1)
    for b in range(nb):
        P, N = sim.polarization(0, edges[b] + 1e-12, edges[b + 1] - 1e-12)
        if N == 0:
            continue
        assert abs(N - c[b]) <= 2
        if N == c[b]:
            np.testing.assert_allclose(sp[b] / c[b], P, rtol=1e-12, atol=1e-14)
    sim.close()


def test_diagnostics_reject_bad_arguments():
    spec = synth.preset("small2d")
    state = synth.make_state(spec)
    sim = S.Simulation(S.config_from_spec(spec, precision="fp64"), state["particles"], state["fields"])
    bad = [lambda: sim.spectrum(2, 0.0, 1.0, 8), lambda: sim.spectrum(0, 1.0, 1.0, 8),
           lambda: sim.spectrum(0, 0.0, 1.0, 0), lambda: sim.spectrum(0, 0.0, 1.0, 1025),
           lambda: sim.spectrum(0, 0.0, float("inf"), 8),
           lambda: sim.phase_space(-1, 0, 0.0, 1.0, 4, 0, -1.0, 1.0, 4),
           lambda: sim.phase_space(0, 2, 0.0, 1.0, 4, 0, -1.0, 1.0, 4),
           lambda: sim.phase_space(0, 0, 0.0, 1.0, 4, 3, -1.0, 1.0, 4),
           lambda: sim.phase_space(0, 0, 0.0, 1.0, 1 << 14, 0, -1.0, 1.0, 1 << 13),
           lambda: sim.density(5)]
    for f in bad:
        with pytest.raises(S.PicError) as e:
            f()
        assert e.value.code == S.PIC_EINVAL
    sim.close()


@pytest.mark.timeout(300)
def test_c2_spectrum_full_size():
    spec = synth.preset("c2")
    _say("c2 fp32 spectrum at full size")
    state = synth.make_state(spec)
    sim = S.Simulation(S.config_from_spec(spec, precision="fp32"), state["particles"], state["fields"])
    del state
    sim.step(5)
    rows = _rows_state(sim, spec)
    c = _check_spectrum(sim, spec, rows, -1, 0.0, 5.0, 1024)
    _check_spectrum(sim, spec, rows, 0, 0.0, 0.5, 256)
    assert c.sum() > 0.9 * sum(r["w"].shape[0] for r in rows)
    H = sim.phase_space(1, 0, 0.0, spec["n"][0] * spec["d"][0], 512, 0, -5.0, 5.0, 128)
    H2 = oracle.phase_space(rows[1]["x"][:, 0], spec["species"][1]["mu"] * rows[1]["u"][:, 0], rows[1]["w"],
                            0.0, spec["n"][0] * spec["d"][0], 512, -5.0, 5.0, 128)
    np.testing.assert_allclose(H, H2, rtol=1e-12, atol=1e-300)
    sim.close()
