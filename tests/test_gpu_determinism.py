"""Deterministic mode and restart from read-back (PIC_FLAG_DETERMINISTIC).

The current deposit of a step is a sum of many contributions per node added
by atomics in whatever order the hardware runs them; in floating point the
order changes the last bits, so two runs of the same state differ by
roundoff.  With PIC_FLAG_DETERMINISTIC the library sums currents (and the
Eq. 4 polarization) as 64-bit fixed-point integers, whose sums do not depend
on the order.  Then:

* two runs from the same state are bitwise identical: every particle's cell,
  offsets, momentum and spin (read back in cell form, exact), every field
  value and the polarization;
* a run stopped after n steps, read back (pic_particles_cells, pic_fields)
  and started again from that state with PIC_FLAG_CELL_ROWS is bitwise
  identical to the uninterrupted run;
* the FP64 deterministic run still matches the oracle like any FP64 run.
"""

import numpy as np
import pytest

import oracle
import synth
from paper_2002_02211_amd import spinpic as S
from parity_util import field_error, max_particle_error, thermal_floor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.load_library()


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _sim(spec, parts, fields, precision, cell_rows=False, **kw):
    cfg = S.config_from_spec(spec, precision=precision, deterministic=True, cell_rows=cell_rows, **kw)
    return S.Simulation(cfg, parts, fields)


def _state(sim, nsp):
    """Everything the run's future depends on, read back exactly."""
    return {"particles": [sim.particles_cells(k) for k in range(nsp)],
            "fields": sim.fields(S.FIELD_NAMES[:9]),
            "P": sim.polarization()[0]}


def _assert_bitwise(a, b, label):
    for k, (pa, pb) in enumerate(zip(a["particles"], b["particles"])):
        assert pa.shape == pb.shape, (label, k)
        assert np.array_equal(pa, pb), "%s: species %d particles differ (max %.3e)" % (
            label, k, np.max(np.abs(pa - pb)) if pa.size else 0.0)
    for nm in S.FIELD_NAMES[:9]:
        assert np.array_equal(a["fields"][nm], b["fields"][nm]), "%s: field %s differs" % (label, nm)
    assert np.array_equal(a["P"], b["P"]), "%s: polarization differs" % label


CASES = [("small2d", "fp64"), ("small2d", "fp32"), ("small3d", "fp64"), ("small3d", "fp32")]


@pytest.mark.parametrize("name,precision", CASES)
def test_two_runs_bitwise_identical(name, precision):
    spec = synth.preset(name)
    state = synth.make_state(spec)
    nsteps = 30 if spec["ndim"] == 2 else 15
    _say("deterministic twice", name, precision, nsteps, "steps")
    out = []
    for _ in range(2):
        sim = _sim(spec, state["particles"], state["fields"], precision)
        sim.step(nsteps)
        out.append(_state(sim, len(spec["species"])))
        sim.close()
    _assert_bitwise(out[0], out[1], "%s %s" % (name, precision))


@pytest.mark.parametrize("name,precision", CASES)
def test_restart_from_readback_bitwise(name, precision):
    spec = synth.preset(name)
    state = synth.make_state(spec)
    n1, n2 = (12, 18) if spec["ndim"] == 2 else (6, 9)
    nsp = len(spec["species"])
    _say("restart", name, precision, n1, "+", n2, "steps")
    whole = _sim(spec, state["particles"], state["fields"], precision)
    whole.step(n1 + n2)
    want = _state(whole, nsp)
    whole.close()
    first = _sim(spec, state["particles"], state["fields"], precision)
    first.step(n1)
    mid = _state(first, nsp)
    first.close()
    # rows in cell form without the id column; ids are the row order (sorted by id)
    rows = [p[:, 1:] for p in mid["particles"]]
    for p in mid["particles"]:
        np.testing.assert_array_equal(p[:, 0], np.arange(p.shape[0]))
    F = np.stack([mid["fields"][nm] for nm in S.FIELD_NAMES[:6]])
    second = _sim(spec, rows, F, precision, cell_rows=True)
    second.step(n2)
    got = _state(second, nsp)
    second.close()
    _assert_bitwise(got, want, "restart %s %s" % (name, precision))


def test_deterministic_fp64_matches_oracle():
    spec = synth.preset("small2d")
    state = synth.make_state(spec)
    _say("deterministic fp64 vs oracle")
    sim = _sim(spec, state["particles"], state["fields"], "fp64")
    ref = oracle.Sim(spec, state)
    sim.step(20)
    ref.step(20)
    for k in range(len(spec["species"])):
        e = max_particle_error(sim.particles(k), ref.particles(k), spec, thermal_floor(spec, k))
        assert e < 1e-9, (k, e)
    F = sim.fields()
    Fo = ref.fields()
    for i, nm in enumerate(S.FIELD_NAMES[:9]):
        assert field_error(F[nm], Fo[i]) < 1e-9, nm
    P, N = sim.polarization()
    Po, No = ref.polarization()
    assert N == No and np.max(np.abs(P - Po)) < 1e-12
    assert sim.energy()[-1] < 1e-11
    sim.close()


def test_deterministic_through_overflow_and_repack():
    """Segments that fill up send particles to the overflow store and are
    repacked; which particles go there depends on the order of the
    insertions, yet both runs end bitwise identical."""
    spec = synth.preset("small2d", n=(64, 32, 1))
    state = synth.make_state(spec)
    e = state["particles"][0]
    left = e[:, 0] < 0.5 * spec["n"][0] * spec["d"][0]
    e[left, 3] = 3.0
    _say("deterministic overflow + repack")
    out = []
    for _ in range(2):
        sim = _sim(spec, state["particles"], state["fields"], "fp64", slack=1e-6)
        overflow = 0
        for _ in range(7):
            sim.step(10)
            overflow = max(overflow, sim.stats()["overflow"])
        st = sim.stats()
        assert overflow > 0 and st["repacks"] >= 1, (overflow, st)
        out.append(_state(sim, 2))
        sim.close()
    _assert_bitwise(out[0], out[1], "overflow")
