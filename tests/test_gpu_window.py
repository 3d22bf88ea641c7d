"""Co-moving window and open x faces (pic_window) on the GPU against the
oracle's window (oracle.Sim(window=...)).

* FP64: particles by id (the ids of injected particles included), every
  field component and Eq. 4 match the oracle to 1e-9 through several
  shifts: uniform injection with 16-cell tiles, a density ramp starting
  inside the injected region with 8-cell tiles, a fixed box with open faces
  (particles leaving), and 3D with a ragged last tile column.
* Shifts with particles in the overflow store (segments without slack).
* FP32 (2D, and 3D with particles matched by id): within the float32-storage
  bound of the oracle.
* Bad parameters are rejected.
* c2 at full size (FP32, the bench's tiles): right after a shift the newest
  particles sit on the injection lattice of the last columns with the
  stated ids, weights and spins and the new columns' fields are zero; one
  further step of sampled particles (newest, near the faces, random)
  matches the oracle pushed from the GPU's own fields.
"""

import numpy as np
import pytest

import oracle
import synth
from paper_2002_02211_amd import spinpic as S
from parity_util import max_particle_error, thermal_floor, field_error, per_particle_error, storage_bounded

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _win(speed=1.0, shift_cells=16, ppc=0, n0=0.0, ramp_start=0.0, ramp_len=0.0, s0=(0.0, 1.0, 0.0)):
    return dict(speed=speed, shift_cells=shift_cells, ppc=ppc, n0=n0, ramp_start=ramp_start,
                ramp_len=ramp_len, s0=s0)


CASES = [
    ("2d-uniform", "small2d", (16, 16, 1), _win(shift_cells=16, ppc=2, n0=0.03), (20, 50)),
    ("2d-ramp-tile8", "small2d", (8, 8, 1),
     _win(shift_cells=8, ppc=3, n0=0.05, ramp_start=26.0, ramp_len=6.0, s0=(0.0, 0.0, 1.0)), (20, 50)),
    ("2d-open-box", "small2d", (16, 16, 1), _win(speed=0.0, shift_cells=16), (20, 30, 40, 50, 60)),
    ("3d", "small3d", (0, 0, 0), _win(shift_cells=6, ppc=1, n0=0.05, s0=(1.0, 0.0, 0.0)), (12, 25)),
    ("2d-two-columns", "small2d", (8, 8, 1),
     _win(shift_cells=16, ppc=1, n0=0.04, ramp_start=24.0, ramp_len=3.0), (30, 50)),
]


def _compare(sim, ref, spec, tol, label):
    st = sim.stats()
    assert st["shifts"] == ref.shifts, (label, st["shifts"], ref.shifts)
    F = sim.fields()
    Fo = ref.fields()
    ferr = {nm: field_error(F[nm], Fo[i]) for i, nm in enumerate(S.FIELD_NAMES[:9])}
    worst = 0.0
    for k in range(len(spec["species"])):
        want = ref.particles(k)
        got = sim.particles(k)
        assert got.shape == want.shape, (label, k, got.shape, want.shape)
        np.testing.assert_array_equal(got[:, 0], want[:, 0])
        e = per_particle_error(got, want, spec, k)
        worst = max(worst, float(e.max(initial=0.0)))
        if e.max(initial=0.0) > tol:
            q = int(np.argmax(e))
            _say(label, "fields", {nm: "%.1e" % v for nm, v in ferr.items()})
            _say(label, "species", k, "worst particle", int(got[q, 0]), "error %.2e" % e[q],
                 "gpu", np.round(got[q], 6).tolist(), "oracle", np.round(want[q], 6).tolist(),
                 "particles over tol", int((e > tol).sum()))
        assert e.max(initial=0.0) <= tol, (label, k, float(e.max()))
    for nm, v in ferr.items():
        assert v <= tol, (label, nm, v)
    P, N = sim.polarization()
    Po, No = ref.polarization()
    assert N == No and np.max(np.abs(P - Po)) < 1e-12
    return worst, st


@pytest.mark.parametrize("name,preset,tile,win,checks", CASES, ids=[c[0] for c in CASES])
def test_window_fp64_matches_oracle(name, preset, tile, win, checks):
    spec = synth.preset(preset)
    state = synth.make_state(spec)
    _say("window fp64", name)
    sim = S.Simulation(S.config_from_spec(spec, precision="fp64", tile=tile), state["particles"], state["fields"])
    sim.window(**win)
    ref = oracle.Sim(spec, state, window=win)
    done = 0
    for n in checks:
        sim.step(n - done)
        ref.step(n - done)
        done = n
        worst, st = _compare(sim, ref, spec, 1e-9, name)
        _say(name, "step", n, "shifts", st["shifts"], "particles", st["per_species"][:2],
             "worst particle error %.2e" % worst)
    assert ref.shifts >= (2 if win["speed"] > 0 else 0)
    if win["speed"] == 0.0:
        assert sum(x.shape[0] for x in ref.xi) < sum(p.shape[0] for p in state["particles"])
    sim.close()


def test_window_opened_after_periodic_steps():
    spec = synth.preset("small2d")
    state = synth.make_state(spec)
    win = _win(shift_cells=16, ppc=2, n0=0.03)
    _say("window fp64 opened after 8 periodic steps")
    sim = S.Simulation(S.config_from_spec(spec, precision="fp64"), state["particles"], state["fields"])
    ref = oracle.Sim(spec, state)
    sim.step(8)
    ref.step(8)
    sim.window(**win)
    ref.enable_window(win)
    sim.step(42)
    ref.step(42)
    worst, st = _compare(sim, ref, spec, 1e-9, "late window")
    _say("late window shifts", st["shifts"], "worst particle error %.2e" % worst)
    assert ref.shifts >= 1
    sim.close()


@pytest.mark.parametrize("shift_cells,speed,ppc,steps", [(8, 2.0, 2, 40), (64, 16.0, 4, 20)],
                         ids=["one-column", "most-columns"])
def test_window_shifts_with_a_full_overflow_store(shift_cells, speed, ppc, steps):
    """Segments sized with almost no slack: injected particles spill into
    the overflow store, which the shifts move along with the rest instead of
    folding it back first; with shifts of most of the box its particles in
    the first columns leave (and the stores grow)."""
    spec = synth.preset("small2d")
    state = synth.make_state(spec)
    win = _win(speed=speed, shift_cells=shift_cells, ppc=ppc, n0=0.03)
    _say("window fp64 with overflow at the shifts", shift_cells, speed)
    sim = S.Simulation(S.config_from_spec(spec, precision="fp64", tile=(8, 8, 1), slack=1e-6),
                       state["particles"], state["fields"])
    sim.window(**win)
    ref = oracle.Sim(spec, state, window=win)
    spilled = 0
    prev = sim.stats()
    for n in range(1, steps + 1):
        sim.step(1)
        ref.step(1)
        st = sim.stats()
        if st["shifts"] > prev["shifts"]:
            spilled = max(spilled, prev["overflow"])
        prev = st
        if n % 10 == 0:
            worst, _ = _compare(sim, ref, spec, 1e-9, "overflow at shifts")
            _say("step", n, "shifts", st["shifts"], "overflow", st["overflow"], "repacks", st["repacks"],
                 "worst particle error %.2e" % worst)
    assert ref.shifts >= 3
    assert spilled > 0, "no shift happened with particles in the overflow store"
    sim.close()


def test_window_fp32_within_storage_bound():
    name, preset, tile, win, _ = CASES[0]
    spec = synth.preset(preset)
    state = synth.make_state(spec)
    _say("window fp32")
    sim = S.Simulation(S.config_from_spec(spec, precision="fp32", tile=tile), state["particles"], state["fields"])
    sim.window(**win)
    ref = oracle.Sim(spec, state, window=win)
    ref32 = oracle.Sim(spec, state, window=win, store_fp32=True)
    for m in (sim, ref, ref32):
        m.step(40)
    assert sim.stats()["shifts"] == ref.shifts == ref32.shifts >= 1
    for k in range(2):
        want = ref.particles(k)
        got = sim.particles(k)
        w32 = ref32.particles(k)
        assert got.shape == want.shape == w32.shape
        np.testing.assert_array_equal(got[:, 0], want[:, 0])
        e32 = per_particle_error(got, want, spec, k)
        eref = per_particle_error(w32, want, spec, k)
        ok, rep = storage_bounded(e32, eref)
        _say("fp32 species", k, rep)
        assert ok, rep
    P, _ = sim.polarization()
    Po, _ = ref.polarization()
    assert np.max(np.abs(P - Po)) < 1e-3
    sim.close()


def test_window_fp32_3d_within_storage_bound():
    """The 3D FP32 path through shifts: particles matched by id (a particle
    within rounding of an open face may leave on one side only), then held
    to the float32-storage bound like the 2D case."""
    name, preset, _, win, _ = CASES[3]
    tile = (6, 6, 6)   # the window shifts by whole tile columns (6 cells)
    spec = synth.preset(preset)
    state = synth.make_state(spec)
    _say("window fp32 3d")
    sim = S.Simulation(S.config_from_spec(spec, precision="fp32", tile=tile), state["particles"], state["fields"])
    sim.window(**win)
    ref = oracle.Sim(spec, state, window=win)
    ref32 = oracle.Sim(spec, state, window=win, store_fp32=True)
    for m in (sim, ref, ref32):
        m.step(25)
    assert sim.stats()["shifts"] == ref.shifts == ref32.shifts >= 2
    for k in range(2):
        want, got, w32 = ref.particles(k), sim.particles(k), ref32.particles(k)
        ids = np.intersect1d(np.intersect1d(want[:, 0], got[:, 0]), w32[:, 0])
        odd = max(want.shape[0], got.shape[0]) - ids.size
        assert odd <= max(2, want.shape[0] // 1000), (k, odd)
        sel = lambda a: a[np.isin(a[:, 0], ids)]
        want, got, w32 = sel(want), sel(got), sel(w32)
        e32 = per_particle_error(got, want, spec, k)
        eref = per_particle_error(w32, want, spec, k)
        ok, rep = storage_bounded(e32, eref)
        _say("fp32 3d species", k, "unmatched", odd, rep)
        assert ok, rep
    P, _ = sim.polarization()
    Po, _ = ref.polarization()
    assert np.max(np.abs(P - Po)) < 1e-3
    sim.close()


def test_window_rejects_bad_parameters():
    spec = synth.preset("small2d")
    state = synth.make_state(spec)
    sim = S.Simulation(S.config_from_spec(spec, precision="fp64"), state["particles"], state["fields"])
    bad = [dict(shift_cells=12), dict(shift_cells=72), dict(shift_cells=0), dict(speed=-1.0),
           dict(ppc=300), dict(ppc=1, s0=(0.0, 0.5, 0.0)), dict(n0=-1.0), dict(ramp_len=float("nan"))]
    for kw in bad:
        args = _win(**{**dict(shift_cells=16), **kw})
        with pytest.raises(S.PicError) as e:
            sim.window(**args)
        assert e.value.code == S.PIC_EINVAL, kw
    sim.close()


@pytest.mark.timeout(600)
def test_c2_window_full_size():
    spec = synth.preset("c2")
    _say("c2 window generate")
    state = synth.make_state(spec)
    counts0 = [p.shape[0] for p in state["particles"]]
    T = 16
    # particles that start in the first T columns: about what the first shift removes
    first_cols = [int(np.sum(p[:, 0] < T * spec["d"][0])) for p in state["particles"]]
    ramp = 50 * 2 * np.pi
    win = _win(shift_cells=T, ppc=8, n0=0.02, ramp_start=0.0, ramp_len=ramp)
    sim = S.Simulation(S.config_from_spec(spec, precision="fp32"), state["particles"], state["fields"])
    del state
    sim.window(**win)
    grid = oracle.Grid(2, spec["n"], spec["d"], spec["dt"], open_x=True)
    nx, ny = spec["n"][0], spec["n"][1]
    # the first shift ends step 24 (24 dt = 16.1 cells of travel)
    sim.step(24)
    st = sim.stats()
    assert st["shifts"] == 1
    _say("c2 window after the first shift", st)
    parts0 = [sim.particles(k) for k in range(2)]
    F0 = sim.fields(("Ex", "Ey", "Ez", "Bx", "By", "Bz"))
    for nm, arr in F0.items():
        assert not arr[..., nx - T:].any(), nm
    per_shift = ny * T * 8
    for k in range(2):
        rows = parts0[k]
        ids = rows[:, 0].astype(np.int64)
        assert np.unique(ids).size == ids.size
        new = rows[ids >= counts0[k]]
        assert new.shape[0] == per_shift
        cx = np.floor(new[:, 1] / spec["d"][0])
        assert cx.min() == nx - T and cx.max() == nx - 1
        f = new[:, 1] / spec["d"][0] - cx
        lat = (np.arange(8) + 0.5) / 8
        assert np.all(np.min(np.abs(f[:, None] - lat[None, :]), axis=1) < 1e-6)
        assert not new[:, 4:7].any()
        assert np.allclose(new[:, 7:10], [0.0, 1.0, 0.0]) and np.allclose(new[:, 10], 0.02 / 8, rtol=1e-6)
        # initial particles removed: about those that started in the first T
        # columns for the protons (thermal motion moves a few across); fewer
        # electrons, which the pulse's front (a0 about 2.5 at x = 0) pushes on
        removed = counts0[k] - int(np.sum(ids < counts0[k]))
        _say("c2 window species", k, "removed", removed, "started in the first columns", first_cols[k])
        if k == 1:
            assert abs(removed - first_cols[k]) <= 0.02 * first_cols[k] + 100
        else:
            assert 0.5 * first_cols[k] < removed <= 1.02 * first_cols[k] + 100
    E0 = np.stack([F0["Ex"], F0["Ey"], F0["Ez"]])
    B0 = np.stack([F0["Bx"], F0["By"], F0["Bz"]])
    del F0
    sim.step(1)
    assert sim.stats()["shifts"] == 1
    parts1 = [sim.particles(k) for k in range(2)]
    rng = np.random.default_rng(11)
    for k, sp in enumerate(spec["species"]):
        r0, r1 = parts0[k], parts1[k]
        # particles that left during the step are absent from r1
        common, i0, i1 = np.intersect1d(r0[:, 0], r1[:, 0], return_indices=True)
        assert r0.shape[0] - common.size < 1000
        x0 = r0[i0, 1] / spec["d"][0]
        near = np.nonzero((x0 < 2) | (x0 > nx - 2))[0]
        newest = np.nonzero(r0[i0, 0] >= counts0[k])[0]
        pick = np.unique(np.concatenate([rng.choice(common.size, 2048, replace=False),
                                         rng.choice(near, min(512, near.size), replace=False),
                                         rng.choice(newest, 512, replace=False)]))
        rows0 = r0[i0[pick]]
        xi = np.zeros((pick.size, 3))
        for a in range(2):
            xi[:, a] = rows0[:, 1 + a] / spec["d"][a]
        Ep, Bp = oracle.gather(E0, B0, xi, grid)
        rr = sp["Z"] / sp["mu"]
        um, up, un, gm = oracle.boris(rows0[:, 4:7], Ep, Bp, rr, grid.dt)
        Om = oracle.tbmt_omega(um, up, gm, Ep, Bp, rr, sp["a"])
        sn = oracle.spin_precess(rows0[:, 7:10], Om, grid.dt)
        xn = oracle.wrap(oracle.move(xi, un, grid), grid)
        want = rows0.copy()
        for a in range(2):
            want[:, 1 + a] = xn[:, a] * spec["d"][a]
        want[:, 4:7] = un
        want[:, 7:10] = sn
        e = per_particle_error(r1[i1[pick]], want, spec, k)
        _say("c2 window species", k, "sampled", pick.size, "near faces", near.size, "max error %.2e" % e.max())
        assert e.max() <= 1e-5
    P, N = sim.polarization()
    s_mean = np.array([sum(np.ascontiguousarray(p[:, 7 + c]).sum() for p in parts1) for c in range(3)]) / N
    assert N == sum(p.shape[0] for p in parts1) and np.max(np.abs(P - s_mean)) < 1e-12
    sim.close()
