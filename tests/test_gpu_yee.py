"""The fused Yee step (one pass over E, B and J per step) on grids whose
blocks and runs of planes end ragged: 2D with 300 columns (one block of 253
and a short one) and 21 rows (runs of 8 planes: 8, 8, 5), 3D with 40 x 20 x
36 cells (in-plane blocks of 32 x 8: short in x and in y; runs of 16 planes:
16, 16, 4).  Fields and particles must match the FP64 oracle to
1e-9 after a few steps with the plasma's currents, and the fields of a
plasma-free run with random initial fields to 1e-12, with periodic faces
and with open x faces (Mur ghosts).
"""

import numpy as np
import pytest

import oracle
import synth
from paper_2002_02211_amd import spinpic as S
from parity_util import field_error, max_particle_error, thermal_floor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(*a):
    print("[gpu-case]", *a, flush=True)


GRIDS = [("2d", "small2d", (300, 21, 1)), ("3d", "small3d", (40, 20, 36))]


def _spec(preset, n):
    spec = dict(synth.preset(preset))
    spec["n"] = n
    return spec


@pytest.mark.parametrize("name,preset,n", GRIDS, ids=[g[0] for g in GRIDS])
def test_yee_step_with_plasma_matches_oracle(name, preset, n):
    spec = _spec(preset, n)
    state = synth.make_state(spec)
    _say("fused Yee with plasma", name, n, [p.shape[0] for p in state["particles"]])
    sim = S.Simulation(S.config_from_spec(spec, precision="fp64", tile=(0, 0, 0)), state["particles"],
                       state["fields"])
    ref = oracle.Sim(spec, state)
    sim.step(4)
    ref.step(4)
    F = sim.fields()
    Fo = ref.fields()
    for i, nm in enumerate(S.FIELD_NAMES[:9]):
        e = field_error(F[nm], Fo[i])
        assert e <= 1e-9, (name, nm, e)
    for k in range(len(spec["species"])):
        e = max_particle_error(sim.particles(k), ref.particles(k), spec, thermal_floor(spec, k))
        assert e <= 1e-9, (name, k, e)
    sim.close()


@pytest.mark.parametrize("name,preset,n", GRIDS, ids=[g[0] for g in GRIDS])
def test_yee_step_vacuum_random_fields(name, preset, n):
    spec = _spec(preset, n)
    shape = (6, n[2], n[1], n[0])
    rng = np.random.default_rng(5)
    fields = rng.standard_normal(shape)
    empty = [np.zeros((0, 10)) for _ in spec["species"]]
    _say("fused Yee in vacuum", name, n)
    sim = S.Simulation(S.config_from_spec(spec, precision="fp64"), empty, fields)
    ref = oracle.Sim(spec, {"particles": empty, "fields": fields})
    sim.step(3)
    ref.step(3)
    F = sim.fields()
    Fo = ref.fields()
    for i, nm in enumerate(S.FIELD_NAMES[:6]):
        e = field_error(F[nm], Fo[i])
        assert e <= 1e-12, (name, nm, e)
    sim.close()


@pytest.mark.parametrize("name,preset,n", GRIDS, ids=[g[0] for g in GRIDS])
def test_yee_step_open_faces_random_fields(name, preset, n):
    """Open x faces (a window that does not move) on the same ragged grids:
    the Mur ghosts of the first and last columns, advanced inside the one
    pass, against the oracle's face by face update."""
    spec = _spec(preset, n)
    shape = (6, n[2], n[1], n[0])
    rng = np.random.default_rng(7)
    fields = rng.standard_normal(shape)
    empty = [np.zeros((0, 10)) for _ in spec["species"]]
    _say("fused Yee with open x faces", name, n)
    sim = S.Simulation(S.config_from_spec(spec, precision="fp64"), empty, fields)
    win = dict(speed=0.0, shift_cells=sim.stats()["tile"][0], ppc=0, n0=0.0, ramp_start=0.0, ramp_len=0.0,
               s0=(0.0, 1.0, 0.0))
    sim.window(**win)
    ref = oracle.Sim(spec, {"particles": empty, "fields": fields}, window=win)
    sim.step(5)
    ref.step(5)
    F = sim.fields()
    Fo = ref.fields()
    for i, nm in enumerate(S.FIELD_NAMES[:6]):
        e = field_error(F[nm], Fo[i])
        assert e <= 1e-12, (name, nm, e)
    sim.close()
