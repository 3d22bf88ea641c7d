"""Full-size parity: the c2 and c3 workloads at their real sizes, in the launch
configuration bench.py times (default tiles, FP32 particles, FP64 shared-memory
current sums), plus c2 and c3 on the FP64 path (the reference the FP32 runs
are compared with over their full length).

The oracle cannot run these whole, so one step (after three warm-up steps, so
that rebinning has happened) is checked piece by piece from the GPU's own
state before the step:

* sampled particles (random, the fastest, and ones that changed cell) pushed
  by the oracle (gather from the GPU's E^n, B^n; Boris; T-BMT; move) against
  the GPU's particles after the step;
* J on interior patches, deposited by the oracle from the GPU's old and new
  positions of every particle that can reach the patch;
* E and B after the step against the oracle's Yee update of E^n, B^n with the
  GPU's J (whole grid);
* properties at any size: particle count and ids, |s| = 1, Eq. 4 against the
  mean of the read-back spins, div E - rho held.
"""

import numpy as np
import pytest

import oracle
import synth
from paper_2002_02211_amd import spinpic as S
from parity_util import per_particle_error

pytestmark = pytest.mark.gpu

WARM = 3
NSAMPLE = 2048
PATCHES = 6


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _xi(rows, grid):
    xi = np.zeros((rows.shape[0], 3))
    for a in range(grid.ndim):
        xi[:, a] = rows[:, 1 + a] / grid.d[a]
    return xi


def _unwrap(xi1, xi0, grid):
    out = xi1.copy()
    for a in range(grid.ndim):
        n = grid.n[a]
        out[:, a] = xi0[:, a] + (np.mod(xi1[:, a] - xi0[:, a] + 0.5 * n, n) - 0.5 * n)
    return out


def _pick(rng, rows0, rows1, grid):
    """Random particles, the fastest, and ones that changed cell."""
    n = rows0.shape[0]
    umag = np.max(np.abs(rows1[:, 4:7]), axis=1)
    fast = np.argpartition(umag, n - 256)[-256:]
    c0 = np.floor(_xi(rows0, grid)[:, :grid.ndim])
    c1 = np.floor(_xi(rows1, grid)[:, :grid.ndim])
    moved = np.nonzero(np.any(c0 != c1, axis=1))[0]
    if moved.size > 512:
        moved = rng.choice(moved, 512, replace=False)
    pick = np.concatenate([rng.choice(n, NSAMPLE, replace=False), fast, moved])
    return np.unique(pick)


def _oracle_push(rows0, E, B, grid, sp):
    Z, mu, a = sp["Z"], sp["mu"], sp["a"]
    r = Z / mu
    xi = _xi(rows0, grid)
    Ep, Bp = oracle.gather(E, B, xi, grid)
    um, up, un, gm = oracle.boris(rows0[:, 4:7], Ep, Bp, r, grid.dt)
    Om = oracle.tbmt_omega(um, up, gm, Ep, Bp, r, a)
    s = oracle.spin_precess(rows0[:, 7:10], Om, grid.dt)
    xi1 = oracle.wrap(oracle.move(xi, un, grid), grid)
    out = rows0.copy()
    for ax in range(grid.ndim):
        out[:, 1 + ax] = xi1[:, ax] * grid.d[ax]
    out[:, 4:7] = un
    out[:, 7:10] = s
    return out


def _patch_current(pos, parts1, spec, grid, lo, size, margin=3):
    """J from the oracle's deposit on a local periodic grid around one patch,
    from every particle whose old position lies within the margin of it.
    pos[k] = (old, new unwrapped) positions of species k in cell units."""
    ndim = grid.ndim
    ln = [size + 2 * margin if a < ndim else 1 for a in range(3)]
    local = oracle.Grid(ndim, ln, grid.d, grid.dt)
    J = np.zeros((3,) + local.shape)
    for k, sp in enumerate(spec["species"]):
        xi0, xi1 = pos[k]
        m = np.ones(xi0.shape[0], dtype=bool)
        for a in range(ndim):
            m &= (xi0[:, a] >= lo[a] - margin) & (xi0[:, a] < lo[a] + size + margin)
        x0 = xi0[m].copy()
        x1 = xi1[m].copy()
        for a in range(ndim):
            x0[:, a] -= lo[a] - margin
            x1[:, a] -= lo[a] - margin
        u1 = parts1[k][m, 4:7]
        gam = np.sqrt(1.0 + np.sum(u1 * u1, axis=1))
        oracle.deposit(J, x0, x1, sp["Z"] * parts1[k][m, 10], u1[:, 2] / gam, local)
    sl = tuple(slice(margin, margin + size) if a < ndim else slice(0, 1) for a in (2, 1, 0))
    return J[(slice(None),) + sl]


# (workload, precision, particle bound, J bound relative to max|J|, field bound
# relative to each component's max).  FP64 bounds allow for the read-back rows
# holding x = (cell + offset) * dx: at 4096 cells its last bit is ~7e-13 of a
# cell, which enters the oracle's shape-factor differences.
CASES = [("c2", "fp32", 1e-5, 1e-6, 1e-12), ("c2", "fp64", 1e-11, 1e-11, 1e-12),
         ("c3", "fp32", 1e-5, 1e-6, 1e-12), ("c3", "fp64", 1e-11, 1e-11, 1e-12)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("workload,precision,ptol,jtol,ftol", CASES,
                         ids=["%s-%s" % (c[0], c[1]) for c in CASES])
def test_full_size_one_step(workload, precision, ptol, jtol, ftol):
    spec = synth.preset(workload)
    _say(workload, precision, "generate")
    state = synth.make_state(spec)
    counts = [p.shape[0] for p in state["particles"]]
    sim = S.Simulation(S.config_from_spec(spec, precision=precision), state["particles"], state["fields"])
    del state
    grid = oracle.Grid(spec["ndim"], spec["n"], spec["d"], spec["dt"])
    sim.step(WARM)
    _say(workload, precision, "read state at step", WARM)
    F0 = sim.fields(("Ex", "Ey", "Ez", "Bx", "By", "Bz"))
    E0 = np.stack([F0["Ex"], F0["Ey"], F0["Ez"]])
    B0 = np.stack([F0["Bx"], F0["By"], F0["Bz"]])
    del F0
    parts0 = [sim.particles(k) for k in range(len(counts))]
    e_before = sim.energy()
    sim.step(1)
    _say(workload, precision, "read state at step", WARM + 1)
    parts1 = [sim.particles(k) for k in range(len(counts))]
    F1 = sim.fields(("Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz"))
    e_after = sim.energy()
    P, N = sim.polarization()
    sim.close()

    # properties at full size
    assert N == sum(counts)
    for k in range(len(counts)):
        assert parts1[k].shape[0] == counts[k]
        np.testing.assert_array_equal(parts1[k][:, 0], np.arange(counts[k]))
        snorm = np.abs(np.sqrt(np.sum(parts1[k][:, 7:10] ** 2, axis=1)) - 1.0)
        assert snorm.max() < (2e-6 if precision == "fp32" else 1e-13), snorm.max()
    # pairwise sums over contiguous columns (a sum along axis 0 of an (N, 3)
    # array adds row after row, which loses ~1e-10 over 1e8 values near 1)
    s_mean = np.array([sum(np.ascontiguousarray(p[:, 7 + c]).sum() for p in parts1)
                       for c in range(3)]) / N
    assert np.max(np.abs(P - s_mean)) < 1e-12
    # div E - rho drift: roundoff of the deposit (FP32 shape factors in FP32)
    rtol = 1e-6 if precision == "fp32" else 1e-11
    _say(workload, precision, "div E - rho drift %.2e %.2e" % (e_before[-1], e_after[-1]))
    assert e_after[-1] < rtol and e_before[-1] < rtol

    # sampled particles, one step through the oracle
    rng = np.random.default_rng(7)
    for k, sp in enumerate(spec["species"]):
        pick = _pick(rng, parts0[k], parts1[k], grid)
        want = _oracle_push(parts0[k][pick], E0, B0, grid, sp)
        e = per_particle_error(parts1[k][pick], want, spec, k)
        _say(workload, precision, "species", k, "sampled", pick.size, "max error %.2e" % e.max())
        assert e.max() <= ptol

    # J on interior patches
    J = np.stack([F1["Jx"], F1["Jy"], F1["Jz"]])
    jscale = np.max(np.abs(J))
    assert jscale > 0
    size = 12 if spec["ndim"] == 2 else 6
    worst = 0.0
    pos = []
    for k in range(len(counts)):
        xi0 = _xi(parts0[k], grid)
        pos.append((xi0, _unwrap(_xi(parts1[k], grid), xi0, grid)))
    for _ in range(PATCHES):
        lo = [int(rng.integers(4, spec["n"][a] - size - 4)) if a < spec["ndim"] else 0 for a in range(3)]
        want = _patch_current(pos, parts1, spec, grid, lo, size)
        sl = tuple(slice(lo[a], lo[a] + size) if a < spec["ndim"] else slice(0, 1) for a in (2, 1, 0))
        got = J[(slice(None),) + sl]
        worst = max(worst, float(np.max(np.abs(got - want))) / jscale)
    del pos
    _say(workload, precision, "J patches max error / max|J| %.2e" % worst)
    assert worst <= jtol

    # fields: the oracle's Yee update with the GPU's J
    oracle.yee_step(E0, B0, J, grid)
    for c, nm in enumerate(("Ex", "Ey", "Ez")):
        sc = max(np.max(np.abs(E0[c])), 1e-30)
        assert np.max(np.abs(F1[nm] - E0[c])) <= ftol * sc, nm
    for c, nm in enumerate(("Bx", "By", "Bz")):
        sc = max(np.max(np.abs(B0[c])), 1e-30)
        assert np.max(np.abs(F1[nm] - B0[c])) <= ftol * sc, nm


def test_c2_full_run_repacks_reuse_allocator_blocks():
    """c2 FP32 over its whole run (about 20 repacks as the laser compresses
    the plasma) through torch's caching allocator, the binding's default: a
    repack frees the old store after building the new one, and the memory
    the allocator holds must stay within a few stores, not grow by a store
    at every repack (which had filled a whole device in one process)."""
    import torch
    _say("c2 full run, allocator")
    spec = synth.preset("c2")
    state = synth.make_state(spec)
    npart = sum(p.shape[0] for p in state["particles"])
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    sim = S.Simulation(S.config_from_spec(spec), state["particles"], state["fields"])
    del state
    torch.cuda.synchronize()
    at_init = torch.cuda.memory_reserved()
    torch.cuda.reset_peak_memory_stats()
    sim.step(spec["steps"])
    torch.cuda.synchronize()
    st = sim.stats()
    grown = torch.cuda.max_memory_reserved() - at_init
    # one FP32 2D store: cell, two offsets, u, s, w, id (44 B a slot) for the
    # particles and the 25 % slack
    store = npart * 1.25 * 44
    _say("repacks %d, allocator grew by %.1f GB (%.1f stores)" % (st["repacks"], grown / 1e9, grown / store))
    sim.close()
    torch.cuda.empty_cache()
    assert st["repacks"] >= 10
    assert grown <= 4 * store
