"""Pins of the oracle's grid operations: gather, deposit, Yee update.

* gather: CIC interpolation from each component's own staggered position
  reproduces any linear field exactly (a wrong half-cell offset does not).
* T8  discrete continuity: rho^(n+1) - rho^n + dt div J = 0 on every node for
      arbitrary moves, and div E - rho stays constant over whole runs.
* T9  single-particle current: sum J_x = Z w dx_moved/dt, sum J_z = Z w v_z.
* J_z (2D3V) distribution of a diagonal move, computed by hand as the time
      integral of the product of the two linear shape factors.
* T10 Yee vacuum: a discrete standing mode oscillates exactly at the Yee
      dispersion frequency; a travelling mode moves in the direction E x B.
* T11 Langmuir oscillation of a cold e/p plasma at the plasma frequency.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import pic as O


# Yee positions written out independently of the oracle's tables: E_a sits
# half a cell along axis a, B_a half a cell along both other axes.
YEE_E = ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5))
YEE_B = ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))


def _grid(ndim, n=(12, 10, 8), d=(0.3, 0.4, 0.5), dt=0.15):
    return O.Grid(ndim, n, d, dt)


@pytest.mark.parametrize("ndim", [2, 3])
def test_gather_reproduces_linear_fields_from_staggered_positions(ndim):
    g = _grid(ndim)
    rng = np.random.default_rng(1)
    nz, ny, nx = g.shape
    k = np.arange(nz)[:, None, None].astype(float)
    j = np.arange(ny)[None, :, None].astype(float)
    i = np.arange(nx)[None, None, :].astype(float)
    coefs = rng.normal(0, 1, (6, 4))
    E = np.zeros((3,) + g.shape)
    B = np.zeros((3,) + g.shape)
    for c in range(3):
        for F, st, cc in ((E, YEE_E[c], coefs[c]), (B, YEE_B[c], coefs[3 + c])):
            val = cc[0] + cc[1] * (i + st[0]) + cc[2] * (j + st[1])
            if ndim == 3:
                val = val + cc[3] * (k + st[2])
            F[c] = np.broadcast_to(val, g.shape)
    # interior particles: no stencil point wraps around the periodic edge
    N = 300
    xi = np.zeros((N, 3))
    for a in range(ndim):
        xi[:, a] = 1.0 + rng.random(N) * (g.n[a] - 3)
    Ep, Bp = O.gather(E, B, xi, g)
    for c in range(3):
        for P, cc in ((Ep, coefs[c]), (Bp, coefs[3 + c])):
            want = cc[0] + cc[1] * xi[:, 0] + cc[2] * xi[:, 1]
            if ndim == 3:
                want = want + cc[3] * xi[:, 2]
            np.testing.assert_allclose(P[:, c], want, rtol=0, atol=1e-12)


def _random_moves(g, N, rng, max_step=0.9):
    xi0 = np.zeros((N, 3))
    xi1 = np.zeros((N, 3))
    for a in range(g.ndim):
        xi0[:, a] = rng.random(N) * g.n[a]
        xi1[:, a] = xi0[:, a] + rng.uniform(-max_step, max_step, N)
    return xi0, xi1


@pytest.mark.parametrize("ndim", [2, 3])
def test_T8_deposit_satisfies_discrete_continuity(ndim):
    g = _grid(ndim)
    rng = np.random.default_rng(2)
    N = 500
    xi0, xi1 = _random_moves(g, N, rng)
    Zw = rng.normal(0, 1, N)
    vz = rng.normal(0, 0.5, N)
    J = np.zeros((3,) + g.shape)
    O.deposit(J, xi0, xi1, Zw, vz, g)
    rho0 = O.charge_density(O.wrap(xi0, g), Zw, g)
    rho1 = O.charge_density(O.wrap(xi1, g), Zw, g)
    resid = (rho1 - rho0) / g.dt + O.div_E(J, g)
    assert np.max(np.abs(resid)) < 1e-12 * np.max(np.abs(rho1 - rho0) / g.dt)


@pytest.mark.parametrize("ndim", [2, 3])
def test_T9_single_particle_current_sums(ndim):
    g = _grid(ndim)
    rng = np.random.default_rng(3)
    for _ in range(50):
        xi0, xi1 = _random_moves(g, 1, rng)
        Zw = np.array([rng.normal()])
        vz = np.array([rng.normal()])
        J = np.zeros((3,) + g.shape)
        O.deposit(J, xi0, xi1, Zw, vz, g)
        for a in range(ndim):
            moved = (xi1[0, a] - xi0[0, a]) * g.d[a]
            assert np.sum(J[a]) == pytest.approx(Zw[0] * moved / g.dt, rel=1e-12, abs=1e-13)
        if ndim == 2:
            assert np.sum(J[2]) == pytest.approx(Zw[0] * vz[0], rel=1e-12, abs=1e-14)


def test_jz_2d3v_diagonal_move_by_hand():
    """(0.2, 0.2) -> (0.8, 0.8) inside cell (3, 4): the x and y shape factors
    of node 3 fall linearly 0.8 -> 0.2 and of node 4 rise 0.2 -> 0.8.  Their
    products integrated over the step: int (0.8-0.6t)^2 dt = 0.28 for the
    diagonal nodes and int (0.8-0.6t)(0.2+0.6t) dt = 0.22 for the others."""
    g = _grid(2)
    xi0 = np.array([[3.2, 4.2, 0.0]])
    xi1 = np.array([[3.8, 4.8, 0.0]])
    J = np.zeros((3,) + g.shape)
    O.deposit(J, xi0, xi1, np.array([2.0]), np.array([0.5]), g)
    Jz = J[2, 0]
    expect = {(3, 4): 0.28, (4, 5): 0.28, (4, 4): 0.22, (3, 5): 0.22}
    for (ix, iy), wgt in expect.items():
        assert Jz[iy, ix] == pytest.approx(1.0 * wgt, rel=1e-13)
    assert np.count_nonzero(Jz) == 4
    # J_x of the same move: each node row y carries the y-shape averaged over
    # the step times Z w dx_moved/dt; rows 4 and 5 get (0.8+0.2)/2 = 0.5 each
    # of the row's share, all at x = 3 + 1/2
    Jx = J[0, 0]
    total = 2.0 * 0.6 * g.d[0] / g.dt
    assert Jx[4, 3] == pytest.approx(0.5 * total, rel=1e-13)
    assert Jx[5, 3] == pytest.approx(0.5 * total, rel=1e-13)
    assert np.count_nonzero(np.abs(Jx) > 1e-15) == 2


def test_jz_2d3v_skewed_move_by_hand():
    """(3.2, 4.3) -> (3.7, 4.5): node-3 x-shape 0.8 -> 0.3, node-4 0.2 -> 0.7,
    node-4 y-shape 0.7 -> 0.5, node-5 0.3 -> 0.5.  Integrating the products of
    these linear functions over the step gives 203/600, 157/600, 127/600 and
    113/600 for the nodes (3,4), (4,4), (3,5), (4,5)."""
    g = _grid(2)
    J = np.zeros((3,) + g.shape)
    O.deposit(J, np.array([[3.2, 4.3, 0.0]]), np.array([[3.7, 4.5, 0.0]]),
              np.array([1.0]), np.array([1.0]), g)
    Jz = J[2, 0]
    for (ix, iy), num in {(3, 4): 203, (4, 4): 157, (3, 5): 127, (4, 5): 113}.items():
        assert Jz[iy, ix] == pytest.approx(num / 600.0, rel=1e-13)
    assert np.count_nonzero(Jz) == 4


def _standing_mode(g, comp, m):
    """cos pattern of E_comp on its staggered points with wave numbers m."""
    nz, ny, nx = g.shape
    st = YEE_E[comp]
    idx = [np.arange(nx)[None, None, :] + st[0],
           np.arange(ny)[None, :, None] + st[1],
           np.arange(nz)[:, None, None] + st[2]]
    kk = [2 * math.pi * m[a] / (g.n[a] * g.d[a]) for a in range(g.ndim)]
    val = np.ones(g.shape)
    for a in range(g.ndim):
        val = val * np.cos(kk[a] * idx[a] * g.d[a])
    return val, kk


@pytest.mark.parametrize("ndim,comp,m", [
    (2, 2, (1, 2, 0)), (2, 2, (3, 0, 0)),
    (3, 2, (1, 1, 0)), (3, 0, (0, 2, 1)), (3, 1, (2, 0, 3)),
])
def test_T10_yee_standing_mode_dispersion(ndim, comp, m):
    g = _grid(ndim, n=(16, 12, 10), d=(0.3, 0.4, 0.35))
    g.dt = 0.9 / math.sqrt(sum(1 / g.d[a] ** 2 for a in range(ndim)))
    val, kk = _standing_mode(g, comp, m)
    # the mode must be divergence-free: E_comp may not vary along axis comp
    assert m[comp] == 0
    E = np.zeros((3,) + g.shape)
    E[comp] = val
    B = np.zeros((3,) + g.shape)
    J = np.zeros((3,) + g.shape)
    s2 = sum((math.sin(kk[a] * g.d[a] / 2) / g.d[a]) ** 2 for a in range(ndim))
    omega = 2 * math.asin(g.dt * math.sqrt(s2)) / g.dt
    for n in range(1, 61):
        O.yee_step(E, B, J, g)
        np.testing.assert_allclose(E[comp], math.cos(omega * n * g.dt) * val, atol=1e-11)
    assert np.max(np.abs(O.div_E(E, g))) < 1e-11


@pytest.mark.parametrize("direction", [1, -1])
def test_T10_yee_travelling_wave_moves_along_E_cross_B(direction):
    """E_y on integer x nodes, B_z on half nodes; B = direction * x_hat x E
    makes the wave travel along direction * x_hat at the Yee phase speed."""
    g = O.Grid(2, (64, 4, 1), (0.25, 0.25, 1.0), 0.2)
    k = 2 * math.pi * 3 / (64 * 0.25)
    omega = 2 * math.asin(g.dt / g.d[0] * math.sin(k * g.d[0] / 2)) / g.dt
    x_e = np.arange(64) * g.d[0]
    x_b = (np.arange(64) + 0.5) * g.d[0]
    E = np.zeros((3,) + g.shape)
    B = np.zeros((3,) + g.shape)
    E[1] = np.cos(k * x_e)[None, None, :]
    # B^n is the mean of the half-step values, hence the cos(omega dt / 2)
    B[2] = direction * math.cos(omega * g.dt / 2) * np.cos(k * x_b)[None, None, :]
    J = np.zeros_like(E)
    for n in range(1, 41):
        O.yee_step(E, B, J, g)
    want = np.cos(k * x_e - direction * omega * 40 * g.dt)
    np.testing.assert_allclose(E[1][0, 0], want, atol=1e-11)


def _run_residual(spec_name, steps):
    import synth
    spec = synth.preset(spec_name)
    sim = oracle.Sim(spec, synth.make_state(spec))
    worst = 0.0
    for _ in range(steps):
        sim.step(1)
        worst = max(worst, sim.energy()[-1])
    return worst, sim


@pytest.mark.parametrize("name", ["small2d", "small3d"])
def test_T8_div_E_minus_rho_constant_over_a_run(name):
    worst, sim = _run_residual(name, 12)
    assert worst < 1e-11
    # the run did move charge around: the residual is not trivially zero
    assert np.max(np.abs(sim.J)) > 1e-4


def test_T11_langmuir_frequency():
    """A cold e/p plasma with a small sinusoidal electron displacement oscillates
    at omega_p sqrt(1 + m_e/m_p), omega_p^2 = n/n_c, up to the grid dispersion."""
    n0, nx, ny, ppc = 0.01, 32, 4, 8
    d = (1.0, 1.0, 1.0)
    dt = 0.95 / math.sqrt(2.0)
    spec = {"ndim": 2, "n": (nx, ny, 1), "d": d, "dt": dt,
            "species": [{"Z": -1.0, "mu": 1.0, "a": 0.0},
                        {"Z": 1.0, "mu": 1836.15267343, "a": 0.0}]}
    L = nx * d[0]
    k = 2 * math.pi / L
    N = nx * ny * ppc
    # quiet start: particles on a regular lattice
    ix = np.repeat(np.arange(nx), ny * ppc)
    rest = np.arange(N) % (ny * ppc)
    x0 = (ix + (rest % ppc + 0.5) / ppc) * d[0]
    y0 = (rest // ppc + 0.5) * d[1]
    parts = []
    for q in (-1, 1):
        p = np.zeros((N, 10))
        p[:, 0] = x0 + (0.05 * np.sin(k * x0) if q == -1 else 0.0)
        p[:, 1] = y0
        p[:, 7] = 1.0
        p[:, 9] = n0 / ppc
        parts.append(p)
    F = np.zeros((6, 1, ny, nx))
    sim = oracle.Sim(spec, {"particles": parts, "fields": F})
    # the displaced electrons left div E - rho = rho at t=0; fields start at 0,
    # so first solve E_x from Gauss's law for a consistent start
    rho = sim.rho()[0]
    ex = np.cumsum(rho.mean(axis=0)) * d[0]
    ex -= ex.mean()
    sim.E[0, 0] = ex[None, :]
    sim.residual0 = O.div_E(sim.E, sim.grid) - sim.rho()
    series = []
    for _ in range(400):
        sim.step(1)
        series.append(sim.E[0, 0].mean(axis=0) @ np.sin(k * (np.arange(nx) + 0.5) * d[0]))
    series = np.array(series)
    t = (np.arange(400) + 1) * dt
    crossings = t[:-1][np.sign(series[:-1]) != np.sign(series[1:])]
    period = 2 * np.mean(np.diff(crossings))
    omega = 2 * math.pi / period
    omega_p = math.sqrt(n0 * (1 + 1 / 1836.15267343))
    print("Langmuir omega", omega, "expected", omega_p)
    assert omega == pytest.approx(omega_p, rel=0.03)
    assert sim.energy()[-1] < 1e-11
