"""Pins of the oracle's Boris push and Thomas-BMT spin rotation.

Each test compares the oracle with a result fixed by the mathematics, not by
re-typing the oracle's formula:

* T1  Boris gyration in a uniform B: the discrete rotation angle per step is
      exactly 2*atan(r|B|dt/(2 gamma)), clockwise about B for r*B > 0.
* T2  g-2 law (section 2 Eq. 2-3 in a transverse B): the spin-momentum angle
      advances by a*gamma*omega_c, exactly in its discrete form.
* T3  a = 0 locks the spin to the momentum in a pure magnetic field.
* T4  longitudinal B: precession at (1+a) r|B|/gamma (pins the Omega_v term).
* T5  pure E parallel to u: u grows linearly, the spin does not move.
* T6  |s| = 1 is conserved.
* T7  gamma is conserved in any static magnetic field.
* Helicity law of Bargmann-Michel-Telegdi in Jackson's form,
      d(beta_hat.s)/dt = -r s_perp.[a beta_hat x B + (a beta - 1/(beta gamma^2)) E],
      which pins the E terms of Eq. 2 and their signs.
* E x B drift: the mean velocity in crossed fields is E x B / B^2.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import pic as O


def _angle_about_z(v):
    return np.arctan2(v[..., 1], v[..., 0])


def _one(v):
    return np.asarray(v, dtype=np.float64)[None, :]


@pytest.mark.parametrize("r", [-1.0, 1.0 / 1836.15267343, 2.5])
@pytest.mark.parametrize("u0", [0.3, 5.0])
def test_T1_boris_gyration_phase(r, u0):
    dt, B0 = 0.2, 0.7
    u = _one([u0, 0.0, 0.0])
    E = _one([0.0, 0.0, 0.0])
    B = _one([0.0, 0.0, B0])
    gamma = math.sqrt(1 + u0 * u0)
    step_angle = -2.0 * math.atan(r * B0 * dt / (2 * gamma))
    for n in range(1, 41):
        _, _, u, _ = O.boris(u, E, B, r, dt)
        expect = math.remainder(n * step_angle, 2 * math.pi)
        got = _angle_about_z(u)[0]
        assert abs(math.remainder(got - expect, 2 * math.pi)) < 1e-12
        assert abs(np.linalg.norm(u) - u0) < 1e-13 * u0


@pytest.mark.parametrize("a", [0.00116, 1.793, -0.1428])
@pytest.mark.parametrize("u0", [0.5, 20.0])
def test_T2_g_minus_2_discrete_and_continuum(a, u0):
    r, B0 = 1.0, 0.4
    gamma = math.sqrt(1 + u0 * u0)
    for dt in (0.3, 0.01):
        u = _one([u0, 0.0, 0.0])
        s = _one([1.0, 0.0, 0.0])
        E = _one([0, 0, 0])
        B = _one([0, 0, B0])
        per_step = -(2 * math.atan((a + 1 / gamma) * r * B0 * dt / 2)
                     - 2 * math.atan(r * B0 * dt / (2 * gamma)))
        nsteps = 25
        for n in range(1, nsteps + 1):
            um, up, u, gm = O.boris(u, E, B, r, dt)
            Om = O.tbmt_omega(um, up, gm, E, B, r, a)
            s = O.spin_precess(s, Om, dt)
            rel = _angle_about_z(s)[0] - _angle_about_z(u)[0]
            assert abs(math.remainder(rel - n * per_step, 2 * math.pi)) < 1e-11
        # continuum g-2 law: d(angle)/dt = -a gamma omega_c, omega_c = r|B|/gamma
        omega_c = r * B0 / gamma
        rate = per_step / dt
        assert rate == pytest.approx(-a * gamma * omega_c, rel=max(2 * (omega_c * gamma * (abs(a) + 1) * dt) ** 2, 1e-12))


def test_T3_a_zero_locks_spin_to_momentum():
    rng = np.random.default_rng(5)
    N = 200
    u = rng.normal(0, 3, (N, 3))
    u[:, 2] = 0.0
    s = u / np.linalg.norm(u, axis=1)[:, None]
    E = np.zeros((N, 3))
    B = np.zeros((N, 3))
    B[:, 2] = rng.normal(0, 1, N)
    for _ in range(200):
        um, up, u, gm = O.boris(u, E, B, -1.0, 0.25)
        Om = O.tbmt_omega(um, up, gm, E, B, -1.0, 0.0)
        s = O.spin_precess(s, Om, 0.25)
    uh = u / np.linalg.norm(u, axis=1)[:, None]
    assert np.max(np.abs(s - uh)) < 1e-12


@pytest.mark.parametrize("a", [0.00116, 1.793])
def test_T4_longitudinal_field(a):
    r, B0, dt, u0 = 1.0 / 1836.15267343, 3.0, 0.5, 2.0
    gamma = math.sqrt(1 + u0 * u0)
    u = _one([0, 0, u0])
    s = _one([1.0, 0, 0])
    E = _one([0, 0, 0])
    B = _one([0, 0, B0])
    per_step = -2 * math.atan((1 + a) * r * B0 * dt / (2 * gamma))
    for n in range(1, 31):
        um, up, u_new, gm = O.boris(u, E, B, r, dt)
        assert np.array_equal(u_new, u)
        Om = O.tbmt_omega(um, up, gm, E, B, r, a)
        s = O.spin_precess(s, Om, dt)
        assert abs(math.remainder(_angle_about_z(s)[0] - n * per_step, 2 * math.pi)) < 1e-12
        u = u_new


def test_T5_pure_E_parallel_to_u():
    r, dt = -1.0, 0.125
    E = _one([0.0, 0.0, 0.5])
    B = _one([0, 0, 0])
    u0 = _one([0.0, 0.0, 0.75])
    u = u0.copy()
    s = _one([0.0, 0.6, 0.8])
    for n in range(1, 51):
        um, up, u, gm = O.boris(u, E, B, r, dt)
        Om = O.tbmt_omega(um, up, gm, E, B, r, 1.793)
        s_new = O.spin_precess(s, Om, dt)
        assert np.array_equal(s_new, s)
        assert u[0, 2] == pytest.approx(0.75 + r * 0.5 * n * dt, abs=1e-14)
        assert u[0, 0] == 0.0 and u[0, 1] == 0.0


def test_T6_spin_norm_conserved_in_random_fields():
    rng = np.random.default_rng(7)
    N = 500
    u = rng.normal(0, 2, (N, 3))
    s = rng.normal(0, 1, (N, 3))
    s /= np.linalg.norm(s, axis=1)[:, None]
    for _ in range(100):
        E = rng.normal(0, 2, (N, 3))
        B = rng.normal(0, 2, (N, 3))
        um, up, u, gm = O.boris(u, E, B, -1.0, 0.2)
        Om = O.tbmt_omega(um, up, gm, E, B, -1.0, 0.00116)
        s = O.spin_precess(s, Om, 0.2)
    assert np.max(np.abs(np.linalg.norm(s, axis=1) - 1.0)) < 1e-14


def _uniform_test_particle_sim(ndim, Bfield, Efield=None, n=(16, 12, 8), ppc=1, seed=3, u_sigma=1.0):
    rng = np.random.default_rng(seed)
    d = (0.3, 0.35, 0.4)
    spec = {"ndim": ndim, "n": n, "d": d, "dt": 0.2,
            "species": [{"Z": -1.0, "mu": 1.0, "a": 0.00116},
                        {"Z": 1.0, "mu": 1836.15267343, "a": 1.793}]}
    shape = (n[2] if ndim == 3 else 1, n[1], n[0])
    F = np.zeros((6,) + shape)
    F[3:6] = Bfield(shape, rng)
    if Efield is not None:
        F[0:3] = Efield(shape, rng)
    parts = []
    for _ in spec["species"]:
        N = 64
        p = np.zeros((N, 10))
        for a in range(ndim):
            p[:, a] = rng.random(N) * n[a] * d[a]
        p[:, 3:6] = rng.normal(0, u_sigma, (N, 3))
        p[:, 6:9] = [0, 1, 0]
        p[:, 9] = 0.01
        parts.append(p)
    return oracle.Sim(spec, {"particles": parts, "fields": F}, test_particle=True)


@pytest.mark.parametrize("ndim", [2, 3])
def test_T7_gamma_conserved_in_static_magnetic_field(ndim):
    sim = _uniform_test_particle_sim(ndim, lambda shp, rng: rng.normal(0, 3.0, (3,) + shp))
    g0 = [np.sqrt(1 + np.sum(u * u, axis=1)) for u in sim.u]
    sim.step(100)
    for k in range(2):
        g1 = np.sqrt(1 + np.sum(sim.u[k] ** 2, axis=1))
        assert np.max(np.abs(g1 - g0[k]) / g0[k]) < 1e-13
        assert np.max(np.abs(np.linalg.norm(sim.s[k], axis=1) - 1)) < 1e-14


@pytest.mark.parametrize("a", [0.0, 0.00116, 1.793])
@pytest.mark.parametrize("r", [-1.0, 0.37])
def test_helicity_law_jackson(a, r):
    """Instantaneous d(beta_hat . s)/dt against the BMT helicity equation."""
    rng = np.random.default_rng(11)
    N = 64
    u = rng.normal(0, 1.5, (N, 3))
    s = rng.normal(0, 1, (N, 3))
    s /= np.linalg.norm(s, axis=1)[:, None]
    E = rng.normal(0, 1, (N, 3))
    B = rng.normal(0, 1, (N, 3))
    dt = 1e-4
    # centre the finite difference on the field time: u and s at -dt/2 and +dt/2
    um, up, u1, gm = O.boris(u, E, B, r, dt)
    Om = O.tbmt_omega(um, up, gm, E, B, r, a)
    s1 = O.spin_precess(s, Om, dt)

    def helicity(uu, ss):
        return np.sum(uu * ss, axis=1) / np.linalg.norm(uu, axis=1)

    fd = (helicity(u1, s1) - helicity(u, s)) / dt
    uc = 0.5 * (u + u1)
    sc = 0.5 * (s + s1)
    gamma = np.sqrt(1 + np.sum(uc * uc, axis=1))
    beta = uc / gamma[:, None]
    bn = np.linalg.norm(beta, axis=1)
    bh = beta / bn[:, None]
    s_perp = sc - bh * np.sum(bh * sc, axis=1)[:, None]
    law = -r * (a * np.sum(s_perp * np.cross(bh, B), axis=1)
                + (a * bn - 1.0 / (bn * gamma ** 2)) * np.sum(s_perp * E, axis=1))
    assert np.max(np.abs(fd - law)) < 1e-6 * max(1.0, np.max(np.abs(law)))


def test_E_cross_B_drift():
    r, dt = -1.0, 0.02
    E0, B0 = 0.3, 1.0
    E = _one([0.0, E0, 0.0])
    B = _one([0.0, 0.0, B0])
    u = _one([0.0, 0.0, 0.0])
    x = 0.0
    vd = E0 / B0
    gamma_d = 1.0 / math.sqrt(1 - vd * vd)
    # one gyration of a particle starting at rest: 2 pi gamma_d^2/(|r| B) in the
    # drift frame, times gamma_d for the lab clock
    period = 2 * math.pi * gamma_d ** 3 / (abs(r) * B0)
    nsteps = int(round(20 * period / dt))
    for _ in range(nsteps):
        _, _, u, _ = O.boris(u, E, B, r, dt)
        gamma = math.sqrt(1 + float(np.sum(u * u)))
        x += dt * u[0, 0] / gamma
    assert x / (nsteps * dt) == pytest.approx(vd, rel=2e-3)
