"""Pins of the test-particle tracking oracle (analytic wakefield, Boris +
Thomas-BMT) and of its complex-step gradient."""

import numpy as np
import pytest

import oracle

MU_P = 1836.15267343
A_P = 1.793


def _beam(n, seed=0, sigma=7.85, kp=0.1):
    rng = np.random.default_rng(seed)
    x = np.c_[rng.normal(0.0, sigma, (n, 2)), rng.uniform(0.0, 2 * np.pi / kp, n)]
    g = rng.normal(20.0, 2.0, n)
    u = np.c_[np.zeros((n, 2)), np.sqrt(g * g - 1.0)]
    s = np.tile([0.0, 0.0, 1.0], (n, 1))
    return x, u, s


def test_wake_fields_values_and_divergence():
    x = np.array([[1.0, -2.0, 3.0], [0.5, 0.25, -7.0]])
    t, E0, kp = 1.5, 0.3, 0.2
    E, B = oracle.wake_fields(x, t, E0, kp)
    xi = x[:, 2] - t
    r = np.hypot(x[:, 0], x[:, 1])
    Er = E0 * kp * r / 2 * np.sin(kp * xi)
    np.testing.assert_allclose(np.hypot(E[:, 0], E[:, 1]), np.abs(Er), rtol=1e-14)
    np.testing.assert_allclose(E[:, 2], E0 * np.cos(kp * xi), rtol=1e-14)
    # B is azimuthal with half the radial field: B . r_hat = 0, |B| = |E_r| / 2
    np.testing.assert_allclose(B[:, 0] * x[:, 0] + B[:, 1] * x[:, 1], 0.0, atol=1e-15)
    np.testing.assert_allclose(np.hypot(B[:, 0], B[:, 1]), np.abs(Er) / 2, rtol=1e-14)
    assert np.all(B[:, 2] == 0)
    # div E = 0 by central differences
    h = 1e-5
    div = np.zeros(2)
    for a in range(3):
        d = np.zeros((2, 3))
        d[:, a] = h
        div += (oracle.wake_fields(x + d, t, E0, kp)[0][:, a] - oracle.wake_fields(x - d, t, E0, kp)[0][:, a]) / (2 * h)
    np.testing.assert_allclose(div, 0.0, atol=1e-9)


def test_free_streaming_without_field():
    x, u, s = _beam(8)
    xN, uN, sN = oracle.tracking_forward(x, u, s, 0.0, 0.1, 0.5, 50, 1.0, MU_P, A_P)
    g = np.sqrt(1 + np.sum(u * u, axis=1))
    np.testing.assert_allclose(xN, x + 50 * 0.5 * u / g[:, None], rtol=1e-13)
    np.testing.assert_array_equal(uN, u)
    np.testing.assert_array_equal(sN, s)


def test_on_axis_particle_gains_momentum_from_Ez_and_keeps_its_spin():
    # on the axis E_r = B = 0: Boris is u_z += r dt E_z(z^n, t^n), beta x E = 0
    x = np.array([[0.0, 0.0, 3.0]])
    u = np.array([[0.0, 0.0, 19.97]])
    s = np.array([[0.0, 0.0, 1.0]])
    E0, kp, dt, r = 0.1, 0.1, 0.5, 1.0 / MU_P
    z, uz = 3.0, 19.97
    for n in range(40):
        uz = uz + r * dt * E0 * np.cos(kp * (z - n * dt))
        z = z + dt * uz / np.sqrt(1 + uz * uz)
    xN, uN, sN = oracle.tracking_forward(x, u, s, E0, kp, dt, 40, 1.0, MU_P, A_P)
    assert abs(uN[0, 2] - uz) < 1e-12 and abs(xN[0, 2] - z) < 1e-10
    np.testing.assert_allclose(sN, s, atol=1e-15)


def test_spin_norm_kept():
    x, u, s = _beam(16, seed=3)
    s = np.random.default_rng(4).normal(size=(16, 3))
    s /= np.linalg.norm(s, axis=1)[:, None]
    _, _, sN = oracle.tracking_forward(x, u, s, 0.5, 0.1, 0.5, 300, 1.0, MU_P, A_P)
    np.testing.assert_allclose(np.linalg.norm(sN, axis=1), 1.0, atol=1e-13)


def _fd4(f, h):
    """Fourth-order central difference of f at 0 (J is ~1 while its
    derivatives are ~1e-8, so the step is moderate and the stencil wide)."""
    return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)


@pytest.mark.parametrize("which", ["E0", "kp", "x0", "u0", "s0"])
def test_complex_step_gradient_matches_central_differences(which):
    x, u, s = _beam(6, seed=5)
    s = s + np.random.default_rng(6).normal(0, 0.1, s.shape)
    s /= np.linalg.norm(s, axis=1)[:, None]
    args = (0.5, 0.1, 0.5, 150, 1.0, MU_P, A_P)
    c = np.array([0.3, -0.2, 1.0])
    dE0, dkp, dx, du, ds = oracle.gradient_complex_step(x, u, s, *args, c)

    def J(x_, u_, s_, e0, k):
        return oracle.objective(oracle.tracking_forward(x_, u_, s_, e0, k, *args[2:])[2], c)

    if which == "E0":
        fd = _fd4(lambda d: J(x, u, s, 0.5 + d, 0.1), 1e-3)
        assert abs(dE0 - fd) <= 1e-7 * abs(fd), (dE0, fd)
        return
    if which == "kp":
        fd = _fd4(lambda d: J(x, u, s, 0.5, 0.1 + d), 1e-4)
        assert abs(dkp - fd) <= 1e-7 * abs(fd), (dkp, fd)
        return
    arr, g, h = {"x0": (x, dx, 1e-2), "u0": (u, du, 1e-2), "s0": (s, ds, 1e-3)}[which]
    for i in (0, 3):
        for k in range(3):
            def f(d):
                a = arr.copy()
                a[i, k] += d
                trip = (a, u, s) if which == "x0" else ((x, a, s) if which == "u0" else (x, u, a))
                return J(*trip, 0.5, 0.1)
            fd = _fd4(f, h)
            assert abs(g[i, k] - fd) <= 1e-6 * abs(fd) + 2e-14, (which, i, k, g[i, k], fd)
