"""FP64 oracle of spin tracking of test particles through an analytic
wakefield, and the gradient of the final polarization.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The particles do not act on the fields.  Each step is the same Boris push and
Thomas-BMT spin rotation as in the PIC oracle (section 2 Eq. 1-3), with the
fields of a linear wake moving at c along z evaluated at the particle:
with xi = z - t,

    E_z = E0 cos(kp xi),  E_r = E0 kp r / 2 sin(kp xi),  B_phi = E_r / 2,

i.e. E_x = E0 kp x / 2 sin, E_y = E0 kp y / 2 sin, B_x = -E0 kp y / 4 sin,
B_y = E0 kp x / 4 sin, B_z = 0.  Positions are at integer times (t^n = n dt),
momenta u = gamma beta and spins at half-integer times.  The objective is
J = c . P with P the polarization of section 2 Eq. 4 over all particles after
the last step.

The gradient is the complex-step derivative of this forward map: every
operation here is analytic, so Im J(theta + i h) / h is the derivative to
rounding for a tiny h, with no subtraction.  Perturbing one initial
component of every particle at once gives all particles' derivatives in one
run, since particles do not interact.  This is an independent route to the
gradient from the hand-written adjoint the library uses.
"""

import numpy as np

from .pic import boris, tbmt_omega, spin_precess


def wake_fields(x, t, E0, kp):
    """E and B, each (N, 3), at positions x (N, 3) and time t."""
    xi = x[:, 2] - t
    S = np.sin(kp * xi)
    C = np.cos(kp * xi)
    E = np.stack([0.5 * E0 * kp * x[:, 0] * S, 0.5 * E0 * kp * x[:, 1] * S, E0 * C], axis=1)
    B = np.stack([-0.25 * E0 * kp * x[:, 1] * S, 0.25 * E0 * kp * x[:, 0] * S, 0.0 * S], axis=1)
    return E, B


def tracking_step(x, u, s, t, E0, kp, dt, r, a):
    """One step: fields at (x^n, t^n), Boris for u, Cayley rotation for s with
    the precession vector at the Boris midpoint, then x^(n+1) = x^n + dt u/gamma."""
    E, B = wake_fields(x, t, E0, kp)
    um, up, un, gm = boris(u, E, B, r, dt)
    Om = tbmt_omega(um, up, gm, E, B, r, a)
    s_new = spin_precess(s, Om, dt)
    gamma = np.sqrt(1.0 + np.sum(un * un, axis=1))
    x_new = x + dt * un / gamma[:, None]
    return x_new, un, s_new


def tracking_forward(x0, u0, s0, E0, kp, dt, nsteps, Z, mu, a, store_fp32=False):
    """Final (x, u, s) after nsteps steps starting at t = 0.  With store_fp32
    the state is rounded to float32 after every step (and at the start): the
    exact method with float32 storage, which bounds what any float32
    trajectory must deviate from the float64 one."""
    r = Z / mu
    x, u, s = x0, u0, s0
    if store_fp32:
        x, u, s = (np.asarray(v, dtype=np.float32).astype(np.float64) for v in (x, u, s))
    for n in range(nsteps):
        x, u, s = tracking_step(x, u, s, n * dt, E0, kp, dt, r, a)
        if store_fp32:
            x, u, s = (v.astype(np.float32).astype(np.float64) for v in (x, u, s))
    return x, u, s


def objective(s, c):
    """J = c . P, P the mean spin (section 2 Eq. 4)."""
    return np.mean(s, axis=0) @ np.asarray(c)


def gradient_complex_step(x0, u0, s0, E0, kp, dt, nsteps, Z, mu, a, c, h=1e-20):
    """dJ/dE0, dJ/dkp and dJ/dx0, dJ/du0, dJ/ds0 (each (N, 3)) by complex step."""
    x0 = np.asarray(x0, dtype=np.complex128)
    u0 = np.asarray(u0, dtype=np.complex128)
    s0 = np.asarray(s0, dtype=np.complex128)
    n = x0.shape[0]

    def J(x, u, s, e0, k):
        _, _, sN = tracking_forward(x, u, s, e0, k, dt, nsteps, Z, mu, a)
        return objective(sN, c)

    dE0 = J(x0, u0, s0, E0 + 1j * h * max(abs(E0), 1.0), kp).imag / (h * max(abs(E0), 1.0))
    dkp = J(x0, u0, s0, E0, kp + 1j * h * max(abs(kp), 1.0)).imag / (h * max(abs(kp), 1.0))
    grads = []
    for which in range(3):
        g = np.zeros((n, 3))
        for k in range(3):
            pert = [x0, u0, s0]
            d = np.zeros((n, 3), dtype=np.complex128)
            d[:, k] = 1j * h
            pert[which] = pert[which] + d
            _, _, sN = tracking_forward(pert[0], pert[1], pert[2], E0, kp, dt, nsteps, Z, mu, a)
            # J is a mean over particles; particle i's own term carries its derivative
            g[:, k] = (sN @ np.asarray(c)).imag / (h * n)
        grads.append(g)
    return dE0, dkp, grads[0], grads[1], grads[2]


def per_particle_complex_step(x0, u0, s0, E0, kp, dt, nsteps, Z, mu, a, c, h=1e-20):
    """Per particle i, the derivatives of c . s_i(final) with respect to E0,
    kp (each (N,)) and to its own initial x, u, s (each (N, 3)), by complex
    step.  The gradient of J = c . mean(s) is these divided by N."""
    x0 = np.asarray(x0, dtype=np.complex128)
    u0 = np.asarray(u0, dtype=np.complex128)
    s0 = np.asarray(s0, dtype=np.complex128)
    n = x0.shape[0]
    cc = np.asarray(c)

    def run(x, u, s, e0, k):
        return tracking_forward(x, u, s, e0, k, dt, nsteps, Z, mu, a)[2] @ cc

    hE = h * max(abs(E0), 1.0)
    hk = h * max(abs(kp), 1.0)
    dE0 = run(x0, u0, s0, E0 + 1j * hE, kp).imag / hE
    dkp = run(x0, u0, s0, E0, kp + 1j * hk).imag / hk
    grads = []
    for which in range(3):
        g = np.zeros((n, 3))
        for k in range(3):
            pert = [x0, u0, s0]
            d = np.zeros((n, 3), dtype=np.complex128)
            d[:, k] = 1j * h
            pert[which] = pert[which] + d
            g[:, k] = run(*pert, E0, kp).imag / h
        grads.append(g)
    return dE0, dkp, grads[0], grads[1], grads[2]
