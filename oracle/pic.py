"""Plain FP64 CPU oracle of one spin-resolved PIC step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It shares no code
with the HIP library: it is slow, vectorized NumPy written to be checked
against the paper by eye.

What it computes, in the order of one step (state: E^n, B^n at integer time,
positions x^n, momenta u^(n-1/2), spins s^(n-1/2)):

1. gather: E and B at every particle by first-order (cloud-in-cell)
   interpolation, each component from its own staggered Yee position;
2. Boris push of u = gamma*beta: half electric kick, magnetic rotation by the
   implicit-midpoint (Cayley) map, half electric kick;
3. Thomas-BMT spin precession, section 2 Eq. 1 with the precession vector of
   Eq. 2 and the coefficients of Eq. 3, integrated by the same implicit
   midpoint map, with gamma and v taken at the time-centred Boris values;
4. move: x^(n+1) = x^n + dt*u^(n+1/2)/gamma, periodic in every axis;
5. charge-conserving current deposit (Esirkepov's density decomposition for
   the CIC shape); in 2D3V J_z uses the time average of the linearly
   interpolated shape product;
6. Yee field update: B half step, E full step with -J, B half step.

Diagnostics: the polarization of section 2 Eq. 4 (mean spin over an ensemble
selected by species and kinetic-energy window), energies, the charge density
and the discrete div E - rho residual; binned: the energy spectrum with the
Eq. 4 polarization of every energy bin (the spectra and polarization-versus-
energy plots of section 3), weighted position-momentum histograms and the
number density of a species.

Units are normalized laser units (time 1/omega0, length c/omega0, fields
m_e c omega0/e, densities n_c).  In them q/(mc) of Eq. 2 becomes r = Z/mu and
v/c becomes beta.  Every function here is pinned by the tests in
``tests/test_oracle_*.py``.
"""

import itertools

import numpy as np

ME_C2_MEV = 0.51099895   # electron rest energy, for kinetic-energy windows

# Half-cell offset of each component's Yee position along (x, y, z).
E_STAGGER = ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5))
B_STAGGER = ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))

# Array axis of each spatial direction in a (nz, ny, nx) field array.
AXIS = (2, 1, 0)


class Grid:
    """Yee grid: ``ndim`` = 2 (x, y; d/dz = 0) or 3; n and d per axis.

    Periodic in every axis, or with ``open_x`` open along x: the fields
    beyond the two x faces read as zero for the gather, current deposited
    there is lost, particles crossing them leave the box, and the field
    update takes its ghost columns from Mur's absorbing condition (see
    MurState)."""

    def __init__(self, ndim, n, d, dt, open_x=False):
        self.open_x = bool(open_x)
        self.ndim = int(ndim)
        self.n = tuple(int(v) for v in n)
        if self.ndim == 2:
            self.n = (self.n[0], self.n[1], 1)
        self.d = tuple(float(v) for v in d)
        self.dt = float(dt)
        self.shape = (self.n[2], self.n[1], self.n[0])
        self.cell_volume = float(np.prod(self.d[:self.ndim]))


# ---------------------------------------------------------------- gather

def interpolate(F, xi, stagger, grid):
    """CIC value of one staggered component F (nz, ny, nx) at positions xi.

    xi holds positions in cell units (x/dx, y/dy, z/dz), shape (N, 3).  Along
    each axis the component sits at index + stagger; the two nearest such
    points straddle the particle and get the linear weights.
    """
    idx, frac = [], []
    for a in range(grid.ndim):
        p = xi[:, a] - stagger[a]
        i = np.floor(p)
        idx.append(i.astype(np.int64))
        frac.append(p - i)
    val = np.zeros(xi.shape[0])
    for corner in itertools.product((0, 1), repeat=grid.ndim):
        weight = np.ones(xi.shape[0])
        ind = [np.zeros(xi.shape[0], dtype=np.int64)] * 3
        inside = np.ones(xi.shape[0], dtype=bool)
        for a in range(grid.ndim):
            weight = weight * (frac[a] if corner[a] else 1.0 - frac[a])
            raw = idx[a] + corner[a]
            if a == 0 and grid.open_x:
                inside = (raw >= 0) & (raw < grid.n[0])
            ind[a] = raw % grid.n[a]
        val += np.where(inside, weight * F[ind[2], ind[1], ind[0]], 0.0)
    return val


def gather(E, B, xi, grid):
    """E and B at the particles, each (N, 3)."""
    Ep = np.stack([interpolate(E[c], xi, E_STAGGER[c], grid) for c in range(3)], axis=1)
    Bp = np.stack([interpolate(B[c], xi, B_STAGGER[c], grid) for c in range(3)], axis=1)
    return Ep, Bp


# ---------------------------------------------------------------- push

def cross_matrix(w):
    """Batched matrix K with K @ x = w x x."""
    K = np.zeros(w.shape[:-1] + (3, 3), dtype=np.result_type(w, np.float64))
    K[..., 0, 1] = -w[..., 2]
    K[..., 0, 2] = w[..., 1]
    K[..., 1, 0] = w[..., 2]
    K[..., 1, 2] = -w[..., 0]
    K[..., 2, 0] = -w[..., 1]
    K[..., 2, 1] = w[..., 0]
    return K


def midpoint_rotate(v, w, dt):
    """One step of dv/dt = v x w by the implicit midpoint rule.

    Solves (v+ - v)/dt = (v+ + v)/2 x w exactly (a 3x3 linear solve per
    particle), which is the Cayley rotation of v about w.
    """
    K = cross_matrix(w) * (0.5 * dt)
    eye = np.eye(3)
    rhs = np.einsum("nij,nj->ni", eye - K, v)
    return np.linalg.solve(eye + K, rhs[..., None])[..., 0]


def boris(u, Ep, Bp, r, dt):
    """Relativistic Boris push of u = gamma*beta, for du/dt = r (E + beta x B).

    Returns (u_minus, u_plus, u_new, gamma_minus): the momentum after the first
    half electric kick, after the magnetic rotation, after the second kick,
    and the Lorentz factor during the rotation.
    """
    eps = 0.5 * r * dt
    u_minus = u + eps * Ep
    gamma_minus = np.sqrt(1.0 + np.sum(u_minus * u_minus, axis=1))
    u_plus = midpoint_rotate(u_minus, r * Bp / gamma_minus[:, None], dt)
    u_new = u_plus + eps * Ep
    return u_minus, u_plus, u_new, gamma_minus


def tbmt_omega(u_minus, u_plus, gamma_minus, Ep, Bp, r, a):
    """Precession vector Omega of section 2 Eq. 2 with the Eq. 3 coefficients.

    In normalized units q/(mc) -> r and v/c -> beta.  gamma is the Boris
    rotation's gamma_minus and beta the mean of the rotation's end points over
    gamma_minus: both at the time of E^n, B^n.
    """
    gamma = gamma_minus[:, None]
    beta = (u_minus + u_plus) / (2.0 * gamma)
    Omega_B = a + 1.0 / gamma
    Omega_v = a * gamma / (gamma + 1.0)
    Omega_E = a + 1.0 / (1.0 + gamma)
    beta_dot_B = np.sum(beta * Bp, axis=1)[:, None]
    return r * (Omega_B * Bp - Omega_v * beta_dot_B * beta - Omega_E * np.cross(beta, Ep))


def spin_precess(s, Omega, dt):
    """One step of section 2 Eq. 1, ds/dt = -Omega x s = s x Omega."""
    return midpoint_rotate(s, Omega, dt)


def move(xi, u_new, grid):
    """Positions (cell units) after dt at velocity u/gamma; not yet wrapped."""
    gamma = np.sqrt(1.0 + np.sum(u_new * u_new, axis=1))
    xi_new = xi.copy()
    for a in range(grid.ndim):
        xi_new[:, a] = xi[:, a] + grid.dt * u_new[:, a] / (gamma * grid.d[a])
    return xi_new


def wrap(xi, grid):
    """Periodic wrap of positions into [0, n) along every active periodic axis."""
    out = xi.copy()
    for a in range(grid.ndim):
        if a == 0 and grid.open_x:
            continue
        p = np.mod(xi[:, a], grid.n[a])
        out[:, a] = np.where(p >= grid.n[a], p - grid.n[a], p)
    return out


# ---------------------------------------------------------------- deposit

def shape_pair(p0, p1):
    """CIC shape factors of the old and new position on three common nodes.

    p0, p1: positions along one axis in cell units, |floor p1 - floor p0| <= 1.
    Returns (b, S0, S1) with node b + k carrying S0[:, k] before and S1[:, k]
    after the move, k = 0, 1, 2.
    """
    i0 = np.floor(p0)
    i1 = np.floor(p1)
    if np.any(np.abs(i1 - i0) > 1):
        raise ValueError("a particle crossed more than one cell in one step")
    b = np.minimum(i0, i1)
    n = p0.shape[0]
    rows = np.arange(n)
    S0 = np.zeros((n, 3))
    S1 = np.zeros((n, 3))
    k0 = (i0 - b).astype(np.int64)
    k1 = (i1 - b).astype(np.int64)
    S0[rows, k0] = 1.0 - (p0 - i0)
    S0[rows, k0 + 1] = p0 - i0
    S1[rows, k1] = 1.0 - (p1 - i1)
    S1[rows, k1 + 1] = p1 - i1
    return b.astype(np.int64), S0, S1


def _scatter(F, ind, values, grid):
    """F[ind] += values with periodic indices; ind is a list (ix, iy, iz).
    With an open x axis, values at x indices outside [0, n) are dropped."""
    values = np.broadcast_to(values, np.shape(ind[0]))
    if grid.open_x:
        keep = (ind[0] >= 0) & (ind[0] < grid.n[0])
        ind = [np.broadcast_to(i, keep.shape)[keep] for i in ind]
        values = values[keep]
    flat = ((ind[2] % grid.n[2]) * grid.n[1] + (ind[1] % grid.n[1])) * grid.n[0] \
        + (ind[0] % grid.n[0])
    F += np.bincount(flat.ravel(), weights=values.ravel(),
                     minlength=F.size).reshape(F.shape)


def deposit(J, xi0, xi1, Zw, vz, grid):
    """Add the current of particles moving xi0 -> xi1 (cell units, unwrapped).

    J_a at the staggered position of E_a.  The x and y (and z in 3D) currents
    are Esirkepov's: with DS = S1 - S0 per axis,
      W_x = DS_x (S0_y S0_z + DS_y S0_z/2 + S0_y DS_z/2 + DS_y DS_z/3)
    (2D: W_x = DS_x (S0_y + DS_y/2)), and J_x(i+1/2) - J_x(i-1/2) =
    -Zw dx/dt W_x(i), summed from the low side where J is zero, so that
    (rho^(n+1) - rho^n)/dt + div J = 0 holds exactly on every node.  In 2D3V
    J_z at the node is Zw v_z times S0x S0y + (DSx S0y + S0x DSy)/2 + DSx DSy/3.
    """
    dt = grid.dt
    bx, S0x, S1x = shape_pair(xi0[:, 0], xi1[:, 0])
    by, S0y, S1y = shape_pair(xi0[:, 1], xi1[:, 1])
    DSx = S1x - S0x
    DSy = S1y - S0y
    k = np.arange(3)
    if grid.ndim == 2:
        Wx = DSx[:, :, None] * (S0y + 0.5 * DSy)[:, None, :]
        Wy = (S0x + 0.5 * DSx)[:, :, None] * DSy[:, None, :]
        Wz = (S0x[:, :, None] * S0y[:, None, :]
              + 0.5 * (DSx[:, :, None] * S0y[:, None, :] + S0x[:, :, None] * DSy[:, None, :])
              + DSx[:, :, None] * DSy[:, None, :] / 3.0)
        Jx = -(Zw * grid.d[0] / dt)[:, None, None] * np.cumsum(Wx, axis=1)
        Jy = -(Zw * grid.d[1] / dt)[:, None, None] * np.cumsum(Wy, axis=2)
        Jz = (Zw * vz)[:, None, None] * Wz
        shp = Jx.shape
        ix = np.broadcast_to(bx[:, None, None] + k[None, :, None], shp)
        iy = np.broadcast_to(by[:, None, None] + k[None, None, :], shp)
        iz = np.zeros(shp, dtype=np.int64)
        for c, Jc in enumerate((Jx, Jy, Jz)):
            _scatter(J[c], [ix, iy, iz], Jc, grid)
        return
    bz, S0z, S1z = shape_pair(xi0[:, 2], xi1[:, 2])
    DSz = S1z - S0z
    X = (slice(None), slice(None), None, None)
    Y = (slice(None), None, slice(None), None)
    Z = (slice(None), None, None, slice(None))
    Wx = DSx[X] * (S0y[Y] * S0z[Z] + 0.5 * DSy[Y] * S0z[Z] + 0.5 * S0y[Y] * DSz[Z]
                   + DSy[Y] * DSz[Z] / 3.0)
    Wy = DSy[Y] * (S0x[X] * S0z[Z] + 0.5 * DSx[X] * S0z[Z] + 0.5 * S0x[X] * DSz[Z]
                   + DSx[X] * DSz[Z] / 3.0)
    Wz = DSz[Z] * (S0x[X] * S0y[Y] + 0.5 * DSx[X] * S0y[Y] + 0.5 * S0x[X] * DSy[Y]
                   + DSx[X] * DSy[Y] / 3.0)
    Jx = -(Zw * grid.d[0] / dt)[:, None, None, None] * np.cumsum(Wx, axis=1)
    Jy = -(Zw * grid.d[1] / dt)[:, None, None, None] * np.cumsum(Wy, axis=2)
    Jz = -(Zw * grid.d[2] / dt)[:, None, None, None] * np.cumsum(Wz, axis=3)
    shp = Jx.shape
    ix = np.broadcast_to(bx[:, None, None, None] + k[None, :, None, None], shp)
    iy = np.broadcast_to(by[:, None, None, None] + k[None, None, :, None], shp)
    iz = np.broadcast_to(bz[:, None, None, None] + k[None, None, None, :], shp)
    for c, Jc in enumerate((Jx, Jy, Jz)):
        _scatter(J[c], [ix, iy, iz], Jc, grid)


def charge_density(xi, Zw, grid):
    """rho on the nodes by CIC deposit of charge Z*w."""
    rho = np.zeros(grid.shape)
    idx, frac = [], []
    for a in range(grid.ndim):
        i = np.floor(xi[:, a])
        idx.append(i.astype(np.int64))
        frac.append(xi[:, a] - i)
    for corner in itertools.product((0, 1), repeat=grid.ndim):
        weight = Zw.copy()
        ind = [np.zeros(xi.shape[0], dtype=np.int64)] * 3
        for a in range(grid.ndim):
            weight = weight * (frac[a] if corner[a] else 1.0 - frac[a])
            ind[a] = idx[a] + corner[a]
        _scatter(rho, ind, weight, grid)
    return rho


# ---------------------------------------------------------------- Yee

def _dplus(F, a, grid, ghost=None):
    """Forward difference along axis a: (F[i+1] - F[i]) / d_a (0 along z in 2D).
    Along an open x axis F[n] is the ghost column (zero if None)."""
    if a == 0 and grid.open_x:
        g = np.zeros_like(F[..., :1]) if ghost is None else ghost
        return (np.concatenate([F[..., 1:], g], axis=-1) - F) / grid.d[0]
    return (np.roll(F, -1, axis=AXIS[a]) - F) / grid.d[a]


def _dminus(F, a, grid, ghost=None):
    """Backward difference along axis a: (F[i] - F[i-1]) / d_a.  Along an open
    x axis F[-1] is the ghost column (zero if None)."""
    if a == 0 and grid.open_x:
        g = np.zeros_like(F[..., :1]) if ghost is None else ghost
        return (F - np.concatenate([g, F[..., :-1]], axis=-1)) / grid.d[0]
    return (F - np.roll(F, 1, axis=AXIS[a])) / grid.d[a]


class MurState:
    """First-order Mur absorbing condition at the two open x faces.

    Beyond each face the Yee update needs one ghost column: E_y and E_z at
    x index n for the B update, B_y and B_z at x index -1 for the E update.
    Each ghost follows the one-way wave equation of a wave leaving through
    its face, discretized midway between the ghost and the first column
    inside and midway between two time levels (Mur 1981):
        ghost(new) = inside(old) + k (inside(new) - ghost(old)),
        k = (c dt - dx) / (c dt + dx),
    with E at integer and B at half-integer times.  The state holds each
    face's ghost and first inside column at the last time level; reset()
    starts both from the first inside column (at the start and after every
    shift of a moving window)."""

    def __init__(self, E, B, grid):
        self.k = (grid.dt - grid.d[0]) / (grid.dt + grid.d[0])
        self.reset(E, B)

    def reset(self, E, B):
        self.hi_ghost = np.stack([E[1][..., -1:], E[2][..., -1:]])
        self.hi_prev = self.hi_ghost.copy()
        self.lo_ghost = np.stack([B[1][..., :1], B[2][..., :1]])
        self.lo_prev = self.lo_ghost.copy()

    def advance_low(self, B):
        """B_y, B_z ghosts at the new half step from the first B column."""
        inside = np.stack([B[1][..., :1], B[2][..., :1]])
        self.lo_ghost = self.lo_prev + self.k * (inside - self.lo_ghost)
        self.lo_prev = inside
        return self.lo_ghost

    def advance_high(self, E):
        """E_y, E_z ghosts at the new integer step from the last E column."""
        inside = np.stack([E[1][..., -1:], E[2][..., -1:]])
        self.hi_ghost = self.hi_prev + self.k * (inside - self.hi_ghost)
        self.hi_prev = inside
        return self.hi_ghost


def curl_E(E, grid, ghost=None):
    """curl E at the B positions (ghost: E_y, E_z beyond an open high x face)."""
    gy = gz = None
    if grid.open_x:
        gy, gz = ghost[0], ghost[1]
    return np.stack([
        _dplus(E[2], 1, grid) - _dplus(E[1], 2, grid),
        _dplus(E[0], 2, grid) - _dplus(E[2], 0, grid, gz),
        _dplus(E[1], 0, grid, gy) - _dplus(E[0], 1, grid),
    ])


def curl_B(B, grid, ghost=None):
    """curl B at the E positions (ghost: B_y, B_z beyond an open low x face)."""
    gy = gz = None
    if grid.open_x:
        gy, gz = ghost[0], ghost[1]
    return np.stack([
        _dminus(B[2], 1, grid) - _dminus(B[1], 2, grid),
        _dminus(B[0], 2, grid) - _dminus(B[2], 0, grid, gz),
        _dminus(B[1], 0, grid, gy) - _dminus(B[0], 1, grid),
    ])


def div_E(E, grid):
    """Discrete divergence of E at the nodes (E beyond an open x face is 0)."""
    return _dminus(E[0], 0, grid) + _dminus(E[1], 1, grid) + _dminus(E[2], 2, grid)


def yee_step(E, B, J, grid, mur=None):
    """B -= dt/2 curl E; E += dt (curl B - J); B -= dt/2 curl E (in place).
    With open x faces the ghost columns come from the Mur state ``mur``."""
    dt = grid.dt
    if not grid.open_x:
        B -= 0.5 * dt * curl_E(E, grid)
        E += dt * (curl_B(B, grid) - J)
        B -= 0.5 * dt * curl_E(E, grid)
        return
    B -= 0.5 * dt * curl_E(E, grid, mur.hi_ghost)
    E += dt * (curl_B(B, grid, mur.advance_low(B)) - J)
    B -= 0.5 * dt * curl_E(E, grid, mur.advance_high(E))


# ---------------------------------------------------------------- Eq. 4

def kinetic_energy_mev(u, mu):
    """mu (gamma - 1) m_e c^2 in MeV."""
    gamma = np.sqrt(1.0 + np.sum(u * u, axis=1))
    return mu * (gamma - 1.0) * ME_C2_MEV


def polarization(s, selected):
    """Section 2 Eq. 4: P = (1/N) sum_i s_i over the selected particles."""
    N = int(np.count_nonzero(selected))
    if N == 0:
        return np.zeros(3), 0
    return s[selected].sum(axis=0) / N, N


# ---------------------------------------------------------------- binned diagnostics

def kinetic_energy_binned(u, mu):
    """mu (gamma - 1) m_e c^2 in MeV with |u|^2 summed as (ux^2 + uy^2) + uz^2,
    the order the binned diagnostics fix so that bin decisions are
    reproducible bit for bit."""
    u2 = (u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1]) + u[:, 2] * u[:, 2]
    return mu * (np.sqrt(1.0 + u2) - 1.0) * ME_C2_MEV


def bin_index(v, lo, hi, nbins):
    """Equal bins over [lo, hi): index floor((v - lo) / (hi - lo) * nbins),
    capped at nbins - 1; -1 for values outside [lo, hi)."""
    inside = (v >= lo) & (v < hi)
    b = np.floor((v - lo) / (hi - lo) * nbins)
    b = np.minimum(b, nbins - 1)
    return np.where(inside, b, -1).astype(np.int64)


def spectrum(u, s, w, mu, emin, emax, nbins):
    """Energy spectrum with the polarization of section 2 Eq. 4 per bin: for
    nbins equal bins of kinetic energy over [emin, emax) MeV, the number of
    macro-particles, the sum of their weights and the sum of their spin
    vectors (so the polarization of bin b is spin[b] / count[b])."""
    b = bin_index(kinetic_energy_binned(u, mu), emin, emax, nbins)
    keep = b >= 0
    count = np.bincount(b[keep], minlength=nbins).astype(np.float64)
    weight = np.bincount(b[keep], weights=w[keep], minlength=nbins)
    spin = np.stack([np.bincount(b[keep], weights=s[keep, k], minlength=nbins)
                     for k in range(3)], axis=1)
    return count, weight, spin


def phase_space(x, p, w, xmin, xmax, nx, pmin, pmax, np_):
    """Weighted 2D histogram over (position, momentum): nx by np_ equal bins
    over [xmin, xmax) x [pmin, pmax); out[ix, ip] = sum of w."""
    bx = bin_index(x, xmin, xmax, nx)
    bp = bin_index(p, pmin, pmax, np_)
    keep = (bx >= 0) & (bp >= 0)
    flat = bx[keep] * np_ + bp[keep]
    return np.bincount(flat, weights=w[keep], minlength=nx * np_).reshape(nx, np_)


# ---------------------------------------------------------------- driver

class Sim:
    """The oracle's counterpart of the library calls: init, step, polarization,
    fields, particles, energy.

    ``spec`` needs ndim, n, d, dt and species (Z, mu, a); ``state`` holds the
    initial particles, one (N, 10) array per species with columns
    x y z ux uy uz sx sy sz w, and fields (6, nz, ny, nx) = Ex Ey Ez Bx By Bz.
    """

    CHUNK = 1 << 20

    def __init__(self, spec, state, test_particle=False, store_fp32=False, window=None):
        # window: a co-moving window (see _advance_window) with open x faces;
        # a dict with speed, shift_cells, ppc, n0, ramp_start, ramp_len, s0
        self.window = dict(window) if window is not None else None
        self.grid = Grid(spec["ndim"], spec["n"], spec["d"], spec["dt"], open_x=window is not None)
        g = self.grid
        self.test_particle = bool(test_particle)
        # store_fp32: after every step, round each particle's in-cell offsets,
        # momentum and spin to float32 (weights once at start), i.e. the exact
        # method with float32 particle storage.  It bounds the error that any
        # float32 particle store must incur; the default is plain float64.
        self.store_fp32 = bool(store_fp32)
        self.species = [(float(sp["Z"]), float(sp["mu"]), float(sp["a"]))
                        for sp in spec["species"]]
        self.xi, self.u, self.s, self.w = [], [], [], []
        for arr in state["particles"]:
            arr = np.asarray(arr, dtype=np.float64)
            xi = np.zeros((arr.shape[0], 3))
            for a in range(g.ndim):
                xi[:, a] = arr[:, a] / g.d[a]
            self.xi.append(wrap(xi, g))
            self.u.append(arr[:, 3:6].copy())
            self.s.append(arr[:, 6:9].copy())
            self.w.append(arr[:, 9].copy())
        if self.store_fp32:
            for k in range(len(self.xi)):
                self._round_fp32(k, 0, self.xi[k].shape[0])
                self.w[k] = self.w[k].astype(np.float32).astype(np.float64)
        # particle ids: the row index of the initial state, then the ids of
        # injected particles (see _inject)
        self.ids = [np.arange(x.shape[0], dtype=np.int64) for x in self.xi]
        self.next_id = [x.shape[0] for x in self.xi]
        self.shifts = 0
        F = np.asarray(state["fields"], dtype=np.float64).reshape((6,) + g.shape)
        self.E = F[0:3].copy()
        self.B = F[3:6].copy()
        self.J = np.zeros((3,) + g.shape)
        self.mur = MurState(self.E, self.B, g) if g.open_x else None
        self.nstep = 0
        self.window_step0 = 0
        self.residual0 = div_E(self.E, g) - self.rho()

    def rho(self):
        g = self.grid
        rho = np.zeros(g.shape)
        for sp, xi, w in zip(self.species, self.xi, self.w):
            rho += charge_density(xi, sp[0] * w, g)
        return rho

    def _round_fp32(self, k, lo, hi):
        """Round the stored state of particles lo:hi of species k to float32."""
        def f32(a):
            return a.astype(np.float32).astype(np.float64)
        xi = self.xi[k][lo:hi]
        for a in range(self.grid.ndim):
            fl = np.floor(xi[:, a])
            off = f32(xi[:, a] - fl)
            up = off >= 1.0                 # rounded up to the next cell edge
            fl = np.where(up, fl + 1.0, fl)
            off = np.where(up, 0.0, off)
            if not (a == 0 and self.grid.open_x):
                fl = np.mod(fl, self.grid.n[a])
            xi[:, a] = fl + off
        self.u[k][lo:hi] = f32(self.u[k][lo:hi])
        self.s[k][lo:hi] = f32(self.s[k][lo:hi])

    def push_species(self, k, lo, hi, deposit_current=True):
        """Gather, Boris, T-BMT, move and deposit for particles lo:hi of species k."""
        g = self.grid
        Z, mu, a = self.species[k]
        r = Z / mu
        xi = self.xi[k][lo:hi]
        Ep, Bp = gather(self.E, self.B, xi, g)
        u_minus, u_plus, u_new, gamma_minus = boris(self.u[k][lo:hi], Ep, Bp, r, g.dt)
        Omega = tbmt_omega(u_minus, u_plus, gamma_minus, Ep, Bp, r, a)
        self.s[k][lo:hi] = spin_precess(self.s[k][lo:hi], Omega, g.dt)
        self.u[k][lo:hi] = u_new
        xi_new = move(xi, u_new, g)
        if deposit_current:
            gamma = np.sqrt(1.0 + np.sum(u_new * u_new, axis=1))
            deposit(self.J, xi, xi_new, Z * self.w[k][lo:hi], u_new[:, 2] / gamma, g)
        self.xi[k][lo:hi] = wrap(xi_new, g)
        if self.store_fp32:
            self._round_fp32(k, lo, hi)

    def step(self, nsteps=1):
        for _ in range(nsteps):
            self.J[...] = 0.0
            for k in range(len(self.species)):
                n = self.xi[k].shape[0]
                for lo in range(0, n, self.CHUNK):
                    self.push_species(k, lo, min(n, lo + self.CHUNK),
                                      deposit_current=not self.test_particle)
                if self.grid.open_x:
                    # particles that crossed an x face leave the box
                    x = self.xi[k][:, 0]
                    self._keep(k, (x >= 0.0) & (x < self.grid.n[0]))
            if not self.test_particle:
                yee_step(self.E, self.B, self.J, self.grid, self.mur)
            self.nstep += 1
            if self.window is not None:
                self._advance_window()

    def _keep(self, k, mask):
        for arrs in (self.xi, self.u, self.s, self.w, self.ids):
            arrs[k] = arrs[k][mask]

    # ------------------------------------------------------------ moving window

    def window_density(self, x):
        """Density of the plasma ahead of the window at lab-frame x: n0 times
        a linear ramp from ramp_start over ramp_len (a step if ramp_len is 0)."""
        w = self.window
        if w["ramp_len"] > 0.0:
            return w["n0"] * np.clip((x - w["ramp_start"]) / w["ramp_len"], 0.0, 1.0)
        return np.where(x >= w["ramp_start"], w["n0"], 0.0)

    def enable_window(self, window):
        """Open the x faces and start a window now (the travel and the lab
        frame count from this step); the div E - rho reference is taken again
        with the open faces."""
        self.window = dict(window)
        self.grid.open_x = True
        self.mur = MurState(self.E, self.B, self.grid)
        self.window_step0 = self.nstep
        self.shifts = 0
        self.residual0 = div_E(self.E, self.grid) - self.rho()

    def _advance_window(self):
        """After step n (counted from the window's start) the window has
        moved n speed dt; every whole shift_cells cells of that it shifts the
        box by shift_cells cells."""
        w, g = self.window, self.grid
        S = int(w["shift_cells"])
        while (self.nstep - self.window_step0) * w["speed"] * g.dt >= (self.shifts + 1) * S * g.d[0]:
            self._shift(S)

    def _shift(self, S):
        """Move the box S cells along +x: fields, currents and particles move
        S cells towards -x in box coordinates, the first S columns leave, the
        last S columns start with zero fields and fresh plasma."""
        g = self.grid
        nx = g.n[0]
        for F in (self.E, self.B, self.J):
            F[..., :nx - S] = F[..., S:].copy()
            F[..., nx - S:] = 0.0
        self.mur.reset(self.E, self.B)
        self.shifts += 1
        for k in range(len(self.species)):
            self.xi[k][:, 0] -= S
            self._keep(k, self.xi[k][:, 0] >= 0.0)
        self._inject(S)

    def _inject(self, S):
        """Cold plasma in the new columns nx-S .. nx-1: in every cell whose
        centre sees density n > 0 (lab frame), ppc particles of every species
        at in-cell offset (q + 1/2)/ppc along every axis, u = 0, spin s0,
        weight n/ppc.  Particle (column col, cell row y, z, q) of a species
        gets id next_id + ((z ny + y) S + col) ppc + q; next_id then advances
        by nz ny S ppc whether or not every cell received particles."""
        w, g = self.window, self.grid
        ppc = int(w["ppc"])
        if ppc <= 0:
            return
        nx, ny = g.n[0], g.n[1]
        nz = g.n[2] if g.ndim == 3 else 1
        origin = self.shifts * S
        cz, cy, col, q = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(S), np.arange(ppc),
                                     indexing="ij")
        cz, cy, col, q = cz.ravel(), cy.ravel(), col.ravel(), q.ravel()
        cx = nx - S + col
        dens = self.window_density((cx + 0.5 + origin) * g.d[0])
        on = dens > 0.0
        f = (q + 0.5) / ppc
        xi = np.zeros((cx.size, 3))
        xi[:, 0] = cx + f
        xi[:, 1] = cy + f
        if g.ndim == 3:
            xi[:, 2] = cz + f
        s0 = np.asarray(w["s0"], dtype=np.float64)
        for k in range(len(self.species)):
            ids = self.next_id[k] + ((cz * ny + cy) * S + col) * ppc + q
            m = int(on.sum())
            self.xi[k] = np.concatenate([self.xi[k], xi[on]])
            self.u[k] = np.concatenate([self.u[k], np.zeros((m, 3))])
            self.s[k] = np.concatenate([self.s[k], np.tile(s0, (m, 1))])
            self.w[k] = np.concatenate([self.w[k], dens[on] / ppc])
            self.ids[k] = np.concatenate([self.ids[k], ids[on]])
            self.next_id[k] += nz * ny * S * ppc

    def select(self, species, emin, emax):
        """Per species, the mask of particles with emin <= E_kin [MeV] < emax."""
        masks = []
        for k, (Z, mu, a) in enumerate(self.species):
            if species not in (-1, k):
                masks.append(np.zeros(self.u[k].shape[0], dtype=bool))
                continue
            ek = kinetic_energy_mev(self.u[k], mu)
            masks.append((ek >= emin) & (ek < emax))
        return masks

    def polarization(self, species=-1, emin=-np.inf, emax=np.inf):
        masks = self.select(species, emin, emax)
        s = np.concatenate(self.s, axis=0)
        return polarization(s, np.concatenate(masks))

    def spectrum(self, species, emin, emax, nbins):
        """Binned energy spectrum of one species (-1: all), see spectrum()."""
        out = [np.zeros(nbins), np.zeros(nbins), np.zeros((nbins, 3))]
        for k, (Z, mu, a) in enumerate(self.species):
            if species not in (-1, k):
                continue
            part = spectrum(self.u[k], self.s[k], self.w[k], mu, emin, emax, nbins)
            for q in range(3):
                out[q] += part[q]
        return tuple(out)

    def phase_space(self, species, axis, xmin, xmax, nx, comp, pmin, pmax, np_):
        """Weighted histogram of position x_axis (c/omega0) against mu u_comp
        (m_e c) for one species."""
        Z, mu, a = self.species[species]
        x = self.xi[species][:, axis] * self.grid.d[axis]
        return phase_space(x, mu * self.u[species][:, comp], self.w[species],
                           xmin, xmax, nx, pmin, pmax, np_)

    def density(self, species):
        """Number density of one species on the nodes (CIC of w)."""
        return charge_density(self.xi[species], self.w[species], self.grid)

    def fields(self):
        """(10, nz, ny, nx): Ex Ey Ez Bx By Bz Jx Jy Jz rho."""
        return np.concatenate([self.E, self.B, self.J, self.rho()[None]], axis=0)

    def particles(self, k):
        """(N, 11): id x y z ux uy uz sx sy sz w, sorted by id (positions in
        box coordinates)."""
        g = self.grid
        n = self.xi[k].shape[0]
        out = np.zeros((n, 11))
        out[:, 0] = self.ids[k]
        for a in range(g.ndim):
            out[:, 1 + a] = self.xi[k][:, a] * g.d[a]
        out[:, 4:7] = self.u[k]
        out[:, 7:10] = self.s[k]
        out[:, 10] = self.w[k]
        return out[np.argsort(self.ids[k], kind="stable")]

    def energy(self):
        """[kinetic energy per species ..., field energy, max|delta(div E - rho)|].

        Energies in m_e c^2 n_c times (c/omega0)^ndim: mu (gamma-1) w V per
        particle and (E^2 + B^2)/2 V per cell, V the cell volume.
        """
        g = self.grid
        out = []
        for (Z, mu, a), u, w in zip(self.species, self.u, self.w):
            gamma = np.sqrt(1.0 + np.sum(u * u, axis=1))
            out.append(float(np.sum(mu * (gamma - 1.0) * w) * g.cell_volume))
        out.append(float(0.5 * (np.sum(self.E ** 2) + np.sum(self.B ** 2)) * g.cell_volume))
        res = div_E(self.E, g) - self.rho()
        out.append(float(np.max(np.abs(res - self.residual0))))
        return np.array(out)
