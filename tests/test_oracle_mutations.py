"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
catch every one of them.

Each mutant replaces one snippet of one oracle function's source (a dropped
term, a flipped sign, a wrong index or stagger, a transposed operand), and
the named pin tests must then fail.  A mutant that survives means the pins
leave that part of the oracle unchecked.
"""

import inspect
import textwrap

import numpy as np
import pytest

from oracle import pic as O

import test_oracle_diag as TD
import test_oracle_grid as TG
import test_oracle_push as TP
import test_oracle_window as TW


def _run_all(checks):
    for chk in checks:
        try:
            chk()
        except Exception:   # noqa: BLE001 - any failure kills the mutant
            return True
    return False


PUSH = [
    lambda: TP.test_T1_boris_gyration_phase(-1.0, 5.0),
    lambda: TP.test_T2_g_minus_2_discrete_and_continuum(1.793, 20.0),
    TP.test_T3_a_zero_locks_spin_to_momentum,
    lambda: TP.test_T4_longitudinal_field(1.793),
    TP.test_T5_pure_E_parallel_to_u,
    lambda: TP.test_helicity_law_jackson(1.793, -1.0),
    lambda: TP.test_helicity_law_jackson(0.0, 0.37),
    TP.test_E_cross_B_drift,
]
GRID = [
    lambda: TG.test_gather_reproduces_linear_fields_from_staggered_positions(2),
    lambda: TG.test_gather_reproduces_linear_fields_from_staggered_positions(3),
    lambda: TG.test_T8_deposit_satisfies_discrete_continuity(2),
    lambda: TG.test_T8_deposit_satisfies_discrete_continuity(3),
    lambda: TG.test_T9_single_particle_current_sums(2),
    lambda: TG.test_T9_single_particle_current_sums(3),
    TG.test_jz_2d3v_diagonal_move_by_hand,
    TG.test_jz_2d3v_skewed_move_by_hand,
    lambda: TG.test_T10_yee_standing_mode_dispersion(2, 2, (1, 2, 0)),
    lambda: TG.test_T10_yee_standing_mode_dispersion(3, 0, (0, 2, 1)),
    lambda: TG.test_T10_yee_standing_mode_dispersion(3, 1, (2, 0, 3)),
    lambda: TG.test_T10_yee_travelling_wave_moves_along_E_cross_B(1),
    lambda: TG.test_T8_div_E_minus_rho_constant_over_a_run("small2d"),
]
DIAG = [
    TD.test_free_streaming_moves_by_u_over_gamma_and_wraps,
    lambda: TD.test_polarization_eq4_against_loops(-1, -np.inf, np.inf),
    lambda: TD.test_polarization_eq4_against_loops(0, 0.05, 0.5),
    lambda: TD.test_polarization_eq4_against_loops(1, 0.2, 1.0),
    TD.test_polarization_at_start_equals_s0,
    TD.test_energy_field_sum_and_kinetic_by_hand,
]

WINDOW = [
    TW.test_open_faces_stay_stable,
    TW.test_oblique_wave_leaves,
    lambda: TW.test_open_faces_absorb_leaving_pulses(1, "y"),
    lambda: TW.test_open_faces_absorb_leaving_pulses(-1, "y"),
    lambda: TW.test_open_faces_absorb_leaving_pulses(1, "z"),
    lambda: TW.test_open_faces_absorb_leaving_pulses(-1, "z"),
    TW.test_window_follows_a_vacuum_pulse,
    TW.test_cold_plasma_in_a_moving_window_stays_uniform,
    TW.test_injected_weights_follow_the_ramp,
    TW.test_particle_leaving_the_box_is_removed_with_interior_continuity,
    TW.test_shift_moves_fields_and_clears_new_columns,
    TW.test_gather_sees_nothing_beyond_the_faces,
    TW.test_no_current_crosses_a_face,
    TW.test_window_started_later_counts_travel_from_its_start,
]

MUTANTS = [
    ("tbmt_omega", "Omega_v * beta_dot_B * beta", "0.0 * beta_dot_B * beta", PUSH),
    ("tbmt_omega", "- Omega_E * np.cross(beta, Ep)", "+ Omega_E * np.cross(beta, Ep)", PUSH),
    ("tbmt_omega", "np.cross(beta, Ep)", "np.cross(Ep, beta)", PUSH),
    ("tbmt_omega", "Omega_E = a + 1.0 / (1.0 + gamma)", "Omega_E = a + 1.0 / gamma", PUSH),
    ("tbmt_omega", "Omega_B = a + 1.0 / gamma", "Omega_B = a + 1.0", PUSH),
    ("tbmt_omega", "Omega_v = a * gamma / (gamma + 1.0)", "Omega_v = a / (gamma + 1.0)", PUSH),
    ("tbmt_omega", "(u_minus + u_plus) / (2.0 * gamma)", "(u_minus + u_plus) / 2.0", PUSH),
    ("tbmt_omega", "(u_minus + u_plus)", "(2.0 * u_minus)", PUSH),
    ("spin_precess", "midpoint_rotate(s, Omega, dt)", "midpoint_rotate(s, -Omega, dt)", PUSH),
    ("midpoint_rotate", "np.linalg.solve(eye + K", "np.linalg.solve(eye - K", PUSH),
    ("boris", "r * Bp / gamma_minus[:, None]", "r * Bp", PUSH),
    ("boris", "u_new = u_plus + eps * Ep", "u_new = u_plus + 2 * eps * Ep", PUSH),
    ("boris", "eps = 0.5 * r * dt", "eps = r * dt", PUSH),
    ("interpolate", "p = xi[:, a] - stagger[a]", "p = xi[:, a] + stagger[a]", GRID),
    ("gather", "E_STAGGER[c]", "E_STAGGER[(c + 1) % 3]", GRID),
    ("gather", "B_STAGGER[c]", "E_STAGGER[c]", GRID),
    ("deposit", "+ DSx[:, :, None] * DSy[:, None, :] / 3.0)", "+ DSx[:, :, None] * DSy[:, None, :] / 2.0)", GRID),
    ("deposit", "(S0y + 0.5 * DSy)", "(S0y + DSy)", GRID),
    ("deposit", "+ DSy[Y] * DSz[Z] / 3.0)", "+ DSy[Y] * DSz[Z] / 2.0)", GRID),
    ("deposit", "np.cumsum(Wx, axis=1)", "Wx", GRID),
    ("deposit", "np.cumsum(Wy, axis=2)", "np.cumsum(Wy, axis=1)", GRID),
    ("deposit", "(Zw * grid.d[0] / dt)[:, None, None] ", "(Zw * grid.d[1] / dt)[:, None, None] ", GRID),
    ("deposit", "Jz = (Zw * vz)[:, None, None] * Wz", "Jz = (Zw * vz)[:, None, None] * Wz.transpose(0, 2, 1)", GRID),
    ("shape_pair", "k0 = (i0 - b)", "k0 = (i1 - b)", GRID),
    ("shape_pair", "S1[rows, k1] = 1.0 - (p1 - i1)", "S1[rows, k1] = 1.0 - (p0 - i0)", GRID),
    ("charge_density", "(frac[a] if corner[a] else 1.0 - frac[a])", "(1.0 - frac[a] if corner[a] else frac[a])", GRID),
    ("yee_step", "E += dt * (curl_B(B, grid) - J)", "E += dt * (curl_B(B, grid) + J)", GRID),
    ("yee_step", "B -= 0.5 * dt * curl_E(E, grid)\n        E +=", "B += 0.5 * dt * curl_E(E, grid)\n        E +=", GRID),
    ("curl_E", "_dplus(E[1], 0, grid, gy) - _dplus(E[0], 1, grid)", "_dplus(E[0], 1, grid) - _dplus(E[1], 0, grid, gy)", GRID),
    ("curl_B", "_dminus(B[0], 2, grid) - _dminus(B[2], 0, grid, gz)", "_dminus(B[0], 2, grid) + _dminus(B[2], 0, grid, gz)", GRID),
    ("_dplus", "np.roll(F, -1, axis=AXIS[a])", "np.roll(F, 1, axis=AXIS[a])", GRID),
    ("div_E", "_dminus(E[1], 1, grid)", "_dminus(E[1], 0, grid)", GRID),
    ("move", "/ (gamma * grid.d[a])", "/ grid.d[a]", DIAG),
    ("wrap", "np.mod(xi[:, a], grid.n[a])", "np.mod(xi[:, a], grid.n[a] - 1)", DIAG),
    ("polarization", "s[selected].sum(axis=0) / N", "s[selected].sum(axis=0) / max(N - 1, 1)", DIAG),
    ("kinetic_energy_mev", "mu * (gamma - 1.0)", "(gamma - 1.0)", DIAG),
    ("MurState.advance_low", "self.lo_prev + self.k * (inside - self.lo_ghost)",
     "self.lo_prev - self.k * (inside - self.lo_ghost)", WINDOW),
    ("MurState.advance_high", "self.hi_prev + self.k * (inside - self.hi_ghost)",
     "inside + self.k * (inside - self.hi_ghost)", WINDOW),
    ("MurState.__init__", "(grid.dt - grid.d[0]) / (grid.dt + grid.d[0])", "0.0", WINDOW),
    ("MurState.advance_high", "np.stack([E[1][..., -1:], E[2][..., -1:]])",
     "np.stack([E[2][..., -1:], E[1][..., -1:]])", WINDOW),
    ("yee_step", "mur.advance_low(B)", "mur.lo_ghost", WINDOW),
    ("_scatter", "(ind[0] < grid.n[0])", "(ind[0] <= grid.n[0])", WINDOW),
    ("interpolate", "inside = (raw >= 0)", "inside = (raw >= -1)", WINDOW),
    ("Sim.step", "(x >= 0.0) & (x < self.grid.n[0])", "(x >= -1.0) & (x < self.grid.n[0])", WINDOW),
    ("Sim._shift", "F[..., :nx - S] = F[..., S:].copy()", "F[..., S:] = F[..., :nx - S].copy()", WINDOW),
    ("Sim._shift", "F[..., nx - S:] = 0.0", "pass", WINDOW),
    ("Sim._shift", "self.xi[k][:, 0] -= S", "self.xi[k][:, 0] -= S - 1", WINDOW),
    ("Sim._inject", "f = (q + 0.5) / ppc", "f = q / ppc", WINDOW),
    ("Sim._inject", "((cz * ny + cy) * S + col) * ppc + q", "((cz * ny + cy) * S + col) + q", WINDOW),
    ("Sim._inject", "(cx + 0.5 + origin) * g.d[0]", "(cx + origin) * g.d[0]", WINDOW),
    ("Sim._inject", "self.next_id[k] += nz * ny * S * ppc", "self.next_id[k] += m", WINDOW),
    ("Sim.window_density", '(x - w["ramp_start"]) / w["ramp_len"]', '(x - w["ramp_start"]) * w["ramp_len"]', WINDOW),
    ("Sim._advance_window", ">= (self.shifts + 1) * S", ">= (self.shifts + 2) * S", WINDOW),
    ("Sim._advance_window", "(self.nstep - self.window_step0)", "self.nstep", WINDOW),
]


@pytest.mark.parametrize("fname,old,new,checks", MUTANTS,
                         ids=["%s:%d" % (m[0], i) for i, m in enumerate(MUTANTS)])
def test_mutant_is_killed(monkeypatch, fname, old, new, checks):
    owner, name = (getattr(O, fname.split(".")[0]), fname.split(".")[1]) if "." in fname else (O, fname)
    src = textwrap.dedent(inspect.getsource(getattr(owner, name)))
    assert old in src, "mutation snippet not found in %s" % fname
    glb = dict(O.__dict__)
    exec(compile(src.replace(old, new, 1), "<mutant %s>" % fname, "exec"), glb)
    monkeypatch.setattr(owner, name, glb[name])
    assert _run_all(checks), "mutant of %s survived: %r -> %r" % (fname, old, new)


def test_unmutated_oracle_passes_every_check():
    for chk in PUSH + GRID + DIAG + WINDOW:
        chk()
