"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a private copy of the oracle source (on the
CPU, in a temporary directory), builds it, and runs the pin suite against
it; the suite must fail. The planted copies are never used for anything
else.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sphx_oracle.c")

# (name, text in the source, planted replacement, unused)
MUTATIONS = [
    ("gradient_direction", "g.e[k] = -dx[k] / g.r;", "g.e[k] = dx[k] / g.r;", None),
    ("kernel_constant_2d", "7.0 / (4.0 * M_PI)", "7.0 / (5.0 * M_PI)", None),
    ("kernel_constant_3d", "21.0 / (16.0 * M_PI)", "21.0 / (15.0 * M_PI)", None),
    ("kernel_derivative_factor", "return -5.0 * wendland_alpha", "return -4.0 * wendland_alpha", None),
    ("kernel_shape_exponent", "* s * s * s * s * (1.0 + 2.0 * q)", "* s * s * s * (1.0 + 2.0 * q)", None),
    ("limiter_direction", "fmax(UL - UR, 0.0)", "fmax(UR - UL, 0.0)", None),
    ("limiter_strength", "fmin(3.0 * fmax", "fmin(1.0 * fmax", None),
    ("ustar_pressure_sign", "(PL - PR) / (2.0 * rho_bar * c)", "(PR - PL) / (2.0 * rho_bar * c)", None),
    ("ustar_dropped_pressure", "+ (PL - PR) / (2.0 * rho_bar * c)", "", None),
    ("momentum_factor_two", "double coef = 2.0 * m * Ps", "double coef = m * Ps", None),
    ("momentum_density_weight", "2.0 * m * Ps / (rho_i * rho_j)", "2.0 * m * Ps / (rho_j * rho_j)", None),
    ("wall_volume_weight", "2.0 * s->vol_w * Ps / rho_i", "2.0 * s->vol_w * Ps / (rho_i * rho_i)", None),
    ("wall_right_velocity", "*UR = -(*UL) + 2.0 * uw;", "*UR = (*UL) + 2.0 * uw;", None),
    ("wall_hydrostatic_sign", "*PR = p_i + rho_i * dot3", "*PR = p_i - rho_i * dot3", None),
    ("continuity_weight", "sum += m / rho_j * (Us - UL)", "sum += m / rho_i * (Us - UL)", None),
    ("continuity_left_state", "sum += m / rho_j * (Us - UL) * g.dW;", "sum += m / rho_j * (Us - UR) * g.dW;", None),
    ("continuity_factor_two", "drho[i] = 2.0 * rho_i * sum;", "drho[i] = rho_i * sum;", None),
    ("reinit_without_self", "double sigma = W0;", "double sigma = 0.0;", None),
    ("reinit_without_walls", "            sigma += orc_kernel_W(s->d, s->p.h, g.r);\n        }\n        double rho_sum",
     "        }\n        double rho_sum", None),
    ("predicate_not_strict", "< s->rc2) idx[w++] = j;", "<= s->rc2) idx[w++] = j;", None),
    ("verlet_full_first_position", "s->x[3 * i + k] += 0.5 * dt * s->v[3 * i + k];\n    }\n    momentum_rate",
     "s->x[3 * i + k] += dt * s->v[3 * i + k];\n    }\n    momentum_rate", None),
    ("acoustic_step_without_flow_speed", "/ (s->p.c0 + vm);", "/ (s->p.c0);", None),
    ("advection_step_no_floor", "/ fmax(vm, s->p.u_ref);", "/ fmax(vm, 1e-300);", None),
    ("eos_sign", "(rho - s->p.rho0); }", "(s->p.rho0 - rho); }", None),
    ("gravity_dropped", "double acc[3] = {s->p.g[0] + s->av[3 * i], s->p.g[1] + s->av[3 * i + 1], s->p.g[2] + s->av[3 * i + 2]};",
     "double acc[3] = {s->av[3 * i], s->av[3 * i + 1], s->av[3 * i + 2]};", None),
    ("viscous_sign", "av[k] += cv * (vi[k] - vj[k]);", "av[k] += cv * (vj[k] - vi[k]);", None),
    ("viscous_factor_two", "double cv = 2.0 * m * eta", "double cv = m * eta", None),
    ("viscous_wall_dropped", "av[k] += cv * (vi[k] - vw[k]);", "av[k] += 0.0 * cv * (vi[k] - vw[k]);", None),
    ("viscous_not_applied", "s->p.g[0] + s->av[3 * i],", "s->p.g[0],", None),
    ("viscous_time_step_missing", "if (s->p.eta > 0.0) *dt_ad", "if (0) *dt_ad", None),
    ("transport_sign", "s->x[3 * i + k] += dt * dt * s->atv[3 * i + k];", "s->x[3 * i + k] -= dt * dt * s->atv[3 * i + k];", None),
    ("no_surface_reinit_keeps_max", "s->rho[i] = s->p.reinit_mode ? rho_sum : fmax(s->rho[i], rho_sum);",
     "s->rho[i] = fmax(s->rho[i], rho_sum);", None),
    ("wall_velocity_sign", "*UR = -(*UL) + 2.0 * uw;", "*UR = -(*UL) - 2.0 * uw;", None),
    ("wall_velocity_factor", "*UR = -(*UL) + 2.0 * uw;", "*UR = -(*UL) + uw;", None),
    ("wall_velocity_dropped", "double uw = -dot3(n, vw);", "double uw = 0.0 * dot3(n, vw);", None),
    ("moving_wall_shear_velocity_dropped", "av[k] += cv * (vi[k] - vw[k]);", "av[k] += cv * vi[k];", None),
    ("wall_speed_without_omega", "v[0] = s->mo.amp[0] * s->mo.omega * co - om * r1;",
     "v[0] = s->mo.amp[0] * co - om * r1;", None),
    ("roll_lever_sign", "v[1] = s->mo.amp[1] * s->mo.omega * co + om * r0;",
     "v[1] = s->mo.amp[1] * s->mo.omega * co - om * r0;", None),
    ("pose_rotation_transposed", "x[0] = (s->mo.pivot[0] + s->mo.amp[0] * sn) + (ct * d0 - st * d1);",
     "x[0] = (s->mo.pivot[0] + s->mo.amp[0] * sn) + (ct * d0 + st * d1);", None),
    ("normal_not_rotated", "n[0] = ct * n0[0] - st * n0[1];", "n[0] = n0[0];", None),
    ("static_flag_ignored", "if (s->moving && s->wmov[w]) wall_velocity(s, x, c, t, v);",
     "if (s->moving) wall_velocity(s, x, c, t, v);", None),
    ("given_wall_velocity_dropped", "for (int k = 0; k < 3; ++k) v[k] += s->vw0[3 * w + k];\n}",
     "for (int k = 0; k < 3; ++k) v[k] += 0.0 * s->vw0[3 * w + k];\n}", None),
    ("given_wall_velocity_sign", "for (int k = 0; k < 3; ++k) v[k] += s->vw0[3 * w + k];\n}",
     "for (int k = 0; k < 3; ++k) v[k] -= s->vw0[3 * w + k];\n}", None),
    ("wall_right_pressure_reference_density", "*PR = p_i + rho_i * dot3(s->p.g, r_fw);",
     "*PR = p_i + s->p.rho0 * dot3(s->p.g, r_fw);", None),
    ("wall_right_density_without_eos", "*rhoR = s->p.rho0 + *PR / (s->p.c0 * s->p.c0);",
     "*rhoR = s->p.rho0;", None),
    ("internal_energy_half", "ei += m * c2 * (log(rr) + 1.0 / rr - 1.0);",
     "ei += 0.5 * m * c2 * (log(rr) + 1.0 / rr - 1.0);", None),
    ("internal_energy_without_log", "ei += m * c2 * (log(rr) + 1.0 / rr - 1.0);",
     "ei += m * c2 * (rr + 1.0 / rr - 2.0);", None),
    ("static_flag_ignored_in_states", "if (s->moving && s->wmov[w]) wall_velocity(s, s->xw + 3 * w, s->wc, t, v);",
     "if (s->moving) wall_velocity(s, s->xw + 3 * w, s->wc, t, v);", None),
]


def _plant(src, old, new):
    assert old in src, f"mutation anchor not found: {old!r}"
    return src.replace(old, new)


@pytest.mark.parametrize("name,old,new,occ", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(name, old, new, occ):
    src = open(SRC).read()
    planted = _plant(src, old, new)
    with tempfile.TemporaryDirectory() as tmp:
        c = os.path.join(tmp, "planted.c")
        so = os.path.join(tmp, "libplanted.so")
        open(c, "w").write(planted)
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC",
                        "-shared", "-o", so, c, "-lm"], check=True)
        env = dict(os.environ, SPHX_ORACLE_LIB=so, OMP_NUM_THREADS="2")
        # a planted mistake that makes a pin run forever also counts as caught
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            "--timeout", "60", "--timeout-method", "thread", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                            os.path.join(ROOT, "tests", "test_oracle_viscous.py"),
                            os.path.join(ROOT, "tests", "test_oracle_moving_walls.py")],
                           env=env, capture_output=True, text=True, cwd=ROOT, timeout=900)
        assert r.returncode != 0, f"planted mistake {name} passed every pin:\n{r.stdout[-2000:]}"
