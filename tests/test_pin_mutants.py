"""Strength of the oracle's pins: each case plants one plausible mistake in a
copy of the oracle (a wrong coefficient, sign, constant, weight or lattice
vector), builds it, and runs the pin that should notice.  That pin must fail.
The correct oracle passes the same pins in test_oracle_pins.py."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbib_oracle.c")

AREA = [(f"fa[2 * v{i}{s}] += 0.5 * fmag * nm{c};", f"fa[2 * v{i}{s}] -= 0.5 * fmag * nm{c};")
        for i in (1, 2) for s, c in (("", "x"), (" + 1", "y"))]

# (name, [(text, replacement)], pin selected with -k)
MUTANTS = [
    ("guo_prefactor", [("double pre = 1.0 - 1.0 / (2.0 * tau);", "double pre = 1.0 - 1.0 / tau;")],
     "test_p2_forcing_moments"),
    ("moments_without_half_force",
     [("s->ux[c] = (jx + 0.5 * s->F[c * 2]) / r;", "s->ux[c] = jx / r;")],
     "test_p4_poiseuille_closed_form"),
    ("zou_he_half_force_sign",
     [("double mx = rw * s->u_bot - 0.5 * Fx;", "double mx = rw * s->u_bot + 0.5 * Fx;")],
     "test_p4_poiseuille_closed_form"),
    ("lattice_vector", [("static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};",
                         "static const int EY[9] = {0, 0, 1, 0, -1, 1, -1, -1, -1};")],
     "test_p1_equilibrium_moments"),
    ("mls_alpha", [("static const double MLS_ALPHA = 0.3;", "static const double MLS_ALPHA = 0.35;")],
     "test_p6_mls_node_centred_closed_form"),
    ("probe_length", [("static const double PROBE_LEN = 1.2;", "static const double PROBE_LEN = 1.0;")],
     "test_hydro_linear_pressure_field"),
    ("area_force_sign", AREA, "test_p9_forces_are_energy_gradients"),
    ("first_order_node_velocity",
     [("k->uv[j] = (1.5 * xn[j] - 2.0 * k->x[j] + 0.5 * k->xm1[j]) / 1.0;",
       "k->uv[j] = xn[j] - k->x[j];")],
     "test_dynamic_first_step_closed_form"),
    ("spreading_weight_one",
     [("spread(s, k->x[2 * v], k->x[2 * v + 1], 0.5 * (ll + lr), Fx, Fy);",
       "spread(s, k->x[2 * v], k->x[2 * v + 1], 1.0, Fx, Fy);")],
     "test_dynamic_forcing_weight_is_arc_length"),
    ("viscous_stress_without_transpose",
     [("tp[a][b] = 1.0 * s->nu * (Gp[a][b] + Gp[b][a]);", "tp[a][b] = 1.0 * s->nu * (Gp[a][b]);"),
      ("tm[a][b] = 1.0 * s->nu * (Gm[a][b] + Gm[b][a]);", "tm[a][b] = 1.0 * s->nu * (Gm[a][b]);")],
     "test_hydro_piecewise"),
    ("bending_force_sign",
     [("double FLx = kb * sn * nLx / la, FLy = kb * sn * nLy / la;",
       "double FLx = -kb * sn * nLx / la, FLy = -kb * sn * nLy / la;")],
     "test_p9_forces_are_energy_gradients"),
    ("contact_exponent",
     [("double mag = C * sqrt(1.0 / (d * d * d * d * d));", "double mag = C * sqrt(1.0 / (d * d * d * d));")],
     "test_contact_force_formula"),
    ("inlet_profile",
     [("double ux = 4.0 * s->u_in * y * (H - y) / (H * H);", "double ux = 4.0 * s->u_in * y * (H - y) / (H * (H + 1));")],
     "test_open_channel_poiseuille"),
    ("taylor_deformation",
     [("out[4] = (a - b) / (a + b);", "out[4] = (a - b) / a;")],
     "test_p10_affine_polygon_taylor"),
    ("swelling_ratio",
     [("out[5] = A / (P * P / (4.0 * M_PI));", "out[5] = A / (P * P / (2.0 * M_PI));")],
     "test_p10_regular_polygon"),
    ("node_mass", [("k->mv = mass / nv;", "k->mv = mass / (nv - 1);")],
     "test_dynamic_first_step_closed_form"),
    ("rigid_rotation_update",
     [("double w = 2.0 / 3.0 * (2.0 * k->w - 0.5 * k->wm1 + aw * 1.0);",
       "double w = 2.0 / 3.0 * (2.0 * k->w - 0.5 * k->wm1 - aw * 1.0);")],
     "test_rigid_disc_rotates_at_half_the_shear_rate"),
    ("outlet_zou_he",
     [("g[7] = g[5] + 0.5 * (g[2] - g[4]) - s->rho_out * uo / 6.0;",
       "g[7] = g[5] - 0.5 * (g[2] - g[4]) - s->rho_out * uo / 6.0;")],
     "test_open_channel_poiseuille"),
    ("kinematic_update_coefficient",
     [("xn[j] = 2.0 / 3.0 * (2.0 * k->x[j] - 0.5 * k->xm1[j] + U[d] * 1.0);",
       "xn[j] = 0.5 * (2.0 * k->x[j] - 0.5 * k->xm1[j] + U[d] * 1.0);")],
     "test_p13_uniform_translation"),
]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name,edits,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_planted_mistake(name, edits, pin, tmp_path):
    src = open(SRC).read()
    for old, new in edits:
        assert src.count(old) == 1, old
        src = src.replace(old, new)
    c = tmp_path / "mutant.c"
    c.write_text(src)
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC",
                           "-shared", "-o", str(lib), str(c), "-lm"])
    env = dict(os.environ, LBIB_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", pin],
                       capture_output=True, text=True, timeout=300, env=env, cwd=ROOT)
    assert r.returncode == 1, f"{name}: pin {pin} did not fail (rc {r.returncode})\n{r.stdout[-2000:]}"
