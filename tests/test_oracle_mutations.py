"""Mutation test of the oracle's pins (CPU only).

Each entry below plants one plausible mistake in a copy of the C oracle -- a
flipped sign, a dropped or wrong factor, a transposed operand, a one-sided
instead of a central face value, a perturbed coefficient -- builds the copy,
and runs the pins named for it in a fresh interpreter against that build
(``NSKR_ORACLE_SO``).  Those pins must fail.  A control build of the
unmodified source passes every pin used here, so a failure is the planted
mistake's doing.  The mistakes are planted in the oracle only, on the CPU;
nothing here touches the HIP library.
"""
import concurrent.futures
import os
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "nskr_oracle.c")

OPS = "tests/test_oracle_operator.py::"
WALLS = "tests/test_oracle_walls_dynamic.py::"
MMS = "tests/test_oracle_convergence.py::test_manufactured_solution_order"
RUS = "tests/test_oracle_rusanov.py::"

# name, text in the source, its replacement, pins that must reject it
MUTATIONS = [
    ("vdw pressure: +a rho^2",
     "return rho * pr->R * T / (1.0 - pr->b * rho) - pr->a * rho * rho;",
     "return rho * pr->R * T / (1.0 - pr->b * rho) + pr->a * rho * rho;",
     ["tests/test_oracle_thermo.py::test_reduced_constants_give_critical_point_one",
      "tests/test_oracle_thermo.py::test_maxwell_matches_table2"]),
    ("Stokes stress: 1/3 div u instead of 2/3",
     "2.0 / 3.0 * div", "1.0 / 3.0 * div",
     [WALLS + "test_slip_wall_normal_traction"]),
    ("Rusanov flux: anti-dissipative jump term",
     "out[v] = a - 0.5 * lam * (sp->U[v] - sm->U[v]);",
     "out[v] = a + 0.5 * lam * (sp->U[v] - sm->U[v]);",
     [WALLS + "test_moving_lid_over_fluid_at_rest"]),
    ("relaxation source: alpha beta (c - rho)",
     "0.5 * pr->alpha * (c * c - rho * rho) * div + pr->gam * (0.5 * gc2 * div - cc);\n"
     "    S[5] = pr->alpha * pr->beta * (rho - c);",
     "0.5 * pr->alpha * (c * c - rho * rho) * div + pr->gam * (0.5 * gc2 * div - cc);\n"
     "    S[5] = pr->alpha * pr->beta * (c - rho);",
     [OPS + "test_uniform_relaxation_follows_stability_polynomial"]),
    ("temperature: kinetic energy |m|^2 / rho without the 1/2",
     "double kin = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / rho;",
     "double kin = 1.0 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / rho;",
     [OPS + "test_init_with_velocities_recovers_temperature_and_densities"]),
    ("energy flux: + gamma c grad c div u",
     "- pr->gam * c * s->gc[i] * div", "+ pr->gam * c * s->gc[i] * div",
     [MMS]),
    ("weak derivative: D_ij instead of D_ji in Dhat",
     "c->Dh[i][j] = -(c->wg[j] / c->wg[i]) * c->D[j][i];",
     "c->Dh[i][j] = -(c->wg[j] / c->wg[i]) * c->D[i][j];",
     [OPS + "test_lift1_exact_for_polynomial_density_and_order_parameter"]),
    ("BR1: one-sided face value of the primitives",
     "val = 0.5 * (prim(Um, k) + prim(Up, k));", "val = prim(Um, k);",
     [OPS + "test_lifted_gradients_of_a_periodic_field_integrate_to_zero"]),
    ("BR1: one-sided face temperature",
     "Ts[f * n2 + fp] = 0.5 * (Tm + Tp);", "Ts[f * n2 + fp] = Tm;",
     [OPS + "test_lifted_gradients_of_a_periodic_field_integrate_to_zero"]),
    ("divergence lifting: jump instead of mean of grad c . n",
     "s += 0.5 * (qm + qp) * nv[m];", "s += 0.5 * (qm - qp) * nv[m];",
     [OPS + "test_divergence_lifting_exact"]),
    ("contact angle: wall energy derivative of the wrong sign",
     "return 6.0 * (c - rl) * (c - rv) / (d * d * d) * sigma * costheta;",
     "return -6.0 * (c - rl) * (c - rv) / (d * d * d) * sigma * costheta;",
     [OPS + "test_contact_angle_wall_c_flux_integral"]),
    ("heat flux dropped from j_e",
     "double je = pr->kappa * s->gT[i]", "double je = 0.0 * s->gT[i]",
     [WALLS + "test_conduction_between_isothermal_walls_is_steady"]),
    ("low-storage RK: a digit of A_2 changed",
     "-567301805773.0 / 1357537059087.0,", "-567301805770.0 / 1357537059087.0,",
     ["tests/test_oracle_basis.py::test_rk_order_conditions"]),
    ("relaxation model 2: p - alpha/2 rho^2",
     "return pr->model == 2 ? p + 0.5 * pr->alpha * rho * rho : p;",
     "return pr->model == 2 ? p - 0.5 * pr->alpha * rho * rho : p;",
     [MMS]),
    ("moving wall: ghost velocity u_w - u instead of 2 u_w - u",
     "sg.U[1 + m] = 2.0 * rho * uw[m] - sm->U[1 + m];",
     "sg.U[1 + m] = rho * uw[m] - sm->U[1 + m];",
     [WALLS + "test_moving_lid_over_fluid_at_rest"]),
    ("slip wall: ghost keeps half the normal momentum",
     "sg.U[1 + m] = sm->U[1 + m] - 2.0 * mn * n[m];",
     "sg.U[1 + m] = sm->U[1 + m] - 1.0 * mn * n[m];",
     [OPS + "test_mass_conservation_walls_and_curved"]),
    ("Navier slip: friction gamma_2 of the wrong sign",
     "- g2 * (ut - (uw[m] - uwn * n[m]));", "+ g2 * (ut - (uw[m] - uwn * n[m]));",
     [WALLS + "test_navier_slip_couette_under_a_moving_lid"]),
    ("heat-transfer wall: gamma_3 flux of the wrong sign",
     "-g3 * (1.0 / wp.Tw - 1.0 / sm->T)", "g3 * (1.0 / wp.Tw - 1.0 / sm->T)",
     [WALLS + "test_conduction_between_heat_transfer_walls_is_steady"]),
    ("dynamic angle: normal instead of tangential grad c in the traction",
     "g1 * div * (sm->gc[m] - gcn * n[m])", "g1 * div * (sm->gc[m] + gcn * n[m])",
     [WALLS + "test_dynamic_angle_traction_is_tangential"]),
    ("HLLC: pressure difference of the wrong sign in the contact speed",
     "double Ss = (p[1] - p[0] + ", "double Ss = (p[0] - p[1] + ",
     ["tests/test_oracle_model2.py::test_hllc_reproduces_linear_acoustics"]),
    ("HLLC: star energy without the pressure work",
     "(Ss - un[k]) * (Ss + p[k] / (rho[k] * (S - un[k]))));", "(Ss - un[k]) * (Ss + 0.0 / (rho[k] * (S - un[k]))));",
     ["tests/test_oracle_model2.py::test_hllc_reproduces_linear_acoustics"]),
    ("surface tension: sqrt(gamma) instead of sqrt(2 gamma)",
     "    return sqrt(2.0 * gam) * I;\n}\n\ndouble orc_sigma(", "    return sqrt(1.0 * gam) * I;\n}\n\ndouble orc_sigma(",
     ["tests/test_oracle_thermo.py::test_sigma_and_interface_width_table1"]),
    ("15-point sigma of the wall table: sqrt(gamma) instead of sqrt(2 gamma)",
     "    return sqrt(2.0 * gam) * I;\n}\n\n/* ", "    return sqrt(1.0 * gam) * I;\n}\n\n/* ",
     ["tests/test_oracle_wall_table.py::test_interpolation_error_bound"]),
    ("time step: CFL factor dropped from the advective limit",
     "double dt_adv = pr->cfl * tN(c->N) * 2.0 / lmax;", "double dt_adv = tN(c->N) * 2.0 / lmax;",
     [OPS + "test_time_step_scales_with_the_cfl_number"]),
    ("time step: CFL factor dropped from the parabolic limit",
     "double dt_par = den > 0.0 ? pr->cfl * RK_REAL / den : INFINITY;",
     "double dt_par = den > 0.0 ? RK_REAL / den : INFINITY;",
     [OPS + "test_time_step_scales_with_the_cfl_number"]),
    ("temperature: relaxation energy alpha (rho - c)^2 without the 1/2",
     "double rel = 0.5 * pr->alpha * (rho - U[5]) * (rho - U[5]);",
     "double rel = 1.0 * pr->alpha * (rho - U[5]) * (rho - U[5]);",
     [OPS + "test_init_recovers_temperature", OPS + "test_init_with_velocities_recovers_temperature_and_densities", MMS]),
    ("temperature: gradient energy of the wrong sign",
     "double reps = U[4] - kin - rel - grd;", "double reps = U[4] - kin - rel + grd;",
     [OPS + "test_init_recovers_temperature", OPS + "test_init_with_velocities_recovers_temperature_and_densities", MMS]),
    ("sound speed: c_v factor (1 + 1/c_v) dropped",
     "return (1.0 + 1.0 / pr->cv) * pr->R * T / (q * q) - 2.0 * pr->a * rho;",
     "return pr->R * T / (q * q) - 2.0 * pr->a * rho;",
     ["tests/test_oracle_thermo.py::test_speed_of_sound_matches_isentropic_derivative"]),
    ("model 2 source: alpha rho grad c of the wrong sign",
     "for (int m = 0; m < 3; ++m) S[1 + m] = pr->alpha * rho * gc[m];",
     "for (int m = 0; m < 3; ++m) S[1 + m] = -pr->alpha * rho * gc[m];",
     [MMS]),
    ("surface lifting: l(+1) weights on the minus faces",
     "c->lhm[j] = c->lm[j] / c->wg[j];", "c->lhm[j] = c->lp[j] / c->wg[j];",
     [OPS + "test_lift1_exact_for_polynomial_density_and_order_parameter"]),
    ("wall temperature: gradient subtracted",
     "w->Tw += tg[0] * x[0] + tg[1] * x[1] + tg[2] * x[2];", "w->Tw -= tg[0] * x[0] + tg[1] * x[1] + tg[2] * x[2];",
     ["tests/test_oracle_wall_table.py::test_isothermal_wall_following_the_fluid_temperature"]),
    ("stage times: every stage at the step's start",
     "c->time = t + RK_C[s] * dt;", "c->time = t;",
     ["tests/test_oracle_wall_table.py::test_rk_stages_use_their_own_times"]),
    ("integrals: kinetic energy without the 1/2",
     "out[6] += wJ * 0.5 * (U6[1] * U6[1] + U6[2] * U6[2] + U6[3] * U6[3]) / rho;",
     "out[6] += wJ * 1.0 * (U6[1] * U6[1] + U6[2] * U6[2] + U6[3] * U6[3]) / rho;",
     [OPS + "test_integrals_against_quadrature_and_thermodynamics"]),
    ("integrals: entropy of the wrong sign",
     "out[18] += -wJ * rho * eta;", "out[18] += wJ * rho * eta;",
     [OPS + "test_integrals_against_quadrature_and_thermodynamics"]),
    ("time step: a digit of T_3 swapped",
     "static const double T[6] = {0, 0, 0.3521, 0.2200, 0.1523, 0.1126};",
     "static const double T[6] = {0, 0, 0.3521, 0.2020, 0.1523, 0.1126};",
     ["tests/test_oracle_dt.py::test_advective_constant"]),
    ("time step: a digit of RHO_3 swapped",
     "static const double R[6] = {0, 0, 64.8, 176.2, 387.0, 745.2};",
     "static const double R[6] = {0, 0, 64.8, 167.2, 387.0, 745.2};",
     ["tests/test_oracle_dt.py::test_parabolic_constant"]),
    ("time step: a digit of the real stability interval swapped",
     "#define RK_REAL 4.6567", "#define RK_REAL 4.5667",
     ["tests/test_oracle_dt.py::test_real_stability_interval_from_the_relaxation_limit"]),
    ("droplets: inverted profile (vapour inside)",
     "double th = tanh((rad[j] - sqrt(d2)) / width);", "double th = tanh((sqrt(d2) - rad[j]) / width);",
     [OPS + "test_droplet_excess_mass_closed_form"]),
    ("droplets: twice the interface width",
     "double th = tanh((rad[j] - sqrt(d2)) / width);", "double th = tanh((rad[j] - sqrt(d2)) / (2.0 * width));",
     [OPS + "test_droplet_excess_mass_closed_form"]),
    ("droplets: no minimum image across periodic sides",
     "if (c->box.periodic[m]) dx -= c->box.len[m] * round(dx / c->box.len[m]);",
     "if (c->box.periodic[m]) dx -= 0.0 * round(dx / c->box.len[m]);",
     [OPS + "test_droplet_excess_mass_closed_form"]),
    ("energy flux: viscous work tau u dropped",
     "Fv[i][4] = Tv[i][0] * u[0] + Tv[i][1] * u[1] + Tv[i][2] * u[2] + je;", "Fv[i][4] = je;",
     [MMS, WALLS + "test_navier_slip_couette_under_a_moving_lid"]),
    ("order-parameter flux: gamma beta grad c without beta",
     "Fv[i][5] = pr->gam * pr->beta * s->gc[i];", "Fv[i][5] = pr->gam * s->gc[i];",
     [MMS, OPS + "test_contact_angle_wall_c_flux_integral"]),
    ("energy flux: zeta_c term of the wrong sign",
     "+ pr->gam * s->gc[i] * zeta;", "- pr->gam * s->gc[i] * zeta;",
     [MMS, OPS + "test_energy_flux_zeta_term_closed_form"]),
    ("zeta_c: alpha (c - rho) instead of alpha (rho - c)",
     "double zeta = pr->beta * (pr->gam * s->lapc + pr->alpha * (rho - c));",
     "double zeta = pr->beta * (pr->gam * s->lapc + pr->alpha * (c - rho));",
     [MMS, OPS + "test_energy_flux_zeta_term_closed_form"]),
    ("HLLC: Davis estimates swapped (min for the right speed)",
     "double SR = fmax(un[0] + a[0], un[1] + a[1]);", "double SR = fmin(un[0] + a[0], un[1] + a[1]);",
     ["tests/test_oracle_model2.py"]),
    ("contact angle: theta in radians taken as degrees",
     "c->wcos[f] = cos(bx->side_theta[f] * M_PI / 180.0);", "c->wcos[f] = cos(bx->side_theta[f]);",
     [OPS + "test_contact_angle_wall_c_flux_integral"]),
    ("Jacobian scaling: + (volume + surface) / J",
     "Ut[v * nn + (size_t)e * n3 + nd] = -acc[v] / J + S[v];", "Ut[v * nn + (size_t)e * n3 + nd] = acc[v] / J + S[v];",
     [OPS + "test_mass_conservation_walls_and_curved", MMS]),
    ("energy source: gamma grad c (x) grad c : grad u of the wrong sign",
     "0.5 * pr->alpha * (c * c - rho * rho) * div + pr->gam * (0.5 * gc2 * div - cc);\n    S[5]",
     "0.5 * pr->alpha * (c * c - rho * rho) * div + pr->gam * (0.5 * gc2 * div + cc);\n    S[5]",
     [MMS]),
    ("energy source: alpha/2 (c^2 - rho^2) div u of the wrong sign",
     "           0.5 * pr->alpha * (c * c - rho * rho) * div", "           0.5 * pr->alpha * (rho * rho - c * c) * div",
     [MMS]),
    ("model 2 energy source: alpha/2 c^2 div u dropped",
     "+ 0.5 * pr->alpha * c * c * div +", "+ 0.0 * pr->alpha * c * c * div +",
     [MMS]),
    ("relaxation wall value: zeta_c = +gamma_1 gamma_4 div u",
     "double zeta = -g1 * g4 * div;", "double zeta = g1 * g4 * div;",
     [WALLS + "test_dynamic_angle_and_relaxation_wall_rates"]),
    ("no-slip wall: BR1 wall velocity taken from the fluid",
     "val = c->box.side_uwall[c->side[e * 6 + f]][k - 1]; /* no-slip */", "val = prim(Um, k); /* no-slip */",
     [WALLS + "test_wall_values_of_the_lifted_velocity"]),
    ("slip wall: BR1 wall velocity keeps its normal part",
     "val = prim(Um, k) - un * n[k - 1];", "val = prim(Um, k);",
     [WALLS + "test_wall_values_of_the_lifted_velocity"]),
    ("isothermal wall: BR1 wall temperature taken from the fluid",
     "Ts[f * n2 + fp] = wall_isothermal(c, kd, sd) ? wp.Tw : Tm;", "Ts[f * n2 + fp] = Tm;",
     [WALLS + "test_conduction_between_isothermal_walls_is_steady", OPS + "test_hot_isothermal_wall_heats_fluid"]),
    ("adiabatic slip wall: BR1 wall temperature set to the wall's",
     "Ts[f * n2 + fp] = wall_isothermal(c, kd, sd) ? wp.Tw : Tm;", "Ts[f * n2 + fp] = wp.Tw;",
     [WALLS + "test_navier_wall_without_coefficients_is_the_slip_wall", WALLS + "test_slip_wall_normal_traction",
      OPS + "test_free_stream_at_rest_with_walls"]),
    ("neutral slip wall: contact-angle flux not zero",
     "                        fs[f * n2 + fp] = 0.0;\n                    } else {",
     "                        fs[f * n2 + fp] = 1e-3;\n                    } else {",
     [WALLS + "test_navier_wall_without_coefficients_is_the_slip_wall", OPS + "test_free_stream_at_rest_with_walls"]),
    ("HLLC: star momentum with (S* + u_n)",
     "Us[1 + m] = f * (U[1 + m] / U[0] + (Ss - un[k]) * n[m]);", "Us[1 + m] = f * (U[1 + m] / U[0] + (Ss + un[k]) * n[m]);",
     ["tests/test_oracle_model2.py"]),
    ("HLLC: order parameter not carried as c / rho",
     "Us[5] = f * U[5] / U[0];", "Us[5] = f;",
     ["tests/test_oracle_model2.py"]),
    ("viscous stress: 2 du_i/dx_j instead of the symmetric part",
     "Tv[i][j] = pr->mu * (gu[i][j] + gu[j][i] - (i == j ? 2.0 / 3.0 * div : 0.0));",
     "Tv[i][j] = pr->mu * (2.0 * gu[i][j] - (i == j ? 2.0 / 3.0 * div : 0.0));",
     [MMS, WALLS + "test_navier_slip_couette_under_a_moving_lid"]),
    ("face traces: l(+1) used on the minus faces",
     "c->lm[j] = lagrange(P, c->xg, j, -1.0);", "c->lm[j] = lagrange(P, c->xg, j, 1.0);",
     ["tests/test_oracle_basis.py::test_face_interpolation", OPS + "test_lift1_exact_for_polynomial_density_and_order_parameter"]),
    ("model 2: wave speed without alpha rho",
     "if (pr->model == 2) a2 += pr->alpha * rho;", "if (pr->model == 2) a2 += 0.0 * rho;",
     ["tests/test_oracle_model2.py", MMS]),
    ("curved metrics: curl form of the wrong sign",
     "JaGL[(i * 3 + n) * sz + nd] = -(s1 - s2);", "JaGL[(i * 3 + n) * sz + nd] = (s1 - s2);",
     [OPS + "test_metrics_satisfy_the_cofactor_identity"]),
    ("Rusanov: the smaller of the two wave speeds",
     "double lam = lm > lp ? lm : lp;", "double lam = lm < lp ? lm : lp;",
     [RUS + "test_rusanov_speed_is_the_larger_of_the_two_sides"]),
    ("Rusanov: wave speed without |u . n|",
     "double lm = fabs(unm) + wave_speed(pr, sm->U[0], sm->T);", "double lm = wave_speed(pr, sm->U[0], sm->T);",
     [RUS + "test_rusanov_speed_of_each_side_is_its_own"]),
    ("model 2: relaxation source alpha beta (c - rho)",
     "S[5] = pr->alpha * pr->beta * (rho - c);\n        return;", "S[5] = pr->alpha * pr->beta * (c - rho);\n        return;",
     [MMS]),
    ("wall table: interpolation weights swapped",
     "out[v] = (1.0 - w) * tab[3 * k + v] + w * tab[3 * (k + 1) + v];",
     "out[v] = w * tab[3 * k + v] + (1.0 - w) * tab[3 * (k + 1) + v];",
     ["tests/test_oracle_wall_table.py::test_interpolation_error_bound"]),
    ("wall time-step limit: traction path divided by the wrong direction's |Ja|",
     "r += sigmaN(c->N) * (lam * an * g1 * gt / rho",
     "r += sigmaN(c->N) * (lam * sqrt(st) * g1 * gt / rho",
     ["tests/test_oracle_dt.py::test_wall_constant_of_the_traction_path"]),
    ("wall time-step limit: c-flux path without beta",
     "sqrt(pr->alpha * pr->beta * g1 * lam * an * st)", "sqrt(pr->alpha * g1 * lam * an * st)",
     ["tests/test_oracle_dt.py::test_wall_constant_of_the_c_flux_path"]),
    ("wall time-step limit: normal direction counted as tangential",
     "            if (d == dn) continue;\n            const double *A = Ja + d * 3;",
     "            const double *A = Ja + d * 3;",
     ["tests/test_oracle_dt.py::test_wall_constant_of_the_c_flux_path"]),
    ("wall time-step limit: the real instead of the imaginary interval",
     "double dt_wall = wmax > 0.0 ? pr->cfl * RK_IMAG / wmax : INFINITY;",
     "double dt_wall = wmax > 0.0 ? pr->cfl * RK_REAL / wmax : INFINITY;",
     ["tests/test_oracle_dt.py::test_wall_constant_of_the_traction_path"]),
    ("wall time-step limit: left out of the minimum",
     "return dt < dt_wall ? dt : dt_wall;", "return dt;",
     ["tests/test_oracle_dt.py::test_sliding_droplet_at_the_printed_gamma_1_is_stable_at_the_rule_step"]),
]


# Mistakes no pin rejects yet (the oracle's header and the design notes call
# the function "parity unpinned"); strict: a pin that starts to reject one
# turns its entry into an unexpected pass, to be moved to the list above.
KNOWN_SURVIVORS = {}


def _build(src_text, path):
    with open(path + ".c", "w") as f:
        f.write(src_text)
    cmd = ["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE", "-o", path,
           path + ".c", "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)


def _run_pins(so, pins):
    env = dict(os.environ, NSKR_ORACLE_SO=so, OMP_NUM_THREADS="2")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-p", "no:randomly", *pins]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


@pytest.fixture(scope="module")
def outcomes():
    with open(SRC) as f:
        src = f.read()
    for name, old, new, _ in MUTATIONS:
        assert src.count(old) == 1, f"mutation site not unique or missing: {name}"
    jobs = [("control", src, sorted({p for *_, pins in MUTATIONS for p in pins}))]
    jobs += [(name, src.replace(old, new), pins) for name, old, new, pins in MUTATIONS]
    with tempfile.TemporaryDirectory() as tmp:
        def one(k):
            name, text, pins = jobs[k]
            so = os.path.join(tmp, f"mut{k}.so")
            _build(text, so)
            return name, _run_pins(so, pins)
        with concurrent.futures.ThreadPoolExecutor(max_workers=6) as ex:
            return dict(ex.map(one, range(len(jobs))))


def test_control_build_passes_every_pin(outcomes):
    rc, out = outcomes["control"]
    assert rc == 0, out


@pytest.mark.parametrize("name", [
    pytest.param(m[0], marks=pytest.mark.xfail(strict=True, reason=KNOWN_SURVIVORS[m[0]]))
    if m[0] in KNOWN_SURVIVORS else m[0] for m in MUTATIONS])
def test_pins_reject_planted_mistake(outcomes, name):
    rc, out = outcomes[name]
    # 1: tests ran and at least one failed (not a crash, a usage error or an
    # empty selection)
    assert rc == 1, f"mutation survived or did not run cleanly (exit {rc}): {name}\n{out}"
