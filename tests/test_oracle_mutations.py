"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake (a dropped term, a flipped sign, a wrong index or
constant) in a copy of the oracle's C source, builds it on the CPU, and runs
the pin tests named for it against that build; the pins must fail.  Nothing
here touches the GPU library."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gdg_oracle.c")
T = "tests/"
SETUP, PHYS, SCHEME = T + "test_oracle_setup.py", T + "test_oracle_physics.py", T + "test_oracle_scheme.py"

BND = T + "test_oracle_boundary.py"
VISC = T + "test_oracle_viscosity.py"
INOUT = T + "test_oracle_inoutflow.py"
MAPPED = T + "test_oracle_mapped.py"
BCPARTS = T + "test_oracle_bcparts.py"
CURVED = T + "test_oracle_curved.py"
UNSTR = T + "test_oracle_unstructured.py"
CG = T + "test_oracle_cg.py"
RK54 = T + "test_oracle_rk54.py"

MUTANTS = {
    # name: (original text, planted text, pin files that must fail)
    "step_start_data_from_the_stage_input": ("                    or_diag *dg) {\n  const int dim = S->dim, m = S->m;",
                                             "                    or_diag *dg) {\n  keep_step_start(S, U);\n"
                                             "  const int dim = S->dim, m = S->m;",
                                             [INOUT + "::test_step_start_data_is_the_state_at_the_step_start"]),
    "rk54_last_stage_takes_u3": ("acc[q] = rk54_a[5][2] * u[2][q]", "acc[q] = rk54_a[5][2] * u[3][q]",
                                 [RK54 + "::test_step_equals_the_butcher_form_with_stage_times"]),
    "rk54_stage_time_from_substep": ("S->t0 + c[k] * tau", "S->t0 + r[k] * tau",
                                     [RK54 + "::test_step_equals_the_butcher_form_with_stage_times"]),
    "rk54_coefficient_digits_swapped": ("{0, 0.368410593050371, 0, 0, 0}", "{0, 0.368410593050317, 0, 0, 0}",
                                        [RK54 + "::test_order_conditions"]),
    "cg_boundary_pair_term_sign": ("          cc[((size_t)i * span + off) * dim + e] -= 0.5 * n * face_integral(S, f, a, b, 1);",
                                   "          cc[((size_t)i * span + off) * dim + e] += 0.5 * n * face_integral(S, f, a, b, 1);",
                                   [CG + "::test_skew_symmetry_and_partition_of_unity"]),
    "cg_mass_not_summed_over_cells": ("      S->mi[i] += S->vx ? tm[0] : cell_integral(S, 2, pa);",
                                      "      S->mi[i] = S->vx ? tm[0] : cell_integral(S, 2, pa);",
                                      [CG + "::test_hand_values_1d_q1"]),
    "unstructured_neighbour_mirrored": ("      if (!same_cell && S->ucp) {", "      if (0) {",
                                        [UNSTR + "::test_renumbered_lattice_gives_the_lattice_result"]),
    "unstructured_face_key_unsorted": ("      qsort(k->key, nc, sizeof(long), long_cmp);\n", "",
                                       [UNSTR + "::test_renumbered_lattice_gives_the_lattice_result"]),
    "curved_map_midpoint_weight": ("(q == 1 ? -4.0 * t * (t - 1.0) : 2.0 * t * (t - 0.5))",
                                   "(q == 1 ? -2.0 * t * (t - 1.0) : 2.0 * t * (t - 0.5))",
                                   [CURVED + "::test_quadratic_points_of_multilinear_cells_give_the_multilinear_mesh"]),
    "curved_map_derivative_sign": ("(q == 1 ? 4.0 - 8.0 * t : 4.0 * t - 1.0)",
                                   "(q == 1 ? 8.0 * t - 4.0 : 4.0 * t - 1.0)",
                                   [CURVED + "::test_identities_on_curved_cells"]),
    "boundary_part_axes_reversed": ("      for (int g = 0; g < dim; ++g) {\n        if (g == e) continue;\n        idx += ki[g] * stride;",
                                    "      for (int g = dim - 1; g >= 0; --g) {\n        if (g == e) continue;\n        idx += ki[g] * stride;",
                                    [BCPARTS + "::test_split_face_is_local_3d"]),
    "boundary_part_face_kind": ("      if (ghost_state(S, g, S->bface[b], S->bkind[b], i, t,",
                                "      if (ghost_state(S, g, S->bface[b], S->bc[S->bface[b]], i, t,",
                                [BCPARTS + "::test_split_face_is_local_2d"]),
    "mapped_gradient_transposed": ("for (int c = 0; c < dim; ++c) ge += Ji[c][e] * g[c];",
                                   "for (int c = 0; c < dim; ++c) ge += Ji[e][c] * g[c];",
                                   [MAPPED + "::test_identities_on_perturbed_cells"]),
    "mapped_mass_without_det": ("else if (kind == 2) out[0] += w * pa * det;",
                                "else if (kind == 2) out[0] += w * pa;", [MAPPED + "::test_cell_areas_are_the_shoelace_areas"]),
    "mapped_normal_transposed": ("out[d] += w * va * vb * sgn * det * Ji[e][d];",
                                 "out[d] += w * va * vb * sgn * det * Ji[d][e];",
                                 [MAPPED + "::test_identities_on_perturbed_cells"]),
    "mapped_corner_mirrored": ("      w *= bit ? xi[e] : 1.0 - xi[e];\n    }",
                               "      w *= bit ? 1.0 - xi[e] : xi[e];\n    }",
                               [MAPPED + "::test_lattice_vertices_give_the_uniform_mesh"]),
    "supersonic_inflow_keeps_state": ("if (un < -a) {\n      data_state(S, f, i, t, Ug);",
                                      "if (un < -1e300) {\n      data_state(S, f, i, t, Ug);",
                                      [BND + "::test_supersonic_inflow_converges_to_riemann_fan"]),
    "supersonic_normal_sign": ("un += (Ui[1 + e] / Ui[0]) * cb[e] / nn;", "un -= (Ui[1 + e] / Ui[0]) * cb[e] / nn;",
                               [BND]),
    "dirichlet_other_face": ("for (int c = 0; c < S->m; ++c) Ud[c] = S->bstate[f][c];",
                             "for (int c = 0; c < S->m; ++c) Ud[c] = S->bstate[f ^ 1][c];",
                             [BND + "::test_dirichlet_inflow_equals_supersonic"]),
    "bar_state_sign": ("(fk[q] - fj[q]) / (2.0 * dij[k])", "(fj[q] - fk[q]) / (2.0 * dij[k])",
                       [SCHEME + "::test_low_order_update_inside_unrelaxed_bounds"]),
    "boundary_term_dropped": (
        "for (int c = 0; c < m; ++c) acc[c] += (fc[c] - fi[c]) - dbd[b] * (Ub[c] - Ui[c]);", ";",
        [SCHEME + "::test_constant_state_preserved", SCHEME + "::test_slip_box_mass_energy"]),
    "kappa_without_plus_one": ("double kap_i = 1.0 / (double)(leni + 1);",
                               "double kap_i = 1.0 / (double)(leni);",
                               [SCHEME + "::test_limiter_bounds_symmetry_and_limits"]),
    "wave_speed_factor": ("double kfac = (g + 1.0) / (2.0 * g);\n  double lam1 = ul",
                          "double kfac = (g - 1.0) / (2.0 * g);\n  double lam1 = ul", [PHYS]),
    "wave_speed_exponent": ("double alpha = (g - 1.0) / (2.0 * g);\n  double num",
                            "double alpha = (g - 1.0) / (g);\n  double num", [PHYS]),
    "entropy_gradient_sign": ("grad[dim + 1] = (g - 1.0) / p;", "grad[dim + 1] = -(g - 1.0) / p;",
                              [SCHEME + "::test_entropy_viscosity_ratio"]),
    "high_order_viscosity_min": ("dH[k] = fmax(dmin, dev);", "dH[k] = fmin(dmin, dev);",
                                 [SCHEME + "::test_vortex_convergence",
                                  SCHEME + "::test_limiter_bounds_symmetry_and_limits"]),
    "limiter_max_not_min": ("lp[k] = fmin(li, lj);", "lp[k] = fmax(li, lj);",
                            [SCHEME + "::test_limiter_bounds_symmetry_and_limits"]),
    "residual_sign": ("rhs[c][a] = -tau * acc[c];", "rhs[c][a] = tau * acc[c];",
                      [SCHEME + "::test_high_low_identity_and_skew_fluxes"]),
    "relaxation_sign": ("Brmin[i] = (1.0 - rel) * rmin;", "Brmin[i] = (1.0 + rel) * rmin;",
                        [SCHEME + "::test_limiter_bounds_symmetry_and_limits"]),
    "cell_boundary_term_sign": ("out[e] = cK - cdK;", "out[e] = cK + cdK;", [SETUP]),
    "face_coupling_half": ("out[e] = 0.5 * n * face_integral(S, f, a, b, 0);",
                           "out[e] = n * face_integral(S, f, a, b, 0);", [SETUP]),
    "slip_half_reflection": ("Ug[1 + e] = Ui[1 + e] - 2.0 * mn * cb[e] / nn;",
                             "Ug[1 + e] = Ui[1 + e] - 1.0 * mn * cb[e] / nn;",
                             [SCHEME + "::test_slip_box_mass_energy"]),
    "mass_flux_sign": ("- mm * (dUH[c * N + j] - dUH[c * N + i]);",
                       "+ mm * (dUH[c * N + j] - dUH[c * N + i]);",
                       [SCHEME + "::test_high_low_identity_and_skew_fluxes"]),
    "density_search_lower_bound": ("if (r + pr < rmin) l = (rmin - r) / pr;", "if (r + pr < rmin) l = 1.0;",
                                   [SCHEME + "::test_limiter_bounds_symmetry_and_limits"]),
    "second_pass_full_flux": ("A2[k * m + c] = (1.0 - l1[k]) * A[k * m + c];", "A2[k * m + c] = A[k * m + c];",
                              [SCHEME + "::test_limiter_bounds_symmetry_and_limits"]),
    "rescaled_entropy_power": ("return pow(U[0], -g) * eps_of(dim, U);",
                               "return pow(U[0], -g + 0.1) * eps_of(dim, U);",
                               [SCHEME + "::test_limiter_bounds_symmetry_and_limits"]),
    "ssp_coefficients": ("Ub[q] = 0.75 * U[q] + 0.25 * Ph[q];", "Ub[q] = 0.5 * U[q] + 0.5 * Ph[q];",
                         [SCHEME + "::test_sod_converges_to_exact", SCHEME + "::test_vortex_convergence"]),
    "min_viscosity_all_faces": ("if (S->kind[k] == OR_KIND_FACE_COLLOC) {", "if (S->kind[k] != OR_KIND_CELL) {",
                                [SCHEME + "::test_vortex_convergence"]),
    "gradient_operand_transposed": ("g = dphi(S, p.b, p.dir, xi) * phi(S, p.a, xi);",
                                    "g = dphi(S, p.a, p.dir, xi) * phi(S, p.b, xi);", [SETUP]),
    "min_viscosity_even_power_zero": ("const double pk = (S->deg % 2 == 0) ? 0.5 : 0.0;",
                                      "const double pk = (S->deg % 2 == 0) ? 0.0 : 0.0;",
                                      [VISC + "::test_face_pair_viscosity_is_the_papers",
                                       VISC + "::test_boundary_viscosity_even_degree"]),
    "min_viscosity_even_power_one": ("const double pk = (S->deg % 2 == 0) ? 0.5 : 0.0;",
                                     "const double pk = (S->deg % 2 == 0) ? 1.0 : 0.0;",
                                     [VISC + "::test_face_pair_viscosity_is_the_papers",
                                      VISC + "::test_boundary_viscosity_even_degree"]),
    "entropy_viscosity_q2_constant": ("case 2: return 0.5;", "case 2: return 1.0;",
                                      [VISC + "::test_face_pair_viscosity_is_the_papers"]),
    "boundary_min_viscosity_dropped": ("double dmin = P->c_k * pow(hh, pk) * dbd[b];", "double dmin = 0.0 * dbd[b];",
                                       [VISC + "::test_boundary_viscosity_even_degree"]),
    "q3_equispaced_nodes": ("double r = 0.5 / sqrt(5.0);\n    S->xg[0] = 0.0;", "double r = 1.0 / 6.0;\n    S->xg[0] = 0.0;",
                            [SETUP + "::test_q3_1d_closed_form"]),
    "entropy_viscosity_q3_constant": ("case 3: return 0.25;", "case 3: return 0.5;",
                                      [VISC + "::test_face_pair_viscosity_is_the_papers"]),
    "q3_quadrature_weights_swapped": ("S->wq[0] = S->wq[3] = 0.5 * wo; S->wq[1] = S->wq[2] = 0.5 * wi;",
                                      "S->wq[0] = S->wq[3] = 0.5 * wi; S->wq[1] = S->wq[2] = 0.5 * wo;",
                                      [SETUP + "::test_q3_1d_closed_form"]),
    "inoutflow_entropy_side_flipped": ("const int in23 = vni <= 0.0;", "const int in23 = vni >= 0.0;",
                                       [INOUT + "::test_subsonic_characteristics"]),
    "inoutflow_outgoing_invariant_from_data": ("const double R4 = vni + 2.0 * ai / (g - 1.0);",
                                               "const double R4 = vnd + 2.0 * ad / (g - 1.0);",
                                               [INOUT + "::test_subsonic_characteristics"]),
    "vortex_data_frozen_in_time": ("vortex_at(S->vortex, x, t, Ud);", "vortex_at(S->vortex, x, 0.0, Ud);",
                                   [INOUT + "::test_vortex_leaving_the_box_converges_with_exact_data"]),
    "ev_normalizer_not_abs_sum": ("D += fabs(grad[q]) * fabs(Sk[q]);", "D += fabs(grad[q] * Sk[q]) * 0.5;",
                                  [SCHEME + "::test_vortex_convergence"]),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    orig, planted, pins = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(orig) >= 1, "mutation site moved: " + name
    path = tmp_path / (name + ".c")
    path.write_text(src.replace(orig, planted, 1))
    lib = tmp_path / ("lib" + name + ".so")
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-o", str(lib),
                           str(path), "-lm"])
    env = dict(os.environ, GDG_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"] + pins,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, "planted mistake %r passed the pins:\n%s" % (name, r.stdout[-800:])
