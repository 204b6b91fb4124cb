"""The oracle's pins catch plausible mistakes.

Each case plants one mistake (a dropped factor, a flipped sign, a transposed
operand, a wrong index) in a copy of el_oracle.c, compiles it on the CPU,
points the oracle wrapper at the copy and runs the pins of
test_oracle_pins.py: at least one of them must fail.  The real oracle is
untouched.
"""
import os
import subprocess

import pytest

import oracle.oracle as oo
from tests import test_frank3_pins as f3
from tests import test_free_walls_pins as fw
from tests import test_obstacle_pins as ob
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oo.__file__), "el_oracle.c")

# (name, text in el_oracle.c, replacement)
MUTATIONS = [
    ("guo_first_moment_sign", "out[i] = weight(i) * (eF / cs2 + contraction", "out[i] = weight(i) * (-eF / cs2 + contraction"),
    ("guo_second_moment_factor", "contraction / (2.0 * cs2 * cs2)", "contraction / (cs2 * cs2)"),
    ("equilibrium_quadratic", "(eu * eu) / (2.0 * cs2 * cs2)", "(eu * eu) / (cs2 * cs2)"),
    ("equilibrium_uu_sign", "- uu / (2.0 * cs2)", "+ uu / (2.0 * cs2)"),
    ("shifted_density_term", "weight(i) * rho * poly + drho * weight(i)", "weight(i) * rho * poly"),
    ("guo_prefactor", "(1.0 - 1.0 / (2.0 * tau)) * S[i]", "(1.0 - 1.0 / tau) * S[i]"),
    ("half_force_in_u", "u_out[a] = (j[a] + 0.5 * Ftot_out[a]) / rho", "u_out[a] = (j[a] + Ftot_out[a]) / rho"),
    ("bounce_back_direction", "s->qn[(int64_t)OPP[i] * s->N + k] = post;", "s->qn[(int64_t)i * s->N + k] = post;"),
    ("stream_direction", "int xd = wrap(x + E[i][0], p->nx);", "int xd = wrap(x - E[i][0], p->nx);"),
    ("weight_edge", "return 1.0 / 36.0;", "return 1.0 / 30.0;"),
    ("laplacian_centre", "- 2.0 * mc +", "- 1.0 * mc +"),
    ("chirality_sign", "h[g] = Km * lap - 2.0 * Kt * p->q0 * curl;", "h[g] = Km * lap + 2.0 * Kt * p->q0 * curl;"),
    ("anchoring_sign", "h[2] += p->W0 * m[2 * st->N + k];", "h[2] -= p->W0 * m[2 * st->N + k];"),
    ("vorticity_transposed", "W[a][m] = 0.5 * (A[m][a] - A[a][m]);", "W[a][m] = 0.5 * (A[a][m] - A[m][a]);"),
    ("alignment_sign", "h[mu] / gamma1 - (gamma2 / gamma1) * align", "h[mu] / gamma1 + (gamma2 / gamma1) * align"),
    ("advection_sign", "- adv + rot", "+ adv + rot"),
    ("heun_half", "0.5 * dt * (s->dn_old", "dt * (s->dn_old"),
    ("heun_predictor_step", "v[a] = s->n[(int64_t)a * s->N + k] + dt * r[a];", "v[a] = s->n[(int64_t)a * s->N + k] + 0.5 * dt * r[a];"),
    ("leslie_a2_transposed", "s += al[1] * n[b] * N[a];", "s += al[1] * n[a] * N[b];"),
    ("leslie_a5_transposed", "s += al[4] * n[b] * Dn[a];", "s += al[4] * n[a] * Dn[b];"),
    ("leslie_a6_transposed", "s += al[5] * n[a] * Dn[b];", "s += al[5] * n[b] * Dn[a];"),
    ("leslie_a1_dropped", "s += al[0] * n[a] * n[b] * nDn;", "s += 0.0 * nDn;"),
    ("N_alignment_sign", "N[a] = (h[a] - gamma2 * Dn[a]) / gamma1;", "N[a] = (h[a] + gamma2 * Dn[a]) / gamma1;"),
    ("alpha4p_factor", "s += p->alpha4p * D[a][b];", "s += 2.0 * p->alpha4p * D[a][b];"),
    ("elastic_transposed", "for (int g = 0; g < 3; ++g) e += G[a][g] * Pi[b][g];",
     "for (int g = 0; g < 3; ++g) e += G[b][g] * Pi[a][g];"),
    ("elastic_chiral_sign", "chiral += eps3(m, b, g) * n[m];", "chiral += eps3(m, g, b) * n[m];"),
    ("divergence_sign", "div += 0.5 * (nb(st, st->sig, 2, a * 3 + b, x, y, z, b, +1) -",
     "div -= 0.5 * (nb(st, st->sig, 2, a * 3 + b, x, y, z, b, +1) -"),
    ("solid_director_value", "if (field_kind == 0) return comp == 2 ? 1.0 : 0.0;",
     "if (field_kind == 0) return comp == 0 ? 1.0 : 0.0;"),
    ("no_corrector_normalisation", "normalise(v);\n                /* n(x) is read only", "/* n(x) is read only"),
    ("checkerboard_projection_sign", "ufull[(int64_t)a * s->N + idx(p, x, y, z)] -= amp * sign;",
     "ufull[(int64_t)a * s->N + idx(p, x, y, z)] += amp * sign;"),
    # the hybrid loop of Sec. II D
    ("fd_before_lbm", "or_step_lbm(s, 1);\n        if (s->t % s->p.fd_ratio == 0) or_step_director(s);",
     "if (s->t % s->p.fd_ratio == 0) or_step_director(s);\n        or_step_lbm(s, 1);"),
    ("fd_on_next_step", "if (s->t % s->p.fd_ratio == 0) or_step_director(s);",
     "if ((s->t + 1) % s->p.fd_ratio == 0) or_step_director(s);"),
    ("no_initial_force", "or_force(s); /* R10: initial force from n0 with u = 0 */", "/* no initial force */"),
    ("no_force_after_fd", "    or_force(s);\n}\n\n/* Hybrid loop", "}\n\n/* Hybrid loop"),
    # tube centroids (R14)
    ("tube_no_minimum_image", "dx -= p->nx * floor(dx / p->nx + 0.5);", ""),
    ("tube_circular_mean_swapped", "atan2(sums[t][2], sums[t][1])", "atan2(sums[t][1], sums[t][2])"),
    ("no_moments_after_stream", "        lbm_step(s);\n        or_moments(s);", "        lbm_step(s);"),
]

# mistakes in the three-constant Frank elasticity (R4'), checked against its own pins
MUTATIONS_FRANK3 = [
    ("frank3_splay_takes_twist_constant", "dh[mu] = a[0] * dS[mu]", "dh[mu] = a[1] * dS[mu]"),
    ("frank3_twist_factor_two", "(nxdT - 2.0 * fp.T * fp.c[mu])", "(nxdT - fp.T * fp.c[mu])"),
    ("frank3_bend_stress_transposed", "ac[2] * (fp.B[b] * n[g] - fp.B[g] * n[b])",
     "ac[2] * (fp.B[g] * n[b] - fp.B[b] * n[g])"),
    ("frank3_chiral_constant", "*Kt = p->K22;", "*Kt = p->K11;"),
    ("frank3_mixed_stencil_sign", "nb2(st, m, 0, g, x, y, z, a, +1, b, +1) - nb2(st, m, 0, g, x, y, z, a, +1, b, -1)",
     "nb2(st, m, 0, g, x, y, z, a, +1, b, +1) + nb2(st, m, 0, g, x, y, z, a, +1, b, -1)"),
    ("frank3_reference_not_minimum", "    if (p->K22 < m) m = p->K22;\n", ""),
    ("frank3_no_div_B", "a[2] * (divB * n[mu] + BdN", "a[2] * (BdN"),
    ("frank3_grad_T_drops_G", "dT[b] += G[b][g] * fp.c[g] + n[g] * dc[b][g];", "dT[b] += n[g] * dc[b][g];"),
    ("frank3_bend_force_sign", "- fp.S * fp.B[mu] - cxB);", "- fp.S * fp.B[mu] + cxB);"),
]

# the unanchored walls (R7') and the obstacles (R7''), against theirs
MUTATIONS_WALLS = [
    ("free_wall_mirror_layer", "return z == 0 ? 1 : p->nz - 2;", "return z == 0 ? 2 : p->nz - 3;"),
    ("free_wall_edges_anchored", "        if (field_kind == 0 && p->free_walls)\n            return f[(int64_t)c * st->N + idx(p, co[0], co[1], mirror_layer(p, co[2]))];\n", ""),
    ("obstacle_not_bounced", "if (is_solid(p, zd) || obstacle(s, xd, yd, zd))", "if (is_solid(p, zd))"),
    ("obstacle_director_moves", "                if (obstacle(s, x, y, z)) { /* fixed director at solid nodes */",
     "                if (0) { /* fixed director at solid nodes */"),
    ("obstacle_velocity_not_held", "if (obstacle(s, x, y, z)) { /* no slip: an obstacle node is at rest */",
     "if (0) { /* no slip: an obstacle node is at rest */"),
    ("obstacle_stress_kept", "if (obstacle(st, x, y, z)) continue; /* sigma = 0 at solid nodes */",
     "/* sigma = 0 at solid nodes */"),
]

PINS = [
    pins.test_lattice_isotropy,
    lambda: pins.test_equilibrium_moments(False),
    lambda: pins.test_equilibrium_moments(True),
    pins.test_guo_source_moments,
    pins.test_uniform_acceleration_exact,
    pins.test_mass_conservation_coupled_channel,
    pins.test_momentum_growth_periodic_with_coupling,
    pins.test_lbm_step_matches_vectorised_implementation,
    pins.test_poiseuille_magic_tau_exact,
    pins.test_poiseuille_curvature_and_slip,
    pins.test_shear_wave_viscosity,
    pins.test_shifted_equals_unshifted_fp64,
    pins.test_director_rhs_exact_on_polynomials,
    pins.test_molecular_field_is_minus_energy_gradient,
    pins.test_director_relaxation_decreases_energy,
    pins.test_helix_is_stationary,
    pins.test_heun_growth_factor_of_linear_mode,
    pins.test_leslie_flow_alignment_angle,
    pins.test_force_summation_by_parts,
    pins.test_alpha4p_term_on_shear_wave,
    pins.test_elastic_stress_satisfies_ericksen_identity,
    pins.test_viscous_stress_power_identity,
    pins.test_checkerboard_velocity_mode_is_undamped,
    pins.test_warm_start_converges_back_to_steady_flow,
    lambda: pins.test_hybrid_loop_matches_numpy_step(4, 4, 6, 2, True),
    lambda: pins.test_hybrid_loop_matches_numpy_step(3, 5, 6, 3, False),
    pins.test_hybrid_loop_variants_match_numpy_step,
    pins.test_tube_centroids_of_analytic_tubes,
]

# cheapest first: the mode-rate pins catch most mistakes in a second
PINS_FRANK3 = [
    f3.test_equal_constants_reduce_to_one_constant,
    lambda: f3.test_single_mode_relaxation_rate(0, 0),
    lambda: f3.test_single_mode_relaxation_rate(1, 1),
    lambda: f3.test_single_mode_relaxation_rate(2, 2),
    lambda: f3.test_elastic_stress_satisfies_ericksen_identity_three_constants(f3.ORDERINGS[0]),
    lambda: f3.test_elastic_stress_satisfies_ericksen_identity_three_constants(f3.ORDERINGS[1]),
    lambda: f3.test_molecular_field_converges_to_variational_derivative(f3.ORDERINGS[0]),
    lambda: f3.test_molecular_field_converges_to_variational_derivative(f3.ORDERINGS[1]),
]

PINS_WALLS = [
    lambda: fw.test_uniform_tilted_director_is_stationary(False),
    lambda: fw.test_uniform_tilted_director_is_stationary(True),
    lambda: fw.test_neumann_mode_growth_factor(False),
    lambda: fw.test_neumann_mode_growth_factor(True),
    fw.test_free_walls_equal_a_mirrored_periodic_box,
    ob.test_mask_layers_reproduce_the_walls,
    ob.test_poiseuille_across_mask_walls_at_magic_tau,
    ob.test_symmetric_post_gives_mirror_symmetric_flow,
    ob.test_mass_conserved_with_obstacles_and_coupling,
]


def _caught(lib, pin_list) -> str:
    saved = oo._lib
    oo._lib = lib
    try:
        for pin in pin_list:
            try:
                pin()
            except Exception as e:  # an assertion or a numerical failure
                return getattr(pin, "__name__", "pin") + f": {type(e).__name__}"
        return ""
    finally:
        oo._lib = saved


@pytest.mark.parametrize("name,old,new,pin_list", [m + (PINS,) for m in MUTATIONS] +
                         [m + (PINS_FRANK3,) for m in MUTATIONS_FRANK3] +
                         [m + (PINS_WALLS,) for m in MUTATIONS_WALLS],
                         ids=[m[0] for m in MUTATIONS + MUTATIONS_FRANK3 + MUTATIONS_WALLS])
def test_planted_mistake_is_caught(name, old, new, pin_list, tmp_path):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {old}"
    mutated = src.replace(old, new, 1)
    cpath = tmp_path / "el_oracle.c"
    cpath.write_text(mutated)
    (tmp_path / "el_oracle.h").write_text(open(SRC.replace(".c", ".h")).read())
    lpath = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o",
                           str(lpath), str(cpath), "-lm"])
    caught_by = _caught(oo.load_library(str(lpath)), pin_list)
    print(f"{name}: caught by {caught_by}")
    assert caught_by, f"no pin fails for the planted mistake {name!r}"
