"""The pins catch plausible mistakes: each case plants one mistake in a copy of
the oracle source (on the CPU), builds it, and requires that at least one pin
fails when the oracle calls are routed to the mutant."""
import os
import shutil
import tempfile

import numpy as np
import pytest

import tests.test_oracle_deam as D
import tests.test_oracle_geometry as Gm
import tests.test_oracle_unrolled as U
import tests.test_oracle_penalty as Pn
import tests.test_oracle_os as Os
import tests.test_oracle_dual as Du
import tests.test_oracle_bowtie as Bt

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "oracle", "deam_oracle.c")

MUTATIONS = {
    "update_sign": ("c[(long)i * V + x] -= log(bt / bh) / Z[i];",
                    "c[(long)i * V + x] += log(bt / bh) / Z[i];"),
    "update_wrong_Z": ("c[(long)i * V + x] -= log(bt / bh) / Z[i];",
                       "c[(long)i * V + x] -= log(bt / bh) / Z[0];"),
    "no_substitution": ("if (metal) ra[i][j] = a[i][j];", "if (0) ra[i][j] = a[i][j];"),
    "midpoint_rule": ("double am = 0.5 * (a0 + a1);", "double am = a0;"),
    "exponent_sign": ("double ex = exp(-(mu1 * l1 + mu2 * l2));",
                      "double ex = exp(-(mu1 * l1 - mu2 * l2));"),
    "basis_swap": ("nadd(&as[1][j], mu2 * q);", "nadd(&as[1][j], mu1 * q);"),
    "dropped_spectrum": ("for (int j = 0; j < 2; ++j) {\n        double q = I0[j * nE + e] * ex;",
                         "for (int j = 0; j < 2; ++j) {\n        double q = I0[0 * nE + e] * ex;"),
    "channel_offset_sign": ("- 0.5 * (g->n_cols - 1) - g->col_offset) * g->dgamma;",
                            "- 0.5 * (g->n_cols - 1) + g->col_offset) * g->dgamma;"),
    "fan_direction": ("double dirx = cg * ux - sg * uy, diry = sg * ux + cg * uy;",
                      "double dirx = cg * ux + sg * uy, diry = -sg * ux + cg * uy;"),
    "helix_direction": ("zs = ((double)v - 0.5 * (g->n_views - 1)) * g->feed_per_rot / g->views_per_rot;",
                        "zs = (0.5 * (g->n_views - 1) - (double)v) * g->feed_per_rot / g->views_per_rot;"),
    "idiv_term": ("term += (dj > 0.0 ? dj * log(dj / g) : 0.0) - dj + g;",
                  "term += (dj > 0.0 ? dj * log(dj / g) : 0.0) + dj - g;"),
    "band_overlap": ("int hi[3] = {g->nx, (b + 1) * band < g->ny ? (b + 1) * band : g->ny,",
                     "int hi[3] = {g->nx, (b + 1) * band < g->ny ? (b + 1) * band + 1 : g->ny,"),
    "grad_weight_sign": ("w[(long)i * R + y] = (ra[i][0] - a[i][0]) + (ra[i][1] - a[i][1]);",
                         "w[(long)i * R + y] = (ra[i][0] - a[i][0]) - (ra[i][1] - a[i][1]);"),
    "ray_length_2d": ("double L = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);",
                      "double L = sqrt(D[0] * D[0] + D[1] * D[1]);"),
    "step_vjp_ratio_term": ("if (!metal && g > 0.0) dwt += dj / (g * g) * a[k][j] * a[i][j];",
                            "if (!metal && g > 0.0) dwt -= dj / (g * g) * a[k][j] * a[i][j];"),
    "step_vjp_moment_index": ("if (metal || g > 0.0) dwt -= r * m[j][i][k];",
                              "if (metal || g > 0.0) dwt -= r * m[j][i][i];"),
    "step_vjp_hat_sign": ("dwh -= m[j][i][k];", "dwh += m[j][i][k];"),
    "step_vjp_upstream_sign": ("u[(long)i * V + x] = act ? -gi / (Z[i] * bt) : 0.0;",
                               "u[(long)i * V + x] = act ? gi / (Z[i] * bt) : 0.0;"),
    "fair_printed_sign": ("return delta * delta * (a - log1p(a));",
                          "return delta * delta * (a + log1p(-a));"),
    "fair_d1_unscaled": ("return t / (1.0 + fabs(t) / delta);", "return t / (1.0 + fabs(t));"),
    "pen_weight_squared": ("w[n] = 1.0 / sqrt(ddx * ddx + ddy * ddy + ddz * ddz);",
                           "w[n] = 1.0 / (ddx * ddx + ddy * ddy + ddz * ddz);"),
    "pen_no_z_neighbours": ("for (int oz = -1; oz <= 1; ++oz)", "for (int oz = 0; oz <= 0; ++oz)"),
    "pen_chain_factor": ("f += 2.0 * lambda * p;", "f += lambda * p;"),
    "pen_neighbour_sign": ("p += w[k] * orc_fair_d1(2.0 * mid - ck - ci[nb[k]], delta);",
                           "p += w[k] * orc_fair_d1(2.0 * mid - ck + ci[nb[k]], delta);"),
    "pen_data_term": ("double f = bt - bh * exp(-Z[i] * (mid - ck));",
                      "double f = bt - bh * exp(Z[i] * (mid - ck));"),
    "pen_bisection_side": ("if (f > 0.0) hi = mid;", "if (f < 0.0) hi = mid;"),
    "pen_skipped_voxel": ("if (!(bt > 0.0 && bh > 0.0)) return ck;",
                          "if (!(bt > 0.0 && bh > 0.0)) return 0.0;"),
    "bowtie_sign": ("double fb = bt ? exp(-(mu1 * bt[kb] + mu2 * bt[n_cols + kb])) : 1.0;",
                    "double fb = bt ? exp(+(mu1 * bt[kb] + mu2 * bt[n_cols + kb])) : 1.0;"),
    "bowtie_channel": ("long kb = bt ? y % n_cols : 0;", "long kb = bt ? (y / n_cols) % n_cols : 0;"),
    "bowtie_basis_swap": ("exp(-(mu1 * bt[kb] + mu2 * bt[n_cols + kb]))",
                          "exp(-(mu2 * bt[kb] + mu1 * bt[n_cols + kb]))"),
    "dual_both_spectra_in_low_scan": ("I0j[e] = j == 0 ? I0[e] : 0.0;", "I0j[e] = I0[e];"),
    "dual_last_scan_only": ("for (long x = 0; x < 4 * V; ++x) b[x] += bs[x];",
                            "for (long x = 0; x < 4 * V; ++x) b[x] = bs[x];"),
    "dual_counts_slot": ("memcpy(dd + (long)j * R[j], d[j],", "memcpy(dd, d[j],"),
    "dilate_one_sided": ("for (long q = k - radius; q <= k + radius; ++q)",
                         "for (long q = k; q <= k + radius; ++q)"),
    "os_subset_order": ("if ((y / per_view) % n_sub != s)", "if ((y / per_view) % n_sub != (s + 1) % n_sub)"),
    "os_no_restriction": ("if ((y / per_view) % n_sub != s)", "if (0)"),
    "os_history_at_last_subset": ("if (s == 0 && obj_hist) obj_hist[k]", "if (obj_hist) obj_hist[k]"),
    "vjp_weight_sign": ("w[(long)i * R + y] = -(v[y] * a[i][0] + v[R + y] * a[i][1]);",
                        "w[(long)i * R + y] = (v[y] * a[i][0] + v[R + y] * a[i][1]);"),
    "vjp_spectrum_index": ("w[(long)i * R + y] = -(v[y] * a[i][0] + v[R + y] * a[i][1]);",
                           "w[(long)i * R + y] = -(v[y] * a[i][0] + v[R + y] * a[i][0]);"),
    "vjp_upstream_swap": ("w[(long)i * R + y] = -(v[y] * a[i][0] + v[R + y] * a[i][1]);",
                          "w[(long)i * R + y] = -(v[R + y] * a[i][0] + v[y] * a[i][1]);"),
    "forward_rays_ignores_list": ("orc_ray(g, rays[s], S, P);", "orc_ray(g, s, S, P);"),
    "forward_rays_layout": ("out[(long)k * n_sel + s] = nval(&acc);",
                            "out[(long)s * nch + k] = nval(&acc);"),
    "pen_history_without_penalty": (
        "obj_hist[k] = orc_sum(R, obj) + orc_penalty(g, c, lambda, delta);",
        "obj_hist[k] = orc_sum(R, obj);"),
}

PINS = [
    lambda o: Gm.test_siddon_matches_voxelwise_clipping(o, Gm.small_fan),
    lambda o: Gm.test_siddon_matches_voxelwise_clipping(o, Gm.small_box3d),
    lambda o: Gm.test_row_sum_is_box_chord(o, "fan64"),
    lambda o: Gm.test_row_sum_is_box_chord(o, "helical_small"),
    lambda o: Gm.test_pixelised_disk_chord_bracket(o, "fan64", -5.0, 8.0, 9.5),
    lambda o: Gm.test_pixelised_disk_chord_bracket(o, "offset", 6.1, -3.3, 7.0),
    lambda o: Gm.test_helical_cylinder_chord_bracket(o),
    lambda o: Gm.test_adjoint_identity(o, "fan64"),
    lambda o: D.test_single_bin_beer_lambert(o),
    lambda o: D.test_flat_attenuation_sums_spectrum(o),
    lambda o: D.test_linear_family_constraint(o),
    lambda o: D.test_idiv_vanishes_on_consistent_data_and_matches_nll(o),
    lambda o: D.test_all_metal_mask_is_noop(o),
    lambda o: D.test_monoenergetic_matches_textbook_am(o),
    lambda o: D.test_masked_idiv_nonincreasing(o, "fan64", 20, True),
    lambda o: D.test_gradient_matches_finite_differences(o),
    lambda o: U.test_step_vjp_matches_finite_differences(o),
    lambda o: Pn.test_fair_potential_closed_forms(o),
    lambda o: Pn.test_penalty_ramp_2d_closed_form(o, 0.7, 1.3),
    lambda o: Pn.test_penalty_ramp_3d_closed_form(o),
    lambda o: Pn.test_update_pen_lambda_zero_is_deam_update(o, Pn.small_box3d),
    lambda o: Pn.test_update_pen_quadratic_limit_lambert_w(o, Pn.small_box3d),
    lambda o: Pn.test_update_pen_minimises_voxel_surrogate(o, Pn.small_fan, 5e5, 0.002),
    lambda o: Pn.test_penalised_objective_decreases(o, 2e5, 0.005),
    lambda o: Os.test_one_subset_is_deam(o),
    lambda o: Os.test_subset_step_is_deam_on_the_subset_scan(o, 3),
    lambda o: Du.test_same_scans_are_deam(o),
    lambda o: Du.test_dilate_mask(o),
    lambda o: Bt.test_filter_is_a_shift_of_the_line_integrals(o, "am"),
    lambda o: D.test_vjp_weights_are_finite_difference_products(o),
    lambda o: Gm.test_forward_rays_equals_forward(o, "fan64"),
]


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="orc_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def test_pins_pass_on_the_real_oracle(orc):
    for pin in PINS:
        pin(orc)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(orc, workdir, name):
    old, new = MUTATIONS[name]
    src = open(ORACLE_SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    path = os.path.join(workdir, f"{name}.c")
    open(path, "w").write(src.replace(old, new))
    lib = orc.compile_library(path, os.path.join(workdir, f"lib{name}.so"))
    caught = None
    with orc.use_library(lib):
        for i, pin in enumerate(PINS):
            try:
                with np.errstate(all="ignore"):
                    pin(orc)
            except (AssertionError, RuntimeError, ValueError, FloatingPointError):
                caught = i
                break
    assert caught is not None, f"no pin caught the mutation {name}"
