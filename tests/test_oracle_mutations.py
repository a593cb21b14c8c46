"""The pins catch plausible mistakes in the oracle (CPU).

Each case copies the oracle's C source, plants one mistake of the kind a
reader could make (a dropped term, a wrong factor, a swapped weight, a
one-sided cleaning rule, a shifted key), builds the copy, points the oracle
loader at it, and checks that at least one of the pins meant for that part
fails.  The committed oracle is never modified.
"""
import os
import subprocess

import pytest

import oracle
import test_clusterizer_oracle as clu
import test_collisions_oracle as col
import test_compression_oracle as cmp
import test_oracle_pins as pins
import test_merge_oracle as mrg
import test_refit_oracle as rft
from conftest import cached_event, cached_oracle

JAC_CASES = [([3.0, -20.0, 0.3, 0.7, -2.5], 40.0), ([10.0, 100.0, 0.05, 1.0, 8.0], -25.0)]

MUTATIONS = [
    ("jacobian_dy_dqpt",
     "    F[0 * 5 + 4] = b;", "    F[0 * 5 + 4] = 0.5 * b;",
     [lambda: [pins.test_jacobian_matches_finite_differences(p, dx) for p, dx in JAC_CASES]]),
    ("propagation_dy",
     "  const double dy = dx * N / D;", "  const double dy = dx * N / (D * 1.0001);",
     [pins.test_propagation_matches_closed_form_crossings]),
    ("kalman_cov_term",
     "      nc[i * 5 + j] = cov[i * 5 + j] - (K[i][0] * cov[0 * 5 + j] + K[i][1] * cov[1 * 5 + j]);",
     "      nc[i * 5 + j] = cov[i * 5 + j] - (K[i][0] * cov[0 * 5 + j]);",
     [pins.test_kalman_equals_batch_least_squares, pins.test_fit_pulls_are_standard_normal]),
    ("seed_half_angle",
     "  const double sa = C * d13 * 0.5;", "  const double sa = C * d13 * 0.45;",
     [pins.test_seed_exact_on_helix]),
    ("score_weights_swapped",
     "(__int128)P->w_y * Ry * Ry + (__int128)P->w_z * Rz * Rz",
     "(__int128)P->w_z * Ry * Ry + (__int128)P->w_y * Rz * Rz",
     [pins.test_golden_neighbour_rule, pins.test_neighbour_score_weights_decide]),
    ("cleaning_one_sided",
     "    upc[m] = (up[m] >= 0 && dn[up[m]] == m) ? up[m] : -1;",
     "    upc[m] = up[m];",
     [pins.test_cleaning_and_chain_invariants]),
    ("constructor_no_pass2_reset",
     "    s = last;\n    cov_init(s.cov, P);\n    s.chi2 = 0;\n    int nfit = 0;",
     "    s = last;\n    s.chi2 = 0;\n    int nfit = 0;",
     [pins.test_constructor_fit_agrees_with_two_pass_fit]),
    ("pickup_weights_swapped",
     "const int64_t s = (int64_t)P->w_y * dY * dY + (int64_t)P->w_z * dZ * dZ;",
     "const int64_t s = (int64_t)P->w_z * dY * dY + (int64_t)P->w_y * dZ * dZ;",
     [pins.test_pickup_score_weights_decide]),
    ("walk_stops_one_miss_early",
     "        } else if (++misses > P->max_miss) {",
     "        } else if (++misses >= P->max_miss) {",
     [pins.test_walk_crosses_max_miss_empty_rows_but_not_more]),
    ("keep_threshold_strict",
     "owned >= P->n_min &&", "owned > P->n_min &&",
     [pins.test_keep_threshold_boundary, pins.test_selection_invariants]),
    ("pickup_tie_reversed",
     "if (s < best_s || (s == best_s && id < best_id)) {", "if (s < best_s || (s == best_s && id > best_id)) {",
     [pins.test_pickup_tie_goes_to_the_smaller_id]),
    ("chi2_z_term_dropped",
     "  *chi2 += r0 * (I00 * r0 + I01 * r1) + r1 * (I01 * r0 + I11 * r1);",
     "  *chi2 += r0 * (I00 * r0 + I01 * r1);",
     [pins.test_fit_chi2_per_degree_of_freedom_is_one]),
    ("pass2_stops_one_miss_early",
     "      } else if (r < r1 && ++misses > P->max_miss) {",
     "      } else if (r < r1 && ++misses >= P->max_miss) {",
     [pins.test_pass2_crosses_max_miss_empty_rows_below_the_chain_but_not_more]),
    ("no_sector_edge_stop",
     "  if (llabs(Yp) > g->H + P->ext_edge_q) {",
     "  if (0 && llabs(Yp) > g->H + P->ext_edge_q) {",
     [pins.test_walk_stops_where_the_prediction_leaves_the_sector]),
    ("fragile_ignores_a_changed_pick",
     "          if (r2.found != r.found || r2.stop != r.stop) *fragile = 1;",
     "          if (r2.stop != r.stop) *fragile = 1;",
     [pins.test_fragile_flag_marks_only_decisions_a_rounding_boundary_can_flip]),
    ("fragile_margin_inverted",
     "    const int ny = fabs(fy - 0.5) < eps, nz = fabs(fz - 0.5) < eps;",
     "    const int ny = fabs(fy - 0.5) > eps, nz = fabs(fz - 0.5) > eps;",
     [pins.test_fragile_flag_marks_only_decisions_a_rounding_boundary_can_flip]),
    ("owner_key_nfit_field",
     "res->trk_key[t] = ((uint32_t)o.nfit << 24) | (0xFFFFFFu - local);",
     "res->trk_key[t] = ((uint32_t)o.nfit << 20) | (0xFFFFFFu - local);",
     [pins.test_owner_is_max_key_over_incidences, pins.test_selection_invariants]),
    ("zdca_arc_sign",
     "  return z + tgl * sT;", "  return z - tgl * sT;",
     [col.test_zdca_is_the_vertex_z_of_generated_helices]),
    ("collision_t0_ignores_side",
     "    c_t0[c] = -(double)c_side[c] * c_zdca[c] / v_drift;", "    c_t0[c] = -c_zdca[c] / v_drift;",
     [col.test_histogram_peaks_and_assignment_hand_worked]),
    ("peak_tie_to_both",
     "if (b - d >= 0 && h[b - d] >= h[b]) peak = 0;", "if (b - d >= 0 && h[b - d] > h[b]) peak = 0;",
     [col.test_histogram_peaks_and_assignment_hand_worked]),
    ("loopers_form_candidates",
     "if (b >= 0 && fabs(k * params[t * 5 + 4]) < c_max) hist", "if (b >= 0) hist",
     [col.test_histogram_peaks_and_assignment_hand_worked]),
    ("loopers_in_the_mean",
     "    if (fabs(k * params[t * 5 + 4]) < c_max) {\n      c_form[c] += 1;",
     "    if (1) {\n      c_form[c] += 1;",
     [col.test_histogram_peaks_and_assignment_hand_worked]),
    ("nearest_tie_to_the_upper_bin",
     "      if (b - d >= 0 && cs[b - d] >= 0) { collision[t] = (int32_t)cs[b - d]; break; }\n"
     "      if (b + d < nb && cs[b + d] >= 0) { collision[t] = (int32_t)cs[b + d]; break; }",
     "      if (b + d < nb && cs[b + d] >= 0) { collision[t] = (int32_t)cs[b + d]; break; }\n"
     "      if (b - d >= 0 && cs[b - d] >= 0) { collision[t] = (int32_t)cs[b - d]; break; }",
     [col.test_histogram_peaks_and_assignment_hand_worked]),
    ("clusterizer_tie_to_the_later_digit",
     "const int later = dp > 0 || (dp == 0 && dt > 0);", "const int later = dp < 0 || (dp == 0 && dt < 0);",
     [clu.test_plateau_and_diagonal_ties_give_one_peak]),
    ("clusterizer_neighbours_across_rows",
     "if (p + dp < 0 || p + dp >= np) continue; /* neighbours stay in the row */",
     "if (j + dp < (int64_t)u * pads_total || j + dp >= (int64_t)(u + 1) * pads_total) continue;",
     [clu.test_neighbours_stay_in_their_row_pad_and_time_window]),
    ("clusterizer_5x5_time_window",
     "pad_range(pad_offsets, time, j + dp, t - 1, t + 1, &a, &b);",
     "pad_range(pad_offsets, time, j + dp, t - 2, t + 2, &a, &b);",
     [clu.test_neighbours_stay_in_their_row_pad_and_time_window, lambda: clu.test_matches_a_dense_map_implementation(1)]),
    ("clusterizer_pad_moment_sign",
     "Sp += w * dp;", "Sp -= w * dp;",
     [clu.test_plateau_and_diagonal_ties_give_one_peak]),
    ("compression_residual_sign",
     "        vy = ((double)y[c] - out[0]) / step;", "        vy = (out[0] - (double)y[c]) / step;",
     [cmp.test_displacements_come_back_as_codes]),
    ("compression_removal_at_the_cut",
     "if (fabs(p[4]) * pt_remove > 1.0) {", "if (fabs(p[4]) * pt_remove >= 1.0) {",
     [cmp.test_removal_cut_and_unattached_rounding]),
    ("compression_model_at_the_row_below",
     "(double)row_x[row[c]], k, sinphi_max, out, NULL)",
     "(double)row_x[row[c] > 0 ? row[c] - 1 : 0], k, sinphi_max, out, NULL)",
     [cmp.test_clusters_on_the_helix_have_code_zero]),
    ("compression_z_against_y",
     "        vz = ((double)z[c] - out[1]) / step;", "        vz = ((double)z[c] - out[0]) / step;",
     [cmp.test_clusters_on_the_helix_have_code_zero]),
    ("refit_not_in_quanta",
     "hits[first[t] + j];\n      X[j] = row_x[row[h]];\n      Y[j] = nearbyint(256.0 * (double)y[h]) / 256.0;",
     "hits[first[t] + j];\n      X[j] = row_x[row[h]];\n      Y[j] = (double)y[h];",
     [rft.test_refit_takes_clusters_in_quanta]),
    ("refit_rounds_half_up",
     "hits[first[t] + j];\n      X[j] = row_x[row[h]];\n      Y[j] = nearbyint(256.0 * (double)y[h]) / 256.0;",
     "hits[first[t] + j];\n      X[j] = row_x[row[h]];\n      Y[j] = floor(256.0 * (double)y[h] + 0.5) / 256.0;",
     [rft.test_refit_takes_clusters_in_quanta]),
    ("refit_x_of_the_row_below",
     "hits[first[t] + j];\n      X[j] = row_x[row[h]];", "hits[first[t] + j];\n      X[j] = row_x[row[h] > 0 ? row[h] - 1 : 0];",
     [rft.test_refit_of_noise_free_helices_gives_the_helix_at_both_ends]),
    ("refit_hit_list_reversed",
     "      const int32_t h = hits[first[t] + j];", "      const int32_t h = hits[first[t] + n - 1 - j];",
     [rft.test_refit_of_noise_free_helices_gives_the_helix_at_both_ends]),
    ("merge_turn_sign",
     "  const double s2 = s * cd - c * sd, c2 = c * cd + s * sd;",
     "  const double s2 = s * cd + c * sd, c2 = c * cd - s * sd;",
     [mrg.test_turn_and_transport_reproduce_the_helix_in_the_next_sector]),
    ("merge_turn_jacobian_y",
     "    J[0 * 5 + 0] = c / c2;", "    J[0 * 5 + 0] = c2 / c;",
     [lambda: [mrg.test_turn_jacobian_matches_finite_differences(c) for c in
               (([3.0, -20.0, 0.3, 0.7, -2.5], 120.0, 0.35), ([20.0, 5.0, 0.6, 0.2, 0.8], 90.0, 0.1))]]),
    ("merge_not_mutual",
     "    if (b >= 0 && ib[b] == a) {", "    if (b >= 0) {",
     [mrg.test_hand_worked_links]),
    ("merge_rows_may_touch",
     "      for (int32_t r = last_row[a] + 1; r <= last_row[a] + max_gap && r < n_rows; ++r) {",
     "      for (int32_t r = last_row[a]; r <= last_row[a] + max_gap && r < n_rows; ++r) {",
     [mrg.test_hand_worked_rules]),
    ("merge_tie_to_the_larger_index",
     "          if (c2 < ib_c[b] || (c2 == ib_c[b] && a < ib[b])) {",
     "          if (c2 < ib_c[b] || (c2 == ib_c[b] && a > ib[b])) {",
     [mrg.test_hand_worked_links]),
    ("merge_no_z_window",
     "          if (!(fabs(p_in[b * 5 + 1] - p_out[a * 5 + 1]) <= dz_max)) continue;\n", "",
     [mrg.test_hand_worked_rules]),
    ("merge_no_y_window",
     "          if (!(fabs(p_in[b * 5] - yc[0]) <= dy_max)) continue;\n", "",
     [mrg.test_hand_worked_rules]),
    ("chain_turn_backwards",
     "        if (turn_state(&s, unit_alpha[u[j]] - unit_alpha[cu], k, P) != 0) return -1;",
     "        if (turn_state(&s, unit_alpha[cu] - unit_alpha[u[j]], k, P) != 0) return -1;",
     [mrg.test_chain_fit_of_helices_across_two_sectors_gives_the_helix]),
    ("chain_pass2_without_turn",
     "      if (turn_state(&s, unit_alpha[u[j]] - unit_alpha[cu], k, P) != 0) return -1;\n      cu = u[j];",
     "      cu = u[j];",
     [mrg.test_chain_fit_of_helices_across_two_sectors_gives_the_helix]),
    ("merge_across_sides",
     "      if (unit_side[w] != unit_side[unit[a]]) continue;\n", "",
     [mrg.test_hand_worked_rules]),
]


def _build_mutant(tmp_path, find, replace):
    src = open(oracle._SRC).read()
    assert src.count(find) == 1, "mutation site not unique: %r" % find
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(find, replace))
    lib = tmp_path / "mutant.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=c11", "-D_POSIX_C_SOURCE=200809L", "-shared",
                           "-fPIC", "-o", str(lib), str(path), "-lm"])
    return str(lib)


@pytest.mark.parametrize("name,find,replace,checks", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, find, replace, checks):
    lib = _build_mutant(tmp_path, find, replace)
    saved = (oracle._LIB, oracle._lib)
    cached_oracle.cache_clear()
    cached_event.cache_clear()
    oracle._LIB, oracle._lib = lib, None
    caught = []
    try:
        for check in checks:
            try:
                check()
            except AssertionError as e:
                caught.append(str(e)[:120])
    finally:
        oracle._LIB, oracle._lib = saved
        cached_oracle.cache_clear()
    assert caught, "no pin caught the planted mistake %s" % name
