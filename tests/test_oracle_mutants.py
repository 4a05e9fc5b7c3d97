"""The pins catch plausible mistakes: each mutant below plants one mistake in
a copy of oracle.c (on the CPU), and at least one pin must fail against it.
The unmutated oracle passes the same pins (test_oracle_pins*)."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_accum_pins as T
import test_oracle_codec_pins as K
import test_oracle_grad_pins as G
import test_oracle_march_pins as M
import test_oracle_policy_pins as R
import test_oracle_spheroid_pins as S
import test_oracle_pins as P

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()

# (name, original text, mutated text): one mistake each
MUTANTS = [
    ("drop transmittance in colour", "C[k] += T * al * SPH(h->id, 4 + k);", "C[k] += al * SPH(h->id, 4 + k);"),
    ("transmittance keeps alpha", "T *= (1.0 - al);", "T *= al;"),
    ("tangent is a miss", "return disc >= 0.0 && t0 > 0.0 && t0 < t_max;", "return disc > 0.0 && t0 > 0.0 && t0 < t_max;"),
    ("exit instead of entry", "double t0 = disc >= 0.0 ? b - sqrt(disc) : NAN;", "double t0 = disc >= 0.0 ? b + sqrt(disc) : NAN;"),
    ("back to front order", "if (a->t0 < b->t0) return -1;\n    if (a->t0 > b->t0) return 1;",
     "if (a->t0 > b->t0) return -1;\n    if (a->t0 < b->t0) return 1;"),
    ("tie broken by larger id", "return (a->id > b->id) - (a->id < b->id);", "return (a->id < b->id) - (a->id > b->id);"),
    ("stop only above the threshold", "int stop = A >= alpha_stop;", "int stop = A > alpha_stop;"),
    ("footprint without factor 2", "double footprint = 2.0 * t * cam->tan_half_fov_y / (double)H;",
     "double footprint = t * cam->tan_half_fov_y / (double)H;"),
    ("rows counted from the bottom", "double sy = (1.0 - (2.0 * (double)y + 1.0) / c->height) * c->tan_half_fov_y;",
     "double sy = ((2.0 * (double)y + 1.0) / c->height - 1.0) * c->tan_half_fov_y;"),
    ("no aspect ratio", "double sx = ((2.0 * (double)x + 1.0) / c->width - 1.0) * c->tan_half_fov_y * aspect;",
     "double sx = ((2.0 * (double)x + 1.0) / c->width - 1.0) * c->tan_half_fov_y;"),
    ("perpendicular offset sign", "double v[3] = {oc[0] - b * d[0], oc[1] - b * d[1], oc[2] - b * d[2]};",
     "double v[3] = {oc[0] + b * d[0], oc[1] + b * d[1], oc[2] + b * d[2]};"),
    ("soft alpha linear falloff", "return a * (1.0 - u) * (1.0 - u);", "return a * (1.0 - u);"),
    ("alpha gradient chain", "acc[8 * j + 7] += dal * (1.0 - u) * (1.0 - u);", "acc[8 * j + 7] += dal * (1.0 - u);"),
    ("remainder ignores transmittance", "R = al * w + (1.0 - al) * R;", "R = al * w + R;"),
    ("radius gradient power", "acc[8 * j + 3] += dal * 4.0 * a * (1.0 - u) * h->q / (r * r * r);",
     "acc[8 * j + 3] += dal * 4.0 * a * (1.0 - u) * h->q / (r * r);"),
    ("half truncates", "double q = rint(ldexp(a, 10 - E));", "double q = floor(ldexp(a, 10 - E));"),
    ("no colour clamp", "col[k] = kc < 0.0 ? 0.0 : (kc > 1.0 ? 1.0 : kc);", "col[k] = kc;"),
    ("premultiplied colour kept", "double kc = (double)rgba[4 * i + k] / A;", "double kc = (double)rgba[4 * i + k];"),
    ("march samples at interval starts", "const double t = t_in + ((double)j + 0.5) * dt;",
     "const double t = t_in + (double)j * dt;"),
    ("march weight without transmittance", "const double w = (1.0 - A) * s;", "const double w = s;"),
    ("trilinear weights swapped", "w *= up ? frac[a] : 1.0 - frac[a];", "w *= up ? 1.0 - frac[a] : frac[a];"),
    ("march colour ramp", "C[1] += w * (4.0 * u * (1.0 - u));", "C[1] += w * (u * (1.0 - u));"),
    ("march never stops", "if (A >= stop_alpha) break;", "if (A > 2.0) break;"),
    ("codec decodes cell corners", "c[a] = lo[a] + ((double)((w >> (18 * a)) & 0x3ffffu) + 0.5) * step;",
     "c[a] = lo[a] + ((double)((w >> (18 * a)) & 0x3ffffu)) * step;"),
    ("codec radius steps", "double code = floor(64.0 * log2(r / r_unit) + 0.5) + 512.0;",
     "double code = floor(32.0 * log2(r / r_unit) + 0.5) + 512.0;"),
    ("codec colour truncates", "w |= (uint32_t)floor(v * 255.0 + 0.5) << (8 * ch);",
     "w |= (uint32_t)floor(v * 255.0) << (8 * ch);"),
    ("codec axis order", "w |= orc_quant(c[a], lo[a], size, 18) << (18 * a);",
     "w |= orc_quant(c[2 - a], lo[a], size, 18) << (18 * a);"),
    ("accumulate reads x for every axis", "double q = floor(((double)cr[a] - lo[a]) / size * (double)grid);",
     "double q = floor(((double)cr[0] - lo[a]) / size * (double)grid);"),
    ("accumulate cells overlap in the key", "key |= (uint64_t)q << (20 * a);", "key |= (uint64_t)q << (2 * a);"),
    ("accumulate one origin for all axes", "double q = floor(((double)cr[a] - lo[a]) / size * (double)grid);",
     "double q = floor(((double)cr[a] - lo[0]) / size * (double)grid);"),
    ("accumulate rounds to the nearest cell", "double q = floor(((double)cr[a] - lo[a]) / size * (double)grid);",
     "double q = rint(((double)cr[a] - lo[a]) / size * (double)grid);"),
    ("opacity radius linear in alpha", "if (mode == 1) r = r * sqrt(A > a_floor ? A : a_floor);",
     "if (mode == 1) r = r * (A > a_floor ? A : a_floor);"),
    ("opacity floor ignored", "if (mode == 1) r = r * sqrt(A > a_floor ? A : a_floor);",
     "if (mode == 1) r = r * sqrt(A);"),
    ("interval centre at its near end", "t = 0.5 * (lo + hi);", "t = lo;"),
    ("interval full length as radius", "half_len = 0.5 * (hi - lo);", "half_len = hi - lo;"),
    ("interval radius ignores the footprint", "if (mode == 2 && kappa * half_len > r) r = kappa * half_len;",
     "if (mode == 2) r = kappa * half_len;"),
    ("interval accepts a reversed interval", "if (!(isfinite(lo) && isfinite(hi) && lo > 0.0 && hi >= lo)) continue;",
     "if (!(isfinite(lo) && isfinite(hi) && lo > 0.0)) continue;"),
    ("interval left open", "if (t_lo != INFINITY && t_hi == INFINITY) t_hi = t_last;", ""),
    ("interval opens at the depth alpha", "if (t_lo == INFINITY && A >= interval_lo) t_lo = t;",
     "if (t_lo == INFINITY && A >= depth_alpha) t_lo = t;"),
    ("accumulate no lower clamp", "if (!(q >= 0.0)) q = 0.0; /* also NaN */", ""),
    ("accumulate no upper clamp", "if (q > (double)(grid - 1)) q = (double)(grid - 1);", ""),
    ("accumulate keeps one frame too long", "if ((int32_t)hist_age[i] + 1 > max_age) continue;",
     "if ((int32_t)hist_age[i] > max_age) continue;"),
    ("spheroid direction scaled by h across", "D[k] = d[k] / r + du * w * u[k];", "D[k] = d[k] / h + du * w * u[k];"),
    ("spheroid axis term reversed", "const double w = 1.0 / h - 1.0 / r;", "const double w = 1.0 / r - 1.0 / h;"),
    ("spheroid exit instead of entry", "const double t0 = disc >= 0.0 ? tm - sqrt(disc / DD) : NAN;",
     "const double t0 = disc >= 0.0 ? tm + sqrt(disc / DD) : NAN;"),
    ("spheroid chord not scaled by D.D", "const double t0 = disc >= 0.0 ? tm - sqrt(disc / DD) : NAN;",
     "const double t0 = disc >= 0.0 ? tm - sqrt(disc) : NAN;"),
    ("spheroid half-length ignores kappa", "const double h = kappa * half_len > r ? kappa * half_len : r;",
     "const double h = half_len > r ? half_len : r;"),
    ("spheroid half-length may fall below r", "const double h = kappa * half_len > r ? kappa * half_len : r;",
     "const double h = kappa * half_len;"),
    ("spheroid axis along the view, not the pixel ray", "for (int k = 0; k < 3; ++k) axis[4 * n + k] = (float)d[k];",
     "for (int k = 0; k < 3; ++k) axis[4 * n + k] = (float)(-cam->forward[k]);"),
    ("spheroid grazing band unscaled", "res[2] = e[1] * r * r;", "res[2] = e[1];"),
]

# pins run against each mutant (parametrised pins with their cases)
PINS = [
    lambda: [P.test_sphere_closed_form(*c) for c in [((0, 0, 5), 1.0, True, 4.0, 0.0),
                                                     ((0.6, 0, 5), 1.0, True, 4.2, 0.36),
                                                     ((1, 0, 5), 1.0, True, 5.0, 1.0)]],
    P.test_sphere_matches_quadratic_roots,
    P.test_two_spheres_hand_computed,
    P.test_stop_at_alpha_hand_computed,
    P.test_first_hit_special_case,
    P.test_equal_depth_tie_breaks_by_id,
    P.test_stop_knife_edge_reports_both_branches,
    P.test_hit_sets_against_quadratic_roots_on_tiny_scene,
    P.test_unproject_eq1_closed_form,
    P.test_unproject_colour_is_straight_and_clamped,
    P.test_unproject_footprint_values,
    P.test_half_rounding_matches_numpy,
    P.test_identity_reprojection_reproduces_source,
    G.test_soft_alpha_closed_form,
    G.test_two_sphere_constant_alpha_derivatives,
    lambda: G.test_analytic_gradient_matches_central_differences(oracle.MODE_SOFT, 0.99),
    lambda: [M.test_constant_volume_closed_form(v) for v in (0.6, 1.7, 12.0)],
    M.test_eye_inside_the_volume,
    M.test_linear_ramp_is_reproduced_and_clamped,
    M.test_trilinear_weights_on_a_single_voxel_pulse,
    M.test_ray_missing_the_cube_is_background,
    M.test_matches_the_input_generators_caster,
    K.test_hand_computed_words,
    K.test_round_trip_error_bounds,
    K.test_decoded_values_encode_to_the_same_words,
    K.test_clamping_and_monotone_codes,
    lambda: [R.test_marcher_interval_closed_form(v, st) for v, st in [(12.0, 0.999), (1.7, 0.999), (0.6, 0.999),
                                                                       (0.3, 0.999), (1.7, 0.5), (0.05, 0.999)]],
    R.test_policies_on_the_axis_hand_computed,
    lambda: [R.test_invalid_interval_drops_the_pixel(b) for b in [(np.inf, 3.0), (1.0, np.inf), (3.0, 1.0),
                                                                  (0.0, 1.0), (-1.0, 1.0), (np.nan, 1.0)]],
    R.test_interval_centre_on_the_pixel_ray,
    R.test_footprint_policy_is_the_plain_unprojection_and_full_opacity_too,
    lambda: [S.test_spheroid_closed_form(*c) for c in [((0, 0, 5), (0, 0, 1), 3.0, 1.0),
                                                         ((0, 0, 5), (1, 0, 0), 4.5, 1.0),
                                                         ((2, 0, 5), (1, 0, 0), 5.0, 0.0)]],
    S.test_spheroid_misses_and_eye_inside,
    S.test_equal_half_length_is_the_sphere,
    S.test_spheroid_matches_quadratic_roots,
    S.test_unproject_spheroids_on_the_axis_hand_computed,
    S.test_unproject_spheroids_lie_along_the_pixel_rays,
    S.test_view_along_the_source_ray_meets_the_tip,
    S.test_spheroid_tangent_pixel_is_flagged_grazing,
    T.test_hand_placed_cells,
    T.test_age_limits,
    lambda: [T.test_random_cells_by_construction(sd) for sd in (0, 1, 2)],
    T.test_merging_a_frame_twice,
    T.test_merged_layout_and_capacity,
]


def caught(lib_path: str) -> list[int]:
    """Indices of the pins that fail against the library at lib_path."""
    saved = oracle._LIB_PATH, oracle._lib
    oracle._LIB_PATH, oracle._lib = lib_path, None
    failed = []
    try:
        for i, pin in enumerate(PINS):
            try:
                pin()
            except (AssertionError, RuntimeError, ValueError, FloatingPointError):
                failed.append(i)
    finally:
        oracle._LIB_PATH, oracle._lib = saved
    return failed


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, orig, mut):
    assert SRC.count(orig) >= 1, f"mutation site not found: {name}"
    src = tmp_path / "mutant.c"
    src.write_text(SRC.replace(orig, mut, 1))  # the first occurrence: the hot-path copy
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-ffp-contract=off",
                           "-o", str(lib), str(src), "-lm"])
    with np.errstate(all="ignore"):
        failed = caught(str(lib))
    assert failed, f"no pin catches the mutant '{name}'"


def test_unmutated_oracle_passes_every_pin():
    assert caught(oracle._LIB_PATH) == []
