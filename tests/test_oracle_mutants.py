"""The oracle's pins against planted mistakes.

Each mutant is a plausible slip in pw_oracle.c (a sign, a face offset, a
transposed operand, a level range, a dropped or misdirected adjoint term, a
wrong fold, a dropped, doubled or signed term of the error magnitudes, an
abs mode left switched on), applied to a temporary copy of the source,
compiled on the CPU with the oracle's flags and routed in with
``oracle.use_library``.  The pins of test_oracle_pins, test_oracle_adjoint,
test_oracle_update and test_oracle_magnitudes must fail for every mutant, and
pass for the unmodified copy built the same way.
"""
import os
import subprocess

import pytest

import test_oracle_adjoint as adj_pins
import test_oracle_magnitudes as mag_pins
import test_oracle_pins as fwd_pins
import test_oracle_update as upd_pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pw_oracle.c")
FLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC"]

PINS = [
    (fwd_pins.test_hand_values, {}),
    (fwd_pins.test_zero_winds, {}),
    (fwd_pins.test_uniform_horizontal_flow_is_steady, {}),
    (fwd_pins.test_single_column_closed_form, {}),
    (fwd_pins.test_quadratic_scaling, {}),
    (fwd_pins.test_x_mirror, {}),
    (fwd_pins.test_y_mirror, {}),
    (fwd_pins.test_xy_transpose, {}),
    (fwd_pins.test_pw_energy_conservation, {}),
    (fwd_pins.test_z_halo_is_never_read, {}),
    (adj_pins.test_adjoint_matches_bruteforce_jacobian, {"shape": (4, 4, 5)}),
    (adj_pins.test_euler_identity, {}),
    (adj_pins.test_dot_product_identity, {}),
    (adj_pins.test_central_differences_on_random_cells, {}),
    (adj_pins.test_fold_is_transpose_of_pad, {}),
    (upd_pins.test_update_of_hand_values, {}),
    (upd_pins.test_euler_step_energy, {}),
    (mag_pins.test_forward_magnitude_hand_values, {}),
    (mag_pins.test_adjoint_magnitude_hand_values, {}),
    (mag_pins.test_magnitudes_ignore_every_sign, {}),
    (mag_pins.test_triangle_inequality_and_equality, {}),
    (mag_pins.test_magnitude_scaling, {}),
    (mag_pins.test_abs_call_leaves_signed_adjoint_alone, {}),
    (mag_pins.test_magnitudes_never_read_z_halo, {}),
]

# (name, text in pw_oracle.c, replacement, which occurrence (0-based))
MUTANTS = [
    ("su_tcx_sign", "s = tcx * (u[SIDX(i - 1, j, k)]", "s = -tcx * (u[SIDX(i - 1, j, k)]", 0),
    ("su_v_face_offset", "(v[SIDX(i, j - 1, k)] + v[SIDX(i + 1, j - 1, k)])",
     "(v[SIDX(i, j - 1, k)] + v[SIDX(i - 1, j - 1, k)])", 0),
    ("su_top_keeps_tzc2", "if (k < nz - 1) {", "if (k < nz) {", 0),
    ("su_level0_computed", "if (k == 0) {", "if (k == -1) {", 0),
    ("sv_transposed_operand", "- v[SIDX(i + 1, j, k)] * (u[c] + u[SIDX(i, j + 1, k)])",
     "- v[SIDX(i + 1, j, k)] * (u[c] + u[SIDX(i + 1, j, k)])", 0),
    ("sv_tcy_sign", "s = s + tcy * (v[SIDX(i, j - 1, k)]", "s = s - tcy * (v[SIDX(i, j - 1, k)]", 0),
    ("sw_tzc_swapped", "s = s + tzc1[k] * w[SIDX(i, j, k - 1)]", "s = s + tzc2[k] * w[SIDX(i, j, k - 1)]", 0),
    ("sw_top_level_computed", "if (k == nz - 1) {\n                    sw[c] = 0.0;",
     "if (k == nz) {\n                    sw[c] = 0.0;", 0),
    ("sw_u_diagonal", "(u[SIDX(i - 1, j, k)] + u[SIDX(i - 1, j, k + 1)])",
     "(u[SIDX(i - 1, j, k)] + u[SIDX(i - 1, j, k - 1)])", 0),
    ("adj_dropped_term", "term(gv, SIDX(i, j - 1, k), gv, c, gv, SIDX(i, j - 1, k), v, v, v, l, tcy);", "", 0),
    ("adj_sign", "term(gw, SIDX(i + 1, j, k), gu, c, gu, SIDX(i, j, k + 1), w, u, u, l, -tcx);",
     "term(gw, SIDX(i + 1, j, k), gu, c, gu, SIDX(i, j, k + 1), w, u, u, l, tcx);", 0),
    ("adj_operand", "gB[b] += lam * coef * A;", "gB[b] += lam * coef * B;", 0),
    ("adj_tzc_index", "u, w, w, l, tzc1[k]);", "u, w, w, l, tzc1[k - 1]);", 0),
    ("adj_level0", "for (k = 1; k < nz; k++) {", "for (k = 0; k < nz; k++) {", 0),
    ("adj_misdirected_target", "term(gu, SIDX(i, j + 1, k), gv, c, gv, SIDX(i + 1, j, k), u, v, v, l, -tcy);",
     "term(gu, SIDX(i, j + 1, k), gv, c, gv, SIDX(i, j + 1, k), u, v, v, l, -tcy);", 0),
    ("fold_assigns", "g[SIDX(ii, jj, k)] += g[s];", "g[SIDX(ii, jj, k)] = g[s];", 0),
    # rounding-error magnitudes T(c) (the scale of every reduced-precision bound)
    ("abs_su_tzc2_dropped", "if (k < nz - 1)\n                    t += fabs(tzc2[k]) * A(u, i, j, k + 1)",
     "if (k < 0)\n                    t += fabs(tzc2[k]) * A(u, i, j, k + 1)", 0),
    ("abs_sv_x_doubled", "t = ax * (A(v, i - 1, j, k)", "t = 2 * ax * (A(v, i - 1, j, k)", 0),
    ("abs_sw_tzc1_doubled", "t += fabs(tzc1[k]) * A(w, i, j, k - 1)", "t += 2 * fabs(tzc1[k]) * A(w, i, j, k - 1)", 0),
    ("abs_su_top_keeps_tzc2", "if (k < nz - 1)\n                    t += fabs(tzc2[k]) * A(u, i, j, k + 1)",
     "if (k < nz)\n                    t += fabs(tzc2[k]) * A(u, i, j, k + 1)", 0),
    ("abs_field_not_abs", "#define A(F, ii, jj, kk) fabs(F[SIDX(ii, jj, kk)])",
     "#define A(F, ii, jj, kk) (F[SIDX(ii, jj, kk)])", 0),
    ("abs_coef_not_abs", "double ax = fabs(tcx), ay = fabs(tcy);", "double ax = tcx, ay = fabs(tcy);", 0),
    ("abs_face_sum_inside", "(A(w, i, j, k) + A(w, i, j, k - 1))",
     "fabs(w[SIDX(i, j, k)] + w[SIDX(i, j, k - 1)])", 0),
    ("abs_adj_lambda_signed", "lam = fabs(lam);", "", 0),
    ("abs_adj_field_signed", "B = fabs(B);", "", 0),
    ("abs_adj_dropped_fabs_coef", "coef = fabs(coef);", "", 0),
    ("abs_mode_left_set", "pw_oracle_adj(u, v, w, lu, lv, lw, tzc1, tzc2, tcx, tcy, nx, ny, nz, h, gu, gv, gw);\n    g_abs_mode = 0;",
     "pw_oracle_adj(u, v, w, lu, lv, lw, tzc1, tzc2, tcx, tcy, nx, ny, nz, h, gu, gv, gw);", 0),
]


def _build(tmp_path, name, text):
    c = tmp_path / (name + ".c")
    so = tmp_path / ("lib" + name + ".so")
    c.write_text(text)
    subprocess.check_call(["gcc"] + FLAGS + [str(c), "-o", str(so), "-lm"])
    return str(so)


def _mutate(text, old, new, occurrence):
    pos = -1
    for _ in range(occurrence + 1):
        pos = text.find(old, pos + 1)
        assert pos >= 0, "mutation site not found: %r" % old
    return text[:pos] + new + text[pos + len(old):]


def _failing_pins(oracle, so):
    failed = []
    with oracle.use_library(so):
        for fn, kw in PINS:
            try:
                fn(oracle, **kw)
            except AssertionError:
                failed.append(fn.__name__)
    return failed


def test_unmodified_copy_passes_every_pin(oracle, tmp_path):
    so = _build(tmp_path, "orig", open(SRC).read())
    assert _failing_pins(oracle, so) == []


@pytest.mark.parametrize("mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(oracle, tmp_path, mutant):
    name, old, new, occ = mutant
    so = _build(tmp_path, name, _mutate(open(SRC).read(), old, new, occ))
    failed = _failing_pins(oracle, so)
    assert failed, "no pin detects mutant %s" % name
