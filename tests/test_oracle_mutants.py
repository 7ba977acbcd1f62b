"""The oracle's pins against planted mistakes.

Each mutant is a plausible slip in pw_oracle.c (a sign, a face offset, a
transposed operand, a level range, a dropped or misdirected adjoint term, a
wrong fold), applied to a temporary copy of the source, compiled on the CPU
with the oracle's flags and routed in with ``oracle.use_library``.  The pins
of test_oracle_pins, test_oracle_adjoint and test_oracle_update must fail for
every mutant, and pass for the unmodified copy built the same way.
"""
import os
import subprocess

import pytest

import test_oracle_adjoint as adj_pins
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
