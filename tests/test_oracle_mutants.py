"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake (a dropped term, a wrong sign or index, a
transposed operand, a strict instead of an inclusive compare, the wrong tie
order) in a private copy of the oracle's C source, builds it on the CPU, and
checks that at least one pin test fails against it."""
import importlib.util
import os
import shutil
import subprocess

import pytest

import test_oracle_hist as H
import test_oracle_join as J
import test_oracle_topk as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "dropped_last_term": ("for (int32_t k = 0; k < d; ++k) {", "for (int32_t k = 0; k < d - 1; ++k) {"),
    "wrong_sign": ("double t = (double)a[k] - (double)b[k];", "double t = (double)a[k] + (double)b[k];"),
    "channels_transposed": ("cnt[(rb * bins + gb) * bins + bb] += 1;", "cnt[(bb * bins + gb) * bins + rb] += 1;"),
    "wrong_pixel_count": ("(double)cnt[k] / (double)npx", "(double)cnt[k] / (double)(npx + 1)"),
    "strict_compare": ("if (dist <= eps) {", "if (dist < eps) {"),
    "strict_count": ("if (sqrt(d2) <= eps) ++c;", "if (sqrt(d2) < eps) ++c;"),
    "tie_larger_j_first": ("return da < db || (da == db && ja < jb);", "return da < db || (da == db && ja > jb);"),
    "reverse_order": ("for (int32_t k = 0; k < d; ++k) {", "for (int32_t k = d - 1; k >= 0; --k) {"),
    "fma_contract": ("d2 = d2 + t * t;", "d2 = fma(t, t, d2);"),
    "crop_area_off_by_one": ("(int64_t)(bx[3] - bx[1]) * (bx[4] - bx[2]);", "(int64_t)(bx[3] - bx[1] + 1) * (bx[4] - bx[2]);"),
    "crop_skips_first_row": ("for (int32_t y = bx[2]; y < bx[4]; ++y) {", "for (int32_t y = bx[2] + 1; y < bx[4]; ++y) {"),
    "self_join_keeps_diagonal": ("for (int64_t j = self ? gi + 1 : 0; j < nS; ++j) {",
                                 "for (int64_t j = self ? gi : 0; j < nS; ++j) {"),
}

PINS = [
    H.test_hand_example,
    lambda o: H.test_matches_histogramdd(o, 8, (7, 5)),
    H.test_mass_and_permutation,
    H.test_crop_hand_example,
    lambda o: H.test_crops_equal_histograms_of_sliced_patches(o, 8),
    J.test_hand_eps_join,
    J.test_pythagorean_closed_form,
    J.test_identity_and_bitwise_symmetry,
    J.test_integer_grid_is_exact,
    lambda o: J.test_canonical_summation_order_golden(o, "order"),
    lambda o: J.test_canonical_summation_order_golden(o, "fma"),
    J.test_self_join_is_upper_half_of_symmetric_full_join,
    J.test_eps_extremes_and_monotone,
    T.test_hand_ties,
    lambda o: T.test_equals_first_k_of_full_sort(o, 5, "grid"),
]


def load_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "dl_oracle.c")).read()
    assert src.count(old) >= 1, name
    d = tmp_path / name
    d.mkdir()
    (d / "dl_oracle.c").write_text(src.replace(old, new))
    shutil.copy(os.path.join(ROOT, "oracle", "__init__.py"), d / "__init__.py")
    spec = importlib.util.spec_from_file_location("oracle_mutant_" + name, d / "__init__.py")
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.build()
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    mod = load_mutant(tmp_path, name)
    caught = []
    for pin in PINS:
        try:
            pin(mod)
        except (AssertionError, ValueError, subprocess.CalledProcessError):
            caught.append(getattr(pin, "__name__", "lambda"))
    assert caught, "no pin caught the planted mistake %r" % name
