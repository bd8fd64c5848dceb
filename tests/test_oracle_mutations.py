"""The CPU reference's pins catch plausible mistakes.

Each case plants one mistake in the CPU reference (a dropped term, a flipped
sign, a transposed operand, an off-by-one, a missing clamp rule) — in a
patched Python helper or in a recompiled copy of the C compositing code, on
the CPU only — and checks that at least one of the pins in `test_oracle.py`
then fails.  Nothing here touches the HIP library.
"""
from __future__ import annotations

import math
import os
import subprocess

import numpy as np
import pytest
import torch

from tests import test_oracle as P


def _mutant_lib(oracle, tmp_path, replacements):
    """Compile a copy of the reference's C code with `replacements`
    (old, new, expected count) applied; returns the path of the library."""
    src = open(os.path.join(os.path.dirname(oracle.__file__), "raster.c")).read()
    for old, new, count in replacements:
        assert src.count(old) >= count, old
        src = src.replace(old, new, count)
    c = tmp_path / "raster_mutant.c"
    c.write_text(src)
    so = tmp_path / "raster_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                           str(c), "-o", str(so), "-lm"])
    return str(so)


@pytest.fixture
def with_c_mutation(oracle, tmp_path, monkeypatch):
    def apply(replacements):
        path = _mutant_lib(oracle, tmp_path, replacements)
        monkeypatch.setattr(oracle, "_LIB_PATH", path)
        monkeypatch.setattr(oracle, "_lib", None)
    return apply


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


# -- compositing (C) ---------------------------------------------------------
FWD_POWER = "const double power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy;"


def test_flipped_cross_term_in_forward_power_is_caught(oracle, with_c_mutation):
    # the first occurrence of the exponent is the forward's
    with_c_mutation([(FWD_POWER, FWD_POWER.replace("- b * dx", "+ b * dx"), 1)])
    _fails(P.test_single_gaussian_closed_form, oracle)


def test_dropped_background_term_in_backward_is_caught(oracle, with_c_mutation):
    with_c_mutation([("(suffix[c3] + Tfin * bg[c3])", "(suffix[c3])", 1)])
    P.test_gradients_match_finite_differences(oracle, (0.0, 0.0, 0.0), 0.0, -1.8)  # black: invisible
    _fails(P.test_gradients_match_finite_differences, oracle, (0.3, 0.6, 0.9), 0.0, -1.8)


def test_derivative_through_the_opacity_clamp_is_caught(oracle, with_c_mutation):
    with_c_mutation([("if (e->g > ALPHA_MAX) continue;", "", 1)])
    _fails(P.test_gradients_match_finite_differences, oracle, (0.3, 0.6, 0.9), 7.0, -0.6)


def test_back_to_front_order_is_caught(oracle, with_c_mutation):
    # sort keys descending: every tile list (and its depth order) reversed
    with_c_mutation([("return a->key < b->key ? -1 : 1;", "return a->key < b->key ? 1 : -1;", 1)])
    _fails(P.test_matches_bruteforce_depth_order, oracle)


def test_wrong_stop_level_is_caught(oracle, with_c_mutation):
    # a lower stop level lets the pixel composite one more Gaussian
    with_c_mutation([("#define T_MIN 1e-4", "#define T_MIN 1e-6", 1)])
    _fails(P.test_opaque_stack_stops_at_transmittance_floor, oracle)


def test_flipped_mean_gradient_in_backward_is_caught(oracle, with_c_mutation):
    line = "d_mean2d_t[j] += dl_dpower * (-(a * e->dx + b * e->dy));"
    with_c_mutation([(line, line.replace("(-(a", "((a"), 1)])
    _fails(P.test_gradients_match_finite_differences, oracle, (0.0, 0.0, 0.0), 0.0, -1.8)


def test_halved_cross_term_of_conic_gradient_is_caught(oracle, with_c_mutation):
    line = "d_conic_t[n + j] += dl_dpower * (-e->dx * e->dy);"
    with_c_mutation([(line, line.replace("(-e->dx", "(-0.5 * e->dx"), 1)])
    _fails(P.test_gradients_match_finite_differences, oracle, (0.0, 0.0, 0.0), 0.0, -1.8)


def test_importance_weight_without_transmittance_is_caught(oracle, with_c_mutation):
    with_c_mutation([("w_t[j] += alpha * T;", "w_t[j] += alpha;", 1)])
    _fails(P.test_importance_sum_identity, oracle)
    _fails(P.test_matches_bruteforce_depth_order, oracle)


def test_emitted_rectangle_off_by_one_is_caught(oracle, with_c_mutation):
    tx1 = "*tx1 = clampi(floordiv(xi + r, TILE) + 1, 0, TX);"
    with_c_mutation([(tx1, tx1.replace(" + 1,", ","), 1)])
    _fails(P.test_binning_covers_radius_box, oracle)


# -- projection (Python) -----------------------------------------------------
def test_missing_screen_space_dilation_is_caught(oracle, monkeypatch):
    monkeypatch.setattr(oracle._proj, "DILATION", 0.0)
    _fails(P.test_isotropic_on_axis_closed_form, oracle, 1.0, 0.1)


def test_transposed_rotation_is_caught(oracle, monkeypatch):
    orig = oracle._proj.quat_to_rotmat
    monkeypatch.setattr(oracle._proj, "quat_to_rotmat", lambda q: orig(q).transpose(1, 2))
    _fails(P.test_screen_covariance_matches_numeric_jacobian, oracle)


def test_sh_sign_flip_is_caught(oracle, monkeypatch):
    orig = oracle.sh_basis

    def flipped(d, *a, **k):
        Y = orig(d, *a, **k).clone()
        Y[:, 1] = -Y[:, 1]
        return Y
    monkeypatch.setattr(oracle, "sh_basis", flipped)
    _fails(P.test_sh_matches_scipy_complex_harmonics, oracle)


def test_tile_count_off_by_one_is_caught(oracle, monkeypatch):
    orig = oracle._proj.tile_rect

    def short(*a):
        tx0, tx1, ty0, ty1 = orig(*a)
        return tx0, torch.maximum(tx0, tx1 - 1), ty0, ty1
    monkeypatch.setattr(oracle._proj, "tile_rect", short)
    _fails(P.test_binning_matches_python_sorted, oracle, 48, 40)


# -- importance, optimizer ---------------------------------------------------
def test_top_mass_without_the_crossing_weight_is_caught(oracle, monkeypatch):
    orig = oracle.top_mass

    def exclusive(w, frac=0.99):
        sel = orig(w, frac)
        if sel.any():
            w = np.asarray(w)
            smallest = np.flatnonzero(sel)[np.argmin(w[sel])]
            sel = sel.copy()
            sel[smallest] = False
        return sel
    monkeypatch.setattr(oracle, "top_mass", exclusive)
    _fails(P.test_top_mass_hand_cases, oracle)


def test_score_without_eps_is_caught(oracle, monkeypatch):
    orig = oracle.importance_fold
    monkeypatch.setattr(oracle, "importance_fold",
                        lambda st, view, w, a, radius, frac=0.99, eps=1e-6: orig(st, view, w, a, radius, frac, 0.0))
    _fails(P.test_importance_fold_and_phi, oracle)


def test_level_gate_in_the_wrong_log_base_is_caught(oracle, monkeypatch):
    orig = oracle.lod_gate_level
    monkeypatch.setattr(oracle, "lod_gate_level",
                        lambda mean, lod, cam_pos, d0, l_max, f=2.0: orig(mean, lod, cam_pos, d0, l_max, math.e))
    _fails(P.test_lod_level_equation_values, oracle)


def test_adam_without_bias_correction_is_caught(oracle, monkeypatch):
    orig = oracle.adam_step
    monkeypatch.setattr(oracle, "adam_step",
                        lambda p, g, m, v, lr, step, **k: orig(p, g, m, v, lr, 10 ** 9, **k))
    _fails(P.test_adam_first_step_and_torch, oracle)


# ---------------------------------------------------------------------------
# LOD levels, L_max(t) and the spawn-gate veto (oracle/levels.py)
# ---------------------------------------------------------------------------
def _levels_mutant(old, new):
    import types

    from oracle import levels
    src = open(levels.__file__).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("levels_mutant")
    exec(compile(src.replace(old, new), "levels_mutant", "exec"), mod.__dict__)
    return mod


LEVEL_MUTATIONS = {
    "representative is the last point of its cube": (
        "order = np.lexsort((idx, code, key))", "order = np.lexsort((-idx, -code, key))"),
    "ties inside a finest cell by descending index": (
        "order = np.lexsort((idx, code, key))", "order = np.lexsort((-idx, code, key))"),
    "label is the finest level represented": (
        "for lvl in range(K - 1, -1, -1):", "for lvl in range(K):"),
    "cube shift off by one": ("sh = K - 1 - lvl", "sh = K - lvl"),
    "x and y swapped in the Z-order code": (
        "code |= ((cells[axis] >> b) & 1) << (3 * b + axis)",
        "code |= ((cells[(1, 0, 2)[axis]] >> b) & 1) << (3 * b + axis)"),
    "cell decision in float64": (
        "q = np.floor((m - o) * s)", "q = np.floor((m.astype(np.float64) - o) / float(delta0) * 2 ** (n_levels - 1))"),
    "unlock times spaced linearly": (
        "u = t0 * (t1 / t0) ** (k / (K - 1))", "u = t0 + (t1 - t0) * k / (K - 1)"),
    "veto count rounded down": (
        "return min(n, max(0, int(math.ceil(float(rho) * n))))", "return min(n, max(0, int(float(rho) * n)))"),
    "veto keeps the lowest survival": (
        "keep[order[:veto_count(n, rho)]] = False", "keep[order[n - veto_count(n, rho):]] = False"),
    "veto ties by descending index": (
        "order = np.lexsort((np.arange(n), p))", "order = np.lexsort((-np.arange(n), p))"),
    "split keeps the parent's level": (
        "lv = np.asarray(parent_level, dtype=np.int64) + (1 if split else 0)",
        "lv = np.asarray(parent_level, dtype=np.int64)"),
    "split level not clamped": (
        "return np.minimum(lv, n_levels - 1).astype(np.uint8)", "return lv.astype(np.uint8)"),
    "stub scorer uses the child's index": (
        "z = np.asarray(opacity_logit, dtype=np.float32)[np.asarray(parents, dtype=np.int64)]",
        "z = np.asarray(opacity_logit, dtype=np.float32)[np.arange(len(parents)) % len(opacity_logit)]"),
    "reference distance by mean instead of median": ("return float(np.median(d))", "return float(np.mean(d))"),
}


@pytest.mark.parametrize("name", sorted(LEVEL_MUTATIONS))
def test_level_mutation_is_caught(name):
    from tests import test_oracle_levels as PL
    mod = _levels_mutant(*LEVEL_MUTATIONS[name])
    failed = []
    for pin in PL.PINS:
        try:
            pin(mod)
        except (AssertionError, IndexError, ValueError):
            failed.append(pin.__name__)
    assert failed, f"no pin catches: {name}"


def test_footprint_count_that_stops_with_the_pixel_is_caught(oracle, with_c_mutation):
    old = "if (footprint) a_t[j] += 1;\n                if (stopped) continue;"
    new = "if (stopped) continue;\n                if (footprint) a_t[j] += 1;"
    with_c_mutation([(old, new, 1)])
    _fails(P.test_importance_footprint_count_ignores_occlusion, oracle)
