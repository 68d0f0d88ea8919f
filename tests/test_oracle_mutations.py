"""Planted mistakes in the oracle must trip at least one pin.

Each case copies the oracle's C source, plants one plausible mistake (a
dropped term, a wrong sign, a wrong index, a transposed operand), builds the
copy in a temporary directory and runs the pins of ``test_oracle_pins``
against it.  This runs on the CPU only and never touches the GPU library.
"""

import os

import pytest

import oracle
import oracle.oracle as oracle_mod
import test_oracle_adjoint as adj
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle_mod.__file__), "wave_oracle.c")

MUTATIONS = {
    "jump_reversed": ("dq[m] = qr[m] - ql[m];", "dq[m] = ql[m] - qr[m];"),
    "left_eigvec_sign": ("e->L[0][0] = -1.0 / (2.0 * Z);", "e->L[0][0] = 1.0 / (2.0 * Z);"),
    "x_limiter_upwind_side": (
        "const int up = (s > 0.0) ? e - 1 : (s < 0.0 ? e + 1 : e);",
        "const int up = (s > 0.0) ? e + 1 : (s < 0.0 ? e - 1 : e);"),
    "y_limiter_upwind_side": (
        "const int up = (s > 0.0) ? f - 1 : (s < 0.0 ? f + 1 : f);",
        "const int up = (s > 0.0) ? f + 1 : (s < 0.0 ? f - 1 : f);"),
    "correction_weight_sign": (
        "const double coef = 0.5 * fabs(s) * (1.0 - dtdx * fabs(s));",
        "const double coef = 0.5 * fabs(s) * (1.0 + dtdx * fabs(s));"),
    "transverse_factor": (
        "Gx_top[GX(j, e) + m] -= 0.5 * dtdx * bp[m];",
        "Gx_top[GX(j, e) + m] -= 1.0 * dtdx * bp[m];"),
    "transverse_swapped_parts": (
        "Gx_bot[GX(j, e) + m] -= 0.5 * dtdx * bm[m];",
        "Gx_bot[GX(j, e) + m] -= 0.5 * dtdx * bp[m];"),
    "y_transverse_swapped_parts": (
        "Fy_right[FY(f - 1, i) + m] -= 0.5 * dtdy * ap[m];",
        "Fy_right[FY(f - 1, i) + m] -= 0.5 * dtdy * am[m];"),
    "dropped_transverse_term": (
        "const double FL = Fc[FC(j, i) + m] + Fy_right[FY(j, i - 1) + m] + Fy_left[FY(j, i) + m];",
        "const double FL = Fc[FC(j, i) + m] + Fy_right[FY(j, i - 1) + m];"),
    "flux_difference_sign": ("dtdx * (FR - FL) - dtdy * (GT - GB);",
                             "dtdx * (FL - FR) - dtdy * (GT - GB);"),
    "y_fluctuation_edges_swapped": (
        "const double fluct_y = apdq_y[AY(j, i) + m] + amdq_y[AY(j + 1, i) + m];",
        "const double fluct_y = apdq_y[AY(j + 1, i) + m] + amdq_y[AY(j, i) + m];"),
    "cfl_wrong_spacing": ("cfl = fmax(cfl, fabs(ey.s[p]) * dtdy);",
                          "cfl = fmax(cfl, fabs(ey.s[p]) * dtdx);"),
    "corner_ghosts_skipped": (
        "for (int i = -2; i < mx + 2; ++i)\n      for (int g = 1; g <= 2; ++g) {\n        if",
        "for (int i = 0; i < mx; ++i)\n      for (int g = 1; g <= 2; ++g) {\n        if"),
    # frozen-branch forward and adjoint
    "frozen_average_sign": ("case 1: out[m] = 0.5 * (w[m] + wup[m]); break;",
                            "case 1: out[m] = 0.5 * (w[m] - wup[m]); break;"),
    "adjoint_upwind_side": ("const int up = (s > 0.0) ? e - 1 : e + 1;",
                            "const int up = (s > 0.0) ? e + 1 : e - 1;"),
    "adjoint_split_parts_swapped": ("lm[m] = -0.5 * dtdx * l_Gx_bot[GX(j, e) + m];",
                                    "lm[m] = -0.5 * dtdx * l_Gx_top[GX(j, e) + m];"),
    "adjoint_ghost_fold_dropped": (
        "lpad[PI(0, j) * NM + m] += lpad[PI(-g, j) * NM + m];", "(void)0;"),
    "adjoint_correction_weight": (
        "const double coef = 0.5 * fabs(s) * (1.0 - dtdx * fabs(s));",
        "const double coef = 0.5 * fabs(s) * (1.0 - dtdy * fabs(s));"),
    "adjoint_jump_sign": ("lpad[PI(e - 1, j) * NM + m] -= ldq[m];",
                          "lpad[PI(e - 1, j) * NM + m] += ldq[m];"),
    # the variant that splits the limited correction transversely
    "tcorr_sign": ("ap[m] -= 2.0 * F[e][m];\n          am[m] += 2.0 * F[e][m];",
                   "ap[m] += 2.0 * F[e][m];\n          am[m] -= 2.0 * F[e][m];"),
    "tcorr_too_much": ("ap[m] -= 2.0 * F[e][m];\n          am[m] += 2.0 * F[e][m];",
                       "ap[m] -= 4.0 * F[e][m];\n          am[m] += 4.0 * F[e][m];"),
    "tcorr_y_dropped": ("bp_[m] -= 2.0 * G[f][m];\n          bm_[m] += 2.0 * G[f][m];", "(void)0;"),
    "tcorr_ignored": ("const int tcorr = (options & OR_OPT_TRANSVERSE_CORR) != 0;",
                      "const int tcorr = 0;"),
    # the batched wrapper that steps every patch of a level
    "step_patches_dx_dy_swapped": ("mx[k], my[k], dx[k],\n                           dy[k], dt[k]",
                                   "mx[k], my[k], dy[k],\n                           dx[k], dt[k]"),
    "step_patches_first_medium": ("dt[k], rho[k], K[k], limiter", "dt[k], rho[0], K[0], limiter"),
    "tcorr_ghost_rows_skipped": ("if (interior || tcorr)\n      for (int e = 0; e <= mx; ++e) {",
                                 "if (interior)\n      for (int e = 0; e <= mx; ++e) {"),
}

# cheapest first; the first failing pin ends a mutant's run
PIN_CALLS = [
    ("ghosts", lambda o: pins.test_extrapolation_ghosts_take_nearest_interior(o)),
    ("cfl", lambda o: pins.test_cfl_closed_form(o)),
    ("step_patches", lambda o: pins.test_step_patches_equals_each_patch_stepped_alone(o, "mc")),
    ("riemann_x", lambda o: pins.test_riemann_solver_eigen_structure(o, 0.7, 2.3, 0)),
    ("riemann_y", lambda o: pins.test_riemann_solver_eigen_structure(o, 0.7, 2.3, 1)),
    ("split_x", lambda o: pins.test_transverse_split_matches_matrix_split(o, 0)),
    ("split_y", lambda o: pins.test_transverse_split_matches_matrix_split(o, 1)),
    ("constant", lambda o: pins.test_constant_state_is_preserved_bitwise(o, False)),
    ("lax_wendroff", lambda o: pins.test_one_dimensional_reduction_lax_wendroff(o, False)),
    ("upwind", lambda o: pins.test_one_dimensional_reduction_upwind(o)),
    ("limited_1d", lambda o: pins.test_one_dimensional_reduction_limited_scheme(o, "mc", False)),
    ("translation", lambda o: pins.test_plane_wave_translates_exactly_at_courant_one(o, "mc", False)),
    ("symmetry", lambda o: pins.test_rotation_and_transpose_symmetry(o, False)),
    ("conservation", lambda o: pins.test_conservation_periodic(o, False)),
    ("frozen_forward", lambda o: adj.test_frozen_forward_equals_nonlinear_step(o)),
    ("dot_product", lambda o: adj.test_dot_product_identity(o, "extrap")),
    ("dense_jacobian", lambda o: adj.test_dense_jacobian_of_small_patch(o)),
    ("second_order", lambda o: pins.test_second_order_convergence_oblique_plane_wave(o, False)),
    # the transverse-correction variant
    ("tc_rejects_masks", lambda o: pins.test_transverse_correction_variant_rejects_masks(o)),
    ("tc_distinct", lambda o: pins.test_transverse_correction_variant_is_distinct_and_reduces_without_correction(o)),
    ("tc_constant", lambda o: pins.test_constant_state_is_preserved_bitwise(o, True)),
    ("tc_lax_wendroff", lambda o: pins.test_one_dimensional_reduction_lax_wendroff(o, True)),
    ("tc_limited_1d", lambda o: pins.test_one_dimensional_reduction_limited_scheme(o, "mc", True)),
    ("tc_conservation", lambda o: pins.test_conservation_periodic(o, True)),
    ("tc_symmetry", lambda o: pins.test_rotation_and_transpose_symmetry(o, True)),
    ("tc_stability", lambda o: pins.test_von_neumann_stable_up_to_courant_one(o, True)),
]


# anchors that occur in both the forward step and the adjoint: which occurrence
# (the heterogeneous-medium step repeats some lines of the homogeneous one, which
# comes first in the file: the mistakes are planted in the homogeneous step)
OCCURRENCE = {"correction_weight_sign": (0, 2), "adjoint_correction_weight": (1, 2),
              "transverse_factor": (0, 2), "transverse_swapped_parts": (0, 2),
              "y_transverse_swapped_parts": (0, 2), "dropped_transverse_term": (0, 2),
              "flux_difference_sign": (0, 2), "y_fluctuation_edges_swapped": (0, 2)}


def _plant(src, name):
    orig, mutated = MUTATIONS[name]
    which, count = OCCURRENCE.get(name, (0, 1))
    assert src.count(orig) == count, f"mutation anchor for {name} occurs {src.count(orig)} times"
    pos = -1
    for _ in range(which + 1):
        pos = src.index(orig, pos + 1)
    return src[:pos] + mutated + src[pos + len(orig):]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    src = open(SRC).read()
    mpath = tmp_path / "mutant.c"
    mpath.write_text(_plant(src, name))
    so = oracle_mod.build(str(mpath), str(tmp_path / "libmutant.so"))
    saved = oracle_mod._lib
    oracle_mod._lib = oracle_mod.load_lib(so)
    caught = None
    try:
        for pin_name, call in PIN_CALLS:
            try:
                call(oracle)
            except (AssertionError, ValueError, RuntimeError, FloatingPointError):
                caught = pin_name
                break
    finally:
        oracle_mod._lib = saved
    assert caught is not None, f"planted mistake {name!r} passed every pin"


# --------------------------------------------------------------------------
# The two-level composite step (oracle/amr.py): mistakes planted in a copy of
# the module, checked against the pins of test_oracle_amr
# --------------------------------------------------------------------------

import importlib.util  # noqa: E402
import sys  # noqa: E402

import oracle.amr as amr_src  # noqa: E402
import test_oracle_amr as amr_pins  # noqa: E402

AMR_MUTATIONS = {
    # the factor printed in front of the coarse second-order term
    "coarse_correction_quarter": (
        'Pc = -Tc["apx"][fp.cj0 + J, e] + Tc["Fx"][fp.cj0 + J, e]',
        'Pc = -Tc["apx"][fp.cj0 + J, e] + 0.25 * Tc["Fx"][fp.cj0 + J, e]'),
    "left_fix_sign": ("qc[:, fp.cj0 + J + 2, fp.ci0 - 1 + 2] -= dt / dxc",
                      "qc[:, fp.cj0 + J + 2, fp.ci0 - 1 + 2] += dt / dxc"),
    "right_fine_fluctuation_side": ('- Tf["apx"][b, mxf] + Tf["Fx"][b, mxf]',
                                    '+ Tf["amx"][b, mxf] + Tf["Fx"][b, mxf]'),
    "c1_dropped_top": ('acc["top"][a] += _fsum(1, rho, K, out, g) - Tf["apy"][myf, a]',
                       'acc["top"][a] += - Tf["apy"][myf, a]'),
    "time_fraction": ("a = k / r\n        Qt = (1.0 - a) * qc + a * qc1",
                      "a = (k + 1) / r\n        Qt = (1.0 - a) * qc + a * qc1"),
    # the recursion of several levels
    "recursion_time_ends_swapped": ("Qt = (1.0 - a) * old[p.parent] + a * new[p.parent]",
                                    "Qt = (1.0 - a) * new[p.parent] + a * old[p.parent]"),
    "recursion_fix_skipped": ("apply_fix(new[p.parent], p, accs[c], Tc[p.parent], dt_l, dx, dy, r, cov)",
                              "pass"),
    # same-level ghosts and the fix next to touching fine patches
    "sibling_ghosts_from_coarse": ("fill_fine_ghosts(new_q[c], fp, Qt, r, sibs)",
                                   "fill_fine_ghosts(new_q[c], fp, Qt, r)"),
    "recursion_sibling_ghosts_from_coarse": ("fill_fine_ghosts(qf, p, Qt, r, sibs)",
                                             "fill_fine_ghosts(qf, p, Qt, r)"),
    "sibling_index_offset": ("si, sj = gi - r * sp.ci0, gj - r * sp.cj0",
                             "si, sj = gi - r * sp.ci0, gj - r * sp.cj0 - 1"),
    "sibling_one_step_ahead": (
        "sibs = [(fines[d], new_q[d]) for d in range(len(fines)) if d != c]",
        "sibs = [(fines[d], O.step(new_q[d], dxf, dyf, dtf, rho, K, limiter)[0])"
        " for d in range(len(fines)) if d != c]"),
    "fix_on_covered_cells": ("apply_fix(qc2, fp, acc, Tc, dt, dxc, dyc, r, cov)",
                             "apply_fix(qc2, fp, acc, Tc, dt, dxc, dyc, r)"),
    "recursion_fix_on_covered_cells": (
        "apply_fix(new[p.parent], p, accs[c], Tc[p.parent], dt_l, dx, dy, r, cov)",
        "apply_fix(new[p.parent], p, accs[c], Tc[p.parent], dt_l, dx, dy, r)"),
    "average_weight": ("sum(axis=1) / (r * r)", "sum(axis=1) / (r * r + 1)"),
    "slope_unlimited": ("return s * np.minimum(np.minimum(2.0 * np.abs(a), 2.0 * np.abs(b)), 0.5 * np.abs(a + b))",
                        "return 0.5 * (a + b)"),
    "ghost_cell_offset": ("X = fp.ci0 + (i + 0.5) / r", "X = fp.ci0 + (i + 1.0) / r"),
}

AMR_PIN_CALLS = [
    ("interp_r2", lambda m: amr_pins.test_interpolation_conservative_linear_exact_and_bounded(2, m)),
    ("interp_r3", lambda m: amr_pins.test_interpolation_conservative_linear_exact_and_bounded(3, m)),
    ("mc_step", lambda m: amr_pins.test_mc_slope_bounds_a_step(m)),
    ("constant", lambda m: amr_pins.test_constant_state_preserved(m)),
    ("ratio_one", lambda m: amr_pins.test_ratio_one_equals_single_level_step(m)),
    ("conserves_r2", lambda m: amr_pins.test_composite_conserves(2, m)),
    ("symmetry", lambda m: amr_pins.test_symmetric_layout_gives_symmetric_result(m)),
    ("one_level_recursion", lambda m: amr_pins.test_one_level_recursion_equals_two_level_step(m)),
    ("three_ratio_one", lambda m: amr_pins.test_three_levels_ratio_one_equal_single_level(m)),
    ("three_conserve", lambda m: amr_pins.test_three_levels_conserve(m)),
    ("split_two_x", lambda m: amr_pins.test_split_patch_equals_whole_patch(2, "x", "two", m)),
    ("split_multi_quadrants",
     lambda m: amr_pins.test_split_patch_equals_whole_patch(3, "quadrants", "multi", m)),
    ("touching_conserve", lambda m: amr_pins.test_touching_patches_conserve(2, m)),
    ("covered_means", lambda m: amr_pins.test_covered_cells_hold_the_means_of_their_fine_cells(m)),
]


@pytest.mark.parametrize("name", sorted(AMR_MUTATIONS))
def test_planted_composite_mistake_is_caught(name, tmp_path):
    orig, mutated = AMR_MUTATIONS[name]
    src = open(amr_src.__file__).read()
    assert src.count(orig) == 1, f"mutation anchor for {name} occurs {src.count(orig)} times"
    src = src.replace(orig, mutated).replace("from . import oracle as O", "import oracle.oracle as O")
    path = tmp_path / "amr_mutant.py"
    path.write_text(src)
    spec = importlib.util.spec_from_file_location("amr_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    sys.modules["amr_mutant"] = mod  # dataclasses look their module up
    try:
        spec.loader.exec_module(mod)
        caught = None
        for pin_name, call in AMR_PIN_CALLS:
            try:
                call(mod)
            except (AssertionError, ValueError, RuntimeError, FloatingPointError, IndexError):
                caught = pin_name
                break
    finally:
        del sys.modules["amr_mutant"]
    assert caught is not None, f"planted mistake {name!r} passed every pin"


# --------------------------------------------------------------------------
# The heterogeneous-medium step: mistakes planted in the C source, checked
# against the pins of test_oracle_var
# --------------------------------------------------------------------------

import test_oracle_var as var_pins  # noqa: E402

VAR_MUTATIONS = {
    "strength_impedance": ("const double a1 = (-dp + Zr * dn) / (Zl + Zr);",
                           "const double a1 = (-dp + Zl * dn) / (Zl + Zr);"),
    "left_wave_speed": ("s[0] = -cl;", "s[0] = -cr;"),
    "transverse_own_impedance": ("const double bd = (-a[0] + Zm * a[n]) / (Zb + Zm);",
                                 "const double bd = (-a[0] + Zm * a[n]) / (Zm + Zm);"),
    "transverse_speed": ("minus[0] = -cb * bd * (-Zb);\n  minus[n] = -cb * bd;",
                         "minus[0] = -ct * bd * (-Zb);\n  minus[n] = -ct * bd;"),
    "transverse_cells_swapped_in_x": (
        "split_var(1, &apdq_x[AX(j, e)], Zc[VIX(e, j - 1)], cc[VIX(e, j - 1)], Zc[VIX(e, j)],\n"
        "                  Zc[VIX(e, j + 1)], cc[VIX(e, j + 1)], bm, bp);",
        "split_var(1, &apdq_x[AX(j, e)], Zc[VIX(e, j + 1)], cc[VIX(e, j + 1)], Zc[VIX(e, j)],\n"
        "                  Zc[VIX(e, j - 1)], cc[VIX(e, j - 1)], bm, bp);"),
    "cfl_smaller_speed": ("cfl = fmax(cfl, fmax(cc[VIX(e - 1, j)], cc[VIX(e, j)]) * dtdx);",
                          "cfl = fmax(cfl, fmin(cc[VIX(e - 1, j)], cc[VIX(e, j)]) * dtdx);"),
}

VAR_PIN_CALLS = [
    ("uniform", lambda L: var_pins.test_uniform_medium_is_the_constant_coefficient_step("mc", L)),
    ("interface_x", lambda L: var_pins.test_interface_riemann_problem_first_step_is_exact(0, L)),
    ("interface_y", lambda L: var_pins.test_interface_riemann_problem_first_step_is_exact(1, L)),
    ("cfl", lambda L: var_pins.test_courant_number_is_the_largest_edge_speed(L)),
    ("transpose", lambda L: var_pins.test_transpose_symmetry(L)),
    ("energy", lambda L: var_pins.test_mc_step_dissipates_energy_on_a_rough_medium(L)),
]


@pytest.mark.parametrize("name", sorted(VAR_MUTATIONS))
def test_planted_medium_mistake_is_caught(name, tmp_path):
    orig, mutated = VAR_MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation anchor for {name} occurs {src.count(orig)} times"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(orig, mutated))
    so = oracle_mod.build(str(mpath), str(tmp_path / "libmutant.so"))
    L = oracle_mod.load_lib(so)
    caught = None
    for pin_name, call in VAR_PIN_CALLS:
        try:
            call(L)
        except (AssertionError, ValueError, RuntimeError, FloatingPointError):
            caught = pin_name
            break
    assert caught is not None, f"planted mistake {name!r} passed every pin"


# --------------------------------------------------------------------------
# The ghost exchange of a tiled level (oracle/tiled.py): mistakes planted in a
# copy of the module, checked against the pins of test_oracle_tiled
# --------------------------------------------------------------------------

import oracle.tiled as tiled_src  # noqa: E402
import test_oracle_tiled as tiled_pins  # noqa: E402

TILED_MUTATIONS = {
    "wrap_off_by_one": ("gx = gx % DX if periodic[0]", "gx = (gx + 1) % DX if periodic[0]"),
    "clamp_short": ("min(max(gy, 0), DY - 1)", "min(max(gy, 0), DY - 2)"),
    "directions_swapped": ("gy = gy % DY if periodic[1]", "gy = gy % DY if periodic[0]"),
    "source_origin_x": ("qs[o][:, sy - oy + 2, sx - ox + 2]", "qs[o][:, sy - oy + 2, sx + 2]"),
    "own_patch_only": ("o = own[sy, sx]", "o = k"),
}

TILED_PIN_CALLS = [
    (f"numpy_pad_{p}", lambda m, p=p: tiled_pins.test_single_patch_exchange_is_numpy_padding(p, m))
    for p in [(True, True), (False, False), (True, False), (False, True)]
] + [
    (f"tiled_{t}_{p}", lambda m, t=t, p=p: tiled_pins.test_tiled_steps_equal_the_single_patch_step(t, p, m))
    for t in sorted(tiled_pins.TILINGS) for p in [(True, True), (False, False), (True, False)]
]


@pytest.mark.parametrize("name", sorted(TILED_MUTATIONS))
def test_planted_exchange_mistake_is_caught(name, tmp_path):
    orig, mutated = TILED_MUTATIONS[name]
    src = open(tiled_src.__file__).read()
    assert src.count(orig) == 1, f"mutation anchor for {name} occurs {src.count(orig)} times"
    path = tmp_path / "tiled_mutant.py"
    path.write_text(src.replace(orig, mutated))
    spec = importlib.util.spec_from_file_location("tiled_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    caught = None
    for pin_name, call in TILED_PIN_CALLS:
        try:
            call(mod)
        except (AssertionError, ValueError, IndexError):
            caught = pin_name
            break
    assert caught is not None, f"planted mistake {name!r} passed every pin"
