"""Planted mistakes in copies of the oracle must each fail at least one pin.

Each mutant is the oracle's C source with one plausible slip (a sign, a
dropped term, a transposed index, a misplaced offset) rebuilt in a temporary
directory; the real oracle source is never touched.  Passing here shows that
the pins in oracle_pins.py constrain every step of the computation.
"""
import os

import pytest

import oracle
import oracle_pins

MUTANTS = {
    "shear_sign": [("*ax = -(g1 * x + g2 * y);", "*ax = (g1 * x + g2 * y);"),
                   ("*ay = -(g2 * x - g1 * y);", "*ay = (g2 * x - g1 * y);")],
    "psf_not_flipped": [("int ii = i + r - a;", "int ii = i - r + a;"),
                        ("int jj = j + r - b;", "int jj = j - r + b;")],
    "psf_periodic_edges": [("if (ii < 0 || ii >= ny) continue;", "ii = (ii + ny) % ny;"),
                           ("if (jj < 0 || jj >= nx) continue;", "jj = (jj + nx) % nx;")],
    "subpixel_offset": [("((double)u + 0.5) / s - 0.5", "(double)u / s - 0.5"),
                        ("((double)v + 0.5) / s - 0.5", "(double)v / s - 0.5")],
    "bin_sum_not_mean": [("acc / ((double)s * s)", "acc / (double)s")],
    "drop_normalisation": [("out[t] = C - 0.5 * chi2;", "out[t] = -0.5 * chi2;")],
    "chi2_whole_image": [("if (mask[i]) {\n                    double r", "{\n                    double r")],
    "sie_normalisation": [("double b = theta_E * sqrt(q);", "double b = theta_E;")],
    "sie_axes_swapped": [("sqrt(q * q * x1 * x1 + x2 * x2)", "sqrt(x1 * x1 + q * q * x2 * x2)")],
    "sie_atanh_atan": [("a2 = b / e * atanh(e * x2 / psi);", "a2 = b / e * atan(e * x2 / psi);")],
    "sersic_rotation_sense": [("double x1 = dx * cos(phi) + dy * sin(phi);", "double x1 = dx * cos(phi) - dy * sin(phi);"),
                              ("double x2 = -dx * sin(phi) + dy * cos(phi);", "double x2 = dx * sin(phi) + dy * cos(phi);")],
    "sersic_q_inverted": [("sqrt(x1 * x1 * q + x2 * x2 / q)", "sqrt(x1 * x1 / q + x2 * x2 * q)")],
    "sersic_drop_minus_one": [("exp(-b_n * (pow(R / R_e, 1.0 / n) - 1.0))", "exp(-b_n * pow(R / R_e, 1.0 / n))")],
    "bn_wrong_quantile": [("if (oracle_gammainc_lower_reg(a, mid) < 0.5) lo = mid;",
                           "if (oracle_gammainc_lower_reg(a, mid) < 0.55) lo = mid;")],
    "gamma_series_term": [("term *= x / ap;", "term *= x / (ap + 1.0);")],
    "lens_equation_sign": [("double bx = x - ax, by = y - ay;", "double bx = x + ax, by = y + ay;")],
    "lens_light_off_mass_centre": [("p[10], p[11], p[3], p[4], x, y)", "p[10], p[11], p[17], p[18], x, y)")],
    "scene_xy_transposed": [("p[10], p[11], p[3], p[4], x, y)", "p[10], p[11], p[3], p[4], y, x)"),
                            ("p[17], p[18], bx, by)", "p[17], p[18], by, bx)")],
    "nnls_no_positivity": [("if (!(cand[c][0] >= 0.0 && cand[c][1] >= 0.0)) continue;", "if (0) continue;")],
    "nnls_weight_one_sigma": [("double w = 1.0 / (sigma[i] * sigma[i]);", "double w = 1.0 / sigma[i];")],
    "nnls_cramer_sign": [("cand[nc][0] = (g1 * F22 - g2 * F12) / det;", "cand[nc][0] = (g1 * F22 + g2 * F12) / det;")],
    "nnls_first_feasible": [("if (chi2 < best) {", "if (best == INFINITY) {")],
    "nnls_amps_swapped": [("out_amp[2 * t] = bl;", "out_amp[2 * t] = bs;"),
                          ("out_amp[2 * t + 1] = bs;", "out_amp[2 * t + 1] = bl;")],
    "light_lens_b_radius": [("double R = (model == 3 && c == 1) ? p[9] : p[8];", "double R = p[8];")],
    "light_source_b_index": [("double n = model == 3 ? nfix[c] : p[14];", "double n = model == 3 ? nfix[2] : p[14];")],
    "light_source_unlensed": [("    double bx = x - ax, by = y - ay;                                       /* Eq. 1 */\n    double R = (model == 3",
                               "    double bx = x, by = y;\n    double R = (model == 3")],
    "light_solve_back_substitution": [("for (int c = r + 1; c < m; ++c) acc -= A[r * m + c] * x[c];",
                                       "for (int c = r + 1; c < m; ++c) acc += A[r * m + c] * x[c];")],
    "light_chi2_drops_component": [("for (int c = 0; c < N; ++c) mval += cand[c] * col[(size_t)c * npix + i];",
                                    "for (int c = 1; c < N; ++c) mval += cand[c] * col[(size_t)c * npix + i];")],
    "light_mass_in_lens_only": [("int mass = model != 1, lens = model != 2, src = model != 1;",
                                 "int mass = 1, lens = model != 2, src = model != 1;")],
    "epl_substitution_power": [("m = 2.0 / (3.0 - gamma);", "m = 1.0 / (3.0 - gamma);")],
    "epl_minor_axis_integral": [("        J1 += f / d;", "        J1 += f;")],
    "epl_slope_exponent": [("p = 0.5 * (gamma - 1.0);", "p = 0.5 * gamma;")],
    "epl_integrals_swapped": [("const double a1 = q * x1 * J0, a2 = q * x2 * J1;",
                               "const double a1 = q * x1 * J1, a2 = q * x2 * J0;")],
    "epl_slope_ignored": [("oracle_epl_deflection(p[0], p[19],", "oracle_epl_deflection(p[0], 2.0,")],
    "philox_no_key_bump": [("            k0 += W0;\n            k1 += W1;\n", "")],
    "philox_words_swapped": [("n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;", "n1 = lo0, n2 = hi0 ^ c3 ^ k1, n3 = lo1;")],
    "stretch_drop_dimension_factor": [("rhs = (d - 1) * log(z[i])", "rhs = 0.0 * log(z[i])")],
    "stretch_partner_same_half": [("const int j = (1 - half) * h +", "const int j = half * h +")],
    "stretch_z_not_squared": [("const double z = w * w / a;", "const double z = w / a;")],
    "stretch_accept_inverted": [("if (lnpY[i] > -INFINITY && lhs < rhs) {", "if (lnpY[i] > -INFINITY && lhs > rhs) {")],
    "stretch_counter_ignores_iteration": [("const uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(uint64_t)t,",
                                           "const uint32_t ctr[4] = {(uint32_t)k, 0u,")],
    "lens_light_not_supersampled": [("acc += orc_scene(p, bl, bs, x, y);",
                                     "acc += orc_scene(p, bl, bs, x, y) - oracle_sersic(p[7], p[8], p[9], bl, p[10], p[11], p[3], p[4], x, y) + oracle_sersic(p[7], p[8], p[9], bl, p[10], p[11], p[3], p[4], ((double)j - 0.5 * (nx - 1)) * dpix, ((double)i - 0.5 * (ny - 1)) * dpix);")],
}


@pytest.fixture(scope="module")
def src():
    with open(oracle.SRC) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, src, tmp_path):
    text = src
    for old, new in MUTANTS[name]:
        assert text.count(old) >= 1, (name, old)
        text = text.replace(old, new)
    path = os.path.join(str(tmp_path), "mutant_%s.c" % name)
    with open(path, "w") as f:
        f.write(text)
    lib = oracle.compile_oracle(path, os.path.join(str(tmp_path), "libmutant_%s.so" % name))
    orc = oracle.Oracle(lib)
    caught = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(orc)
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
    assert caught, "planted mistake %r passed every pin" % name
