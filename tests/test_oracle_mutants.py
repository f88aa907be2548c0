"""Each plausible mistake planted in the oracle (on the CPU) fails a pin.

The oracle source is copied, one mistake is substituted into the copy, the
copy is compiled with the oracle's own flags, and every pin is run against
it: at least one pin must fail.  Together with ``test_oracle_pins`` this shows
the pins constrain every step of the oracle (point distance, inverse order,
max/min, threshold, tie-break, label, distance, the paper's discard tests).
"""
import os

import pytest

import oracle
import pins

SRC = open(oracle.SRC).read()

MUTANTS = {
    "inverse_index_off_by_one": ("b + 3 * (NP - 1 - i)", "b + 3 * ((NP - i) % NP)"),
    "dropped_dz_term": ("fmaf(dz, dz, fmaf(dy, dy, dx * dx))", "fmaf(dy, dy, dx * dx)"),
    "wrong_sign": ("float dz = a[2] - b[2];", "float dz = a[2] + b[2];"),
    "transposed_operand": ("float dy = a[1] - b[1];", "float dy = a[1] - b[2];"),
    "no_fma_rounding": ("fmaf(dz, dz, fmaf(dy, dy, dx * dx))", "dz * dz + (dy * dy + dx * dx)"),
    "max_of_orders": ("float d = md < mi ? md : mi;", "float d = md > mi ? md : mi;"),
    "direct_order_only": ("float d = md < mi ? md : mi;", "float d = md;"),
    "min_over_points": ("md = x > md ? x : md;\n    mi = y > mi ? y : mi;\n  }\n  *d_dir",
                        "md = (i == 0 || x < md) ? x : md;\n    mi = y > mi ? y : mi;\n  }\n  *d_dir"),
    "exclusive_threshold": ("if (d <= t2) {", "if (d < t2) {"),
    "threshold_of_centroid": ("float tt = t2[bid[c]];", "float tt = t2[c % nb];"),
    "last_tie_wins": ("if (ok && (bestc < 0 || D < bestd))", "if (ok && (bestc < 0 || D <= bestd))"),
    "first_found_wins": ("if (ok && (bestc < 0 || D < bestd))", "if (ok && bestc < 0)"),
    "label_is_centroid": ("labels[f] = bid[bestc];", "labels[f] = (int32_t)bestc;"),
    "squared_distance_out": ("dists[f] = sqrtf(bestd);", "dists[f] = bestd;"),
    "threshold_not_squared": ("return t >= 0.0f ? t * t : -1.0f;", "return t >= 0.0f ? t : -1.0f;"),
    "cut_test2_inverse_wrong": ("float y0 = d2_f32(a, b + 3 * (NP - 1)), y1 = d2_f32(a + 3 * (NP - 1), b);",
                                "float y0 = d2_f32(a, b), y1 = d2_f32(a + 3 * (NP - 1), b + 3 * (NP - 1));"),
    "cut_test3_inverse_wrong": ("float y = d2_f32(a + 3 * i, b + 3 * (NP - 1 - i));\n    if (y > t2) alive_i = 0; else mi = y > mi ? y : mi;\n  }\n  if (!alive_d && !alive_i) return 0;\n  /* test4",
                                "float y = d2_f32(a + 3 * i, b + 3 * i);\n    if (y > t2) alive_i = 0; else mi = y > mi ? y : mi;\n  }\n  if (!alive_d && !alive_i) return 0;\n  /* test4"),
    "cut_skips_a_point": ("if (i == CENTER || i == 4 || i == 8 || i == 12 || i == 16) continue;\n    float x",
                          "if (i == CENTER || i == 4 || i == 8 || i == 12 || i == 16 || i == 7) continue;\n    float x"),
    "f64_rounded_difference": ("double dx = (double)a[0] - (double)b[0];", "double dx = (double)(a[0] - b[0]);"),
    "f64_exclusive_threshold": ("if (d <= t * t && (bestc < 0 || d < bestd))", "if (d < t * t && (bestc < 0 || d < bestd))"),
    "tn_not_squared": ("float uu = u * u;", "float uu = u;"),
    "tn_min_length": ("float mx = ls > lc ? ls : lc;", "float mx = ls < lc ? ls : lc;"),
    "tn_not_added": ("v = sqrtf(D) + oracle_tn_f32(ls, lc[c]);", "v = sqrtf(D);"),
    "tn_squared_metric": ("v = sqrtf(D) + oracle_tn_f32(ls, lc[c]);", "v = D + oracle_tn_f32(ls, lc[c]);"),
    "tn_threshold_ignored": ("if (!(v <= thr[bid[c]])) continue;", "(void)0;"),
    "tn_arc_skips_segment": ("for (int i = 0; i + 1 < NP; ++i) {\n    float dx = p[3 * (i + 1)] - p[3 * i];",
                             "for (int i = 1; i + 1 < NP; ++i) {\n    float dx = p[3 * (i + 1)] - p[3 * i];"),
    "tn_distance_is_dme": ("dists[f] = (flags & VAR_TN) ? bestv : sqrtf(bestv);", "dists[f] = sqrtf(bestv);"),
    "dir_tie_inverse": ("int direct = ed <= ei;\n  float mx = 0.0f;", "int direct = ed < ei;\n  float mx = 0.0f;"),
    "dir_picks_larger": ("int direct = ed <= ei;\n  float mx = direct ? ed : ei;", "int direct = ed > ei;\n  float mx = direct ? ed : ei;"),
    "dir_ignored_brute": ("if (flags & VAR_DIR)\n        ok = mode == ORACLE_CUT ? eval_dir_cut_f32(a, b, tt, &D) : eval_dir_brute_f32(a, b, tt, &D);",
                          "if (flags & VAR_DIR)\n        ok = mode == ORACLE_CUT ? eval_dir_cut_f32(a, b, tt, &D) : eval_brute_f32(a, b, tt, &D);"),
    "multi_first_found": ("if (!seen[k] || v < best[k]) best[k] = v;", "if (!seen[k]) best[k] = v;"),
    "multi_last_found": ("if (!seen[k] || v < best[k]) best[k] = v;", "best[k] = v;"),
    "multi_drops_last_bundle": ("for (int32_t b = 0; b < nb; ++b) {\n          if (!seen[b]) continue;",
                                "for (int32_t b = 0; b < nb - 1; ++b) {\n          if (!seen[b]) continue;"),
    "multi_squared_distance": ("dists[at] = (flags & VAR_TN) ? best[b] : sqrtf(best[b]);",
                               "dists[at] = best[b];"),
    "multi_counts_set_not_added": ("bundle_counts[bundles[i]] += 1;", "bundle_counts[bundles[i]] = 1;"),
    "multi_threshold_of_bundle_zero": ("    float tt = t2[bid[c]];\n    int ok;\n    if (flags & VAR_DIR)\n      ok = mode == ORACLE_CUT ? eval_dir_cut_f32(a, b, tt, &D) : eval_dir_brute_f32(a, b, tt, &D);\n    else\n      ok = mode == ORACLE_CUT ? eval_cut_f32(a, b, tt, &D) : eval_brute_f32(a, b, tt, &D);\n    if (!ok) continue;\n    float v = D;\n    if (flags & VAR_TN) {\n      v = sqrtf(D) + oracle_tn_f32(ls, lc[c]);\n      if (!(v <= thr[bid[c]])) continue;\n    }\n    int32_t k",
                                       "    float tt = t2[0];\n    int ok;\n    if (flags & VAR_DIR)\n      ok = mode == ORACLE_CUT ? eval_dir_cut_f32(a, b, tt, &D) : eval_dir_brute_f32(a, b, tt, &D);\n    else\n      ok = mode == ORACLE_CUT ? eval_cut_f32(a, b, tt, &D) : eval_brute_f32(a, b, tt, &D);\n    if (!ok) continue;\n    float v = D;\n    if (flags & VAR_TN) {\n      v = sqrtf(D) + oracle_tn_f32(ls, lc[c]);\n      if (!(v <= thr[bid[c]])) continue;\n    }\n    int32_t k"),
    "accepted_threshold_of_bundle_zero": ("thr2_f32(thr[bid[c]]), &D)) {\n        if (cnt < cap)",
                                          "thr2_f32(thr[0]), &D)) {\n        if (cnt < cap)"),
    "accepted_skips_last_centroid": ("for (int64_t c = 0; c < m; ++c) {\n      float D;\n      if (eval_brute_f32(a, cen + (size_t)c * 3 * NP, thr2_f32(thr[bid[c]])",
                                     "for (int64_t c = 0; c < m - 1; ++c) {\n      float D;\n      if (eval_brute_f32(a, cen + (size_t)c * 3 * NP, thr2_f32(thr[bid[c]])"),
    "resample_k_over_21": ("int64_t t = (L / 20) * k + ((L % 20) * k) / 20;",
                           "int64_t t = (L / 21) * k + ((L % 21) * k) / 21;"),
    "resample_target_rounded": ("int64_t t = (L / 20) * k + ((L % 20) * k) / 20;",
                                "int64_t t = (L / 20) * k + ((L % 20) * k + 10) / 20;"),
    "resample_strict_tie": ("while (j + 1 < P && !(t <= S[j + 1])) ++j;",
                            "while (j + 1 < P && !(t < S[j + 1])) ++j;"),
    "resample_no_saturation": ("if (!(g < 16384.0f)) return (int64_t)1 << 38;",
                               "if (!(g < 1e9f)) return (int64_t)1 << 38;"),
    "resample_float_accumulation": (
        "S[j + 1] = S[j] + seg_fixed(sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))));",
        "S[j + 1] = seg_fixed((float)S[j] / 16777216.0f + sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))));"),
    "resample_from_far_end": ("out[3 * k + c] = fmaf(w, b - a, a);", "out[3 * k + c] = fmaf(w, a - b, b);"),
    "resample_by_index": ("S[j + 1] = S[j] + seg_fixed(sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))));",
                          "S[j + 1] = S[j] + 16777216;"),
    "resample_last_point_off_by_one": ("out[3 * (NP - 1) + c] = p[3 * (P - 1) + c];",
                                       "out[3 * (NP - 1) + c] = p[3 * (P > 1 ? P - 2 : 0) + c];"),
    "resample_skips_first_segment": ("for (int64_t j = 0; j + 1 < P; ++j) {\n    float dx = p[3 * (j + 1)] - p[3 * j];",
                                     "S[1] = 0;\n  for (int64_t j = 1; j + 1 < P; ++j) {\n    float dx = p[3 * (j + 1)] - p[3 * j];"),
    "resample_accepts_long": ("if (off[i + 1] - off[i] > ((int64_t)1 << 24)) return -2;", ""),
    "resample_accepts_empty": ("off[i + 1] <= off[i]) return -2;", "off[i + 1] < off[i]) return -2;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    assert SRC.count(old) >= 1, f"mutation site for {name} not found"
    src = tmp_path / "mutant.c"
    src.write_text(SRC.replace(old, new, 1))
    lib = oracle.compile_oracle(str(src), str(tmp_path / "libmutant.so"))
    O = oracle.Oracle(lib)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(O)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"no pin catches mutant {name}"
