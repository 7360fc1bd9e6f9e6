"""Planted mistakes in copies of the oracle must fail its pins (CPU only).

Each mutant is the oracle source with one plausible slip (a dropped term, a
wrong sign, a wrong tie-break, the other reading of "largest distance to all
chosen surfels", a wrong operand, ...), compiled with the oracle's own flags
into a temporary library.  The pin battery must reject every one of them;
the unmodified source must pass it.
"""
import pytest

import oracle
from tests import pins

MUTANTS = {
    "dropped_dz_term": ("    float s = xx + yy;\n    return s + zz;",
                        "    float s = xx + yy;\n    (void)zz;\n    return s;"),
    "wrong_sign_dz": ("    float dz = a[2] - b[2];", "    float dz = a[2] + b[2];"),
    "highest_index_tie": ("            if (best < 0 || m[i] > m[best]) best = i;\n        }\n        c = best;\n        mc = m[c];",
                          "            if (best < 0 || m[i] >= m[best]) best = i;\n        }\n        c = best;\n        mc = m[c];"),
    "max_sum_reading": ("                if (d < m[i]) { m[i] = d; ++dec; }",
                        "                { m[i] = isinf(m[i]) ? d : m[i] + d; ++dec; }"),
    "distance_to_start_only": ("                float d = d2_f32(P + 3 * i, P + 3 * c);\n                ++live;",
                               "                float d = d2_f32(P + 3 * i, P + 3 * start);\n                ++live;"),
    "radius_is_d2": ("        if (radius) radius[t] = sqrtf(mc);\n    }\n    free(m);",
                     "        if (radius) radius[t] = mc;\n    }\n    free(m);"),
    "reselect_picked": ("        for (int64_t i = 0; i < n; ++i) {\n            if (sel[i]) continue;\n            if (best < 0 || m[i] > m[best]) best = i;\n        }\n        c = best;\n        mc",
                        "        for (int64_t i = 0; i < n; ++i) {\n            if (best < 0 || m[i] > m[best]) best = i;\n        }\n        c = best;\n        mc"),
    "ball_counts_ties": ("                if (d < mc) ++ball;\n                if (d < m[i]) { m[i] = d; ++dec; }",
                         "                if (d <= mc) ++ball;\n                if (d < m[i]) { m[i] = d; ++dec; }"),
    "ball_against_own_m": ("                if (d < mc) ++ball;\n                if (d < m[i]) { m[i] = d; ++dec; }",
                           "                if (d < m[i]) ++ball;\n                if (d < m[i]) { m[i] = d; ++dec; }"),
    "dec_counts_ties": ("                if (d < m[i]) { m[i] = d; ++dec; }",
                        "                if (d <= m[i]) { m[i] = d; ++dec; }"),
    "grid_ball_ties": ("                if (d < mc) ++ball;\n                if (d < m[i]) m[i] = d;",
                       "                if (d <= mc) ++ball;\n                if (d < m[i]) m[i] = d;"),
    "grid_span_no_margin": ("        double rr = sqrt(((double)mc + 1e-37) / (1.0 - 1e-5));\n"
                            "        int64_t span = isinf(rr) ? INT64_MAX : (int64_t)floor(rr / h) + 2;",
                            "        double rr = sqrt((double)mc);\n"
                            "        int64_t span = isinf(rr) ? INT64_MAX : (int64_t)floor(rr / h) + 1;"),
    "philox_multiplier": ("        uint64_t p0 = (uint64_t)0xD2511F53u * x0;", "        uint64_t p0 = (uint64_t)0xD2511F55u * x0;"),
    "philox_key_bump": ("            k1 += 0xBB67AE85u;", "            k1 += 0x9E3779B9u;"),
    "philox_no_first_key": ("        if (r > 0) {\n            k0 += 0x9E3779B9u;", "        {\n            k0 += 0x9E3779B9u;"),
    "sampler_growth_late": ("        int64_t q = K < 0 ? 1 : 1 + round / (K > 0 ? K : 1);",
                            "        int64_t q = K < 0 ? 1 : 1 + (round + 1) / (K > 0 ? K : 1);"),
    "sampler_highest_index_tie": ("(m[i] == m[best] && i < best)", "(m[i] == m[best] && i > best)"),
    "sampler_draw_modulo": ("                    int64_t idx = (int64_t)(((uint64_t)u[0] * (uint64_t)n) >> 32);",
                            "                    int64_t idx = (int64_t)((uint64_t)u[0] % (uint64_t)n);"),
    "sampler_draws_removed": ("                    if (!alive[idx]) continue;\n                    int dup = 0;",
                              "                    int dup = 0;"),
    "sampler_counter_swapped": ("                    const uint32_t ctr[4] = {(uint32_t)round, (uint32_t)j, a, 0u};",
                                "                    const uint32_t ctr[4] = {(uint32_t)j, (uint32_t)round, a, 0u};"),
    "sampler_vicinity_ties": ("                if (alive[i] && m[i] < thr) { alive[i] = 0; --remaining; }",
                              "                if (alive[i] && m[i] <= thr) { alive[i] = 0; --remaining; }"),
    "sampler_radius_after_removal": ("            if (radius) radius[t] = sqrtf(m[c]);\n            alive[c] = 0;\n            --remaining;",
                                     "            if (radius) radius[t] = sqrtf(m[c] * 0.5f);\n            alive[c] = 0;\n            --remaining;"),
    "prefix_nn_self": ("            if (b != a) {\n                float d = d2_f32(pa,", "            {\n                float d = d2_f32(pa,"),
    "capture_farthest_hit": ("                    if (t < tbest) {\n                        tbest = t;",
                             "                    if (t > tbest || tbest == INFINITY) {\n                        tbest = t;"),
    "capture_box_normal_sign": ("        nl[axis] = dl[axis] > 0.0f ? -1.0f : 1.0f;", "        nl[axis] = dl[axis] > 0.0f ? 1.0f : -1.0f;"),
    "capture_pixel_corner": ("                float fa = (float)(2 * i + 1) / (float)R - 1.0f;",
                             "                float fa = (float)(2 * i) / (float)R - 1.0f;"),
    "capture_image_axis": ("    u[1] = -d[0];\n    u[2] = 0.0f;", "    u[1] = d[0];\n    u[2] = 0.0f;"),
    "capture_cylinder_exit": ("                float t = t0 - sqrtf(h2 / a);\n                float z", "                float t = t0 + sqrtf(h2 / a);\n                float z"),
    "capture_sphere_exit": ("        float t = t0 - sqrtf(h2 / a);\n        if (!(t > 0.0f)) return 0;", "        float t = t0 + sqrtf(h2 / a);\n        if (!(t > 0.0f)) return 0;"),
    "grid_prunes_too_much": ("if (bd * (1.0 - 1e-5) - 1e-37 >= (double)mc) continue;",
                             "if (bd * 4.0 >= (double)mc) continue;"),
    "splitmix_constant": ("z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;",
                          "z = (z ^ (z >> 27)) * 0x94D049BB133111EAull;"),
    "fp64_dropped_dz": ("    double dz = a[2] - b[2];", "    double dz = 0.0 * (a[2] - b[2]);"),
    "oct_no_fold": ("    if (nrm[2] < 0.0f) {\n        float qx", "    if (0) {\n        float qx"),
    "oct_fold_swapped": ("        float qx = (1.0f - fabsf(py)) * sgn_nz(px);",
                         "        float qx = (1.0f - fabsf(px)) * sgn_nz(px);"),
    "oct_truncates": ("    return (int16_t)lrintf(c * 32767.0f);", "    return (int16_t)(c * 32767.0f);"),
    "oct_l2_norm": ("    float l1 = s + az;", "    float l1 = sqrtf(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);"),
    "emit_alpha_zero": ("                col[3] = 255;\n            } else {", "                col[3] = 0;\n            } else {"),
    "median_lower_middle": ("    else *out_rm = 0.5f * (nn[pm / 2 - 1] + nn[pm / 2]);",
                            "    else *out_rm = nn[pm / 2 - 1];"),
    "nn_includes_self": ("            if (b == a) continue;\n            float d = d2_f32",
                         "            float d = d2_f32"),
    "prefix_linear": ("    double p = ceil((double)pm * (r_m / r) * (r_m / r));",
                      "    double p = ceil((double)pm * (r_m / r));"),
    "along_order_max": ("            if (d < best) best = d;\n        }\n        r64[t] = sqrt(best);",
                        "            if (d > best || isinf(best)) best = d;\n        }\n        r64[t] = sqrt(best);"),
}


def test_unmodified_passes_battery():
    pins.pin_battery()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = oracle.source_text()
    assert src.count(old) == 1, "mutation target not unique: " + name
    lib = oracle.compile_variant(src.replace(old, new), str(tmp_path / ("m_%s.so" % name)))
    with pytest.raises((AssertionError, oracle.OracleError)):
        pins.pin_battery(lib)
