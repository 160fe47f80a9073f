"""Planted mistakes in the oracle, each caught by a pin.

Every case copies the oracle package (``oracle/``) into a temporary
directory, changes one line of one function (a dropped term, a wrong index,
sign, norm or rounding rule), builds the copy with the same compiler flags
and runs a named pin of ``test_oracle_pins.py`` / ``test_oracle_weighted.py``
against it: the pin must fail.  The real oracle passes the same pins in the
ordinary test run.  The table below is the evidence that no part of the
oracle is pinned only by itself.
"""
import importlib.util
import inspect
import os
import shutil
import sys

import pytest

import test_oracle_pins as pins
import test_oracle_weighted as wpins

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")

C, PY, W = "abft_oracle.c", "oracle.py", "weighted.py"

# (oracle function, file, original text, planted text, pin, pin arguments)
MUTATIONS = [
    ("orc_encode_rows", C, "const double *src = A + (g * br + r) * lda;",
     "const double *src = A + (g * br) * lda;", pins.test_encoding_block_sums_exact, dict(br=2, bc=3)),
    ("orc_encode_cols", C, "for (int64_t h = 0; h < G; ++h) s += row[h * bc + c];",
     "for (int64_t h = 1; h < G; ++h) s += row[h * bc + c];", pins.test_encoding_block_sums_exact, dict(br=2, bc=3)),
    ("orc_gemm", C, "double a = A[i * lda + l];", "double a = (l + 1 < K) ? A[i * lda + l] : 0.0;",
     pins.test_gemm_integer_exact, {}),
    ("orc_dot", C, "for (int64_t l = 0; l < K; ++l) s += a[l * inca] * b[l * incb];",
     "for (int64_t l = 1; l < K; ++l) s += a[l * inca] * b[l * incb];",
     pins.test_gemm_matches_library_within_gamma_bound, {}),
    ("orc_row_norms", C, "out[i] = sqrt(s);", "out[i] = s;", pins.test_norms_bound_the_tight_sum, {}),
    ("orc_group_abs_row_norms", C, "t[l] += fabs(A[(g * br + r) * lda + l]);", "t[l] += A[(g * br + r) * lda + l];",
     pins.test_det_threshold_hand_value_b2, {}),
    ("orc_col_norms", C, "for (int64_t l = 0; l < K; ++l) s += B[l * ldb + j] * B[l * ldb + j];",
     "for (int64_t l = 1; l < K; ++l) s += B[l * ldb + j] * B[l * ldb + j];",
     pins.test_det_threshold_hand_value_b1, {}),
    ("orc_group_abs_col_norms", C, "for (int64_t h = 0; h < G; ++h) t += fabs(B[l * ldb + h * bc + c]);",
     "for (int64_t h = 0; h < G; ++h) t += B[l * ldb + h * bc + c];", pins.test_det_threshold_hand_value_b2, {}),
    ("orc_tau_det: gamma_{G+1} -> gamma_G", C, "2.0 * orc_gamma((double)(m / br + 1), u64)",
     "2.0 * orc_gamma((double)(m / br), u64)", pins.test_det_threshold_hand_value_b1, {}),
    ("orc_tau_det: u_st dropped", C, "2.0 * orc_gamma((double)(m / br + 1), u64) + u_st);",
     "2.0 * orc_gamma((double)(m / br + 1), u64));", pins.test_det_threshold_hand_value_b1, {}),
    ("orc_tau_det: gamma_k -> gamma_{k-1}",
     C, "double cc = kappa * (2.0 * orc_gamma((double)k, u_acc)",
     "double cc = kappa * (2.0 * orc_gamma((double)(k - 1), u_acc)", pins.test_det_threshold_hand_value_b1, {}),
    ("orc_tau_det: row norm of B for the grouped norm", C, "tau_r[i * bc + c] = cr * na[i] * nb_abs[c];",
     "tau_r[i * bc + c] = cr * na[i] * nb[c];", pins.test_det_threshold_hand_value_b2, {}),
    ("orc_tau_stat: checksum row dropped from v", C, "for (int64_t g = 0; g <= Gr; ++g) {",
     "for (int64_t g = 0; g < Gr; ++g) {", pins.test_stat_threshold_hand_value_b2, {}),
    ("orc_tau_stat: ||b||_4 for ||b||_4^2", C,
     "double n4sq = sqrt(s4);\n            for (int64_t r = 0; r < br; ++r)",
     "double n4sq = sqrt(sqrt(s4));\n            for (int64_t r = 0; r < br; ++r)",
     pins.test_stat_model_block_checksums_simulated_fp32, dict(b=4, lo=0.45, hi=0.8)),
    ("orc_tau_stat: ||a||_4 for ||a||_4^2", C,
     "double n4sq = sqrt(s4);\n            for (int64_t c = 0; c < bc; ++c)",
     "double n4sq = sqrt(sqrt(s4));\n            for (int64_t c = 0; c < bc; ++c)",
     pins.test_stat_threshold_hand_value_b2, {}),
    ("orc_tau_stat: T/2 -> T", C, "double coef = u_acc * u_acc / 3.0 * (T / 2.0 + s_store);",
     "double coef = u_acc * u_acc / 3.0 * (T + s_store);", pins.test_stat_model_matches_simulated_fp32_accumulation,
     {}),
    ("orc_tau_stat: stored-total rounding dropped", C, "double cst = u_acc * u_acc / 3.0 * (1.0 + T_c / 3.0);",
     "double cst = 0.0;",
     pins.test_stat_threshold_hand_value_b2, {}),
    ("orc_tau_stat: accumulated stored totals' drift dropped", C,
     "double cst = u_acc * u_acc / 3.0 * (1.0 + T_c / 3.0);", "double cst = u_acc * u_acc / 3.0 * (1.0 + T_c / 6.0);",
     pins.test_stat_threshold_hand_value_b2, {}),
    ("orc_tau_stat: non-finite stored total kept in the rounding term", C,
     "double t = Cf && isfinite(Cf[(m + r) * ldc + j]) ? Cf[(m + r) * ldc + j] : 0.0;",
     "double t = Cf ? Cf[(m + r) * ldc + j] : 0.0;", pins.test_stat_threshold_hand_value_b2, {}),
    ("orc_tau_stat: b = 1 GEMV squares", C, "q += v[l] * (Bf[l * ldb + j] * Bf[l * ldb + j]);",
     "q += v[l] * fabs(Bf[l * ldb + j]);", pins.test_stat_q_matches_library_gemv, {}),
    ("orc_verify: a block dropped from the column sum", C,
     "for (int64_t g = 0; g < Gr; ++g) s += C[(g * br + r) * ldc + j];",
     "for (int64_t g = 1; g < Gr; ++g) s += C[(g * br + r) * ldc + j];",
     pins.test_eq_abft_gemm_consistency_exact, dict(br=3, bc=2)),
    ("orc_verify: NaN passes the column test", C,
     "if (!(fabs(d) <= t)) {\n                if (!isfinite(d)) rep->n_nonfinite++;\n                if (rep->n_flag_c",
     "if (fabs(d) > t) {\n                if (!isfinite(d)) rep->n_nonfinite++;\n                if (rep->n_flag_c",
     pins.test_nonfinite_value_fails_both_relations, {}),
    ("orc_verify: erased-relation test on the wrong residue", C, "if (i % br == r) return 1;",
     "if (i % br != r) return 1;", pins.test_known_erasure_skips_exactly_its_relations, {}),
    ("orc_classify: column congruence not checked", C, "if (i % br != r || j % bc != c) return ORC_MULTI;",
     "if (j % bc != c) return ORC_MULTI;", pins.test_classify_rules_on_hand_made_reports, {}),
    ("orc_classify: residual consistency not checked", C,
     "if (!(fabs(sc * dc - sr * dr) <= tol)) return ORC_MULTI;", "(void)tol;",
     pins.test_classify_rules_on_hand_made_reports, {}),
    ("orc_classify: sign of a stored total", C, "double sc = (i < m) ? 1.0 : -1.0,", "double sc = 1.0,",
     pins.test_every_element_every_bit_located_and_restored, dict(m=4, n=4, k=6, br=2, bc=2)),
    ("orc_rebuild_value: a checksum entry rebuilt as a data entry", C,
     "return (i < m) ? C[(m + r) * ldc + j] - s : s;", "return C[(m + r) * ldc + j] - s;",
     pins.test_every_element_every_bit_located_and_restored, dict(m=4, n=4, k=6, br=2, bc=2)),
    ("orc_recover: one row too many accepted", C, "if (!use_rows && h > br) return -4;",
     "if (!use_rows && h > br + 3) return -4;", pins.test_taller_than_checksum_block_is_unrecoverable, {}),
    ("orc_residual: ||x|| dropped", C, "return rmax / ((double)k * u * cnorm * xnorm);",
     "return rmax / ((double)k * u * cnorm * xnorm * 1e6);", pins.test_residual_check, {}),
    ("orc_to_bf16: ties away from zero", C, "if (lo > 0x8000u || (lo == 0x8000u && (hi & 1u))) hi += 1;",
     "if (lo >= 0x8000u) hi += 1;", pins.test_bf16_rne_matches_torch, {}),
    ("orc_e4m3_value: subnormal scale", C, "if (e == 0) v = ldexp((double)f, -9);",
     "if (e == 0) v = ldexp((double)f, -10);", pins.test_e4m3_decode_table_matches_torch, {}),
    ("orc_to_e4m3: ties away from zero", C,
     "if (rem > 0.5 || (rem == 0.5 && fmod(fl, 2.0) == 1.0)) qv = fl + 1.0;", "if (rem >= 0.5) qv = fl + 1.0;",
     pins.test_e4m3_rne_matches_torch_in_range, {}),
    ("orc_to_e4m3: infinities to NaN", C, "if (isinf(v)) { out[q] = (uint8_t)(sign | 0x7E); continue; }",
     "if (isinf(v)) { out[q] = 0x7F; continue; }", pins.test_e4m3_saturation_and_nonfinite, {}),
    ("orc_e4m3_scale_exp: one binade low", C, "while (ldexp(amax, e + 1) <= 448.0) ++e;",
     "while (ldexp(amax, e + 2) <= 448.0) ++e;", pins.test_e4m3_scale_is_largest_power_of_two, {}),
    ("oracle.tau_det_chained: |B| dropped", PY, "return tc + _f64(tau_c_prev)[:, :k] @ np.abs(Bf), tr",
     "return tc + _f64(tau_c_prev)[:, :k] @ Bf, tr", pins.test_chained_threshold_bounds_and_needs_the_inherited_term,
     {}),
    ("oracle.tau_det_chained: roundoffs not passed on", PY,
     "tc, tr = tau_det(Af, Bf, m, n, br, bc, u_acc=u_acc, u_st=u_st, kappa=kappa)",
     "tc, tr = tau_det(Af, Bf, m, n, br, bc, kappa=kappa)",
     pins.test_chained_threshold_binary32_bounds_single_precision_products, {}),
    ("oracle.outer_update: one update skipped", PY, "for l in range(k0, k1):", "for l in range(k0 + 1, k1):",
     pins.test_outer_product_does_not_transpose_or_skip, {}),
    ("oracle.block_cyclic_owner: local index", PY, "return I % P, (I // P) * nb + ii",
     "return I % P, I * nb + ii", pins.test_block_cyclic_owner_by_hand, {}),
    ("weighted.wencode: one block dropped", W, "for g in range(Gr):\n            acc += Wr[r, g] * A[g * br:(g + 1) * br]",
     "for g in range(Gr - 1):\n            acc += Wr[r, g] * A[g * br:(g + 1) * br]",
     wpins.test_section_2_1_checksums_by_hand, {}),
    ("weighted.wtau_det: summation terms dropped", W, "cc = kappa * (2 * gamma(k, u_acc) + u_st + 3 * gamma(Gr + 1))",
     "cc = kappa * (2 * gamma(k, u_acc) + u_st)", wpins.test_det_threshold_needs_its_summation_term,
     dict(wlo=0.5, whi=1.5)),
    ("weighted.wtau_det: product roundoff always binary64", W,
     "cc = kappa * (2 * gamma(k, u_acc) + u_st + 3 * gamma(Gr + 1))",
     "cc = kappa * (2 * gamma(k) + u_st + 3 * gamma(Gr + 1))",
     wpins.test_det_threshold_binary32_bounds_binary32_residuals,
     dict(m=64, n=32, k=4096, br=8, bc=4, fr=2, fc=2, positive=True)),
    ("weighted.fit_group: ratio test without the threshold", W,
     "fit = all(abs(d[r] - w[r] * delta) <= t[r] + eps * (abs(d[r]) + abs(w[r] * delta)) for r in range(f))",
     "fit = all(abs(d[r] - w[r] * delta) <= 0.0 for r in range(f))",
     wpins.test_every_element_every_exponent_bit_located_and_corrected, dict(fr=2, fc=1)),
    ("weighted._rebuild_line: lost checksum not recomputed", W, "    for r in Lc:\n        v[m + r * b + res] = S[r]",
     "    for r in Lc:\n        pass", wpins.test_any_f_lost_blocks_rebuilt_exactly, dict(direction=0)),
    ("weighted.erased_groups: skip rule off by one", W, "if (jj - j0) % bc < w:", "if (jj - j0) % bc <= w:",
     wpins.test_known_erasure_skips_exactly_its_groups, {}),
]


def _mutant_package(tmp_path, tag, fname, old, new):
    """Copy of the oracle package with one planted change, imported under its
    own name and built into its own directory."""
    name = "orcmut_" + tag
    d = tmp_path / name
    d.mkdir()
    for f in ("__init__.py", C, PY, W):
        text = open(os.path.join(ORACLE_DIR, f)).read()
        if f == fname:
            assert text.count(old) == 1, f"planted text must match once in {f}: {old!r}"
            text = text.replace(old, new)
        (d / f).write_text(text)
    spec = importlib.util.spec_from_file_location(name, str(d / "__init__.py"), submodule_search_locations=[str(d)])
    pkg = importlib.util.module_from_spec(spec)
    sys.modules[name] = pkg
    spec.loader.exec_module(pkg)
    orc = importlib.import_module(name + ".oracle")
    orc.build(force=True)
    wo = importlib.import_module(name + ".weighted")
    return name, orc, wo


@pytest.mark.parametrize("case", range(len(MUTATIONS)), ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(case, tmp_path, monkeypatch):
    func, fname, old, new, pin, kwargs = MUTATIONS[case]
    name, orc, wo = _mutant_package(tmp_path, str(case), fname, old, new)
    try:
        monkeypatch.setattr(wpins, "wo", wo)
        if "orc" in inspect.signature(pin).parameters:
            kwargs = dict(kwargs, orc=orc)
        with pytest.raises(AssertionError):
            pin(**kwargs)
    finally:
        for mod in [k for k in sys.modules if k == name or k.startswith(name + ".")]:
            del sys.modules[mod]
        shutil.rmtree(str(tmp_path / name), ignore_errors=True)
