"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (a dropped
term, a wrong bound, floor for ceil, a wrong index ...), builds it, and runs
the pin suite against the broken copy in a child process; the suite must fail
(a crash of the broken copy counts as caught).  The real oracle is untouched.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ssp_oracle.c")

MUTANTS = {
    "floor_instead_of_ceil": ("return (uint64_t)((num + den - 1) / den);",
                              "return (uint64_t)(num / den);"),
    "flop_counts_row_not_rowlen": ("f += (uint64_t)(Brpt[k + 1] - Brpt[k]);", "f += 1;"),
    "flop_off_by_one_row": ("f += (uint64_t)(Brpt[k + 1] - Brpt[k]);",
                            "f += (uint64_t)(Brpt[k + 1] - Brpt[k]) + (k == 0);"),
    "distinct_counts_all": ("if (buf[q] != buf[q - 1]) ++distinct;", "++distinct;"),
    "splitmix_counter_from_zero": ("uint64_t z = seed + (i + 1u) * 0x9E3779B97F4A7C15ULL;",
                                   "uint64_t z = seed + i * 0x9E3779B97F4A7C15ULL;"),
    "splitmix_wrong_shift": ("z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;",
                             "z = (z ^ (z >> 29)) * 0x94D049BB133111EBULL;"),
    "sample_le_threshold": ("if ((orc_splitmix64(seed, (uint64_t)i) >> 11) < T)",
                            "if ((orc_splitmix64(seed, (uint64_t)i) >> 12) < T)"),
    "wide_division_drops_low_bits": ("rem = (rem << 1) | ((bits_lo >> b) & 1u);", "rem = (rem << 1);"),
    "wide_division_drops_carry": ("u128 rem = (low >> 64) + high;", "u128 rem = high;"),
    "reference_drops_M": ("u128 q = (u128)st->sample_nnz * (uint64_t)M;",
                          "u128 q = (u128)st->sample_nnz;"),
    "reference_uses_sample_flop": ("u128 d = (u128)st->n_sampled * st->total_flop;",
                                   "u128 d = (u128)st->n_sampled * st->sample_flop;"),
    "predict_ratio_inverted": ("ceil_div_u128((u128)rf[i] * st->sample_nnz, st->sample_flop)",
                               "ceil_div_u128((u128)rf[i] * st->sample_flop, st->sample_nnz)"),
    "no_empty_fallback": ("nnz_pred[i] = (int64_t)rf[i]; sum += rf[i];", "nnz_pred[i] = 0;"),
    "paper_sample_num_round": ("int64_t s = (int64_t)(0.003 * (double)M);",
                               "int64_t s = (int64_t)(0.003 * (double)M + 0.5);"),
    "paper_sample_cap": ("return s < 300 ? s : 300;", "return s;"),
    "paper_draw_mod_not_scale": ("rows[r] = (int32_t)(((u128)(uint64_t)M * u53) >> 53);",
                                 "rows[r] = (int32_t)(u53 % (uint64_t)M);"),
    "paper_draw_stream_seed_plus_one": (
        "uint64_t u53 = orc_splitmix64(seed, (uint64_t)r) >> 11;",
        "uint64_t u53 = orc_splitmix64(seed + 1u, (uint64_t)r) >> 11;"),
    "paper_draw_rounds": ("rows[r] = (int32_t)(((u128)(uint64_t)M * u53) >> 53);",
                          "rows[r] = (int32_t)(((u128)(uint64_t)M * u53 + ((u128)1 << 52)) >> 53);"),
    "sample_sums_skip_last": ("for (int64_t s = 0; s < n; ++s) {\n        fs +=",
                              "for (int64_t s = 0; s + 1 < n; ++s) {\n        fs +="),
    "exact_sum_dropped_row": ("Z += z;", "Z += (i ? z : 0);"),
    "spgemm_assigns_not_adds": ("acc[j] += p;", "acc[j] = p;"),
    "spgemm_adds_not_multiplies": ("const double p = a * Bval[q];", "const double p = a + Bval[q];"),
    "spgemm_drops_last_b_entry": (
        "for (int64_t q = Brpt[k]; q < Brpt[k + 1]; ++q) {\n                const int32_t j",
        "for (int64_t q = Brpt[k]; q + 1 < Brpt[k + 1]; ++q) {\n                const int32_t j"),
    "spgemm_wrong_a_value": ("const double a = Aval[e];", "const double a = Aval[Arpt[i]];"),
    "spgemm_signed_abs": ("aab[j] += p < 0 ? -p : p;", "aab[j] += p;"),
    "spgemm_terms_not_counted": ("terms[j] += 1;", "terms[j] = 1;"),
    "spgemm_unsorted_rows": ("qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);", ""),
    "spgemm_row_offset_shift": ("const int64_t o = Crpt[i] + s;", "const int64_t o = Crpt[i] + s + (s > 0 && i == 0);"),
    "kmv_counts_duplicates": ("        if (s > 0 && h[s] == h[s - 1]) continue;\n", ""),
    "kmv_column_seed": ("colk[j] = (orc_splitmix64(seed + 1u, (uint64_t)j) >> 11) < T;",
                        "colk[j] = (orc_splitmix64(seed, (uint64_t)j) >> 11) < T;"),
    "kmv_pair_transposed": ("(uint64_t)i * (uint64_t)N + (uint64_t)j) >> 11;",
                            "(uint64_t)j * (uint64_t)M + (uint64_t)i) >> 11;"),
    "kmv_kth_off_by_one": ("if (d == k) kv = h[s];", "if (d == k + 1) kv = h[s];"),
    "kmv_unsampled_columns": ("                if (!colk[j]) continue;\n", ""),
}
PIN_FILES = ("test_oracle_pins.py", "test_oracle_spgemm_pins.py", "test_oracle_kmv_pins.py")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new, 1))
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(lib), str(mut)])
    env = dict(os.environ, SSP_ORACLE_LIB_OVERRIDE=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *[os.path.join(ROOT, "tests", f) for f in PIN_FILES]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
