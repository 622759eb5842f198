"""Planted mistakes in copies of the oracle must each fail at least one pin.

Each mutation is a plausible slip (a dropped term, a wrong index, a transposed
operand, a wrong sign or bias, single-precision accumulation, a rounding rule)
applied to a temporary copy of oracle/normalize_oracle.c, compiled with the
same flags. The real oracle source is never modified.
"""
import os

import pytest

import oracle
from oracle_pins import ALL_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "normalize_oracle.c")

MUTATIONS = {
    "dropped_first_term": ("for (int64_t j = begin; j < end; ++j)", "for (int64_t j = begin + 1; j < end; ++j)"),
    "dropped_last_term": ("for (int64_t j = begin; j < end; ++j)", "for (int64_t j = begin; j < end - 1; ++j)"),
    "reversed_index": ("for (int64_t i = 0; i < n; ++i) out[i] = load(in, dtype, i) / s;",
                       "for (int64_t i = 0; i < n; ++i) out[i] = load(in, dtype, n - 1 - i) / s;"),
    "transposed_divide": ("for (int64_t i = 0; i < n; ++i) out[i] = load(in, dtype, i) / s;",
                          "for (int64_t i = 0; i < n; ++i) out[i] = s / load(in, dtype, i);"),
    "float_accumulator": ("  double s = 0.0;\n  for (int64_t j", "  float s = 0.0f;\n  for (int64_t j"),
    "bf16_lost_sign": ("    v = ldexp(128.0 + (double)f, e - 127 - 7);\n  }\n  return s ? -v : v;",
                       "    v = ldexp(128.0 + (double)f, e - 127 - 7);\n  }\n  return v;"),
    "bf16_wrong_bias": ("e - 127 - 7", "e - 126 - 7"),
    "bf16_subnormal_scale": ("ldexp((double)f, -126 - 7)", "ldexp((double)f, -127 - 7)"),
    "f16_subnormal_scale": ("ldexp((double)f, -14 - 10)", "ldexp((double)f, -15 - 10)"),
    "round_ties_away": ("else kr = fmod(kf, 2.0) == 0.0 ? kf : kf + 1.0;", "else kr = kf + 1.0;"),
    "round_truncates": ("if (rem > 0.5) kr = kf + 1.0;", "if (rem > 2.0) kr = kf + 1.0;"),
    "batched_sum_from_zero": ("double s = e > b ? sum_seq(in, dtype, b, e) : 0.0;",
                              "double s = e > b ? sum_seq(in, dtype, 0, e) : 0.0;"),
    "naive_skips_last": ("if (tid < n) out[tid] = load(in, dtype, tid) / val;",
                         "if (tid < n - 1) out[tid] = load(in, dtype, tid) / val;\n      else if (tid < n) out[tid] = 0.0;"),
    "sum_skips_first": ("return sum_seq(in, dtype, 0, n);", "return sum_seq(in, dtype, 1, n);"),
    "sum_guard_drops_single": ("if (n <= 0 || !valid_dtype(dtype) || !in) return 0.0;",
                               "if (n <= 1 || !valid_dtype(dtype) || !in) return 0.0;"),
    "perblock_wrong_range": ("double shared_val = sum_seq(in, dtype, 0, n);",
                             "double shared_val = sum_seq(in, dtype, b * block, n);"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert old in src, "mutation site vanished from the oracle source: %s" % name
    mutated = tmp_path / "mutated.c"
    mutated.write_text(src.replace(old, new, 1))
    lib = oracle.build(force=True, src=str(mutated), out=str(tmp_path / ("lib_%s.so" % name)))
    orc = oracle.Oracle(lib)
    failed = []
    for pin in ALL_PINS:
        try:
            pin(orc)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, "planted mistake %r passed every pin" % name


# ---- the row-softmax / log-sum-exp oracle (softmax_oracle.c) ----------------

from softmax_pins import SOFTMAX_PINS  # noqa: E402

SOFTMAX_SRC = os.path.join(os.path.dirname(oracle.__file__), "softmax_oracle.c")

SOFTMAX_MUTATIONS = {
    "no_max_shift": ("for (int64_t j = b; j < e; ++j) s += exp((double)x[j] - m);",
                     "for (int64_t j = b; j < e; ++j) s += exp((double)x[j]);"),
    "max_skips_second": ("for (int64_t j = b + 1; j < e; ++j)", "for (int64_t j = b + 2; j < e; ++j)"),
    "sum_skips_first": ("for (int64_t j = b; j < e; ++j) s += exp", "for (int64_t j = b + 1; j < e; ++j) s += exp"),
    "lse_without_max": ("if (lse) lse[r] = m + log(s);", "if (lse) lse[r] = log(s);"),
    "lse_log2": ("if (lse) lse[r] = m + log(s);", "if (lse) lse[r] = m + log2(s);"),
    "map_shifted_index": ("out[i] = exp((double)x[i] - m) / s;", "out[i] = exp((double)x[i < e - 1 ? i + 1 : i] - m) / s;"),
    "map_sign": ("out[i] = exp((double)x[i] - m) / s;", "out[i] = exp(m - (double)x[i]) / s;"),
    "float_accumulator": ("  double s = 0.0;\n  for (int64_t j = b; j < e; ++j) s += exp",
                          "  float s = 0.0f;\n  for (int64_t j = b; j < e; ++j) s += exp"),
    "row_end_short": ("const int64_t b = offsets[r], e = offsets[r + 1];",
                      "const int64_t b = offsets[r], e = offsets[r + 1] > b ? offsets[r + 1] - 1 : b;"),
    "empty_row_lse_zero": ("if (lse) lse[r] = -INFINITY;", "if (lse) lse[r] = 0.0;"),
    "min_not_max": ("if ((double)x[j] > m) m = (double)x[j];", "if ((double)x[j] < m) m = (double)x[j];"),
}


@pytest.mark.parametrize("name", sorted(SOFTMAX_MUTATIONS))
def test_softmax_mutation_is_caught(tmp_path, name):
    old, new = SOFTMAX_MUTATIONS[name]
    src = open(SOFTMAX_SRC).read()
    assert old in src, "mutation site vanished from the softmax oracle source: %s" % name
    mutated = tmp_path / "mutated_softmax.c"
    mutated.write_text(src.replace(old, new, 1))
    lib = oracle.build(force=True, softmax_src=str(mutated), out=str(tmp_path / ("lib_sm_%s.so" % name)))
    orc = oracle.Oracle(lib)
    failed = []
    for pin in SOFTMAX_PINS:
        try:
            pin(orc)
        except (AssertionError, FloatingPointError):
            failed.append(pin.__name__)
    assert failed, "planted mistake %r passed every softmax pin" % name


# ---- the forward NLL-loss oracle (nll_oracle.c) -----------------------------

from nll_pins import NLL_PINS  # noqa: E402

NLL_SRC = os.path.join(os.path.dirname(oracle.__file__), "nll_oracle.c")

NLL_MUTATIONS = {
    "sign": ("const double l = -w * (double)logp[i * c + t];", "const double l = w * (double)logp[i * c + t];"),
    "wrong_class": ("const double l = -w * (double)logp[i * c + t];",
                    "const double l = -w * (double)logp[i * c + (t + 1) % c];"),
    "weight_ignored": ("const double w = weight ? (double)weight[t] : 1.0;", "const double w = 1.0;"),
    "mean_over_n": ("if (reduction == ORC_NLL_MEAN) out[0] = loss / wsum;",
                    "if (reduction == ORC_NLL_MEAN) out[0] = loss / (double)n;"),
    "ignored_weight_counted": ("      if (reduction == ORC_NLL_NONE) out[i] = 0.0;\n      continue;",
                               "      if (reduction == ORC_NLL_NONE) out[i] = 0.0;\n      wsum += 1.0;\n      continue;"),
    "float_accumulator": ("double loss = 0.0, wsum = 0.0;", "float loss = 0.0f; double wsum = 0.0;"),
    "target_bound_off_by_one": ("if (t < 0 || t >= c) return ORC_NLL_EINVAL;",
                                "if (t < 0 || t > c) return ORC_NLL_EINVAL;"),
    "negative_target_accepted": ("if (t < 0 || t >= c) return ORC_NLL_EINVAL;",
                                 "if (t >= c) return ORC_NLL_EINVAL;\n    if (t < 0) continue;"),
    "sum_skips_first": ("for (int64_t i = 0; i < n; ++i) {", "for (int64_t i = 1; i < n; ++i) {"),
}


@pytest.mark.parametrize("name", sorted(NLL_MUTATIONS))
def test_nll_mutation_is_caught(tmp_path, name):
    old, new = NLL_MUTATIONS[name]
    src = open(NLL_SRC).read()
    assert old in src, "mutation site vanished from the NLL oracle source: %s" % name
    mutated = tmp_path / "mutated_nll.c"
    mutated.write_text(src.replace(old, new, 1))
    lib = oracle.build(force=True, nll_src=str(mutated), out=str(tmp_path / ("lib_nll_%s.so" % name)))
    orc = oracle.Oracle(lib)
    failed = []
    for pin in NLL_PINS:
        try:
            pin(orc)
        except (AssertionError, ValueError):
            failed.append(pin.__name__)
    assert failed, "planted mistake %r passed every NLL pin" % name


# ---- the Fig. 9-shaped tile kernel oracle (layerforward_oracle.c) ------------

from layerforward_pins import LAYERFORWARD_PINS  # noqa: E402

LF_SRC = os.path.join(os.path.dirname(oracle.__file__), "layerforward_oracle.c")

LF_MUTATIONS = {
    "no_input_factor": ("s += (double)hidden[j * LF_TILE + x] * (double)input[j];",
                        "s += (double)hidden[j * LF_TILE + x];"),
    "transposed_tile": ("s += (double)hidden[j * LF_TILE + x] * (double)input[j];",
                        "s += (double)hidden[(b * LF_TILE + x) * LF_TILE + k] * (double)input[j];"),
    "span_off_by_one": ("for (int k = y; k < y + span; ++k) {", "for (int k = y; k < y + span - 1; ++k) {"),
    "span_highest_bit": ("static int span_of(int y) { return y == 0 ? LF_TILE : (y & -y); }",
                         "static int span_of(int y) { return y == 0 ? LF_TILE : (y & -y) * (y > 8 ? 1 : 2) > LF_TILE - y ? LF_TILE - y : (y & -y) * (y > 8 ? 1 : 2); }"),
    "output_from_last_row": ("if (y == 0) output[b * LF_TILE + x] = s;", "if (y == 8) output[b * LF_TILE + x] = s;"),
    "input_wrong_row": ("s += (double)hidden[j * LF_TILE + x] * (double)input[j];",
                        "s += (double)hidden[j * LF_TILE + x] * (double)input[b * LF_TILE];"),
}


@pytest.mark.parametrize("name", sorted(LF_MUTATIONS))
def test_layerforward_mutation_is_caught(tmp_path, name):
    old, new = LF_MUTATIONS[name]
    src = open(LF_SRC).read()
    assert old in src, "mutation site vanished from the layerforward oracle source: %s" % name
    mutated = tmp_path / "mutated_lf.c"
    mutated.write_text(src.replace(old, new, 1))
    lib = oracle.build(force=True, lf_src=str(mutated), out=str(tmp_path / ("lib_lf_%s.so" % name)))
    orc = oracle.Oracle(lib)
    failed = []
    for pin in LAYERFORWARD_PINS:
        try:
            pin(orc)
        except (AssertionError, ValueError):
            failed.append(pin.__name__)
    assert failed, "planted mistake %r passed every layerforward pin" % name
