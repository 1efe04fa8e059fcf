"""The pins catch planted mistakes.

Each case copies oracle/oracle.c, plants one plausible mistake (a flipped or off-by-one
comparison, a 32-bit wrap in the band arithmetic, a dropped record, a transposed operand, a sum
instead of a product), builds the copy on the CPU, and runs the pins of test_oracle_pins.py
against it: at least one pin must fail.  The real oracle is untouched.
"""
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "lt_as_le": ("case ORC_LT: return r < s;", "case ORC_LT: return r <= s;"),
    "gt_operands_swapped": ("case ORC_GT: return r > s;", "case ORC_GT: return s > r;"),
    "ne_as_lt": ("case ORC_NE: return r != s;", "case ORC_NE: return r < s;"),
    "band_32bit_wrap": ("int64_t d = (int64_t)r - (int64_t)s;",
                        "int64_t d = (int32_t)((uint32_t)r - (uint32_t)s);"),
    "band_strict": ("return d <= w;", "return d < w;"),
    "sortmerge_drops_record": ("for (int64_t a = i; a < i2; ++a)",
                               "for (int64_t a = i + 1; a < i2; ++a)"),
    "sortmerge_swaps_columns": ("out[2 * k] = r[a].rid;\n                        out[2 * k + 1] = s[b].rid;",
                                "out[2 * k] = s[b].rid;\n                        out[2 * k + 1] = r[a].rid;"),
    "count_equi_sum_not_product": (
        "total += (uint64_t)(i2 - i) * (uint64_t)(j2 - j);\n        i = i2;",
        "total += (uint64_t)(i2 - i) + (uint64_t)(j2 - j);\n        i = i2;"),
    "count_lt_off_by_one": ("if (s[mid] <= Ra[i]) lo = mid + 1;",
                            "if (s[mid] < Ra[i]) lo = mid + 1;"),
    # both loops of the window join (count and write) get the same mistake
    "window_upper_bound_strict": ("(int64_t)s[j].key <= hi", "(int64_t)s[j].key < hi"),
    "nlj_ignores_second_column": ("if (ok && op_c != ORC_NONE) ok = orc_holds(op_c, Rc[i], Sc[j], w);\n            c +=",
                                  "c +="),
}

PIN_FUNCS = [
    pins.test_golden_equi_duplicates, pins.test_golden_theta_ops, pins.test_golden_band_extremes,
    pins.test_golden_band_and_lt_with_payload,
    lambda: pins.test_equi_pairs_equal_pandas_merge(11),
    lambda: pins.test_lt_count_equals_searchsorted(21),
    pins.test_lt_pairs_equal_per_row_slices,
    lambda: pins.test_trichotomy_and_complements(31),
    lambda: pins.test_mirror_symmetry("lt", "gt"),
    lambda: pins.test_mirror_symmetry("gt", "lt"),
    pins.test_band_zero_is_equality,
    pins.test_band_monotone_and_conjunction_is_intersection,
    pins.test_band_counts_by_direct_window_definition,
    lambda: pins.test_sortmerge_and_window_match_bruteforce(71),
    pins.test_equi_count_is_sum_of_multiplicity_products,
]


def _build_variant(tmp_path, name, old, new):
    src = open(SRC).read()
    sites = src.count(old)
    assert sites == (2 if name == "window_upper_bound_strict" else 1), (name, sites)
    mutated = src.replace(old, new)
    c = tmp_path / f"oracle_{name}.c"
    so = tmp_path / f"liboracle_{name}.so"
    c.write_text(mutated)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", str(c),
                           "-o", str(so)])
    return str(so)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    so = _build_variant(tmp_path, name, old, new)
    real = oracle._load()
    monkeypatch.setattr(oracle, "_LIB", so)
    monkeypatch.setattr(oracle, "_lib", None)
    oracle._load()
    caught = []
    try:
        for f in PIN_FUNCS:
            try:
                f()
            except AssertionError:
                caught.append(getattr(f, "__name__", "pin"))
            except Exception as e:  # a hypothesis failure wraps the assertion
                if "Falsifying" in str(e) or isinstance(e, AssertionError):
                    caught.append(getattr(f, "__name__", "pin"))
                else:
                    raise
    finally:
        monkeypatch.setattr(oracle, "_lib", real)
    assert caught, f"no pin caught the planted mistake {name}"
