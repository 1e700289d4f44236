"""The oracle's pins catch plausible mistakes (no GPU).

Each case copies the oracle's C source to a temporary directory, plants one
plausible mistake by text substitution (a strict compare, a dropped pair, a
wrong tie rule, a lost missing-value check, a wrong mask bit, ...), compiles
it with the same flags, and checks that at least one pin fails on the broken
copy. Mistakes are planted only in these CPU copies.
"""
import functools
import os

import pytest

import oracle
from tests import oracle_pins as pins

MUTANTS = {
    "strict_ge": ("if (!(v >= prev)) pos = 0;", "if (!(v > prev)) pos = 0;"),
    "strict_le": ("if (!(v <= prev)) neg = 0;", "if (!(v < prev)) neg = 0;"),
    "swapped_ge": ("if (!(v >= prev)) pos = 0;", "if (!(prev >= v)) pos = 0;"),
    "tie_to_negative": ("const int n_bit = counted && neg && !pos;",
                        "const int n_bit = counted && neg;"),
    "no_prev_update": ("prev = v;\n", "\n"),
    "skip_first_pair": ("for (int32_t j = 1; counted", "for (int32_t j = 2; counted"),
    "last_pair_dropped": ("(pos || neg) && j < k; ++j)", "(pos || neg) && j < k - 1; ++j)"),
    "and_instead_of_or": ("const int m_bit = counted && (pos || neg);",
                          "const int m_bit = counted && (pos && neg);"),
    "neg_always_on": ("int neg = neg_on;", "int neg = 1;"),
    "first_missing_ignored": ("if (oracle_missing(prev, sentinel)) {",
                              "if (0 && oracle_missing(prev, sentinel)) {"),
    "modes_swapped": ("const int include = (flags & ORACLE_NAN_INCLUDE) != 0;",
                      "const int include = (flags & ORACLE_NAN_INCLUDE) == 0;"),
    "sentinel_ignored": ("return isnan(v) || v == sentinel;", "return isnan(v);"),
    "fill_ignored": ("if (include) v = fill;", "if (include) v = v;"),
    "mask_bit_index": ("mrow[r >> 6] |= (uint64_t)1 << (r & 63);",
                       "mrow[r >> 6] |= (uint64_t)1 << (r & 31);"),
    "column_bound_off_by_one": ("c[j] >= cols", "c[j] > cols"),
    "length_zero_valid": ("int valid = k >= 1;", "int valid = k >= 0;"),
    "first_col_from_second": ("float prev = row[c[0]];", "float prev = row[c[k > 1]];"),
    "negative_counts_all_neg": ("n_negative += n_bit;", "n_negative += neg;"),
}


@functools.lru_cache(maxsize=None)
def _build_mutant(name, tmpdir):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    path_c = os.path.join(tmpdir, f"m_{name}.c")
    with open(path_c, "w") as f:
        f.write(mutated)
    path_so = os.path.join(tmpdir, f"libm_{name}.so")
    oracle.build(path_c, path_so)
    return path_so


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path_factory):
    tmpdir = str(tmp_path_factory.getbasetemp())
    so = _build_mutant(name, tmpdir)
    ev = functools.partial(oracle.eval_population, lib_path=so)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(ev)
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"no pin detects mutant {name}"
