"""Plant plausible mistakes in copies of the C oracle and check the pins catch each.

Every mutant is a one-place edit of oracle/ig_oracle.c compiled into a temporary
library; the pins of test_oracle_pins (worked example, exhaustive enumeration,
patterns given as code rows, t(b) by scanning) must fail on it.  This runs on the CPU only.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "ig_oracle.c")

MUTANTS = {
    # Eq. 6 operands transposed: "r inside b" instead of "b inside r"
    "subset_transposed": ("if ((b[k] & r[k]) != b[k]) return 0;", "if ((b[k] & r[k]) != r[k]) return 0;"),
    # Eq. 2 with |b| instead of |b|^2
    "weight_not_squared": ("m->S[c][p] = (int64_t)f * (int64_t)len * (int64_t)len;",
                           "m->S[c][p] = (int64_t)f * (int64_t)len;"),
    # Eq. 1 without the records themselves
    "no_signatures": ("if (is_empty(X + i * K, K)) continue;\n        memcpy",
                      "if (1) continue;\n        memcpy"),
    # support counted in the other class
    "support_other_class": ("uint32_t f = support(b, Xc, nc, K);", "uint32_t f = support(b, Xo, no, K);"),
    # Eq. 5 bit order reversed inside a word
    "msb_first": ("out[i * K + bit / 64] |= (uint64_t)1 << (bit % 64);",
                  "out[i * K + bit / 64] |= (uint64_t)1 << (63 - bit % 64);"),
    # Eq. 4 with the classes exchanged
    "scores_swapped": ("if (subset(m->words[1] + p * K, x, K)) a += m->S[1][p];",
                       "if (subset(m->words[1] + p * K, x, K)) nn += m->S[1][p];"),
    # Eq. 3 against the same class
    "coherence_same_class": ("rc = fit_class(Xs[c], ns[c], Xs[1 - c], ns[1 - c], K, m, c);",
                             "rc = fit_class(Xs[c], ns[c], Xs[c], ns[c], K, m, c);"),
    # feature offsets off by one
    "offset_off_by_one": ("for (uint32_t f = 0; f < d; ++f) { off[f] = acc; acc += nbins[f]; }",
                          "for (uint32_t f = 0; f < d; ++f) { acc += nbins[f]; off[f] = acc - 1; }"),
    # pairs restricted to neighbours
    "pairs_neighbours_only": ("for (uint64_t j = i + 1; j < n; ++j) {\n            uint64_t *b = rows + m * K;",
                              "for (uint64_t j = i + 1; j < n && j < i + 2; ++j) {\n            uint64_t *b = rows + m * K;"),
    # first-cover position counted from zero
    "t_off_by_one": ("if (subset(b, Xo + t * K, K)) return t + 1;", "if (subset(b, Xo + t * K, K)) return t + 2;"),
    # Eq. 2 with |b| instead of |b|^2 for patterns given as code rows
    "from_patterns_not_squared": ("m->S[c][p] = (int64_t)fs[c][p] * (int64_t)len * (int64_t)len;",
                                  "m->S[c][p] = (int64_t)fs[c][p] * (int64_t)len;"),
    # |b| of given patterns without their last word
    "from_patterns_last_word_dropped": ("uint32_t len = popcount_row(m->words[c] + p * K, K);",
                                        "uint32_t len = popcount_row(m->words[c] + p * K, K - 1);"),
    # the supports of given patterns taken from the other class's list
    "from_patterns_f_swapped": ("m->f[c][p] = fs[c][p];", "m->f[c][p] = fs[1 - c][p < ms[1 - c] ? p : 0];"),
    # t(b) of a coherent pair counted as zero instead of every other-class record
    "pair_facts_t_coherent_zero": ("out_t[q] = t ? t : ns[1 - cls];", "out_t[q] = t;"),
}


def _run_pins():
    """Return True when every pin passes with the currently loaded oracle library."""
    try:
        pins.test_worked_example_c_oracle()
        for s in range(12):
            pins.test_exhaustive_enumeration(s)
        pins.test_pack_bit_order()
        pins.test_one_and_two_records()
        pins.test_model_from_patterns_worked_example()
        pins.test_model_from_patterns_weights_by_hand()
        for s in range(4):
            pins.test_model_from_patterns_reproduces_a_fit(s)
        for s in range(6):
            pins.test_pair_facts_t_by_scanning(s)
    except (AssertionError, oracle.OracleError):
        return False
    return True


@pytest.fixture(scope="module")
def src_text():
    return open(SRC).read()


def test_pins_pass_on_unmodified_oracle():
    assert _run_pins()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, src_text, tmp_path):
    old, new = MUTANTS[name]
    assert src_text.count(old) == 1, f"mutation site of {name} not found exactly once"
    mut = src_text.replace(old, new)
    c_path = tmp_path / "mut.c"
    so_path = tmp_path / "libmut.so"
    c_path.write_text(mut)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(so_path),
                    str(c_path)], check=True)
    try:
        oracle.use_library(str(so_path))
        oracle.lib()
        caught = not _run_pins()
    finally:
        oracle.use_library(None)
    assert caught, f"mutant {name} passed every pin"


# ---------------------------------------------- regulations and metrics
REG_SRC = os.path.join(os.path.dirname(SRC), "regulations.py")
REG_MUTANTS = {
    # Regulation 1 with ties going to normal
    "r1_strict": ("lab, rule = (1 if a >= n else 0), R1", "lab, rule = (1 if a > n else 0), R1"),
    # Regulation 2 dropped
    "r2_missing": ("if use_r2 and a == 0 and n == 0:", "if False:"),
    # Regulation 3 applied to flows already labelled attack
    "r3_on_attack_too": ("if use_r3 and lab == 0 and regulation3_fires(n, st, r):",
                         "if use_r3 and regulation3_fires(n, st, r):"),
    # Regulation 3's gap reversed
    "r3_gap_reversed": ("gap = st.mu - n_x", "gap = n_x - st.mu"),
    # sample instead of population variance
    "sample_variance": ("return Fraction(self.count * self.total_sq - self.total * self.total, self.count * self.count)",
                        "return Fraction(self.count * self.total_sq - self.total * self.total, "
                        "self.count * (self.count - 1))"),
    # ties counted as wins in the AUC
    "auc_ties_full": ("num += 2 * below + (upto - below)", "num += 2 * upto"),
    # recall over predicted positives
    "recall_is_precision": ("return self.tp / (self.tp + self.fn) if self.tp + self.fn else 0.0",
                            "return self.tp / (self.tp + self.fp) if self.tp + self.fp else 0.0"),
}


def _run_regulation_pins(mod):
    from tests import test_oracle_regulations as rp
    saved = rp.reg
    rp.reg = mod
    try:
        rp.test_worked_example_labels()
        rp.test_textbook_moments()
        for r, f in [(1.0, 3), (0.5, 4), (0.0, 5), (2.0, 1), (2.5, 0)]:
            rp.test_regulation3_threshold_is_exact(r, f)
        rp.test_regulation3_only_turns_normal_into_attack()
        rp.test_regulation3_with_a_non_dyadic_r()
        for s in range(8):
            rp.test_metrics_against_sklearn_and_brute_force(s)
        rp.test_auc_closed_forms()
    except AssertionError:
        return False
    finally:
        rp.reg = saved
    return True


def _module_from(text, name):
    import sys
    import types
    mod = types.ModuleType(name)
    sys.modules[name] = mod          # dataclasses look their module up there
    try:
        exec(compile(text, name, "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


def test_regulation_pins_pass_on_unmodified_oracle():
    assert _run_regulation_pins(_module_from(open(REG_SRC).read(), "reg_ok"))


@pytest.mark.parametrize("name", sorted(REG_MUTANTS))
def test_regulation_pins_catch_mutant(name):
    text = open(REG_SRC).read()
    old, new = REG_MUTANTS[name]
    assert text.count(old) == 1, f"mutation site of {name} not found exactly once"
    assert not _run_regulation_pins(_module_from(text.replace(old, new), "reg_" + name)), \
        f"mutant {name} passed every pin"
