"""Pins of the regulations and detection-metric oracle (oracle/regulations.py)
against facts fixed by the paper and by mathematics:

* the hand-worked example's flows t1..t4 (Appendix of tests/golden/worked_example.md):
  normal, attack, attack by Regulation 2, normal
* Regulation 3 on a textbook sample whose mean (5) and population standard
  deviation (2) are known in closed form, at thresholds hit exactly
* Regulation 3 never turns an attack label into normal, and only acts on flows
  Regulation 1 labels normal
* accuracy, recall, precision and AUC against scikit-learn's routines, and the
  AUC against a brute-force count over every (attack, normal) pair
* closed forms: perfectly separated margins give AUC 1, reversed 0, all equal 1/2
"""
import json
import os
import random

import numpy as np
import pytest

import oracle
from oracle import regulations as reg

GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def test_worked_example_labels():
    g = json.load(open(GOLD))
    # Regulation 3 off (no statistics needed): R1 and R2 alone
    labels, rules = reg.classify(g["A"], g["N"], use_r3=False)
    assert labels == [0, 1, 1, 0]
    assert rules == [reg.R1, reg.R1, reg.R2, reg.R1]


def test_textbook_moments():
    N = [2, 4, 4, 4, 5, 5, 7, 9]
    st = reg.normal_stats(N + [100, 0], [0] * 8 + [1, 1])   # attack rows do not count
    assert (st.count, st.total, st.total_sq) == (8, 40, 232)
    assert st.mu == 5 and st.var == 4
    assert st.mu_float() == 5.0 and st.sigma_float() == 2.0


@pytest.mark.parametrize("r,fires_below", [(1.0, 3), (0.5, 4), (0.0, 5), (2.0, 1), (2.5, 0)])
def test_regulation3_threshold_is_exact(r, fires_below):
    # mu - r sigma = 5 - 2r exactly; N fires iff N < 5 - 2r (strict)
    st = reg.normal_stats([2, 4, 4, 4, 5, 5, 7, 9], [0] * 8)
    for n in range(-2, 10):
        assert reg.regulation3_fires(n, st, r) == (n < fires_below), (r, n)


def test_regulation3_only_turns_normal_into_attack():
    st = reg.normal_stats([2, 4, 4, 4, 5, 5, 7, 9], [0] * 8)
    A = [5, 1, 0, 0, 3]
    N = [2, 2, 0, 4, 3]
    labels, rules = reg.classify(A, N, st, 1.0)
    # flow 0: A >= N -> attack by R1 although N = 2 < 3
    # flow 1: A < N, N = 2 < 3 -> attack by R3
    # flow 2: A = N = 0 -> attack by R2 (R3 does not override it)
    # flow 3: A < N, N = 4 >= 3 -> normal
    # flow 4: A = N = 3 -> attack by R1 (ties go to attack)
    assert labels == [1, 1, 1, 0, 1]
    assert rules == [reg.R1, reg.R3, reg.R2, reg.R1, reg.R1]


def test_regulation3_with_a_non_dyadic_r():
    # r = 0.568 is not exact in binary: the decision uses the double's exact value
    from fractions import Fraction
    st = reg.normal_stats([0, 10], [0, 0])      # mu = 5, sigma = 5: threshold 5 - 5 r
    r = 0.568
    thr = 5 - 5 * Fraction(r)                   # 2.16 minus a tiny amount
    for n in range(0, 6):
        assert reg.regulation3_fires(n, st, r) == (n < thr)
    assert reg.regulation3_fires(2, st, r) and not reg.regulation3_fires(3, st, r)


def _brute_auc2(margins, truth):
    num = 0
    P = [m for m, t in zip(margins, truth) if t == 1]
    Q = [m for m, t in zip(margins, truth) if t == 0]
    for p in P:
        for q in Q:
            num += 2 if p > q else (1 if p == q else 0)
    return num, 2 * len(P) * len(Q)


@pytest.mark.parametrize("seed", range(8))
def test_metrics_against_sklearn_and_brute_force(seed):
    from sklearn.metrics import accuracy_score, precision_score, recall_score, roc_auc_score
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(5, 300))
    A = rng.integers(0, 6 + seed * 3, size=n)          # small ranges: many ties
    N = rng.integers(0, 6 + seed * 3, size=n)
    truth = rng.integers(0, 2, size=n)
    truth[0], truth[1] = 0, 1
    pred = rng.integers(0, 2, size=n)
    m = reg.metrics(pred, truth, A, N)
    assert (m.auc_num, m.auc_den) == _brute_auc2((A - N).tolist(), truth.tolist())
    assert m.tp + m.fp + m.tn + m.fn == n
    assert m.accuracy == pytest.approx(accuracy_score(truth, pred), abs=1e-15)
    assert m.recall == pytest.approx(recall_score(truth, pred, zero_division=0), abs=1e-15)
    assert m.precision == pytest.approx(precision_score(truth, pred, zero_division=0), abs=1e-15)
    assert m.auc == pytest.approx(roc_auc_score(truth, A - N), abs=1e-12)


def test_auc_closed_forms():
    truth = [0, 0, 0, 1, 1]
    assert reg.metrics(truth, truth, [0, 0, 0, 9, 9], [5, 4, 3, 0, 0]).auc == 1.0   # separated
    assert reg.metrics(truth, truth, [9, 9, 9, 0, 0], [0, 0, 0, 1, 1]).auc == 0.0   # reversed
    assert reg.metrics(truth, truth, [3] * 5, [3] * 5).auc == 0.5                    # all tied
    m = reg.metrics([1, 1], [1, 1], [1, 2], [0, 0])                                  # no normal flow
    assert m.auc_den == 0 and m.recall == 1.0 and m.precision == 1.0


def test_regulations_on_an_oracle_model():
    # the statistics come from N of the normal training records, scored by the
    # model fitted on them; with r = 0 Regulation 3 fires exactly below the mean
    from paper_2507_14222_amd import synth
    w = synth.make_tiny(0)
    om = oracle.fit(w.codes, w.labels, w.nbins)
    A_tr, N_tr = oracle.score(om, w.codes, w.nbins)
    st = reg.normal_stats(N_tr.tolist(), w.labels.tolist())
    assert st.count == int((w.labels == 0).sum())
    A, N = oracle.score(om, w.test_codes, w.nbins)
    labels, rules = reg.classify(A.tolist(), N.tolist(), st, 0.0)
    for a, n, lab, rule in zip(A.tolist(), N.tolist(), labels, rules):
        if rule == reg.R3:
            assert a < n and n * st.count < st.total
        elif a < n:
            assert lab == 0 and n * st.count >= st.total
