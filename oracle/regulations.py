"""Classifier regulations and detection metrics -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark may import this module.
It applies the three regulations of Section 3.1 to the evidence (A, N) of each
flow (Eq. 4) and computes the detection metrics of Table 2, in plain Python with
exact integers and fractions: nothing here rounds before the final conversion of
a metric to a float.

Readings taken where the paper is silent:
  - mu_N and sigma_N of Regulation 3 are the mean and the population standard
    deviation of N(x) over the normal training records x; r is a given constant
    (Table 2's header names 0.568).
  - Regulation 3 is decided exactly: N < mu_N - r sigma_N with mu_N and
    sigma_N the exact real values and r the exact value of the given double.
  - Regulation 2 overrides Regulation 1 (both label attack, so only the
    reported deciding regulation differs); Regulation 3 only turns a normal
    label into attack.
  - Positive class = attack (label 1).  The AUC ranks flows by the margin
    A(x) - N(x), the quantity Regulation 1 compares with zero; ties between an
    attack and a normal flow count one half.
"""
from __future__ import annotations

import bisect
from dataclasses import dataclass
from fractions import Fraction
from typing import List, Sequence, Tuple

import numpy as np

R1, R2, R3 = 1, 2, 3   # the regulation that decided a label


@dataclass
class NormalStats:
    count: int        # normal training records
    total: int        # sum of N over them
    total_sq: int     # sum of N^2 over them

    @property
    def mu(self) -> Fraction:
        return Fraction(self.total, self.count)

    @property
    def var(self) -> Fraction:
        """Population variance: mean of N^2 minus the squared mean."""
        return Fraction(self.count * self.total_sq - self.total * self.total, self.count * self.count)

    def mu_float(self) -> float:
        return float(self.mu)

    def sigma_float(self) -> float:
        import math
        return math.sqrt(self.var)


def normal_stats(N: Sequence[int], labels: Sequence[int]) -> NormalStats:
    """Moments of N(x) over the records labelled normal (label 0)."""
    vals = [int(v) for v, lab in zip(N, labels) if int(lab) == 0]
    return NormalStats(len(vals), sum(vals), sum(v * v for v in vals))


def regulation3_fires(n_x: int, st: NormalStats, r: float) -> bool:
    """N(x) < mu_N - r sigma_N, exactly.  With r >= 0 and sigma_N >= 0 this holds
    iff mu_N - N(x) > 0 and (mu_N - N(x))^2 > r^2 sigma_N^2."""
    gap = st.mu - n_x
    rr = Fraction(r)
    return gap > 0 and gap * gap > rr * rr * st.var


def classify(A: Sequence[int], N: Sequence[int], st: NormalStats = None, r: float = 0.0,
             use_r2: bool = True, use_r3: bool = True) -> Tuple[List[int], List[int]]:
    """Labels (1 attack, 0 normal) and the deciding regulation of each flow."""
    labels, rules = [], []
    for a, n in zip(A, N):
        a, n = int(a), int(n)
        lab, rule = (1 if a >= n else 0), R1                  # Regulation 1
        if use_r2 and a == 0 and n == 0:                      # Regulation 2
            lab, rule = 1, R2
        if use_r3 and lab == 0 and regulation3_fires(n, st, r):   # Regulation 3
            lab, rule = 1, R3
        labels.append(lab)
        rules.append(rule)
    return labels, rules


@dataclass
class Metrics:
    tp: int
    fp: int
    tn: int
    fn: int
    auc_num: int      # twice the Mann-Whitney U of the margins (attack above normal)
    auc_den: int      # twice (attack flows) x (normal flows)

    @property
    def accuracy(self) -> float:
        return (self.tp + self.tn) / (self.tp + self.fp + self.tn + self.fn)

    @property
    def recall(self) -> float:
        return self.tp / (self.tp + self.fn) if self.tp + self.fn else 0.0

    @property
    def precision(self) -> float:
        return self.tp / (self.tp + self.fp) if self.tp + self.fp else 0.0

    @property
    def auc(self) -> float:
        return self.auc_num / self.auc_den if self.auc_den else 0.0


def metrics(pred: Sequence[int], truth: Sequence[int], A: Sequence[int], N: Sequence[int]) -> Metrics:
    """Confusion counts of the labels against the truth (attack = positive) and the
    AUC of the margins A - N: the probability that an attack flow's margin exceeds
    a normal flow's, ties one half, counted pair by pair through a sorted list of
    the normal flows' margins."""
    pred = np.asarray(pred, np.int64)
    truth = np.asarray(truth, np.int64)
    tp = int(np.sum((pred == 1) & (truth == 1)))
    fp = int(np.sum((pred == 1) & (truth == 0)))
    tn = int(np.sum((pred == 0) & (truth == 0)))
    fn = int(np.sum((pred == 0) & (truth == 1)))
    margin = [int(a) - int(n) for a, n in zip(A, N)]
    pos = [m for m, t in zip(margin, truth) if t == 1]
    neg = sorted(m for m, t in zip(margin, truth) if t == 0)
    num = 0
    for m in pos:
        below = bisect.bisect_left(neg, m)       # normal flows with a smaller margin
        upto = bisect.bisect_right(neg, m)       # ... plus those with the same margin
        num += 2 * below + (upto - below)
    return Metrics(tp, fp, tn, fn, num, 2 * len(pos) * len(neg))
