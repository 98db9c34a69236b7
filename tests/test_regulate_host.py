"""Host logic of the classifier: the integer cut of Regulation 3 (ig_r3_threshold)
against the oracle's exact decision N < mu_N - r sigma_N (Section 3.1), on
moments of many samples, for values of r that stress the exact arithmetic.  Runs
on the CPU: the threshold is computed on the host and needs no device."""
import numpy as np
import pytest

from oracle import regulations as R
from paper_2507_14222_amd import ig

RS = [0.0, 0.568, 1.0, 2.5, 1e-9, 1e-300, 3.0e6, 0.1 + 0.2]


def moments_of(vals):
    mo = ig.Moments()
    tot = sum(vals)
    sq = sum(v * v for v in vals)
    mo.count = len(vals)
    mo.sum[0], mo.sum[1] = tot & (2 ** 64 - 1), tot >> 64
    for i in range(3):
        mo.sumsq[i] = (sq >> (64 * i)) & (2 ** 64 - 1)
    return mo, R.normal_stats(vals, [0] * len(vals))


def check_cut(vals, r):
    mo, st = moments_of(vals)
    T = ig.r3_threshold(mo, r)
    assert T >= 0
    for N in range(max(0, T - 3), T + 4):
        assert R.regulation3_fires(N, st, r) == (N < T), (vals[:5], r, T, N)
    if T == 0:
        assert not R.regulation3_fires(0, st, r)


@pytest.mark.parametrize("r", RS)
def test_cut_matches_exact_decision_small(r):
    rng = np.random.default_rng(7)
    for trial in range(40):
        n = int(rng.integers(1, 30))
        vals = [int(v) for v in rng.integers(0, 1000, n)]
        check_cut(vals, r)


@pytest.mark.parametrize("r", RS)
def test_cut_matches_exact_decision_wide(r):
    """Values near 2^62 (sums beyond 64 bits, squares beyond 128)."""
    rng = np.random.default_rng(11)
    for trial in range(12):
        n = int(rng.integers(2, 300))
        base = int(rng.integers(0, 2 ** 62))
        vals = [base + int(v) for v in rng.integers(0, 2 ** 40, n)]
        check_cut(vals, r)


def test_cut_closed_forms():
    # all values equal: sigma = 0, the cut is the mean (N < mu exactly)
    check_cut([5, 5, 5], 0.568)
    mo, _ = moments_of([5, 5, 5])
    assert ig.r3_threshold(mo, 0.568) == 5
    mo, _ = moments_of([4, 6])           # mu 5, sigma 1: N < 5 - r
    assert ig.r3_threshold(mo, 1.0) == 4  # N < 4
    assert ig.r3_threshold(mo, 0.5) == 5  # N < 4.5: N <= 4
    assert ig.r3_threshold(mo, 5.0) == 0  # N < 0: never for N >= 0
    mo, _ = moments_of([0, 0, 10])       # mu 10/3 = 3.33.., r = 0: N < mu
    assert ig.r3_threshold(mo, 0.0) == 4


def test_cut_rejects_bad_arguments():
    mo, _ = moments_of([1, 2, 3])
    for r in (-0.1, float("nan"), float("inf")):
        with pytest.raises(ig.IGError) as e:
            ig.r3_threshold(mo, r)
        assert e.value.status == ig.IG_E_INVAL
    with pytest.raises(ig.IGError) as e:
        ig.r3_threshold(ig.Moments(), 0.5)
    assert e.value.status == ig.IG_E_INVAL
