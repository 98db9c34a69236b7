"""Invariants the IG definitions imply, checked on the C oracle.

They hold at any size and are reused by the GPU tests on outputs too large for
the oracle.  Each names the property it checks:

I1 every pattern is a record or lies inside two records of its class
I2 no pattern lies inside a record of the other class
I3 output is unchanged by any permutation of the input records
I4 swapping the labels swaps the two classes' outputs
I5 a record with no superset in the other class is a pattern of its class
I6 duplicating a record leaves P unchanged and adds one to f of each pattern inside it;
   adding an other-class record can only remove patterns
I7 one token per feature: at most one bit per feature block, popcount <= d
I8 f >= 1, and f >= 2 unless the pattern equals a record
I9 scores are additive over any split of the pattern set
I11 f <= n_c
"""
import numpy as np
import pytest

import oracle
from paper_2507_14222_amd import synth


def _sub(b, x):
    return bool(np.all((b & x) == b))


def _fit(p):
    return oracle.fit(p.codes, p.labels, p.nbins)


def _problem(seed, n=70, d=7):
    return synth.make_random_problem(seed, n, d, bins_lo=2, bins_hi=6)


def _rows(m, c):
    return [tuple(int(v) for v in r) for r in m.patterns[c]]


@pytest.mark.parametrize("seed", range(6))
def test_I1_I2_I5_I7_I8_I11(seed):
    p = _problem(seed)
    m = _fit(p)
    R = oracle.pack(p.codes, p.nbins)
    off = np.concatenate([[0], np.cumsum(p.nbins.astype(np.int64))])
    for c in (0, 1):
        Xc = R[p.labels == c]
        Xo = R[p.labels != c]
        recs = set(tuple(int(v) for v in r) for r in Xc)
        for b, f in zip(m.patterns[c], m.f[c]):
            sup = [x for x in Xc if _sub(b, x)]
            assert len(sup) == f                                       # f definition
            assert 1 <= f <= Xc.shape[0]                               # I8, I11
            if tuple(int(v) for v in b) not in recs:
                assert f >= 2                                          # I8
                # I1: b is exactly the AND of some pair of its supersets
                found = any(np.array_equal(sup[i] & sup[j], b)
                            for i in range(len(sup)) for j in range(i + 1, len(sup)))
                assert found
            assert not any(_sub(b, x) for x in Xo)                     # I2
            bits = np.unpackbits(b.view(np.uint8), bitorder="little")
            pos = np.flatnonzero(bits)
            blocks = np.searchsorted(off, pos, side="right") - 1
            assert len(set(blocks.tolist())) == len(pos) <= p.d        # I7
        pats = set(_rows(m, c))
        for x in Xc:                                                   # I5
            if not any(_sub(x, y) for y in Xo):
                assert tuple(int(v) for v in x) in pats


@pytest.mark.parametrize("seed", range(4))
def test_I3_permutation(seed):
    p = _problem(20 + seed)
    m = _fit(p)
    perm = np.random.default_rng(seed).permutation(p.n)
    m2 = oracle.fit(p.codes[perm], p.labels[perm], p.nbins)
    for c in (0, 1):
        assert np.array_equal(m.patterns[c], m2.patterns[c])
        assert np.array_equal(m.f[c], m2.f[c]) and np.array_equal(m.S[c], m2.S[c])


def test_I4_label_swap():
    p = _problem(31)
    m = _fit(p)
    m2 = oracle.fit(p.codes, (1 - p.labels).astype(np.uint8), p.nbins)
    for c in (0, 1):
        assert np.array_equal(m.patterns[c], m2.patterns[1 - c])
        assert np.array_equal(m.S[c], m2.S[1 - c])
    A, N = oracle.score(m, p.codes[:20], p.nbins)
    A2, N2 = oracle.score(m2, p.codes[:20], p.nbins)
    assert np.array_equal(A, N2) and np.array_equal(N, A2)


def test_I6_duplicate_and_added_record():
    p = _problem(41)
    m = _fit(p)
    R = oracle.pack(p.codes, p.nbins)
    i = 3
    codes = np.concatenate([p.codes, p.codes[i:i + 1]])
    labels = np.concatenate([p.labels, p.labels[i:i + 1]])
    m2 = oracle.fit(codes, labels, p.nbins)
    c = int(p.labels[i])
    assert np.array_equal(m.patterns[c], m2.patterns[c])
    inside = np.array([_sub(b, R[i]) for b in m.patterns[c]], dtype=np.int64)
    assert np.array_equal(m2.f[c].astype(np.int64), m.f[c].astype(np.int64) + inside)
    assert np.array_equal(m.patterns[1 - c], m2.patterns[1 - c])
    # an extra other-class record can only remove patterns of class c
    extra = np.array([[int(v) % int(nb) for v, nb in zip(p.codes[i] + 1, p.nbins)]], np.uint16)
    codes3 = np.concatenate([p.codes, extra])
    labels3 = np.concatenate([p.labels, np.array([1 - c], np.uint8)])
    m3 = oracle.fit(codes3, labels3, p.nbins)
    assert set(_rows(m3, c)) <= set(_rows(m, c))


def test_I9_additivity():
    p = _problem(51)
    m = _fit(p)
    flows = p.codes[:25]
    A, N = oracle.score(m, flows, p.nbins)
    R = oracle.pack(flows, p.nbins)
    for c, tot in ((1, A), (0, N)):
        half = m.patterns[c].shape[0] // 2
        parts = []
        for sl in (slice(0, half), slice(half, None)):
            parts.append(np.array([sum(int(S) for b, S in zip(m.patterns[c][sl], m.S[c][sl]) if _sub(b, x))
                                   for x in R], dtype=np.int64))
        assert np.array_equal(parts[0] + parts[1], tot)


def test_weights_are_support_times_squared_length():
    p = _problem(61)
    m = _fit(p)
    for c in (0, 1):
        pc = np.unpackbits(m.patterns[c].view(np.uint8), axis=1).sum(axis=1).astype(np.int64)
        assert np.array_equal(m.S[c], m.f[c].astype(np.int64) * pc * pc)
