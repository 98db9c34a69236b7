"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

* the hand-worked example (Eq. 1-4 applied by hand, tests/golden/worked_example.*)
* exhaustive enumeration of every subset of a tiny token universe, a loop order
  unrelated to the oracle's (pairs -> sort -> scan)
* special cases with textbook answers (empty other class, one or two records)
* the C oracle against the set-based definitional oracle on random problems
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import definitional as dfn
from paper_2507_14222_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def _tokset_to_words(b, nbins):
    """Eq. 5 for a set of (feature, bin) tokens -- written here, not taken from the oracle."""
    off = np.concatenate([[0], np.cumsum(np.asarray(nbins, dtype=np.int64))[:-1]])
    L = int(np.sum(nbins))
    K = (L + 63) // 64
    w = [0] * K
    for f, c in b:
        bit = int(off[f]) + int(c)
        w[bit // 64] |= 1 << (bit % 64)
    return tuple(w)


def _definitional_as_arrays(model, nbins):
    out = {}
    for c in (0, 1):
        rows = sorted((_tokset_to_words(b, nbins), f, S) for b, (f, S) in model[c].items())
        out[c] = rows
    return out


def _oracle_as_rows(m):
    out = {}
    for c in (0, 1):
        out[c] = [(tuple(int(x) for x in m.patterns[c][p]), int(m.f[c][p]), int(m.S[c][p]))
                  for p in range(m.patterns[c].shape[0])]
    return out


# ------------------------------------------------------------ worked example
def test_worked_example_c_oracle():
    g = json.load(open(GOLD))
    codes = np.array(g["codes"], np.uint16)
    labels = np.array(g["labels"], np.uint8)
    nbins = np.array(g["nbins"], np.uint16)
    m = oracle.fit(codes, labels, nbins)
    for c in ("0", "1"):
        exp = [(int(h, 16), f, S) for h, f, S in g["patterns"][c]]
        got = [(int(m.patterns[int(c)][p, 0]), int(m.f[int(c)][p]), int(m.S[int(c)][p]))
               for p in range(m.patterns[int(c)].shape[0])]
        assert got == exp, c
    for k in ("pairs", "distinct", "coherent", "tests"):
        assert m.stats[k] == g["stats"][k], k
    A, N = oracle.score(m, np.array(g["flows"], np.uint16), nbins)
    assert A.tolist() == g["A"]
    assert N.tolist() == g["N"]
    A2, N2 = oracle.score_direct(codes, labels, nbins, np.array(g["flows"], np.uint16))
    assert A2.tolist() == g["A"] and N2.tolist() == g["N"]


def test_worked_example_definitional():
    g = json.load(open(GOLD))
    model = dfn.fit(g["codes"], g["labels"])
    got = _definitional_as_arrays(model, g["nbins"])
    for c in (0, 1):
        exp = [((int(h, 16),), f, S) for h, f, S in g["patterns"][str(c)]]
        assert got[c] == exp
    sc = dfn.score(model, g["flows"])
    assert [a for a, _ in sc] == g["A"]
    assert [n for _, n in sc] == g["N"]


def test_pack_bit_order():
    # Eq. 5 with the least-significant-bit-first reading: token j -> word j//64, bit j%64
    nbins = np.array([64, 3, 70], np.uint16)       # L = 137, K = 3
    codes = np.array([[0, 0, 0], [63, 2, 69], [5, 1, 60]], np.uint16)
    w = oracle.pack(codes, nbins)
    assert w.shape == (3, 3)
    assert w[0].tolist() == [1, 1 | (1 << 3), 0]
    # bit 63; bit 64+2 = 66; bit 67+69 = 136 -> word 2 bit 8
    assert w[1].tolist() == [1 << 63, 1 << 2, 1 << 8]
    # bit 5; bit 65; bit 127 -> word 1 bit 63
    assert w[2].tolist() == [1 << 5, (1 << 1) | (1 << 63), 0]
    absent = np.array([[0xFFFF, 1, 0xFFFF]], np.uint16)
    assert oracle.pack(absent, nbins)[0].tolist() == [0, 1 << 1, 0]
    with pytest.raises(oracle.OracleError):
        oracle.pack(np.array([[64, 0, 0]], np.uint16), nbins)


# ------------------------------------------------- exhaustive enumeration
def _enumerate_expected(codes, labels, nbins):
    """Every non-empty subset b of the universe: b is a candidate of class c when
    it equals a record or the AND of two distinct-index records; coherent when no
    other-class record contains it; f counts class records containing it.
    Scores sum over every subset of the flow."""
    off = np.concatenate([[0], np.cumsum(nbins.astype(np.int64))[:-1]])
    L = int(nbins.sum())
    recs = []
    for row in codes:
        m = 0
        for f, c in enumerate(row):
            m |= 1 << int(off[f] + c)
        recs.append(m)
    X = {c: [r for r, lab in zip(recs, labels) if lab == c] for c in (0, 1)}
    pats = {0: {}, 1: {}}
    for c in (0, 1):
        Xc, Xo = X[c], X[1 - c]
        members = set(Xc)
        for i in range(len(Xc)):
            for j in range(i + 1, len(Xc)):
                members.add(Xc[i] & Xc[j])
        for b in range(1, 1 << L):
            if b not in members:
                continue
            if any((b & r) == b for r in Xo):
                continue
            f = sum(1 for x in Xc if (b & x) == b)
            pats[c][b] = (f, f * bin(b).count("1") ** 2)
    return pats, recs


@pytest.mark.parametrize("seed", range(12))
def test_exhaustive_enumeration(seed):
    rng = np.random.default_rng(100 + seed)
    d = int(rng.integers(2, 5))
    nbins = rng.integers(2, 4, size=d).astype(np.uint16)    # L <= 12
    n = int(rng.integers(2, 14))
    codes = np.stack([rng.integers(0, nb, size=n) for nb in nbins], axis=1).astype(np.uint16)
    labels = rng.integers(0, 2, size=n).astype(np.uint8)
    pats, _ = _enumerate_expected(codes, labels, nbins)
    m = oracle.fit(codes, labels, nbins)
    for c in (0, 1):
        got = {int(m.patterns[c][p, 0]): (int(m.f[c][p]), int(m.S[c][p]))
               for p in range(m.patterns[c].shape[0])}
        assert got == pats[c]
        # canonical order is ascending
        w = m.patterns[c][:, 0]
        assert np.all(w[1:] > w[:-1])
    flows = np.stack([rng.integers(0, nb, size=9) for nb in nbins], axis=1).astype(np.uint16)
    A, N = oracle.score(m, flows, nbins)
    off = np.concatenate([[0], np.cumsum(nbins.astype(np.int64))[:-1]])
    for t, row in enumerate(flows):
        x = 0
        for f, cc in enumerate(row):
            x |= 1 << int(off[f] + cc)
        expA = sum(S for b, (_, S) in pats[1].items() if (b & x) == b)
        expN = sum(S for b, (_, S) in pats[0].items() if (b & x) == b)
        # every subset of x, enumerated bit by bit
        sub = x
        expA2 = expN2 = 0
        while sub:
            expA2 += pats[1].get(sub, (0, 0))[1]
            expN2 += pats[0].get(sub, (0, 0))[1]
            sub = (sub - 1) & x
        assert (int(A[t]), int(N[t])) == (expA, expN) == (expA2, expN2)


# ------------------------------------------------------------ special cases
def _rand_problem(rng, n, d=4, bmax=4):
    nbins = rng.integers(2, bmax + 1, size=d).astype(np.uint16)
    codes = np.stack([rng.integers(0, nb, size=n) for nb in nbins], axis=1).astype(np.uint16)
    return codes, nbins


def test_empty_other_class_keeps_every_candidate():
    # With no record of the other class, Eq. 3 removes nothing: P = B (without the empty set).
    rng = np.random.default_rng(7)
    codes, nbins = _rand_problem(rng, 9)
    labels = np.zeros(9, np.uint8)
    m = oracle.fit(codes, labels, nbins)
    X = [dfn.tokens(r) for r in codes]
    B = set(X)
    for i in range(9):
        for j in range(i + 1, 9):
            if X[i] & X[j]:
                B.add(X[i] & X[j])
    assert m.stats["coherent"][0] == len(B) == m.stats["distinct"][0]
    assert m.stats["coherent"][1] == 0 and m.patterns[1].shape[0] == 0


def test_one_and_two_records():
    nbins = np.array([3, 3, 3], np.uint16)
    # one normal record, one attack record that shares nothing
    m = oracle.fit(np.array([[0, 0, 0], [1, 1, 1]], np.uint16), np.array([0, 1], np.uint8), nbins)
    assert m.patterns[0].shape[0] == 1 and m.patterns[1].shape[0] == 1
    assert m.f[0].tolist() == [1] and m.S[0].tolist() == [9]
    # two normal records: candidates {x1, x2, x1 & x2}
    codes = np.array([[0, 0, 0], [0, 1, 0], [2, 2, 2]], np.uint16)
    m = oracle.fit(codes, np.array([0, 0, 1], np.uint8), nbins)
    got = sorted((int(w[0]), int(f), int(S)) for w, f, S in zip(m.patterns[0], m.f[0], m.S[0]))
    x1 = 1 | (1 << 3) | (1 << 6)
    x2 = 1 | (1 << 4) | (1 << 6)
    assert got == sorted([(x1, 1, 9), (x2, 1, 9), (x1 & x2, 2, 8)])


def test_duplicates_and_contradictions():
    nbins = np.array([2, 2], np.uint16)
    # a record present in both classes can never be a pattern of either class
    codes = np.array([[0, 0], [0, 0], [0, 0], [1, 1]], np.uint16)
    labels = np.array([0, 0, 1, 1], np.uint8)
    m = oracle.fit(codes, labels, nbins)
    assert m.patterns[0].shape[0] == 0
    assert [int(w[0]) for w in m.patterns[1]] == [0b1010]
    # duplicated record: counted twice in f, present once
    m = oracle.fit(np.array([[0, 0], [0, 0], [1, 1]], np.uint16), np.array([0, 0, 1], np.uint8), nbins)
    assert m.f[0].tolist() == [2] and m.S[0].tolist() == [8]


# ----------------------------------------------- C vs set-based oracle
@pytest.mark.parametrize("seed", range(20))
def test_c_oracle_matches_definitional(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 40))
    d = int(rng.integers(1, 9))
    nbins = rng.integers(1, 12, size=d).astype(np.uint16)
    codes = np.stack([rng.integers(0, nb, size=n) for nb in nbins], axis=1).astype(np.uint16)
    labels = (rng.random(n) < rng.uniform(0.1, 0.9)).astype(np.uint8)
    m = oracle.fit(codes, labels, nbins)
    model = dfn.fit(codes, labels)
    assert _oracle_as_rows(m) == _definitional_as_arrays(model, nbins)
    flows = np.stack([rng.integers(0, nb, size=15) for nb in nbins], axis=1).astype(np.uint16)
    A, N = oracle.score(m, flows, nbins)
    assert list(zip(A.tolist(), N.tolist())) == dfn.score(model, flows)
    A2, N2 = oracle.score_direct(codes, labels, nbins, flows)
    assert A2.tolist() == A.tolist() and N2.tolist() == N.tolist()


def test_multiword_universe_against_definitional():
    # K > 1 with a ragged last word: 9 features of 30 bins -> L = 270, K = 5
    p = synth.make_random_problem(5, 60, 9, bins_lo=30, bins_hi=30, concentration=0.3)
    m = oracle.fit(p.codes, p.labels, p.nbins)
    assert m.K == 5
    model = dfn.fit(p.codes, p.labels)
    assert _oracle_as_rows(m) == _definitional_as_arrays(model, p.nbins)


def test_pair_facts_and_direct_score():
    p = synth.make_random_problem(11, 50, 6, bins_lo=3, bins_hi=5)
    m = oracle.fit(p.codes, p.labels, p.nbins)
    n0 = int((p.labels == 0).sum())
    pi = np.array([0, 1, 2, 3, 4], np.uint64)
    pj = np.array([0, 5, 9, 3, n0 - 1], np.uint64)
    words, coh, f, t = oracle.pair_facts(p.codes, p.labels, p.nbins, 0, pi, pj)
    pats = {tuple(int(x) for x in r): (int(ff), int(S)) for r, ff, S in zip(m.patterns[0], m.f[0], m.S[0])}
    for q in range(5):
        key = tuple(int(x) for x in words[q])
        assert (key in pats) == bool(coh[q])
        if coh[q]:
            assert pats[key][0] == int(f[q])
    flows = p.codes[:10]
    A, N = oracle.score(m, flows, p.nbins)
    A2, N2 = oracle.score_direct(p.codes, p.labels, p.nbins, flows)
    assert A.tolist() == A2.tolist() and N.tolist() == N2.tolist()


# --------------------------------------------- patterns given as code rows
def _words_to_codes(W, nbins):
    """Code rows of one-token-per-feature bitsets (the inverse of Eq. 5, written
    here): the set bit of a feature's block gives its bin, no bit gives 0xFFFF."""
    nbins = np.asarray(nbins, np.int64)
    off = np.concatenate([[0], np.cumsum(nbins)])
    out = np.full((W.shape[0], nbins.size), 0xFFFF, np.uint16)
    for r in range(W.shape[0]):
        x = 0
        for k in range(W.shape[1]):
            x |= int(W[r, k]) << (64 * k)
        for f in range(nbins.size):
            block = (x >> int(off[f])) & ((1 << int(nbins[f])) - 1)
            if block:
                assert block & (block - 1) == 0, "more than one bin of a feature"
                out[r, f] = block.bit_length() - 1
    return out


def test_model_from_patterns_worked_example():
    # Eq. 2 on the hand-worked patterns: the given supports, S = f |b|^2 by hand
    g = json.load(open(GOLD))
    nbins = np.array(g["nbins"], np.uint16)
    rows = {c: np.array([[int(h, 16)] for h, _, _ in g["patterns"][str(c)]], np.uint64) for c in (0, 1)}
    f = {c: np.array([ff for _, ff, _ in g["patterns"][str(c)]], np.uint32) for c in (0, 1)}
    S = {c: [SS for _, _, SS in g["patterns"][str(c)]] for c in (0, 1)}
    codes = {c: _words_to_codes(rows[c], nbins) for c in (0, 1)}
    m = oracle.model_from_patterns(codes[0], f[0], codes[1], f[1], nbins)
    for c in (0, 1):
        assert m.patterns[c].tolist() == rows[c].tolist()
        assert m.f[c].tolist() == f[c].tolist()
        assert m.S[c].tolist() == S[c]
    A, N = oracle.score(m, np.array(g["flows"], np.uint16), nbins)
    assert A.tolist() == g["A"] and N.tolist() == g["N"]


@pytest.mark.parametrize("seed", range(4))
def test_model_from_patterns_reproduces_a_fit(seed):
    # the patterns of a fit, given back as code rows with their supports, make the
    # same words, f and S (in the order given, here shuffled) and the same scores
    p = synth.make_random_problem(300 + seed, 45, 6 + 3 * seed, bins_lo=3, bins_hi=9 + 8 * seed)
    om = oracle.fit(p.codes, p.labels, p.nbins)
    rng = np.random.default_rng(seed)
    perm = [rng.permutation(om.patterns[c].shape[0]) for c in (0, 1)]
    codes = [_words_to_codes(om.patterns[c][perm[c]], p.nbins) for c in (0, 1)]
    m = oracle.model_from_patterns(codes[0], om.f[0][perm[0]], codes[1], om.f[1][perm[1]], p.nbins)
    for c in (0, 1):
        assert np.array_equal(m.patterns[c], om.patterns[c][perm[c]])
        assert np.array_equal(m.f[c], om.f[c][perm[c]])
        assert np.array_equal(m.S[c], om.S[c][perm[c]])
    flows = np.stack([rng.integers(0, nb, size=40) for nb in p.nbins], axis=1).astype(np.uint16)
    A, N = oracle.score(m, flows, p.nbins)
    A2, N2 = oracle.score(om, flows, p.nbins)
    assert A.tolist() == A2.tolist() and N.tolist() == N2.tolist()


def test_model_from_patterns_weights_by_hand():
    # one pattern of 3 tokens over two words (L = 70 + 30): S = f * 9 for any f
    nbins = np.array([70, 30], np.uint16)
    codes = np.array([[0xFFFF, 5], [69, 0xFFFF], [3, 29]], np.uint16)
    f = np.array([7, 1, 3], np.uint32)
    m = oracle.model_from_patterns(codes, f, codes[:0], f[:0], nbins)
    assert m.patterns[0].tolist() == [[0, 1 << 11], [0, 1 << 5], [1 << 3, 1 << 35]]
    assert m.S[0].tolist() == [7 * 1, 1 * 1, 3 * 4]
    assert m.patterns[1].shape == (0, 2)


# ----------------------------------------------------- t(b) by scanning
def _bits(codes, nbins):
    off = np.concatenate([[0], np.cumsum(np.asarray(nbins, np.int64))[:-1]])
    out = []
    for row in codes:
        x = 0
        for f, c in enumerate(row):
            x |= 1 << int(off[f] + c)
        out.append(x)
    return out


@pytest.mark.parametrize("seed", range(6))
def test_pair_facts_t_by_scanning(seed):
    # t(b): other-class records examined in input order up to and including the
    # first that contains b, all of them when none does (Eq. 3's scan); checked on
    # every pair i <= j of both classes, and summed over the distinct candidates it
    # is the fit's test count
    rng = np.random.default_rng(500 + seed)
    d = int(rng.integers(2, 6))
    nbins = rng.integers(2, 5, size=d).astype(np.uint16)
    n = int(rng.integers(3, 30))
    codes = np.stack([rng.integers(0, nb, size=n) for nb in nbins], axis=1).astype(np.uint16)
    labels = (rng.random(n) < 0.5).astype(np.uint8)
    if seed == 5:
        labels[:] = 0          # no other class: t = 0 and every candidate is coherent
    x = _bits(codes, nbins)
    om = oracle.fit(codes, labels, nbins)
    for c in (0, 1):
        Xc = [v for v, lab in zip(x, labels) if lab == c]
        Xo = [v for v, lab in zip(x, labels) if lab != c]
        if not Xc:
            continue
        pi, pj = zip(*[(i, j) for i in range(len(Xc)) for j in range(i, len(Xc))])
        words, coh, f, t = oracle.pair_facts(codes, labels, nbins, c, np.array(pi), np.array(pj))
        seen = {}
        for q, (i, j) in enumerate(zip(pi, pj)):
            b = Xc[i] & Xc[j]
            exp_t = next((r + 1 for r, o in enumerate(Xo) if b & o == b), len(Xo))
            assert int(t[q]) == exp_t, (c, i, j)
            assert bool(coh[q]) == (b != 0 and all(b & o != b for o in Xo))
            assert int(f[q]) == sum(1 for v in Xc if b & v == b)
            if b:
                seen[b] = exp_t
        assert sum(seen.values()) == om.stats["tests"][c]
