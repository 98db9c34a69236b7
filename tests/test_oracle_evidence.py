"""Pins of the evidence oracle (oracle/evidence.py) against facts fixed by the
paper and by mathematics, and plausible mistakes planted in copies of it:

* the hand-worked example (tests/golden/worked_example.md): the normal patterns
  inside t1 = (0,0,1) are {0,2,5} (S 9), {0,2} (S 8), {2,5} (S 8), in that order
  (equal weights by ascending words); the attack patterns inside t2 = (0,1,1)
  are {0,3,5} (S 9) and {3,5} (S 8)
* additivity with Eq. 4: the weights of all the patterns inside a flow sum to
  the C oracle's A(t) and N(t)
* brute force on small problems with Python integers and Python's sort
"""
import json
import os
import sys
import types

import numpy as np
import pytest

import oracle
from oracle import evidence as ev
from paper_2507_14222_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")
SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "evidence.py")


def _worked(mod):
    g = json.load(open(GOLD))
    nb = np.array(g["nbins"], np.uint16)
    om = oracle.fit(np.array(g["codes"], np.uint16), np.array(g["labels"], np.uint8), nb)
    out = mod.evidence(om, np.array(g["flows"], np.uint16), nb, 8)
    cnt, w, f, S = out[0][0]                      # t1, normal patterns
    assert cnt == 3 and [int(x) for x in w[:, 0]] == [0x25, 0x05, 0x24] and S.tolist() == [9, 8, 8]
    assert f.tolist() == [1, 2, 2]
    assert out[0][1][0] == 0                      # t1: no attack pattern inside
    cnt, w, f, S = out[1][1]                      # t2, attack patterns
    assert cnt == 2 and [int(x) for x in w[:, 0]] == [0x29, 0x28] and S.tolist() == [9, 8]
    cnt, w, f, S = ev.evidence(om, np.array(g["flows"][:1], np.uint16), nb, 2)[0][0]   # top 2 of 3
    assert cnt == 3 and [int(x) for x in w[:, 0]] == [0x25, 0x05]


def _additive(mod):
    for seed in (3, 4):
        p = synth.make_random_problem(seed, 80, 9, bins_lo=2, bins_hi=5)
        om = oracle.fit(p.codes, p.labels, p.nbins)
        flows = np.concatenate([p.codes[:25], synth.make_random_problem(seed + 50, 25, 9, 2, 5).codes % p.nbins])
        A, N = oracle.score(om, flows, p.nbins)
        out = mod.evidence(om, flows, p.nbins, 10 ** 9)
        for t in range(flows.shape[0]):
            assert int(out[t][0][3].sum()) == int(N[t]) and int(out[t][1][3].sum()) == int(A[t])
            assert out[t][0][0] == out[t][0][1].shape[0] and out[t][1][0] == out[t][1][1].shape[0]


def _brute(mod):
    # K = 1 and K = 2; models with rows in canonical order (fits) and shuffled
    for seed, d, blo, bhi in ((5, 7, 2, 4), (6, 7, 2, 4), (7, 20, 4, 6), (8, 24, 4, 5)):
        p = synth.make_random_problem(seed, 60, d, bins_lo=blo, bins_hi=bhi)
        fitted = oracle.fit(p.codes, p.labels, p.nbins)
        rng = np.random.default_rng(seed)
        perms = [rng.permutation(fitted.patterns[c].shape[0]) for c in (0, 1)]
        shuffled = types.SimpleNamespace(patterns=[fitted.patterns[c][perms[c]] for c in (0, 1)],
                                         f=[fitted.f[c][perms[c]] for c in (0, 1)],
                                         S=[fitted.S[c][perms[c]] for c in (0, 1)])
        for om in (fitted, shuffled):
            _brute_model(mod, om, p)


def _brute_model(mod, om, p):
    flows = p.codes[:20]
    fw = oracle.pack(flows, p.nbins)
    for k in (1, 3, 50):
        out = mod.evidence(om, flows, p.nbins, k)
        for t in range(flows.shape[0]):
            tv = [int(x) for x in fw[t]]
            for c in (0, 1):
                rows = []
                for i in range(om.patterns[c].shape[0]):
                    wv = [int(x) for x in om.patterns[c][i]]
                    if all(a & ~b == 0 for a, b in zip(wv, tv)):
                        rows.append((-int(om.S[c][i]), wv, int(om.f[c][i])))
                rows.sort()
                cnt, w, f, S = out[t][c]
                assert cnt == len(rows)
                got = [(-int(s), [int(x) for x in ww], int(ff)) for s, ww, ff in zip(S, w, f)]
                assert got == rows[:k]


def test_worked_example():
    _worked(ev)


def test_additive_with_eq4():
    _additive(ev)


def test_brute_force():
    _brute(ev)


MUTANTS = {
    # weights ascending
    "ascending_weight": ("keys.append(-S[idx])", "keys.append(S[idx])"),
    # ties left in index order instead of word order
    "no_word_tiebreak": ("keys = [patterns[idx, k] for k in range(patterns.shape[1] - 1, -1, -1)]", "keys = []"),
    # words compared with the last word most significant
    "last_word_first": ("keys = [patterns[idx, k] for k in range(patterns.shape[1] - 1, -1, -1)]",
                        "keys = [patterns[idx, k] for k in range(patterns.shape[1])]"),
    # Eq. 6 operands transposed
    "subset_transposed": ("return np.all((patterns & ~flow_words[None, :]) == 0, axis=1)",
                          "return np.all((flow_words[None, :] & ~patterns) == 0, axis=1)"),
    # count of the reported list instead of every pattern inside
    "count_truncated": ("per.append((int(idx.size), P[top], f[top], S[top]))",
                        "per.append((int(top.size), P[top], f[top], S[top]))"),
    # classes exchanged
    "classes_swapped": ("P, f, S = model.patterns[c], model.f[c], model.S[c]",
                        "P, f, S = model.patterns[1 - c], model.f[1 - c], model.S[1 - c]"),
}


def _module(text, name):
    mod = types.ModuleType(name)
    text = text.replace("from . import pack", "from oracle import pack")
    exec(compile(text, name, "exec"), mod.__dict__)
    return mod


def _pins_pass(mod):
    try:
        _worked(mod)
        _additive(mod)
        _brute(mod)
    except AssertionError:
        return False
    return True


def test_pins_pass_on_unmodified_copy():
    assert _pins_pass(_module(open(SRC).read(), "ev_ok"))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name):
    text = open(SRC).read()
    old, new = MUTANTS[name]
    assert text.count(old) == 1, name
    assert not _pins_pass(_module(text.replace(old, new), "ev_" + name)), f"mutant {name} passed every pin"
