"""Batched fitting (ig_fit_batch): every model equals the one ig_fit builds for
the same problem -- patterns, supports, weights and counters -- whatever the
grouping, widths, sizes and tuning; small problems also equal the oracle."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2507_14222_amd import ig, synth, tune

pytestmark = pytest.mark.gpu


def say(*a):
    print("[batch]", *a, flush=True)
    sys.stdout.flush()


def _problems():
    ps = []
    specs = [(1, 1, 3, 2, 3), (2, 2, 3, 2, 3), (3, 40, 6, 2, 4), (4, 65, 8, 2, 6), (5, 200, 30, 4, 8),
             (6, 150, 40, 6, 10), (7, 170, 41, 10, 14), (8, 130, 60, 12, 16), (9, 120, 80, 12, 16),
             (10, 100, 80, 28, 32), (11, 300, 12, 2, 3), (12, 257, 6, 2, 2), (13, 90, 41, 10, 14)]
    for seed, n, d, lo, hi in specs:
        ps.append(synth.make_random_problem(seed, n, d, bins_lo=lo, bins_hi=hi))
    # one class only; no records; contradictions
    p = synth.make_random_problem(20, 50, 5, bins_lo=3, bins_hi=4)
    ps.append(synth.Problem(p.codes, np.zeros(p.n, np.uint8), p.nbins))
    ps.append(synth.Problem(np.zeros((0, 4), np.uint16), np.zeros(0, np.uint8), np.array([2, 3, 4, 5], np.uint16)))
    c = np.array([[1, 2, 3], [1, 2, 3], [0, 0, 0], [1, 0, 3]], np.uint16)
    ps.append(synth.Problem(c, np.array([0, 1, 1, 0], np.uint8), np.array([2, 3, 4], np.uint16)))
    return ps


def _same(a, b, tests=True):
    for c in (0, 1):
        for x, y in zip(a.export(c), b.export(c)):
            assert np.array_equal(x, y)
    sa, sb = a.stats(), b.stats()
    # tests and support_tests count the pairs the kernels examined: equal for the same kernels
    for k in ("n_class", "pairs", "distinct", "coherent") + (("tests", "support_tests") if tests else ()):
        assert getattr(sa, k) == getattr(sb, k), k


def test_batch_equals_plain_and_oracle():
    P = _problems()
    say("batch of", len(P))
    B = ig.fit_batch(P)                    # matrix cores where the operands fit 8 words
    BV = ig.fit_batch(P, kernels="valu")   # early-exit VALU path everywhere
    for p, mb, mv in zip(P, B, BV):
        _same(mb, ig.fit(p.codes, p.labels, p.nbins))                   # same kernels, same counters
        _same(mv, ig.fit(p.codes, p.labels, p.nbins, kernels="valu"))
        _same(mb, mv, tests=False)
        om = oracle.fit(p.codes, p.labels, p.nbins)
        for c in (0, 1):
            w, f, S = mb.export(c)
            assert np.array_equal(w, om.patterns[c]) and np.array_equal(f, om.f[c]) and np.array_equal(S, om.S[c])
        assert list(mv.stats().tests) == om.stats["tests"]


def test_groups_split_by_memory_and_tuning_give_same_models():
    P = _problems()
    say("small groups + tuning table")
    B0 = ig.fit_batch(P)
    table = [{"ks": 0, "min_pairs": 0, "filter_cpl": 2, "grid_per_cu": 4, "support_cpl": 1},
             {"ks": 8, "min_pairs": 1000, "filter_cpl": 1, "grid_per_cu": 16, "support_cpl": 2}]
    B1 = ig.fit_batch(P, mem_budget_bytes=40 * 30_000, tune=table)   # several groups, some problems alone
    for a, b in zip(B0, B1):
        _same(a, b)
        assert a.digest(0) == b.digest(0) and a.digest(1) == b.digest(1)


def test_digest_detects_differences():
    p = synth.make_random_problem(31, 120, 10, bins_lo=3, bins_hi=6)
    a = ig.fit(p.codes, p.labels, p.nbins)
    b = ig.fit(p.codes, p.labels, p.nbins)
    assert a.digest(0) == b.digest(0) and a.digest(1) == b.digest(1)
    q = synth.Problem(p.codes[:-1], p.labels[:-1], p.nbins)
    c = ig.fit(q.codes, q.labels, q.nbins)
    assert (a.digest(0), a.digest(1)) != (c.digest(0), c.digest(1))


def test_autotuner_small():
    say("autotune")
    t = tune.autotune([3, 8], sizes=(300,), reps=1)
    assert {e["ks"] for e in t["entries"]} == {3, 8}
    p = synth.make_random_problem(41, 200, 30, bins_lo=10, bins_hi=12)
    a = ig.fit(p.codes, p.labels, p.nbins, kernels="valu")
    b = ig.fit(p.codes, p.labels, p.nbins, tune=t["entries"], kernels="valu")
    _same(a, b)


# ------------------------------------------------ the 64-problem workload
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch64_small.json")


def _export_digest(m):
    h = hashlib.sha256()
    for c in (0, 1):
        w, f, S = m.export(c)
        h.update(np.ascontiguousarray(w, dtype="<u8").tobytes())
        h.update(np.ascontiguousarray(f, dtype="<u4").tobytes())
        h.update(np.ascontiguousarray(S, dtype="<i8").tobytes())
    return h.hexdigest()


def _check_golden(m, e):
    st = m.stats()
    for k in ("n_class", "pairs", "distinct", "coherent"):
        assert list(getattr(st, k)) == e["stats"][k], k
    assert _export_digest(m) == e["model_sha256"]


@pytest.mark.timeout(600)
def test_small_problems_of_the_64_problem_workload_match_the_oracle():
    """Every problem of the 64-problem workload (seed 3) with at most 5,000 records,
    fitted batched and one by one, against the oracle's stored digests."""
    g = json.load(open(GOLD))
    probs = synth.make_batch()
    idx = sorted(int(k) for k in g["problems"])
    say("seed-3 problems with n <= %d:" % g["max_n"], idx)
    ms = ig.fit_batch([probs[i] for i in idx])
    say("batched fit done")
    for i, m in zip(idx, ms):
        _check_golden(m, g["problems"][str(i)])
        m.free()
        say("batched problem", i, "ok")
    for i in idx:
        p = probs[i]
        m = ig.fit(p.codes, p.labels, p.nbins)
        _check_golden(m, g["problems"][str(i)])
        m.free()
        say("problem", i, "ok")


@pytest.mark.timeout(900)
def test_64_problem_workload_batched_equals_plain():
    """All 64 problems (seed 3): ig_fit_batch over memory-sized slices against 64
    plain ig_fit calls, model by model (device digests of the set of rows, f and S,
    plus every counter but the timings)."""
    import torch
    probs = synth.make_batch()
    dev = [(torch.from_numpy(p.codes.view(np.int16)).cuda(), torch.from_numpy(p.labels).cuda(), p.nbins)
           for p in probs]

    class P:
        def __init__(self, c, l, nb):
            self.codes, self.labels, self.nbins = c, l, nb

    def key(m):
        st = m.stats()
        return (m.digest(0), m.digest(1), st.n_class, st.pairs, st.distinct, st.coherent, st.tests,
                st.support_tests)

    batched = {}
    for sl in tune.slices_by_memory(probs):
        ms = ig.fit_batch([P(*dev[i]) for i in sl])
        for i, m in zip(sl, ms):
            batched[i] = key(m)
            m.free()
        say("batched slice", sl[0], "..", sl[-1])
    for i in range(len(probs)):
        m = ig.fit(*dev[i])
        assert key(m) == batched[i], f"problem {i}"
        m.free()
        if i % 8 == 7:
            say("plain fits equal up to", i)
