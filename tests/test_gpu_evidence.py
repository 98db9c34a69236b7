"""ig_evidence against the evidence oracle (oracle/evidence.py): for each flow and
class, the number of patterns inside the flow and the k heaviest of them (weight
descending, then words ascending), words, supports and weights bit for bit."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import evidence as ev
from paper_2507_14222_amd import ig, synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def say(*a):
    print("[evidence]", *a, flush=True)
    sys.stdout.flush()


def gpu_evidence(m, flows, k):
    import torch
    cnt, w, f, S = ig.evidence(m, flows, k)
    torch.cuda.synchronize()
    return (cnt.cpu().numpy().view(np.uint32), w.cpu().numpy().view(np.uint64), f.cpu().numpy().view(np.uint32),
            S.cpu().numpy())


def compare(m, om, flows, nbins, k, invalid=()):
    cnt, w, f, S = gpu_evidence(m, flows, k)
    ok = [t for t in range(flows.shape[0]) if t not in set(invalid)]
    want = ev.evidence(om, flows[ok], nbins, k)
    for j, t in enumerate(ok):
        for c in (0, 1):
            oc, ow, of, oS = want[j][c]
            q = ow.shape[0]
            assert cnt[t, c] == oc, (t, c)
            assert np.array_equal(w[t, c, :q], ow) and np.array_equal(f[t, c, :q], of) and np.array_equal(S[t, c, :q], oS)
            assert not w[t, c, q:].any() and not f[t, c, q:].any() and not S[t, c, q:].any()
    for t in invalid:
        assert (cnt[t] == 0xFFFFFFFF).all() and not S[t].any()


def test_worked_example():
    g = json.load(open(GOLD))
    nb = np.array(g["nbins"], np.uint16)
    m = ig.fit(np.array(g["codes"], np.uint16), np.array(g["labels"], np.uint8), nb)
    cnt, w, f, S = gpu_evidence(m, np.array(g["flows"], np.uint16), 2)
    assert cnt[0].tolist() == [3, 0] and [int(x) for x in w[0, 0, :, 0]] == [0x25, 0x05] and S[0, 0].tolist() == [9, 8]
    assert cnt[1].tolist() == [0, 2] and [int(x) for x in w[1, 1, :, 0]] == [0x29, 0x28] and f[1, 1].tolist() == [1, 2]


CASES = [(3, 80, 9, 2, 5), (7, 129, 10, 3, 9), (8, 200, 30, 4, 8), (11, 170, 41, 10, 14), (14, 120, 80, 12, 16)]


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}-n{c[1]}-d{c[2]}" for c in CASES])
def test_random_problems(case):
    seed, n, d, blo, bhi = case
    p = synth.make_random_problem(seed, n, d, bins_lo=blo, bins_hi=bhi)
    m = ig.fit(p.codes, p.labels, p.nbins)
    om = oracle.fit(p.codes, p.labels, p.nbins)
    rng = np.random.default_rng(seed)
    flows = np.concatenate([p.codes[:40], np.stack([rng.integers(0, b, 30) for b in p.nbins], 1)]).astype(np.uint16)
    flows[5, 1] = p.nbins[1]   # a code out of range
    say(case, "bucketed", m.bucketed, "patterns", m.n_patterns())
    for k in (1, 5, 64, 256):
        compare(m, om, flows, p.nbins, k, invalid=(5,))


def test_valu_model_scans_every_pattern():
    p = synth.make_random_problem(12, 140, 50, bins_lo=10, bins_hi=14)
    m = ig.fit(p.codes, p.labels, p.nbins, kernels="valu")
    om = oracle.fit(p.codes, p.labels, p.nbins)
    say("no buckets", m.bucketed)
    compare(m, om, p.codes[:30], p.nbins, 20)


@pytest.mark.timeout(600)
def test_15k_workload_sample():
    w = synth.make_15k()
    m = ig.fit(w.codes, w.labels, w.nbins)
    om = oracle.fit(w.codes, w.labels, w.nbins)
    say("15k: 10 flows")
    compare(m, om, w.test_codes[:10], w.nbins, 32)
    with pytest.raises(ig.IGError) as e:
        ig.evidence(m, w.test_codes[:2], 257)
    assert e.value.status == ig.IG_E_INVAL
