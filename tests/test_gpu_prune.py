"""Pruned scoring (ig_score_ex, IG_SCORE_PRUNED): each flow meets only the token
buckets of its own tokens.  Exactness is the claim -- a pattern inside a flow holds
no token the flow lacks, so no weight of Eq. 4 may be lost -- so every case
compares the pruned sums with the dense kernel's and with the oracle, bit for bit."""
import sys

import numpy as np
import pytest

import oracle
from paper_2507_14222_amd import ig, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[prune]", *a, flush=True)
    sys.stdout.flush()


def scores(m, flows, mode):
    import torch
    out = ig.score(m, flows, mode=mode)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return o[:, 0], o[:, 1]


def all_modes_equal_oracle(m, om, flows, nbins):
    oA, oN = oracle.score(om, flows, nbins)
    for mode in ("pruned", "dense", "auto"):
        A, N = scores(m, flows, mode)
        assert np.array_equal(A, oA) and np.array_equal(N, oN), mode


CASES = [
    # seed, n, d, bins_lo, bins_hi, attack_frac: L below and above 256 tokens,
    # one-hot and factored operands, flows of one bucket spanning several blocks
    (4, 63, 8, 2, 6, 0.5),
    (7, 129, 10, 3, 9, 0.5),
    (8, 200, 30, 4, 8, 0.5),
    (11, 170, 41, 10, 14, 0.55),
    (18, 300, 12, 2, 3, 0.5),
    (19, 257, 6, 2, 2, 0.9),
    (21, 400, 41, 3, 70, 0.47),
]


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}-n{c[1]}-d{c[2]}" for c in CASES])
@pytest.mark.parametrize("kernels", ["auto", "mfma_onehot"])
def test_pruned_equals_dense_and_oracle(case, kernels):
    seed, n, d, blo, bhi, af = case
    p = synth.make_random_problem(seed, n, d, bins_lo=blo, bins_hi=bhi, attack_frac=af)
    if kernels == "mfma_onehot" and p.L > 1024:
        pytest.skip("one-hot matrix-core operands hold at most 16 words")
    m = ig.fit(p.codes, p.labels, p.nbins, kernels=kernels)
    say(case, kernels, "L", p.L, "patterns", m.n_patterns(), "bucketed", m.bucketed)
    if not m.bucketed:
        pytest.skip("scoring stays on the vector ALUs for this model")
    om = oracle.fit(p.codes, p.labels, p.nbins)
    rng = np.random.default_rng(seed)
    flows = np.stack([rng.integers(0, b, 700) for b in p.nbins], 1).astype(np.uint16)
    flows = np.concatenate([flows, p.codes, np.repeat(p.codes[:1], 600, axis=0)])   # one crowded bucket set
    all_modes_equal_oracle(m, om, flows, p.nbins)


def test_invalid_and_empty_flows():
    p = synth.make_random_problem(31, 150, 12, bins_lo=3, bins_hi=7)
    m = ig.fit(p.codes, p.labels, p.nbins)
    assert m.bucketed
    say("invalid flows")
    flows = p.codes[:40].copy()
    flows[3, 2] = p.nbins[2]          # out of range
    flows[17, 0] = 0xFFFF
    A, N = scores(m, flows, "pruned")
    assert A[3] == -1 and N[3] == -1 and A[17] == -1 and N[17] == -1
    om = oracle.fit(p.codes, p.labels, p.nbins)
    ok = np.ones(40, bool)
    ok[[3, 17]] = False
    oA, oN = oracle.score(om, flows[ok], p.nbins)
    assert np.array_equal(A[ok], oA) and np.array_equal(N[ok], oN)
    A, N = scores(m, np.zeros((0, p.d), np.uint16), "pruned")
    assert A.size == 0


def test_one_class_and_empty_models():
    nb = np.array([2, 3, 4], np.uint16)
    say("one class / empty")
    for codes, labels in [
        (np.zeros((0, 3)), np.zeros(0)),
        (np.array([[1, 2, 3], [1, 2, 3], [0, 0, 0]]), np.array([0, 0, 0])),
        (np.array([[1, 2, 3], [0, 1, 1]]), np.array([1, 1])),
    ]:
        codes = codes.astype(np.uint16)
        labels = labels.astype(np.uint8)
        m = ig.fit(codes, labels, nb)
        om = oracle.fit(codes, labels, nb)
        flows = np.array([[1, 2, 3], [0, 0, 0], [0, 1, 1], [1, 0, 2]], np.uint16)
        if m.bucketed:
            all_modes_equal_oracle(m, om, flows, nb)
        else:
            A, N = scores(m, flows, "auto")
            oA, oN = oracle.score(om, flows, nb)
            assert np.array_equal(A, oA) and np.array_equal(N, oN)


def test_imported_model_buckets_by_bins():
    nb = synth.mixture41_nbins()
    ps = synth.make_pattern_set(seed=43, per_class=4000)
    say("import", [c.shape for c in ps.codes])
    m = ig.import_patterns(ps.codes[0], ps.f[0], ps.codes[1], ps.f[1], nb)
    assert m.bucketed
    om = oracle.model_from_patterns(ps.codes[0], ps.f[0], ps.codes[1], ps.f[1], nb)
    flows = synth.make_flows(seed=44, n=1500)
    all_modes_equal_oracle(m, om, flows, nb)


def test_pruned_rejected_without_buckets():
    p = synth.make_random_problem(12, 140, 50, bins_lo=10, bins_hi=14)   # 9-10 one-hot words
    m = ig.fit(p.codes, p.labels, p.nbins, kernels="valu")
    say("no buckets", m.info().mfma_words, m.bucketed)
    if m.bucketed:
        pytest.skip("this model is bucketed")
    with pytest.raises(ig.IGError) as e:
        ig.score(m, p.codes[:4], mode="pruned")
    assert e.value.status == ig.IG_E_UNSUPPORTED
    om = oracle.fit(p.codes, p.labels, p.nbins)
    A, N = scores(m, p.codes[:50], "auto")
    oA, oN = oracle.score(om, p.codes[:50], p.nbins)
    assert np.array_equal(A, oA) and np.array_equal(N, oN)


def test_15k_workload_pruned_equals_dense():
    w = synth.make_15k()
    say("15k workload", w.codes.shape, w.test_codes.shape)
    m = ig.fit(w.codes, w.labels, w.nbins)
    assert m.bucketed
    A, N = scores(m, w.test_codes, "pruned")
    dA, dN = scores(m, w.test_codes, "dense")
    assert np.array_equal(A, dA) and np.array_equal(N, dN)
    # and in request-sized slices (every flow of a slice in its own lists)
    at = 0
    for k in (1, 7, 64, 255, 256, 257, 1000, 2000):
        a, n = scores(m, w.test_codes[at:at + k], "pruned")
        assert np.array_equal(a, A[at:at + k]) and np.array_equal(n, N[at:at + k]), k
        at += k


def _token_counts(codes, nbins):
    off = np.concatenate([[0], np.cumsum(nbins.astype(np.int64))])
    cnt = np.zeros(int(off[-1]), np.int64)
    for f in range(codes.shape[1]):
        np.add.at(cnt, off[f] + codes[:, f].astype(np.int64), 1)
    return cnt


@pytest.mark.parametrize("kernels,dense", [("auto", False), ("auto", True), ("valu", False)])
def test_bucket_of_each_pattern_is_its_rarest_token(kernels, dense):
    """Every pattern is filed under its token held by the fewest training records of
    its own class (lowest token on ties), whichever path fitted it: the bucket sizes
    equal a histogram of that rule over the exported patterns."""
    p = synth.make_random_problem(11, 170, 41, bins_lo=10, bins_hi=14, attack_frac=0.55)
    m = ig.fit(p.codes, p.labels, p.nbins, kernels=kernels, dense=dense)
    assert m.bucketed
    for c in (0, 1):
        cost = _token_counts(p.codes[p.labels == c], p.nbins)
        L = int(cost.size)
        w, _, _ = m.export(c)
        bits = np.unpackbits(w.view(np.uint8), axis=1, bitorder="little")[:, :L].astype(bool)
        keyed = np.where(bits, cost[None, :], np.iinfo(np.int64).max)
        key = np.argmin(keyed, axis=1)          # first minimum: the lowest token on ties
        want = np.bincount(key, minlength=L)
        got = m.bucket_sizes(c)
        assert got.sum() == w.shape[0] and np.array_equal(got, want), c
