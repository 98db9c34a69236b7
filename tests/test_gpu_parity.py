"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer, exact work: every comparison is bit-exact (patterns, f, S, counters,
scores).  Small sizes compare whole outputs; the 15k workload compares digests
of the whole output with the oracle's stored ones; the 148k workload compares
oracle facts on sampled pairs and flows plus properties that hold at any size.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2507_14222_amd import ig, synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print("[parity]", *a, flush=True)
    sys.stdout.flush()


def gpu_arrays(m):
    return [m.export(c) for c in (0, 1)]


def assert_same_model(m, om, K):
    for c in (0, 1):
        w, f, S = m.export(c)
        ow = om.patterns[c]
        assert w.shape == ow.shape, (c, w.shape, ow.shape)
        assert np.array_equal(w, ow), f"class {c}: pattern words differ"
        assert np.array_equal(f, om.f[c]), f"class {c}: supports differ"
        assert np.array_equal(S, om.S[c]), f"class {c}: weights differ"


def assert_same_stats(m, om):
    """Counters equal the oracle's, including the input-order sums of t(b)."""
    st = m.stats()
    assert list(st.pairs) == om.stats["pairs"]
    assert list(st.distinct) == om.stats["distinct"]
    assert list(st.coherent) == om.stats["coherent"]
    assert list(st.n_class) == om.stats["n_class"]
    assert list(st.tests) == om.stats["tests"]


def gpu_scores(m, flows):
    out = ig.score(m, flows)
    import torch
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return o[:, 0], o[:, 1]


# ------------------------------------------------------------ worked example
def test_worked_example():
    g = json.load(open(os.path.join(GOLD, "worked_example.json")))
    say("worked example")
    m = ig.fit(np.array(g["codes"], np.uint16), np.array(g["labels"], np.uint8), np.array(g["nbins"], np.uint16),
               kernels="valu")
    for c in ("0", "1"):
        w, f, S = m.export(int(c))
        got = [(int(w[p, 0]), int(f[p]), int(S[p])) for p in range(w.shape[0])]
        assert got == [(int(h, 16), ff, SS) for h, ff, SS in g["patterns"][c]]
    st = m.stats()
    assert list(st.pairs) == g["stats"]["pairs"] and list(st.distinct) == g["stats"]["distinct"]
    assert list(st.coherent) == g["stats"]["coherent"] and list(st.tests) == g["stats"]["tests"]
    A, N = gpu_scores(m, np.array(g["flows"], np.uint16))
    assert A.tolist() == g["A"] and N.tolist() == g["N"]


# ------------------------------------------------------------ tiny workload
def test_tiny_workload_full_parity():
    w = synth.make_tiny(0)
    say("tiny workload", w.codes.shape)
    om = oracle.fit(w.codes, w.labels, w.nbins)
    m = ig.fit(w.codes, w.labels, w.nbins, kernels="valu")
    assert_same_model(m, om, om.K)
    assert_same_stats(m, om)
    m = ig.fit(w.codes, w.labels, w.nbins)   # default kernels
    assert_same_model(m, om, om.K)
    A, N = gpu_scores(m, w.test_codes)
    oA, oN = oracle.score(om, w.test_codes, w.nbins)
    assert np.array_equal(A, oA) and np.array_equal(N, oN)


# ----------------------------------------------- random problems, all widths
CASES = [
    # seed, n, d, bins_lo, bins_hi, attack_frac   (K = ceil(sum bins / 64))
    (1, 1, 3, 2, 3, 0.5),
    (2, 2, 3, 2, 3, 0.5),
    (3, 3, 2, 2, 2, 0.34),
    (4, 63, 8, 2, 6, 0.5),
    (5, 64, 8, 2, 6, 0.3),
    (6, 65, 8, 2, 6, 0.7),
    (7, 129, 10, 3, 9, 0.5),      # K = 1..2
    (8, 200, 30, 4, 8, 0.5),      # K = 3
    (9, 150, 40, 6, 10, 0.45),    # K = 5
    (10, 180, 30, 12, 18, 0.5),   # K = 7
    (11, 170, 41, 10, 14, 0.55),  # K = 8
    (12, 140, 50, 10, 14, 0.5),   # K = 9..10
    (13, 130, 60, 12, 16, 0.5),   # K = 13..14
    (14, 120, 80, 12, 16, 0.5),   # K = 18..20
    (15, 110, 80, 20, 26, 0.5),   # K = 29..32
    (16, 100, 80, 28, 32, 0.5),   # K = 38..40
    (17, 90, 120, 28, 32, 0.5),   # K = 57..60
    (18, 300, 12, 2, 3, 0.5),     # dense overlaps, many duplicates
    (19, 257, 6, 2, 2, 0.9),      # L = 12, heavy repetition, unbalanced
]


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}-n{c[1]}-d{c[2]}" for c in CASES])
def test_random_problem_parity(case):
    seed, n, d, blo, bhi, af = case
    p = synth.make_random_problem(seed, n, d, bins_lo=blo, bins_hi=bhi, attack_frac=af)
    say("random problem", case, "L", p.L)
    om = oracle.fit(p.codes, p.labels, p.nbins)
    m = ig.fit(p.codes, p.labels, p.nbins, kernels="valu")
    assert m.K == om.K
    assert_same_model(m, om, om.K)
    assert_same_stats(m, om)
    m = ig.fit(p.codes, p.labels, p.nbins)   # default kernels (matrix cores when K <= 8)
    assert_same_model(m, om, om.K)
    info = m.info()
    # matrix cores whenever the operands (factored, else one-hot) fit 8 words
    assert info.mfma_words == (om.K if not info.flags & ig.IG_MODEL_FACTORED else info.mfma_words)
    assert m.score_on_matrix_cores == (info.mfma_words <= 8 and max(info.max_weight) < 2 ** 28)
    flows = synth.make_random_problem(seed + 1000, 97, d, bins_lo=blo, bins_hi=bhi).codes
    flows = np.minimum(flows, p.nbins[None, :] - 1).astype(np.uint16)
    flows = np.concatenate([flows, p.codes[: min(40, p.n)]])
    A, N = gpu_scores(m, flows)
    oA, oN = oracle.score(om, flows, p.nbins)
    assert np.array_equal(A, oA) and np.array_equal(N, oN)


def test_filter_lanes_per_candidate_agree():
    p = synth.make_random_problem(21, 333, 20, bins_lo=3, bins_hi=7)
    say("cpl 1 vs 2")
    a = ig.fit(p.codes, p.labels, p.nbins, filter_cpl=1, kernels="valu")
    b = ig.fit(p.codes, p.labels, p.nbins, filter_cpl=2, kernels="valu")
    for c in (0, 1):
        for x, y in zip(a.export(c), b.export(c)):
            assert np.array_equal(x, y)
    assert a.stats().tests == b.stats().tests


# ------------------------------------------------------- chunked pair space
def test_chunked_pair_space_gives_same_model():
    w = synth.make_tiny(0)
    say("chunked fit")
    om = oracle.fit(w.codes, w.labels, w.nbins)
    m = ig.fit(w.codes, w.labels, w.nbins, mem_budget_bytes=40 * 50_000)
    st = m.stats()
    assert st.chunks[0] > 1 and st.chunks[1] > 1
    assert_same_model(m, om, om.K)
    assert list(st.coherent) == om.stats["coherent"]


# ----------------------------------------------------------- packed inputs
def test_fit_packed_matches_codes_path():
    p = synth.make_random_problem(31, 211, 14, bins_lo=3, bins_hi=9)
    say("fit_packed")
    words = oracle.pack(p.codes, p.nbins)
    a = ig.fit(p.codes, p.labels, p.nbins)
    b = ig.fit_packed(words, p.labels)
    for c in (0, 1):
        for x, y in zip(a.export(c), b.export(c)):
            assert np.array_equal(x, y)
    fl = oracle.pack(p.codes[:50], p.nbins)
    out = ig.score_packed(b, fl).cpu().numpy()
    A, N = gpu_scores(a, p.codes[:50])
    assert np.array_equal(out[:, 0], A) and np.array_equal(out[:, 1], N)
    # a model fitted from codes scores packed flows too (on the VALU kernel when its
    # matrix-core operands are factored), including flows holding two bins of a feature
    out = ig.score_packed(a, fl).cpu().numpy()
    assert np.array_equal(out[:, 0], A) and np.array_equal(out[:, 1], N)
    wide = fl | oracle.pack(p.codes[50:100], p.nbins)
    om = oracle.fit(p.codes, p.labels, p.nbins)
    out = ig.score_packed(a, wide).cpu().numpy()
    for c, col in ((1, 0), (0, 1)):   # Eq. 4 by its definition on the words
        inside = np.all((om.patterns[c][None, :, :] & ~wide[:, None, :]) == 0, axis=2)
        assert np.array_equal(out[:, col], inside.astype(np.int64) @ om.S[c].astype(np.int64))


# ---------------------------------------------------------- imported sets
def test_import_patterns_and_score():
    rng = np.random.default_rng(41)
    nb = synth.mixture41_nbins()
    ps = synth.make_pattern_set(seed=41, per_class=3000)
    say("import", [c.shape for c in ps.codes])
    m = ig.import_patterns(ps.codes[0], ps.f[0], ps.codes[1], ps.f[1], nb)
    om = oracle.model_from_patterns(ps.codes[0], ps.f[0], ps.codes[1], ps.f[1], nb)
    for c in (0, 1):
        order = np.lexsort(om.patterns[c].T[::-1])
        w, f, S = m.export(c)
        assert np.array_equal(w, om.patterns[c][order])
        assert np.array_equal(f, om.f[c][order]) and np.array_equal(S, om.S[c][order])
    flows = synth.make_flows(seed=42, n=700)
    A, N = gpu_scores(m, flows)
    oA, oN = oracle.score(om, flows, nb)
    assert np.array_equal(A, oA) and np.array_equal(N, oN)
    # repeated pattern -> rejected
    dup = np.concatenate([ps.codes[0][:5], ps.codes[0][:1]])
    with pytest.raises(ig.IGError) as e:
        ig.import_patterns(dup, np.ones(6, np.uint32), ps.codes[1][:3], np.ones(3, np.uint32), nb)
    assert e.value.status == ig.IG_E_INVAL


# --------------------------------------------------- invalid and degenerate
def test_invalid_codes_and_labels():
    nb = np.array([3, 3], np.uint16)
    say("invalid inputs")
    with pytest.raises(ig.IGError) as e:
        ig.fit(np.array([[0, 3], [1, 1]], np.uint16), np.array([0, 1], np.uint8), nb)
    assert e.value.status == ig.IG_E_INVAL
    with pytest.raises(ig.IGError) as e:
        ig.fit(np.array([[0, 2], [1, 1]], np.uint16), np.array([0, 2], np.uint8), nb)
    assert e.value.status == ig.IG_E_INVAL
    m = ig.fit(np.array([[0, 2], [1, 1], [0, 1]], np.uint16), np.array([0, 1, 0], np.uint8), nb)
    A, N = gpu_scores(m, np.array([[0, 2], [0, 7], [9, 0]], np.uint16))
    assert A[1] == -1 and N[1] == -1 and A[2] == -1 and N[2] == -1
    assert N[0] > 0


def test_degenerate_sizes():
    nb = np.array([2, 3, 4], np.uint16)
    say("degenerate sizes")
    # no records at all
    m = ig.fit(np.zeros((0, 3), np.uint16), np.zeros(0, np.uint8), nb)
    assert m.n_patterns() == (0, 0)
    A, N = gpu_scores(m, np.array([[0, 0, 0]], np.uint16))
    assert A[0] == 0 and N[0] == 0
    for codes, labels in [
        (np.array([[1, 2, 3]]), np.array([1])),                        # one record
        (np.array([[1, 2, 3], [1, 2, 3], [0, 0, 0]]), np.array([0, 0, 0])),   # one class only
        (np.array([[1, 2, 3], [1, 2, 3]]), np.array([0, 1])),         # contradiction
        (np.array([[0, 0, 0], [1, 1, 1], [0, 1, 2], [1, 0, 3]]), np.array([0, 0, 1, 1])),  # empty pair ANDs
    ]:
        codes = codes.astype(np.uint16)
        labels = labels.astype(np.uint8)
        om = oracle.fit(codes, labels, nb)
        m = ig.fit(codes, labels, nb, kernels="valu")
        assert_same_model(m, om, om.K)
        assert_same_stats(m, om)
        assert_same_model(ig.fit(codes, labels, nb), om, om.K)


def test_scores_do_not_depend_on_batching():
    w = synth.make_tiny(0)
    say("score batching")
    m = ig.fit(w.codes, w.labels, w.nbins)
    A, N = gpu_scores(m, w.test_codes)
    rng = np.random.default_rng(3)
    at = 0
    while at < w.test_codes.shape[0]:
        k = int(rng.integers(1, 70))
        a, n = gpu_scores(m, w.test_codes[at:at + k])
        assert np.array_equal(a, A[at:at + k]) and np.array_equal(n, N[at:at + k])
        at += k


def test_binding_calls_on_a_non_current_stream():
    """Calls on a stream other than torch's current one, with host inputs and with
    device inputs that the binding converts: the conversions run on the call's
    stream after it waits for the caller's stream (here kept busy, so that an
    unordered read would see an unfinished copy), and the temporaries are not
    reused while the call runs.  Results equal those of the default path."""
    import torch
    w = synth.make_tiny(0)
    say("non-current stream")
    m = ig.fit(w.codes, w.labels, w.nbins)
    A, N = gpu_scores(m, w.test_codes)
    s = torch.cuda.Stream()
    outs = []
    for rep in range(3):
        torch.cuda._sleep(20_000_000)                            # the caller's stream is busy
        d64 = torch.from_numpy(w.test_codes.astype(np.int64)).cuda()   # queued behind it
        outs.append(ig.score(m, d64, stream=s))                 # converted to int16 on s
        del d64
        outs.append(ig.score(m, w.test_codes, stream=s))        # host flows
        junk = torch.full((1 << 22,), -1, dtype=torch.int64, device="cuda")   # reuse pressure
        del junk
    s.synchronize()
    for o in outs:
        o = o.cpu().numpy()
        assert np.array_equal(o[:, 0], A) and np.array_equal(o[:, 1], N)
    torch.cuda._sleep(20_000_000)
    dcodes = torch.from_numpy(w.codes.astype(np.int64)).cuda()
    m2 = ig.fit(dcodes, w.labels, w.nbins, stream=s)
    om = oracle.fit(w.codes, w.labels, w.nbins)
    assert_same_model(m2, om, om.K)


def test_scoring_shapes_beyond_the_launch_cache():
    """Scoring launches of 20 flow-block counts, then the same in reverse: the
    launcher keeps its last 16 range choices, so the sequence both evicts and
    reuses them.  Every slice equals the matching rows of one launch over all
    flows, and a sample of those equals the oracle."""
    p = synth.make_random_problem(11, 170, 41, bins_lo=10, bins_hi=14, attack_frac=0.55)
    say("scoring shapes", p.codes.shape)
    m = ig.fit(p.codes, p.labels, p.nbins, kernels="mfma")
    assert m.score_on_matrix_cores
    rng = np.random.default_rng(5)
    sizes = [256 * k - 7 * k for k in range(1, 21)]   # k flow blocks of 256 flows
    flows = np.stack([rng.integers(0, b, sum(sizes)) for b in p.nbins], 1).astype(np.uint16)
    flows[: p.codes.shape[0]] = p.codes             # records score non-zero
    A, N = gpu_scores(m, flows)
    pick = np.concatenate([np.arange(p.codes.shape[0]), rng.choice(flows.shape[0], 400, replace=False)])
    om = oracle.fit(p.codes, p.labels, p.nbins)
    oA, oN = oracle.score(om, flows[pick], p.nbins)
    assert np.array_equal(A[pick], oA) and np.array_equal(N[pick], oN)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    for k in list(range(20)) + list(range(19, -1, -1)):
        a, n = gpu_scores(m, flows[starts[k]:starts[k + 1]])
        assert np.array_equal(a, A[starts[k]:starts[k + 1]]) and np.array_equal(n, N[starts[k]:starts[k + 1]]), k


# ----------------------------------------------------- full-size workloads
def _model_digest(m):
    h = hashlib.sha256()
    for c in (0, 1):
        w, f, S = m.export(c)
        h.update(np.ascontiguousarray(w, dtype="<u8").tobytes())
        h.update(np.ascontiguousarray(f, dtype="<u4").tobytes())
        h.update(np.ascontiguousarray(S, dtype="<i8").tobytes())
    return h.hexdigest()


def test_15k_workload_matches_oracle_digest():
    g = json.load(open(os.path.join(GOLD, "mixture41_15k.json")))
    w = synth.make_15k()
    say("15k workload", w.codes.shape, w.test_codes.shape)
    m = ig.fit(w.codes, w.labels, w.nbins, kernels="valu")
    assert list(m.stats().tests) == g["stats"]["tests"]
    assert _model_digest(m) == g["model_sha256"]
    del m
    m = ig.fit(w.codes, w.labels, w.nbins)   # the configuration the benchmark times
    st = m.stats()
    assert list(st.pairs) == g["stats"]["pairs"]
    assert list(st.distinct) == g["stats"]["distinct"]
    assert list(st.coherent) == g["stats"]["coherent"]
    assert _model_digest(m) == g["model_sha256"]
    assert m.info().flags & ig.IG_MODEL_FIT_BUCKETS
    md = ig.fit(w.codes, w.labels, w.nbins, dense=True)   # every candidate against every record
    assert not md.info().flags & ig.IG_MODEL_FIT_BUCKETS and _model_digest(md) == g["model_sha256"]
    del md
    A, N = gpu_scores(m, w.test_codes)
    assert A[:16].tolist() == g["scores_head"]["A"] and N[:16].tolist() == g["scores_head"]["N"]
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(A, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(N, dtype="<i8").tobytes())
    assert h.hexdigest() == g["scores_sha256"]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kernels", ["auto", "mfma_onehot", "valu"])
def test_148k_workload_matches_oracle_digest(kernels):
    """The 148k workload (14.8k training records, 133,200 flows) at full output:
    both pattern sets with f and S, and the scores of every held-out flow, against
    the oracle's stored digests."""
    g = json.load(open(os.path.join(GOLD, "mixture41_148k.json")))
    w = synth.make_148k()
    say("148k workload", kernels, w.codes.shape, w.test_codes.shape)
    m = ig.fit(w.codes, w.labels, w.nbins, kernels=kernels)
    st = m.stats()
    assert list(st.pairs) == g["stats"]["pairs"]
    assert list(st.distinct) == g["stats"]["distinct"]
    assert list(st.coherent) == g["stats"]["coherent"]
    if kernels == "valu":
        assert list(st.tests) == g["stats"]["tests"]
    assert _model_digest(m) == g["model_sha256"]
    if kernels != "auto":
        return
    A, N = gpu_scores(m, w.test_codes)
    assert A[:16].tolist() == g["scores_head"]["A"] and N[:16].tolist() == g["scores_head"]["N"]
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(A, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(N, dtype="<i8").tobytes())
    assert h.hexdigest() == g["scores_sha256"]


def _check_structure(m, nbins):
    """Properties of any fitted model: strictly ascending rows, S = f |b|^2,
    f >= 1, one token per feature block."""
    off = np.concatenate([[0], np.cumsum(nbins.astype(np.int64))])
    for c in (0, 1):
        w, f, S = m.export(c)
        if w.shape[0] == 0:
            continue
        # strictly ascending in (w_0, ..., w_{K-1})
        a, b = w[:-1], w[1:]
        lt = np.zeros(a.shape[0], bool)
        eq = np.ones(a.shape[0], bool)
        for k in range(w.shape[1]):
            lt |= eq & (a[:, k] < b[:, k])
            eq &= a[:, k] == b[:, k]
        assert lt.all(), "rows not strictly ascending"
        bits = np.unpackbits(w.view(np.uint8), axis=1, bitorder="little")
        pc = bits.sum(axis=1).astype(np.int64)
        assert (f >= 1).all() and np.array_equal(S, f.astype(np.int64) * pc * pc)
        # at most one token inside each feature's block
        blk = np.add.reduceat(bits[:, : off[-1]], off[:-1], axis=1)
        assert blk.max() <= 1


def test_148k_workload_sampled():
    w = synth.make_148k()
    say("148k workload", w.codes.shape, w.test_codes.shape)
    m = ig.fit(w.codes, w.labels, w.nbins)
    _check_structure(m, w.nbins)
    rng = np.random.default_rng(148)
    for c in (0, 1):
        words, f, S = m.export(c)
        rows = {tuple(r): (int(ff), int(ss)) for r, ff, ss in zip(words.tolist(), f.tolist(), S.tolist())}
        nc = int((w.labels == c).sum())
        pi = rng.integers(0, nc, size=96).astype(np.uint64)
        pj = rng.integers(0, nc, size=96).astype(np.uint64)
        pj[:8] = pi[:8]   # record signatures too
        ow, coh, of, _ = oracle.pair_facts(w.codes, w.labels, w.nbins, c, pi, pj)
        for q in range(pi.size):
            key = tuple(int(x) for x in ow[q])
            if coh[q]:
                assert key in rows, f"class {c}: coherent pair ({pi[q]},{pj[q]}) missing"
                assert rows[key][0] == int(of[q])
            else:
                assert key not in rows, f"class {c}: incoherent pair ({pi[q]},{pj[q]}) present"
    idx = rng.choice(w.test_codes.shape[0], size=12, replace=False)
    flows = w.test_codes[idx]
    A, N = gpu_scores(m, flows)
    oA, oN = oracle.score_direct(w.codes, w.labels, w.nbins, flows)
    assert np.array_equal(A, oA) and np.array_equal(N, oN)


# ------------------------------------------- coherence on the matrix cores
MFMA_CASES = [c for c in CASES if c[0] in (1, 2, 4, 6, 7, 8, 9, 10, 11, 18, 19)]   # K <= 8
# factored operands of 6 .. 13 words for one-hot widths K = 10 .. 38 (16 words at most)
WIDE_CASES = [c for c in CASES if c[0] in (12, 13, 14, 15, 16)]
MFMA_RUNS = ([(c, k) for c in MFMA_CASES for k in ("mfma", "mfma_onehot")] +
             [(c, "mfma") for c in WIDE_CASES] + [(CASES[11], "mfma_onehot"), (CASES[12], "mfma_onehot")])


# storage width above K (K = 9, 11, 13, 15 are held in 10, 12, 14, 16 words): the
# factoring walks every storage word, including the padding ones
PADDED_CASES = [(32, 60, 32, 14, 18, 0.5), (30, 60, 41, 14, 18, 0.5), (30, 60, 50, 14, 18, 0.5),
                (32, 60, 56, 14, 18, 0.5)]
MFMA_RUNS += [(c, k) for c in PADDED_CASES for k in ("mfma", "mfma_onehot")]
# one-hot storage of 20 (K = 17, padded), 24 and 28 words, factored into 6 to 9 words
WIDE_STORAGE_CASES = [(35, 80, 70, 14, 16, 0.5), (33, 80, 80, 16, 19, 0.5), (34, 80, 80, 20, 23, 0.5)]
MFMA_RUNS += [(c, "mfma") for c in WIDE_STORAGE_CASES]
# factored tokens with presence tokens, and the ternary bit tokens, each forced
MFMA_RUNS += [(c, k) for c in MFMA_CASES + WIDE_CASES + PADDED_CASES + WIDE_STORAGE_CASES
              for k in ("mfma_presence", "mfma_ternary")]


@pytest.mark.parametrize("case,kernels", MFMA_RUNS, ids=[f"s{c[0]}-d{c[2]}-{k}" for c, k in MFMA_RUNS])
def test_matrix_core_coherence_matches_oracle(case, kernels):
    seed, n, d, blo, bhi, af = case
    p = synth.make_random_problem(seed, n, d, bins_lo=blo, bins_hi=bhi, attack_frac=af)
    say("mfma coherence", case, kernels)
    om = oracle.fit(p.codes, p.labels, p.nbins)
    m = ig.fit(p.codes, p.labels, p.nbins, kernels=kernels)
    assert_same_model(m, om, om.K)
    st = m.stats()
    assert list(st.coherent) == om.stats["coherent"] and list(st.distinct) == om.stats["distinct"]
    info = m.info()
    for c in (0, 1):   # dense: every candidate against every other-class record
        dense = om.stats["distinct"][c] * om.stats["n_class"][1 - c]
        if info.flags & ig.IG_MODEL_FIT_BUCKETS:
            assert 0 < st.tests[c] <= dense or dense == 0
        else:
            assert st.tests[c] == dense
    assert info.mfma_tokens <= 64 * info.mfma_words
    if info.flags & ig.IG_MODEL_FACTORED:
        assert info.mfma_words < om.K and info.mfma_tokens < p.L
    flows = synth.make_random_problem(seed + 2000, 61, d, bins_lo=blo, bins_hi=bhi).codes
    flows = np.minimum(flows, p.nbins[None, :] - 1).astype(np.uint16)
    bad = np.zeros(len(flows), bool)
    bad[::7] = True
    flows[bad, 0] = p.nbins[0]   # a code out of range: (-1, -1)
    A, N = gpu_scores(m, flows)
    assert np.all(A[bad] == -1) and np.all(N[bad] == -1)
    oA, oN = oracle.score(om, flows[~bad], p.nbins)
    assert np.array_equal(A[~bad], oA) and np.array_equal(N[~bad], oN)


@pytest.mark.parametrize("kernels", ["mfma", "mfma_presence", "mfma_ternary"])
def test_factored_patterns_without_tokens(kernels):
    """A pattern of one-bin features only has no factored tokens: its support must
    not count the padding rows of the last record tile, and an invalid flow must
    keep its (-1, -1) although such a pattern meets every operand with zero."""
    say("token-free factored patterns", kernels)
    rng = np.random.default_rng(11)
    nb = np.array([1, 70, 2], np.uint16)   # 73 one-hot tokens in 2 words; factored, 1 word
    n = 40                                  # the last record tile holds 8 of 32 rows
    codes = np.stack([np.zeros(n, np.int64), rng.integers(0, 70, n), rng.integers(0, 2, n)], 1).astype(np.uint16)
    labels = np.zeros(n, np.uint8)          # one class: every candidate is coherent
    om = oracle.fit(codes, labels, nb)
    m = ig.fit(codes, labels, nb, kernels=kernels)
    info = m.info()
    assert info.flags & ig.IG_MODEL_FACTORED and m.score_on_matrix_cores
    assert_same_model(m, om, om.K)
    flows = np.array([[0, 5, 1], [0, 69, 0], [0, 70, 0], [0, 3, 2], [0, 12, 1]], np.uint16)
    bad = np.array([False, False, True, True, False])
    A, N = gpu_scores(m, flows)
    assert np.all(A[bad] == -1) and np.all(N[bad] == -1)
    oA, oN = oracle.score(om, flows[~bad], nb)
    assert np.array_equal(A[~bad], oA) and np.array_equal(N[~bad], oN)


def _bias_span_problem():
    """Class 0 holds a zero row and, for every t = 0 .. T (T = 140 bit tokens), a row
    that agrees with it on features worth exactly t bit tokens and differs on all
    others, so the candidates of the ternary contraction take every size |P| from 0
    to T (every quotient and remainder of the bias slots' 1 - |P|).  Class 1: random
    rows and near copies of the zero row, which cover some of the candidates."""
    rng = np.random.default_rng(5)
    nb = np.array([2] * 10 + [4] * 10 + [16] * 10 + [128] * 10, np.uint16)
    bits = np.array([1] * 10 + [2] * 10 + [4] * 10 + [7] * 10)
    T, d = int(bits.sum()), len(nb)
    order = np.argsort(-bits, kind="stable")
    rows = [np.zeros(d, np.int64)]
    for t in range(T + 1):
        keep, left = np.zeros(d, bool), t
        for f in order:
            if bits[f] <= left:
                keep[f], left = True, left - bits[f]
        assert left == 0
        r = rng.integers(1, nb.astype(np.int64))
        r[keep] = 0
        rows.append(r)
    near = np.zeros((20, d), np.int64)
    for i in range(20):
        fl = rng.choice(d, size=1 + i % 3, replace=False)
        near[i, fl] = rng.integers(1, nb[fl].astype(np.int64))
    codes = np.concatenate([np.array(rows), rng.integers(0, nb.astype(np.int64), size=(20, d)), near])
    labels = np.concatenate([np.zeros(len(rows)), np.ones(40)]).astype(np.uint8)
    return codes.astype(np.uint16), labels, nb, T


@pytest.mark.parametrize("kernels", ["mfma", "mfma_presence", "mfma_ternary"])
def test_ternary_bias_spans_every_candidate_size(kernels):
    codes, labels, nb, T = _bias_span_problem()
    say("ternary bias span", kernels, T)
    om = oracle.fit(codes, labels, nb)
    m = ig.fit(codes, labels, nb, kernels=kernels)
    info = m.info()
    if kernels == "mfma_ternary":
        slots = 3 + (T - 1) // 36
        assert info.fit_tokens == T and info.fit_words == (T + slots + 63) // 64
    assert_same_model(m, om, om.K)
    st = m.stats()
    assert list(st.coherent) == om.stats["coherent"] and list(st.distinct) == om.stats["distinct"]
    assert 0 < om.stats["coherent"][0] < om.stats["distinct"][0]   # some candidates are covered


def _bucket_tests(codes, labels, nbins, om):
    """The subset tests of the token-bucketed contractions, from their definition:
    each distinct candidate of class c (Eq. 1: the records and the non-empty pair
    intersections) meets the other class's records that hold its token held by the
    fewest of them (the lowest such token on ties); each pattern of class c meets
    its own class's records that hold its token held by the fewest of those."""
    nb = nbins.astype(np.int64)
    off = np.concatenate([[0], np.cumsum(nb)[:-1]])
    L = int(nb.sum())
    tok = codes.astype(np.int64) + off
    coh, sup = [], []
    for c in (0, 1):
        Xc, Xo = tok[labels == c], tok[labels != c]
        cnt_o = np.bincount(Xo.ravel(), minlength=L)
        cnt_c = np.bincount(Xc.ravel(), minlength=L)
        cands = {tuple(r) for r in Xc}
        for i in range(len(Xc)):
            eq = Xc[i + 1:] == Xc[i]
            for j in np.nonzero(eq.any(1))[0]:
                cands.add(tuple(Xc[i][eq[j]]))
        coh.append(sum(int(min((cnt_o[t], t) for t in b)[0]) for b in cands))
        words = om.patterns[c]
        total = 0
        for row in words:
            toks = [64 * k + b for k in range(len(row)) for b in range(64) if (int(row[k]) >> b) & 1]
            total += int(min((cnt_c[t], t) for t in toks)[0])
        sup.append(total)
    return coh, sup


# widths where the ternary view takes fewer words than the one-hot words (K >= 3)
BUCKET_CASES = [c for c in CASES if c[0] in (8, 9, 10, 11, 12, 13)]


@pytest.mark.parametrize("case", BUCKET_CASES, ids=[f"s{c[0]}-n{c[1]}-d{c[2]}" for c in BUCKET_CASES])
def test_fit_token_buckets_match_dense_and_oracle(case):
    """The bucketed coherence and support contractions (ternary tokens) give the
    dense ones' model, the oracle's, and test exactly the pairs of each candidate
    with the records of its bucket."""
    seed, n, d, blo, bhi, af = case
    p = synth.make_random_problem(seed, n, d, bins_lo=blo, bins_hi=bhi, attack_frac=af)
    say("fit buckets", case)
    om = oracle.fit(p.codes, p.labels, p.nbins)
    mb = ig.fit(p.codes, p.labels, p.nbins, kernels="mfma_ternary")
    md = ig.fit(p.codes, p.labels, p.nbins, kernels="mfma_ternary", dense=True)
    ib, idn = mb.info(), md.info()
    assert ib.flags & ig.IG_MODEL_FIT_BUCKETS and not idn.flags & ig.IG_MODEL_FIT_BUCKETS
    assert_same_model(mb, om, om.K)
    assert_same_model(md, om, om.K)
    coh, sup = _bucket_tests(p.codes, p.labels, p.nbins, om)
    sb, sd = mb.stats(), md.stats()
    assert list(sb.tests) == coh and list(sb.support_tests) == sup
    assert list(sd.tests) == [om.stats["distinct"][c] * om.stats["n_class"][1 - c] for c in (0, 1)]
    assert list(sd.support_tests) == [om.stats["coherent"][c] * om.stats["n_class"][c] for c in (0, 1)]


def _boundary_codes(rng, nb, n):
    """Codes that reach each feature's extreme bin indices: 0, nb - 1, every
    all-ones index 2^k - 1 below nb and its neighbours, plus a few random bins,
    so the bin popcounts span 0 up to ceil(log2 nb)."""
    cols = []
    for b in nb:
        b = int(b)
        vals = {0, b - 1}
        k = 1
        while (1 << k) - 1 < b:
            vals.update(v for v in ((1 << k) - 1, (1 << k) - 2, 1 << k) if 0 <= v < b)
            k += 1
        vals.update(int(v) for v in rng.integers(0, b, 3))
        vals = np.array(sorted(vals))
        cols.append(vals[rng.integers(0, len(vals), n)])
    return np.stack(cols, 1).astype(np.uint16)


@pytest.mark.parametrize("kernels", ["mfma", "mfma_presence", "mfma_ternary"])
@pytest.mark.parametrize("nb,n", [
    ([2, 3, 9, 16, 17, 33, 65, 513], 90),   # 1 to 4 bit tokens with one presence token, 5 to 10 with two
    ([1024], 120),                           # bin 1023: 10 bits set, presence parts 6 + 4
])
def test_factored_bin_boundaries(nb, n, kernels):
    """Features whose bin counts sit at the factored encoding's boundaries, with
    bins of every popcount up to the feature's bit count: model and scores on the
    matrix cores against the oracle, including flows one bit away from a pattern."""
    nb = np.array(nb, np.uint16)
    say("factored bin boundaries", list(nb))
    rng = np.random.default_rng(int(nb.sum()))
    codes = _boundary_codes(rng, nb, n)
    labels = (rng.random(n) < 0.5).astype(np.uint8)
    om = oracle.fit(codes, labels, nb)
    m = ig.fit(codes, labels, nb, kernels=kernels)
    info = m.info()
    assert info.flags & ig.IG_MODEL_FACTORED and m.score_on_matrix_cores
    assert_same_model(m, om, om.K)
    st = m.stats()
    for key in ("pairs", "distinct", "coherent", "n_class"):
        assert list(getattr(st, key)) == om.stats[key], key
    if info.flags & ig.IG_MODEL_FIT_BUCKETS:
        # each candidate against the other-class records of its token bucket
        coh, sup = _bucket_tests(codes, labels, nb, om)
        assert list(st.tests) == coh and list(st.support_tests) == sup
    else:
        # every distinct candidate against every other-class record
        assert list(st.tests) == [om.stats["distinct"][c] * om.stats["n_class"][1 - c] for c in (0, 1)]
    flows = _boundary_codes(rng, nb, 300)
    near = flows.copy()   # one bin bit flipped where the result stays a valid bin
    for j, b in enumerate(nb):
        flip = near[:, j] ^ (1 << rng.integers(0, max(int(b - 1).bit_length(), 1), len(near)))
        near[:, j] = np.where(flip < b, flip, near[:, j])
    flows = np.concatenate([flows, near, codes])
    A, N = gpu_scores(m, flows)
    oA, oN = oracle.score(om, flows, nb)
    assert np.array_equal(A, oA) and np.array_equal(N, oN)


def test_matrix_core_coherence_15k_digest():
    g = json.load(open(os.path.join(GOLD, "mixture41_15k.json")))
    w = synth.make_15k()
    say("mfma coherence 15k")
    m = ig.fit(w.codes, w.labels, w.nbins, kernels="mfma")
    assert list(m.stats().coherent) == g["stats"]["coherent"]
    assert _model_digest(m) == g["model_sha256"]
