"""The classifier and detection metrics on the device (ig_normal_moments,
ig_classify, ig_detection_metrics; Section 3.1 Regulations 1-3, Table 2) against
the oracle's exact integer/fraction implementation: moments equal, labels and
deciding rules equal flow by flow, confusion counts and the AUC fraction equal."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import regulations as R
from paper_2507_14222_amd import ig, synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")
R_TABLE2 = 0.568


def say(*a):
    print("[regulate]", *a, flush=True)
    sys.stdout.flush()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def check_against_oracle(scores, train_scores, train_labels, truth, r):
    """moments, threshold, labels, rules and metrics against the oracle"""
    mo = ig.normal_moments(train_scores, train_labels)
    tN = train_scores[:, 1].tolist()
    st = R.normal_stats(tN, train_labels.tolist())
    assert (int(mo.count), mo.total, mo.total_sq) == (st.count, st.total, st.total_sq)
    T = ig.r3_threshold(mo, r)
    lab, rule = ig.classify(scores, T)
    lab, rule = host(lab), host(rule)
    A, N = scores[:, 0].tolist(), scores[:, 1].tolist()
    olab, orule = R.classify(A, N, st, r)
    assert lab.tolist() == olab and rule.tolist() == orule
    mt = ig.detection_metrics(scores, lab, truth)
    om = R.metrics(olab, truth.tolist(), A, N)
    assert (int(mt.tp), int(mt.fp), int(mt.tn), int(mt.fn)) == (om.tp, om.fp, om.tn, om.fn)
    assert (int(mt.auc_num), int(mt.auc_den)) == (om.auc_num, om.auc_den)
    assert int(mt.invalid) == 0
    return mt


def test_worked_example_flows():
    g = json.load(open(GOLD))
    m = ig.fit(np.array(g["codes"], np.uint16), np.array(g["labels"], np.uint8), np.array(g["nbins"], np.uint16))
    out = host(ig.score(m, np.array(g["flows"], np.uint16)))
    lab, rule = ig.classify(out)
    assert host(lab).tolist() == [0, 1, 1, 0]
    assert host(rule).tolist() == [R.R1, R.R1, R.R2, R.R1]
    lab, rule = ig.classify(out, use_r2=False)
    assert host(rule).tolist() == [R.R1, R.R1, R.R1, R.R1]


def test_tiny_workload_split():
    w = synth.make_tiny(0)
    m = ig.fit(w.codes, w.labels, w.nbins)
    say("tiny", w.codes.shape, w.test_codes.shape)
    tr = host(ig.score(m, w.codes))
    te = host(ig.score(m, w.test_codes))
    for r in (0.0, R_TABLE2, 1.0, 3.0):
        check_against_oracle(te, tr, w.labels, w.test_labels, r)


def test_15k_workload_split():
    w = synth.make_15k()
    m = ig.fit(w.codes, w.labels, w.nbins)
    say("15k", w.codes.shape, w.test_codes.shape)
    tr = host(ig.score(m, w.codes))
    te = host(ig.score(m, w.test_codes))
    mt = check_against_oracle(te, tr, w.labels, w.test_labels, R_TABLE2)
    say("15k metrics", mt.as_dict())


def test_threshold_boundary_scores():
    """Normal-record N values chosen so that mu_N - r sigma_N falls on and next to
    integers; flows with N on each side of the cut."""
    rng = np.random.default_rng(5)
    train_N = np.array([2, 4, 4, 4, 5, 5, 7, 9] * 3, np.int64)   # mu 5, sigma 2
    tr = np.stack([np.zeros_like(train_N), train_N], 1)
    labels = np.zeros(train_N.size, np.uint8)
    N = np.arange(0, 12, dtype=np.int64).repeat(3)
    A = np.concatenate([np.zeros(12, np.int64), N[12:24] - 1, rng.integers(0, 12, 12)])
    te = np.stack([A[: N.size], N], 1)
    truth = rng.integers(0, 2, N.size).astype(np.uint8)
    for r in (0.5, 1.0, 1.5, 2.0, 2.5, R_TABLE2):
        check_against_oracle(te, tr, labels, truth, r)


def test_invalid_scores_and_bad_truth():
    sc = np.array([[-1, -1], [3, 1], [0, 4], [-1, -1]], np.int64)
    lab, rule = ig.classify(sc, 2)
    assert host(lab).tolist() == [255, 1, 0, 255] and host(rule).tolist() == [0, 1, 1, 0]
    mt = ig.detection_metrics(sc, host(lab), np.array([1, 1, 0, 0], np.uint8))
    assert (int(mt.tp), int(mt.tn), int(mt.invalid)) == (1, 1, 2)
    assert (int(mt.auc_num), int(mt.auc_den)) == (2, 2)
    with pytest.raises(ig.IGError) as e:
        ig.detection_metrics(sc, host(lab), np.array([1, 2, 0, 0], np.uint8))
    assert e.value.status == ig.IG_E_INVAL
    with pytest.raises(ig.IGError) as e:
        ig.normal_moments(sc, np.array([0, 3, 0, 0], np.uint8))
    assert e.value.status == ig.IG_E_INVAL
