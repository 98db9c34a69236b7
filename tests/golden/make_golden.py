"""Write the oracle's expected values for the 15k workload (calls oracle/ only).

Usage: python tests/golden/make_golden.py  ->  tests/golden/mixture41_15k.json
The digests cover the sorted pattern words, supports and weights of both classes
and the (A, N) scores of the held-out flows, all as little-endian bytes.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2507_14222_amd import synth  # noqa: E402


def model_digest(words, f, S) -> str:
    h = hashlib.sha256()
    for c in (0, 1):
        h.update(np.ascontiguousarray(words[c], dtype="<u8").tobytes())
        h.update(np.ascontiguousarray(f[c], dtype="<u4").tobytes())
        h.update(np.ascontiguousarray(S[c], dtype="<i8").tobytes())
    return h.hexdigest()


def score_digest(A, N) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(A, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(N, dtype="<i8").tobytes())
    return h.hexdigest()


def main():
    w = synth.make_15k()
    t0 = time.time()
    m = oracle.fit(w.codes, w.labels, w.nbins)
    t1 = time.time()
    A, N = oracle.score(m, w.test_codes, w.nbins)
    t2 = time.time()
    out = {
        "_source": "oracle/ (C oracle) on paper_2507_14222_amd.synth.make_15k(); written by tests/golden/make_golden.py",
        "workload": w.name,
        "n_train": int(w.n), "n_test": int(w.test_codes.shape[0]),
        "stats": m.stats,
        "model_sha256": model_digest(m.patterns, m.f, m.S),
        "scores_sha256": score_digest(A, N),
        "scores_head": {"A": A[:16].tolist(), "N": N[:16].tolist()},
        "oracle_seconds": {"fit": round(t1 - t0, 2), "score": round(t2 - t1, 2),
                           "threads": oracle.max_threads()},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mixture41_15k.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
