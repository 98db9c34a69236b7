"""Write the oracle's expected values for the full-size workloads (calls oracle/ only).

Usage: python tests/golden/make_golden.py [15k] [148k] [batch]
  15k    -> tests/golden/mixture41_15k.json   fit of the 10.5k training records, 4,500 flows
  148k   -> tests/golden/mixture41_148k.json  fit of the 14.8k training records, all 133,200 flows
  batch  -> tests/golden/batch64_small.json   every problem of the 64-problem workload with
                                              at most 5,000 records

The digests cover the sorted pattern words, supports and weights of both classes
(as little-endian bytes) and the (A, N) scores of the held-out flows.
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

HERE = os.path.dirname(os.path.abspath(__file__))
BATCH_MAX_N = 5000


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


def _write(name, out):
    with open(os.path.join(HERE, name), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1)[:2000], flush=True)


def workload(w, fname):
    t0 = time.time()
    m = oracle.fit(w.codes, w.labels, w.nbins)
    t1 = time.time()
    print(f"[golden] {w.name}: fit {t1 - t0:.1f} s, {m.stats['coherent']} patterns", flush=True)
    # scored in slices so that progress shows; the digest covers every flow in order
    A = np.zeros(w.test_codes.shape[0], np.int64)
    N = np.zeros_like(A)
    step = 4500
    for a in range(0, A.size, step):
        A[a:a + step], N[a:a + step] = oracle.score(m, w.test_codes[a:a + step], w.nbins)
        print(f"[golden] {w.name}: scored {min(a + step, A.size)} / {A.size}", flush=True)
    t2 = time.time()
    _write(fname, {
        "_source": f"oracle/ (C oracle) on paper_2507_14222_amd.synth ({w.name}); "
                   "written by tests/golden/make_golden.py",
        "workload": w.name,
        "n_train": int(w.n), "n_test": int(w.test_codes.shape[0]),
        "stats": m.stats,
        "model_sha256": model_digest(m.patterns, m.f, m.S),
        "scores_sha256": score_digest(A, N),
        "scores_head": {"A": A[:16].tolist(), "N": N[:16].tolist()},
        "oracle_seconds": {"fit": round(t1 - t0, 2), "score": round(t2 - t1, 2),
                           "threads": oracle.max_threads()},
    })


def batch():
    probs = synth.make_batch()
    rows = {}
    for i, p in enumerate(probs):
        if p.n > BATCH_MAX_N:
            continue
        t0 = time.time()
        m = oracle.fit(p.codes, p.labels, p.nbins)
        rows[str(i)] = {"n": p.n, "d": p.d, "L": p.L, "stats": m.stats,
                        "model_sha256": model_digest(m.patterns, m.f, m.S),
                        "oracle_seconds": round(time.time() - t0, 2)}
        print(f"[golden] batch problem {i}: n={p.n} K={(p.L + 63) // 64} {rows[str(i)]['oracle_seconds']} s",
              flush=True)
        del m
    _write("batch64_small.json", {
        "_source": "oracle/ (C oracle) on paper_2507_14222_amd.synth.make_batch(); every problem with at most "
                   f"{BATCH_MAX_N} records; written by tests/golden/make_golden.py",
        "max_n": BATCH_MAX_N, "threads": oracle.max_threads(), "problems": rows,
    })


def main(argv):
    targets = argv or ["15k"]
    for t in targets:
        if t == "15k":
            workload(synth.make_15k(), "mixture41_15k.json")
        elif t == "148k":
            workload(synth.make_148k(), "mixture41_148k.json")
        elif t == "batch":
            batch()
        else:
            raise SystemExit(f"unknown target {t}")


if __name__ == "__main__":
    main(sys.argv[1:])
