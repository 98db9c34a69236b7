"""Autotuner for the launch shapes of libig's fit kernels.

Two families of shapes are tuned.  The VALU coherence and support kernels (the
path for operands wider than the matrix-core kernels take): for each storage
width KS and problem-size bucket a seeded synthetic problem of that width and
size is fitted with every candidate shape (coherence: candidates per lane x
workgroups per CU; support: patterns per lane), timed by the library's own event
pairs.  The matrix-core contractions: for each operand width (factored words)
and size bucket, the 32-column sets per wave of the coherence and the support
contraction, timed by the library's event pairs around those launches
(ig_stats.kernel_ms).  The result is a table of ig_tune_entry rows, cached as
JSON and passed to ig_fit / ig_fit_batch.  Tuning never changes results.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, List, Optional

import numpy as np

from . import ig, synth

COHERENCE_SHAPES = [(cpl, g) for cpl in (1, 2) for g in (4, 8, 16)]
SUPPORT_CPL = (1, 2)


def _problem_for(ks: int, n: int, seed: int) -> synth.Problem:
    """A Dirichlet(0.5) problem whose token universe needs exactly `ks` storage words."""
    rng = np.random.default_rng(seed)
    target_L = max(2, 64 * ks - 32)            # inside the width bucket
    d = int(np.clip(target_L // 16, 2, 80))
    nbins = np.full(d, target_L // d)
    nbins[: target_L - int(nbins.sum())] += 1
    return synth.make_problem(rng, n, d, nbins.astype(np.int64), 0.5)


def _time(p, tune, reps: int):
    best_c = best_s = float("inf")
    for _ in range(reps):
        m = ig.fit(p.codes, p.labels, p.nbins, tune=tune, kernels="valu")
        st = m.stats()
        best_c = min(best_c, st.ms[4])
        best_s = min(best_s, st.ms[6])
        m.free()
    return best_c, best_s


def autotune(widths: Iterable[int], sizes=(1200, 5000), reps: int = 2, seed: int = 7) -> Dict:
    """Measure every shape on each (width, size) bucket; returns the table and the timings."""
    entries: List[Dict] = []
    measured = []
    for ks in sorted(set(int(w) for w in widths)):
        for n in sizes:
            p = _problem_for(ks, n, seed + ks * 1000 + n)
            n1 = int(p.labels.sum())
            n0 = p.n - n1
            pairs = n0 * (n0 - 1) // 2 + n1 * (n1 - 1) // 2
            rows = []
            for cpl, g in COHERENCE_SHAPES:
                for scpl in SUPPORT_CPL:
                    t = [{"ks": ks, "min_pairs": 0, "filter_cpl": cpl, "grid_per_cu": g, "support_cpl": scpl}]
                    c_ms, s_ms = _time(p, t, reps)
                    rows.append((cpl, g, scpl, c_ms, s_ms))
            best_coh = min(rows, key=lambda r: r[3])
            best_sup = min(rows, key=lambda r: r[4])
            lo = 0 if n == min(sizes) else pairs
            entries.append({"ks": ks, "min_pairs": int(lo), "filter_cpl": best_coh[0],
                            "grid_per_cu": best_coh[1], "support_cpl": best_sup[2]})
            measured.append({"ks": ks, "n": n, "pairs": int(pairs),
                             "shapes": [dict(zip(("filter_cpl", "grid_per_cu", "support_cpl", "coherence_ms",
                                                  "support_ms"), r)) for r in rows]})
    return {"arch": "gfx950", "entries": entries, "measured": measured}


MFMA_SETS = (1, 2, 3)


def _problem_for_words(ko: int, n: int, seed: int) -> synth.Problem:
    """A Dirichlet(0.5) problem whose factored operands take `ko` words: features
    of 8 bins take 3 bit tokens and 1 presence token, so 16 ko - 4 of them fill
    ko words but the last few tokens."""
    rng = np.random.default_rng(seed)
    d = max(2, 16 * ko - 4)
    return synth.make_problem(rng, n, d, np.full(d, 8, np.int64), 0.5)


def _time_mfma(p, tune, reps: int):
    best_c = best_s = float("inf")
    for _ in range(reps):
        m = ig.fit(p.codes, p.labels, p.nbins, tune=tune)
        st = m.stats()
        best_c = min(best_c, st.kernel_ms[0])
        best_s = min(best_s, st.kernel_ms[1])
        m.free()
    return best_c, best_s


def autotune_mfma(words: Iterable[int], sizes=(1500, 6000), reps: int = 2, seed: int = 11) -> Dict:
    """Column sets per wave of the matrix-core coherence and support contractions,
    per operand width and size bucket."""
    entries: List[Dict] = []
    measured = []
    for ko in sorted(set(int(w) for w in words)):
        for n in sizes:
            p = _problem_for_words(ko, n, seed + ko * 1000 + n)
            n1 = int(p.labels.sum())
            n0 = p.n - n1
            pairs = n0 * (n0 - 1) // 2 + n1 * (n1 - 1) // 2
            rows = []
            for sets in MFMA_SETS:
                t = [{"mfma_words": ko, "min_pairs": 0, "coherence_sets": sets, "support_sets": sets}]
                c_ms, s_ms = _time_mfma(p, t, reps)
                rows.append((sets, c_ms, s_ms))
            best_c = min(rows, key=lambda r: r[1])
            best_s = min(rows, key=lambda r: r[2])
            lo = 0 if n == min(sizes) else pairs
            entries.append({"ks": 0, "min_pairs": int(lo), "mfma_words": ko,
                            "coherence_sets": best_c[0], "support_sets": best_s[0]})
            measured.append({"mfma_words": ko, "n": n, "pairs": int(pairs),
                             "shapes": [dict(zip(("sets", "coherence_ms", "support_ms"), r)) for r in rows]})
    return {"entries": entries, "measured": measured}


def save(table: Dict, path: str) -> None:
    with open(path, "w") as f:
        json.dump(table, f, indent=1)


def load(path: str) -> Optional[List[Dict]]:
    """Tuning rows from a cache file, or None when there is none."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    return t.get("entries")


def model_bytes_estimate(p) -> int:
    """Upper estimate of the device bytes a fit of problem p holds at once: every
    pair intersection and record of both classes as a candidate row plus its
    12-byte sort entry."""
    n1 = int(np.asarray(p.labels).sum())
    n0 = int(p.n) - n1
    K = ig_storage_words((int(p.L) + 63) // 64)
    return (n0 * (n0 + 1) // 2 + n1 * (n1 + 1) // 2) * (K * 8 + 12)


def slices_by_memory(problems, budget_bytes: float = 90e9) -> List[List[int]]:
    """Consecutive slices of the problem list whose estimated bytes stay within
    the budget (a slice holds at least one problem): the 64 models of the batch
    workload together are larger than device memory, so a caller fits and
    releases them slice by slice."""
    slices, cur, acc = [], [], 0
    for i, p in enumerate(problems):
        b = model_bytes_estimate(p)
        if cur and acc + b > budget_bytes:
            slices.append(cur)
            cur, acc = [], 0
        cur.append(i)
        acc += b
    if cur:
        slices.append(cur)
    return slices


def widths_of(problems) -> List[int]:
    return sorted(set(ig_storage_words((p.L + 63) // 64) for p in problems))


def ig_storage_words(K: int) -> int:
    """The compiled storage width that holds K words (same rule as the library)."""
    for v in (1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 40, 48, 56, 64):
        if K <= v:
            return v
    raise ValueError("K beyond 64")


def main(argv=None) -> None:
    """Tune the VALU-path widths of the batched-fit workload and write the table:
    python -m paper_2507_14222_amd.tune --out paper_2507_14222_amd/tuning_gfx950.json"""
    import argparse
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--sizes", type=int, nargs="+", default=[1200, 5000])
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--mfma-words", type=int, nargs="+", default=list(range(3, 11)),
                    help="operand widths of the matrix-core contractions to tune (the 64-problem "
                         "workload factors into 3 to 10 words)")
    a = ap.parse_args(argv)
    # widths beyond the matrix-core kernels' 8 one-hot words may fall to the VALU path
    widths = [w for w in widths_of(synth.make_batch()) if w > 8]
    table = autotune(widths, sizes=tuple(a.sizes), reps=a.reps)
    print("[tune] VALU rows:", len(table["entries"]), flush=True)
    mf = autotune_mfma(a.mfma_words, reps=a.reps)
    table["entries"] += mf["entries"]
    table["measured_mfma"] = mf["measured"]
    save(table, a.out)
    print(json.dumps({"widths": widths, "entries": table["entries"]}), flush=True)
    sys.stdout.flush()


if __name__ == "__main__":
    main()
