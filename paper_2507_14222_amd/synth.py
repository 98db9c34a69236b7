"""Seeded synthetic workloads shaped like the paper's intrusion-detection data.

The paper measures on NSL-KDD, UNSW-NB15 and UKM-IDS20 (Section 4). None of
those datasets is used here: every generator below draws records from seeded
random distributions whose *shapes* follow the workloads the paper describes
(record counts, 41 features with 3/70/11-level categoricals, the 10/90
small-train regime of Table 2).  No dataset record is reproduced.

This module is shared by the CPU oracle's tests and by the HIP path.  It holds
none of the method's arithmetic: it emits per-feature bin codes, labels and bin
counts only.  Packing into bitsets (Eq. 5), intersections, coherence and scores
are computed separately by each side.

Every generator returns a ``Workload``:

* ``codes``  uint16 [n, d]  bin code of every feature (one token per feature)
* ``labels`` uint8  [n]     0 = normal, 1 = attack
* ``nbins``  uint16 [d]     number of bins of each feature
* ``test_codes`` / ``test_labels``  the held-out flows that are scored

The anti-contradiction step of the paper's pipeline (Section 4: records that
carry the same tokens in both classes are removed before training) is done on
code rows: with one token per feature, two records have the same token set
exactly when their code rows are equal.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

ABSENT = 0xFFFF  # code meaning "feature not part of this pattern" (pattern sets only)


@dataclass
class Workload:
    name: str
    codes: np.ndarray
    labels: np.ndarray
    nbins: np.ndarray
    test_codes: np.ndarray
    test_labels: np.ndarray
    meta: Dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.codes.shape[0])

    @property
    def d(self) -> int:
        return int(self.codes.shape[1])

    @property
    def L(self) -> int:
        return int(self.nbins.astype(np.int64).sum())


def drop_contradictions(codes: np.ndarray, labels: np.ndarray) -> np.ndarray:
    """Boolean keep-mask removing every copy of a code row present in both classes."""
    if codes.shape[0] == 0:
        return np.zeros(0, dtype=bool)
    _, inv = np.unique(codes, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    nuniq = int(inv.max()) + 1
    has0 = np.zeros(nuniq, dtype=bool)
    has1 = np.zeros(nuniq, dtype=bool)
    has0[inv[labels == 0]] = True
    has1[inv[labels == 1]] = True
    bad = has0 & has1
    return ~bad[inv]


def _draw_categorical(rng: np.random.Generator, probs: np.ndarray, size: int) -> np.ndarray:
    """Vectorised draws from one categorical distribution."""
    cdf = np.cumsum(probs)
    cdf[-1] = 1.0
    return np.searchsorted(cdf, rng.random(size), side="right").astype(np.int64)


# --------------------------------------------------------------------------
# Tiny workload: 20 one-hot categorical features with 8 bins each.
# --------------------------------------------------------------------------
def make_tiny(seed: int = 0, n_per_class: int = 750, n_train_per_class: int = 600,
              d: int = 20, bins: int = 8, n_shared: int = 5) -> Workload:
    """1,200 training + 300 test records, 20 features x 8 bins (L = 160, K = 3).

    Per class and feature the bin probabilities are Dirichlet(0.5); the first
    ``n_shared`` features use one distribution for both classes.
    """
    rng = np.random.default_rng(seed)
    p = np.empty((2, d, bins))
    for f in range(d):
        if f < n_shared:
            q = rng.dirichlet([0.5] * bins)
            p[0, f] = q
            p[1, f] = q
        else:
            p[0, f] = rng.dirichlet([0.5] * bins)
            p[1, f] = rng.dirichlet([0.5] * bins)
    rows, labs = [], []
    for c in (0, 1):
        cc = np.empty((n_per_class, d), dtype=np.int64)
        for f in range(d):
            cc[:, f] = _draw_categorical(rng, p[c, f], n_per_class)
        rows.append(cc)
        labs.append(np.full(n_per_class, c, dtype=np.uint8))
    codes = np.concatenate(rows)
    labels = np.concatenate(labs)
    keep = drop_contradictions(codes, labels)
    codes, labels = codes[keep], labels[keep]
    tr, te = [], []
    for c in (0, 1):
        idx = np.flatnonzero(labels == c)
        tr.append(idx[:n_train_per_class])
        te.append(idx[n_train_per_class:])
    tr = np.concatenate(tr)
    te = np.concatenate(te)
    tr = tr[rng.permutation(tr.size)]
    return Workload(
        name="tiny-1200",
        codes=codes[tr].astype(np.uint16), labels=labels[tr],
        nbins=np.full(d, bins, dtype=np.uint16),
        test_codes=codes[te].astype(np.uint16), test_labels=labels[te],
        meta={"seed": seed, "d": d, "bins": bins})


# --------------------------------------------------------------------------
# 41-feature mixture generator (15k and 148k workloads, flows of the server).
# --------------------------------------------------------------------------
CAT_LEVELS = (3, 70, 11)
N_NUMERIC = 38
NUM_BINS = 10
N_COMP = 4


def _mixture_params(rng: np.random.Generator) -> List[Dict]:
    """Per-class 4-component mixture parameters; the attack class reuses the
    normal class's parameters on 8 numeric features and on the first
    categorical, and shifts the log-mean of the other numeric features."""
    shared_num = 8
    params = []
    for c in (0, 1):
        w = rng.dirichlet([2.0] * N_COMP)
        cat = [[rng.dirichlet([0.5] * lv) for _ in range(N_COMP)] for lv in CAT_LEVELS]
        mu = rng.normal(0.0, 1.0, size=(N_COMP, N_NUMERIC))
        sig = rng.uniform(0.25, 1.0, size=(N_COMP, N_NUMERIC))
        if c == 1:
            base = params[0]
            cat[0] = [q.copy() for q in base["cat"][0]]
            mu[:, :shared_num] = base["mu"][:, :shared_num]
            sig[:, :shared_num] = base["sig"][:, :shared_num]
            mu[:, shared_num:] = base["mu"][:, shared_num:] + rng.normal(
                0.0, 0.5, size=(N_COMP, N_NUMERIC - shared_num))
            sig[:, shared_num:] = base["sig"][:, shared_num:]
        params.append({"w": w, "cat": cat, "mu": mu, "sig": sig})
    return params


def _mixture_raw(rng: np.random.Generator, params: Dict, n: int):
    comp = _draw_categorical(rng, params["w"], n)
    cats = np.empty((n, len(CAT_LEVELS)), dtype=np.int64)
    for f, lv in enumerate(CAT_LEVELS):
        for k in range(N_COMP):
            sel = np.flatnonzero(comp == k)
            cats[sel, f] = _draw_categorical(rng, params["cat"][f][k], sel.size)
    z = rng.standard_normal((n, N_NUMERIC))
    num = np.exp(params["mu"][comp] + params["sig"][comp] * z)
    return cats, num


def _bin_numeric(num: np.ndarray, edges: np.ndarray) -> np.ndarray:
    out = np.empty(num.shape, dtype=np.int64)
    for f in range(num.shape[1]):
        out[:, f] = np.searchsorted(edges[f], num[:, f], side="right")
    return out


def mixture41_nbins() -> np.ndarray:
    return np.array(list(CAT_LEVELS) + [NUM_BINS] * N_NUMERIC, dtype=np.uint16)


def make_mixture41(seed: int, n: int, normal_frac: float = 0.53,
                   train_frac: float = 0.7, name: Optional[str] = None) -> Workload:
    """41 features: categoricals with 3, 70, 11 levels and 38 log-normal numeric
    features binned at the deciles of all pooled values (L = 464, K = 8)."""
    rng = np.random.default_rng(seed)
    params = _mixture_params(rng)
    n0 = int(round(n * normal_frac))
    n1 = n - n0
    cats0, num0 = _mixture_raw(rng, params[0], n0)
    cats1, num1 = _mixture_raw(rng, params[1], n1)
    num = np.concatenate([num0, num1])
    qs = np.linspace(0.1, 0.9, NUM_BINS - 1)
    edges = np.quantile(num, qs, axis=0).T  # [38, 9]
    codes = np.concatenate([np.concatenate([cats0, cats1]), _bin_numeric(num, edges)], axis=1)
    labels = np.concatenate([np.zeros(n0, np.uint8), np.ones(n1, np.uint8)])
    keep = drop_contradictions(codes, labels)
    codes, labels = codes[keep], labels[keep]
    perm = rng.permutation(codes.shape[0])
    ntr = int(round(train_frac * codes.shape[0]))
    tr, te = perm[:ntr], perm[ntr:]
    return Workload(
        name=name or f"mixture41-{n}",
        codes=codes[tr].astype(np.uint16), labels=labels[tr],
        nbins=mixture41_nbins(),
        test_codes=codes[te].astype(np.uint16), test_labels=labels[te],
        meta={"seed": seed, "n_total": n, "train_frac": train_frac,
              "dropped_contradictions": int((~keep).sum())})


def make_15k(seed: int = 1) -> Workload:
    """15,000 records (53% normal / 47% attack), 70/30 seeded split."""
    return make_mixture41(seed, 15000, train_frac=0.7, name="mixture41-15k")


def make_148k(seed: int = 2) -> Workload:
    """148,000 records, 10/90 train/test split (about 14.8k train, 133k test)."""
    return make_mixture41(seed, 148000, train_frac=0.1, name="mixture41-148k")


# --------------------------------------------------------------------------
# 64 independent problems of uneven size and width (batched fitting).
# --------------------------------------------------------------------------
@dataclass
class Problem:
    codes: np.ndarray
    labels: np.ndarray
    nbins: np.ndarray

    @property
    def n(self) -> int:
        return int(self.codes.shape[0])

    @property
    def d(self) -> int:
        return int(self.codes.shape[1])

    @property
    def L(self) -> int:
        return int(self.nbins.astype(np.int64).sum())


def make_problem(rng: np.random.Generator, n: int, d: int, nbins: np.ndarray,
                 attack_frac: float, shared_frac: float = 0.25) -> Problem:
    """Dirichlet(0.5) categorical records; a quarter of the features share one
    distribution between the classes."""
    n1 = int(round(n * attack_frac))
    n0 = n - n1
    n_shared = int(round(shared_frac * d))
    codes = np.empty((n, d), dtype=np.int64)
    for f in range(d):
        nb = int(nbins[f])
        p0 = rng.dirichlet([0.5] * nb)
        p1 = p0 if f < n_shared else rng.dirichlet([0.5] * nb)
        codes[:n0, f] = _draw_categorical(rng, p0, n0)
        codes[n0:, f] = _draw_categorical(rng, p1, n1)
    labels = np.concatenate([np.zeros(n0, np.uint8), np.ones(n1, np.uint8)])
    keep = drop_contradictions(codes, labels)
    codes, labels = codes[keep], labels[keep]
    perm = rng.permutation(codes.shape[0])
    return Problem(codes[perm].astype(np.uint16), labels[perm], nbins.astype(np.uint16))


def make_batch(seed: int = 3, n_problems: int = 64, n_lo: int = 500, n_hi: int = 20000,
               d_lo: int = 20, d_hi: int = 80, b_lo: int = 4, b_hi: int = 32,
               r_lo: float = 0.2, r_hi: float = 0.8) -> List[Problem]:
    """64 problems: n ~ U{500..20000}, d ~ U{20..80}, bins ~ U{4..32},
    attack ratio ~ U(0.2, 0.8); one child seed per problem."""
    children = np.random.SeedSequence(seed).spawn(n_problems)
    probs = []
    for ss in children:
        rng = np.random.default_rng(ss)
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.integers(d_lo, d_hi + 1))
        nbins = rng.integers(b_lo, b_hi + 1, size=d)
        ratio = float(rng.uniform(r_lo, r_hi))
        probs.append(make_problem(rng, n, d, nbins, ratio))
    return probs


# --------------------------------------------------------------------------
# Served scoring: a large resident pattern set and a Poisson request stream.
# --------------------------------------------------------------------------
@dataclass
class PatternSet:
    """Pattern sets given as code rows; ABSENT marks a feature the pattern does
    not constrain.  ``f`` is the support attached to each pattern."""
    codes: List[np.ndarray]   # per class: uint16 [m, d]
    f: List[np.ndarray]       # per class: uint32 [m]
    nbins: np.ndarray


def make_pattern_set(seed: int = 4, per_class: int = 1_000_000, keep_p: float = 0.15,
                     f_max: int = 8000) -> PatternSet:
    """Per class: take generated records of that class, keep each feature with
    probability ``keep_p`` (at least one), drop repeats, top up to ``per_class``
    distinct patterns, and attach a support drawn uniformly from 1..f_max."""
    rng = np.random.default_rng(seed)
    params = _mixture_params(rng)
    # decile edges from a pooled reference sample, as in the record generator
    c0, n0 = _mixture_raw(rng, params[0], 50000)
    c1, n1 = _mixture_raw(rng, params[1], 50000)
    edges = np.quantile(np.concatenate([n0, n1]), np.linspace(0.1, 0.9, NUM_BINS - 1), axis=0).T
    out_codes, out_f = [], []
    d = len(CAT_LEVELS) + N_NUMERIC
    for c in (0, 1):
        have = np.zeros((0, d), dtype=np.uint16)
        while have.shape[0] < per_class:
            m = int((per_class - have.shape[0]) * 1.3) + 1024
            cats, num = _mixture_raw(rng, params[c], m)
            rows = np.concatenate([cats, _bin_numeric(num, edges)], axis=1).astype(np.uint16)
            keep = rng.random((m, d)) < keep_p
            empty = ~keep.any(axis=1)
            keep[empty, rng.integers(0, d, size=int(empty.sum()))] = True
            rows[~keep] = ABSENT
            allrows = np.concatenate([have, rows])
            _, first = np.unique(allrows, axis=0, return_index=True)
            first.sort()
            have = allrows[first]
        have = have[:per_class]
        out_codes.append(have)
        out_f.append(rng.integers(1, f_max + 1, size=per_class).astype(np.uint32))
    return PatternSet(out_codes, out_f, mixture41_nbins())


def make_flows(seed: int = 5, n: int = 200_000) -> np.ndarray:
    """Flows to be served, drawn from the 41-feature mixture (both classes)."""
    w = make_mixture41(seed, n, train_frac=0.0)
    return w.test_codes


@dataclass
class Request:
    arrival_s: float
    start: int      # offset into the flow pool
    size: int


def make_requests(seed: int, rate_flows_per_s: float, n_requests: int,
                  pool_size: int, max_size: int = 4096) -> List[Request]:
    """Poisson arrivals; sizes floor(exp(U(0, ln(max_size+1)))) clipped to [1, max_size]."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(0.0, np.log(max_size + 1), size=n_requests))).astype(np.int64)
    sizes = np.clip(sizes, 1, max_size)
    mean_size = (max_size) / np.log(max_size + 1)
    req_rate = rate_flows_per_s / mean_size
    gaps = rng.exponential(1.0 / req_rate, size=n_requests)
    arr = np.cumsum(gaps)
    starts = rng.integers(0, max(1, pool_size - max_size), size=n_requests)
    return [Request(float(a), int(s), int(z)) for a, s, z in zip(arr, starts, sizes)]


# --------------------------------------------------------------------------
# Small random problems for parity sweeps (ragged sizes, many widths).
# --------------------------------------------------------------------------
def make_random_problem(seed: int, n: int, d: int, bins_lo: int = 2, bins_hi: int = 8,
                        attack_frac: float = 0.5, concentration: float = 0.5) -> Problem:
    rng = np.random.default_rng(seed)
    nbins = rng.integers(bins_lo, bins_hi + 1, size=d)
    n1 = int(round(n * attack_frac))
    n0 = n - n1
    codes = np.empty((n, d), dtype=np.int64)
    for f in range(d):
        nb = int(nbins[f])
        for lo, hi in ((0, n0), (n0, n)):
            p = rng.dirichlet([concentration] * nb)
            codes[lo:hi, f] = _draw_categorical(rng, p, hi - lo)
    labels = np.concatenate([np.zeros(n0, np.uint8), np.ones(n1, np.uint8)])
    perm = rng.permutation(n)
    return Problem(codes[perm].astype(np.uint16), labels[perm], nbins.astype(np.uint16))
