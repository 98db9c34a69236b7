"""Evidence of a decision -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark may import this module.
For a flow t and a class c, the evidence is the set of coherent patterns of P^c
that lie inside t: exactly the terms that Eq. 4 adds into A(t) (c = 1) or N(t)
(c = 0).  The paper presents these matched patterns as the readable account of
a decision (Sections 2 and 5); this module lists them.

Reading taken where the paper is silent: a caller asks for at most k of them;
the k reported are the heaviest, ordered by weight S descending and, between
equal weights, by the patterns' words in ascending canonical order (w_0 most
significant, compared as unsigned 64-bit), so that the list is unique.

Plain numpy on packed rows (oracle.pack); no blocking, no pruning.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from . import pack


def inside_mask(patterns: np.ndarray, flow_words: np.ndarray) -> np.ndarray:
    """Eq. 6 for every pattern of a class against one flow: b AND NOT t == 0 on
    every word."""
    if patterns.shape[0] == 0:
        return np.zeros(0, bool)
    return np.all((patterns & ~flow_words[None, :]) == 0, axis=1)


def evidence_order(patterns: np.ndarray, S: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """The indices idx sorted by S descending, then by the rows' words ascending."""
    if idx.size == 0:
        return idx
    # np.lexsort sorts by the last key first: words K-1 .. 0 (w_0 most significant), then -S
    keys = [patterns[idx, k] for k in range(patterns.shape[1] - 1, -1, -1)]
    keys.append(-S[idx])
    return idx[np.lexsort(keys)]


def evidence(model, flows, nbins, k: int) -> List[List[Tuple[int, np.ndarray, np.ndarray, np.ndarray]]]:
    """For each flow and class: (count inside, words [min(k, count), K], f, S) of the
    heaviest patterns inside the flow, in evidence order."""
    fw = pack(flows, nbins)
    out = []
    for t in range(fw.shape[0]):
        per = []
        for c in (0, 1):
            P, f, S = model.patterns[c], model.f[c], model.S[c]
            idx = np.nonzero(inside_mask(P, fw[t]))[0]
            top = evidence_order(P, S, idx)[:k]
            per.append((int(idx.size), P[top], f[top], S[top]))
        out.append(per)
    return out
