"""Definitional IG oracle on Python sets -- TEST INFRASTRUCTURE ONLY.

Only the test suite may import this module.  It works on token sets, never on
packed words: a record is the frozenset of its (feature, bin) tokens (Section
3.1), intersections are Python's set ``&`` and subset tests are ``<=``.  It is
meant for small inputs (pure-Python loops) and serves as the second,
independent oracle that the C oracle is cross-checked against.

Readings of the paper (same as the C oracle): f_c(b) is the number of class-c
records containing b; |b| is the number of tokens; the empty set is never a
pattern; label 1 (attack) is class "+", scored into A.
"""
from __future__ import annotations

from typing import Dict, FrozenSet, Iterable, List, Sequence, Tuple

Token = Tuple[int, int]
TokenSet = FrozenSet[Token]


def tokens(row: Sequence[int], absent: int = 0xFFFF) -> TokenSet:
    """Section 3.1: every value is tied to its column, giving one token per feature."""
    return frozenset((f, int(c)) for f, c in enumerate(row) if int(c) != absent)


def candidates(X: List[TokenSet]) -> set:
    """Eq. 1: the records and the intersections of every pair (taken once);
    the empty set is never a candidate."""
    B = set(x for x in X if x)
    for i in range(len(X)):
        for j in range(i + 1, len(X)):
            b = X[i] & X[j]
            if b:
                B.add(b)
    return B


def coherent(B: Iterable[TokenSet], X_other: List[TokenSet]) -> set:
    """Eq. 3: keep b when no record of the other class contains it."""
    return set(b for b in B if not any(b <= x for x in X_other))


def support(b: TokenSet, X: List[TokenSet]) -> int:
    """f_c(b) of Eq. 2: records of the class containing b."""
    return sum(1 for x in X if b <= x)


def weight(b: TokenSet, X: List[TokenSet]) -> int:
    """Eq. 2: S_c(b) = f_c(b) * |b|^2."""
    return support(b, X) * len(b) ** 2


def fit(codes, labels) -> Dict[int, Dict[TokenSet, Tuple[int, int]]]:
    """Per class c (0 normal, 1 attack): {pattern: (f, S)} for every coherent pattern."""
    X = {0: [], 1: []}
    for row, lab in zip(codes, labels):
        X[int(lab)].append(tokens(row))
    out = {}
    for c in (0, 1):
        P = coherent(candidates(X[c]), X[1 - c])
        out[c] = {b: (support(b, X[c]), weight(b, X[c])) for b in P}
    return out


def score(model, flows) -> List[Tuple[int, int]]:
    """Eq. 4: (A, N) per flow; A sums the attack patterns, N the normal ones."""
    res = []
    for row in flows:
        x = tokens(row)
        A = sum(S for b, (_, S) in model[1].items() if b <= x)
        N = sum(S for b, (_, S) in model[0].items() if b <= x)
        res.append((A, N))
    return res
