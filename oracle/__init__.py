"""CPU oracle of the IG hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product path never calls it.  It wraps the plain C oracle
(``ig_oracle.c``) with ctypes and numpy; ``definitional`` is a second,
set-based oracle for small inputs.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import build_oracle

_lib = None
_lib_path = None   # another build of ig_oracle.c to load instead of build_oracle.LIB


class _Model(C.Structure):
    _fields_ = [
        ("K", C.c_uint32), ("L", C.c_uint32), ("d", C.c_uint32),
        ("n_class", C.c_uint64 * 2), ("pairs", C.c_uint64 * 2),
        ("distinct", C.c_uint64 * 2), ("tests", C.c_uint64 * 2),
        ("count", C.c_uint64 * 2),
        ("words", C.POINTER(C.c_uint64) * 2),
        ("f", C.POINTER(C.c_uint32) * 2),
        ("S", C.POINTER(C.c_int64) * 2),
    ]


def lib():
    global _lib
    if _lib is None:
        path = _lib_path or build_oracle.build(force=False)   # rebuilt when the source is newer
        L = C.CDLL(path)
        p = C.c_void_p
        L.igo_pack.argtypes = [p, C.c_uint64, C.c_uint32, p, C.c_uint32, p]
        L.igo_fit.argtypes = [p, C.c_uint64, C.c_uint32, p, p, C.POINTER(_Model)]
        L.igo_free.argtypes = [C.POINTER(_Model)]
        L.igo_free.restype = None
        L.igo_score.argtypes = [C.POINTER(_Model), p, C.c_uint64, C.c_uint32, p, p, p]
        L.igo_score_packed.argtypes = [C.POINTER(_Model), p, C.c_uint64, p, p]
        L.igo_model_from_patterns.argtypes = [p, p, C.c_uint64, p, p, C.c_uint64, C.c_uint32, p,
                                              C.POINTER(_Model)]
        L.igo_score_direct.argtypes = [p, C.c_uint64, C.c_uint32, p, p, p, C.c_uint64, p, p]
        L.igo_pair_facts.argtypes = [p, C.c_uint64, C.c_uint32, p, p, C.c_int, p, p, C.c_uint64,
                                     p, p, p, p]
        L.igo_max_threads.restype = C.c_int
        L.igo_set_threads.argtypes = [C.c_int]
        L.igo_set_threads.restype = None
        _lib = L
    return _lib


def use_library(path: Optional[str]) -> None:
    """Load the oracle from another build of the same source (the benchmark's
    host-tuned copy); None returns to the default build."""
    global _lib, _lib_path
    _lib = None
    _lib_path = path


def _ptr(a: np.ndarray):
    return C.c_void_p(a.ctypes.data) if a.size else C.c_void_p(0)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class OracleError(RuntimeError):
    pass


def universe(nbins) -> tuple:
    L = int(np.asarray(nbins, dtype=np.int64).sum())
    return L, (L + 63) // 64


def pack(codes, nbins) -> np.ndarray:
    """Eq. 5 packing of code rows (0xFFFF = feature absent)."""
    codes = _c(codes, np.uint16)
    nbins = _c(nbins, np.uint16)
    n, d = codes.shape
    _, K = universe(nbins)
    out = np.zeros((n, K), dtype=np.uint64)
    rc = lib().igo_pack(_ptr(codes), n, d, _ptr(nbins), K, _ptr(out))
    if rc:
        raise OracleError(f"igo_pack failed ({rc})")
    return out


@dataclass
class OracleModel:
    K: int
    L: int
    d: int
    patterns: List[np.ndarray]   # per class: uint64 [m, K], ascending
    f: List[np.ndarray]          # per class: uint32 [m]
    S: List[np.ndarray]          # per class: int64 [m]
    stats: Dict = field(default_factory=dict)
    _m: Optional[_Model] = None

    def __del__(self):
        if self._m is not None and _lib is not None:
            _lib.igo_free(C.byref(self._m))
            self._m = None


def _wrap(m: _Model) -> OracleModel:
    K = m.K
    pats, fs, Ss = [], [], []
    for c in (0, 1):
        cnt = int(m.count[c])
        if cnt:
            w = np.ctypeslib.as_array(m.words[c], shape=(cnt * K,)).reshape(cnt, K).copy()
            f = np.ctypeslib.as_array(m.f[c], shape=(cnt,)).copy()
            S = np.ctypeslib.as_array(m.S[c], shape=(cnt,)).copy()
        else:
            w = np.zeros((0, K), np.uint64)
            f = np.zeros(0, np.uint32)
            S = np.zeros(0, np.int64)
        pats.append(w); fs.append(f); Ss.append(S)
    stats = {
        "n_class": [int(m.n_class[0]), int(m.n_class[1])],
        "pairs": [int(m.pairs[0]), int(m.pairs[1])],
        "distinct": [int(m.distinct[0]), int(m.distinct[1])],
        "tests": [int(m.tests[0]), int(m.tests[1])],
        "coherent": [int(m.count[0]), int(m.count[1])],
    }
    return OracleModel(int(m.K), int(m.L), int(m.d), pats, fs, Ss, stats, m)


def fit(codes, labels, nbins) -> OracleModel:
    """Eq. 1-3 and Eq. 2 weights for both classes."""
    codes = _c(codes, np.uint16)
    labels = _c(labels, np.uint8)
    nbins = _c(nbins, np.uint16)
    n, d = codes.shape
    m = _Model()
    rc = lib().igo_fit(_ptr(codes), n, d, _ptr(labels), _ptr(nbins), C.byref(m))
    if rc:
        raise OracleError(f"igo_fit failed ({rc})")
    return _wrap(m)


def model_from_patterns(codes0, f0, codes1, f1, nbins) -> OracleModel:
    """A model from given pattern code rows (0xFFFF = feature absent) and supports:
    Eq. 5 packing and Eq. 2 weights, rows in the order given."""
    codes0 = _c(codes0, np.uint16); codes1 = _c(codes1, np.uint16)
    f0 = _c(f0, np.uint32); f1 = _c(f1, np.uint32)
    nbins = _c(nbins, np.uint16)
    d = codes0.shape[1]
    m = _Model()
    rc = lib().igo_model_from_patterns(_ptr(codes0), _ptr(f0), codes0.shape[0], _ptr(codes1),
                                       _ptr(f1), codes1.shape[0], d, _ptr(nbins), C.byref(m))
    if rc:
        raise OracleError(f"igo_model_from_patterns failed ({rc})")
    return _wrap(m)


def score(model: OracleModel, codes, nbins):
    """Eq. 4: returns (A, N) int64 arrays."""
    codes = _c(codes, np.uint16)
    nbins = _c(nbins, np.uint16)
    n, d = codes.shape
    A = np.zeros(n, np.int64)
    N = np.zeros(n, np.int64)
    rc = lib().igo_score(C.byref(model._m), _ptr(codes), n, d, _ptr(nbins), _ptr(A), _ptr(N))
    if rc:
        raise OracleError(f"igo_score failed ({rc})")
    return A, N


def score_direct(codes, labels, nbins, flows):
    """(A, N) of each flow from the definitions, without fitting a model."""
    codes = _c(codes, np.uint16); labels = _c(labels, np.uint8)
    nbins = _c(nbins, np.uint16); flows = _c(flows, np.uint16)
    n, d = codes.shape
    m = flows.shape[0]
    A = np.zeros(m, np.int64)
    N = np.zeros(m, np.int64)
    rc = lib().igo_score_direct(_ptr(codes), n, d, _ptr(labels), _ptr(nbins), _ptr(flows), m,
                                _ptr(A), _ptr(N))
    if rc:
        raise OracleError(f"igo_score_direct failed ({rc})")
    return A, N


def pair_facts(codes, labels, nbins, cls: int, pi, pj):
    """For class-c record pairs (i, j) (indices within the class, input order):
    b = x_i AND x_j, coherent flag, support f and t(b)."""
    codes = _c(codes, np.uint16); labels = _c(labels, np.uint8)
    nbins = _c(nbins, np.uint16)
    pi = _c(pi, np.uint64); pj = _c(pj, np.uint64)
    n, d = codes.shape
    _, K = universe(nbins)
    q = pi.size
    words = np.zeros((q, K), np.uint64)
    coh = np.zeros(q, np.uint8)
    f = np.zeros(q, np.uint32)
    t = np.zeros(q, np.uint64)
    rc = lib().igo_pair_facts(_ptr(codes), n, d, _ptr(labels), _ptr(nbins), cls, _ptr(pi), _ptr(pj),
                              q, _ptr(words), _ptr(coh), _ptr(f), _ptr(t))
    if rc:
        raise OracleError(f"igo_pair_facts failed ({rc})")
    return words, coh.astype(bool), f, t


def max_threads() -> int:
    return int(lib().igo_max_threads())


def set_threads(n: int) -> None:
    lib().igo_set_threads(int(n))
