"""Python binding of libig (ctypes): argument marshalling only.

Every step of the IG hot path runs in the HIP kernels of ``libig.so``;
PyTorch only provides device memory and streams.  The binding fails loudly when
the library has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libig.so")

IG_OK, IG_E_INVAL, IG_E_NOMEM, IG_E_DEVICE, IG_E_OVERFLOW, IG_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
_NAMES = {0: "IG_OK", -1: "IG_E_INVAL", -2: "IG_E_NOMEM", -3: "IG_E_DEVICE", -4: "IG_E_OVERFLOW",
          -5: "IG_E_UNSUPPORTED"}
ABSENT = 0xFFFF
IG_MODEL_SCORE_MFMA = 1   # ModelInfo.flags: scoring runs on the matrix cores
IG_MODEL_FACTORED = 2     # ModelInfo.flags: matrix-core operands use factored tokens
IG_MODEL_BUCKETED = 4     # ModelInfo.flags: scoring tiles grouped by token (pruned scoring)
IG_MODEL_FIT_BUCKETS = 8  # ModelInfo.flags: the fit's contractions used token buckets
SCORE_MODES = {"auto": 0, "dense": 1, "pruned": 2}


class IGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class TuneEntry(C.Structure):
    _fields_ = [("ks", C.c_uint32), ("min_pairs", C.c_uint32), ("filter_cpl", C.c_uint32),
                ("grid_per_cu", C.c_uint32), ("support_cpl", C.c_uint32), ("mfma_words", C.c_uint32),
                ("coherence_sets", C.c_uint32), ("support_sets", C.c_uint32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    """ig_allocator: a caller's device allocator (see torch_allocator())."""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class FitOpts(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_uint64), ("filter_cpl", C.c_uint32), ("score_fpl", C.c_uint32),
                ("block", C.c_uint32), ("n_tune", C.c_uint32), ("tune", C.POINTER(TuneEntry)),
                ("coherence_mfma", C.c_uint32), ("fit_dense", C.c_uint32), ("alloc", C.POINTER(Allocator))]


def torch_allocator(fail_after: Optional[int] = None) -> Allocator:
    """An ig_allocator over torch's caching allocator: the library's model buffers
    and fit scratch then come from torch's pool, stream-ordered on the stream the
    library passes.  fail_after = n makes every allocation after the first n fail
    (for tests of the failure path).  The returned object keeps its callbacks alive;
    keep it (the models built with it keep a reference)."""
    torch = _torch()
    state = {"n": 0, "live": {}}

    def _alloc(nbytes, stream, ctx):
        if fail_after is not None and state["n"] >= fail_after:
            return None
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), int(stream or 0))
        except Exception:
            return None
        state["n"] += 1
        state["live"][p] = int(nbytes)
        return p

    def _free(ptr, stream, ctx):
        if ptr:
            state["live"].pop(ptr, None)
            torch.cuda.caching_allocator_delete(ptr)

    a = Allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
    a._state = state          # allocations made and blocks still held (tests)
    return a


class Stats(C.Structure):
    _fields_ = [("n_class", C.c_uint64 * 2), ("pairs", C.c_uint64 * 2), ("distinct", C.c_uint64 * 2),
                ("coherent", C.c_uint64 * 2), ("tests", C.c_uint64 * 2), ("support_tests", C.c_uint64 * 2),
                ("chunks", C.c_uint32 * 2), ("ms", C.c_float * 8), ("kernel_ms", C.c_float * 2)]


class ModelInfo(C.Structure):
    _fields_ = [("K", C.c_uint32), ("L", C.c_uint32), ("d", C.c_uint32), ("flags", C.c_uint32),
                ("mfma_tokens", C.c_uint32), ("mfma_words", C.c_uint32),
                ("n_patterns", C.c_uint64 * 2), ("max_weight", C.c_int64 * 2),
                ("fit_tokens", C.c_uint32), ("fit_words", C.c_uint32)]


class Moments(C.Structure):
    """Exact moments of N over the normal records (ig_moments)."""
    _fields_ = [("count", C.c_uint64), ("sum", C.c_uint64 * 2), ("sumsq", C.c_uint64 * 3)]

    @property
    def total(self) -> int:
        return int(self.sum[0]) | int(self.sum[1]) << 64

    @property
    def total_sq(self) -> int:
        return int(self.sumsq[0]) | int(self.sumsq[1]) << 64 | int(self.sumsq[2]) << 128


class Metrics(C.Structure):
    """Confusion counts and the exact AUC fraction (ig_metrics)."""
    _fields_ = [("tp", C.c_uint64), ("fp", C.c_uint64), ("tn", C.c_uint64), ("fn", C.c_uint64),
                ("auc_num", C.c_uint64), ("auc_den", C.c_uint64), ("invalid", C.c_uint64)]

    def as_dict(self) -> dict:
        tp, fp, tn, fn = int(self.tp), int(self.fp), int(self.tn), int(self.fn)
        n = tp + fp + tn + fn
        return {"tp": tp, "fp": fp, "tn": tn, "fn": fn, "invalid": int(self.invalid),
                "accuracy": (tp + tn) / n if n else 0.0,
                "recall": tp / (tp + fn) if tp + fn else 0.0,
                "precision": tp / (tp + fp) if tp + fp else 0.0,
                "auc": int(self.auc_num) / int(self.auc_den) if self.auc_den else 0.0}


class Problem(C.Structure):
    _fields_ = [("d_codes", C.c_void_p), ("d_labels", C.c_void_p), ("n", C.c_uint32), ("d", C.c_uint32),
                ("h_nbins", C.c_void_p)]


_lib = None

# every symbol the headers under include/ declare
EXPORTS = ("ig_fit", "ig_fit_packed", "ig_fit_batch", "ig_score", "ig_score_ex", "ig_score_noalloc", "ig_score_packed", "ig_model_get_info",
           "ig_model_export", "ig_model_import", "ig_model_digest", "ig_fit_stats", "ig_model_free",
           "ig_last_error", "ig_version", "ig_probe_mfma_fp4", "ig_probe_hbm_copy", "ig_normal_moments",
           "ig_r3_threshold", "ig_classify", "ig_detection_metrics", "ig_evidence", "ig_model_bucket_sizes", "ig_release_memory", "ig_memory_stats")
IG_CLASSIFY_R3, IG_CLASSIFY_NO_R2 = 1, 2


def lib():
    """Load libig.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise IGError(IG_E_DEVICE, f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, u32, u64 = C.c_void_p, C.c_uint32, C.c_uint64
    L.ig_fit.argtypes = [vp, vp, u32, u32, vp, C.POINTER(FitOpts), vp, C.POINTER(vp)]
    L.ig_fit_packed.argtypes = [vp, vp, u32, u32, C.POINTER(FitOpts), vp, C.POINTER(vp)]
    L.ig_fit_batch.argtypes = [C.POINTER(Problem), u32, C.POINTER(FitOpts), vp, C.POINTER(vp)]
    L.ig_score.argtypes = [vp, vp, u32, vp, vp]
    L.ig_score_ex.argtypes = [vp, vp, u32, vp, u32, vp]
    L.ig_score_noalloc.argtypes = [vp, vp, u32, vp, vp]
    L.ig_score_packed.argtypes = [vp, vp, u32, vp, vp]
    L.ig_model_get_info.argtypes = [vp, C.POINTER(ModelInfo)]
    L.ig_model_export.argtypes = [vp, u32, vp, vp, vp]
    L.ig_model_import.argtypes = [C.POINTER(vp), C.POINTER(vp), C.POINTER(u64), u32, vp, vp, C.POINTER(vp)]
    L.ig_fit_stats.argtypes = [vp, C.POINTER(Stats)]
    L.ig_model_digest.argtypes = [vp, u32, C.POINTER(u64)]
    L.ig_model_free.argtypes = [vp]
    L.ig_model_free.restype = None
    L.ig_last_error.restype = C.c_char_p
    L.ig_version.restype = C.c_char_p
    L.ig_probe_mfma_fp4.argtypes = [u32, vp, C.POINTER(C.c_double), C.POINTER(C.c_float)]
    L.ig_probe_hbm_copy.argtypes = [vp, vp, C.c_size_t, vp, C.POINTER(C.c_double), C.POINTER(C.c_float)]
    L.ig_normal_moments.argtypes = [vp, vp, u32, C.POINTER(Moments), vp]
    L.ig_evidence.argtypes = [vp, vp, u32, u32, vp, vp, vp, vp, vp]
    L.ig_model_bucket_sizes.argtypes = [vp, u32, vp]
    L.ig_release_memory.argtypes = []
    L.ig_memory_stats.argtypes = [C.POINTER(u64), C.POINTER(u64), C.POINTER(u64)]
    L.ig_r3_threshold.argtypes = [C.POINTER(Moments), C.c_double, C.POINTER(C.c_int64)]
    L.ig_classify.argtypes = [vp, u32, C.c_int64, u32, vp, vp, vp]
    L.ig_detection_metrics.argtypes = [vp, vp, vp, u32, C.POINTER(Metrics), vp]
    for name in ("ig_fit", "ig_fit_packed", "ig_fit_batch", "ig_score", "ig_score_ex", "ig_score_noalloc", "ig_score_packed", "ig_model_get_info",
                 "ig_model_export", "ig_model_import", "ig_model_digest", "ig_fit_stats", "ig_probe_mfma_fp4",
                 "ig_probe_hbm_copy", "ig_normal_moments", "ig_r3_threshold", "ig_classify",
                 "ig_detection_metrics", "ig_evidence", "ig_model_bucket_sizes", "ig_release_memory", "ig_memory_stats"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(status: int) -> None:
    if status != IG_OK:
        raise IGError(status, lib().ig_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> C.c_void_p:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class _OnStream:
    """Context for one library call on `stream` (None = torch's current stream).

    Inside it torch's current stream is the call's stream, so the temporaries the
    binding makes (host-to-device copies, dtype conversions, default outputs) are
    enqueued and allocated on the stream the library then launches on.  That
    stream first waits for work already queued on the caller's current stream
    (which may have produced the inputs), and every device tensor handed to the
    library is marked as used on it, so that torch's caching allocator does not
    reuse its memory while the call is still in flight."""

    def __init__(self, stream):
        torch = _torch()
        self.caller = torch.cuda.current_stream()
        self.s = stream if stream is not None else self.caller
        self._ctx = torch.cuda.stream(self.s)

    def __enter__(self):
        if self.s != self.caller:
            self.s.wait_stream(self.caller)
        self._ctx.__enter__()
        return self

    def __exit__(self, *exc):
        return self._ctx.__exit__(*exc)

    def use(self, t):
        """Mark a device tensor as read or written by the call."""
        if self.s != self.caller:
            t.record_stream(self.s)
        return t

    @property
    def handle(self) -> C.c_void_p:
        return C.c_void_p(self.s.cuda_stream)


def _dev(a, dtype):
    """A contiguous device tensor of the given torch dtype (copies host arrays)."""
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a
        if t.dtype != dtype:
            t = t.to(dtype)
        if not t.is_cuda:
            t = t.cuda()
        return t.contiguous()
    arr = np.ascontiguousarray(a)
    # keep the bits: unsigned 16/64-bit arrays travel as their signed views
    if arr.dtype == np.uint16:
        arr = arr.view(np.int16)
    elif arr.dtype == np.uint64:
        arr = arr.view(np.int64)
    t = torch.from_numpy(arr).to(device="cuda")
    return (t if t.dtype == dtype else t.to(dtype)).contiguous()


def _np_u16(a) -> np.ndarray:
    if hasattr(a, "cpu"):
        a = a.cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.uint16)


def _opts(mem_budget_bytes: int = 0, filter_cpl: int = 0, score_fpl: int = 0, tune=None,
          kernels: str = "auto", allocator=None, dense: bool = False) -> FitOpts:
    """Fit options; `tune` is a list of dicts with the fields of ig_tune_entry;
    kernels = "auto" | "mfma" | "valu" | "mfma_onehot" | "mfma_presence" |
    "mfma_ternary" selects the coherence/support kernels ("mfma_onehot": matrix cores
    on the one-hot words, no factored tokens; "mfma_presence": factored tokens with
    presence tokens; "mfma_ternary": the ternary bit tokens whenever the fit has
    them; "mfma" and "auto" take whichever of the two needs fewer words);
    dense = True tests every candidate against every record on the ternary tokens
    instead of the records of its token bucket (same results);
    allocator = None (the library's arena), "torch" (torch's caching allocator) or an
    Allocator."""
    o = FitOpts()
    if allocator is not None:
        a = torch_allocator() if allocator == "torch" else allocator
        o.alloc = C.pointer(a)
        o._alloc = a
    o.fit_dense = 1 if dense else 0
    o.coherence_mfma = {"auto": 0, "mfma": 1, "valu": 2, "mfma_onehot": 3, "mfma_presence": 4,
                        "mfma_ternary": 5}[kernels]
    o.mem_budget_bytes = int(mem_budget_bytes)
    o.filter_cpl = int(filter_cpl)
    o.score_fpl = int(score_fpl)
    if tune:
        arr = (TuneEntry * len(tune))()
        for i, e in enumerate(tune):
            for k in ("ks", "min_pairs", "filter_cpl", "grid_per_cu", "support_cpl", "mfma_words",
                      "coherence_sets", "support_sets"):
                setattr(arr[i], k, int(e.get(k, 0)))
        o.n_tune = len(tune)
        o.tune = C.cast(arr, C.POINTER(TuneEntry))
        o._keep = arr   # keep the table alive with the options
    return o


@dataclass
class FitStats:
    n_class: Tuple[int, int]
    pairs: Tuple[int, int]
    distinct: Tuple[int, int]
    coherent: Tuple[int, int]
    tests: Tuple[int, int]
    support_tests: Tuple[int, int]
    chunks: Tuple[int, int]
    ms: Tuple[float, ...]
    kernel_ms: Tuple[float, float] = (0.0, 0.0)   # subset-test kernels alone: coherence, support


class Model:
    """A device-resident pair of coherent pattern sets (P^0 normal, P^1 attack)."""

    def __init__(self, handle: C.c_void_p, keep=None):
        self._h = handle
        self._keep = keep   # a caller allocator the model's buffers came from

    @property
    def handle(self) -> C.c_void_p:
        if not self._h:
            raise IGError(IG_E_INVAL, "model already freed")
        return self._h

    def info(self) -> ModelInfo:
        i = ModelInfo()
        _check(lib().ig_model_get_info(self.handle, C.byref(i)))
        return i

    @property
    def K(self) -> int:
        return int(self.info().K)

    @property
    def score_on_matrix_cores(self) -> bool:
        return bool(self.info().flags & IG_MODEL_SCORE_MFMA)

    @property
    def bucketed(self) -> bool:
        return bool(self.info().flags & IG_MODEL_BUCKETED)

    def n_patterns(self) -> Tuple[int, int]:
        i = self.info()
        return int(i.n_patterns[0]), int(i.n_patterns[1])

    def stats(self) -> FitStats:
        s = Stats()
        _check(lib().ig_fit_stats(self.handle, C.byref(s)))
        t = lambda a: (int(a[0]), int(a[1]))
        return FitStats(t(s.n_class), t(s.pairs), t(s.distinct), t(s.coherent), t(s.tests), t(s.support_tests),
                        t(s.chunks), tuple(float(x) for x in s.ms), tuple(float(x) for x in s.kernel_ms))

    def export(self, cls: int):
        """(words uint64 [n, K], f uint32 [n], S int64 [n]) of class ``cls``, ascending."""
        i = self.info()
        n, K = int(i.n_patterns[cls]), int(i.K)
        w = np.zeros((n, K), np.uint64)
        f = np.zeros(n, np.uint32)
        S = np.zeros(n, np.int64)
        ptr = lambda a: C.c_void_p(a.ctypes.data) if a.size else None
        _check(lib().ig_model_export(self.handle, cls, ptr(w), ptr(f), ptr(S)))
        return w, f, S

    def bucket_sizes(self, cls: int) -> np.ndarray:
        """Patterns of class ``cls`` per token bucket (uint32 [L])."""
        out = np.zeros(int(self.info().L), np.uint32)
        _check(lib().ig_model_bucket_sizes(self.handle, cls, C.c_void_p(out.ctypes.data)))
        return out

    def digest(self, cls: int) -> int:
        """Device-computed digest of class ``cls`` (rows, f, S in canonical order)."""
        h = C.c_uint64()
        _check(lib().ig_model_digest(self.handle, cls, C.byref(h)))
        return int(h.value)

    def free(self) -> None:
        if self._h:
            lib().ig_model_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def fit(codes, labels, nbins, mem_budget_bytes: int = 0, filter_cpl: int = 0, tune=None,
        kernels: str = "auto", stream=None, allocator=None, dense: bool = False) -> Model:
    """ig_fit: codes [n, d] bin codes, labels [n] (0 normal / 1 attack), nbins [d]."""
    torch = _torch()
    with _OnStream(stream) as on:
        dc = on.use(_dev(codes, torch.int16))
        dl = on.use(_dev(labels, torch.uint8))
        n, d = (int(dc.shape[0]), int(dc.shape[1])) if dc.dim() == 2 else (0, 0)
        nb = _np_u16(nbins)
        h = C.c_void_p()
        o = _opts(mem_budget_bytes, filter_cpl, tune=tune, kernels=kernels, allocator=allocator, dense=dense)
        _check(lib().ig_fit(C.c_void_p(dc.data_ptr()), C.c_void_p(dl.data_ptr()), n, d or nb.size,
                            C.c_void_p(nb.ctypes.data), C.byref(o), on.handle, C.byref(h)))
    return Model(h, getattr(o, "_alloc", None))


def fit_packed(words, labels, mem_budget_bytes: int = 0, stream=None) -> Model:
    """ig_fit_packed: words [n, K] uint64 bitsets (Eq. 5 layout), labels [n]."""
    torch = _torch()
    with _OnStream(stream) as on:
        dw = on.use(_dev(np.ascontiguousarray(words).view(np.int64) if isinstance(words, np.ndarray) else words,
                         torch.int64))
        dl = on.use(_dev(labels, torch.uint8))
        n, K = int(dw.shape[0]), int(dw.shape[1])
        h = C.c_void_p()
        o = _opts(mem_budget_bytes)
        _check(lib().ig_fit_packed(C.c_void_p(dw.data_ptr()), C.c_void_p(dl.data_ptr()), n, K, C.byref(o),
                                   on.handle, C.byref(h)))
    return Model(h)


def fit_batch(problems: Sequence, mem_budget_bytes: int = 0, tune=None, kernels: str = "auto",
              stream=None, allocator=None, dense: bool = False) -> List[Model]:
    """ig_fit_batch over problems with attributes codes, labels, nbins."""
    torch = _torch()
    keep = []
    arr = (Problem * len(problems))()
    with _OnStream(stream) as on:
        for p, pr in enumerate(problems):
            dc = on.use(_dev(pr.codes, torch.int16))
            dl = on.use(_dev(pr.labels, torch.uint8))
            nb = _np_u16(pr.nbins)
            keep += [dc, dl, nb]
            arr[p].d_codes = dc.data_ptr()
            arr[p].d_labels = dl.data_ptr()
            arr[p].n = int(dc.shape[0])
            arr[p].d = int(nb.size)
            arr[p].h_nbins = nb.ctypes.data
        outs = (C.c_void_p * len(problems))()
        o = _opts(mem_budget_bytes, tune=tune, kernels=kernels, allocator=allocator, dense=dense)
        _check(lib().ig_fit_batch(arr, len(problems), C.byref(o), on.handle, outs))
    keep = getattr(o, "_alloc", None)
    return [Model(C.c_void_p(outs[p]), keep) for p in range(len(problems))]


def score(model: Model, flows, out=None, stream=None, mode: str = "auto"):
    """ig_score / ig_score_ex: (A, N) per flow as an int64 device tensor [n, 2],
    asynchronous on `stream` (torch's current stream when None): the result is
    ready once that stream reaches the call.  mode = "auto" | "dense" | "pruned"."""
    torch = _torch()
    with _OnStream(stream) as on:
        dc = on.use(_dev(flows, torch.int16))
        n = int(dc.shape[0])
        if out is None:
            out = torch.empty((n, 2), dtype=torch.int64, device=dc.device)
        on.use(out)
        if mode == "auto":
            _check(lib().ig_score(model.handle, C.c_void_p(dc.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                  on.handle))
        else:
            _check(lib().ig_score_ex(model.handle, C.c_void_p(dc.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                     SCORE_MODES[mode], on.handle))
    return out


def score_noalloc(model: Model, flows, out, stream=None):
    """ig_score_noalloc: as score(), through the entry point that allocates no device
    memory (its scratch is a fixed array in the library); `flows` must already be a
    contiguous int16/uint16-bit device tensor and `out` an int64 device tensor
    [n, 2], so that the binding allocates nothing either."""
    torch = _torch()
    assert flows.is_cuda and flows.dtype == torch.int16 and flows.is_contiguous()
    assert out.is_cuda and out.dtype == torch.int64 and out.is_contiguous()
    n = int(flows.shape[0])
    with _OnStream(stream) as on:
        on.use(flows)
        on.use(out)
        _check(lib().ig_score_noalloc(model.handle, C.c_void_p(flows.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                      on.handle))
    return out


def score_packed(model: Model, words, out=None, stream=None):
    """ig_score_packed: as score() for flows given as packed words [n, K]."""
    torch = _torch()
    with _OnStream(stream) as on:
        dw = on.use(_dev(np.ascontiguousarray(words).view(np.int64) if isinstance(words, np.ndarray) else words,
                         torch.int64))
        n = int(dw.shape[0])
        if out is None:
            out = torch.empty((n, 2), dtype=torch.int64, device=dw.device)
        on.use(out)
        _check(lib().ig_score_packed(model.handle, C.c_void_p(dw.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                     on.handle))
    return out


def import_patterns(codes0, f0, codes1, f1, nbins, stream=None) -> Model:
    """ig_model_import from pattern code rows (ABSENT = feature not in the pattern)."""
    c = [np.ascontiguousarray(codes0, np.uint16), np.ascontiguousarray(codes1, np.uint16)]
    f = [np.ascontiguousarray(f0, np.uint32), np.ascontiguousarray(f1, np.uint32)]
    nb = _np_u16(nbins)
    pc = (C.c_void_p * 2)(*[x.ctypes.data for x in c])
    pf = (C.c_void_p * 2)(*[x.ctypes.data for x in f])
    cnt = (C.c_uint64 * 2)(c[0].shape[0], c[1].shape[0])
    h = C.c_void_p()
    _check(lib().ig_model_import(pc, pf, cnt, int(nb.size), C.c_void_p(nb.ctypes.data),
                                 _stream_handle(stream), C.byref(h)))
    return Model(h)


def evidence(model: Model, flows, k: int, stream=None):
    """ig_evidence: for each flow and class the number of patterns inside the flow
    and the k heaviest of them (weight descending, then words ascending).
    Returns device tensors count [n, 2] (int32 view of uint32; -1 marks a flow with
    a code out of range), words [n, 2, k, K] (int64 view of uint64), f [n, 2, k]
    (int32 view of uint32) and S [n, 2, k]; slots past the count are zero."""
    torch = _torch()
    K = model.K
    with _OnStream(stream) as on:
        dc = on.use(_dev(flows, torch.int16))
        n = int(dc.shape[0])
        cnt = on.use(torch.empty((n, 2), dtype=torch.int32, device=dc.device))
        words = on.use(torch.empty((n, 2, k, K), dtype=torch.int64, device=dc.device))
        f = on.use(torch.empty((n, 2, k), dtype=torch.int32, device=dc.device))
        S = on.use(torch.empty((n, 2, k), dtype=torch.int64, device=dc.device))
        _check(lib().ig_evidence(model.handle, C.c_void_p(dc.data_ptr()), n, int(k), C.c_void_p(cnt.data_ptr()),
                                 C.c_void_p(words.data_ptr()), C.c_void_p(f.data_ptr()), C.c_void_p(S.data_ptr()),
                                 on.handle))
    return cnt, words, f, S


def normal_moments(scores, labels, stream=None) -> Moments:
    """ig_normal_moments: exact count, sum and sum of squares of N over the records
    labelled 0 (scores: the [n, 2] (A, N) of those records)."""
    torch = _torch()
    mo = Moments()
    with _OnStream(stream) as on:
        ds = on.use(_dev(scores, torch.int64))
        dl = on.use(_dev(labels, torch.uint8))
        _check(lib().ig_normal_moments(C.c_void_p(ds.data_ptr()), C.c_void_p(dl.data_ptr()), int(ds.shape[0]),
                                       C.byref(mo), on.handle))
    return mo


def r3_threshold(moments: Moments, r: float) -> int:
    """ig_r3_threshold: T with N < mu_N - r sigma_N exactly when N < T (N >= 0)."""
    t = C.c_int64()
    _check(lib().ig_r3_threshold(C.byref(moments), float(r), C.byref(t)))
    return int(t.value)


def classify(scores, r3_threshold: Optional[int] = None, use_r2: bool = True, stream=None):
    """ig_classify: (label, rule) uint8 device tensors [n]; Regulation 3 applies
    when a threshold is given."""
    torch = _torch()
    with _OnStream(stream) as on:
        ds = on.use(_dev(scores, torch.int64))
        n = int(ds.shape[0])
        lab = on.use(torch.empty(n, dtype=torch.uint8, device=ds.device))
        rule = on.use(torch.empty(n, dtype=torch.uint8, device=ds.device))
        flags = (IG_CLASSIFY_R3 if r3_threshold is not None else 0) | (0 if use_r2 else IG_CLASSIFY_NO_R2)
        _check(lib().ig_classify(C.c_void_p(ds.data_ptr()), n, int(r3_threshold or 0), flags,
                                 C.c_void_p(lab.data_ptr()), C.c_void_p(rule.data_ptr()), on.handle))
    return lab, rule


def detection_metrics(scores, pred, truth, stream=None) -> Metrics:
    """ig_detection_metrics: confusion counts of pred against truth and the exact
    AUC of the margins A - N."""
    torch = _torch()
    mt = Metrics()
    with _OnStream(stream) as on:
        ds = on.use(_dev(scores, torch.int64))
        dp = on.use(_dev(pred, torch.uint8))
        dt = on.use(_dev(truth, torch.uint8))
        _check(lib().ig_detection_metrics(C.c_void_p(ds.data_ptr()), C.c_void_p(dp.data_ptr()),
                                          C.c_void_p(dt.data_ptr()), int(ds.shape[0]), C.byref(mt), on.handle))
    return mt


def release_memory() -> None:
    """ig_release_memory: the library's cached scratch and free arena chunks back."""
    _check(lib().ig_release_memory())


def memory_stats() -> dict:
    """ig_memory_stats of the current device: reserved, in use, cached bytes."""
    r, u, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
    _check(lib().ig_memory_stats(C.byref(r), C.byref(u), C.byref(c)))
    return {"reserved": int(r.value), "in_use": int(u.value), "cached": int(c.value)}


def version() -> str:
    return lib().ig_version().decode()


def probe_mfma_fp4(iters: int = 20000, stream=None) -> Tuple[float, float]:
    """Measured fp4 matrix-core rate of the device: (operations/s, launch ms)."""
    r, ms = C.c_double(), C.c_float()
    with _OnStream(stream) as on:
        _check(lib().ig_probe_mfma_fp4(int(iters), on.handle, C.byref(r), C.byref(ms)))
    return float(r.value), float(ms.value)


def probe_hbm_copy(src, dst, stream=None) -> Tuple[float, float]:
    """Measured HBM copy rate between two equal device tensors: (bytes/s read +
    written, launch ms)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    r, ms = C.c_double(), C.c_float()
    with _OnStream(stream) as on:
        on.use(src)
        on.use(dst)
        _check(lib().ig_probe_hbm_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, on.handle,
                                       C.byref(r), C.byref(ms)))
    return float(r.value), float(ms.value)
