"""The C-ABI library: it loads, exports every symbol the headers under include/
declare, and rejects bad arguments that need no device data before touching the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2507_14222_amd import ig

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")


def _declared():
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(INCLUDE, h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(ig_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_is_built():
    assert os.path.exists(ig.LIB_PATH), "run __graft_entry__.build() first"


def test_every_declared_symbol_is_exported():
    L = ig.lib()
    declared = _declared()
    assert set(declared) == set(ig.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_version_and_no_error_initially():
    assert "gfx950" in ig.version()
    assert ig.lib().ig_last_error() in (b"",)


def _fit_raw(codes_ptr, labels_ptr, n, d, nbins, out=True):
    h = C.c_void_p()
    nb = np.ascontiguousarray(nbins, np.uint16) if nbins is not None else None
    st = ig.lib().ig_fit(codes_ptr, labels_ptr, n, d,
                         C.c_void_p(nb.ctypes.data) if nb is not None else None,
                         None, None, C.byref(h) if out else None)
    return st, h


def test_fit_rejects_null_out():
    st, _ = _fit_raw(None, None, 0, 2, [2, 2], out=False)
    assert st == ig.IG_E_INVAL
    assert b"out" in ig.lib().ig_last_error()


def test_fit_rejects_bad_nbins():
    st, h = _fit_raw(None, None, 0, 3, [2, 0, 2])
    assert st == ig.IG_E_INVAL and not h.value
    assert b"nbins[1]" in ig.lib().ig_last_error()
    st, _ = _fit_raw(None, None, 0, 2, None)
    assert st == ig.IG_E_INVAL
    st, _ = _fit_raw(None, None, 0, 0, [1])
    assert st == ig.IG_E_INVAL


def test_fit_rejects_too_wide_universe():
    st, _ = _fit_raw(None, None, 0, 2, [4000, 200])
    assert st == ig.IG_E_UNSUPPORTED
    assert b"4096" in ig.lib().ig_last_error()


def test_fit_rejects_null_codes():
    st, _ = _fit_raw(None, None, 10, 2, [2, 2])
    assert st == ig.IG_E_INVAL


def test_fit_packed_rejects_bad_width():
    h = C.c_void_p()
    assert ig.lib().ig_fit_packed(None, None, 0, 65, None, None, C.byref(h)) == ig.IG_E_UNSUPPORTED
    assert ig.lib().ig_fit_packed(None, None, 0, 0, None, None, C.byref(h)) == ig.IG_E_UNSUPPORTED


def test_model_calls_reject_null():
    info = ig.ModelInfo()
    assert ig.lib().ig_model_get_info(None, C.byref(info)) == ig.IG_E_INVAL
    st = ig.Stats()
    assert ig.lib().ig_fit_stats(None, C.byref(st)) == ig.IG_E_INVAL
    ig.lib().ig_model_free(None)   # NULL-safe
    assert ig.lib().ig_score(None, None, 0, None, None) == ig.IG_E_INVAL
    assert ig.lib().ig_model_export(None, 0, None, None, None) == ig.IG_E_INVAL


def test_import_rejects_null():
    h = C.c_void_p()
    assert ig.lib().ig_model_import(None, None, None, 1, None, None, C.byref(h)) == ig.IG_E_INVAL


def test_error_text_is_thread_local():
    import threading
    _fit_raw(None, None, 0, 2, [4000, 200])
    main_msg = ig.lib().ig_last_error()
    seen = []

    def other():
        seen.append(ig.lib().ig_last_error())

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert main_msg and seen == [b""]
