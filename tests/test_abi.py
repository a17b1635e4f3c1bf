"""The C ABI library loads on a machine without a GPU and exports every function that
include/pfn.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(pfn_[a-z0-9_]+)\s*\(", text))
    return names


def test_header_declares_the_three_pipeline_calls():
    names = declared_functions()
    for n in ("pfn_trace_photon_cache", "pfn_train_field", "pfn_render_frame",
              "pfn_render_batch", "pfn_field_query", "pfn_render_path_traced"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2304_07338_amd import _ffi
    if not os.path.exists(_ffi.LIB_PATH):
        pytest.fail("libpfn.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_ffi.LIB_PATH)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares exactly the header's functions
    assert set(_ffi.SIGNATURES) == declared_functions()


def test_null_context_is_rejected_without_a_gpu():
    from paper_2304_07338_amd import _ffi
    lib = _ffi.load()
    assert lib.pfn_sync(None) == _ffi.PFN_ERR_INVALID_ARG
    assert lib.pfn_render_frame(None, None, None, None) == _ffi.PFN_ERR_INVALID_ARG
    assert lib.pfn_last_error(None) == b"null context"
    assert lib.pfn_create(0, None, None) == _ffi.PFN_ERR_INVALID_ARG
