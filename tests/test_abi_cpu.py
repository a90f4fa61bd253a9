"""Host-side checks of the C-ABI library (no GPU compute): it loads, exports
every function declared in include/bbc.h, maps status codes, and refuses a
context when no GPU is visible."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bbc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bbc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def bbc():
    from paper_2605_03603_amd import bbc as B
    return B


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["bbc_build_csr", "bbc_count_global", "bbc_count_per_vertex", "bbc_submit", "bbc_poll",
              "bbc_count_batch", "bbc_ctx_create", "bbc_status_string"]:
        assert n in names


def test_library_exports_every_declared_symbol(bbc):
    lib = ctypes.CDLL(bbc.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(bbc.EXPORTED) == declared_functions()


def test_status_strings(bbc):
    for code, name in bbc.STATUS_NAMES.items():
        assert bbc.status_string(code)
    assert bbc.status_string(0) == "ok"
    assert bbc.status_string(99) == "unknown status"


def test_null_arguments_rejected(bbc):
    L = bbc.lib
    assert L.bbc_ctx_create(0, None, 0, None) == 1           # BBC_E_INVAL
    assert L.bbc_count_global(None, None, 3, 3, None) == 1
    assert L.bbc_poll(None, 1, None) == 1
    assert L.bbc_last_error(None) == b"null context"


def test_no_device_means_no_context(bbc):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    st = bbc.lib.bbc_ctx_create(0, None, 0, ctypes.byref(h))
    assert st == 10   # BBC_E_HIP
    with pytest.raises(bbc.BBCError):
        bbc.Context(0)


def test_sign_packing_roundtrip(bbc):
    import numpy as np
    s = np.array([1, -1, -1, 1, 1, -1, 1], np.int8)
    p = bbc.pack_signs_2bit(s)
    codes = [(p[e >> 2] >> (2 * (e & 3))) & 3 for e in range(s.size)]
    assert codes == [1 if x > 0 else 3 for x in s]
