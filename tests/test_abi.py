"""The C-ABI library builds, loads and exports every function include/bos.h
declares (no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bos.h")
LIB = os.path.join(ROOT, "paper_2008_01765_amd", "libbos.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bos_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libbos():
    if not os.path.exists(LIB):
        from paper_2008_01765_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("bos_orp", "bos_sort", "bos_sort_batched", "bos_workspace_bytes", "bos_status_string"):
        assert required in names


def test_every_declared_symbol_is_exported(libbos):
    missing = [f for f in declared_functions() if not hasattr(libbos, f)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2008_01765_amd import bos
    assert sorted(bos.EXPORTS) == declared_functions()


def test_status_strings(libbos):
    libbos.bos_status_string.restype = ctypes.c_char_p
    for s in range(7):
        assert libbos.bos_status_string(s)


def test_no_gpu_calls_fail_cleanly(libbos):
    # Without a GPU every entry point reports UNSUPPORTED instead of crashing.
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    libbos.bos_orp.restype = ctypes.c_int
    st = libbos.bos_orp(None, None, ctypes.c_uint64(10), 8, None, None, ctypes.c_size_t(0), None, None)
    assert st == 6
