"""The C-ABI library loads and exports every function include/taches.h
declares (CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "taches.h")
LIB = os.path.join(ROOT, "paper_2401_01607_amd", "libtaches.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(taches_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_four_core_calls():
    names = declared_functions()
    for core in ("taches_open", "taches_set_ir", "taches_process", "taches_close"):
        assert core in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtaches.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtaches.so not built")
def test_binding_wraps_every_declared_symbol():
    from paper_2401_01607_amd import taches as T
    missing = [n for n in declared_functions() if not hasattr(T, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtaches.so not built")
def test_config_default_and_bytes_need_no_gpu():
    from paper_2401_01607_amd import taches as T
    c = T.taches_config_default(256, 65536)
    assert (c.block_size, c.max_ir_len, c.channels, c.ir_slots) == (256, 65536, 1, 2)
    b = T.taches_bytes_for(c)
    # tail >= (Lmax - 1 + B) FP32 slots, two IR slots
    assert b >= (65536 - 1 + 256) * 4 + 2 * 65536 * 4
    c.max_ir_len = 0
    assert T.taches_bytes_for(c) == -1
