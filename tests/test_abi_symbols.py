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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtaches.so not built")
def test_binding_structs_match_the_header_layout(tmp_path):
    """Compile the header with the host C compiler and compare every
    struct's size and field offsets with the ctypes mirrors."""
    import shutil
    import subprocess
    from paper_2401_01607_amd import taches as T
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"taches_config": T.taches_config, "taches_info": T.taches_info,
               "taches_pool_info": T.taches_pool_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "taches.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        name, field, val = line.split()
        cls = structs[name]
        want = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert int(val) == want, (name, field, int(val), want)
