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
def test_auto_tail_rule_needs_no_gpu():
    """AUTO keeps an FP64 tail for IRs of >= 2^18 taps or more than 1024
    chunk sums per output (chunk = min(B, 256)); explicit tails win."""
    from paper_2401_01607_amd import taches as T
    cases = [(32, 32_768, 0), (32, 32_769, 1), (64, 65_536, 0), (64, 65_537, 1), (128, 131_072, 0),
             (128, 131_073, 1), (256, 262_143, 0), (512, 262_143, 0), (512, 262_144, 1), (1024, 262_143, 0),
             (64, 1024, 0)]
    for B, L, want in cases:
        c = T.taches_config_default(B, L)
        assert T.taches_tail_is_fp64(c) == want, (B, L)
    c = T.taches_config_default(32, 1 << 20)
    c.tail = T.TACHES_TAIL_FP32
    assert T.taches_tail_is_fp64(c) == 0
    c = T.taches_config_default(512, 16)
    c.tail = T.TACHES_TAIL_FP64
    assert T.taches_tail_is_fp64(c) == 1
    c.max_ir_len = 0
    assert T.taches_tail_is_fp64(c) == T.TACHES_EINVAL


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
               "taches_pool_info": T.taches_pool_info, "taches_server_tick_info": T.taches_server_tick_info,
               "taches_server_stats": T.taches_server_stats}
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
