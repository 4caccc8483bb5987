"""The C-ABI library loads on the host and exports every symbol its header declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2602_14450_amd", "libqcd.so")
HEADER = os.path.join(ROOT, "include", "qcd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qcd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("qcd_gauge_upload", "qcd_dslash", "qcd_bicgstab", "qcd_solve_mixed_ir"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqcd.so not built")
def test_library_exports_all_declared_symbols():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    lib.qcd_last_error.restype = ctypes.c_char_p
    assert lib.qcd_last_error() == b""


def test_fastdiv_matches_integer_division():
    # host mirror of the round-up multiplier division used for site decoding
    def make(d):
        s = 0
        while (1 << s) < d:
            s += 1
        m = ((1 << 32) * ((1 << s) - d)) // d + 1
        return m & 0xFFFFFFFF, s

    import random
    rnd = random.Random(3)
    for d in list(range(1, 130)) + [192, 255, 256, 1000, 4096, 12345]:
        m, s = make(d)
        for n in [0, 1, d - 1, d, d + 1, 2**31 - 1] + [rnd.randrange(2**31) for _ in range(2000)]:
            q = (((n * m) >> 32) + n) >> s
            assert q == n // d, (d, n)


def test_binding_declares_every_exported_symbol():
    # the Python binding's list of entry points matches the header
    import importlib.util
    spec = importlib.util.find_spec("paper_2602_14450_amd")
    src = open(spec.origin).read()
    for name in declared_functions():
        assert f'"{name}"' in src, name


def test_header_is_plain_c(tmp_path):
    # the boundary is a C ABI: the header compiles as C11 with no C++ or torch types
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "use.c"
    src.write_text('#include "qcd.h"\nint f(void) { qcd_ir_params p = {0}; return (int)p.inner_prec; }\n')
    r = subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-fsyntax-only", "-I", os.path.dirname(HEADER),
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqcd.so not built")
def test_binding_covers_exactly_the_header():
    # the Python binding names every entry point the header declares, and no other
    import sys
    sys.path.insert(0, ROOT)
    import paper_2602_14450_amd as q
    assert sorted(q.EXPORTED) == declared_functions()
