"""The C ABI library loads and exports every function include/*.h declares
(no compute call: this runs without a GPU)."""
import ctypes as C
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2010_05975_amd", "libcfx.so")


def declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(cfx_[a-z0-9_]+)\s*\(", text))
    return names


def test_header_declares_the_boundary():
    need = {"cfx_create", "cfx_destroy", "cfx_getrf", "cfx_getrf_buffer_size", "cfx_getrs",
            "cfx_tslu", "cfx_version"}
    assert need <= declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcfx.so not built")
def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    missing = [n for n in sorted(declared()) if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcfx.so not built")
def test_version_string():
    lib = C.CDLL(LIB)
    lib.cfx_version.restype = C.c_char_p
    assert b"gfx950" in lib.cfx_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcfx.so not built")
def test_argument_errors_without_gpu():
    """Argument checks run on the host before any device work."""
    lib = C.CDLL(LIB)
    lib.cfx_getrf.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    assert lib.cfx_getrf(None, 4, None, 4, None, None, None, None, 0, None) == -1
    lib.cfx_create.argtypes = [C.c_void_p]
    assert lib.cfx_create(None) == -1
