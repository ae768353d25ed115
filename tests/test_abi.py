"""The C-ABI library loads and exports every entry point include/fr.h
declares; the host-only name table agrees with the oracle's.  No compute
call is made (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2609_19190_amd", "libflashrad.so")
HDR = os.path.join(ROOT, "include", "fr.h")


def declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fr_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert {"fr_discretise", "fr_map", "fr_map_matrices", "fr_map_count", "fr_map_name",
            "fr_last_error"} <= set(names)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in fr.h but not exported"


def test_binding_lists_every_symbol():
    src = open(os.path.join(ROOT, "paper_2609_19190_amd", "binding.py")).read()
    for n in declared():
        assert n in src, f"{n} missing from the Python binding"


def test_name_table_matches_oracle(lib):
    from oracle import oracle as O
    lib.fr_map_name.restype = ctypes.c_char_p
    lib.fr_map_name.argtypes = [ctypes.c_uint32, ctypes.c_int32]
    lib.fr_map_count.argtypes = [ctypes.c_uint32]
    for fam in (63, 1, 2, 3, 12, 48, 33, 62):
        n = lib.fr_map_count(fam)
        assert n == O.map_count(fam)
        got = [lib.fr_map_name(fam, k).decode() for k in range(n)]
        assert got == O.map_names(fam)
        assert lib.fr_map_name(fam, n) is None
    assert lib.fr_map_count(64) == 0


def test_library_is_gfx950_code():
    blob = open(LIB, "rb").read()
    assert b"gfx950" in blob


def test_library_built_from_this_tree(lib):
    """fr_source_hash() names the sources the library was compiled from; the
    build runs before the tests, so it is this tree's."""
    import sys
    sys.path.insert(0, ROOT)
    from paper_2609_19190_amd import build as PB
    lib.fr_source_hash.restype = ctypes.c_char_p
    assert lib.fr_source_hash().decode() == PB.source_hash()


def test_one_error_message_for_every_family(lib):
    """A failing call of any family sets the one thread-local message that
    fr_last_error() and the family getters return; a later successful call
    clears it (fr_scalar runs on the host, so this needs no GPU)."""
    import numpy as np
    for n in ("fr_last_error", "fr_scalar_last_error", "fr_batch_last_error", "fr_server_last_error"):
        getattr(lib, n).restype = ctypes.c_char_p
    vol = np.zeros((4, 4, 4), np.int16)
    msk = np.zeros((4, 4, 4), np.uint8)
    msk[1:3, 1:3, 1:3] = 1
    sp = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    out = np.empty(93, np.float64)
    call = lambda m, cap: lib.fr_scalar(ctypes.c_void_p(vol.ctypes.data), 1, 4, 4, 4,
                                        ctypes.c_void_p(m.ctypes.data), sp, 2, ctypes.c_double(8.0),
                                        ctypes.c_double(float("nan")), ctypes.c_uint32(63),
                                        ctypes.c_void_p(out.ctypes.data), cap)
    assert call(np.zeros_like(msk), 93) < 0  # empty mask
    msg = lib.fr_last_error()
    assert msg
    for n in ("fr_scalar_last_error", "fr_batch_last_error", "fr_server_last_error"):
        assert getattr(lib, n)() == msg
    assert call(msk, 93) == 0
    assert lib.fr_last_error() == b""
