"""CPU checks of the C-ABI library: it loads and exports every symbol that
include/ttsg.h declares (no compute call is made without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2409_09471_amd", "libttsg.so")


def _declared():
    txt = open(os.path.join(ROOT, "include", "ttsg.h")).read()
    return sorted(set(re.findall(r"\b(ttsg_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2409_09471_amd import build_lib
        build_lib.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["ttsg_matvec", "ttsg_kr_sketch", "ttsg_stta_sketch", "ttsg_round_rand",
                     "ttsg_sgmres_solve"]:
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_lists_every_declared_symbol():
    from paper_2409_09471_amd import ttsg
    assert sorted(ttsg.EXPORTED) == _declared()


def test_version_and_error_strings(lib):
    lib.ttsg_version.restype = ctypes.c_char_p
    lib.ttsg_last_error.restype = ctypes.c_char_p
    assert b"gfx950" in lib.ttsg_version()
    assert isinstance(lib.ttsg_last_error(), bytes)


def test_argument_validation_without_gpu(lib):
    # bad shapes are rejected before any device work
    n = (ctypes.c_int32 * 3)(4, 4, 4)
    r = (ctypes.c_int32 * 4)(2, 1, 1, 1)     # r[0] != 1
    R = (ctypes.c_int32 * 4)(1, 2, 2, 1)
    p = (ctypes.c_void_p * 3)(1, 1, 1)
    rc = lib.ttsg_matvec(3, n, R, p, r, p, 0, p, None)
    assert rc == -1
    lib.ttsg_last_error.restype = ctypes.c_char_p
    assert b"boundary ranks" in lib.ttsg_last_error()


def test_autotune_table_round_trip(tmp_path):
    """The tile table is host state: saving, clearing and loading it needs no GPU."""
    from paper_2409_09471_amd import ttsg
    ttsg.autotune_clear()
    assert ttsg.autotune_save(str(tmp_path / "empty.txt")) == 0
    table = tmp_path / "t.txt"
    table.write_text("# comment\n0 6 6 12 0 1 1 0 3\n1 5 8 6 10 0 0 1 2\n0 1 1 1 1 0 0 0 9\n")
    assert ttsg.autotune_load(str(table)) == 2          # the variant-9 line is rejected
    out = tmp_path / "out.txt"
    assert ttsg.autotune_save(str(out)) == 2
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert sorted(lines) == sorted(["0 6 6 12 0 1 1 0 3", "1 5 8 6 10 0 0 1 2"])
    assert ttsg.autotune_clear() == 2
    with pytest.raises(ttsg.TTSGError):
        ttsg.autotune_load(str(tmp_path / "missing.txt"))
