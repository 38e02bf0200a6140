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


def test_expsum_coefficients_match_the_oracle():
    """ttsg_expsum (host arithmetic in the library) and oracle.precond implement
    the same quadrature independently; both must give the same terms and meet
    the accuracy bound on the interval."""
    import numpy as np
    from oracle import precond as opc
    from paper_2409_09471_amd import ttsg
    for zmin, zmax, tol in [(1.0, 100.0, 1e-2), (197.0, 1.33e6, 1e-3), (0.3, 5e4, 1e-6)]:
        a, b = ttsg.expsum(zmin, zmax, tol)
        ao, bo = opc.expsum_coefficients(zmin, zmax, tol)
        assert len(a) == len(ao)
        assert np.allclose(a, ao, rtol=1e-13) and np.allclose(b, bo, rtol=1e-13)
        z = np.geomspace(zmin, zmax, 5001)
        assert np.max(np.abs(z * opc.expsum_eval(a, b, z) - 1.0)) <= tol
    with pytest.raises(ttsg.TTSGError) as e:
        ttsg.expsum(1.0, 1e6, 1e-8, max_terms=4)
    assert e.value.code == ttsg.ERR_CAPACITY
    with pytest.raises(ttsg.TTSGError) as e:
        ttsg.expsum(2.0, 1.0, 1e-2)
    assert e.value.code == ttsg.ERR_ARG


def test_workspace_queries_without_gpu(lib):
    """Workspace sizes are host arithmetic: they grow with the options that need
    buffers, and an unknown precision is rejected with TTSG_ERR_DTYPE."""
    from paper_2409_09471_amd import ttsg
    d = 4
    n = (ctypes.c_int32 * d)(16, 16, 16, 16)
    R = (ctypes.c_int32 * (d + 1))(1, 2, 2, 2, 1)
    rb = (ctypes.c_int32 * (d + 1))(1, 2, 2, 2, 1)
    rx = (ctypes.c_int32 * (d + 1))(1, 16, 32, 16, 1)
    rho = (ctypes.c_int32 * (d + 1))(1, 16, 52, 36, 1)
    opts = ttsg.SgmresOpts(maxit=40, q=1, tol=1e-6, round_tol=1e-8, stop_safety=0.1, rcond=1e-12)
    sizes = []
    for ext in [None, ttsg.SgmresExt(ls_mode=ttsg.LS_WHITEN), ttsg.SgmresExt(zeta=9, alpha=1, beta=1, ls_mode=0)]:
        if ext is not None and ext.zeta:
            a = (ctypes.c_double * 9)(*[1.0] * 9)
            b = (ctypes.c_double * 9)(*[float(j) for j in range(9)])
            ext.alpha = ctypes.cast(a, ctypes.c_void_p)
            ext.beta = ctypes.cast(b, ctypes.c_void_p)
        nb = ctypes.c_size_t(0)
        rc = lib.ttsg_sgmres_workspace_size(d, n, R, rb, 80, rho, rx, ctypes.byref(opts),
                                            ctypes.byref(ext) if ext is not None else None, ctypes.byref(nb))
        assert rc == 0
        sizes.append(nb.value)
    assert sizes[0] > 0 and sizes[1] > sizes[0] and sizes[2] > sizes[0]
    opts.precision = 7
    nb = ctypes.c_size_t(0)
    assert lib.ttsg_sgmres_workspace_size(d, n, R, rb, 80, rho, rx, ctypes.byref(opts), None,
                                          ctypes.byref(nb)) == ttsg.ERR_DTYPE
    assert lib.ttsg_kr_sketch_workspace_size(d, n, 80, R, rb, 7, ctypes.byref(nb)) == ttsg.ERR_DTYPE
    assert lib.ttsg_stta_sketch_workspace_size(d, n, rho, rx, None, rb, 0, ctypes.byref(nb)) == 0
    assert nb.value > 0
    # a rank of b above the STTA target ranks is a capacity error
    big = (ctypes.c_int32 * (d + 1))(1, 32, 2, 2, 1)
    opts.precision = 0
    assert lib.ttsg_sgmres_workspace_size(d, n, R, big, 80, rho, rx, ctypes.byref(opts), None,
                                          ctypes.byref(nb)) == ttsg.ERR_CAPACITY


def test_noalloc_sketch_rejects_shapes_beyond_its_buffer(lib):
    """ttsg_stta_sketch_noalloc refuses shapes whose scratch exceeds its static
    buffer with TTSG_ERR_WS before touching the device (d = 20, n = 128,
    ranks 128, rho 160, operator rank 3 needs about 264 MiB)."""
    from paper_2409_09471_amd import ttsg
    d = 20
    I = lambda v: (ctypes.c_int32 * len(v))(*v)  # noqa: E731
    n = I([128] * d)
    r = I([1] + [128] * (d - 1) + [1])
    rx = I([1] + [128] * (d - 1) + [1])
    rho = I([1, 128] + [160] * (d - 3) + [128, 1])
    R = I([1] + [3] * (d - 1) + [1])
    nb = ctypes.c_size_t(0)
    assert lib.ttsg_stta_sketch_workspace_size(d, n, rho, rx, R, r, 0, ctypes.byref(nb)) == 0
    assert nb.value > (128 << 20)
    fake = (ctypes.c_void_p * d)(*([16] * d))    # never dereferenced: the size check comes first
    rc = lib.ttsg_stta_sketch_noalloc(d, n, rho, fake, rx, fake, R, fake, r, fake, fake, fake, 0, None)
    assert rc == ttsg.ERR_WS
    lib.ttsg_last_error.restype = ctypes.c_char_p
    assert b"static buffer" in lib.ttsg_last_error()
    # the C2-shaped sketch of A v_k (d = 10, n = 64, ranks 64, rho 84, R = 3) fits
    d = 10
    n, r, rx = I([64] * d), I([1] + [64] * 9 + [1]), I([1] + [64] * 9 + [1])
    rho, R = I([1, 64] + [84] * 7 + [64, 1]), I([1] + [3] * 9 + [1])
    assert lib.ttsg_stta_sketch_workspace_size(d, n, rho, rx, R, r, 0, ctypes.byref(nb)) == 0
    assert nb.value <= (128 << 20)
