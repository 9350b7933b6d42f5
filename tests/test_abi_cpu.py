"""The C-ABI library loads and exports every symbol the header declares; host-side
argument checks fail cleanly without touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1510_06916_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "nxgraph.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nxg_[a-z_0-9]+)\s*\(", text)) - {"nxg_alloc_fn", "nxg_free_fn"})


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libnxgraph.so is not built")
    return _lib.lib()


def test_every_declared_symbol_is_exported(L):
    syms = header_symbols()
    assert len(syms) >= 8
    for s in syms:
        assert hasattr(L, s), s
        assert s in _lib.SIGNATURES, "binding lacks " + s


def test_version_and_error_text(L):
    hdr = open(os.path.join(ROOT, "include", "nxgraph.h")).read()
    assert L.nxg_abi_version() == int(re.search(r"#define NXG_ABI_VERSION (\d+)", hdr).group(1))
    assert L.nxg_last_error() == b""


def test_host_side_argument_errors(L):
    out = ctypes.c_void_p(123)
    assert L.nxg_dsss_build(None, None, ctypes.byref(out)) == _lib.NXG_EINVAL
    assert out.value is None
    assert b"desc" in L.nxg_last_error()
    d = _lib.BuildDesc(n=0, m=0)
    assert L.nxg_dsss_build(ctypes.byref(d), None, ctypes.byref(out)) == _lib.NXG_EINVAL
    d = _lib.BuildDesc(n=10, m=-1)
    assert L.nxg_dsss_build(ctypes.byref(d), None, ctypes.byref(out)) == _lib.NXG_EINVAL
    d = _lib.BuildDesc(n=10, m=5)  # null edge arrays
    assert L.nxg_dsss_build(ctypes.byref(d), None, ctypes.byref(out)) == _lib.NXG_EINVAL
    d = _lib.BuildDesc(n=10, m=0, flags=0x1000)
    assert L.nxg_dsss_build(ctypes.byref(d), None, ctypes.byref(out)) == _lib.NXG_EINVAL
    d = _lib.BuildDesc(n=10, m=0, flags=_lib.NXG_BUILD_PAIRS | _lib.NXG_BUILD_SYMMETRIZE)
    assert L.nxg_dsss_build(ctypes.byref(d), None, ctypes.byref(out)) == _lib.NXG_EINVAL
    d = _lib.BuildDesc(n=10, m=0, flags=_lib.NXG_BUILD_SYMMETRIZE | _lib.NXG_BUILD_KEEP_PERM)
    assert L.nxg_dsss_build(ctypes.byref(d), None, ctypes.byref(out)) == _lib.NXG_EINVAL
    d = _lib.BuildDesc(n=10, m=0, flags=_lib.NXG_BUILD_SCATTER | _lib.NXG_BUILD_RELABEL)
    assert L.nxg_dsss_build(ctypes.byref(d), None, ctypes.byref(out)) == _lib.NXG_EINVAL
    d = _lib.BuildDesc(n=10, m=0, interval=11)
    assert L.nxg_dsss_build(ctypes.byref(d), None, ctypes.byref(out)) == _lib.NXG_EINVAL
    assert L.nxg_dsss_destroy(None) == _lib.NXG_OK
    assert L.nxg_run(None, None, None, None) == _lib.NXG_EINVAL
    assert L.nxg_dsss_info_get(None, None) == _lib.NXG_EINVAL
    bad_free = _lib.FREE_FN(0)
    assert L.nxg_set_allocator(_lib.ALLOC_FN(lambda b, s, c: None), bad_free, None) == _lib.NXG_EINVAL


def test_package_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libnxgraph.so")
    with pytest.raises(RuntimeError, match="not built"):
        _lib.lib()
