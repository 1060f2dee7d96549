"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/gs2d.h declares, and its pure-host calls validate
arguments."""
import ctypes
import os
import re

import pytest

from paper_2505_09324_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(gs2d_[a-z0-9_]+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgs2d.so not built (run python -m paper_2505_09324_amd.build)")
    return _lib.lib()


def test_every_declared_symbol_is_exported_and_bound(lib):
    declared = _declared()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(_lib.exported_symbols())


def test_status_strings(lib):
    assert _lib.status_str(0) == "ok"
    assert "capacity" in _lib.status_str(-3)


def test_workspace_bytes_validation(lib):
    ok = _lib.make_shape(1920, 1080, 30000, 16)
    n = _lib.workspace_bytes(ok)
    assert n > 0 and n % 256 == 0
    bigger = _lib.make_shape(1920, 1080, 30000, 16, max_pairs=ok.max_pairs * 2)
    assert _lib.workspace_bytes(bigger) > n
    for bad in (_lib.Shape(0, 10, 5, 16, 100, 1), _lib.Shape(10, 10, 0, 16, 100, 1),
                _lib.Shape(10, 10, 70000, 16, 100, 1), _lib.Shape(10, 10, 5, 12, 100, 1),
                _lib.Shape(10, 10, 5, 16, 0, 1), _lib.Shape(8192, 8192, 5, 8, 100, 1),
                _lib.Shape(64, 64, 5, 8, 100, 2), _lib.Shape(64, 64, 5, 16, 100, 3),
                _lib.Shape(64, 64, 5, 32, 100, 8)):
        assert lib.gs2d_workspace_bytes(ctypes.byref(bad)) == 0
    # the limits themselves: N = 65536 and 256 x 256 tiles are accepted, one
    # Gaussian or one tile row / column more is not
    assert lib.gs2d_workspace_bytes(ctypes.byref(_lib.make_shape(2048, 2048, 65536, 8))) > 0
    for bad in (_lib.make_shape(2048, 2048, 65537, 8), _lib.make_shape(2049, 2048, 100, 8),
                _lib.make_shape(2048, 2049, 100, 8)):
        assert lib.gs2d_workspace_bytes(ctypes.byref(bad)) == 0


def test_bins_view_checks_space_and_alignment(lib):
    s = _lib.make_shape(64, 64, 10, 16)
    need = _lib.workspace_bytes(s)
    b = _lib.Bins()
    fake = 1 << 40  # never dereferenced by this host-only call
    assert lib.gs2d_bins_view(ctypes.byref(s), ctypes.c_void_p(fake), need, ctypes.byref(b)) == 0
    assert b.n_tiles == 16 and b.tiles_x == 4 and b.tiles_y == 4
    assert lib.gs2d_bins_view(ctypes.byref(s), ctypes.c_void_p(fake), need - 1, ctypes.byref(b)) == -2
    assert lib.gs2d_bins_view(ctypes.byref(s), ctypes.c_void_p(fake + 4), need, ctypes.byref(b)) == -1
    assert lib.gs2d_bins_view(ctypes.byref(s), None, need, ctypes.byref(b)) == -1


def test_null_arguments_rejected_before_any_launch(lib):
    s = _lib.make_shape(64, 64, 10, 16)
    need = _lib.workspace_bytes(s)
    fake = ctypes.c_void_p(1 << 40)
    assert lib.gs2d_project_bin(ctypes.byref(s), None, fake, fake, need, None) == -1
    assert lib.gs2d_render_fwd(ctypes.byref(s), fake, need, None, None, None, None, None, None) == -1
    # dl_dimg without a target is invalid
    assert lib.gs2d_render_fwd(ctypes.byref(s), fake, need, fake, None, None, fake, None, None) == -1
    assert lib.gs2d_render_bwd(ctypes.byref(s), fake, need, fake, None, fake, fake, fake, None) == -1
    cfg = _lib.adam_cfg()
    assert lib.gs2d_adam_step(0, fake, fake, fake, fake, fake, fake, fake, fake, fake,
                              ctypes.byref(cfg), None, 0, None) == -1
