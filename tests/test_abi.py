"""The C-ABI library loads and exports every entry point include/pwa.h declares (CPU only)."""
import os
import re

import pytest

import paper_1108_5882_amd as pwa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pwa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pwa_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert sorted(pwa.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    if not os.path.exists(pwa.LIB_PATH):
        pytest.skip("libpwa.so not built")
    lib = pwa.load()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_errors_without_gpu_or_context():
    if not os.path.exists(pwa.LIB_PATH):
        pytest.skip("libpwa.so not built")
    import ctypes
    lib = pwa.load()
    # null output pointer and null contexts are rejected without touching a device
    assert lib.pwa_create(None, 0, 0, None) == 1
    assert lib.pwa_destroy(None) == 0
    assert lib.pwa_set_mc_mode(None, 0, 0) == 1
    assert b"null" in lib.pwa_last_error(None)


def test_mlp_host_side_checks():
    """Parameter count of the 32 -> 256 -> 256 -> 1 network and argument checks
    that need no device."""
    if not os.path.exists(pwa.LIB_PATH):
        pytest.skip("libpwa.so not built")
    import ctypes
    lib = pwa.load()
    assert lib.pwa_mlp_param_count(32, 256) == 32 * 256 + 256 + 256 * 256 + 256 + 256 + 1 == 74497
    assert lib.pwa_mlp_param_count(0, 256) == -1
    assert lib.pwa_mlp_create(None, 0, 32, 256, 64, None) == 1
    h = ctypes.c_void_p()
    assert lib.pwa_mlp_create(ctypes.byref(h), 0, 0, 256, 64, None) == 1
    assert b"shape" in lib.pwa_mlp_last_error(None)
    assert lib.pwa_mlp_destroy(None) == 0
    assert lib.pwa_mlp_set_params(None, None, 0) == 1
