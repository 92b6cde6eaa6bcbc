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


def _fake_context(prec="f32", k=4):
    """A Context object with no library handle, for the binding's own argument checks."""
    import numpy as np
    from paper_1108_5882_amd import _lib
    c = _lib.Context.__new__(_lib.Context)
    c.device, c.prec, c.k = 0, {"f32": _lib.F32, "f64": _lib.F64}[prec], k
    c.real = np.float32 if prec == "f32" else np.float64
    c.cplx = np.complex64 if prec == "f32" else np.complex128
    c._borrowed, c._vbuf, c._obuf = {}, None, None
    c.h = None
    return c


def test_binding_rejects_host_tensors_for_device_arguments():
    """The device-side calls of the binding refuse CPU tensors, wrong dtypes and
    wrong sizes before anything reaches the library (no device needed)."""
    torch = pytest.importorskip("torch")
    from paper_1108_5882_amd import _lib
    c = _fake_context(k=4)
    with pytest.raises(TypeError):
        c.nll_grad_async(torch.zeros(8, dtype=torch.float64), torch.zeros(10, dtype=torch.float64))
    with pytest.raises(TypeError):
        c.nll_batch_async(torch.zeros((2, 8), dtype=torch.float64), torch.zeros((2, 10), dtype=torch.float64))
    with pytest.raises(TypeError):
        c._check_device_tensor(torch.zeros(8, dtype=torch.float32), "V_dev", torch.float64)
    with pytest.raises(TypeError):
        c.set_amplitudes("data", torch.zeros((3, 4), dtype=torch.complex64), borrow=True)
    with pytest.raises(TypeError):
        c.set_amplitudes("data", __import__("numpy").zeros((3, 4), dtype="complex64"), borrow=True)
    # V of the wrong length for the synchronous calls
    with pytest.raises(ValueError):
        c._stage_v(__import__("numpy").ones(3, dtype=complex))
    vp, op = c._stage_v(__import__("numpy").arange(4) * (1 + 1j))
    assert list(c._vbuf) == [0, 0, 1, 1, 2, 2, 3, 3] and vp and op
    assert _lib.BORROW == 2


def test_kinematic_context_host_checks():
    """Argument checks of the kinematic context that need no device."""
    if not os.path.exists(pwa.LIB_PATH):
        pytest.skip("libpwa.so not built")
    import ctypes
    import numpy as np
    lib = pwa.load()
    sp = np.array([0, 2, 5], dtype=np.int32)
    h = ctypes.c_void_p()
    assert lib.pwa_kin_create(None, 0, 3, sp.ctypes.data, None) == 1
    assert lib.pwa_kin_create(ctypes.byref(h), 0, 3, sp.ctypes.data, None) == 6     # spin 5 not supported
    assert b"spin" in lib.pwa_kin_last_error(None)
    assert lib.pwa_kin_create(ctypes.byref(h), 0, 0, sp.ctypes.data, None) == 1
    assert lib.pwa_kin_destroy(None) == 0
    assert lib.pwa_kin_set_mode(None, 0) == 1
