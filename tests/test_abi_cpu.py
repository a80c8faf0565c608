"""CPU checks of the C ABI: the library exports every function include/gmrf.h declares, the
binding mirrors them, argument validation happens before any device access, and without a
GPU the compute entry points fail loudly with GMRF_EDEVICE (there is no CPU fallback)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmrf.h")


def _ensure_lib():
    from paper_1312_1476_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    from paper_1312_1476_amd import _abi
    return _abi


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gmrf_[a-z0-9_]+)\s*\(", text)))


def test_header_functions_exported_and_bound():
    abi = _ensure_lib()
    names = declared_functions()
    assert len(names) >= 15
    handle = C.CDLL(abi.LIB_PATH)
    for nm in names:
        assert hasattr(handle, nm), f"{nm} declared in gmrf.h but not exported"
        assert nm in abi.SIGNATURES, f"{nm} has no binding"
    assert set(abi.SIGNATURES) == set(names)


def test_errors_without_device_or_with_bad_args():
    abi = _ensure_lib()
    L = abi.lib()
    h = C.c_void_p()
    shape = (C.c_int64 * 2)(8, 8)
    # argument errors are reported before touching the device
    assert L.gmrf_op_create_lattice(0, shape, 1, 0.1, 1.0, 0, 0, C.byref(h)) == abi.GMRF_EINVAL
    assert L.gmrf_op_create_lattice(2, shape, 3, 0.1, 1.0, 0, 0, C.byref(h)) == abi.GMRF_EINVAL
    assert L.gmrf_op_create_lattice(2, shape, 1, 0.1, -1.0, 0, 0, C.byref(h)) == abi.GMRF_EINVAL
    assert b"order" in L.gmrf_last_error() or b"tau" in L.gmrf_last_error()
    assert L.gmrf_sample(None, None, 1, 1e-8, 10, 0, None, None, None) == abi.GMRF_EINVAL
    # NULL handles of the later entry points: refused before any device call
    assert L.gmrf_solve(None, None, 1, 1e-8, 10, 0, None, None, None) == abi.GMRF_EINVAL
    assert L.gmrf_sample_two_pass(None, None, 1, 1e-8, 10, None, None, None) == abi.GMRF_EINVAL
    assert L.gmrf_sample_noalloc(None, None, 1, 1e-8, 10, 0, None, None, None) == abi.GMRF_EINVAL
    assert L.gmrf_op_set_diagonal(None, None) == abi.GMRF_EINVAL
    assert L.gmrf_op_set_ichol_precond(None, 1, -1.0, None) == abi.GMRF_EINVAL
    assert L.gmrf_ichol_info(None, None, None, None) == abi.GMRF_EINVAL
    assert L.gmrf_logdet_coloured(None, 2, 10, 0, None, 1, None, None, None, None) == abi.GMRF_EINVAL
    assert L.gmrf_distance_colouring(None, 1, None, None) == abi.GMRF_EINVAL
    assert L.gmrf_strerror(abi.GMRF_ENOTSPD).startswith(b"operator is not")
    import torch
    if not torch.cuda.is_available():
        st = L.gmrf_op_create_lattice(2, shape, 1, 0.1, 1.0, 0, 0, C.byref(h))
        assert st == abi.GMRF_EDEVICE
        assert L.gmrf_rademacher(1, 100, 1, C.c_void_p(1), None) == abi.GMRF_EDEVICE


def test_missing_library_fails_loudly(monkeypatch):
    from paper_1312_1476_amd import _abi
    monkeypatch.setattr(_abi, "LIB_PATH", "/nonexistent/libgmrf.so")
    monkeypatch.setattr(_abi, "_lib", None)
    with pytest.raises(ImportError):
        _abi.lib()


def test_product_never_touches_oracle():
    pkg = os.path.join(ROOT, "paper_1312_1476_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f), errors="replace").read()
                assert not re.search(r"\bimport\s+oracle\b|\bfrom\s+oracle\b|oracle/", txt), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith(".py"):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert not re.search(r"\bimport\s+paper_1312_1476_amd|\bfrom\s+paper_1312_1476_amd", txt), f
