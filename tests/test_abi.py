"""The C-ABI library loads and exports every function include/mlcc.h declares
(CPU only: no device call is made)."""
import ctypes
import os
import re

from paper_2006_05226_amd import mlcc


def header_functions(root):
    text = open(os.path.join(root, "include", "mlcc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mlcc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(root):
    names = header_functions(root)
    assert len(names) >= 18
    lib = ctypes.CDLL(mlcc.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(mlcc.EXPORTS) == names


def test_binding_declares_signatures():
    lib = mlcc.load()
    for n in mlcc.EXPORTS:
        assert getattr(lib, n).argtypes is not None


def test_create_error_without_gpu_is_reported():
    """Without a device the context call fails with a status, never a crash."""
    import torch
    if torch.cuda.is_available():
        return
    lib = mlcc.load()
    h = ctypes.c_void_p()
    st = lib.mlcc_context_create(0, None, 0, ctypes.byref(h))
    assert st < 0
    assert len(lib.mlcc_last_error(None)) > 0
