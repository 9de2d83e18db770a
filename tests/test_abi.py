"""The C-ABI library loads and exports every entry point its header declares;
argument checks that need no device behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def _lib_path():
    from paper_2305_15693_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    return B.LIB


def declared_functions():
    names = []
    for fn in sorted(os.listdir(HEADER_DIR)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(fresco_[a-z0-9_]+)\s*\(",
                             text, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ["fresco_create", "fresco_destroy", "fresco_structure_factor",
                     "fresco_loss_grad", "fresco_error_string"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_invalid_arguments_without_device():
    lib = ctypes.CDLL(_lib_path())
    lib.fresco_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.fresco_create.restype = ctypes.c_int
    assert lib.fresco_create(None, None, None) == -1
    h = ctypes.c_void_p()
    assert lib.fresco_create(ctypes.byref(h), None, None) == -1
    assert h.value is None
    lib.fresco_destroy.argtypes = [ctypes.c_void_p]
    assert lib.fresco_destroy(None) == 0
    lib.fresco_error_string.restype = ctypes.c_char_p
    assert lib.fresco_error_string(-5) == b"non-finite position"
    for fn in ["fresco_structure_factor", "fresco_loss_grad", "fresco_loss_grad_async"]:
        f = getattr(lib, fn)
        f.restype = ctypes.c_int
        assert f(None, None, None, None) == -1


def test_problem_validation_without_device():
    """Invalid problems are rejected before any device work."""
    from paper_2305_15693_amd import fresco as F
    lib = F.lib()

    def create(**kw):
        p = F.Problem()
        p.dim, p.dtype, p.n = 2, F.F32, 100
        p.box[0] = p.box[1] = 10.0
        p.kmax[0] = p.kmax[1] = 4
        p.k_cut, p.tol, p.upsampfac = 4.0, 1e-6, 2.0
        for k, v in kw.items():
            if k == "box":
                p.box[0] = v
            else:
                setattr(p, k, v)
        h = ctypes.c_void_p()
        return lib.fresco_create(ctypes.byref(h), ctypes.byref(p), None)

    assert create(dim=4) == F.EINVAL
    assert create(dtype=7) == F.EINVAL
    assert create(n=0) == F.EINVAL
    assert create(box=-1.0) == F.EINVAL
    assert create(tol=0.5) == F.EINVAL
    assert create(tol=0.0) == F.EINVAL
    assert create(upsampfac=1.25) == F.EINVAL
    assert create(weight_mode=9) == F.EINVAL
    assert create(n=1 << 40) == F.ENOTSUP
