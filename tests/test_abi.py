"""CPU-side checks of the boundary: the HIP library loads and exports every
function include/rc.h declares, the binding's record layouts match the ABI,
and the product package never reaches the oracle."""
import ctypes
import os
import re

from paper_1308_3203_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rc.h")).read()
    return sorted(set(re.findall(r"^\s*(?:rc_status|const char\*)\s+(rc_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    assert "rc_check" in names and "rc_prog_load" in names and len(names) >= 15


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(B.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(B.EXPORTS) == declared_functions()


def test_binding_loads_library_and_layouts():
    lib = B.load_library()
    assert lib.rc_last_error() == b""
    assert B.RECORD_DTYPE.itemsize == 40 and B.SUMMARY_DTYPE.itemsize == 40


def test_context_creation_fails_cleanly_without_device():
    import torch
    if torch.cuda.is_available():
        return
    lib = B.load_library()
    out = ctypes.c_void_p()
    st = lib.rc_ctx_create(0, None, ctypes.byref(out))
    assert st == B.RC_E_HIP and b"device" in lib.rc_last_error()


def test_product_code_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_1308_3203_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "oracle.h" not in text and "liboracle" not in text, f
