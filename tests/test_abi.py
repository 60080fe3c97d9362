"""CPU checks of the C ABI: the library loads and exports every symbol the header declares."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fe.h")
LIB = os.path.join(ROOT, "paper_2607_03413_amd", "libfe.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fe_apply", "patch_fdm_inverse", "pcg_solve", "fe_problem_create", "fe_dss",
                     "fe_gather", "fe_assemble", "fe_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfe.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if " T " in line)
    assert set(declared_functions()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfe.so not built")
def test_error_path_without_gpu_work():
    """Argument validation happens before any device call."""
    lib = ctypes.CDLL(LIB)
    lib.fe_last_error.restype = ctypes.c_char_p
    lib.fe_problem_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.fe_problem_create(None, None, None) == -1
    assert b"null" in lib.fe_last_error()
    lib.fe_apply.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int, ctypes.c_void_p]
    assert lib.fe_apply(None, None, None, 0, None) == -1


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2607_03413_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
