"""The C-ABI library loads and exports every symbol the public header declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]
LIB = os.path.join(ROOT, "paper_2203_11025_amd", "libhelm.so")


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"^typedef[^;]*;", "", text, flags=re.M | re.S)  # function-pointer types
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M):
            name = m.group(1)
            if name not in ("if", "for", "while", "return", "sizeof", "defined"):
                names.append(name)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ["helm_setup", "helm_apply", "helm_sl_vcycle", "helm_fgmres_solve",
                     "helm_destroy", "helm_last_error"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhelm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhelm.so not built")
def test_last_error_callable_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.helm_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.helm_last_error(), bytes)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhelm.so not built")
def test_binding_names_match_header():
    from paper_2203_11025_amd import helm, unet

    names = declared_functions()
    for n in helm.EXPORTS + unet.EXPORTS:
        assert n in names
