"""The C-ABI library loads and exports every function include/rw.h declares
(no compute: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rw.h")
LIB = os.path.join(ROOT, "paper_2108_07205_amd", "librw.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rw_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("rw_ctx_create", "rw_wall_build", "rw_refine", "rw_coarsen", "rw_solve",
                     "rw_hbs_apply", "rw_nodes", "rw_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librw.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    import paper_2108_07205_amd as rw
    assert set(declared_functions()) == set(rw.EXPORTED_SYMBOLS)


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2108_07205_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
