"""The C-ABI library loads and exports every function include/scdg.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_1911_02366_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1911_02366_amd import build
        build.build()
    return _lib.LIB_PATH


def declared_functions():
    text = open(os.path.join(ROOT, "include", "scdg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scdg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for call in ("scdg_assemble", "scdg_factor", "scdg_condense", "scdg_condense_rhs",
                 "scdg_solve_condensed", "scdg_backsolve", "scdg_solve", "scdg_residual"):
        assert call in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol(lib_path):
    from paper_1911_02366_amd import _lib
    assert sorted(_lib.EXPORTED) == declared_functions()
    _lib.load(lib_path)


def test_status_strings_without_gpu(lib_path):
    from paper_1911_02366_amd import _lib
    lib = _lib.load(lib_path)
    assert lib.scdg_status_string(0) == b"ok"
    assert lib.scdg_status_string(-5) == b"singular pivot"


def test_create_rejects_bad_structure_without_gpu(lib_path):
    # argument checks return before any device call
    from paper_1911_02366_amd import _lib
    lib = _lib.load(lib_path)
    handle = ctypes.c_void_p()
    assert lib.scdg_plan_create(ctypes.byref(handle), None, None, -1) == -1
