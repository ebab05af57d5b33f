"""CPU-side checks of the C ABI library: it is built, loads, and exports every
entry point declared in include/pdschur.h (no compute call without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pdschur.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pd_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_four_core_entry_points():
    names = _declared()
    for core in ["pd_schur_build", "pd_collision_update", "pd_global_solve",
                 "pd_local_step_region"]:
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2008_01541_amd import library_path, load_library
    assert os.path.exists(library_path()), "build the library first (__graft_entry__.build())"
    lib = load_library()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert missing == []


def test_binding_names_match_abi():
    from paper_2008_01541_amd._lib import _SIGS
    declared = set(_declared())
    assert set(_SIGS) <= declared
    assert declared - set(_SIGS) <= {"pd_last_error"}


def test_null_arguments_rejected_without_gpu():
    from paper_2008_01541_amd import load_library
    lib = load_library()
    assert lib.pd_schur_build(None, None, None) == -1
    out = ctypes.c_void_p()
    assert lib.pd_schur_build(None, None, ctypes.byref(out)) == -1
    assert lib.pd_destroy(None) == -1
    assert lib.pd_query(None, None, None, None, None, None) == -1
