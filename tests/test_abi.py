"""The C ABI: libeik.so loads without a GPU and exports every function that
include/eik.h declares; the binding marshals the same names."""
import os
import re

import pytest

import paper_1805_04198_amd as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "eik.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(eik_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("eik_solve", "eik_dd_solve", "eik_adjoint", "eik_last_error"):
        assert n in names
    assert sorted(E.SYMBOLS) == names


@pytest.mark.skipif(not os.path.exists(E.LIB_PATH), reason="libeik.so not built")
def test_library_exports_every_declared_symbol():
    L = E.load_library()
    for n in declared():
        assert hasattr(L, n), n
    assert L.eik_version().startswith(b"eik-mi355x")


@pytest.mark.skipif(not os.path.exists(E.LIB_PATH), reason="libeik.so not built")
def test_null_arguments_are_rejected_without_touching_a_device():
    L = E.load_library()
    st = L.eik_dd_solve(None, None, None, None, None, None, None, None, None)
    assert st == E.EIK_ERR_ARG
    assert b"NULL" in L.eik_last_error()
    assert L.eik_adjoint(None, None, None, None, None, None, None, None) == E.EIK_ERR_ARG
    assert L.eik_adjoint_batch(None, None, 0, None, None, None, None, None, None, 1, None, None) == E.EIK_ERR_ARG
