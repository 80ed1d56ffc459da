"""The C-ABI library loads and exports every entry point include/l1_alm.h
declares (no GPU work)."""
import os
import re

import paper_1007_3753_amd as pkg
from paper_1007_3753_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "l1_alm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"\b(l1_alm_[a-z_]+)\s*\(", src))


def test_header_declares_the_boundary():
    names = _declared()
    assert {"l1_alm_plan", "l1_alm_solve", "l1_alm_backward"} <= names
    assert names == set(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = pkg.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.l1_alm_last_error() == b""


def test_desc_layout_matches_header():
    # the ctypes mirror has the field order and types of l1_alm_desc
    src = open(os.path.join(ROOT, "include", "l1_alm.h")).read()
    body = src[src.index("typedef struct {"):src.index("} l1_alm_desc;")]
    decl = re.findall(r"^\s*(int|double)\s+(\w+);", body, flags=re.M)
    fields = _lib.l1_alm_desc._fields_
    assert len(decl) == len(fields)
    for (ctype, cname), (pname, ptype) in zip(decl, fields):
        assert (ctype == "int") == (ptype.__name__ == "c_int"), cname
        assert cname == pname or (cname, pname) == ("lambda", "lam")
