"""Host-side checks of the C ABI: the library loads, exports every entry point
include/mad.h declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import os
import re

import pytest

import paper_1506_03872_amd as mad

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mad.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(mad_\w+|mips_\w+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declarations_are_known():
    names = declared_functions()
    assert "mad_plan_topk" in names and "mad_topk" in names
    assert set(names) == set(mad.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = mad.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_invalid_arguments_rejected_without_gpu():
    L = mad.lib()
    h = C.c_void_p()
    # NULL plan pointer
    assert L.mad_plan_create_dense(None, 10, None, 10, 4, 0, None, None) == \
        mad.MAD_EINVAL
    # bad shapes are checked before any device call
    assert L.mad_plan_create_dense(None, 0, None, 10, 4, 0, None,
                                   C.byref(h)) == mad.MAD_EINVAL
    assert L.mad_plan_create_dense(None, 10, None, 10, 0, 0, None,
                                   C.byref(h)) == mad.MAD_EINVAL
    assert L.mad_plan_create_dense(None, 1 << 31, None, 10, 4, 0, None,
                                   C.byref(h)) == mad.MAD_EINVAL
    # NULL inputs
    assert L.mad_plan_create_dense(None, 10, None, 10, 4, 0, None,
                                   C.byref(h)) == mad.MAD_EINVAL
    assert b"device" in L.mad_last_error()
    # calls on a NULL plan
    assert L.mad_plan_topk(None, 1, 10, 1, 0, None, None, None) == mad.MAD_EINVAL
    assert L.mad_plan_refresh(None, None) == mad.MAD_EINVAL
    assert L.mad_plan_stats(None, None, None, None, None, None) == mad.MAD_EINVAL
    L.mad_plan_destroy(None)  # no-op


def test_sparse_entry_rejects_null_output():
    L = mad.lib()
    rc = L.mad_plan_create_csr(None, None, None, 1, None, None, None, 1, 1,
                               0, None, None)
    assert rc in (mad.MAD_EINVAL, mad.MAD_EUNSUPPORTED)
