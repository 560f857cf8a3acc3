"""The C-ABI library loads on a machine without a GPU, exports every entry
point include/mask.h declares, and its host-only logic (level schedule,
argument checks) behaves as documented.  No compute call is made."""
import ctypes
import os
import re

import pytest

import paper_2208_02734_amd as pk
from oracle import mask_oracle as mo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "mask.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:mask_status|const char\*|double)\s+(mask_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(pk.LIB_PATH):
        pytest.skip("library not built")
    return pk.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["mask_build", "mask_query", "mask_free", "mask_plan_levels",
                     "mask_export_level", "mask_import", "mask_query_debug", "mask_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(_declared()) == sorted(pk.EXPORTED)


def _header_arg_counts():
    with open(os.path.join(ROOT, "include", "mask.h")) as f:
        text = f.read()
    out = {}
    for m in re.finditer(r"^\s*(?:mask_status|const char\*|double)\s+(mask_\w+)\s*\(([^)]*)\)",
                         text, re.M):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_every_entry_point_declares_its_argument_types(L):
    # without argtypes ctypes passes a Python int as a C int and masks a
    # 64-bit pointer to its low 32 bits
    counts = _header_arg_counts()
    for name in pk.EXPORTED:
        fn = getattr(L, name)
        assert fn.argtypes is not None, name
        assert len(fn.argtypes) == counts[name], name


def test_plan_levels_matches_oracle_and_paper(L):
    for n, lg, nc in [(80, 10, 5), (1600, 16, 8), (80000, 10, 5), (80000, 110, 55), (7, 10, 5)]:
        assert pk.mask_plan_levels(n, lg, nc) == mo.plan_levels(n, lg, nc)


def test_plan_levels_rejects_non_shrinking(L):
    with pytest.raises(pk.MaskError) as e:
        pk.mask_plan_levels(100, 4, 4)
    assert e.value.status == 1


def test_invalid_arguments_are_reported_without_device_work(L):
    h = ctypes.c_void_p()
    st = L.mask_build(None, None, None, None, ctypes.byref(h))
    assert st == 1 and h.value is None
    assert b"NULL" in L.mask_last_error()
    m = pk.mask_matrix()
    m.layout, m.n, m.dim, m.ld, m.x = 0, 100, 8, 0, 1234
    # level with more chunks than items
    p, lv = pk._params([(200, 2)], 5, 0, "l2", "fp32", 4, None)
    st = L.mask_build(ctypes.byref(m), ctypes.byref(p), None, None, ctypes.byref(h))
    assert st == 1 and b"more chunks than items" in L.mask_last_error()
    # group boundaries that do not end at n, or leave a group empty
    for off in ([0, 50, 99], [0, 50, 50, 100][:3], [0, 60, 60]):
        p, lv = pk._params([(2, 4)], 5, 0, "l2", "fp32", 4, None, group_off=off)
        st = L.mask_build(ctypes.byref(m), ctypes.byref(p), None, None, ctypes.byref(h))
        assert st == 1 and b"group_off" in L.mask_last_error(), off
    with pytest.raises(pk.MaskError):
        pk._params([(2, 4)], 5, 0, "l2", "fp32", 4, None, group_off=[0, 100])
    # unknown init, and k-means++ with L1
    p, lv = pk._params([(2, 4)], 5, 0, "l2", "fp32", 4, None)
    p.init = 7
    st = L.mask_build(ctypes.byref(m), ctypes.byref(p), None, None, ctypes.byref(h))
    assert st == 1 and b"init" in L.mask_last_error()
    p, lv = pk._params([(2, 4)], 5, 0, "l1", "fp32", 4, None, init="kmeans++")
    st = L.mask_build(ctypes.byref(m), ctypes.byref(p), None, None, ctypes.byref(h))
    assert st == 4
    # point query and relocation on a NULL index
    assert L.mask_point_query(None, ctypes.byref(m), None, None, None, None, None) == 1
    ng = ctypes.c_int32()
    assert L.mask_relocate(None, None, None, None, None, 0, ctypes.byref(ng), None, None) == 1
    # query on a NULL index
    st = L.mask_query(None, ctypes.byref(m), 10, 4, None, None, None)
    assert st == 1
    # k out of range is rejected before the index is touched
    assert L.mask_free(None) == 0


def test_unsupported_requests(L):
    h = ctypes.c_void_p()
    m = pk.mask_matrix()
    m.layout, m.n, m.dim, m.ld, m.x = 0, 1000, 300, 0, 1234
    p, lv = pk._params([(2, 10)], 5, 0, "l2", "fp32", 4, None)
    st = L.mask_build(ctypes.byref(m), ctypes.byref(p), None, None, ctypes.byref(h))
    assert st == 4
    # the low-precision forms are L2 only
    m.dim = 16
    for prec in ("bf16", "fp8"):
        p2, lv2 = pk._params([(2, 10)], 5, 0, "l1", prec, 4, None)
        assert L.mask_build(ctypes.byref(m), ctypes.byref(p2), None, None, ctypes.byref(h)) == 4


def test_csr_arguments_are_checked_before_device_work(L):
    h = ctypes.c_void_p()
    m = pk.mask_matrix()
    m.layout, m.n, m.dim = 1, 1000, 20_000
    m.indptr, m.indices, m.values, m.nnz = 1234, 1234, 1234, 5000
    p, lv = pk._params([(2, 10)], 5, 0, "l2", "fp32", 4, None)
    # more columns than the descent can stage in LDS
    st = L.mask_build(ctypes.byref(m), ctypes.byref(p), None, None, ctypes.byref(h))
    assert st == 4 and b"16384" in L.mask_last_error()
    m.dim = 1000
    # CSR data: L2 metric and FP32 form only
    p1, lv1 = pk._params([(2, 10)], 5, 0, "l1", "fp32", 4, None)
    assert L.mask_build(ctypes.byref(m), ctypes.byref(p1), None, None, ctypes.byref(h)) == 4
    p2, lv2 = pk._params([(2, 10)], 5, 0, "l2", "bf16", 4, None)
    assert L.mask_build(ctypes.byref(m), ctypes.byref(p2), None, None, ctypes.byref(h)) == 4
    # negative nnz and missing arrays are invalid
    m.nnz = -1
    assert L.mask_build(ctypes.byref(m), ctypes.byref(p), None, None, ctypes.byref(h)) == 1
    m.nnz, m.indices = 10, None
    assert L.mask_build(ctypes.byref(m), ctypes.byref(p), None, None, ctypes.byref(h)) == 1
    assert h.value is None
