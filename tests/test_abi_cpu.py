"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function include/odmd.h declares, and
reject bad arguments on the host before any device call.  The product
package must never reach the CPU oracle.
"""
import ctypes
import os
import re

import pytest

from paper_2311_18715_amd import odmd as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "odmd.h")

needs_lib = pytest.mark.skipif(not os.path.exists(B.LIB_PATH), reason="libodmd.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(odmd_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for core in ["odmd_create", "odmd_update", "odmd_eigs", "odmd_predict", "odmd_destroy"]:
        assert core in names
    assert set(names) == set(B.EXPORTS)


@needs_lib
def test_library_exports_every_declared_symbol():
    L = B.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


@needs_lib
def test_state_bytes_is_host_only():
    L = B.lib()
    n64 = L.odmd_state_bytes(160000, 40, B.F64, B.F64)
    n32 = L.odmd_state_bytes(160000, 40, B.F32, B.F32)
    assert n64 > 160000 * 40 * 8 and n32 > 160000 * 40 * 4
    assert n64 - n32 >= 160000 * 41 * 4 - 4096
    assert L.odmd_state_bytes(0, 4, B.F64, B.F64) == 0
    assert L.odmd_state_bytes(100, 65, B.F64, B.F64) == 0       # above the rank cap
    assert L.odmd_state_bytes(10, 11, B.F64, B.F64) == 0        # r_max > n
    assert L.odmd_state_bytes(100, 8, B.F64, B.F32) == 0        # io must match basis
    assert L.odmd_state_bytes(100, 8, B.BF16, B.F32) > 0        # BF16 basis, FP32 snapshots
    assert L.odmd_state_bytes(100, 8, B.BF16, B.BF16) == 0      # BF16 snapshots are not offered
    # general pairs: a second stored-column set (B = T R), its state and records
    g64 = L.odmd_state_bytes_general(160000, 40, B.F64, B.F64)
    assert g64 - n64 >= 160000 * 56 * 8
    assert L.odmd_state_bytes_general(100, 65, B.F64, B.F64) == 0
    assert L.odmd_state_bytes_general(100, 8, B.BF16, B.F32) > L.odmd_state_bytes(100, 8, B.BF16, B.F32)


@needs_lib
def test_create_general_rejects_bad_arguments():
    L = B.lib()
    h = ctypes.c_void_p(12345)
    assert L.odmd_create_general(100, 65, 1e-8, B.F64, B.F64, None, None, 0, ctypes.byref(h)) == 1
    assert h.value is None
    assert L.odmd_create_general(100, 4, 1e-8, B.F64, B.F32, None, None, 0, ctypes.byref(h)) == 1
    assert L.odmd_create_general(100, 4, 1e-8, B.F64, B.F64, None, None, 0, None) == 1


@needs_lib
@pytest.mark.parametrize("n,r_max,tol", [
    (0, 4, 1e-8), (-5, 4, 1e-8), (100, 0, 1e-8), (100, 65, 1e-8), (5, 6, 1e-8),
    (100, 4, -1e-3), (100, 4, 1.0), (100, 4, float("nan")), (100, 4, float("inf")),
])
def test_create_rejects_bad_arguments(n, r_max, tol):
    h = ctypes.c_void_p(12345)
    assert B.lib().odmd_create(n, r_max, tol, ctypes.byref(h)) == 1     # ODMD_EINVAL
    assert h.value is None                                              # *h cleared


@needs_lib
def test_null_arguments_are_rejected():
    L = B.lib()
    assert L.odmd_create(100, 4, 1e-8, None) == 1
    assert L.odmd_update(None, None, None) == 1
    assert L.odmd_sync(None) == 1
    assert L.odmd_destroy(None) == 1
    assert L.odmd_release(None) == 1
    assert L.odmd_predict(None, 5, None) == 1
    assert L.odmd_update_batch(None, None, None, 1) == 1
    assert L.odmd_update_batch_noalloc(None, None, None, 1) == 1
    r = ctypes.c_int32()
    assert L.odmd_eigs(None, 4, ctypes.byref(r), None, None, None, None) == 1
    assert L.odmd_get_info(None, None) == 1
    assert L.odmd_profile(None, 1) == 1
    assert L.odmd_profile_latency(None, 1) == 1


@needs_lib
def test_workspace_checks_happen_before_device_use():
    L = B.lib()
    h = ctypes.c_void_p()
    need = L.odmd_state_bytes(1000, 8, B.F64, B.F64)
    # too small a workspace, misaligned workspace, bytes without a buffer
    assert L.odmd_create_ex(1000, 8, 1e-8, B.F64, B.F64, None, ctypes.c_void_p(4096), need - 1,
                            ctypes.byref(h)) == 2
    assert L.odmd_create_ex(1000, 8, 1e-8, B.F64, B.F64, None, ctypes.c_void_p(4096 + 8), need,
                            ctypes.byref(h)) == 1
    assert L.odmd_create_ex(1000, 8, 1e-8, B.F64, B.F64, None, None, 64, ctypes.byref(h)) == 1


@needs_lib
def test_status_strings():
    L = B.lib()
    for code in range(8):
        assert len(L.odmd_status_str(code)) > 0
    assert L.odmd_status_str(99) == b"unknown status"


def test_product_never_reaches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2311_18715_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, re.M), f
                assert "odmd_oracle" not in text, f


@needs_lib
def test_launch_shape_entry_points_are_host_checked():
    L = B.lib()
    t, r, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert L.odmd_default_shape(160000, ctypes.byref(t), ctypes.byref(r), ctypes.byref(c)) == 0
    assert (t.value, r.value, c.value) == (512, 256, 256)
    assert L.odmd_default_shape(131071, ctypes.byref(t), ctypes.byref(r), ctypes.byref(c)) == 0
    assert (t.value, r.value, c.value) == (256, 512, 512)
    assert L.odmd_default_shape(0, ctypes.byref(t), ctypes.byref(r), ctypes.byref(c)) == 1
    assert L.odmd_default_shape(10, None, ctypes.byref(r), ctypes.byref(c)) == 1
    # the default shape's bytes equal the plain entry points'
    for n in (100, 160000):
        d = B.default_shape(n)
        assert L.odmd_state_bytes_shaped(n, 16, B.F32, B.F32, *d, 0) == \
            L.odmd_state_bytes(n, 16, B.F32, B.F32)
        assert L.odmd_state_bytes_shaped(n, 16, B.F64, B.F64, *d, 1) == \
            L.odmd_state_bytes_general(n, 16, B.F64, B.F64)
    # more workgroups, more partial-sum records
    assert L.odmd_state_bytes_shaped(160000, 16, B.F64, B.F64, 256, 16, 65536, 0) > \
        L.odmd_state_bytes_shaped(160000, 16, B.F64, B.F64, 256, 16, 1, 0)
    bad = [(384, 256, 256, 0), (128, 256, 256, 0), (512, 8, 256, 0), (512, 24, 256, 0),
           (512, 1 << 25, 256, 0), (512, 256, 0, 0), (512, 256, 65537, 0), (512, 256, 256, 2)]
    h = ctypes.c_void_p(12345)
    for shape in bad:
        assert L.odmd_state_bytes_shaped(1000, 8, B.F64, B.F64, *shape) == 0, shape
        assert L.odmd_create_shaped(1000, 8, 1e-8, B.F64, B.F64, None, *shape, None, 0,
                                    ctypes.byref(h)) == 1, shape
        assert h.value is None
    # the size and type checks of odmd_create_ex still apply
    assert L.odmd_create_shaped(1000, 65, 1e-8, B.F64, B.F64, None, 512, 256, 256, 0, None, 0,
                                ctypes.byref(h)) == 1
    assert L.odmd_create_shaped(1000, 8, 1e-8, B.F64, B.F64, None, 512, 256, 256, 0, None, 0,
                                None) == 1


@needs_lib
def test_autotune_rejects_bad_arguments_before_device_use():
    L = B.lib()
    t, r, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    b, d = ctypes.c_double(), ctypes.c_double()
    outs = [ctypes.byref(v) for v in (t, r, c, b, d)]
    for n, rmax, basis, io, streams in [(0, 8, B.F64, B.F64, 1), (100, 65, B.F64, B.F64, 1),
                                        (100, 8, B.F64, B.F32, 1), (100, 8, B.F64, B.F64, 0),
                                        (100, 8, B.F64, B.F64, 1025)]:
        assert L.odmd_autotune(n, rmax, basis, io, streams, None, *outs) == 1
    assert L.odmd_autotune(100, 8, B.F64, B.F64, 1, None, None, *outs[1:]) == 1


@needs_lib
def test_plan_entry_points_check_arguments_on_the_host():
    L = B.lib()
    p = ctypes.c_void_p(12345)
    assert L.odmd_plan_create(None, None, None, 1, ctypes.byref(p)) == 1
    assert p.value is None
    assert L.odmd_plan_create(None, None, None, 1, None) == 1
    H = (ctypes.c_void_p * 1)(None)
    assert L.odmd_plan_create(H, H, H, 0, ctypes.byref(p)) == 1     # count >= 1
    assert L.odmd_plan_create(H, H, H, 1, ctypes.byref(p)) == 1     # NULL handle
    assert L.odmd_plan_launch(None) == 1
    assert L.odmd_plan_destroy(None) == 1


def test_info_struct_matches_the_header():
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{(.*?)\} odmd_info;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"(int32_t|int64_t|double)\s+(\w+);", body)
    ctype = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double}
    assert [(n, ctype[t]) for t, n in fields] == list(B.Info._fields_)


@needs_lib
def test_noalloc_batch_limits_are_host_checked():
    """The no-allocation batched update rejects more streams than its fixed
    tables hold, and NULL entries, on the host (no handle is dereferenced,
    no device call is made)."""
    L = B.lib()
    cnt = B.NOALLOC_MAX_STREAMS + 1
    H = (ctypes.c_void_p * cnt)()
    X = (ctypes.c_void_p * cnt)()
    Y = (ctypes.c_void_p * cnt)()
    assert L.odmd_update_batch_noalloc(H, X, Y, cnt) == 1
    assert L.odmd_update_batch_noalloc(H, X, Y, -1) == 1
    assert L.odmd_update_batch_noalloc(H, X, Y, 0) == 0          # nothing to do
    assert L.odmd_update_batch_noalloc(H, X, Y, 2) == 1          # NULL handles
