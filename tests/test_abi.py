"""The C ABI on the CPU: the scan library loads, exports every function that
include/pq.h declares, and rejects bad arguments on the host before any GPU
work (nothing here touches a device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pq.h")

PQ_OK, PQ_EINVAL, PQ_ECORRUPT = 0, -1, -2


def _declared():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(pq_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2602_17335_amd import build as b
    srcs = [os.path.join(b.HERE, s) for s in b.SOURCES] + [HEADER]
    if not os.path.exists(b.SO) or os.path.getmtime(b.SO) < max(os.path.getmtime(s) for s in srcs):
        b.build()
    L = ctypes.CDLL(b.SO)
    vp = ctypes.c_void_p
    L.pq_open_device.argtypes = [vp, ctypes.c_uint64, vp, ctypes.POINTER(vp)]
    L.pq_open_device.restype = ctypes.c_int
    L.pq_last_error.restype = ctypes.c_char_p
    for name in ("pq_num_columns", "pq_num_row_groups"):
        getattr(L, name).argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.pq_plan.argtypes = [vp, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, vp]
    L.pq_scan_check.argtypes = [vp, vp, vp]
    L.pq_profile.argtypes = [vp, ctypes.c_int32]
    L.pq_close.argtypes = [vp]
    L.pq_close.restype = None
    return L


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("pq_open_device", "pq_plan", "pq_scan", "pq_scan_check", "pq_close", "pq_last_error"):
        assert n in names
    assert len(names) >= 15


def _declarations():
    """(name, comment text between the previous declaration and this one)."""
    text = open(HEADER).read()
    body = text[text.index("extern \"C\""):]
    out, last = [], 0
    for m in re.finditer(r"^\s*(?:pq_status|void|const char\*)\s+(pq_[a-z0-9_]+)\s*\(", body, flags=re.M):
        between = body[last:m.start()]
        out.append((m.group(1), " ".join(re.findall(r"/\*(.*?)\*/", between, flags=re.S))))
        last = body.index(";", m.end()) + 1
    return out


def test_every_declared_call_cites_the_paper():
    """Each entry point's comment (or the comment of the group it is declared
    in, for declarations with no comment of their own) names the paper
    section that defines the operation, or the callers it exists for."""
    prev_cited = False
    decls = _declarations()
    assert len(decls) >= 15
    for name, comment in decls:
        if comment.strip():
            prev_cited = "Sec." in comment or "callers" in comment
        assert prev_cited, f"{name}: no citation in its comment"


def test_every_declared_function_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, f"declared in pq.h but not exported: {missing}"


def test_open_rejects_bad_arguments_on_the_host(lib):
    out = ctypes.c_void_p(123)
    assert lib.pq_open_device(None, 100, None, ctypes.byref(out)) == PQ_EINVAL
    assert out.value is None  # cleared on failure
    assert b"dev_buf" in lib.pq_last_error()
    # a non-NULL pointer that is not 16-byte aligned is refused before any access
    assert lib.pq_open_device(ctypes.c_void_p(0x1001), 100, None, ctypes.byref(out)) == PQ_EINVAL
    assert b"aligned" in lib.pq_last_error()
    # too short to be a Parquet file: refused before the footer is read
    assert lib.pq_open_device(ctypes.c_void_p(0x1000), 11, None, ctypes.byref(out)) == PQ_ECORRUPT
    assert lib.pq_open_device(ctypes.c_void_p(0x1000), 100, None, None) == PQ_EINVAL


def test_null_handle_is_rejected(lib):
    n = ctypes.c_int32(-1)
    assert lib.pq_num_columns(None, ctypes.byref(n)) == PQ_EINVAL
    assert lib.pq_num_row_groups(None, ctypes.byref(n)) == PQ_EINVAL
    assert lib.pq_plan(None, 1, 0, 1, None) == PQ_EINVAL
    assert lib.pq_scan_check(None, None, None) != PQ_OK  # no GPU here: the scratch array cannot be found
    assert lib.pq_profile(None, 0) == PQ_OK  # NULL: the recorder of batched scans
    lib.pq_close(None)  # a no-op


def test_batch_calls_reject_bad_arguments_on_the_host(lib):
    vp, u64 = ctypes.c_void_p, ctypes.c_uint64
    lib.pq_plan_batch.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(u64), vp, ctypes.c_int32]
    lib.pq_scan_batch.argtypes = [vp, ctypes.c_int32, vp, vp, u64, vp]
    ws = u64(0)
    assert lib.pq_plan_batch(None, 0, ctypes.byref(ws), None, 0) == PQ_OK  # an empty batch
    assert ws.value >= 256
    assert lib.pq_plan_batch(None, 1, ctypes.byref(ws), None, 0) == PQ_EINVAL
    assert lib.pq_plan_batch(None, 0, None, None, 0) == PQ_EINVAL
    assert lib.pq_scan_batch(None, 0, None, None, 0, None) == PQ_EINVAL  # NULL workspace
