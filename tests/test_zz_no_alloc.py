"""pq_scan_noalloc (the allocation-free variant of pq_scan, whose workspace
is the library's file-scope device array) against pq_scan, through the C
ABI: two calls in a row on one GPU, the second with a smaller input, each
byte-identical (outputs pre-filled with 0xAB, guard regions untouched) to
pq_scan of the same request; and a scan whose workspace would not fit the
array is refused before anything is enqueued."""
import ctypes

import pytest

import datagen as dg
from tests.gpu_util import GUARD, POISON, check_guards

pytestmark = pytest.mark.gpu


def _noalloc(f, cols, rb, re_):
    import torch
    import paper_2602_17335_amd as pqs
    L = pqs.lib()
    L.pq_scan_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.POINTER(pqs.ColumnOut), ctypes.c_int32, ctypes.c_void_p]
    L.pq_scan_noalloc.restype = ctypes.c_int
    mask, rg_end, ws, outs, tens = f.allocate(cols, rb, re_, poison=POISON, guard=GUARD)
    del ws  # not used: the scan's workspace is the library's array
    arr = (pqs.ColumnOut * len(outs))(*outs)
    s = torch.cuda.current_stream()
    pqs._check(L.pq_scan_noalloc(f._h, mask, rb, rg_end, arr, len(outs), ctypes.c_void_p(s.cuda_stream)))
    pqs._check(L.pq_scan_check(f._h, None, ctypes.c_void_p(s.cuda_stream)))
    return tens


def _same(tens, ref, label):
    import torch
    import paper_2602_17335_amd as pqs
    for c, t in tens.items():
        r = ref[c]
        rows = t["rows"]
        assert torch.equal(t["validity_buf"][: pqs.validity_bytes(rows)], r["validity_words"]), (label, c)
        guards = [t["validity_buf"][t["validity_bytes"]:]]
        if "offsets" in t:
            assert torch.equal(t["offsets"], r["offsets"]), (label, c)
            assert torch.equal(t["chars_buf"][: t["chars_bytes"]], r["chars"]), (label, c)
            guards += [t["offsets_buf"][8 * (rows + 1):], t["chars_buf"][max(t["chars_bytes"], 1):]]
        else:
            assert torch.equal(t["values_buf"][:rows], r["values"]), (label, c)
            guards.append(t["values_raw"][t["value_bytes"]:])
        check_guards({"guards": guards}, f"{label} col{c}")


def test_noalloc_matches_pq_scan_twice():
    import paper_2602_17335_amd as pqs
    big = dg.write(dg.wide_table(300_007, 120_000, 64 * dg.KiB))
    small = dg.write(dg.wide_table(41_003, 20_000, 16 * dg.KiB, seed=0x5EED0011))
    for data, cols, rb, re_, label in ((big, list(range(16)), 0, 3, "first, 300K rows x 16 columns"),
                                       (small, [0, 3, 6, 9, 12, 15], 1, 3, "second, smaller")):
        print(f"[gpu] noalloc: {label}", flush=True)
        buf, n = pqs.to_device(data)
        f = pqs.DeviceFile(buf, n)
        ref = f.scan(cols, rb, re_, poison=POISON, guard=GUARD)
        got = _noalloc(f, cols, rb, re_)
        _same(got, ref, label)


def test_noalloc_refuses_a_workspace_above_the_array():
    import paper_2602_17335_amd as pqs
    data = dg.write(dg.snappy_wide_table(1_500_000, 1_500_000, 1 * dg.MiB))
    buf, n = pqs.to_device(data)
    f = pqs.DeviceFile(buf, n)
    assert f.plan((1 << 16) - 1, 0, 1).workspace_bytes > (64 << 20)
    with pytest.raises(pqs.PqError) as e:
        _noalloc(f, list(range(16)), 0, 1)
    assert e.value.code == pqs.PQ_ECAPACITY
