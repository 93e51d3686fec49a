"""GPU parity of the streamed scan of a host-resident file (Sec. 4.1,
overlapped reading): the file stays in pinned host memory, each row group's
selected column chunks are copied into one of two device staging slots while
the previous row group decodes, and every output buffer must equal the
oracle's byte for byte -- uncompressed and Snappy, V1 and V2 pages,
dictionary, PLAIN, DELTA, BYTE_STREAM_SPLIT, DELTA_LENGTH_BYTE_ARRAY and
DELTA_BYTE_ARRAY columns, column subsets, row-group sub-ranges (so that a
slot is reused many times) and the single-row-group file.  A host handle is refused by the
device-resident scan calls."""
import numpy as np
import pytest

import datagen as dg
import oracle
from tests.gpu_util import GUARD, POISON, compare_column

pytestmark = pytest.mark.gpu


def _streamed(data, columns=None, rg_begin=0, rg_end=None, label=""):
    import paper_2602_17335_amd as pqs
    print(f"[gpu] streamed {label}: {len(data)} bytes cols={columns} rg=[{rg_begin},{rg_end})", flush=True)
    f = pqs.HostFile(data)
    if columns is None:
        columns = list(range(f.num_columns))
    out = f.scan(columns, rg_begin, rg_end, poison=POISON, guard=GUARD)
    of = oracle.File(data)
    if rg_end is None:
        rg_end = of.num_row_groups
    for c, g in out.items():
        compare_column(of.read(c, rg_begin, rg_end), g, f"streamed {label} col{c}")
    return f


def _mixed(version, codec, rows=300_017, rg=40_000, page=32 * dg.KiB):
    return dg.FileSpec(cols=[
        dg.Col(dg.INT64, dg.RLE_DICTIONARY, True, dg.DICTVALS, 0.1, hi=1000),
        dg.Col(dg.INT32, dg.PLAIN, False, dg.UNIFORM, lo=-2**31, hi=2**31),
        dg.Col(dg.INT64, dg.DELTA_BINARY_PACKED, True, dg.SORTED, 0.1, lo=0, hi=1 << 40, gap_max=8),
        dg.Col(dg.BYTE_ARRAY, dg.RLE_DICTIONARY, True, dg.STRINGS, 0.2, hi=500, str_min=8, str_max=44),
        dg.Col(dg.BYTE_ARRAY, dg.PLAIN, True, dg.STRINGS, 0.1, hi=100_000, str_min=0, str_max=30),
        dg.Col(dg.DOUBLE, dg.BYTE_STREAM_SPLIT, True, dg.UNIFORM, 0.3),
        dg.Col(dg.BYTE_ARRAY, dg.DELTA_LENGTH_BYTE_ARRAY, True, dg.STRINGS, 0.1, hi=100_000, str_min=8, str_max=44),
        dg.Col(dg.DOUBLE, dg.RLE_DICTIONARY, False, dg.DICTVALS, hi=40_000),
        dg.Col(dg.BYTE_ARRAY, dg.DELTA_BYTE_ARRAY, True, dg.STRINGS, 0.1, hi=3000, str_min=0, str_max=30),
    ], num_rows=rows, rg_rows=rg, page_bytes=page, page_version=version, codec=codec,
        name=f"streamed-v{version}-c{codec}")


@pytest.mark.parametrize("version,codec", [(1, dg.UNCOMPRESSED), (2, dg.UNCOMPRESSED), (1, dg.SNAPPY), (2, dg.SNAPPY)])
def test_streamed_all_columns(version, codec):
    _streamed(dg.write(_mixed(version, codec)), label=f"v{version} codec{codec}")


def test_streamed_subsets_and_ranges():
    data = dg.write(_mixed(1, dg.SNAPPY))
    _streamed(data, [0, 3, 6, 8], 2, 7, label="cols 0,3,6,8 rg[2,7)")
    _streamed(data, [5], 7, 8, label="col 5 last row group")
    _streamed(data, [1, 4], 3, 3, label="empty range")


def test_streamed_single_row_group():
    _streamed(dg.write(dg.small_table(rows=200_000, page_bytes=64 * dg.KiB)), label="small table one row group")


def test_streamed_equals_device_scan():
    """The same file scanned device-resident and streamed: equal bytes."""
    import paper_2602_17335_amd as pqs
    data = dg.write(_mixed(2, dg.SNAPPY, rows=200_003, rg=25_000))
    buf, n = pqs.to_device(data)
    d = pqs.DeviceFile(buf, n).scan(list(range(9)))
    h = pqs.HostFile(data).scan(list(range(9)))
    for c in range(9):
        for k in ("values", "offsets", "chars", "validity_words"):
            if k in d[c]:
                assert np.array_equal(d[c][k].cpu().numpy(), h[c][k].cpu().numpy()), (c, k)


def test_host_handle_refused_by_device_scans():
    import paper_2602_17335_amd as pqs
    f = pqs.HostFile(dg.write(dg.small_table(rows=50_000, page_bytes=64 * dg.KiB)))
    mask, rg_end, ws, outs, _ = f.allocate([0, 1])
    with pytest.raises(pqs.PqError) as e:
        pqs.DeviceFile.scan_into(f, mask, 0, rg_end, outs, ws)
    assert e.value.code == pqs.PQ_EINVAL
    with pytest.raises(pqs.PqError) as e:
        pqs.Batch([(f, [0, 1], 0, None)])
    assert e.value.code == pqs.PQ_EINVAL
    with pytest.raises(pqs.PqError) as e:
        pqs.Server([f], budget_bytes=1 << 26)
    assert e.value.code == pqs.PQ_EINVAL
