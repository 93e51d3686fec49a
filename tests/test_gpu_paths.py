"""GPU parity on the decode paths that only some legal files take, each
compared with the CPU oracle byte for byte through the C ABI:

- dictionary-index streams whose bit-width byte is wider than the minimum
  (25, 31 and 32 bits: one load per value instead of a packed piece);
- streams of 256 MiB or more, where every walk switches to 64-bit positions;
- DELTA_BINARY_PACKED blocks other than the common 128/4 and 256/4 shapes
  (512 values in 8 miniblocks), and the shape the scanner does not support
  (1024 values in 32 miniblocks), which must be refused at open;
- the small two-column table at its full size (1,000,000 rows, 1 MiB pages);
- one handle scanned on two streams at once, each scan with its own
  workspace, against the single-stream result;
- the library's streaming copy used as the bench's practical ceiling.
"""
import sys

import numpy as np
import pytest

import datagen as dg
import oracle
from tests.gpu_util import GUARD, POISON, check_file, compare_column

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("width", [25, 31, 32])
def test_index_width_wider_than_minimal(width):
    spec = dg.FileSpec(cols=[
        dg.Col(dg.INT64, dg.RLE_DICTIONARY, True, dg.DICTVALS, 0.1, hi=1000),
        dg.Col(dg.INT32, dg.RLE_DICTIONARY, False, dg.ZIPF, hi=1 << 12, zipf_s=1.1),
        dg.Col(dg.BYTE_ARRAY, dg.RLE_DICTIONARY, True, dg.STRINGS, 0.2, hi=500, str_min=8, str_max=44),
        dg.Col(dg.DOUBLE, dg.RLE_DICTIONARY, True, dg.DICTVALS, 0.05, hi=40_000),
    ], num_rows=150_007, rg_rows=70_000, page_bytes=64 * dg.KiB, index_width=width, name=f"idxw{width}")
    check_file(dg.write(spec), label=f"index width {width}")


def test_streams_over_256MiB():
    """One row group, one page per column: a 504 MB PLAIN INT64 value stream
    (OPTIONAL, 10% nulls) and a 280 MB dictionary-index stream at 32 bits."""
    rows = 70_000_000
    spec = dg.FileSpec(cols=[
        dg.Col(dg.INT64, dg.PLAIN, True, dg.UNIFORM, 0.1, lo=-2**62, hi=2**62),
        dg.Col(dg.INT32, dg.RLE_DICTIONARY, False, dg.DICTVALS, hi=1000),
    ], num_rows=rows, rg_rows=rows, page_bytes=1 << 30, index_width=32, name="big_streams")
    check_file(dg.write(spec, nthreads=8), label="streams over 256 MiB")


def _delta_spec(block, mini):
    return dg.FileSpec(cols=[
        dg.Col(dg.INT64, dg.DELTA_BINARY_PACKED, True, dg.SORTED, 0.1, lo=0, hi=1 << 40, gap_max=8),
        dg.Col(dg.INT32, dg.DELTA_BINARY_PACKED, False, dg.UNIFORM, lo=-2**31, hi=2**31),
        dg.Col(dg.INT64, dg.DELTA_BINARY_PACKED, True, dg.UNIFORM, 0.3, lo=-2**62, hi=2**62),
    ], num_rows=90_011, rg_rows=40_000, page_bytes=48 * dg.KiB, delta_block=block, delta_mini=mini,
        name=f"delta{block}_{mini}")


def test_delta_block_512_of_8():
    check_file(dg.write(_delta_spec(512, 8)), label="delta 512/8")


def test_delta_block_1024_of_32_unsupported():
    """32 miniblocks per block is valid Parquet (the oracle decodes it, see
    the CPU tests) but above the scanner's 16: refused at open."""
    import paper_2602_17335_amd as pqs
    data = dg.write(_delta_spec(1024, 32))
    buf, n = pqs.to_device(data)
    with pytest.raises(pqs.PqError) as e:
        pqs.DeviceFile(buf, n)
    assert e.value.code == pqs.PQ_EUNSUPPORTED


def test_small_table_full_size():
    """The two-column table at its stated size: 1,000,000 rows, one row
    group, 1 MiB pages, INT32 PLAIN and INT64 dictionary (1024 entries)."""
    check_file(dg.write(dg.small_table()), label="small 1M rows")


def test_two_streams_one_handle():
    """Two scans of one handle in flight on two streams (separate workspaces
    and outputs) give the bytes of the same scans run one at a time."""
    import torch
    import paper_2602_17335_amd as pqs
    data = dg.write(dg.wide_table(400_003, 100_000, 64 * dg.KiB))
    buf, n = pqs.to_device(data)
    f = pqs.DeviceFile(buf, n)
    jobs = [(list(range(16)), 0, 4), ([0, 5, 6, 9, 13, 15], 1, 3)]
    alone = [f.scan(c, b, e, poison=POISON, guard=GUARD) for c, b, e in jobs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    pending = []
    for (cols, b, e), s in zip(jobs, streams):
        mask, rg_end, ws, outs, tens = f.allocate(cols, b, e, poison=POISON, guard=GUARD)
        f.scan_into(mask, b, rg_end, outs, ws, stream=s)
        pending.append((ws, tens, s))
    print("[gpu] two streams enqueued", flush=True)
    for (ws, tens, s), ref in zip(pending, alone):
        f.check(ws, stream=s)
        for c, t in tens.items():
            r = ref[c]
            rows = t["rows"]
            assert torch.equal(t["validity_buf"][: pqs.validity_bytes(rows)], r["validity_words"]), c
            if "offsets" in t:
                assert torch.equal(t["offsets"], r["offsets"]), c
                assert torch.equal(t["chars_buf"][: t["chars_bytes"]], r["chars"]), c
            else:
                assert torch.equal(t["values_buf"][:rows], r["values"]), c
    of = oracle.File(data)
    for (cols, b, e), res in zip(jobs, alone):
        for c in cols:
            compare_column(of.read(c, b, e), res[c], f"two-streams col{c} rg[{b},{e})")


def test_copy_probe():
    """The library's streaming copy (the bench's "% of copy" reference)
    copies every byte, including a ragged tail past the last 16-byte chunk,
    and leaves the bytes after the destination range alone."""
    import torch
    import paper_2602_17335_amd as pqs
    for n in (1, 15, 16, 4097, (3 << 20) + 7, 64 << 20):
        src = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda")
        dst = torch.full((n + 64,), 0xAB, dtype=torch.uint8, device="cuda")
        pqs.copy_probe(dst, src, n)
        torch.cuda.synchronize()
        assert torch.equal(dst[:n], src), n
        assert bool((dst[n:] == 0xAB).all()), n
