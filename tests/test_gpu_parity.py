"""GPU parity: every output buffer of the HIP scan (through the C ABI)
equals the CPU oracle's, byte for byte, on seeded files that span several
tiles and ragged tails, on pyarrow-written files (V1/V2, Snappy,
dictionary fallback, DELTA), on row-group sub-ranges and projections, and on
edge cases.  Integer work, so the bar is exact equality."""
import io

import numpy as np
import pyarrow as pa
import pyarrow.parquet as pq
import pytest

import datagen as dg
from tests.gpu_util import check_file, gpu_scan

pytestmark = pytest.mark.gpu


def _spec_cases():
    cases = {
        "small2col": dg.small_table(300_011, 64 * dg.KiB),
        "wide_v1": dg.wide_table(250_003, 100_000, 64 * dg.KiB),
        "wide_v2": dg.wide_table(250_003, 100_000, 64 * dg.KiB, page_version=2),
        "wide_bigpage": dg.wide_table(200_000, 200_000, 1 * dg.MiB),
        "wide_snappy": dg.snappy_wide_table(250_003, 100_000, 64 * dg.KiB),
        "wide_tinypages": dg.wide_table(20_000, 7_000, 700),
    }
    s = dg.snappy_wide_table(150_000, 150_000, 128 * dg.KiB)
    s.page_version = 2
    s.dict_cap = 32 * dg.KiB
    cases["wide_snappy_v2_fallback"] = s
    # literal-only Snappy streams: one literal spans every 64 KiB output block
    # of a 256 KiB page, so the pages are decompressed sequentially (no
    # block index), beside the block-parallel path of the other files
    lit = dg.snappy_wide_table(120_000, 120_000, 256 * dg.KiB)
    lit.snappy_literal_only = True
    cases["wide_snappy_literal_only"] = lit
    # every Snappy tag form in turn (literal lengths in 0-4 extra bytes,
    # copies with 1-, 2- and 4-byte offsets), V1 and V2 pages
    for v in (1, 2):
        vf = dg.snappy_wide_table(130_000, 130_000, 256 * dg.KiB)
        vf.page_version = v
        vf.snappy_varied_forms = True
        cases[f"wide_snappy_varied_forms_v{v}"] = vf
    cases["edge"] = dg.FileSpec(cols=[
        dg.Col(dg.INT32, dg.PLAIN, True, dg.UNIFORM, 1.0),
        dg.Col(dg.INT64, dg.RLE_DICTIONARY, True, dg.CONST, 0.3, lo=-5),
        dg.Col(dg.INT32, dg.DELTA_BINARY_PACKED, False, dg.UNIFORM, lo=-2**31, hi=2**31),
        dg.Col(dg.INT64, dg.DELTA_BINARY_PACKED, True, dg.UNIFORM, 0.5, lo=-2**62, hi=2**62),
        dg.Col(dg.BYTE_ARRAY, dg.PLAIN, True, dg.STRINGS, 0.25, hi=0, str_min=0, str_max=3),
        dg.Col(dg.INT32, dg.RLE_DICTIONARY, True, dg.RUNS, 0.0, lo=0, hi=7, run_len=5000),
        dg.Col(dg.DOUBLE, dg.RLE_DICTIONARY, False, dg.DICTVALS, hi=3),
        dg.Col(dg.BYTE_ARRAY, dg.RLE_DICTIONARY, False, dg.STRINGS, hi=1, str_min=5, str_max=5),
        dg.Col(dg.INT64, dg.DELTA_BINARY_PACKED, True, dg.SORTED, 0.9, lo=0, hi=1 << 40, gap_max=3),
        dg.Col(dg.INT32, dg.PLAIN, True, dg.UNIFORM, 0.999, lo=0, hi=100),
    ], num_rows=40_011, rg_rows=13_000, page_bytes=20_000, name="edge")
    # string dictionaries: entries of 45..60 chars (slots, four pieces per
    # slot), of 61..300 chars (no slots; 128-entry regions larger than the
    # LDS buffer), of 0..2 chars (slots holding empty strings), and of 8..44
    # chars with fewer than 4 rows per entry (short enough for slots, but
    # decoded from (position, length) pairs)
    cases["dict_strings"] = dg.FileSpec(cols=[
        dg.Col(dg.BYTE_ARRAY, dg.RLE_DICTIONARY, True, dg.STRINGS, 0.2, hi=3000, str_min=45, str_max=60),
        dg.Col(dg.BYTE_ARRAY, dg.RLE_DICTIONARY, True, dg.STRINGS, 0.1, hi=2000, str_min=61, str_max=300),
        dg.Col(dg.BYTE_ARRAY, dg.RLE_DICTIONARY, False, dg.STRINGS, 0.0, hi=700, str_min=0, str_max=2),
        dg.Col(dg.BYTE_ARRAY, dg.RLE_DICTIONARY, True, dg.STRINGS, 0.1, hi=40_000, str_min=8, str_max=44),
    ], num_rows=70_001, rg_rows=30_000, page_bytes=256 * dg.KiB, name="dict_strings")
    # string dictionaries past the size whose length chain is walked in
    # segments side by side at open: short entries (thousands per segment),
    # 50-70-char entries (the chain often enters a segment past the
    # candidate positions, so the page is walked whole), one with a single
    # huge segment count; uncompressed and Snappy (dictionary in the
    # decompression buffer)
    for codec, tag in ((dg.UNCOMPRESSED, ""), (dg.SNAPPY, "_snappy")):
        cases["dict_chains" + tag] = dg.FileSpec(cols=[
            dg.Col(dg.BYTE_ARRAY, dg.RLE_DICTIONARY, True, dg.STRINGS, 0.1, hi=300_000, str_min=0, str_max=6),
            dg.Col(dg.BYTE_ARRAY, dg.RLE_DICTIONARY, False, dg.STRINGS, 0.0, hi=20_000, str_min=50, str_max=70),
            dg.Col(dg.BYTE_ARRAY, dg.RLE_DICTIONARY, True, dg.STRINGS, 0.3, hi=400_000, str_min=8, str_max=44),
        ], num_rows=400_003, rg_rows=400_003, page_bytes=1 * dg.MiB, codec=codec, name="dict_chains" + tag)
    # long definition-level streams (pages of 10^5 optional rows and more),
    # walked in segments side by side at open: bit-packed runs (50% nulls),
    # long RLE runs (0.1% nulls), pages of few values (99.9% nulls), all
    # null, strings; V1 and V2, uncompressed and Snappy (V1 levels in the
    # decompression buffer)
    ll_cols = [
        dg.Col(dg.INT32, dg.PLAIN, True, dg.UNIFORM, 0.5, lo=-(1 << 31), hi=1 << 31),
        dg.Col(dg.INT64, dg.RLE_DICTIONARY, True, dg.DICTVALS, 0.001, hi=100),
        dg.Col(dg.INT64, dg.DELTA_BINARY_PACKED, True, dg.SORTED, 0.999, lo=0, hi=1 << 40, gap_max=8),
        dg.Col(dg.INT32, dg.PLAIN, True, dg.UNIFORM, 1.0),
        dg.Col(dg.BYTE_ARRAY, dg.PLAIN, True, dg.STRINGS, 0.3, hi=0, str_min=0, str_max=12),
    ]
    for ver in (1, 2):
        for codec, tag in ((dg.UNCOMPRESSED, ""), (dg.SNAPPY, "_snappy")):
            cases[f"long_levels_v{ver}{tag}"] = dg.FileSpec(
                cols=ll_cols, num_rows=600_011, rg_rows=300_007, page_bytes=1 * dg.MiB, codec=codec,
                page_version=ver, name=f"long_levels_v{ver}{tag}")
    # bit-packed level runs of 1000 and 3000 groups (no RLE runs): the chain enters
    # segments past the candidate positions (1000) or leaves the staged bytes
    # (3000), so those pages are walked whole by one wave
    for groups in (1000, 3000):
        cases[f"long_levels_bp{groups}"] = dg.FileSpec(
            cols=[ll_cols[0], ll_cols[4]], num_rows=300_007, rg_rows=300_007, page_bytes=1 * dg.MiB,
            max_bp_groups=groups, rle_min=1 << 30, name=f"long_levels_bp{groups}")
    # long DELTA_BINARY_PACKED streams, whose block chains are walked in
    # segments side by side at open: narrow blocks (sorted keys), wide
    # blocks of about 1 KiB (uniform 64-bit values: chains enter segments
    # past the candidate positions, so those pages are walked whole), and
    # the length streams of DELTA_LENGTH_BYTE_ARRAY strings; blocks of
    # 128 x 4, 256 x 8 and 1024 x 1 values; V1 and V2 Snappy
    dl_cols = [
        dg.Col(dg.INT32, dg.DELTA_BINARY_PACKED, False, dg.SORTED, 0.0, lo=0, hi=1 << 30, gap_max=8),
        dg.Col(dg.INT64, dg.DELTA_BINARY_PACKED, True, dg.SORTED, 0.1, lo=0, hi=1 << 40, gap_max=1000),
        dg.Col(dg.INT64, dg.DELTA_BINARY_PACKED, True, dg.UNIFORM, 0.2, lo=-2**62, hi=2**62),
        dg.Col(dg.BYTE_ARRAY, dg.DELTA_LENGTH_BYTE_ARRAY, True, dg.STRINGS, 0.1, hi=0, str_min=0, str_max=20),
    ]
    for blk, mini in ((128, 4), (256, 8), (1024, 1)):
        for ver, codec, tag in ((1, dg.UNCOMPRESSED, ""), (2, dg.SNAPPY, "_v2_snappy")):
            cases[f"long_delta_{blk}x{mini}{tag}"] = dg.FileSpec(
                cols=dl_cols, num_rows=400_003, rg_rows=400_003, page_bytes=1 * dg.MiB, codec=codec,
                page_version=ver, delta_block=blk, delta_mini=mini, name=f"long_delta_{blk}x{mini}{tag}")
    # long dictionary-index streams, walked in segments side by side at
    # open: index widths 1, 7, 10 (Zipf ranks: RLE runs among bit-packed
    # ones), 14 (strings), 16 (bit-packed runs of 1009 bytes, the widest the
    # candidates cover) and 20 (wider: those pages are walked whole); V1
    # and V2 Snappy
    di_cols = [
        dg.Col(dg.INT32, dg.RLE_DICTIONARY, False, dg.DICTVALS, 0.0, hi=2),
        dg.Col(dg.INT64, dg.RLE_DICTIONARY, True, dg.DICTVALS, 0.1, hi=100),
        dg.Col(dg.INT32, dg.RLE_DICTIONARY, True, dg.ZIPF, 0.1, hi=1024, zipf_s=1.1),
        dg.Col(dg.BYTE_ARRAY, dg.RLE_DICTIONARY, True, dg.STRINGS, 0.1, hi=10_000, str_min=8, str_max=44),
        dg.Col(dg.INT32, dg.RLE_DICTIONARY, True, dg.DICTVALS, 0.05, hi=65536),
        dg.Col(dg.INT64, dg.RLE_DICTIONARY, True, dg.DICTVALS, 0.05, hi=1_000_000),
    ]
    for ver, codec, tag in ((1, dg.UNCOMPRESSED, ""), (2, dg.SNAPPY, "_v2_snappy")):
        cases[f"long_dict{tag}"] = dg.FileSpec(
            cols=di_cols, num_rows=1_500_007, rg_rows=1_500_007, page_bytes=1 * dg.MiB, codec=codec,
            page_version=ver, name=f"long_dict{tag}")
    return cases


CASES = _spec_cases()


@pytest.mark.parametrize("name", sorted(CASES))
def test_parity_writer_files(name):
    spec = CASES[name]
    data = dg.write(spec)
    check_file(data, label=name)


def test_parity_subrange_and_projection():
    spec = dg.wide_table(300_000, 70_000, 32 * dg.KiB)
    data = dg.write(spec)
    check_file(data, columns=[0, 6, 9, 15], rg_begin=1, rg_end=4, label="sub")
    check_file(data, columns=[13], rg_begin=2, rg_end=3, label="one")
    check_file(data, columns=[5, 6], rg_begin=3, rg_end=3, label="empty-range")


def test_parity_snappy_subrange_and_projection():
    """Snappy pages of several 64 KiB blocks under row-group sub-ranges and
    projections (a scan's block-indexed blocks are taken in buckets of
    element count: only the selected pages' blocks may enter them)."""
    spec = dg.snappy_wide_table(300_000, 70_000, 256 * dg.KiB)
    data = dg.write(spec)
    check_file(data, columns=[0, 6, 9, 15], rg_begin=1, rg_end=4, label="snappy-sub")
    check_file(data, columns=[13], rg_begin=2, rg_end=3, label="snappy-one")
    check_file(data, columns=[3, 4, 5], rg_begin=0, rg_end=5, label="snappy-three")


def _arrow_table(n, seed):
    rng = np.random.default_rng(seed)
    m = rng.random(n) < 0.1
    strs = np.array([("k" * int(k % 37)) + str(k) for k in rng.integers(0, 3000, n)], dtype=object)
    dbl = rng.random(n) * 1e6
    dbl[::97] = np.nan
    dbl[1::89] = -0.0
    return pa.table({
        "i32": pa.array(rng.integers(-2**31, 2**31, n).astype(np.int32), mask=m),
        "i64sorted": pa.array(np.cumsum(rng.integers(1, 9, n)).astype(np.int64), mask=rng.random(n) < 0.05),
        "i64few": pa.array(rng.integers(0, 50, n).astype(np.int64)),
        "i64ext": pa.array(rng.choice(np.array([0, -1, 2**63 - 1, -2**63, 7], dtype=np.int64), n)),
        "dbl": pa.array(dbl, mask=m),
        "str": pa.array(strs, mask=rng.random(n) < 0.2, type=pa.binary()),
        "strreq": pa.array(strs, type=pa.binary()),
        "allnull": pa.array(np.zeros(n, dtype=np.int32), mask=np.ones(n, dtype=bool)),
    })


@pytest.mark.parametrize("version", ["1.0", "2.0"])
@pytest.mark.parametrize("compression", ["none", "snappy"])
@pytest.mark.parametrize("encoding", ["dict", "plain", "delta"])
def test_parity_pyarrow_files(version, compression, encoding):
    n = 60_000
    t = _arrow_table(n, 5)
    kw = dict(data_page_version=version, compression=compression, data_page_size=16384,
              row_group_size=25_000, dictionary_pagesize_limit=4096)
    if encoding == "dict":
        kw["use_dictionary"] = True
    elif encoding == "plain":
        kw["use_dictionary"] = False
    else:
        kw["use_dictionary"] = ["str", "dbl"]
        kw["column_encoding"] = {"i32": "DELTA_BINARY_PACKED", "i64sorted": "DELTA_BINARY_PACKED",
                                 "i64few": "DELTA_BINARY_PACKED", "i64ext": "DELTA_BINARY_PACKED"}
    bio = io.BytesIO()
    pq.write_table(t, bio, **kw)
    check_file(np.frombuffer(bio.getvalue(), dtype=np.uint8), label=f"arrow-{version}-{compression}-{encoding}")


def test_repeat_scan_identical():
    """The same scan twice on one handle gives identical bytes."""
    import torch
    spec = dg.wide_table(200_000, 100_000, 48 * dg.KiB)
    data = dg.write(spec)
    f, a = gpu_scan(data)
    b = f.scan(list(range(16)))
    for c in a:
        for k in a[c]:
            if isinstance(a[c][k], torch.Tensor):
                assert torch.equal(a[c][k], b[c][k]), (c, k)


def test_corrupt_dictionary_index_reported():
    import paper_2602_17335_amd as pqs
    spec = dg.FileSpec(cols=[dg.Col(dg.INT64, dg.RLE_DICTIONARY, False, dg.DICTVALS, hi=4)],
                       num_rows=64, rg_rows=64, page_bytes=1 << 20)
    b = dg.write(spec).copy()
    raw = b.tobytes()
    dict_end = raw.index(b"\x15\x00", 4 + 20)
    body = dict_end + len(raw[dict_end:].split(b"\x00\x00", 1)[0]) + 2
    assert b[body] == 2
    b[body] = 3  # indices now decode at width 3 past the 4-entry dictionary or the page
    buf, n = pqs.to_device(b)
    try:
        f = pqs.DeviceFile(buf, n)
        f.scan([0])
        raise AssertionError("corruption not reported")
    except pqs.PqError as e:
        assert e.code == pqs.PQ_ECORRUPT


def _level_page(data):
    """(body offset, level bytes) of the first page of a one-column V1
    uncompressed file without a dictionary page."""
    import oracle
    raw = data.tobytes()
    h, n = oracle.page_header(raw[4:4 + 256])
    assert h.type == 0 and h.compressed_size == h.uncompressed_size
    body = 4 + n
    return body, int.from_bytes(raw[body:body + 4], "little")


@pytest.mark.parametrize("how", ["truncated", "empty", "bad_run"])
def test_corrupt_long_level_stream_reported(how):
    """A long definition-level stream that ends before the page's last row
    (length prefix halved, or zero) or holds an RLE run of value 5 is
    reported as corrupt at open, as the oracle reports it."""
    import oracle
    import paper_2602_17335_amd as pqs
    spec = dg.FileSpec(cols=[dg.Col(dg.INT32, dg.PLAIN, True, dg.UNIFORM, 0.5, lo=0, hi=1000)],
                       num_rows=500_000, rg_rows=500_000, page_bytes=4 * dg.MiB)
    b = dg.write(spec).copy()
    body, L = _level_page(b)
    assert L > 3 * 16384  # several segments of the parallel walk
    if how == "truncated":
        b[body:body + 4] = np.frombuffer((L // 2).to_bytes(4, "little"), dtype=np.uint8)
    elif how == "empty":
        b[body:body + 4] = 0
    else:
        at = body + 4 + L // 2
        b[at:at + 200] = np.tile(np.array([0x02, 0x05], dtype=np.uint8), 100)
    with pytest.raises(oracle.OracleError):
        oracle.File(b).read(0)
    buf, n = pqs.to_device(b)
    with pytest.raises(pqs.PqError) as e:
        f = pqs.DeviceFile(buf, n)
        f.scan([0])
    assert e.value.code == pqs.PQ_ECORRUPT


def _uleb(raw, pos):
    v = sh = 0
    while True:
        b = raw[pos]
        pos += 1
        v |= (b & 0x7F) << sh
        sh += 7
        if not b & 0x80:
            return v, pos


@pytest.mark.parametrize("how", ["bad_width", "unused_width"])
def test_long_delta_stream_widths(how):
    """A miniblock bit width above 32 in the middle of a long INT32 DELTA
    stream is reported as corrupt at open, as the oracle reports it; a width
    of 255 for a miniblock of the last block that holds no values is
    ignored, by both."""
    import oracle
    import paper_2602_17335_amd as pqs
    spec = dg.FileSpec(cols=[dg.Col(dg.INT32, dg.DELTA_BINARY_PACKED, False, dg.SORTED, 0.0, lo=0, hi=1 << 30,
                                    gap_max=8)], num_rows=300_000, rg_rows=300_000, page_bytes=4 * dg.MiB)
    b = dg.write(spec).copy()
    raw = b.tobytes()
    h, n = oracle.page_header(raw[4:4 + 256])
    assert h.type == 0 and h.compressed_size == h.uncompressed_size
    pos = 4 + n
    B, pos = _uleb(raw, pos)
    M, pos = _uleb(raw, pos)
    total, pos = _uleb(raw, pos)
    _, pos = _uleb(raw, pos)
    per, nblocks = B // M, (total - 1 + B - 1) // B
    blocks = []
    for k in range(nblocks):
        _, pos = _uleb(raw, pos)
        used_mb = (min(total - 1 - k * B, B) + per - 1) // per
        blocks.append((pos, used_mb))
        pos += M + sum(per * w // 8 for w in raw[pos:pos + used_mb])
    assert pos - (4 + n) > 4 * 16384  # several segments of the parallel walk
    if how == "bad_width":
        b[blocks[nblocks // 2][0]] = 0xFF
        with pytest.raises(oracle.OracleError):
            oracle.File(b).read(0)
        buf, n2 = pqs.to_device(b)
        with pytest.raises(pqs.PqError) as e:
            f = pqs.DeviceFile(buf, n2)
            f.scan([0])
        assert e.value.code == pqs.PQ_ECORRUPT
    else:
        wpos, used_mb = blocks[-1]
        assert used_mb < M
        b[wpos + used_mb] = 0xFF
        check_file(b, label="unused-width")


def test_corrupt_long_index_stream_reported():
    """3000 bytes of 0xFF in the middle of a long dictionary-index stream
    (every run header there is an overlong ULEB128) are reported as corrupt
    at open, as the oracle reports them."""
    import oracle
    import paper_2602_17335_amd as pqs
    spec = dg.FileSpec(cols=[dg.Col(dg.INT64, dg.RLE_DICTIONARY, False, dg.DICTVALS, 0.0, hi=100)],
                       num_rows=400_000, rg_rows=400_000, page_bytes=4 * dg.MiB)
    b = dg.write(spec).copy()
    raw = b.tobytes()
    h, n = oracle.page_header(raw[4:4 + 256])
    assert h.type == 2  # the dictionary page
    at = 4 + n + h.compressed_size
    h, n = oracle.page_header(raw[at:at + 256])
    assert h.type == 0 and h.compressed_size == h.uncompressed_size and h.compressed_size > 4 * 32768
    mid = at + n + h.compressed_size // 2
    b[mid:mid + 3000] = 0xFF
    with pytest.raises(oracle.OracleError):
        oracle.File(b).read(0)
    buf, n2 = pqs.to_device(b)
    with pytest.raises(pqs.PqError) as e:
        f = pqs.DeviceFile(buf, n2)
        f.scan([0])
    assert e.value.code == pqs.PQ_ECORRUPT


def test_bad_magic_rejected_before_gpu_work():
    import paper_2602_17335_amd as pqs
    b = dg.write(dg.small_table(1000, 4096)).copy()
    b[-1] = 0
    buf, n = pqs.to_device(b)
    with pytest.raises(pqs.PqError) as e:
        pqs.DeviceFile(buf, n)
    assert e.value.code == pqs.PQ_ECORRUPT


def test_column_encodings_match_page_headers():
    """pq_column_encodings equals the set of data-page encodings found by
    walking every chunk's page headers with the oracle's header parser."""
    import oracle
    import paper_2602_17335_amd as pqs
    spec = CASES["wide_snappy_v2_fallback"]
    data = dg.write(spec)
    md = pq.ParquetFile(io.BytesIO(data.tobytes())).metadata
    raw = data.tobytes()
    want = [0] * md.num_columns
    for rg in range(md.num_row_groups):
        for c in range(md.num_columns):
            cm = md.row_group(rg).column(c)
            at = cm.dictionary_page_offset if cm.has_dictionary_page else cm.data_page_offset
            end = at + cm.total_compressed_size
            while at < end:
                h, n = oracle.page_header(raw[at:at + 256])
                if h.type in (0, 3):  # DATA_PAGE, DATA_PAGE_V2
                    want[c] |= 1 << h.encoding
                at += n + h.compressed_size
    buf, n = pqs.to_device(data)
    f = pqs.DeviceFile(buf, n)
    got = [f.column_encodings(c) for c in range(f.num_columns)]
    assert got == want
    assert any(bin(m).count("1") > 1 for m in want)  # the dictionary fallback mixes encodings


def _string_spec():
    return dg.FileSpec(cols=[
        dg.Col(dg.BYTE_ARRAY, dg.PLAIN, True, dg.STRINGS, 0.1, hi=5000, str_min=0, str_max=40),
        dg.Col(dg.BYTE_ARRAY, dg.RLE_DICTIONARY, True, dg.STRINGS, 0.1, hi=300, str_min=8, str_max=44),
        dg.Col(dg.BYTE_ARRAY, dg.RLE_DICTIONARY, False, dg.STRINGS, 0.0, hi=200, str_min=61, str_max=200),
    ], num_rows=40_011, rg_rows=15_000, page_bytes=32 * dg.KiB, name="strings")


def test_chars_capacity_reported_and_respected():
    """A chars buffer below the planned size: pq_scan_check reports
    PQ_ECAPACITY and no byte past chars_capacity is written (PLAIN strings,
    slot dictionary, dictionary without slots)."""
    import torch
    import paper_2602_17335_amd as pqs
    buf, n = pqs.to_device(dg.write(_string_spec()))
    f = pqs.DeviceFile(buf, n)
    for c in range(3):
        mask, rg_end, ws, outs, tens = f.allocate([c])
        need = tens[c]["chars_bytes"]
        assert need > 1000, (c, need)
        cap = need // 2 + 3
        guard = torch.full((need + 4096,), 0xAB, dtype=torch.uint8, device="cuda")
        outs[0].chars = guard.data_ptr()
        outs[0].chars_capacity = cap
        print(f"[gpu] capacity col{c}: need {need}, capacity {cap}", flush=True)
        f.scan_into(mask, 0, rg_end, outs, ws)
        with pytest.raises(pqs.PqError) as e:
            f.check(ws)
        assert e.value.code == pqs.PQ_ECAPACITY, (c, e.value.code)
        assert bool((guard[cap:] == 0xAB).all()), f"col{c}: bytes written past chars_capacity"
        # the same handle scans correctly afterwards
        out = f.scan([c])
        assert int(out[c]["offsets"][-1]) == need


def test_workspace_too_small_rejected_before_gpu_work():
    import torch
    import paper_2602_17335_amd as pqs
    buf, n = pqs.to_device(dg.write(_string_spec()))
    f = pqs.DeviceFile(buf, n)
    mask, rg_end, ws, outs, tens = f.allocate([0, 1, 2])
    small = torch.zeros(max(ws.numel() // 2, 256), dtype=torch.uint8, device="cuda")
    with pytest.raises(pqs.PqError) as e:
        f.scan_into(mask, 0, rg_end, outs, small)
    assert e.value.code == pqs.PQ_ECAPACITY
    torch.cuda.synchronize()
    assert int(small.count_nonzero()) == 0  # nothing was enqueued: the workspace is untouched
    f.check(small)


def test_plan_chars_bytes_match_oracle():
    """pq_plan (host-only, from the tile prefix built at open) gives every
    string column's exact chars size on every row-group range."""
    import oracle
    import paper_2602_17335_amd as pqs
    data = dg.write(_string_spec())
    buf, n = pqs.to_device(data)
    f = pqs.DeviceFile(buf, n)
    of = oracle.File(data)
    nrg = f.num_row_groups
    for rb in range(nrg + 1):
        for re_ in range(rb, nrg + 1):
            sz = f.plan(0b111, rb, re_)
            for c in range(3):
                assert int(sz.chars_bytes[c]) == of.read(c, rb, re_)["chars"].size, (c, rb, re_)
