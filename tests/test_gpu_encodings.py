"""GPU parity of the encodings the paper's encoding search adds (Sec. 3,
Encoding Flexibility): BYTE_STREAM_SPLIT (INT32, INT64, DOUBLE),
DELTA_LENGTH_BYTE_ARRAY and DELTA_BYTE_ARRAY strings, in files of the
project's writer (V1 and V2, Snappy, nulls, empty strings) and of pyarrow
(sorted strings with long shared prefixes), in the file the writer's encoding
search and 10% compression rule produce, and through the batched and
per-page forms; every buffer compared with the oracle byte for byte.  A
DELTA_BYTE_ARRAY page with a value longer than the expansion buffer (16 KiB)
is valid Parquet the scanner does not decode: scanning its column reports
PQ_EUNSUPPORTED, and the file's other columns scan normally."""
import io

import numpy as np
import pyarrow as pa
import pyarrow.parquet as pq
import pytest

import datagen as dg
import oracle
from tests.gpu_util import GUARD, POISON, check_file, compare_column

pytestmark = pytest.mark.gpu


def _spec(version, codec, rows=150_007, rg=60_000, page=32 * dg.KiB):
    return dg.FileSpec(cols=[
        dg.Col(dg.INT32, dg.BYTE_STREAM_SPLIT, True, dg.UNIFORM, 0.1, lo=-2**31, hi=2**31),
        dg.Col(dg.INT64, dg.BYTE_STREAM_SPLIT, False, dg.UNIFORM, lo=-2**62, hi=2**62),
        dg.Col(dg.DOUBLE, dg.BYTE_STREAM_SPLIT, True, dg.UNIFORM, 0.3),
        dg.Col(dg.BYTE_ARRAY, dg.DELTA_LENGTH_BYTE_ARRAY, True, dg.STRINGS, 0.1, hi=100_000, str_min=8, str_max=44),
        dg.Col(dg.BYTE_ARRAY, dg.DELTA_LENGTH_BYTE_ARRAY, False, dg.STRINGS, 0.0, hi=5000, str_min=0, str_max=3),
        dg.Col(dg.BYTE_ARRAY, dg.DELTA_LENGTH_BYTE_ARRAY, True, dg.STRINGS, 0.5, hi=2000, str_min=100, str_max=300),
        dg.Col(dg.INT32, dg.PLAIN, True, dg.UNIFORM, 0.999, lo=0, hi=100),
        dg.Col(dg.BYTE_ARRAY, dg.DELTA_BYTE_ARRAY, True, dg.STRINGS, 0.1, hi=2000, str_min=0, str_max=40),
    ], num_rows=rows, rg_rows=rg, page_bytes=page, page_version=version, codec=codec,
        name=f"enc-v{version}-c{codec}")


@pytest.mark.parametrize("version,codec", [(1, dg.UNCOMPRESSED), (2, dg.UNCOMPRESSED), (1, dg.SNAPPY), (2, dg.SNAPPY)])
def test_new_encodings_writer_files(version, codec):
    check_file(dg.write(_spec(version, codec)), label=f"bss/dlba/dba v{version} codec{codec}")


@pytest.mark.parametrize("version", ["1.0", "2.0"])
def test_new_encodings_pyarrow_files(version):
    rng = np.random.default_rng(21)
    n = 50_000
    words = np.array([("w" * int(k % 29)) + str(k) for k in rng.integers(0, 10_000, n)], dtype=object)
    dbl = rng.random(n) * 1e6
    dbl[::101] = np.nan
    # sorted keys with long shared prefixes for DELTA_BYTE_ARRAY
    keys = sorted("customer/%05d/order/%07d" % (int(a), int(b)) for a, b in
                  zip(rng.integers(0, 300, n), rng.integers(0, 10**7, n)))
    t = pa.table({
        "i32": pa.array(rng.integers(-2**31, 2**31, n).astype(np.int32), mask=rng.random(n) < 0.1),
        "i64": pa.array(rng.integers(-2**62, 2**62, n).astype(np.int64)),
        "dbl": pa.array(dbl, mask=rng.random(n) < 0.05),
        "s": pa.array(words, mask=rng.random(n) < 0.2, type=pa.binary()),
        "k": pa.array(keys, mask=rng.random(n) < 0.05, type=pa.binary()),
    })
    bio = io.BytesIO()
    pq.write_table(t, bio, use_dictionary=False, data_page_version=version, data_page_size=8192, row_group_size=20_000,
                   column_encoding={"i32": "BYTE_STREAM_SPLIT", "i64": "BYTE_STREAM_SPLIT", "dbl": "BYTE_STREAM_SPLIT",
                                    "s": "DELTA_LENGTH_BYTE_ARRAY", "k": "DELTA_BYTE_ARRAY"})
    check_file(np.frombuffer(bio.getvalue(), dtype=np.uint8), label=f"arrow bss/dlba {version}")


def test_encoding_search_preset_file():
    spec = dg.wide_table(300_000, 100_000, 64 * dg.KiB, codec=dg.SNAPPY)
    spec.encoding_search = True
    spec.min_saving_pct = 10
    check_file(dg.write(spec), label="wide table, encoding search + 10% compression rule")


@pytest.mark.parametrize("codec", [dg.UNCOMPRESSED, dg.SNAPPY])
def test_delta_byte_array_pyarrow_snappy_and_pages(codec):
    """pyarrow DELTA_BYTE_ARRAY pages of several sizes (many pages, each its
    own prefix chain), with and without Snappy."""
    rng = np.random.default_rng(5)
    n = 120_000
    keys = sorted("%s/%08d" % ("abcdefghij"[int(a)] * int(1 + a), int(b)) for a, b in
                  zip(rng.integers(0, 10, n), rng.integers(0, 10**8, n)))
    t = pa.table({"k": pa.array(keys, mask=rng.random(n) < 0.02, type=pa.binary()),
                  "e": pa.array([b""] * n, type=pa.binary())})
    bio = io.BytesIO()
    pq.write_table(t, bio, use_dictionary=False, data_page_size=4096, row_group_size=50_000,
                   compression="snappy" if codec == dg.SNAPPY else "none",
                   column_encoding={"k": "DELTA_BYTE_ARRAY", "e": "DELTA_BYTE_ARRAY"})
    check_file(np.frombuffer(bio.getvalue(), dtype=np.uint8), label=f"arrow dba codec{codec}")


def test_delta_byte_array_long_values_unsupported_others_scan():
    import paper_2602_17335_amd as pqs
    spec = dg.FileSpec(cols=[
        dg.Col(dg.BYTE_ARRAY, dg.DELTA_BYTE_ARRAY, True, dg.STRINGS, 0.1, hi=50, str_min=20000, str_max=20000),
        dg.Col(dg.INT64, dg.DELTA_BINARY_PACKED, True, dg.SORTED, 0.1, lo=0, hi=1 << 40),
    ], num_rows=3_000, rg_rows=3_000, page_bytes=1 << 20)
    data = dg.write(spec)
    buf, n = pqs.to_device(data)
    f = pqs.DeviceFile(buf, n)
    with pytest.raises(pqs.PqError) as e:
        f.scan([0])
    assert e.value.code == pqs.PQ_EUNSUPPORTED
    out = f.scan([1], poison=POISON, guard=GUARD)
    compare_column(oracle.File(data).read(1), out[1], "DELTA column beside a DELTA_BYTE_ARRAY one")


@pytest.mark.parametrize("form", [0, 1])
def test_new_encodings_batched(form):
    import paper_2602_17335_amd as pqs
    datas = [dg.write(_spec(v, c, rows=40_000 + 7 * i, rg=15_000, page=16 * dg.KiB))
             for i, (v, c) in enumerate([(1, dg.UNCOMPRESSED), (2, dg.SNAPPY), (1, dg.SNAPPY)])]
    files = []
    for d in datas:
        buf, n = pqs.to_device(d)
        files.append(pqs.DeviceFile(buf, n))
    b = pqs.Batch([(f, list(range(8)), 0, None) for f in files], poison=POISON, guard=GUARD)
    t = pqs.tuning_default()
    t.form = form
    b.scan(t)
    b.check()
    for i, d in enumerate(datas):
        of = oracle.File(d)
        for c in range(8):
            compare_column(of.read(c), b.outputs[i][c], f"batch form{form} file{i} col{c}")
