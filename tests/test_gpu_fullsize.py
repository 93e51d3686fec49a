"""GPU parity at full size: the benchmark's own workloads -- the 16-column
wide table of 64,000,000 rows in one 64M-row row group with 1 MiB pages,
uncompressed, the same table Snappy-compressed with a 1 MiB dictionary cap
(PLAIN fallback for the high-cardinality columns), and the two ends of the
row-group x page-size sweep -- scanned in the
launch configuration bench.py times (one pq_scan of all sixteen columns)
and compared with the oracle byte for byte over every row of every column
(values, validity, offsets, chars).  The oracle reads the columns on
several host threads (each read is an independent single-threaded decode
of one column)."""
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

import datagen as dg
import oracle
from tests.gpu_util import GUARD, POISON, compare_column

pytestmark = pytest.mark.gpu

ROWS = 64_000_000


def _full_parity(spec, label):
    import paper_2602_17335_amd as pqs
    print(f"[gpu] {label}: generating {ROWS} rows", flush=True)
    data = dg.write(spec, nthreads=16)
    print(f"[gpu] {label}: {len(data)} bytes, scanning all columns", flush=True)
    sys.stdout.flush()
    buf, n = pqs.to_device(data)
    f = pqs.DeviceFile(buf, n)
    cols = list(range(f.num_columns))
    out = f.scan(cols, poison=POISON, guard=GUARD)
    of = oracle.File(data)
    with ThreadPoolExecutor(max_workers=8) as ex:
        for c, o in zip(cols, ex.map(of.read, cols)):
            compare_column(o, out[c], f"{label} col{c}")
            out[c] = None
    print(f"[gpu] {label}: all {len(cols)} columns equal", flush=True)


def test_full_size_uncompressed():
    _full_parity(dg.wide_table(ROWS, ROWS, 1 << 20), "wide16 64M uncompressed")


def test_full_size_snappy():
    _full_parity(dg.snappy_wide_table(ROWS, ROWS, 1 << 20), "wide16 64M snappy")


@pytest.mark.parametrize("rg_rows,page_bytes", [(1_000_000, 64 * 1024), (ROWS, 8 << 20)])
def test_full_size_sweep_extremes(rg_rows, page_bytes):
    """The two ends of the row-group x page-size sweep: 64 row groups of 1M
    rows with 64 KiB pages (576 dictionaries, about 49K pages), and one
    row group with 8 MiB pages (pages of up to 20M rows)."""
    _full_parity(dg.wide_table(ROWS, rg_rows, page_bytes), f"wide16 64M rg{rg_rows} page{page_bytes}")
