"""Seeded synthetic Parquet files: the shared INPUT GENERATOR.

Both the CPU oracle and the GPU reader consume the bytes produced here; this
module holds no decoding arithmetic.  The C core (``pqgen.c``) encodes; the
recipes below fix the workloads (column mixes, null rates, distributions,
row-group and page sizes, codec) used by tests and by the benchmark.

The file knobs are the four the paper studies (Sec. 1, Sec. 3: page count /
page size, row-group size, encoding, compression).  The column mix of the wide
table stands in for the paper's TPC-H ``lineitem`` workload (Sec. 3 setup),
which is not reproduced: every value here is synthetic.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libpqgen.so")

INT32, INT64, DOUBLE, BYTE_ARRAY = 1, 2, 5, 6
PLAIN, PLAIN_DICTIONARY, RLE, DELTA_BINARY_PACKED, RLE_DICTIONARY = 0, 2, 3, 5, 8
DELTA_LENGTH_BYTE_ARRAY, DELTA_BYTE_ARRAY, BYTE_STREAM_SPLIT = 6, 7, 9
UNIFORM, ZIPF, SORTED, DICTVALS, STRINGS, CONST, RUNS = 0, 1, 2, 3, 4, 5, 6
UNCOMPRESSED, SNAPPY = 0, 1

KiB = 1024
MiB = 1024 * 1024


class _Col(ctypes.Structure):
    _fields_ = [
        ("ptype", ctypes.c_int32), ("encoding", ctypes.c_int32), ("optional", ctypes.c_int32),
        ("dist", ctypes.c_int32), ("null_prob", ctypes.c_double),
        ("lo", ctypes.c_int64), ("hi", ctypes.c_int64),
        ("dlo", ctypes.c_double), ("dhi", ctypes.c_double), ("zipf_s", ctypes.c_double),
        ("str_min", ctypes.c_int32), ("str_max", ctypes.c_int32),
        ("gap_max", ctypes.c_int32), ("run_len", ctypes.c_int32),
    ]


class _Spec(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64), ("num_rows", ctypes.c_int64), ("rg_rows", ctypes.c_int64),
        ("page_bytes", ctypes.c_int64), ("dict_cap", ctypes.c_int64),
        ("codec", ctypes.c_int32), ("page_version", ctypes.c_int32),
        ("delta_block", ctypes.c_int32), ("delta_mini", ctypes.c_int32),
        ("max_bp_groups", ctypes.c_int32), ("rle_min", ctypes.c_int32),
        ("ncols", ctypes.c_int32), ("nthreads", ctypes.c_int32),
        ("snappy_skip", ctypes.c_int32), ("index_width", ctypes.c_int32),
        ("encoding_search", ctypes.c_int32), ("min_saving_pct", ctypes.c_int32),
    ]


@dataclasses.dataclass
class Col:
    ptype: int
    encoding: int = PLAIN
    optional: bool = False
    dist: int = UNIFORM
    null_prob: float = 0.0
    lo: int = 0
    hi: int = 1 << 20
    dlo: float = 0.0
    dhi: float = 1e6
    zipf_s: float = 1.1
    str_min: int = 8
    str_max: int = 44
    gap_max: int = 8
    run_len: int = 16


@dataclasses.dataclass
class FileSpec:
    cols: List[Col]
    num_rows: int
    rg_rows: int
    page_bytes: int = 1 * MiB
    dict_cap: int = 0
    codec: int = UNCOMPRESSED
    page_version: int = 1
    delta_block: int = 128
    delta_mini: int = 4
    max_bp_groups: int = 63
    rle_min: int = 8
    seed: int = 0x5EED0000
    snappy_literal_only: bool = False
    snappy_varied_forms: bool = False  # every Snappy tag form in turn (decoder fixture)
    index_width: int = 0  # dictionary index bit width byte when wider than the minimum (legal; 0 = minimal)
    encoding_search: bool = False  # per chunk, the candidate encoding of smallest encoded size
    min_saving_pct: int = 0  # >0: chunks whose Snappy pages save no more than this stay uncompressed
    name: str = "custom"

    def _c(self, nthreads: int):
        sp = _Spec()
        sp.seed = self.seed & 0xFFFFFFFFFFFFFFFF
        sp.num_rows = self.num_rows
        sp.rg_rows = max(1, self.rg_rows)
        sp.page_bytes = self.page_bytes
        sp.dict_cap = self.dict_cap
        sp.codec = self.codec
        sp.page_version = self.page_version
        sp.delta_block = self.delta_block
        sp.delta_mini = self.delta_mini
        sp.max_bp_groups = self.max_bp_groups
        sp.rle_min = self.rle_min
        sp.ncols = len(self.cols)
        sp.nthreads = nthreads
        sp.snappy_skip = 1 if self.snappy_literal_only else 2 if self.snappy_varied_forms else 0
        sp.index_width = self.index_width
        sp.encoding_search = 1 if self.encoding_search else 0
        sp.min_saving_pct = self.min_saving_pct
        arr = (_Col * len(self.cols))()
        for i, c in enumerate(self.cols):
            for f in dataclasses.fields(Col):
                v = getattr(c, f.name)
                setattr(arr[i], f.name, int(v) if isinstance(v, bool) else v)
        return sp, arr


_lib = None


def build(force: bool = False) -> str:
    """Compile the C writer into datagen/libpqgen.so."""
    src = os.path.join(_HERE, "pqgen.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-pthread", src, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        L.pqg_write.restype = ctypes.c_void_p
        L.pqg_write.argtypes = [ctypes.POINTER(_Spec), ctypes.POINTER(_Col), ctypes.POINTER(ctypes.c_size_t)]
        L.pqg_free.argtypes = [ctypes.c_void_p]
        L.pqg_snappy.restype = ctypes.c_void_p
        L.pqg_snappy.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.pqg_expected_fixed.argtypes = [ctypes.POINTER(_Spec), ctypes.POINTER(_Col), ctypes.c_int,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        L.pqg_expected_strings.restype = ctypes.c_int64
        L.pqg_expected_strings.argtypes = [ctypes.POINTER(_Spec), ctypes.POINTER(_Col), ctypes.c_int,
                                           ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]
        _lib = L
    return _lib


def write(spec: FileSpec, nthreads: Optional[int] = None) -> np.ndarray:
    """Encode `spec` into a Parquet file; returns its bytes as a uint8 array."""
    L = lib()
    nt = nthreads or min(16, os.cpu_count() or 1)
    sp, arr = spec._c(nt)
    n = ctypes.c_size_t(0)
    p = L.pqg_write(ctypes.byref(sp), arr, ctypes.byref(n))
    try:
        out = np.empty(n.value, dtype=np.uint8)
        ctypes.memmove(out.ctypes.data, p, n.value)
    finally:
        L.pqg_free(p)
    return out


def snappy_compress(data: bytes, literal_only: bool = False, varied_forms: bool = False) -> bytes:
    """The fixture compressor: greedy matcher; one literal (literal_only); or
    the greedy matcher's elements in every tag form in turn (varied_forms)."""
    L = lib()
    buf = ctypes.create_string_buffer(bytes(data), len(data))
    n = ctypes.c_size_t(0)
    p = L.pqg_snappy(buf, len(data), 1 if literal_only else 2 if varied_forms else 0, ctypes.byref(n))
    try:
        return ctypes.string_at(p, n.value)
    finally:
        L.pqg_free(p)


_NP = {INT32: np.int32, INT64: np.int64, DOUBLE: np.float64}


def expected(spec: FileSpec, col: int, row0: int = 0, nrows: Optional[int] = None) -> dict:
    """Decoded rows [row0, row0+nrows) of column `col`, straight from the seeds.

    Returns {"values"| "offsets"+"chars", "validity"} in the reader's output
    layout: null slots zero, LSB-first validity, int64 offsets from 0.
    """
    L = lib()
    sp, arr = spec._c(1)
    n = spec.num_rows - row0 if nrows is None else nrows
    c = spec.cols[col]
    validity = np.zeros((n + 7) // 8, dtype=np.uint8)
    if c.ptype == BYTE_ARRAY:
        offsets = np.zeros(n + 1, dtype=np.int64)
        total = L.pqg_expected_strings(ctypes.byref(sp), arr, col, row0, n, offsets.ctypes.data, None, None)
        chars = np.zeros(max(total, 1), dtype=np.uint8)
        L.pqg_expected_strings(ctypes.byref(sp), arr, col, row0, n, offsets.ctypes.data, chars.ctypes.data,
                               validity.ctypes.data)
        return {"offsets": offsets, "chars": chars[:total], "validity": validity}
    vals = np.zeros(n, dtype=_NP[c.ptype])
    L.pqg_expected_fixed(ctypes.byref(sp), arr, col, row0, n, vals.ctypes.data, validity.ctypes.data)
    return {"values": vals, "validity": validity}


# --------------------------------------------------------------------------
# Workload recipes
# --------------------------------------------------------------------------

def small_table(rows: int = 1_000_000, page_bytes: int = 1 * MiB, seed: int = 0x5EED0000) -> FileSpec:
    """One uncompressed row group, all REQUIRED: an INT32 PLAIN column uniform
    in [0, 2^20) and an INT64 RLE_DICTIONARY column with 1024 distinct
    uniformly random values (index bit width 10)."""
    return FileSpec(
        cols=[
            Col(INT32, PLAIN, False, UNIFORM, lo=0, hi=1 << 20),
            Col(INT64, RLE_DICTIONARY, False, DICTVALS, hi=1024),
        ],
        num_rows=rows, rg_rows=rows, page_bytes=page_bytes, seed=seed, name="small_2col")


def wide_cols(null_prob: float = 0.10, plain_hicard_strings: bool = False) -> List[Col]:
    """The 16-column fact table: 6 INT32, 4 INT64, 3 DOUBLE, 3 BYTE_ARRAY,
    every column OPTIONAL with Bernoulli(null_prob) nulls."""
    p = null_prob
    return [
        Col(INT32, PLAIN, True, UNIFORM, p, lo=-(1 << 31), hi=1 << 31),        # c0
        Col(INT32, PLAIN, True, UNIFORM, p, lo=0, hi=1 << 20),                 # c1
        Col(INT32, PLAIN, True, UNIFORM, p, lo=0, hi=1 << 31),                 # c2
        Col(INT32, RLE_DICTIONARY, True, ZIPF, p, hi=1 << 10, zipf_s=1.1),     # c3
        Col(INT32, RLE_DICTIONARY, True, ZIPF, p, hi=1 << 16, zipf_s=1.1),     # c4
        Col(INT32, RLE_DICTIONARY, True, ZIPF, p, hi=1 << 20, zipf_s=1.1),     # c5
        Col(INT64, DELTA_BINARY_PACKED, True, SORTED, p, lo=0, hi=1 << 40, gap_max=8),  # c6
        Col(INT64, RLE_DICTIONARY, True, DICTVALS, p, hi=100),                 # c7
        Col(INT64, RLE_DICTIONARY, True, DICTVALS, p, hi=10_000),              # c8
        Col(INT64, RLE_DICTIONARY, True, DICTVALS, p, hi=1_000_000),           # c9
        Col(DOUBLE, PLAIN, True, UNIFORM, p, dlo=0.0, dhi=1e6),                # c10
        Col(DOUBLE, PLAIN, True, UNIFORM, p, dlo=0.0, dhi=1e6),                # c11
        Col(DOUBLE, PLAIN, True, UNIFORM, p, dlo=0.0, dhi=1e6),                # c12
        Col(BYTE_ARRAY, RLE_DICTIONARY, True, STRINGS, p, hi=100, str_min=8, str_max=44),        # c13
        Col(BYTE_ARRAY, RLE_DICTIONARY, True, STRINGS, p, hi=10_000, str_min=8, str_max=44),     # c14
        Col(BYTE_ARRAY, RLE_DICTIONARY, True, STRINGS, p, hi=1_000_000, str_min=8, str_max=44),  # c15
    ]


def wide_table(rows: int = 64_000_000, rg_rows: int = 64_000_000, page_bytes: int = 1 * MiB,
               seed: int = 0x5EED0001, codec: int = UNCOMPRESSED, dict_cap: int = 0,
               page_version: int = 1) -> FileSpec:
    """The wide fact table (16 columns, 10% nulls).  Uncompressed with no
    dictionary cap by default; with codec=SNAPPY and dict_cap=1 MiB it is the
    compressed variant whose high-cardinality dictionary columns fall back to
    PLAIN."""
    return FileSpec(cols=wide_cols(), num_rows=rows, rg_rows=rg_rows, page_bytes=page_bytes,
                    seed=seed, codec=codec, dict_cap=dict_cap, page_version=page_version,
                    name="wide16")


def snappy_wide_table(rows: int = 64_000_000, rg_rows: int = 64_000_000, page_bytes: int = 1 * MiB,
                      seed: int = 0x5EED0002) -> FileSpec:
    return wide_table(rows, rg_rows, page_bytes, seed, codec=SNAPPY, dict_cap=1 * MiB)


def batch_cols(null_prob: float = 0.05) -> List[Col]:
    """The 8 columns of the many-files workload: INT32 uniform PLAIN, INT32
    Zipf(1.1) ranks over [1, 2^16] dictionary, INT64 sorted keys DELTA,
    INT64 10^4-distinct dictionary, 2 x DOUBLE uniform PLAIN, 2 x BYTE_ARRAY
    dictionary strings (10^2 and 10^4 distinct, length 8..44); every column
    OPTIONAL with Bernoulli(null_prob) nulls."""
    p = null_prob
    return [
        Col(INT32, PLAIN, True, UNIFORM, p, lo=-(1 << 31), hi=1 << 31),
        Col(INT32, RLE_DICTIONARY, True, ZIPF, p, hi=1 << 16, zipf_s=1.1),
        Col(INT64, DELTA_BINARY_PACKED, True, SORTED, p, lo=0, hi=1 << 40, gap_max=8),
        Col(INT64, RLE_DICTIONARY, True, DICTVALS, p, hi=10_000),
        Col(DOUBLE, PLAIN, True, UNIFORM, p, dlo=0.0, dhi=1e6),
        Col(DOUBLE, PLAIN, True, UNIFORM, p, dlo=0.0, dhi=1e6),
        Col(BYTE_ARRAY, RLE_DICTIONARY, True, STRINGS, p, hi=100, str_min=8, str_max=44),
        Col(BYTE_ARRAY, RLE_DICTIONARY, True, STRINGS, p, hi=10_000, str_min=8, str_max=44),
    ]


def batch_specs(nfiles: int = 4096, max_rows: int = 4_000_000, min_rows: int = 10_000,
                rg_rows: int = 1_000_000, page_kib=(8, 16, 32, 64, 128, 256, 512, 1024),
                seed: int = 0x5EED0003) -> List[FileSpec]:
    """The many-files workload: file of Zipf rank i (1-based) holds
    max(min_rows, floor(max_rows * i^-1.1)) rows, the files in a seeded
    random order; each file's page-size target is drawn uniformly from
    `page_kib` (a log-uniform choice over 8 KiB .. 1 MiB by default), and a
    seeded half of the files is Snappy-compressed.  File i's values come from
    seed + 0x1000 * (i + 1)."""
    rng = np.random.default_rng(seed)
    ranks = np.arange(1, nfiles + 1, dtype=np.float64)
    rows = np.maximum(min_rows, np.floor(max_rows * ranks ** -1.1)).astype(np.int64)
    rows = rows[rng.permutation(nfiles)]
    pages = rng.integers(0, len(page_kib), nfiles)
    snappy = rng.random(nfiles) < 0.5
    out = []
    for i in range(nfiles):
        out.append(FileSpec(cols=batch_cols(), num_rows=int(rows[i]), rg_rows=rg_rows,
                            page_bytes=int(page_kib[pages[i]]) * KiB, codec=SNAPPY if snappy[i] else UNCOMPRESSED,
                            seed=(seed + 0x1000 * (i + 1)) & 0xFFFFFFFFFFFFFFFF, name=f"batch{i}"))
    return out


def serve_catalog(nfiles: int = 256, min_bytes: int = 1_000_000, max_bytes: int = 2_000_000_000,
                  seed: int = 0x5EED0004) -> List[FileSpec]:
    """The serving catalog: file i's target encoded size is log-uniform in
    [min_bytes, max_bytes]; its recipe cycles through the wide table
    (uncompressed), the wide table Snappy-compressed with a 1 MiB dictionary
    cap, and the 8-column many-files recipe, with rows set from the size at
    the recipe's measured bytes per row (about 50, 48 and 42), 1M-row row
    groups (smaller files: at least 4 row groups), and a page-size target
    drawn from 64 KiB .. 1 MiB."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(min_bytes), np.log(max_bytes), nfiles))
    pages = rng.integers(0, 5, nfiles)
    out = []
    for i in range(nfiles):
        kind = i % 3
        bpr = (50.0, 48.0, 42.0)[kind]
        rows = max(4_000, int(sizes[i] / bpr))
        rg = min(1_000_000, max(1_000, rows // 4))
        pb = (64 << (int(pages[i]))) * KiB
        s = (seed + 0x1000 * (i + 1)) & 0xFFFFFFFFFFFFFFFF
        if kind == 0:
            sp = wide_table(rows, rg, pb, seed=s)
        elif kind == 1:
            sp = snappy_wide_table(rows, rg, pb, seed=s)
        else:
            sp = FileSpec(cols=batch_cols(), num_rows=rows, rg_rows=rg, page_bytes=pb, seed=s)
        sp.name = f"serve{i}"
        out.append(sp)
    return out


# The paper's file-configuration steps (Sec. 3) on the wide table, cumulative
# as in its ablation: the DuckDB-like baseline, then more pages per chunk
# (Insight 1), million-row row groups (Insight 2), the per-chunk encoding
# search (Insight 3) and compression kept only where it saves more than 10%
# (Insight 4).
PRESETS = ("baseline", "+pages", "+rowgroups", "+encodings", "+no_compression")


def preset(name: str, rows: int = 16_000_000, seed: int = 0x5EED0005) -> FileSpec:
    """The wide table under one step of the paper's configuration sequence.
    baseline: 122,880-row row groups, one page per column chunk, V1 pages,
    PLAIN or dictionary encodings only (the sorted key column PLAIN),
    Snappy everywhere.  +pages: pages of about 1/100 of a chunk (4 KiB).
    +rowgroups: 10M-row row groups with 256 KiB pages (still >= 100 pages
    per chunk).  +encodings: every chunk takes its smallest candidate
    encoding (V2 encodings included).  +no_compression: Snappy is kept only
    where it saves more than 10%."""
    steps = PRESETS[: PRESETS.index(name) + 1]
    cols = wide_cols()
    cols[6] = dataclasses.replace(cols[6], encoding=PLAIN)  # V1 defaults: no DELTA
    spec = FileSpec(cols=cols, num_rows=rows, rg_rows=122_880, page_bytes=1 << 30, codec=SNAPPY,
                    seed=seed, name=f"preset {name}")
    if "+pages" in steps:
        spec.page_bytes = 4 * KiB
    if "+rowgroups" in steps:
        spec.rg_rows = 10_000_000
        spec.page_bytes = 256 * KiB
    if "+encodings" in steps:
        spec.encoding_search = True
    if "+no_compression" in steps:
        spec.min_saving_pct = 10
    return spec
