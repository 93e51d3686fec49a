"""CPU oracle for the Parquet column-chunk scan.

TEST INFRASTRUCTURE ONLY: the plain, single-threaded reader in ``oracle.c``
that the GPU reader is checked against bit for bit.  Only ``tests/``, the
smoke check and the benchmark's CPU-baseline leg use it; the GPU product path
never imports it, and it shares no code with that path.

Every function here only marshals arguments; the decoding itself is in
``oracle.c`` (see its header for the rules it follows and where they come
from).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
# A test may point this at a deliberately broken build of oracle.c to show
# that the pins catch the mistake.
_SO = os.environ.get("PQ_ORACLE_SO", _SO)

ORC_OK, ORC_EINVAL, ORC_ECORRUPT, ORC_EUNSUPPORTED, ORC_ENOMEM = 0, -1, -2, -3, -4


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class _Column(ctypes.Structure):
    _fields_ = [
        ("rows", ctypes.c_int64), ("values", ctypes.c_void_p), ("validity", ctypes.c_void_p),
        ("offsets", ctypes.c_void_p), ("chars", ctypes.c_void_p), ("chars_len", ctypes.c_int64),
        ("pages", ctypes.c_int64), ("dict_pages", ctypes.c_int64),
    ]


class PageHeader(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "type", "uncompressed_size", "compressed_size", "num_values", "encoding", "num_nulls",
        "num_rows", "def_len", "rep_len", "is_compressed", "has_sub")]


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", src, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        vp, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
        L.orc_open.argtypes = [vp, u64, ctypes.POINTER(vp)]
        L.orc_close.argtypes = [vp]
        L.orc_num_columns.argtypes = [vp]
        L.orc_num_row_groups.argtypes = [vp]
        L.orc_row_group_rows.argtypes = [vp, ctypes.c_int]
        L.orc_row_group_rows.restype = i64
        L.orc_column_type.argtypes = [vp, ctypes.c_int]
        L.orc_column_optional.argtypes = [vp, ctypes.c_int]
        L.orc_read_column.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Column)]
        L.orc_column_free.argtypes = [ctypes.POINTER(_Column)]
        L.orc_last_error.restype = ctypes.c_char_p
        L.orc_hybrid_decode.argtypes = [vp, u64, ctypes.c_int, i64, vp]
        L.orc_hybrid_decode.restype = i64
        L.orc_delta_decode.argtypes = [vp, u64, ctypes.c_int, i64, vp]
        L.orc_delta_decode.restype = i64
        L.orc_byte_stream_split_decode.argtypes = [vp, u64, ctypes.c_int, i64, vp]
        L.orc_byte_stream_split_decode.restype = i64
        L.orc_delta_length_decode.argtypes = [vp, u64, i64, vp, vp]
        L.orc_delta_length_decode.restype = i64
        L.orc_delta_byte_array_decode.argtypes = [vp, u64, i64, ctypes.POINTER(vp), ctypes.POINTER(u64), vp, vp]
        L.orc_delta_byte_array_decode.restype = i64
        L.orc_snappy_decompress.argtypes = [vp, u64, vp, u64]
        L.orc_snappy_decompress.restype = i64
        L.orc_page_header_parse.argtypes = [vp, u64, ctypes.POINTER(PageHeader)]
        L.orc_page_header_parse.restype = i64
        _lib = L
    return _lib


def _err(code: int):
    raise OracleError(code, lib().orc_last_error().decode())


def _buf(data):
    a = np.frombuffer(bytes(data), dtype=np.uint8) if not isinstance(data, np.ndarray) else data
    return np.ascontiguousarray(a, dtype=np.uint8)


def hybrid_decode(data, bit_width: int, count: int):
    """RLE/bit-packed hybrid stream -> (values uint32[count], bytes consumed)."""
    b = _buf(data)
    out = np.zeros(max(count, 1), dtype=np.uint32)
    n = lib().orc_hybrid_decode(b.ctypes.data, b.size, bit_width, count, out.ctypes.data)
    if n < 0:
        raise OracleError(int(n), "hybrid stream")
    return out[:count], int(n)


def delta_decode(data, is32: bool, count: int):
    """DELTA_BINARY_PACKED stream -> (values uint64[count], bytes consumed)."""
    b = _buf(data)
    out = np.zeros(max(count, 1), dtype=np.uint64)
    n = lib().orc_delta_decode(b.ctypes.data, b.size, 1 if is32 else 0, count, out.ctypes.data)
    if n < 0:
        raise OracleError(int(n), "delta stream")
    return out[:count], int(n)


def byte_stream_split_decode(data, width: int, count: int):
    """(values as uint64 array, bytes used) of a BYTE_STREAM_SPLIT stream."""
    b = _buf(data)
    out = np.zeros(max(count, 1), dtype=np.uint64)
    n = lib().orc_byte_stream_split_decode(b.ctypes.data, b.size, width, count, out.ctypes.data)
    if n < 0:
        _err(n)
    return out[:count], n


def delta_length_decode(data, count: int):
    """(list of byte strings, bytes used) of a DELTA_LENGTH_BYTE_ARRAY stream."""
    b = _buf(data)
    pos = np.zeros(max(count, 1), dtype=np.uint64)
    ln = np.zeros(max(count, 1), dtype=np.uint32)
    n = lib().orc_delta_length_decode(b.ctypes.data, b.size, count, pos.ctypes.data, ln.ctypes.data)
    if n < 0:
        _err(n)
    raw = b.tobytes()
    return [raw[int(pos[k]):int(pos[k]) + int(ln[k])] for k in range(count)], n


def delta_byte_array_decode(data, count: int):
    """(list of byte strings, bytes used) of a DELTA_BYTE_ARRAY stream."""
    b = _buf(data)
    pos = np.zeros(max(count, 1), dtype=np.uint64)
    ln = np.zeros(max(count, 1), dtype=np.uint32)
    mat = ctypes.c_void_p()
    cap = ctypes.c_uint64(0)
    n = lib().orc_delta_byte_array_decode(b.ctypes.data, b.size, count, ctypes.byref(mat), ctypes.byref(cap),
                                          pos.ctypes.data, ln.ctypes.data)
    try:
        if n < 0:
            _err(n)
        raw = ctypes.string_at(mat.value, cap.value) if mat.value else b""
        return [raw[int(pos[k]):int(pos[k]) + int(ln[k])] for k in range(count)], n
    finally:
        if mat.value:
            ctypes.CDLL(None).free(mat)


def snappy_decompress(data, cap: int) -> bytes:
    b = _buf(data)
    out = np.zeros(max(cap, 1), dtype=np.uint8)
    n = lib().orc_snappy_decompress(b.ctypes.data, b.size, out.ctypes.data, cap)
    if n < 0:
        raise OracleError(int(n), "snappy stream")
    return out[:n].tobytes()


def page_header(data):
    """-> (PageHeader, header length)."""
    b = _buf(data)
    h = PageHeader()
    n = lib().orc_page_header_parse(b.ctypes.data, b.size, ctypes.byref(h))
    if n < 0:
        raise OracleError(int(n), "page header")
    return h, int(n)


_NP = {1: np.int32, 2: np.int64, 5: np.float64}


class File:
    """An opened Parquet file held in host memory."""

    def __init__(self, data):
        self._buf = _buf(data)
        self._h = ctypes.c_void_p()
        rc = lib().orc_open(self._buf.ctypes.data, self._buf.size, ctypes.byref(self._h))
        if rc != 0:
            _err(rc)

    def close(self):
        if self._h:
            lib().orc_close(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_columns(self) -> int:
        return lib().orc_num_columns(self._h)

    @property
    def num_row_groups(self) -> int:
        return lib().orc_num_row_groups(self._h)

    def row_group_rows(self, rg: int) -> int:
        return lib().orc_row_group_rows(self._h, rg)

    def column_type(self, col: int) -> int:
        return lib().orc_column_type(self._h, col)

    def column_optional(self, col: int) -> bool:
        return bool(lib().orc_column_optional(self._h, col))

    def decode_seconds(self, col: int, rg_begin: int = 0, rg_end: Optional[int] = None):
        """Times one call of the oracle's column decode (its own output
        allocation included, no copy into Python arrays); returns (seconds,
        decoded bytes: validity + values, or offsets + chars)."""
        import time
        if rg_end is None:
            rg_end = self.num_row_groups
        c = _Column()
        t0 = time.perf_counter()
        rc = lib().orc_read_column(self._h, col, rg_begin, rg_end, ctypes.byref(c))
        dt = time.perf_counter() - t0
        if rc != 0:
            _err(rc)
        try:
            rows = c.rows
            t = self.column_type(col)
            n = (rows + 7) // 8
            n += 8 * (rows + 1) + c.chars_len if t == 6 else rows * np.dtype(_NP[t]).itemsize
            return dt, n
        finally:
            lib().orc_column_free(ctypes.byref(c))

    def read(self, col: int, rg_begin: int = 0, rg_end: Optional[int] = None) -> dict:
        """Decoded rows of `col` over [rg_begin, rg_end): a dict with
        "values" (fixed width) or "offsets"+"chars" (BYTE_ARRAY), "validity",
        and page counts."""
        if rg_end is None:
            rg_end = self.num_row_groups
        c = _Column()
        rc = lib().orc_read_column(self._h, col, rg_begin, rg_end, ctypes.byref(c))
        if rc != 0:
            _err(rc)
        try:
            rows = c.rows
            t = self.column_type(col)
            nb = (rows + 7) // 8
            out = {"rows": rows, "pages": c.pages, "dict_pages": c.dict_pages}
            v = np.zeros(nb, dtype=np.uint8)
            if nb:
                ctypes.memmove(v.ctypes.data, c.validity, nb)
            out["validity"] = v
            if t == 6:
                off = np.zeros(rows + 1, dtype=np.int64)
                ctypes.memmove(off.ctypes.data, c.offsets, 8 * (rows + 1))
                ch = np.zeros(c.chars_len, dtype=np.uint8)
                if c.chars_len:
                    ctypes.memmove(ch.ctypes.data, c.chars, c.chars_len)
                out["offsets"], out["chars"] = off, ch
            else:
                vals = np.zeros(rows, dtype=_NP[t])
                if rows:
                    ctypes.memmove(vals.ctypes.data, c.values, vals.nbytes)
                out["values"] = vals
            return out
        finally:
            lib().orc_column_free(ctypes.byref(c))
