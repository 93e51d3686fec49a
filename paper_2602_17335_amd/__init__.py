"""MI355X Parquet column-chunk scanner: Python binding of libpqscan.so.

Argument marshalling only.  Every step of the scan runs in the HIP kernels
behind the C ABI in include/pq.h; PyTorch supplies device memory and the
stream.  There is no CPU fallback: importing fails loudly when the library is
missing, and the scan needs a GPU.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpqscan.so")

PQ_OK, PQ_EINVAL, PQ_ECORRUPT, PQ_EUNSUPPORTED, PQ_ENOMEM, PQ_EHIP, PQ_ECAPACITY, PQ_EBUSY = 0, -1, -2, -3, -4, -5, -7, -8
INT32, INT64, DOUBLE, BYTE_ARRAY = 1, 2, 5, 6
_WIDTH = {INT32: 4, INT64: 8, DOUBLE: 8}

EXPORTS = ("pq_open_device", "pq_num_row_groups", "pq_num_columns", "pq_column_info_get", "pq_row_group_rows",
           "pq_file_stats_get", "pq_column_bytes", "pq_column_encodings", "pq_plan", "pq_scan", "pq_scan_check", "pq_profile",
           "pq_profile_read", "pq_close", "pq_last_error", "pq_tuning_default", "pq_plan_batch", "pq_scan_batch",
           "pq_autotune_batch", "pq_scan_noalloc", "pq_server_create", "pq_server_submit", "pq_server_wait",
           "pq_server_release", "pq_server_stats_get", "pq_server_destroy", "pq_server_last_error",
           "pq_open_host", "pq_scan_streamed", "pq_copy_probe")
FORM_BATCHED, FORM_PER_PAGE = 0, 1
TUNE_CLASSES = 54


class PqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pq error {code}: {msg}")
        self.code = code


class ColumnInfo(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("nullable", ctypes.c_int32), ("name", ctypes.c_char * 64)]


class ScanSizes(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("workspace_bytes", ctypes.c_uint64), ("chars_bytes", ctypes.c_int64 * 64)]


class ColumnOut(ctypes.Structure):
    _fields_ = [("values", ctypes.c_void_p), ("validity", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("chars", ctypes.c_void_p), ("chars_capacity", ctypes.c_uint64)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


class FileStats(ctypes.Structure):
    _fields_ = [("pages", ctypes.c_int64), ("dict_pages", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("compressed_pages", ctypes.c_int64), ("encoded_bytes", ctypes.c_uint64),
                ("uncompressed_bytes", ctypes.c_uint64), ("open_ms_device", ctypes.c_double),
                ("device_bytes", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("file", ctypes.c_void_p), ("col_mask", ctypes.c_uint64), ("rg_begin", ctypes.c_int32),
                ("rg_end", ctypes.c_int32), ("outs", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32), ("queues", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("tiles_per_unit", ctypes.c_uint8 * TUNE_CLASSES),
                ("pad2_", ctypes.c_uint8 * 2)]

    def to_dict(self):
        return {"form": self.form, "waves_per_cu": self.waves_per_cu, "queues": self.queues,
                "tiles_per_unit": list(self.tiles_per_unit)}

    @classmethod
    def from_dict(cls, d):
        t = tuning_default()
        t.form, t.waves_per_cu, t.queues = d["form"], d["waves_per_cu"], d["queues"]
        for i, v in enumerate(d["tiles_per_unit"]):
            t.tiles_per_unit[i] = v
        return t


class Served(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_outs", ctypes.c_int32), ("shared", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("rows", ctypes.c_int64), ("decoded_bytes", ctypes.c_uint64),
                ("queue_ms", ctypes.c_double), ("latency_ms", ctypes.c_double), ("outs", ColumnOut * 64)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "failed", "batches", "cache_hits", "evictions",
                                               "decoded_bytes", "budget_bytes", "used_bytes", "resident_results")]


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libpqscan.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2602_17335_amd.build` "
                              "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, i32, i64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
        L.pq_open_device.argtypes = [vp, u64, vp, ctypes.POINTER(vp)]
        L.pq_open_host.argtypes = [vp, u64, vp, ctypes.POINTER(vp)]
        L.pq_copy_probe.argtypes = [vp, vp, u64, vp]
        L.pq_scan_streamed.argtypes = [vp, u64, i32, i32, ctypes.POINTER(ColumnOut), i32, vp, u64, vp, vp]
        L.pq_num_row_groups.argtypes = [vp, ctypes.POINTER(i32)]
        L.pq_num_columns.argtypes = [vp, ctypes.POINTER(i32)]
        L.pq_column_info_get.argtypes = [vp, i32, ctypes.POINTER(ColumnInfo)]
        L.pq_row_group_rows.argtypes = [vp, i32, ctypes.POINTER(i64)]
        L.pq_file_stats_get.argtypes = [vp, ctypes.POINTER(FileStats)]
        L.pq_plan.argtypes = [vp, u64, i32, i32, ctypes.POINTER(ScanSizes)]
        L.pq_column_bytes.argtypes = [vp, i32, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.pq_column_encodings.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_uint32)]
        L.pq_profile.argtypes = [vp, i32]
        L.pq_profile_read.argtypes = [vp, ctypes.POINTER(KernelTime), i32, ctypes.POINTER(i32)]
        L.pq_scan.argtypes = [vp, u64, i32, i32, ctypes.POINTER(ColumnOut), i32, vp, u64, vp]
        L.pq_scan_check.argtypes = [vp, vp, vp]
        L.pq_tuning_default.argtypes = [ctypes.POINTER(Tuning)]
        L.pq_plan_batch.argtypes = [ctypes.POINTER(Request), i32, ctypes.POINTER(u64), ctypes.POINTER(i64), i32]
        L.pq_scan_batch.argtypes = [ctypes.POINTER(Request), i32, ctypes.POINTER(Tuning), vp, u64, vp]
        L.pq_autotune_batch.argtypes = [ctypes.POINTER(Request), i32, vp, u64, vp, i32, ctypes.POINTER(Tuning),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.pq_server_create.argtypes = [ctypes.POINTER(vp), i32, u64, i32, i32, ctypes.POINTER(Tuning), ctypes.POINTER(vp)]
        L.pq_server_submit.argtypes = [vp, i32, u64, i32, i32, ctypes.POINTER(u64)]
        L.pq_server_wait.argtypes = [vp, u64, i32, ctypes.POINTER(Served)]
        L.pq_server_release.argtypes = [vp, u64]
        L.pq_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.pq_server_destroy.argtypes = [vp]
        L.pq_server_destroy.restype = None
        L.pq_server_last_error.restype = ctypes.c_char_p
        L.pq_close.argtypes = [vp]
        L.pq_close.restype = None
        L.pq_last_error.restype = ctypes.c_char_p
        for name in ("pq_open_device", "pq_num_row_groups", "pq_num_columns", "pq_column_info_get",
                     "pq_row_group_rows", "pq_file_stats_get", "pq_plan", "pq_scan", "pq_scan_check",
                     "pq_column_bytes", "pq_column_encodings", "pq_profile", "pq_profile_read",
                     "pq_tuning_default", "pq_plan_batch", "pq_scan_batch", "pq_autotune_batch",
                     "pq_server_create", "pq_server_submit", "pq_server_wait", "pq_server_release",
                     "pq_server_stats_get", "pq_open_host", "pq_scan_streamed", "pq_copy_probe"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != PQ_OK:
        raise PqError(rc, lib().pq_last_error().decode(errors="replace"))


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def copy_probe(dst, src, nbytes: int, stream=None):
    """Enqueues the library's plain streaming copy of nbytes from device
    tensor src to device tensor dst (the "% of copy" reference)."""
    _check(lib().pq_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                               ctypes.c_void_p(_stream_ptr(stream))))


def validity_bytes(rows: int) -> int:
    """Bytes the library writes for a validity bitmap of `rows` rows."""
    return (rows + 31) // 32 * 4


def to_device(data, device="cuda"):
    """Copies file bytes (numpy uint8 / bytes) into a fresh device buffer that
    is 16-byte aligned and padded to a multiple of 16 bytes."""
    import numpy as np
    import torch
    a = np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray)) else np.asarray(data, dtype=np.uint8)
    n = a.size
    buf = torch.empty((n + 15) // 16 * 16 + 16, dtype=torch.uint8, device=device)
    buf[:n].copy_(torch.from_numpy(a), non_blocking=False)
    return buf, n


class DeviceFile:
    """A Parquet file resident in device memory, opened for scanning."""

    def __init__(self, dev_buf, nbytes: Optional[int] = None, stream=None):
        self._buf = dev_buf  # keep the borrowed buffer alive
        n = dev_buf.numel() if nbytes is None else nbytes
        h = ctypes.c_void_p()
        _check(lib().pq_open_device(ctypes.c_void_p(dev_buf.data_ptr()), n, ctypes.c_void_p(_stream_ptr(stream)),
                                    ctypes.byref(h)))
        self._h = h
        self.nbytes = n

    def close(self):
        if self._h:
            lib().pq_close(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_columns(self) -> int:
        n = ctypes.c_int32()
        _check(lib().pq_num_columns(self._h, ctypes.byref(n)))
        return n.value

    @property
    def num_row_groups(self) -> int:
        n = ctypes.c_int32()
        _check(lib().pq_num_row_groups(self._h, ctypes.byref(n)))
        return n.value

    def row_group_rows(self, rg: int) -> int:
        n = ctypes.c_int64()
        _check(lib().pq_row_group_rows(self._h, rg, ctypes.byref(n)))
        return n.value

    def column_info(self, col: int) -> ColumnInfo:
        ci = ColumnInfo()
        _check(lib().pq_column_info_get(self._h, col, ctypes.byref(ci)))
        return ci

    def stats(self) -> FileStats:
        s = FileStats()
        _check(lib().pq_file_stats_get(self._h, ctypes.byref(s)))
        return s

    def column_bytes(self, col: int):
        """(encoded data-page bytes, dictionary-page bytes) of a column."""
        d, k = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().pq_column_bytes(self._h, col, ctypes.byref(d), ctypes.byref(k)))
        return d.value, k.value

    def column_encodings(self, col: int) -> int:
        """Bit mask of the Parquet encodings (Encoding enum values) used by the
        column's data pages."""
        m = ctypes.c_uint32()
        _check(lib().pq_column_encodings(self._h, col, ctypes.byref(m)))
        return m.value

    def profile(self, enable: bool):
        _check(lib().pq_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> Dict[str, tuple]:
        """{kernel: (launches, total device ms)} since profile(True)."""
        arr = (KernelTime * 16)()
        n = ctypes.c_int32()
        _check(lib().pq_profile_read(self._h, arr, 16, ctypes.byref(n)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(min(n.value, 16))}

    def plan(self, mask: int, rg_begin: int, rg_end: int) -> ScanSizes:
        sz = ScanSizes()
        _check(lib().pq_plan(self._h, mask, rg_begin, rg_end, ctypes.byref(sz)))
        return sz

    def scan_into(self, mask: int, rg_begin: int, rg_end: int, outs: Sequence[ColumnOut], workspace, stream=None):
        """Enqueues pq_scan with caller-provided buffers (no synchronisation)."""
        arr = (ColumnOut * max(len(outs), 1))(*outs)
        _check(lib().pq_scan(self._h, mask, rg_begin, rg_end, arr, len(outs), ctypes.c_void_p(workspace.data_ptr()),
                             workspace.numel(), ctypes.c_void_p(_stream_ptr(stream))))

    def check(self, workspace, stream=None):
        """Synchronises `stream` and raises the device error of the scan that
        last used `workspace`, if any."""
        _check(lib().pq_scan_check(self._h, ctypes.c_void_p(workspace.data_ptr()),
                                   ctypes.c_void_p(_stream_ptr(stream))))

    def allocate(self, columns: Sequence[int], rg_begin: int = 0, rg_end: Optional[int] = None,
                 poison: Optional[int] = None, guard: int = 0):
        """Plans a scan and allocates its workspace and output tensors.
        `poison`: byte every output buffer is filled with first (None: left
        uninitialised); `guard`: bytes after each buffer, filled with 0xAB,
        that the scan must not touch.  Returns (mask, rg_end, workspace,
        outs, tensors)."""
        import torch
        if rg_end is None:
            rg_end = self.num_row_groups
        mask = 0
        for c in columns:
            mask |= 1 << c
        sz = self.plan(mask, rg_begin, rg_end)
        ws = torch.empty(max(int(sz.workspace_bytes), 256), dtype=torch.uint8, device="cuda")
        cols = sorted(columns)
        rows = int(sz.rows)

        def buf(nbytes):
            t = torch.empty(nbytes + guard, dtype=torch.uint8, device="cuda")
            if poison is not None:
                t.fill_(poison)
            if guard:
                t[nbytes:].fill_(0xAB)
            return t

        outs, tensors = [], {}
        for k, c in enumerate(cols):
            ci = self.column_info(c)
            vbytes = max(validity_bytes(rows), 4)
            vb = buf(vbytes)
            o = ColumnOut()
            o.validity = vb.data_ptr()
            t = {"validity_buf": vb, "validity_bytes": vbytes, "rows": rows, "guard": guard}
            if ci.type == BYTE_ARRAY:
                ob = buf(8 * (rows + 1))
                nch = int(sz.chars_bytes[k])
                chars = buf(max(nch, 1))
                o.offsets, o.chars, o.chars_capacity = ob.data_ptr(), chars.data_ptr(), nch
                t.update(offsets_buf=ob, offsets=ob[: 8 * (rows + 1)].view(torch.int64), chars_buf=chars,
                         chars_bytes=nch, chars_alloc=max(nch, 1))
            else:
                dt = {INT32: torch.int32, INT64: torch.int64, DOUBLE: torch.float64}[ci.type]
                w = _WIDTH[ci.type]
                vals = buf(max(rows, 1) * w)
                o.values = vals.data_ptr()
                t.update(values_raw=vals, values_buf=vals[: max(rows, 1) * w].view(dt), value_bytes=max(rows, 1) * w)
            outs.append(o)
            tensors[c] = t
        return mask, rg_end, ws, outs, tensors

    def scan(self, columns: Sequence[int], rg_begin: int = 0, rg_end: Optional[int] = None, stream=None,
             check: bool = True, poison: Optional[int] = None, guard: int = 0) -> Dict[int, dict]:
        """Scans `columns` over row groups [rg_begin, rg_end) into new device
        tensors: {col: {"values"| "offsets","chars", "validity",
        "validity_words"}} ("validity_words": all bytes the library writes,
        whole 32-bit words)."""
        mask, rg_end, ws, outs, tensors = self.allocate(columns, rg_begin, rg_end, poison, guard)
        self.scan_into(mask, rg_begin, rg_end, outs, ws, stream)
        if check:
            self.check(ws, stream)
        res = {}
        for c, t in tensors.items():
            rows = t["rows"]
            vb = t["validity_buf"]
            d = {"validity": vb[: (rows + 7) // 8], "validity_words": vb[: validity_bytes(rows)], "rows": rows}
            guards = [vb[t["validity_bytes"]:]]
            if "offsets" in t:
                d["offsets"] = t["offsets"]
                d["chars"] = t["chars_buf"][: t["chars_bytes"]]
                guards += [t["offsets_buf"][8 * (rows + 1):], t["chars_buf"][t["chars_alloc"]:]]
            else:
                d["values"] = t["values_buf"][:rows]
                guards.append(t["values_raw"][t["value_bytes"]:])
            d["guards"] = guards
            res[c] = d
        return res


class HostFile(DeviceFile):
    """A Parquet file resident in pinned host memory (pq_open_host), scanned
    with its row groups streamed to the device while the previous one is
    decoded (pq_scan_streamed).  The copies run on `copy_stream` (a stream of
    the handle's own unless given)."""

    def __init__(self, data, stream=None, pinned: bool = True):
        import numpy as np
        import torch
        a = np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray)) else np.asarray(data, dtype=np.uint8)
        n = a.size
        buf = torch.empty(max(n, 1), dtype=torch.uint8, pin_memory=pinned)
        buf[:n].copy_(torch.from_numpy(a))
        self._buf = buf  # borrowed by the handle until close
        self._copy_stream = None
        h = ctypes.c_void_p()
        _check(lib().pq_open_host(ctypes.c_void_p(buf.data_ptr()), n, ctypes.c_void_p(_stream_ptr(stream)),
                                  ctypes.byref(h)))
        self._h = h
        self.nbytes = n

    def scan_into(self, mask: int, rg_begin: int, rg_end: int, outs: Sequence[ColumnOut], workspace, stream=None,
                  copy_stream=None):
        """Enqueues pq_scan_streamed (no synchronisation)."""
        import torch
        if copy_stream is None:
            if self._copy_stream is None:
                self._copy_stream = torch.cuda.Stream()
            copy_stream = self._copy_stream
        arr = (ColumnOut * max(len(outs), 1))(*outs)
        _check(lib().pq_scan_streamed(self._h, mask, rg_begin, rg_end, arr, len(outs),
                                      ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                      ctypes.c_void_p(copy_stream.cuda_stream), ctypes.c_void_p(_stream_ptr(stream))))


# ---------------------------------------------------------------------------
# batched scans
# ---------------------------------------------------------------------------

def tuning_default() -> Tuning:
    t = Tuning()
    _check(lib().pq_tuning_default(ctypes.byref(t)))
    return t


def batch_profile(enable: bool):
    """Per-kernel HIP-event timing of batched scans (pq_profile(NULL, ..))."""
    _check(lib().pq_profile(None, 1 if enable else 0))


def batch_profile_read() -> Dict[str, tuple]:
    arr = (KernelTime * 16)()
    n = ctypes.c_int32()
    _check(lib().pq_profile_read(None, arr, 16, ctypes.byref(n)))
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(min(n.value, 16))}


class Batch:
    """Several scan requests (file, columns, row-group range), over one or
    more DeviceFiles, planned and scanned together through pq_scan_batch.
    `requests`: [(DeviceFile, columns, rg_begin, rg_end or None)]."""

    def __init__(self, requests, poison: Optional[int] = None, guard: int = 0):
        import torch
        self.requests = []
        self._keep = []
        for f, cols, rb, re_ in requests:
            if re_ is None:
                re_ = f.num_row_groups
            mask = 0
            for c in cols:
                mask |= 1 << c
            self.requests.append((f, sorted(cols), rb, re_, mask))
        n = len(self.requests)
        self._reqs = (Request * max(n, 1))()
        for i, (f, cols, rb, re_, mask) in enumerate(self.requests):
            self._reqs[i].file = f._h.value
            self._reqs[i].col_mask = mask
            self._reqs[i].rg_begin = rb
            self._reqs[i].rg_end = re_
        ncols = sum(len(r[1]) for r in self.requests)
        ws = ctypes.c_uint64()
        chars = (ctypes.c_int64 * max(ncols, 1))()
        _check(lib().pq_plan_batch(self._reqs, n, ctypes.byref(ws), chars, ncols))
        self.workspace = torch.empty(max(int(ws.value), 256), dtype=torch.uint8, device="cuda")
        self.outputs = []  # per request {col: tensors}
        self._outs = []
        self.decoded_bytes = 0
        k = 0

        def buf(nbytes):
            t = torch.empty(nbytes + guard, dtype=torch.uint8, device="cuda")
            if poison is not None:
                t.fill_(poison)
            if guard:
                t[nbytes:].fill_(0xAB)
            return t

        for i, (f, cols, rb, re_, mask) in enumerate(self.requests):
            rows = sum(f.row_group_rows(g) for g in range(rb, re_))
            arr = (ColumnOut * max(len(cols), 1))()
            res = {}
            for j, c in enumerate(cols):
                ci = f.column_info(c)
                vbytes = max(validity_bytes(rows), 4)
                vb = buf(vbytes)
                o = arr[j]
                o.validity = vb.data_ptr()
                d = {"rows": rows, "validity": vb[: (rows + 7) // 8], "validity_words": vb[: validity_bytes(rows)],
                     "guards": [vb[vbytes:]]}
                self.decoded_bytes += (rows + 7) // 8
                if ci.type == BYTE_ARRAY:
                    ob = buf(8 * (rows + 1))
                    nch = int(chars[k])
                    ch = buf(max(nch, 1))
                    o.offsets, o.chars, o.chars_capacity = ob.data_ptr(), ch.data_ptr(), nch
                    d.update(offsets=ob[: 8 * (rows + 1)].view(torch.int64), chars=ch[:nch])
                    d["guards"] += [ob[8 * (rows + 1):], ch[max(nch, 1):]]
                    self.decoded_bytes += 8 * (rows + 1) + nch
                else:
                    dt = {INT32: torch.int32, INT64: torch.int64, DOUBLE: torch.float64}[ci.type]
                    w = _WIDTH[ci.type]
                    vals = buf(max(rows, 1) * w)
                    o.values = vals.data_ptr()
                    d["values"] = vals[: max(rows, 1) * w].view(dt)[:rows]
                    d["guards"].append(vals[max(rows, 1) * w:])
                    self.decoded_bytes += rows * w
                res[c] = d
                k += 1
            self._outs.append(arr)
            self._reqs[i].outs = ctypes.cast(arr, ctypes.c_void_p).value
            self.outputs.append(res)

    def scan(self, tuning: Optional[Tuning] = None, stream=None):
        """Enqueues the batch (no synchronisation)."""
        tp = ctypes.byref(tuning) if tuning is not None else None
        _check(lib().pq_scan_batch(self._reqs, len(self.requests), tp, ctypes.c_void_p(self.workspace.data_ptr()),
                                   self.workspace.numel(), ctypes.c_void_p(_stream_ptr(stream))))

    def check(self, stream=None):
        _check(lib().pq_scan_check(None, ctypes.c_void_p(self.workspace.data_ptr()),
                                   ctypes.c_void_p(_stream_ptr(stream))))

    def autotune(self, reps: int = 3, stream=None):
        """Runs the library's autotuner; returns (best Tuning, best ms, default ms)."""
        best = Tuning()
        bms, dms = ctypes.c_double(), ctypes.c_double()
        _check(lib().pq_autotune_batch(self._reqs, len(self.requests), ctypes.c_void_p(self.workspace.data_ptr()),
                                       self.workspace.numel(), ctypes.c_void_p(_stream_ptr(stream)), reps,
                                       ctypes.byref(best), ctypes.byref(bms), ctypes.byref(dms)))
        return best, bms.value, dms.value


# ---------------------------------------------------------------------------
# the scan server
# ---------------------------------------------------------------------------

_hip = None


def _hip_memcpy_d2h(dst_numpy, src_ptr: int):
    """Copies device bytes into a host numpy array (HIP runtime, which torch
    has already loaded)."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    if dst_numpy.nbytes:
        rc = _hip.hipMemcpy(dst_numpy.ctypes.data, ctypes.c_void_p(src_ptr), dst_numpy.nbytes, 2)
        if rc != 0:
            raise PqError(PQ_EHIP, f"hipMemcpy failed ({rc})")


def _server_check(rc: int):
    if rc != PQ_OK:
        raise PqError(rc, lib().pq_server_last_error().decode(errors="replace"))


class Server:
    """pq_server over a catalog of DeviceFiles: submit(file index, columns,
    rg range) -> id; wait(id) -> Served; fetch(id) copies a result to host
    numpy arrays; release(id)."""

    def __init__(self, files, budget_bytes: int, slots: int = 4, max_batch: int = 64,
                 tuning: Optional[Tuning] = None):
        self.files = list(files)
        arr = (ctypes.c_void_p * len(self.files))(*[f._h.value for f in self.files])
        h = ctypes.c_void_p()
        tp = ctypes.byref(tuning) if tuning is not None else None
        _server_check(lib().pq_server_create(arr, len(self.files), budget_bytes, slots, max_batch, tp,
                                             ctypes.byref(h)))
        self._h = h
        self._cols = {}

    def close(self):
        if self._h:
            lib().pq_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, file: int, columns: Sequence[int], rg_begin: int, rg_end: int) -> int:
        mask = 0
        for c in columns:
            mask |= 1 << c
        rid = ctypes.c_uint64()
        _server_check(lib().pq_server_submit(self._h, file, mask, rg_begin, rg_end, ctypes.byref(rid)))
        self._cols[rid.value] = (file, sorted(columns))
        return rid.value

    def wait(self, rid: int, timeout_ms: int = -1) -> Served:
        out = Served()
        rc = lib().pq_server_wait(self._h, rid, timeout_ms, ctypes.byref(out))
        if rc != PQ_OK:
            _server_check(rc)
        return out

    def fetch(self, rid: int, served: Served) -> Dict[int, dict]:
        """The request's columns as host numpy arrays: validity (whole words),
        values or offsets + chars."""
        import numpy as np
        file, cols = self._cols[rid]
        f = self.files[file]
        rows = served.rows
        res = {}
        for k, c in enumerate(cols):
            o = served.outs[k]
            d = {"rows": rows}
            vw = np.empty(validity_bytes(rows), dtype=np.uint8)
            _hip_memcpy_d2h(vw, o.validity)
            d["validity_words"] = vw
            d["validity"] = vw[: (rows + 7) // 8]
            t = f.column_info(c).type
            if t == BYTE_ARRAY:
                off = np.empty(rows + 1, dtype=np.int64)
                _hip_memcpy_d2h(off, o.offsets)
                ch = np.empty(int(off[-1]) if rows >= 0 else 0, dtype=np.uint8)
                _hip_memcpy_d2h(ch, o.chars)
                d["offsets"], d["chars"] = off, ch
            else:
                v = np.empty(rows, dtype={INT32: np.int32, INT64: np.int64, DOUBLE: np.float64}[t])
                _hip_memcpy_d2h(v, o.values)
                d["values"] = v
            res[c] = d
        return res

    def release(self, rid: int):
        _server_check(lib().pq_server_release(self._h, rid))
        self._cols.pop(rid, None)

    def stats(self) -> dict:
        st = ServerStats()
        _server_check(lib().pq_server_stats_get(self._h, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in ServerStats._fields_}
