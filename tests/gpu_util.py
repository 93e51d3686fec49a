"""Helpers shared by the GPU tests: run the HIP scan through the C ABI and
compare every output buffer with the CPU oracle, byte for byte.

Every output buffer is pre-filled with 0xAB and followed by a 4 KiB guard
region of 0xAB, so a byte the scan should write and does not (a skipped
validity word, a null slot, an offset) differs from the oracle, and a byte
written past a buffer shows up in its guard."""
import sys

import numpy as np

import oracle

POISON = 0xAB
GUARD = 4096


def gpu_scan(data, columns=None, rg_begin=0, rg_end=None):
    import paper_2602_17335_amd as pqs
    buf, n = pqs.to_device(data)
    f = pqs.DeviceFile(buf, n)
    if columns is None:
        columns = list(range(f.num_columns))
    out = f.scan(columns, rg_begin, rg_end, poison=POISON, guard=GUARD)
    return f, out


def check_guards(g, name=""):
    for k, gd in enumerate(g.get("guards", [])):
        a = gd.cpu().numpy()
        if not (a == 0xAB).all():
            bad = np.nonzero(a != 0xAB)[0]
            raise AssertionError(f"{name}: guard region {k} written at bytes {bad[:10]} (of {bad.size})")


def _np(x):
    return x if isinstance(x, np.ndarray) else x.cpu().numpy()


def compare_column(o, g, name=""):
    """o: oracle dict, g: GPU dict of torch tensors (or host numpy arrays)."""
    rows = o["rows"]
    assert g["rows"] == rows, (name, g["rows"], rows)
    gv = _np(g["validity"])
    assert gv.size == o["validity"].size
    if not (gv == o["validity"]).all():
        bad = np.nonzero(gv != o["validity"])[0]
        raise AssertionError(f"{name}: validity differs at bytes {bad[:10]} (of {bad.size})")
    if "validity_words" in g:
        # the whole 32-bit words the library writes: bits past `rows` are 0
        words = _np(g["validity_words"])
        exp = np.zeros(words.size, dtype=np.uint8)
        exp[: o["validity"].size] = o["validity"]
        if not (words == exp).all():
            bad = np.nonzero(words != exp)[0]
            raise AssertionError(f"{name}: validity word tail differs at bytes {bad[:10]} (of {bad.size})")
    if "offsets" in o:
        goff = _np(g["offsets"])
        if not (goff == o["offsets"]).all():
            bad = np.nonzero(goff != o["offsets"])[0]
            raise AssertionError(f"{name}: offsets differ at rows {bad[:10]} (of {bad.size}): "
                                 f"gpu {goff[bad[:5]]} oracle {o['offsets'][bad[:5]]}")
        gch = _np(g["chars"])
        assert gch.size == o["chars"].size, (name, gch.size, o["chars"].size)
        if not (gch == o["chars"]).all():
            bad = np.nonzero(gch != o["chars"])[0]
            raise AssertionError(f"{name}: chars differ at {bad[:10]} (of {bad.size})")
    else:
        gvals = _np(g["values"]).view(np.uint8)
        ov = o["values"].view(np.uint8)
        if not (gvals == ov).all():
            w = o["values"].itemsize
            bad = np.nonzero((gvals != ov).reshape(-1, w).any(axis=1))[0]
            raise AssertionError(f"{name}: values differ at rows {bad[:10]} (of {bad.size}): "
                                 f"gpu {_np(g['values'])[bad[:5]]} oracle {o['values'][bad[:5]]}")
    check_guards(g, name)


def check_file(data, columns=None, rg_begin=0, rg_end=None, label=""):
    print(f"[gpu] {label}: {len(data)} bytes cols={columns} rg=[{rg_begin},{rg_end})", flush=True)
    sys.stdout.flush()
    f, out = gpu_scan(data, columns, rg_begin, rg_end)
    ofile = oracle.File(data)
    if rg_end is None:
        rg_end = ofile.num_row_groups
    for c, g in out.items():
        compare_column(ofile.read(c, rg_begin, rg_end), g, f"{label} col{c}")
    return f
