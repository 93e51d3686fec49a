"""Pins for the CPU oracle's building blocks, each against something other
than the oracle itself: hand-derived byte fixtures (tests/golden/), a
brute-force bit reader on tiny inputs, closed forms, Python big-integer
arithmetic, and pyarrow's independent Snappy codec."""
import itertools

import numpy as np
import io

import pyarrow as pa
import pyarrow.parquet as pq
import pytest

import datagen as dg
import oracle
from tests import golden_io

# ---------------------------------------------------------------------------
# hand-derived fixtures
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("fx", golden_io.fixtures("hybrid"), ids=lambda d: d["_name"])
def test_hybrid_golden(fx):
    w, n = int(fx["bit_width"]), int(fx["count"])
    if fx["kind"] == "hybrid_error":
        with pytest.raises(oracle.OracleError):
            oracle.hybrid_decode(fx["bytes"], w, n)
        return
    vals, used = oracle.hybrid_decode(fx["bytes"], w, n)
    assert vals.tolist() == [int(x) for x in fx["values"].split()]
    assert used == len(fx["bytes"])


@pytest.mark.parametrize("fx", golden_io.fixtures("snappy"), ids=lambda d: d["_name"])
def test_snappy_golden(fx):
    if fx["kind"] == "snappy_error":
        with pytest.raises(oracle.OracleError):
            oracle.snappy_decompress(fx["bytes"], 64)
        return
    assert oracle.snappy_decompress(fx["bytes"], 4096) == fx["text"].encode()


def _signed(v, is32):
    bits = 32 if is32 else 64
    v = int(v) & ((1 << bits) - 1)
    return v - (1 << bits) if v >> (bits - 1) else v


@pytest.mark.parametrize("fx", golden_io.fixtures("delta"), ids=lambda d: d["_name"])
def test_delta_golden(fx):
    is32, n = bool(int(fx["is32"])), int(fx["count"])
    if fx["kind"] == "delta_error":
        with pytest.raises(oracle.OracleError):
            oracle.delta_decode(fx["bytes"], is32, n)
        return
    vals, used = oracle.delta_decode(fx["bytes"], is32, n)
    assert [_signed(v, is32) for v in vals.tolist()] == [int(x) for x in fx["values"].split()]
    assert used == len(fx["bytes"])


@pytest.mark.parametrize("fx", golden_io.fixtures("page_header"), ids=lambda d: d["_name"])
def test_page_header_golden(fx):
    h, n = oracle.page_header(fx["bytes"])
    assert n == int(fx["header_len"])
    for k in ("type", "uncompressed_size", "compressed_size", "num_values", "encoding",
              "num_nulls", "num_rows", "def_len", "rep_len", "is_compressed"):
        if k in fx:
            assert getattr(h, k) == int(fx[k]), k


# ---------------------------------------------------------------------------
# brute force on tiny inputs: a trivially written bit reader
# ---------------------------------------------------------------------------


def _bits_lsb_first(data: bytes):
    for byte in data:
        for j in range(8):
            yield (byte >> j) & 1


def _brute_bitpacked(payload: bytes, w: int, n: int):
    bits = list(_bits_lsb_first(payload))
    return [sum(bits[i * w + j] << j for j in range(w)) for i in range(n)]


@pytest.mark.parametrize("w", [1, 2, 3, 5, 7, 8])
def test_hybrid_bitpacked_bruteforce(w):
    # every 1-group bit-packed run whose w-byte payload is one of a set of
    # exhaustive (w<=2: all 2^(8w) strings) or sampled byte strings
    rng = np.random.default_rng(w)
    if w <= 2:
        payloads = [bytes(t) for t in itertools.product(range(256), repeat=w)]
    else:
        payloads = [rng.integers(0, 256, w, dtype=np.uint8).tobytes() for _ in range(3000)]
    for p in payloads:
        got, used = oracle.hybrid_decode(b"\x03" + p, w, 8)
        assert got.tolist() == _brute_bitpacked(p, w, 8)
        assert used == 1 + w


def test_hybrid_random_streams_vs_bruteforce():
    # random mixes of RLE and bit-packed runs, encoded here by hand-rolled
    # Python (value -> bytes), decoded by the oracle
    rng = np.random.default_rng(7)
    for _ in range(300):
        w = int(rng.integers(0, 33))
        stream, expect = bytearray(), []
        for _ in range(int(rng.integers(1, 6))):
            if rng.random() < 0.5:
                run = int(rng.integers(0, 40))
                v = int(rng.integers(0, 1 << w)) if w else 0
                hdr = run << 1
                while True:
                    b = hdr & 0x7F
                    hdr >>= 7
                    stream.append(b | (0x80 if hdr else 0))
                    if not hdr:
                        break
                stream += v.to_bytes((w + 7) // 8, "little")
                expect += [v] * run
            else:
                g = int(rng.integers(1, 5))
                vals = [int(x) for x in rng.integers(0, 1 << w, 8 * g, dtype=np.uint64)] if w else [0] * (8 * g)
                acc = 0
                for i, v in enumerate(vals):
                    acc |= v << (i * w)
                stream.append((g << 1) | 1)
                stream += acc.to_bytes(g * w, "little")
                expect += vals
        n = len(expect)
        got, _ = oracle.hybrid_decode(bytes(stream), w, n)
        assert got.tolist() == expect


# ---------------------------------------------------------------------------
# DELTA_BINARY_PACKED: closed forms and big-integer arithmetic
# ---------------------------------------------------------------------------


def _uleb(v):
    out = bytearray()
    while True:
        b = v & 0x7F
        v >>= 7
        out.append(b | (0x80 if v else 0))
        if not v:
            return bytes(out)


def _zz(v):
    return (v << 1) ^ (v >> 63) if v >= 0 else ((-v) << 1) - 1


def _delta_stream(values, is32, block=128, mini=4):
    """Encoder written from the format description, with Python integers."""
    bits = 32 if is32 else 64
    mask = (1 << bits) - 1
    out = bytearray(_uleb(block) + _uleb(mini) + _uleb(len(values)))
    out += _uleb(_zz(_signed(values[0], is32) if values else 0))
    per = block // mini
    deltas = [_signed((values[i] - values[i - 1]) & mask, is32) for i in range(1, len(values))]
    for b0 in range(0, len(deltas), block):
        blk = deltas[b0:b0 + block]
        mn = min(blk)
        out += _uleb(_zz(mn))
        us = [(d - mn) & mask for d in blk]
        nm = (len(us) + per - 1) // per
        widths = [max(u.bit_length() for u in us[m * per:(m + 1) * per]) if m < nm else 0 for m in range(mini)]
        out += bytes(widths)
        for m in range(nm):
            chunk = us[m * per:(m + 1) * per] + [0] * (per - len(us[m * per:(m + 1) * per]))
            acc = 0
            for i, u in enumerate(chunk):
                acc |= u << (i * widths[m])
            out += acc.to_bytes(per * widths[m] // 8, "little")
    return bytes(out)


def test_delta_arithmetic_progression_closed_form():
    for first, step, n in [(0, 0, 1), (5, 3, 1000), (-7, -2, 513), (1 << 40, 12345, 300)]:
        vals = [first + step * k for k in range(n)]
        data = _delta_stream([v & ((1 << 64) - 1) for v in vals], False)
        got, used = oracle.delta_decode(data, False, n)
        assert [_signed(v, False) for v in got.tolist()] == vals
        assert used == len(data)


@pytest.mark.parametrize("is32", [False, True])
def test_delta_random_vs_bigint(is32):
    rng = np.random.default_rng(11 + is32)
    bits = 32 if is32 else 64
    for _ in range(40):
        n = int(rng.integers(1, 700))
        kind = rng.integers(0, 3)
        if kind == 0:   # full-range random: widths up to the physical width
            vals = [int(x) for x in rng.integers(0, 1 << 62, n)]
            vals = [(v * 4 + int(rng.integers(0, 4))) & ((1 << bits) - 1) for v in vals]
        elif kind == 1:  # extremes, wrap-around deltas
            ext = [0, (1 << (bits - 1)) - 1, 1 << (bits - 1), (1 << bits) - 1, 1]
            vals = [ext[int(i)] for i in rng.integers(0, len(ext), n)]
        else:            # sorted keys with small gaps
            start = int(rng.integers(0, 1 << 30))
            vals = list(np.cumsum(rng.integers(1, 9, n)) + start)
            vals = [int(v) & ((1 << bits) - 1) for v in vals]
        block = int(rng.choice([128, 256]))
        mini = int(rng.choice([1, 2, 4])) if block == 128 else int(rng.choice([2, 4, 8]))
        data = _delta_stream(vals, is32, block, mini)
        got, used = oracle.delta_decode(data + b"\xab\xcd", is32, n)   # trailing bytes are ignored
        assert [int(v) & ((1 << bits) - 1) for v in got.tolist()] == vals
        assert used == len(data)


def test_delta_rejects_bad_header():
    with pytest.raises(oracle.OracleError):   # block size not a multiple of 128
        oracle.delta_decode(_uleb(100) + _uleb(4) + _uleb(1) + _uleb(0), False, 1)
    with pytest.raises(oracle.OracleError):   # miniblock size not a multiple of 32
        oracle.delta_decode(_uleb(128) + _uleb(8) + _uleb(1) + _uleb(0), False, 1)
    # INT32 miniblock wider than 32 bits
    bad = _uleb(128) + _uleb(4) + _uleb(2) + _uleb(0) + _uleb(0) + bytes([33, 0, 0, 0]) + bytes(33 * 4)
    with pytest.raises(oracle.OracleError):
        oracle.delta_decode(bad, True, 2)


# ---------------------------------------------------------------------------
# Snappy against an independent implementation (pyarrow)
# ---------------------------------------------------------------------------


def _snappy_inputs():
    rng = np.random.default_rng(3)
    yield b""
    yield b"a"
    yield bytes(range(256)) * 300                                   # periodic: copy-heavy
    yield rng.integers(0, 256, 200_000, dtype=np.uint8).tobytes()    # incompressible
    yield b"x" * 100_000                                           # long run, overlapping copies
    yield rng.integers(97, 101, 150_000, dtype=np.uint8).tobytes()   # small alphabet
    yield (b"parquet-page-" * 9000)[:100_003]


@pytest.mark.parametrize("data", list(_snappy_inputs()), ids=lambda d: f"len{len(d)}")
def test_snappy_vs_pyarrow(data):
    codec = pa.Codec("snappy")
    comp = codec.compress(data, asbytes=True)
    assert oracle.snappy_decompress(comp, len(data) + 16) == data


def _tag_forms(stream):
    """(length-byte counts of the literals, tag forms of the copies) in a raw
    Snappy stream, by a walk over its element tags."""
    i = 0
    while stream[i] & 0x80:  # the uncompressed length
        i += 1
    i += 1
    lit, cop = set(), set()
    while i < len(stream):
        t = stream[i]
        if t & 3 == 0:
            nb = max(0, (t >> 2) - 59)
            n = (int.from_bytes(stream[i + 1:i + 1 + nb], "little") if nb else t >> 2) + 1
            lit.add(nb)
            i += 1 + nb + n
        else:
            cop.add(t & 3)
            i += (2, 3, 5)[(t & 3) - 1]
    return lit, cop


@pytest.mark.parametrize("data", list(_snappy_inputs())[2:], ids=lambda d: f"len{len(d)}")
def test_snappy_every_tag_form(data):
    """The fixture writer's varied-forms streams (literal lengths in 0-4 extra
    bytes, copies with 1-, 2- and 4-byte offsets) decode to the input with
    pyarrow's codec and with the oracle."""
    comp = dg.snappy_compress(data, varied_forms=True)
    assert pa.Codec("snappy").decompress(comp, len(data), asbytes=True) == data
    assert oracle.snappy_decompress(comp, len(data) + 16) == data


def test_snappy_varied_forms_cover_every_tag_form():
    """On an input with many short matches the varied-forms stream holds
    every literal length form and every copy form."""
    data = np.random.default_rng(3).integers(97, 101, 150_000, dtype=np.uint8).tobytes()
    lit, cop = _tag_forms(dg.snappy_compress(data, varied_forms=True))
    assert lit == {0, 1, 2, 3, 4} and cop == {1, 2, 3}
    lit0, cop0 = _tag_forms(dg.snappy_compress(data))
    assert 3 not in cop0  # the plain matcher never writes 4-byte offsets


# ---------------------------------------------------------------------------
# BYTE_STREAM_SPLIT, DELTA_LENGTH_BYTE_ARRAY, DELTA_BYTE_ARRAY
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("fx", golden_io.fixtures("bss"), ids=lambda d: d["_name"])
def test_byte_stream_split_golden(fx):
    vals, used = oracle.byte_stream_split_decode(fx["bytes"], int(fx["width"]), int(fx["count"]))
    assert [int(v) for v in vals] == [int(x) for x in fx["values"].split()]
    assert used == len(fx["bytes"])


def test_byte_stream_split_is_a_transpose():
    """Brute force: the decode is the byte transpose of the value matrix
    (numpy's own view of the little-endian bytes)."""
    rng = np.random.default_rng(11)
    for w, dt in ((4, np.uint32), (8, np.uint64)):
        for n in (0, 1, 7, 100):
            v = rng.integers(0, np.iinfo(dt).max, n, dtype=dt, endpoint=True)
            enc = v.view(np.uint8).reshape(n, w).T.copy().tobytes()
            got, used = oracle.byte_stream_split_decode(enc, w, n)
            assert (got.astype(dt) == v).all() and used == n * w
    with pytest.raises(oracle.OracleError):
        oracle.byte_stream_split_decode(b"\x00" * 7, 4, 2)


@pytest.mark.parametrize("fx", golden_io.fixtures("dlba"), ids=lambda d: d["_name"])
def test_delta_length_golden(fx):
    strs, used = oracle.delta_length_decode(fx["bytes"], int(fx["count"]))
    assert strs == [s.encode() for s in fx["strings"].split()]
    assert used == len(fx["bytes"])


@pytest.mark.parametrize("fx", golden_io.fixtures("dba"), ids=lambda d: d["_name"])
def test_delta_byte_array_golden(fx):
    strs, used = oracle.delta_byte_array_decode(fx["bytes"], int(fx["count"]))
    assert strs == [s.encode() for s in fx["strings"].split()]
    assert used == len(fx["bytes"])


def test_delta_byte_array_rejects_bad_prefixes():
    """A first prefix length above 0, or a prefix longer than the previous
    string, is corrupt (the golden stream with its prefix lengths edited)."""
    fx = golden_io.fixtures("dba")[0]
    b = bytearray(fx["bytes"])
    b[4] = 0x02  # first prefix length 1 (zigzag 2)
    with pytest.raises(oracle.OracleError):
        oracle.delta_byte_array_decode(bytes(b), 4)
    b = bytearray(fx["bytes"])
    b[5] = 0x05  # min delta -3: prefix lengths 0 1 1 -2
    with pytest.raises(oracle.OracleError):
        oracle.delta_byte_array_decode(bytes(b), 4)


def test_string_delta_encodings_vs_pyarrow():
    """Random strings with long shared prefixes (sorted), empty strings and
    repeats, written by pyarrow as DELTA_LENGTH_BYTE_ARRAY and
    DELTA_BYTE_ARRAY: the oracle's column equals pyarrow's read."""
    rng = np.random.default_rng(12)
    words = sorted(("%s/%d/%s" % ("p" * int(rng.integers(0, 30)), int(rng.integers(0, 1000)),
                                 "x" * int(rng.integers(0, 5)))).encode() for _ in range(5000))
    words += [b"", b"", words[3], words[3]]
    t = pa.table({"dlba": pa.array(words, type=pa.binary()), "dba": pa.array(words, type=pa.binary())})
    bio = io.BytesIO()
    pq.write_table(t, bio, use_dictionary=False, data_page_size=4096, data_page_version="2.0",
                   column_encoding={"dlba": "DELTA_LENGTH_BYTE_ARRAY", "dba": "DELTA_BYTE_ARRAY"})
    f = oracle.File(np.frombuffer(bio.getvalue(), dtype=np.uint8))
    for c in range(2):
        o = f.read(c)
        ch, off = o["chars"].tobytes(), o["offsets"]
        assert [ch[off[i]:off[i + 1]] for i in range(len(words))] == words
