#!/usr/bin/env python3
"""Benchmark of the GPU Parquet scan: decoded GB/s and % of HBM peak.

One step = one pq_scan of every selected column of a device-resident file
(Snappy decompression when the file is compressed, dictionary decode, and
the decode kernels; DELTA carries and string offsets come from the tile
prefix that pq_open_device builds once per file, outside the timed region
and reported as open_ms), with the file already in HBM when the timed
region starts.  The default workload is the 16-column
wide fact table: 64,000,000 rows, one 64M-row row group, 1 MiB pages,
uncompressed, every column OPTIONAL with 10% nulls (synthetic, seeded; it
stands in for the paper's TPC-H lineitem scans, Sec. 3 setup).

Prints one JSON line.  Per-kernel device times come from HIP events that the
library records around each kernel on the scan's stream; the dominant
kernel's algorithmic bytes over its average duration give the roofline
fraction against the MI355X's 8 TB/s HBM peak.  The CPU baseline is the
plain single-threaded oracle run over the same file on one host core.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Parquet scan decoded GB/s & % HBM peak; batched vs plain form; p99 latency"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in ("paper_2602_17335_amd/csrc/pq_scan_kernels.hip", "paper_2602_17335_amd/csrc/pq_device.hpp",
                "paper_2602_17335_amd/csrc/pq_internal.h"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def decoded_bytes(out_tensors, types):
    """Bytes of the decoded result: values (null slots included), the
    validity bitmap, int64 offsets and chars."""
    total = 0
    for c, t in out_tensors.items():
        rows = t["rows"]
        total += (rows + 7) // 8
        if "offsets" in t:
            total += 8 * (rows + 1) + t["chars_bytes"]
        else:
            total += rows * (4 if types[c] == 1 else 8)
    return total


ENC_PLAIN, ENC_PLAIN_DICT, ENC_DELTA, ENC_RLE_DICT = 0, 2, 5, 8


def decode_kernel(f, c, types):
    """The decode kernel that handles every data page of column c, or None
    when its pages mix encodings that different kernels decode."""
    if types[c] == 6:
        return "k_decode_str"  # k_decode_str<true> (slot dictionaries) or <false>
    m = f.column_encodings(c)
    wide = 2 if types[c] != 1 else 0
    if m == 1 << ENC_DELTA:
        return "k_decode_delta"
    if m == 1 << ENC_PLAIN:
        return f"k_decode_fixed<{wide}>"
    if m and not (m & ~((1 << ENC_PLAIN_DICT) | (1 << ENC_RLE_DICT))):
        return f"k_decode_fixed<{wide + 1}>"
    return None


def algorithmic_bytes(kernel, f, cols, types, out_tensors, rows):
    """Bytes one launch of `kernel` must move: the encoded data-page bytes of
    the columns it decodes (levels and values) plus the decoded bytes it
    writes (values or offsets + chars, and the validity bitmap).  Dictionary
    gathers are served by the caches and not counted.  None when the kernel
    has no such figure (or a column's pages are split between kernels)."""
    b, any_col = 0, False
    for c in cols:
        k = decode_kernel(f, c, types)
        if k is None and types[c] != 6:
            return None
        if k != kernel and not (k == "k_decode_str" and kernel.startswith("k_decode_str<")):
            continue
        any_col = True
        data, _ = f.column_bytes(c)
        t = out_tensors[c]
        if "offsets" in t:
            b += data + 8 * (rows + 1) + t["chars_bytes"] + (rows + 7) // 8
        else:
            b += data + rows * (4 if types[c] == 1 else 8) + (rows + 7) // 8
    return b if any_col else None


def host_cpu():
    """Model name and core counts of the host the benchmark runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def oracle_seconds(data, columns=None, reps=1):
    """The oracle (single-threaded C) decoding `columns` of a file held in
    host memory, pinned to one host core (the second of this process's
    allowed cores): per rep the sum of the per-column decode calls, the
    median over reps.  Returns (seconds, decoded bytes, core)."""
    import oracle
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[2] if len(allowed) > 2 else allowed[0]
    os.sched_setaffinity(0, {core})
    try:
        f = oracle.File(data)
        cols = list(range(f.num_columns)) if columns is None else columns
        times, nbytes = [], 0
        for _ in range(reps):
            tot, nbytes = 0.0, 0
            for c in cols:
                dt, nb = f.decode_seconds(c)
                tot += dt
                nbytes += nb
            times.append(tot)
        f.close()
    finally:
        os.sched_setaffinity(0, set(allowed))
    times.sort()
    return times[len(times) // 2], nbytes, core


def pyarrow_seconds(data, reps=3):
    """pyarrow.parquet.read_table over the whole file on all host cores
    (third-party context, not the oracle): median seconds."""
    import io
    import pyarrow.parquet as papq
    raw = bytes(data)
    v = []
    for _ in range(reps):
        t0 = time.perf_counter()
        papq.read_table(io.BytesIO(raw), use_threads=True)
        v.append(time.perf_counter() - t0)
    v.sort()
    return v[len(v) // 2]


def cpu_baseline(data, nbytes_label):
    """The oracle (single-threaded) over every column of the benchmark file
    itself, in host memory, pinned to one host core; only the decode calls
    are timed."""
    dt, tot, core = oracle_seconds(data)
    cpu = host_cpu()
    return {"value": round(tot / dt / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"the benchmark file itself ({nbytes_label}), all columns, {tot / 1e9:.2f} GB decoded "
                      f"in {dt:.1f} s on host core {core}",
            "cpu_model": cpu["model"], "nproc": cpu["nproc"], "cores_allowed": cpu["affinity"]}


def read_traffic(key):
    """Measured HBM bytes per launch recorded by a rocprofv3 counter run
    (profiles/traffic.txt: `key source_hash fetch_bytes write_bytes` per
    line); None unless the kernel sources still hash the same."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    h = kernel_source_hash()
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 4 and parts[0] == key and parts[1] == h:
                return int(parts[2]) + int(parts[3])
    return None


def bench_batch(nfiles, reps, log):
    """The many-files workload (Zipf row counts, 8 OPTIONAL columns, mixed
    page sizes, Snappy on half the files) scanned three ways, every column of
    every file, into the same output buffers: one batched scan (one persistent
    decode launch; default and autotuned schedule), the per-page form (one
    launch per page and decoder), and one pq_scan per file (one launch per
    decoder per file).  Each time is the median over `reps` runs between HIP
    events on one stream, inputs resident in HBM."""
    import torch
    import datagen as dg
    import paper_2602_17335_amd as pqs
    t0 = time.perf_counter()
    specs = dg.batch_specs(nfiles)
    total_rows = sum(sp.num_rows for sp in specs)
    datas = [dg.write(sp, nthreads=min(16, os.cpu_count() or 1)) for sp in specs]
    log(f"batch: generated {nfiles} files, {sum(d.size for d in datas) / 1e9:.2f} GB in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    files = []
    for d in datas:
        buf, n = pqs.to_device(d)
        files.append(pqs.DeviceFile(buf, n))
    torch.cuda.synchronize()
    open_s = time.perf_counter() - t0
    file_bytes = sum(d.size for d in datas)
    del datas
    pages = sum(f.stats().pages for f in files)
    tiles = sum(f.stats().tiles for f in files)
    log(f"batch: opened {nfiles} files ({pages} data pages, {tiles} tiles) in {open_s:.1f} s")
    b = pqs.Batch([(f, list(range(8)), 0, None) for f in files])
    dec = b.decoded_bytes
    stream = torch.cuda.current_stream()

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        v = []
        for _ in range(n):
            a = torch.cuda.Event(enable_timing=True)
            z = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            z.record(stream)
            torch.cuda.synchronize()
            v.append(a.elapsed_time(z))
        v.sort()
        return v[len(v) // 2]

    batched_ms = timed(lambda: b.scan(), reps)
    b.check()
    best, tuned_ms_at_tune, default_ms_at_tune = b.autotune(reps=3)
    tuned_ms = timed(lambda: b.scan(best), reps)
    b.check()
    pqs.batch_profile(True)
    b.scan(best)
    torch.cuda.synchronize()
    prof = pqs.batch_profile_read()
    pqs.batch_profile(False)
    pp = pqs.tuning_default()
    pp.form = pqs.FORM_PER_PAGE
    per_page_ms = timed(lambda: b.scan(pp), max(2, reps // 4))
    b.check()
    # one pq_scan per file, into the batch's own output buffers
    need = max(f.plan(mask, rb, re_).workspace_bytes for f, cols, rb, re_, mask in b.requests)
    ws = torch.empty(max(int(need), 256), dtype=torch.uint8, device="cuda")

    def per_file():
        for i, (f, cols, rb, re_, mask) in enumerate(b.requests):
            f.scan_into(mask, rb, re_, list(b._outs[i])[: len(cols)], ws)

    per_file_ms = timed(per_file, max(2, reps // 4))
    files[0].check(ws)
    gbps = lambda ms: round(dec / (ms / 1e3) / 1e9, 2)
    out = {
        "workload": f"{nfiles} files, Zipf(1.1) row counts 10,000..4,000,000 ({total_rows:,} rows), "
                    "8 OPTIONAL columns with 5% nulls (INT32 PLAIN, INT32 dictionary, INT64 DELTA, INT64 dictionary, "
                    "2 DOUBLE PLAIN, 2 string dictionary), pages 8 KiB..1 MiB, Snappy on half the files, 1M-row row groups",
        "file_bytes": file_bytes, "pages": pages, "tiles": tiles, "decoded_bytes": dec, "open_s": round(open_s, 2),
        "batched_ms": round(batched_ms, 3), "batched_gbps": gbps(batched_ms),
        "autotuned_ms": round(tuned_ms, 3), "autotuned_gbps": gbps(tuned_ms),
        "per_page_ms": round(per_page_ms, 3), "per_page_gbps": gbps(per_page_ms),
        "per_file_ms": round(per_file_ms, 3), "per_file_gbps": gbps(per_file_ms),
        "speedup_vs_per_page": round(per_page_ms / tuned_ms, 2), "speedup_vs_per_file": round(per_file_ms / tuned_ms, 2),
        "autotuner": {"default_ms": round(default_ms_at_tune, 3), "best_ms": round(tuned_ms_at_tune, 3),
                      "waves_per_cu": best.waves_per_cu, "queues": best.queues,
                      "tiles_per_unit": list(best.tiles_per_unit)},
        "kernels": {k: {"launches": n, "avg_ms": round(t / max(n, 1), 4)} for k, (n, t) in prof.items()},
    }
    log(f"batch: batched {batched_ms:.2f} ms (autotuned {tuned_ms:.2f}), per-page {per_page_ms:.2f} ms, "
        f"per-file {per_file_ms:.2f} ms for {dec / 1e9:.2f} GB decoded")
    for f in files:
        f.close()
    return out


def bench_serve(nfiles, max_bytes, budget_bytes, qps_list, seconds, log, seed=0x5EED0006):
    """The scan server under Poisson load: a catalog of resident files
    (encoded sizes log-uniform in [1 MB, max_bytes]; plain and Snappy wide
    tables and the 8-column recipe), requests of 1-8 random columns over a
    random contiguous row-group range of a random file, arriving as a Poisson
    process at each rate of `qps_list` for `seconds`.  Latency is the
    server's submit-to-completion time (completion = the stream callback after
    the batch that decoded the request); decoded GB/s = decoded bytes of the
    completed requests over the wall time of the run."""
    import queue
    import threading
    import numpy as np
    import torch
    import datagen as dg
    import paper_2602_17335_amd as pqs
    t0 = time.perf_counter()
    files, enc = [], 0
    for sp in dg.serve_catalog(nfiles, max_bytes=max_bytes):
        d = dg.write(sp, nthreads=min(16, os.cpu_count() or 1))
        enc += d.size
        buf, n = pqs.to_device(d)
        del d
        files.append(pqs.DeviceFile(buf, n))
    torch.cuda.synchronize()
    log(f"serve: {nfiles} files, {enc / 1e9:.2f} GB encoded, generated and opened in {time.perf_counter() - t0:.1f} s")
    meta = [(f.num_columns, f.num_row_groups) for f in files]
    srv = pqs.Server(files, budget_bytes, slots=4, max_batch=64)
    rng = np.random.default_rng(seed)
    points = []
    for qps in qps_list:
        n = max(1, int(rng.poisson(qps * seconds)))
        gaps = rng.exponential(1.0 / qps, n)
        reqs = []
        for _ in range(n):
            i = int(rng.integers(0, nfiles))
            nc, nrg = meta[i]
            cols = sorted(rng.choice(nc, size=int(rng.integers(1, min(8, nc) + 1)), replace=False).tolist())
            b = int(rng.integers(0, nrg))
            e = int(rng.integers(b + 1, nrg + 1))
            reqs.append((i, cols, b, e))
        ids = queue.Queue()
        lat, qms, dec, bad = [], [], [0], [0]

        def waiter():
            while True:
                rid = ids.get()
                if rid is None:
                    return
                sv = srv.wait(rid)
                lat.append(sv.latency_ms)
                qms.append(sv.queue_ms)
                dec[0] += sv.decoded_bytes
                bad[0] += sv.status != 0
                srv.release(rid)

        th = threading.Thread(target=waiter)
        th.start()
        start = time.perf_counter()
        at = start
        for g, r in zip(gaps, reqs):
            at += g
            while True:
                dt = at - time.perf_counter()
                if dt <= 0:
                    break
                time.sleep(min(dt, 0.0005))
            ids.put(srv.submit(*r))
        ids.put(None)
        th.join()
        wall = time.perf_counter() - start
        lat.sort()
        qms.sort()
        pct = lambda v, q: round(v[min(len(v) - 1, int(round(q * (len(v) - 1))))], 3)
        offered = n / (at - start) if at > start else 0.0
        pt = {"qps_offered": round(offered, 1), "requests": n, "failed": bad[0],
              "p50_ms": pct(lat, 0.5), "p99_ms": pct(lat, 0.99), "queue_p50_ms": pct(qms, 0.5),
              "queue_p99_ms": pct(qms, 0.99), "decoded_gbps": round(dec[0] / wall / 1e9, 2),
              "qps_served": round(n / wall, 1)}
        log(f"serve: {qps} QPS offered -> p50 {pt['p50_ms']} ms, p99 {pt['p99_ms']} ms, {pt['decoded_gbps']} GB/s decoded")
        points.append(pt)
    st = srv.stats()
    srv.close()
    for f in files:
        f.close()
    return {"workload": f"{nfiles} resident files, {enc / 1e9:.2f} GB encoded (sizes log-uniform 1 MB..{max_bytes / 1e6:.0f} MB; "
                        "wide tables plain and Snappy, 8-column recipe), Poisson arrivals, 1-8 random columns over a random "
                        "row-group range per request",
            "budget_bytes": budget_bytes, "slots": 4, "max_batch": 64, "seconds_per_point": seconds, "points": points,
            "batches": st["batches"], "shared_results": st["cache_hits"], "evictions": st["evictions"]}


def bench_presets(rows, reps, log):
    """The paper's file-configuration sequence (Sec. 3, Insights 1-4, its
    ablation of effective bandwidth) on the wide table with the file in HBM:
    for each cumulative step, the encoded file size, the compression ratio
    (decoded bytes / encoded bytes), the median GPU scan time of all 16
    columns, and the effective bandwidth (decoded bytes / scan time).  With
    storage instead of HBM the file would arrive at a link rate R; the
    'at_link' figures model an overlapped reader, decoded bytes /
    max(scan time, file bytes / R), for R of the paper's 1-4 SSDs (about 6.5
    GB/s each) and of a PCIe 5 x16 link (64 GB/s)."""
    import torch
    import datagen as dg
    import paper_2602_17335_amd as pqs
    out = []
    for name in dg.PRESETS:
        spec = dg.preset(name, rows)
        data = dg.write(spec, nthreads=min(16, os.cpu_count() or 1))
        buf, n = pqs.to_device(data)
        del data
        f = pqs.DeviceFile(buf, n)
        st = f.stats()
        mask, rg_end, ws, outs, tens = f.allocate(list(range(16)))
        dec = decoded_bytes(tens, {c: f.column_info(c).type for c in range(16)})
        v = []
        for i in range(reps + 1):
            a = torch.cuda.Event(enable_timing=True)
            z = torch.cuda.Event(enable_timing=True)
            a.record()
            f.scan_into(mask, 0, rg_end, outs, ws)
            z.record()
            torch.cuda.synchronize()
            if i:
                v.append(a.elapsed_time(z))
        f.check(ws)
        v.sort()
        ms = v[len(v) // 2]
        encs = sorted({e for c in range(16) for e in range(32) if (f.column_encodings(c) >> e) & 1})
        row = {"preset": name, "file_bytes": n, "decoded_bytes": dec, "ratio": round(dec / n, 3),
               "pages": st.pages, "row_groups": f.num_row_groups, "compressed_pages": st.compressed_pages,
               "encodings": encs, "scan_ms": round(ms, 3), "effective_gbps": round(dec / ms / 1e6, 1),
               "at_link_gbps": {str(r): round(dec / max(ms / 1e3, n / (r * 1e9)) / 1e9, 1)
                                for r in (6.5, 13.0, 26.0, 64.0)}}
        log(f"preset {name:16s} {n / 1e9:6.3f} GB file, ratio {row['ratio']:5.2f}, scan {ms:7.2f} ms, "
            f"{row['effective_gbps']:7.1f} GB/s effective")
        out.append(row)
        del ws, outs, tens
        f.close()
        del buf
        torch.cuda.empty_cache()
    return {"workload": f"wide16 table, {rows:,} rows, 16 OPTIONAL columns with 10% nulls, all columns scanned",
            "steps": out}


def bench_streamed(rows, rg_rows, reps, log):
    """Sec. 4.1's overlapped reader with pinned host memory as the source:
    the wide table in row groups of `rg_rows` is scanned (all 16 columns)
    three ways -- device-resident (decode alone), a plain host-to-device
    copy of the whole file (the link alone), and pq_scan_streamed, which
    copies row group g+1 while row group g decodes.  The streamed rate
    includes the PCIe transfer; it is reported beside the headline figure,
    never as it.  `overlap` = max(copy, decode) / streamed (1.0: the slower
    of the two hides the other completely)."""
    import torch
    import datagen as dg
    import paper_2602_17335_amd as pqs
    data = dg.write(dg.wide_table(rows, rg_rows, 1 << 20), nthreads=min(16, os.cpu_count() or 1))
    hf = pqs.HostFile(data)
    buf, n = pqs.to_device(data)
    del data
    df = pqs.DeviceFile(buf, n)
    cols = list(range(df.num_columns))
    types = {c: df.column_info(c).type for c in cols}

    def med(fn):
        v = []
        for i in range(reps + 1):
            a = torch.cuda.Event(enable_timing=True)
            z = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            z.record()
            torch.cuda.synchronize()
            if i:
                v.append(a.elapsed_time(z))
        v.sort()
        return v[len(v) // 2]

    mask, rg_end, ws, outs, tens = df.allocate(cols)
    dec = decoded_bytes(tens, types)
    t_dec = med(lambda: df.scan_into(mask, 0, rg_end, outs, ws))
    df.check(ws)
    dst = torch.empty(n, dtype=torch.uint8, device="cuda")
    src = hf._buf[:n]
    t_copy = med(lambda: dst.copy_(src, non_blocking=True))
    del dst
    mask2, _, ws2, outs2, tens2 = hf.allocate(cols)
    t_str = med(lambda: hf.scan_into(mask2, 0, rg_end, outs2, ws2))
    hf.check(ws2)
    same = all(torch.equal(tens[c][k], tens2[c][k]) for c in cols
               for k in ("values_buf", "offsets", "validity_buf") if k in tens[c])
    row = {"workload": f"wide16 table, {rows:,} rows in row groups of {rg_rows:,}, 1 MiB pages, uncompressed, "
                       "pinned host memory, all 16 columns",
           "file_bytes": n, "row_groups": df.num_row_groups, "decoded_bytes": dec,
           "staging_bytes": int(hf.plan(mask2, 0, rg_end).workspace_bytes) - int(df.plan(mask, 0, rg_end).workspace_bytes),
           "decode_only_ms": round(t_dec, 3), "copy_only_ms": round(t_copy, 3),
           "link_gbps": round(n / t_copy / 1e6, 2), "streamed_ms": round(t_str, 3),
           "streamed_decoded_gbps": round(dec / t_str / 1e6, 2), "streamed_file_gbps": round(n / t_str / 1e6, 2),
           "overlap": round(max(t_copy, t_dec) / t_str, 3), "outputs_equal_device_scan": bool(same)}
    log(f"streamed: file {n / 1e9:.3f} GB in {row['row_groups']} row groups; decode alone {t_dec:.2f} ms, "
        f"copy alone {t_copy:.2f} ms ({row['link_gbps']} GB/s), streamed {t_str:.2f} ms "
        f"({row['streamed_decoded_gbps']} GB/s decoded, overlap {row['overlap']})")
    del ws, outs, tens, ws2, outs2, tens2
    df.close()
    hf.close()
    del buf
    torch.cuda.empty_cache()
    return row


def bench_configs(path, reps, log, with_oracle=True):
    """One JSON line per configuration (written to `path`): the 2-column
    table at 1,000,000 rows; the 16-column table over the row-group x
    page-size sweep (1M / 8M / 64M-row row groups x 64 KiB / 1 MiB / 8 MiB
    pages); the Snappy table (64M-row row group, 1 MiB pages, 1 MiB
    dictionary cap) for the projections P1 = {c15}, P4 = {c0, c6, c10,
    c13} and P16 = all columns.  Per configuration: open time, the warm
    and cold (L2 and MALL evicted by a 512 MiB write before each scan)
    median scan times over `reps` scans, the open-inclusive cold figure
    (open + first scan), decoded GB/s, algorithmic bytes (encoded read +
    decoded written; for Snappy also the staged form, decompression and
    decode each reading and writing its own bytes) as a fraction of 8 TB/s
    and of the library's plain copy of the same byte count, decompression
    and decode time apart (per-kernel events), the oracle on one pinned
    host core and pyarrow on all host cores (context)."""
    import io
    import json
    import torch
    import pyarrow.parquet as papq
    import datagen as dg
    import paper_2602_17335_amd as pqs
    nth = min(16, os.cpu_count() or 1)
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    cpu = host_cpu()

    def timed(fn, n, cold):
        v = []
        for _ in range(n):
            if cold:
                flush.fill_(1)
            a = torch.cuda.Event(enable_timing=True)
            z = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            z.record()
            torch.cuda.synchronize()
            v.append(a.elapsed_time(z))
        v.sort()
        return v[len(v) // 2]

    def copy_gbps(nbytes):
        nbytes = max(16, nbytes // 16 * 16)
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        pqs.copy_probe(dst, src, nbytes)
        ms = timed(lambda: pqs.copy_probe(dst, src, nbytes), 5, False)
        del src, dst
        return 2 * nbytes / ms / 1e6

    out = open(path, "w")

    def run(name, spec, projections, workload):
        t0 = time.perf_counter()
        data = dg.write(spec, nthreads=nth)
        md = papq.ParquetFile(io.BytesIO(bytes(data))).metadata
        buf, n = pqs.to_device(data)
        torch.cuda.synchronize()
        log(f"config {name}: {n / 1e9:.3f} GB file generated in {time.perf_counter() - t0:.1f} s")
        flush.fill_(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = pqs.DeviceFile(buf, n)
        torch.cuda.synchronize()
        open_ms = (time.perf_counter() - t0) * 1e3
        st = f.stats()
        types = {c: f.column_info(c).type for c in range(f.num_columns)}
        pya_s = pyarrow_seconds(data, 3)
        for pname, cols in projections:
            mask, rg_end, ws, outs, tens = f.allocate(cols)
            dec = decoded_bytes(tens, types)
            scan = lambda: f.scan_into(mask, 0, rg_end, outs, ws)
            first_ms = timed(scan, 1, False) if pname == projections[0][0] else None
            for _ in range(3):
                scan()
            f.check(ws)
            warm = timed(scan, reps, False)
            cold = timed(scan, reps, True)
            f.check(ws)
            f.profile(True)
            scan()
            torch.cuda.synchronize()
            prof = f.profile_read()
            f.profile(False)
            dec_ms = sum(t for k, (nl, t) in prof.items() if not k.startswith("k_snappy"))
            dcmp_ms = sum(t for k, (nl, t) in prof.items() if k.startswith("k_snappy"))
            comp = sum(sum(f.column_bytes(c)) for c in cols)
            unc = sum(md.row_group(g).column(c).total_uncompressed_size for g in range(md.num_row_groups) for c in cols)
            alg = comp + dec
            row = {"config": name, "projection": pname, "workload": workload, "columns": cols,
                   "file_bytes": n, "pages": st.pages, "dict_pages": st.dict_pages, "row_groups": f.num_row_groups,
                   "decoded_bytes": dec, "encoded_bytes": comp, "open_ms": round(open_ms, 2),
                   "warm_p50_ms": round(warm, 4), "cold_p50_ms": round(cold, 4), "reps": reps,
                   "decoded_gbps_warm": round(dec / warm / 1e6, 1), "decoded_gbps_cold": round(dec / cold / 1e6, 1),
                   "algorithmic_bytes": alg, "algorithmic_gbps": round(alg / warm / 1e6, 1),
                   "frac_of_8tbs": round(alg / warm / 1e6 / HBM_PEAK_GBS, 4)}
            cg = copy_gbps(alg // 2)
            row["copy_gbps_same_bytes"] = round(cg, 1)
            row["pct_of_copy"] = round(100 * (alg / warm / 1e6) / cg, 1)
            if first_ms is not None:
                row["open_inclusive_cold_ms"] = round(open_ms + first_ms, 2)
                row["open_inclusive_gbps"] = round(dec / (open_ms + first_ms) / 1e6, 2)
            if dcmp_ms > 0:
                row.update({"uncompressed_bytes": unc, "decompress_ms": round(dcmp_ms, 3),
                            "decode_ms": round(dec_ms, 3),
                            "staged_algorithmic_bytes": (comp + unc) + (unc + dec),
                            "decompress_gbps": round((comp + unc) / dcmp_ms / 1e6, 1),
                            "decode_gbps": round((unc + dec) / dec_ms / 1e6, 1)})
            if with_oracle:
                osec, ob, core = oracle_seconds(data, cols)
                row["oracle"] = {"seconds": round(osec, 3), "gbps": round(ob / osec / 1e9, 4), "core": core,
                                 "cpu_model": cpu["model"], "nproc": cpu["nproc"]}
            row["pyarrow_all_cores_s"] = round(pya_s, 3)
            log(f"config {name} {pname}: warm {warm:.3f} ms, cold {cold:.3f} ms, {row['decoded_gbps_warm']} GB/s "
                f"decoded, {row['pct_of_copy']}% of copy" + (f", oracle {row['oracle']['gbps']} GB/s" if with_oracle else ""))
            out.write(json.dumps(row) + "\n")
            out.flush()
            del ws, outs, tens
        f.close()
        del buf, data
        torch.cuda.empty_cache()

    run("C0", dg.small_table(), [("all", [0, 1])],
        "2 REQUIRED columns, 1,000,000 rows, 1 row group, 1 MiB pages, uncompressed")
    for rg in (1_000_000, 8_000_000, 64_000_000):
        for page in (64 * 1024, 1 << 20, 8 << 20):
            run(f"C1 rg{rg // 1_000_000}M page{page // 1024}KiB", dg.wide_table(64_000_000, rg, page),
                [("P16", list(range(16)))],
                f"wide16, 64,000,000 rows, row groups of {rg:,}, {page // 1024} KiB pages, uncompressed")
    run("C2", dg.snappy_wide_table(64_000_000, 64_000_000, 1 << 20),
        [("P1", [15]), ("P4", [0, 6, 10, 13]), ("P16", list(range(16)))],
        "wide16, 64,000,000 rows, one row group, 1 MiB pages, Snappy, 1 MiB dictionary cap")
    out.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rows", type=int, default=64_000_000)
    ap.add_argument("--rg-rows", type=int, default=64_000_000)
    ap.add_argument("--page-bytes", type=int, default=1 << 20)
    ap.add_argument("--codec", choices=["none", "snappy"], default="none")
    ap.add_argument("--columns", default="all", help="comma-separated column indices, or 'all'")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--batch-files", type=int, default=4096,
                    help="files of the many-files workload (batched vs plain forms); 0 skips it")
    ap.add_argument("--serve-files", type=int, default=64,
                    help="files of the serving catalog (0 skips the serving run; 256 with --serve-max-mb 2000 "
                         "is the full catalog)")
    ap.add_argument("--serve-max-mb", type=int, default=256, help="largest catalog file, MB")
    ap.add_argument("--serve-budget-gb", type=int, default=64, help="device-memory budget of the server, GB")
    ap.add_argument("--serve-qps", default="200,1000,4000", help="offered request rates")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--preset-rows", type=int, default=16_000_000,
                    help="rows of the file-configuration sequence (0 skips it)")
    ap.add_argument("--stream-rows", type=int, default=64_000_000,
                    help="rows of the streamed-from-host-memory run (0 skips it)")
    ap.add_argument("--stream-rg-rows", type=int, default=4_000_000, help="row-group rows of the streamed run")
    ap.add_argument("--configs-report", default=None,
                    help="write one JSON line per configuration (sweep, Snappy projections, C0) to this path "
                         "and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: this scanner is built and measured on one GPU "
              "(each GPU would scan its own shard of the files or row groups independently)", file=sys.stderr)
        sys.exit(2)

    import torch
    import datagen as dg
    import paper_2602_17335_amd as pqs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.configs_report:
        bench_configs(args.configs_report, args.steps, log, not args.no_cpu_baseline)
        return
    if args.codec == "snappy":
        def spec_fn(rows, rg):
            return dg.snappy_wide_table(rows, rg, args.page_bytes)
    else:
        def spec_fn(rows, rg):
            return dg.wide_table(rows, rg, args.page_bytes)
    spec = spec_fn(args.rows, args.rg_rows)
    t0 = time.perf_counter()
    data = dg.write(spec, nthreads=min(16, os.cpu_count() or 1))
    log(f"generated {len(data) / 1e9:.3f} GB file in {time.perf_counter() - t0:.1f} s")
    buf, nbytes = pqs.to_device(data)
    if args.no_cpu_baseline:
        del data
    torch.cuda.synchronize()

    if args.copy_probe:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        bcopy = torch.empty_like(a)
        bcopy.copy_(a)
        torch.cuda.synchronize()
        del a, bcopy
        log("copy probe: 1 GiB device-to-device copy done")

    t0 = time.perf_counter()
    f = pqs.DeviceFile(buf, nbytes)
    torch.cuda.synchronize()
    open_ms = (time.perf_counter() - t0) * 1e3
    st = f.stats()
    log(f"opened: {st.pages} data pages, {st.dict_pages} dictionary pages, {st.tiles} tiles, "
        f"open {open_ms:.1f} ms wall ({st.open_ms_device:.1f} ms device)")
    ncols = f.num_columns
    cols = list(range(ncols)) if args.columns == "all" else [int(x) for x in args.columns.split(",")]
    types = {c: f.column_info(c).type for c in range(ncols)}
    mask, rg_end, ws, outs, tens = f.allocate(cols)
    rows = next(iter(tens.values()))["rows"]
    dec = decoded_bytes(tens, types)
    stream = torch.cuda.current_stream()

    # the first scan after the open, timed alone (the open-inclusive figure)
    e_a = torch.cuda.Event(enable_timing=True)
    e_b = torch.cuda.Event(enable_timing=True)
    e_a.record(stream)
    f.scan_into(mask, 0, rg_end, outs, ws)
    e_b.record(stream)
    torch.cuda.synchronize()
    first_ms = e_a.elapsed_time(e_b)
    for _ in range(args.warmup):
        f.scan_into(mask, 0, rg_end, outs, ws)
    f.check(ws)
    log(f"warmup done ({args.warmup} scans; the first scan after the open took {first_ms:.3f} ms)")

    f.profile(True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        f.scan_into(mask, 0, rg_end, outs, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    f.check(ws)
    prof = f.profile_read()
    f.profile(False)
    ms = total_ms / args.steps
    value = dec / (ms / 1e3) / 1e9
    log(f"{args.steps} scans: {ms:.3f} ms/scan, {value:.1f} GB/s decoded")
    kern = {k: {"launches": n, "avg_ms": round(t / n, 4), "share": round(t / total_ms, 3)} for k, (n, t) in prof.items()}
    for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["avg_ms"]):
        log(f"  {k:16s} {v['avg_ms']:8.3f} ms/launch  {v['share'] * 100:5.1f}% of the timed region")

    # per-scan latency: each scan between its own events, warm (back to back)
    # and cold (L2 and the 256 MB MALL evicted by a 512 MiB write first)
    def timed_scans(n, flush):
        out = []
        scratch = torch.empty(512 << 20, dtype=torch.uint8, device="cuda") if flush else None
        for _ in range(n):
            if flush:
                scratch.fill_(1)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            f.scan_into(mask, 0, rg_end, outs, ws)
            b.record(stream)
            torch.cuda.synchronize()
            out.append(a.elapsed_time(b))
        f.check(ws)
        return sorted(out)
    warm = timed_scans(args.steps, False)
    cold = timed_scans(max(3, args.steps // 4), True)
    def pct(v, q):
        return round(v[min(len(v) - 1, int(round(q * (len(v) - 1))))], 4)
    latency = {"scans": len(warm), "p50_ms": pct(warm, 0.5), "p99_ms": pct(warm, 0.99),
               "evicted_scans": len(cold), "evicted_p50_ms": pct(cold, 0.5), "evicted_p99_ms": pct(cold, 0.99),
               "evicted_gbps": round(dec / (pct(cold, 0.5) / 1e3) / 1e9, 2),
               "open_inclusive_ms": round(open_ms + first_ms, 2),
               "open_inclusive_gbps": round(dec / ((open_ms + first_ms) / 1e3) / 1e9, 2)}
    log(f"latency: warm p50 {latency['p50_ms']} ms, p99 {latency['p99_ms']} ms; "
        f"L2/MALL evicted before each scan p50 {latency['evicted_p50_ms']} ms = {latency['evicted_gbps']} GB/s; "
        f"open + first scan {latency['open_inclusive_ms']} ms = {latency['open_inclusive_gbps']} GB/s")
    # the practical ceiling: the library's plain copy of the scan's
    # algorithmic bytes (encoded read + decoded written), moved as a copy
    enc = sum(sum(f.column_bytes(c)) for c in cols)
    half = (enc + dec) // 32 * 16
    csrc = torch.empty(half, dtype=torch.uint8, device="cuda")
    cdst = torch.empty(half, dtype=torch.uint8, device="cuda")
    pqs.copy_probe(cdst, csrc, half)
    cv = []
    for _ in range(5):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        pqs.copy_probe(cdst, csrc, half)
        b.record(stream)
        torch.cuda.synchronize()
        cv.append(a.elapsed_time(b))
    del csrc, cdst
    cv.sort()
    copy_gbps = 2 * half / cv[2] / 1e6
    scan_alg_gbps = (enc + dec) / ms / 1e6
    copy_ref = {"bytes_moved": 2 * half, "ms": round(cv[2], 4), "gbps": round(copy_gbps, 1),
                "scan_algorithmic_gbps": round(scan_alg_gbps, 1), "pct_of_copy": round(100 * scan_alg_gbps / copy_gbps, 1)}
    log(f"copy of the same {2 * half / 1e9:.2f} GB: {copy_gbps:.0f} GB/s; the scan moves its algorithmic bytes at "
        f"{scan_alg_gbps:.0f} GB/s = {copy_ref['pct_of_copy']}% of copy")

    key = f"rows={args.rows}:rg={args.rg_rows}:page={args.page_bytes}:codec={args.codec}:cols={args.columns}"
    per = {}
    n_str = sum(1 for k in prof if k.startswith("k_decode_str"))
    for k, (n_l, t_l) in prof.items():
        if k.startswith("k_decode_str") and n_str > 1:
            continue  # string tiles split between the two instantiations: no per-launch figure
        alg = algorithmic_bytes(k, f, cols, types, tens, rows)
        if alg is None or n_l == 0:
            continue
        ach = alg / (t_l / n_l / 1e3) / 1e9
        per[k] = {"achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4), "avg_ms": round(t_l / n_l, 4),
                  "algorithmic_bytes_per_launch": alg, "traffic": read_traffic(f"{k}:{key}")}
    roof = None
    if per:
        dom = max(per, key=lambda k: prof[k][1])
        d = per[dom]
        roof = {"bound": "hbm", "achieved": d["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": d["frac"],
                "traffic": d["traffic"], "kernel": dom, "algorithmic_bytes_per_launch": d["algorithmic_bytes_per_launch"],
                "traffic_key": f"{dom}:{key}", "decode_kernels": per}
        for k, v in per.items():
            log(f"  roofline {k:18s} {v['achieved']:8.1f} GB/s = {v['frac'] * 100:5.1f}% of HBM peak")

    batch = None
    if args.batch_files > 0:
        del ws, outs, tens
        f.close()
        del buf
        torch.cuda.empty_cache()
        batch = bench_batch(args.batch_files, max(5, args.steps // 2), log)

    presets = None
    if args.preset_rows > 0:
        presets = bench_presets(args.preset_rows, 5, log)

    streamed = None
    if args.stream_rows > 0:
        streamed = bench_streamed(args.stream_rows, args.stream_rg_rows, 5, log)

    serve = None
    if args.serve_files > 0:
        serve = bench_serve(args.serve_files, args.serve_max_mb * 1_000_000, args.serve_budget_gb << 30,
                            [float(x) for x in args.serve_qps.split(",")], args.serve_seconds, log)

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU baseline: oracle over the same file ...")
        cpu = cpu_baseline(data, f"{nbytes / 1e9:.2f} GB, {args.rows:,} rows")
        log(f"CPU baseline: {cpu['value']} GB/s")

    workload = (f"wide16: {args.rows:,} rows, row groups of {args.rg_rows:,}, {args.page_bytes // 1024} KiB pages, "
                f"{'Snappy' if args.codec == 'snappy' else 'uncompressed'}, 16 OPTIONAL columns with 10% nulls "
                f"(6 INT32, 4 INT64, 3 DOUBLE, 3 BYTE_ARRAY; PLAIN / dictionary / DELTA)")
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": workload, "rows": rows, "row_group_rows": args.rg_rows, "page_bytes": args.page_bytes,
                   "codec": args.codec, "columns": len(cols), "file_bytes": nbytes, "decoded_bytes_per_step": dec,
                   "pages": st.pages, "dict_pages": st.dict_pages, "tiles": st.tiles,
                   "open_ms": round(open_ms, 2), "open_ms_device": round(st.open_ms_device, 2),
                   "form": "plain (one launch per kernel kind per scan)", "kernels": kern,
                   "latency": latency, "copy_reference": copy_ref},
        "roofline": roof,
        "batched_vs_plain": batch,
        "serving": serve,
        "streamed_from_host": streamed,
        "file_configurations": presets,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
