"""The scan server (pq_server_*): requests of 1-8 random columns over random
row-group ranges of a catalog of resident files (plain and Snappy wide
tables, the many-files recipe) give byte-identical results when each runs
alone and when all run in a mix (submitted together, batched continuously,
overlapping on several streams, sharing identical results), under a roomy
budget and under one small enough to force waiting for memory and
evictions; every result also equals the CPU oracle's."""
import numpy as np
import pytest

import datagen as dg
import oracle
from tests.gpu_util import compare_column

pytestmark = pytest.mark.gpu


def _catalog():
    specs = [
        dg.wide_table(200_003, 50_000, 64 * dg.KiB, seed=0x5EED0201),
        dg.snappy_wide_table(150_001, 40_000, 32 * dg.KiB, seed=0x5EED0202),
        dg.wide_table(90_000, 90_000, 256 * dg.KiB, seed=0x5EED0203),
    ]
    specs += dg.batch_specs(3, max_rows=160_000, min_rows=20_000, rg_rows=30_000, page_kib=(8, 32, 128),
                            seed=0x5EED0204)
    specs[1].dict_cap = 64 * dg.KiB
    return [dg.write(s) for s in specs]


def _requests(files, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        i = int(rng.integers(0, len(files)))
        f = files[i]
        nc = f.num_columns
        cols = sorted(rng.choice(nc, size=int(rng.integers(1, min(8, nc) + 1)), replace=False).tolist())
        nrg = f.num_row_groups
        b = int(rng.integers(0, nrg))
        e = int(rng.integers(b + 1, nrg + 1))
        out.append((i, cols, b, e))
    return out


def _run(server, reqs, together):
    res = []
    if together:
        ids = [server.submit(*r) for r in reqs]
        for rid in ids:
            sv = server.wait(rid)
            assert sv.status == 0
            res.append((server.fetch(rid, sv), sv.shared))
            server.release(rid)
    else:
        for r in reqs:
            rid = server.submit(*r)
            sv = server.wait(rid)
            assert sv.status == 0
            res.append((server.fetch(rid, sv), sv.shared))
            server.release(rid)
    return res


def _same(a, b, label):
    for c in a:
        for k in a[c]:
            if isinstance(a[c][k], np.ndarray):
                assert a[c][k].dtype == b[c][k].dtype and (a[c][k].view(np.uint8) == b[c][k].view(np.uint8)).all(), \
                    (label, c, k)


@pytest.mark.parametrize("budget_mb,slots", [(1024, 4), (48, 2)])
def test_alone_equals_mix(budget_mb, slots):
    import paper_2602_17335_amd as pqs
    datas = _catalog()
    files = []
    for d in datas:
        buf, n = pqs.to_device(d)
        files.append(pqs.DeviceFile(buf, n))
    reqs = _requests(files, 60, seed=0x5EED0205 + budget_mb)
    reqs += reqs[:10]  # identical requests: shared while in flight or resident
    print(f"[gpu] serve: {len(reqs)} requests, budget {budget_mb} MB, {slots} slots", flush=True)
    # alone: one request in flight at a time, on a server of its own
    srv = pqs.Server(files, budget_mb << 20, slots=slots, max_batch=16)
    alone = _run(srv, reqs, together=False)
    srv.close()
    print("[gpu] serve: alone done", flush=True)
    # the mix: every request submitted at once to a fresh server
    srv = pqs.Server(files, budget_mb << 20, slots=slots, max_batch=16)
    mixed = _run(srv, reqs, together=True)
    st = srv.stats()
    print(f"[gpu] serve: mix done {st}", flush=True)
    assert st["failed"] == 0 and st["completed"] == len(reqs)
    assert st["batches"] >= 2
    if budget_mb < 100:
        assert st["evictions"] > 0
    for k, ((ra, _), (rm, _)) in enumerate(zip(alone, mixed)):
        _same(ra, rm, f"request {k} {reqs[k]}")
    ofs = {}
    for k, (i, cols, b, e) in enumerate(reqs[:60]):
        of = ofs.setdefault(i, oracle.File(datas[i]))
        for c in cols:
            g = dict(alone[k][0][c])
            g["validity_words"] = g["validity_words"]
            compare_column(of.read(c, b, e), g, f"serve req{k} file{i} col{c} rg[{b},{e})")
    srv.close()
