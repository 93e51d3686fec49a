"""GPU parity of batched scans (pq_scan_batch): many files of uneven size
(a scaled-down copy of the many-files workload: Zipf row counts, mixed page
sizes, Snappy on half the files, 8 OPTIONAL columns of every decoder kind)
decoded together, in the persistent one-launch form under several
schedules and in the one-launch-per-page form, every output buffer compared
with the CPU oracle byte for byte (buffers pre-filled with 0xAB, guard
regions checked)."""
import pytest

import datagen as dg
import oracle
from tests.gpu_util import GUARD, POISON, compare_column

pytestmark = pytest.mark.gpu


def _files(n=40, seed=0x5EED0103):
    specs = dg.batch_specs(n, max_rows=120_000, min_rows=1_500, rg_rows=40_000, page_kib=(8, 16, 32, 64, 128),
                           seed=seed)
    return [dg.write(s) for s in specs]


def _open(datas):
    import paper_2602_17335_amd as pqs
    out = []
    for d in datas:
        buf, n = pqs.to_device(d)
        out.append(pqs.DeviceFile(buf, n))
    return out


def _check_batch(b, datas, label):
    ofs = {}
    for i, (f, cols, rb, re_, mask) in enumerate(b.requests):
        j = next(k for k, h in enumerate(b._files) if h is f)
        of = ofs.setdefault(j, oracle.File(datas[j]))
        for c in cols:
            compare_column(of.read(c, rb, re_), b.outputs[i][c], f"{label} req{i} file{j} col{c} rg[{rb},{re_})")


def _batch(files, reqs):
    import paper_2602_17335_amd as pqs
    b = pqs.Batch(reqs, poison=POISON, guard=GUARD)
    b._files = files
    return b


def test_batch_all_files_all_columns():
    import paper_2602_17335_amd as pqs
    datas = _files()
    files = _open(datas)
    reqs = [(f, list(range(8)), 0, None) for f in files]
    print(f"[gpu] batch: {len(files)} files, default schedule", flush=True)
    b = _batch(files, reqs)
    b.scan()
    b.check()
    _check_batch(b, datas, "batched")
    # one shared queue, other waves per CU and units of 1 and 16 tiles
    t = pqs.tuning_default()
    t.queues, t.waves_per_cu = 1, 4
    for k in range(pqs.TUNE_CLASSES):
        t.tiles_per_unit[k] = 1 if k % 2 else 16
    print("[gpu] batch: one queue, mixed unit sizes", flush=True)
    b2 = _batch(files, reqs)
    b2.scan(t)
    b2.check()
    _check_batch(b2, datas, "batched-q1")
    print("[gpu] batch: per-page launches", flush=True)
    t.form = pqs.FORM_PER_PAGE
    b3 = _batch(files, reqs)
    b3.scan(t)
    b3.check()
    _check_batch(b3, datas, "per-page")


def test_batch_subranges_projections_shared_files():
    """Requests with row-group sub-ranges and projections, several on one
    file, empty ranges among them."""
    datas = _files(12, seed=0x5EED0104)
    files = _open(datas)
    reqs = []
    for i, f in enumerate(files):
        nrg = f.num_row_groups
        reqs.append((f, [0, 3, 6], 0, nrg))
        reqs.append((f, [1, 2, 7], min(1, nrg), nrg))
        reqs.append((f, [4, 5], nrg // 2, nrg // 2))
    print(f"[gpu] batch: {len(reqs)} requests over {len(files)} files", flush=True)
    b = _batch(files, reqs)
    b.scan()
    b.check()
    _check_batch(b, datas, "subranges")


def test_autotuned_schedule_is_exact():
    """The autotuner's schedule decodes the same bytes (and its timings are
    positive)."""
    datas = _files(24, seed=0x5EED0105)
    files = _open(datas)
    reqs = [(f, list(range(8)), 0, None) for f in files]
    b = _batch(files, reqs)
    print("[gpu] autotune", flush=True)
    best, best_ms, default_ms = b.autotune(reps=2)
    assert best_ms > 0 and default_ms > 0 and best_ms <= default_ms * 1.0001
    b2 = _batch(files, reqs)
    b2.scan(best)
    b2.check()
    _check_batch(b2, datas, "autotuned")
