"""Host logic of bench.py (no GPU): the request stream of the serving run, the FIFO replay of
the FP64 baseline, the sweeps' byte-count ratio and the validity check of the stored counter
traffic."""
import hashlib
import json
import os
import shutil

import numpy as np

import bench


def test_fifo_timeline_by_hand():
    # a request waits for the one before it; an idle server starts at the arrival
    done = bench.fifo_timeline([0.0, 1.0, 10.0, 10.5], [3.0, 2.0, 1.0, 4.0])
    np.testing.assert_allclose(done, [3.0, 5.0, 11.0, 15.0])


def test_serve_requests_seeded_and_in_range():
    a = bench.serve_requests(40)
    b = bench.serve_requests(40)
    assert len(a) == 40
    times = [r[0] for r in a]
    assert all(t1 > t0 for t0, t1 in zip(times, times[1:]))
    for (t, op, src), (t2, op2, src2) in zip(a, b):
        assert t == t2 and op == op2 and np.array_equal(src, src2)
        assert 0 <= op < len(bench.SERVE_FREQS)
        assert 1 <= len(src) <= 128
        assert len({tuple(x) for x in src}) == len(src)  # distinct grid points
        assert np.all(src[:, 2] == 0.5)
    # the first 40 requests of the stream hold 726 sources (the serving profile's figure)
    assert sum(len(r[2]) for r in a) == 726


def test_plain_count_ratio_by_hand():
    # one level: 10 stored factor entries, 3 pivots, fronts of 5 rows in all, s = 2, e = 8
    lv = [{"factor_useful": 10, "sum_pivots": 3, "sum_front": 5}]
    r = bench._plain_count_ratio(lv, 2, 8.0)
    plain = 8.0 * (10 + 2.0 * 3 * 2)
    assert abs(r["oras_fwd"] - plain / (8.0 * (10 + 2.0 * 5 * 2))) < 1e-15
    assert abs(r["oras_bwd"] - plain / (8.0 * (10 + (5 + 3) * 2))) < 1e-15


def test_counter_traffic_voided_when_source_changes(tmp_path, monkeypatch):
    """The stored HBM traffic of a kernel class is reported only while the source file it was
    measured on is unchanged."""
    src_rel = "paper_2004_07930_amd/csrc/spmm.hip"
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_2004_07930_amd" / "csrc").mkdir(parents=True)
    shutil.copy(os.path.join(bench.ROOT, src_rel), tmp_path / src_rel)
    sha = hashlib.sha256(open(tmp_path / src_rel, "rb").read()).hexdigest()
    rec = {"spmm": {"traffic_bytes_per_launch": 2.5e9, "source": src_rel, "source_sha256": sha}}
    (tmp_path / "profiles" / "traffic_w.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("spmm", "w") == 2.5
    assert bench.counter_traffic("oras_fwd", "w") is None
    assert bench.counter_traffic("spmm", "other") is None
    with open(tmp_path / src_rel, "a") as f:
        f.write("\n// edited\n")
    assert bench.counter_traffic("spmm", "w") is None

