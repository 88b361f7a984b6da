"""Host-side logic that needs no GPU: autotuner signature and cache,
bench's one-GPU contract, option validation in the binding."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


class FakeCtx:
    def __init__(self, n, nl, ns, fp64=False):
        self.nx = self.ny = self.nz = n
        self.nl, self.ns, self.fp64 = nl, ns, fp64


def test_autotune_signature_and_cache(tmp_path, monkeypatch):
    from paper_1203_2941_amd import autotune
    a = [FakeCtx(64, 40, 3), FakeCtx(128, 100, 3)]
    b = [FakeCtx(64, 40, 3), FakeCtx(128, 100, 3)]
    c = [FakeCtx(64, 41, 3), FakeCtx(128, 100, 3)]
    assert autotune.signature(a, "bw_ticket") == autotune.signature(b, "bw_ticket")
    assert autotune.signature(a, "bw_ticket") != autotune.signature(c, "bw_ticket")
    assert autotune.signature(a, "bw_ticket") != autotune.signature(a, "frozen")
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "t.json"))
    key = autotune.signature(a, "bw_ticket")
    hit = {"queue_depth": 1 << 20, "walk_blocks_per_cu": 4, "blocks_per_cu": 2,
           "packets_per_s": 1.0, "rates": {}, "sample_packets": 1}
    (tmp_path / "t.json").write_text(json.dumps({key: hit}))
    # a cached entry is returned without touching the GPU
    assert autotune.tune(a, [1, 1], [0, 1], mode="bw_ticket") == hit


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_run_opts_modes():
    from paper_1203_2941_amd import context, _lib
    o = context.run_opts(mode="bw_epoch", epoch_packets=7, record=True)
    assert o.mode == _lib.BW_EPOCH and o.epoch_packets == 7 and o.record == 1
    with pytest.raises(KeyError):
        context.run_opts(mode="nonsense")


def test_traffic_summary_round_trip(tmp_path):
    """Counter summary for the walk's HBM traffic: each counter is scaled by
    its reading of a copy of known size; the two runs may differ in launch
    count; bench reads back per-launch and per-step bytes."""
    import sqlite3
    from paper_1203_2941_amd import profiling as pf

    def db(path, counter, calib, walk):
        con = sqlite3.connect(path)
        con.execute("create table counters_collection (dispatch_id int, kernel_name text, "
                    "counter_name text, value real)")
        rows = [(0, "vectorized_elementwise_kernel<MulFunctor>", counter, calib)]
        rows += [(i + 1, f"void mcrt::{pf.TRANSPORT_KERNEL}(args)", counter, v)
                 for i, v in enumerate(walk)]
        con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
        con.commit()
        con.close()

    mib = 4
    nbytes = mib << 20
    db(tmp_path / "f.db", "FETCH_SIZE", nbytes / 2048.0, [100.0, 300.0])       # 2048 B per unit
    db(tmp_path / "w.db", "WRITE_SIZE", nbytes / 1024.0, [10.0, 20.0, 30.0])   # 1024 B per unit
    text = pf.traffic_md(str(tmp_path / "f.db"), str(tmp_path / "w.db"), mib, "cmd")
    out = tmp_path / "t.md"
    out.write_text(text)
    got = pf.read_traffic(str(out))
    per_launch = 200.0 * 2048 + 20.0 * 1024
    assert abs(got["per_launch"] - per_launch) / per_launch < 1e-5
    assert abs(got["per_step"] - per_launch * 2.5) / (per_launch * 2.5) < 1e-5
    # a summary taken from other transport sources is not reported
    out.write_text(text.replace(pf.source_digest(), "0" * 64))
    assert pf.read_traffic(str(out)) is None
