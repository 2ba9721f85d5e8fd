"""Host logic of bench.py on the CPU: the saturated-rate slope, the guard
on the committed traffic counters, the serving driver (latencies and the
queueing delay from the server's queue length, by Little's law) against
a scripted stand-in server, and the one-GPU contract."""
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_saturated_rate_is_the_middle_slope():
    # 100 equal requests finishing every 10 ms after a 1 s start-up and
    # with a slow tail: the 10 %-70 % slope is 100 units/s
    done = [(1.0 + 0.01 * i, 1.0) for i in range(90)] + [(5.0 + i, 1.0) for i in range(10)]
    assert abs(bench.saturated_rate(done) - 100.0) < 1e-9


def test_traffic_counters_only_for_their_kernel_and_tiling(tmp_path, monkeypatch):
    import hashlib
    import workloads as W
    sha = hashlib.sha256(open(bench.KERNEL_SRC, "rb").read()).hexdigest()
    prof = tmp_path / "counters.txt"
    prof.write_text("# scaled counters\n"
                    f"kernel_source_sha256: {sha}\ncells_per_lane: 16\nblock_steps: 48\n"
                    "fetch_bytes_per_update: 0.4\nwrite_bytes_per_update: 0.2\n")
    monkeypatch.setitem(bench.COUNTERS, W.F32, str(prof))
    v = bench.measured_traffic_per_update(16, 48)
    assert v is not None and abs(v - 0.6) < 1e-12
    assert bench.measured_traffic_per_update(16, 56) is None
    assert bench.measured_traffic_per_update(12, 48) is None
    other = tmp_path / "kernels.hip"
    other.write_text("// not the profiled source\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(other))
    assert bench.measured_traffic_per_update(16, 48) is None


def test_counters_list_takes_the_matching_tiling(tmp_path, monkeypatch):
    """A precision may have counters at several tilings; the lookup takes
    the file taken at the run's tiling."""
    import hashlib
    import workloads as W
    sha = hashlib.sha256(open(bench.KERNEL_SRC, "rb").read()).hexdigest()
    files = []
    for C, f in ((16, 1.0), (12, 2.0)):
        prof = tmp_path / f"c{C}.txt"
        prof.write_text(f"kernel_source_sha256: {sha}\ncells_per_lane: {C}\nblock_steps: 48\n"
                        f"fetch_bytes_per_update: {f}\nwrite_bytes_per_update: 0.5\n")
        files.append(str(prof))
    monkeypatch.setitem(bench.COUNTERS, W.F64, files)
    assert bench.measured_traffic_per_update(16, 48, W.F64) == 1.5
    assert bench.measured_traffic_per_update(12, 48, W.F64) == 2.5
    assert bench.measured_traffic_per_update(8, 48, W.F64) is None


def test_roofline_of_launches_on_two_streams(monkeypatch):
    """With the runs split over two streams, each stream is busy for the
    whole stepping phase: a launch lasts 2 x step time / launches, and the
    achieved rate is the flops of all launches over the phase."""
    import workloads as W
    monkeypatch.setattr(bench, "measured_traffic_per_update", lambda C, T, p=W.F32: 0.5)
    st = {"step_ms": 1000.0, "launches": 400, "streams": 2, "cells_per_lane": 16,
          "block_steps": 48, "tile_waves": 1, "graph": 0}
    updates = 2.0e12
    r = bench.kernel_roofline(st, updates, W.F32)
    assert r["concurrent_streams"] == 2
    assert abs(r["avg_launch_ms"] - 5.0) < 1e-12
    assert abs(r["achieved"] - updates * bench.FLOPS_PER_UPDATE / 1e12) < 1e-3
    # traffic per launch at 0.5 B an update, both streams' launches over 1 s
    assert abs(r["traffic"] - 0.5 * updates / 400) < 1e-6
    assert abs(r["measured_hbm_GBs"] - 0.5 * updates / 1e9) < 0.1
    one = bench.kernel_roofline(dict(st, streams=1), updates, W.F32)
    assert abs(one["avg_launch_ms"] - 2.5) < 1e-12 and one["achieved"] == r["achieved"]


class _FakeServer:
    """One request in service at a time, each needing `work` progress
    calls; the rest wait in the queue."""

    def __init__(self, work, **kw):
        self.work = work
        self.queue, self.live, self.left, self.done = [], None, 0, set()
        self.next_id = 1

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False

    def submit(self, prob):
        rid = self.next_id
        self.next_id += 1
        self.queue.append(rid)
        return rid

    def progress(self, max_blocks=1):
        if self.live is None and self.queue:
            self.live, self.left = self.queue.pop(0), self.work
        if self.live is not None:
            self.left -= 1
            if self.left == 0:
                self.done.add(self.live)
                self.live = None
        return (0 if self.live is None else 1), len(self.queue)

    def ready(self, rid):
        return rid in self.done

    def poll(self, rid):
        self.done.discard(rid)
        return {"status": 0}


def test_2d_roofline_and_its_counters(tmp_path, monkeypatch):
    """The 2D kernel's roofline: algorithmic 6 words per cell-update over
    the average launch; measured traffic only from counters taken on the
    same kernel source and tiling."""
    import hashlib
    import workloads as W
    sha = hashlib.sha256(open(bench.KERNEL2D_SRC, "rb").read()).hexdigest()
    prof = tmp_path / "c2d.txt"
    prof.write_text(f"kernel_source_sha256: {sha}\ncells_per_lane: 4\ncolumns_per_wave: 8\n"
                    "fetch_bytes_per_update: 14.5\nwrite_bytes_per_update: 12.0\n")
    monkeypatch.setitem(bench.COUNTERS_2D, (W.TE, W.F32), str(prof))
    st = {"launches": 100, "step_ms": 10.0, "cell_updates": 100 * 2.0e7,
          "cells_per_lane": 4, "columns_per_wave": 8, "waves": 1000, "block_steps": 1}
    r = bench.kernel_roofline_2d(st, W.TE, W.F32)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["achieved"] - 2.0e7 * 24 / 1e-4 / 1e9) < 0.1      # 4800 GB/s
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-4
    assert abs(r["traffic"] - 26.5 * 2.0e7) < 1.0
    st["columns_per_wave"] = 16
    assert bench.kernel_roofline_2d(st, W.TE, W.F32)["traffic"] is None
    assert bench.kernel_roofline_2d(st, W.TM, W.F32)["traffic"] is None
    other = tmp_path / "kernels2d.hip"
    other.write_text("// not the profiled source\n")
    monkeypatch.setattr(bench, "KERNEL2D_SRC", str(other))
    st["columns_per_wave"] = 8
    assert bench.kernel_roofline_2d(st, W.TE, W.F32)["traffic"] is None
    # two steps a launch: each launch still moves 6 words a cell, 3 per
    # cell-update; the single-step equivalent doubles
    st.update(block_steps=2, cell_updates=100 * 4.0e7)
    r2 = bench.kernel_roofline_2d(st, W.TE, W.F32)
    assert abs(r2["achieved"] - r["achieved"]) < 0.1 and r2["bytes_per_update"] == 12
    assert abs(r2["single_step_hbm_equiv_GBs"] - 2 * r["achieved"]) < 0.2
    assert r2["traffic"] is None                       # counters were taken at T = 1


def test_serving_driver_counts_latency_and_queueing(monkeypatch):
    clock = {"t": 0.0}
    monkeypatch.setattr(bench.time, "perf_counter", lambda: clock["t"])
    monkeypatch.setattr(bench.time, "sleep", lambda s: None)
    fake = _FakeServer(work=3)

    def Server(**kw):
        return fake

    # each progress call takes 1 s of the fake clock
    orig = fake.progress

    def progress(max_blocks=1):
        clock["t"] += 1.0
        return orig(max_blocks)

    fake.progress = progress
    P = types.SimpleNamespace(Server=Server, GfdtdError=RuntimeError)
    prob = types.SimpleNamespace(nz=10, steps=5)
    stream = [(0.0, prob)] * 4            # four requests at t = 0
    res = bench.serve(P, stream, 1 << 20, 8, closed=True)
    assert res["rejected"] == 0 and len(res["latency_s"]) == 4
    assert res["updates"] == 4 * 50
    # served one after another, 3 s each: done at 3, 6, 9, 12 s
    assert sorted(res["latency_s"]) == [3.0, 6.0, 9.0, 12.0]
    # waits for admission: 0, 3, 6, 9 s (the queue, as sampled after each
    # progress call, holds 3, 2, 1 requests for 3 s each) -> mean 4.5 s
    assert abs(res["queue_wait_mean_s"] - 4.5) < 1e-9
    # time averages of the sampled live and queued counts
    assert 0.0 < res["live_mean"] <= 1.0 and 0.0 < res["queue_mean"] <= 3.0


def test_alone_latency_driver(monkeypatch):
    clock = {"t": 0.0}
    monkeypatch.setattr(bench.time, "perf_counter", lambda: clock["t"])
    fake = _FakeServer(work=2)
    orig = fake.progress

    def progress(max_blocks=1):
        clock["t"] += 0.5
        return orig(max_blocks)

    fake.progress = progress
    P = types.SimpleNamespace(Server=lambda **kw: fake)
    prob = types.SimpleNamespace(nz=10, steps=5)
    assert bench.alone_latencies(P, [prob, prob], 1 << 20, 8) == [1.0, 1.0]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
