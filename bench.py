"""Benchmark: batched generalized-FDTD solves on one MI355X.

A "step" is one pass of the whole hot path over one batch: every run of the
batched moving-bilayer-crystal workload (4096 runs, grid lengths
log-uniform in [4096, 65536], 4 nz time steps each) stepped from zero
fields to its last step, source, ends, probes and probe DFTs included.
Inputs (rest profiles, probes, frequencies) are resident in HBM before the
timed region.  `value` is total cell-updates (sum over runs of nz * steps)
per second of the timed passes.

Printed beside it, in the same JSON line:
  roofline     -- the stepping kernel (k_tiles) of the timed pass against
                  the chip's vector-ALU peak, timed with HIP events on the
                  library's stream;
  batched_f64  -- the same batch in FP64, with its kernel roofline;
  serving      -- the continuous-batching server on the serving mix (grid
                  lengths log-uniform in [1e3, 1e6], 2 GiB pool): saturated
                  rate, and at each offered load the throughput, p50/p99
                  latency, mean queueing delay, rejections and (at the
                  lowest load) each request's slowdown against its alone
                  time;
  plain        -- the plain single-run form of the interface (2000 cells x
                  4000 steps), slab (65536 x 131072) and moving-matter
                  gradient (2^20 x 2^18) workloads, FP32 and FP64: rate,
                  kernel roofline, error against the FP64 oracle (the
                  gradient on its 2^14 x 2^12 downscaled copy, and FP32
                  against FP64 at full size) and the oracle's own rate on
                  the host;
  tmm_sweep    -- the batched transfer-matrix evaluator: call and kernel
                  time;
  twod         -- the 2D TE / TM path on a moving slab (4096 x 4096 cells,
                  x periodic, 4096 steps at S = 0.25), FP32 and FP64: rate,
                  the step kernel (k_step2d) against the HBM peak at its
                  algorithmic 6 words per cell-update, FP32 against FP64 at
                  full size, and the 2D oracle's error and host rate on a
                  64-column copy of 1024 steps;
  error        -- the FP32 batch's probe spectra against the oracle on a
                  sample of its runs at their full step counts;
  cpu_baseline -- the oracle on the host cores on that sample.
"""
import argparse
import json
import math
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = ("cell-updates/sec batched-served vs plain at fixed error; "
          "p50/p99 solve latency")

# Algorithmic arithmetic of one cell-update: eq. (10a)-(10d) with the
# Table 1 terms as printed, one flop per add, subtract, multiply, divide:
# (10a) 6, (10d) 5, (10b) 6, (10c) 5 for a moving modulation.
FLOPS_PER_UPDATE = 22
# Algorithmic HBM bytes of one cell-update: read and write D and B once.
BYTES_PER_UPDATE = {W.F32: 16, W.F64: 32}
# MI355X vector-ALU peaks: FP64 256 CUs x 64 lanes x 2 flops (FMA) x 2.4 GHz
# = 78.6 TFLOP/s; FP32 twice that, 157.3 TFLOP/s (two VALU instructions
# can issue per SIMD and cycle slot: the FP32 stepping kernel measures 1.2
# VALU wave-instructions per 4 cycles per SIMD without packed FP32 math).
ALU_PEAK_TFLOPS = {W.F32: 256 * 64 * 2 * 2.4e9 * 2 / 1e12,
                   W.F64: 256 * 64 * 2 * 2.4e9 / 1e12}
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Counter summaries per precision, one per tiling the autotuner picks on the
# crystal batch (FP64 lands on 12 or 16 cells per lane, about 2 % apart).
COUNTERS = {
    W.F32: [os.path.join(ROOT, "profiles", "k_tiles_f32_crystals4096_hbm_counters.txt")],
    W.F64: [os.path.join(ROOT, "profiles", "k_tiles_f64_crystals4096_hbm_counters.txt"),
            os.path.join(ROOT, "profiles", "k_tiles_f64_c12_crystals4096_hbm_counters.txt")],
}
KERNEL_SRC = os.path.join(ROOT, "paper_2304_06586_amd", "csrc", "kernels.hip")
KERNEL2D_SRC = os.path.join(ROOT, "paper_2304_06586_amd", "csrc", "kernels2d.hip")
COUNTERS_2D = {
    (W.TE, W.F32): os.path.join(ROOT, "profiles", "k_step2d_f32_te_slab4096_hbm_counters.txt"),
    (W.TE, W.F64): os.path.join(ROOT, "profiles", "k_step2d_f64_te_slab4096_hbm_counters.txt"),
    (W.TM, W.F32): os.path.join(ROOT, "profiles", "k_step2d_f32_tm_slab4096_hbm_counters.txt"),
    (W.TM, W.F64): os.path.join(ROOT, "profiles", "k_step2d_f64_tm_slab4096_hbm_counters.txt"),
}
# Algorithmic HBM bytes of one 2D cell-update: read and write D, B and C once.
BYTES_PER_UPDATE_2D = {W.F32: 24, W.F64: 48}


def measured_traffic_per_update(C, T, precision=W.F32):
    """HBM bytes per cell-update of k_tiles from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE counters (scaled by a plain copy), or None when
    the kernel source has changed since they were taken or they were taken
    at another tiling (cells per lane C, steps per launch T)."""
    import hashlib
    paths = COUNTERS[precision]
    if isinstance(paths, str):
        paths = [paths]
    try:
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    for path in paths:
        try:
            kv = {}
            for line in open(path):
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
            if kv.get("kernel_source_sha256") != sha:
                continue
            if int(kv["cells_per_lane"]) != C or int(kv["block_steps"]) != T:
                continue
            return float(kv["fetch_bytes_per_update"]) + float(kv["write_bytes_per_update"])
        except (OSError, KeyError, ValueError):
            continue
    return None


def measured_traffic_2d(pol, precision, C, xch, T=1):
    """HBM bytes per cell-update of k_step2d from committed rocprofv3
    FETCH_SIZE/WRITE_SIZE counters (copy-calibrated), or None when there
    are none for this polarization and precision, the kernel source has
    changed since, or they were taken at another tiling."""
    import hashlib
    path = COUNTERS_2D.get((pol, precision))
    if path is None:
        return None
    try:
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        sha = hashlib.sha256(open(KERNEL2D_SRC, "rb").read()).hexdigest()
        if kv.get("kernel_source_sha256") != sha:
            return None
        if (int(kv["cells_per_lane"]) != C or int(kv["columns_per_wave"]) != xch
                or int(kv.get("block_steps", 1)) != T):
            return None
        return float(kv["fetch_bytes_per_update"]) + float(kv["write_bytes_per_update"])
    except (OSError, KeyError, ValueError):
        return None


def kernel_roofline_2d(st, pol, precision):
    """k_step2d of the last pass against the HBM peak.  A launch of T steps
    reads and writes D, B and C of every cell once: algorithmic bytes per
    launch are 6 words a cell (24 B FP32, 48 B FP64), i.e. 6/T words per
    cell-update, over the average launch time from the library's HIP
    events around the pass's stepping launches.  The single-step figure
    (6 words per cell-update, what the same rate would need without
    temporal blocking) is given beside it."""
    launches = max(1, int(st["launches"]))
    avg_launch_ms = st["step_ms"] / launches
    upd_per_launch = st["cell_updates"] / launches
    T = max(1, int(st.get("block_steps", 1)))
    alg = upd_per_launch * BYTES_PER_UPDATE_2D[precision] / T
    achieved = alg / (avg_launch_ms * 1e-3) / 1e9 if avg_launch_ms > 0 else 0.0
    per_update = measured_traffic_2d(pol, precision, int(st["cells_per_lane"]),
                                     int(st["columns_per_wave"]), T)
    traffic = per_update * upd_per_launch if per_update is not None else None
    return {
        "kernel": "k_step2d",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                        "copy-calibrated)",
        "algorithmic_bytes_per_launch": alg,
        "bytes_per_update": BYTES_PER_UPDATE_2D[precision] / T,
        "single_step_hbm_equiv_GBs": (round(alg * T / (avg_launch_ms * 1e-3) / 1e9, 1)
                                      if avg_launch_ms > 0 else 0.0),
        "block_steps": T,
        "kernel_cell_updates_per_s": (st["cell_updates"] / (st["step_ms"] * 1e-3)
                                      if st["step_ms"] > 0 else 0.0),
        "launches_per_pass": launches,
        "avg_launch_ms": round(avg_launch_ms, 4),
        "cells_per_lane": int(st["cells_per_lane"]),
        "columns_per_wave": int(st["columns_per_wave"]),
        "waves_per_launch": int(st["waves"]),
    }


def twod_leg(P, args):
    """The 2D path on the moving-slab workload, both polarizations and
    precisions: one untimed pass, then a timed pass (inputs resident)."""
    import torch
    out = {}
    full = {}
    cases = set(args.twod_cases.split(","))
    for pol, pname in ((W.TE, "te"), (W.TM, "tm")):
        for prec, dname in ((W.F32, "f32"), (W.F64, "f64")):
            if f"{pname}_{dname}" not in cases:
                continue
            p = W.slab_run_2d(args.seed, pol=pol, precision=prec)
            if args.twod_steps:
                p = p.replace(steps=args.twod_steps)
            with P.Run2D(p, fields=False) as r:
                r.run()
                r.collect()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r.run()
                res = r.collect()
                dt = time.perf_counter() - t0
                st = r.stats()
            full[(pname, dname)] = res
            out[f"{pname}_{dname}"] = {
                "value": p.cell_updates / dt, "unit": "cell-updates/s",
                "ms": dt * 1e3, "nx": p.nx, "nz": p.nz, "steps": p.steps,
                "beta": p.beta, "status": res["status"],
                "roofline": kernel_roofline_2d(st, pol, prec)}
            log(f"2d {pname}_{dname}: {p.cell_updates / dt:.4g} cell-updates/s, "
                f"{dt * 1e3:.1f} ms, k_step2d {out[f'{pname}_{dname}']['roofline']['achieved']}"
                f" GB/s (C={st['cells_per_lane']}, {st['columns_per_wave']} columns/wave, "
                f"T={st['block_steps']})")
    for pname in ("te", "tm"):
        if (pname, "f64") not in full or (pname, "f32") not in full:
            continue
        a, b = full[(pname, "f64")], full[(pname, "f32")]
        out[f"{pname}_f32"]["error_vs_gpu_f64"] = {
            "trace_rel_l2": rel(b["trace"], a["trace"]),
            "dft_rel_l2": rel(b["dft"], a["dft"])}
    if not args.no_cpu and not args.twod_steps:
        from oracle import stepper2d
        for pol, pname in ((W.TE, "te"), (W.TM, "tm")):
            if f"{pname}_f32" not in out or f"{pname}_f64" not in out:
                continue
            q = W.slab_run_2d(args.seed, pol=pol, precision=W.F64, nx=64, steps=1024)
            t0 = time.perf_counter()
            ref = stepper2d.solve(q, fields=False)
            odt = time.perf_counter() - t0
            for prec, dname in ((W.F32, "f32"), (W.F64, "f64")):
                g = P.gfdtd2d_solve(q.replace(precision=prec), fields=False)
                out[f"{pname}_{dname}"]["error_vs_oracle_downscaled"] = {
                    "trace_rel_l2": rel(g["trace"], ref["trace"]),
                    "dft_rel_l2": rel(g["dft"], ref["dft"])}
            out[f"{pname}_f64"]["oracle"] = {
                "value": q.cell_updates / odt, "unit": "cell-updates/s", "cores": 1,
                "seconds": round(odt, 2),
                "sample": "the same workload on 64 columns for 1024 steps"}
    return out


def kernel_roofline(st, updates, precision):
    """k_tiles of the last pass against the vector-ALU peak, from the
    library's HIP events around the pass's stepping launches.  When the
    batch splits its runs over two streams, launches of the two halves run
    concurrently: each stream is busy for the whole stepping phase, so a
    launch lasts streams x step time / launches on average, and `achieved`
    is the flops of all launches over the phase (the two streams' launches
    summed)."""
    step_s = st["step_ms"] / 1e3
    launches = max(1, int(st["launches"]))
    streams = max(1, int(st.get("streams", 1)))
    avg_launch_ms = st["step_ms"] * streams / launches
    k_rate = updates / step_s if step_s > 0 else 0.0
    achieved = k_rate * FLOPS_PER_UPDATE / 1e12
    per_update = measured_traffic_per_update(int(st["cells_per_lane"]),
                                             int(st["block_steps"]), precision)
    upd_per_launch = updates / launches
    traffic = per_update * upd_per_launch if per_update is not None else None
    hbm_equiv = k_rate * BYTES_PER_UPDATE[precision] / 1e9
    return {
        "kernel": "k_tiles",
        "bound": "alu",
        "achieved": round(achieved, 3),
        "peak": round(ALU_PEAK_TFLOPS[precision], 1),
        "unit": "TFLOP/s",
        "frac": round(achieved / ALU_PEAK_TFLOPS[precision], 4),
        "traffic": traffic,
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                        "copy-calibrated)",
        "measured_hbm_GBs": (round(streams * traffic / (avg_launch_ms * 1e-3) / 1e9, 1)
                             if traffic is not None and avg_launch_ms > 0 else None),
        "algorithmic_bytes_per_launch": upd_per_launch * BYTES_PER_UPDATE[precision],
        "flops_per_update": FLOPS_PER_UPDATE,
        "kernel_cell_updates_per_s": k_rate,
        "launches_per_pass": launches,
        "concurrent_streams": streams,
        "avg_launch_ms": round(avg_launch_ms, 4),
        "cells_per_lane": int(st["cells_per_lane"]),
        "block_steps": int(st["block_steps"]),
        "tile_waves": int(st["tile_waves"]),
        "graph": int(st["graph"]),
        "single_step_hbm_equiv_GBs": round(hbm_equiv, 1),
        "single_step_hbm_frac": round(hbm_equiv / HBM_PEAK_GBS, 3),
    }


def gpu_pass_rate(P, problems, passes, warmup, tune=True, collect=False,
                  record_trace=False, **exec_kw):
    """Seconds for `passes` passes of a batch (after autotuning and
    warm-up, both outside the timed region), its stats, and its results
    when `collect`."""
    import torch
    with P.Batch(problems, record_trace=record_trace, fields=False, **exec_kw) as b:
        if tune:
            b.autotune(trial_blocks=4)
        for _ in range(warmup):
            b.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(passes):
            b.run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = b.stats()
        out = b.collect() if collect else None
    return dt, st, out


def rel(a, b):
    den = np.linalg.norm(np.ravel(b))
    num = np.linalg.norm(np.ravel(a) - np.ravel(b))
    return float(num / den) if den > 0 else float(num)


# ------------------------------------------------------------------ serving

def serve(P, stream, pool_bytes, max_slots, blocks_per_call=64, closed=False):
    """Drive the continuous-batching server with a request stream of
    (arrival time, problem).  closed=True submits everything at t = 0.
    Returns a dict: the seconds from the first arrival to the last
    completion, each request's latency in stream order (s, None if
    rejected), total cell-updates, the (completion time, cell-updates) of
    every request, rejections, and the mean time a request waits for
    admission: by Little's law the time integral of the server's queue
    length divided by the requests that entered it."""
    n = len(stream)
    lat = [None] * n
    done = []
    updates = 0
    rejected = 0
    queue_area = 0.0
    live_area = 0.0
    last_q, last_live, last_t = 0, 0, 0.0
    accepted = 0
    finished = 0
    with P.Server(pool_bytes=pool_bytes, max_slots=max_slots) as srv:
        pending = {}
        i = 0
        t0 = time.perf_counter()
        while finished + rejected < n:
            now = time.perf_counter() - t0
            while i < n and (closed or stream[i][0] <= now):
                prob = stream[i][1]
                try:
                    rid = srv.submit(prob)
                except P.GfdtdError:
                    rejected += 1
                    i += 1
                    continue
                pending[rid] = (i, 0.0 if closed else stream[i][0], prob.nz * prob.steps)
                updates += prob.nz * prob.steps
                accepted += 1
                i += 1
            if pending:
                now = time.perf_counter() - t0
                queue_area += last_q * (now - last_t)
                live_area += last_live * (now - last_t)
                last_live, last_q = srv.progress(max_blocks=blocks_per_call)
                last_t = now
                for rid in list(pending):
                    if srv.ready(rid):
                        now = time.perf_counter() - t0
                        r = srv.poll(rid)
                        assert r["status"] == 0
                        k, arr, work = pending.pop(rid)
                        lat[k] = now - arr
                        done.append((now, work))
                        finished += 1
            elif i < n:
                time.sleep(max(0.0, min(0.01, stream[i][0] - now)))
        total = time.perf_counter() - t0
    return {"total_s": total, "latency_s": lat, "updates": updates,
            "done": sorted(done), "rejected": rejected,
            "queue_wait_mean_s": queue_area / max(1, accepted),
            "live_mean": live_area / max(total, 1e-9),
            "queue_mean": queue_area / max(total, 1e-9)}


def alone_latencies(P, problems, pool_bytes, max_slots, blocks_per_call=64):
    """Latency of each request served alone, by the same server and loop."""
    out = []
    with P.Server(pool_bytes=pool_bytes, max_slots=max_slots) as srv:
        for p in problems:
            t0 = time.perf_counter()
            rid = srv.submit(p)
            while not srv.ready(rid):
                srv.progress(max_blocks=blocks_per_call)
            srv.poll(rid)
            out.append(time.perf_counter() - t0)
    return out


def saturated_rate(done, lo=0.1, hi=0.7):
    """Cell-updates/s of a saturated server: the slope of completed work
    against time between lo and hi of the total work (the start, while the
    pipeline fills, and the drain, while the last long requests finish
    alone, are left out)."""
    t = np.array([d[0] for d in done])
    w = np.cumsum([d[1] for d in done])
    W_ = w[-1]
    i0 = int(np.searchsorted(w, lo * W_))
    i1 = int(np.searchsorted(w, hi * W_))
    if i1 <= i0 or t[i1] <= t[i0]:
        return W_ / t[-1]
    return float((w[i1] - w[i0]) / (t[i1] - t[i0]))


def serving_leg(P, args):
    pool = int(args.serve_budget_gib * (1 << 30))
    slots = args.serve_slots
    sat_stream = W.serving_stream(args.seed, args.serve_sat_requests, 1.0,
                                  nz_hi=args.serve_nz_hi)
    sat = serve(P, sat_stream, pool, slots, closed=True)
    cap = saturated_rate(sat["done"])
    mean_work = sat["updates"] / len(sat_stream)
    cap_rps = cap / mean_work
    log(f"serving: saturated {cap:.4g} cell-updates/s ({cap_rps:.2f} req/s)")
    loads = []
    for li, frac in enumerate([float(x) for x in args.serve_loads.split(",") if x]):
        rate = frac * cap_rps
        n = max(args.serve_min_requests, int(round(rate * args.serve_seconds)))
        stream = W.serving_stream(args.seed + 1 + li, n, rate, nz_hi=args.serve_nz_hi)
        res = serve(P, stream, pool, slots)
        lat = np.array([x for x in res["latency_s"] if x is not None])
        entry = {
            "offered_fraction": frac,
            "offered_requests_per_s": round(rate, 3),
            "requests": n,
            "offered_seconds": round(stream[-1][0], 2),
            "cell_updates_per_s": res["updates"] / res["total_s"],
            "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
            "queue_wait_mean_ms": res["queue_wait_mean_s"] * 1e3,
            "queued_mean": round(res["queue_mean"], 2),
            "live_mean": round(res["live_mean"], 2),
            "rejected": res["rejected"],
        }
        if li == 0 and args.serve_alone:
            # each request of the lightest load served alone, same server
            idx = [k for k, x in enumerate(res["latency_s"]) if x is not None]
            alone = alone_latencies(P, [stream[k][1] for k in idx], pool, slots)
            slow = np.array([res["latency_s"][k] / a for k, a in zip(idx, alone)])
            entry["slowdown_vs_alone"] = {
                "p50": float(np.percentile(slow, 50)),
                "p99": float(np.percentile(slow, 99)),
                "max": float(np.max(slow)),
                "requests": len(slow),
                "note": "latency in the mix / latency of the same request served "
                        "alone by the same server",
            }
        loads.append(entry)
        log(f"serving at {frac:.2f} of capacity ({rate:.2f} req/s, {n} requests): "
            f"p50 {entry['p50_latency_ms']:.1f} ms p99 {entry['p99_latency_ms']:.1f} ms, "
            f"queueing {entry['queue_wait_mean_ms']:.1f} ms, live {entry['live_mean']}, "
            f"queued {entry['queued_mean']}"
            + (f", slowdown p99 {entry['slowdown_vs_alone']['p99']:.2f}"
               if "slowdown_vs_alone" in entry else ""))
    return {
        "saturated_cell_updates_per_s": cap,
        "saturated_requests_per_s": cap_rps,
        "saturated_note": "slope of completed work vs time between 10 % and "
                          "70 % of the total, all requests submitted at t = 0",
        "makespan_cell_updates_per_s": sat["updates"] / sat["total_s"],
        "saturated_requests": len(sat_stream),
        "loads": loads,
        "mix": f"interface/slab/crystal/gradient, nz log-uniform in "
               f"[1e3, {args.serve_nz_hi:.0e}], steps U[2,4] nz, "
               "FP32 or FP64 with p = 1/2, Poisson arrivals",
        "budget_GiB": args.serve_budget_gib,
        "max_slots": slots,
    }


# ----------------------------------------------------------- oracle (host)

class OracleJobs(threading.Thread):
    """The oracle on a list of (name, problem) in one host thread (the C
    stepper releases the interpreter lock), timing each run."""

    def __init__(self, jobs):
        super().__init__(daemon=True)
        self.jobs = jobs
        self.results = {}
        self.error = None

    def run(self):
        try:
            import oracle
            for name, p in self.jobs:
                t0 = time.perf_counter()
                out = oracle.solve(p, fields=False)
                dt = time.perf_counter() - t0
                self.results[name] = (out, dt, p.nz * p.steps)
        except Exception as e:          # reported in the line, not raised
            self.error = repr(e)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--runs", type=int, default=4096)
    ap.add_argument("--precision", choices=["f32", "f64"], default="f32")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cells-per-lane", type=int, default=0)
    ap.add_argument("--block-steps", type=int, default=0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample-updates", type=float, default=6e10,
                    help="cell-updates of the oracle sample of the batch (runs at "
                         "full length, in batch order, each at most 4e9)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default tiling instead of autotuning it")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-tmm", action="store_true")
    ap.add_argument("--no-2d", action="store_true")
    ap.add_argument("--twod-cases", default="te_f32,te_f64,tm_f32,tm_f64",
                    help="2D cases to run (polarization_precision, comma-separated)")
    ap.add_argument("--twod-steps", type=int, default=0, metavar="N",
                    help="run the 2D cases for N steps instead of 4096 (profiling)")
    ap.add_argument("--serve-loads", default="0.25,0.5,0.75,0.9,1.1",
                    help="offered loads as fractions of the saturated request "
                         "rate, comma separated (the first also gets alone times)")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="seconds of arrivals per offered load")
    ap.add_argument("--serve-min-requests", type=int, default=24)
    ap.add_argument("--serve-sat-requests", type=int, default=160)
    ap.add_argument("--serve-nz-hi", type=float, default=1e6)
    ap.add_argument("--serve-budget-gib", type=float, default=2.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--no-serve-alone", dest="serve_alone", action="store_false")
    ap.add_argument("--steps-cap", type=int, default=0, metavar="N",
                    help="cap every run at N steps: a shorter workload with the "
                         "same runs, tiles and launch shape, for counter "
                         "collection (the reported value then covers it)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times), "
                         "the reference for HBM byte counters")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "copies": 5}), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the "
              "batched workload shards by runs with no communication, so the "
              "per-GPU figure is the one reported.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2304_06586_amd as P
    assert torch.cuda.is_available(), "no GPU"
    P.load_library()
    prec = W.F32 if args.precision == "f32" else W.F64
    exec_kw = dict(cells_per_lane=args.cells_per_lane, block_steps=args.block_steps,
                   tune=not args.no_tune and not args.cells_per_lane
                   and not args.block_steps)

    # ---------------------------------------------------------------- batched
    log(f"generating {args.runs} crystal runs (seed {args.seed})")
    probs = W.crystal_runs(args.seed, count=args.runs, precision=prec)
    if args.steps_cap:
        probs = [q.replace(steps=min(q.steps, args.steps_cap)) for q in probs]
    updates = float(sum(p.nz * p.steps for p in probs))
    log(f"cell-updates per pass: {updates:.4g}")
    dt, st, batch_out = gpu_pass_rate(P, probs, args.steps, args.warmup,
                                      collect=not args.no_cpu, **exec_kw)
    value = updates * args.steps / dt
    ms_per_step = dt * 1e3 / args.steps
    log(f"batched: {value:.4g} cell-updates/s, {ms_per_step:.1f} ms per pass")
    roofline = kernel_roofline(st, updates, prec)

    # --------------------------------------------------- batched, other dtype
    batched_f64 = None
    if not args.no_f64 and prec == W.F32 and not args.steps_cap:
        probs64 = [q.replace(precision=W.F64) for q in probs]
        dt64, st64, _ = gpu_pass_rate(P, probs64, 1, 1, **exec_kw)
        batched_f64 = {"value": updates / dt64, "ms": dt64 * 1e3,
                       "roofline": kernel_roofline(st64, updates, W.F64),
                       "hbm_equiv_frac": round(updates / dt64 * 32 / 8e12, 3)}
        log(f"batched f64: {batched_f64['value']:.4g} cell-updates/s")
        del probs64

    # ---------------------------------- oracle of the plain configs, host thread
    plain_defs = [
        ("interface", lambda pr: W.interface_run(args.seed, precision=pr)),
        ("slab", lambda pr: W.slab_run(args.seed, precision=pr)),
        ("gradient", lambda pr: W.gradient_run(args.seed, precision=pr)),
    ]
    oracle_jobs = None
    if not args.no_plain and not args.no_cpu:
        oracle_jobs = OracleJobs([
            ("interface", W.interface_run(args.seed, precision=W.F64)),
            ("gradient_downscaled", W.gradient_run(args.seed, precision=W.F64,
                                                   downscaled=True)),
            ("slab", W.slab_run(args.seed, precision=W.F64)),
        ])
        oracle_jobs.start()         # overlaps the serving leg on one host core

    # ---------------------------------------------------------------- served
    serving = None
    if not args.no_serve:
        serving = serving_leg(P, args)

    # ------------------------------------------------------------------ plain
    plain = None
    if not args.no_plain:
        plain = {}
        gpu_out = {}
        for name, maker in plain_defs:
            for pname, pr in (("f32", W.F32), ("f64", W.F64)):
                p = maker(pr)
                pdt, pst, pout = gpu_pass_rate(P, [p], 1, 1, tune=not args.no_tune,
                                               collect=True, record_trace=True)
                gpu_out[(name, pname)] = pout[0]
                plain[f"{name}_{pname}"] = {
                    "value": p.nz * p.steps / pdt, "ms": pdt * 1e3,
                    "nz": p.nz, "steps": p.steps,
                    "roofline": kernel_roofline(pst, float(p.nz * p.steps), pr)}
                log(f"plain {name}_{pname}: {plain[f'{name}_{pname}']['value']:.4g} "
                    f"cell-updates/s, {pdt * 1e3:.2f} ms (C={pst['cells_per_lane']}, "
                    f"T={pst['block_steps']})")
        # the gradient's downscaled copy, against the oracle
        for pname, pr in (("f32", W.F32), ("f64", W.F64)):
            q = W.gradient_run(args.seed, precision=pr, downscaled=True)
            gpu_out[("gradient_downscaled", pname)] = P.gfdtd_solve(q, fields=False)
        # FP32 against FP64 at full gradient size (probe spectra and traces)
        g32, g64 = gpu_out[("gradient", "f32")], gpu_out[("gradient", "f64")]
        plain["gradient_f32"]["error_vs_gpu_f64"] = {
            "dft_rel_l2": rel(g32["dft"], g64["dft"]),
            "trace_rel_l2": rel(g32["trace"], g64["trace"])}
        if oracle_jobs is not None:
            oracle_jobs.join()
            if oracle_jobs.error:
                plain["oracle_error"] = oracle_jobs.error
            for oname, key in (("interface", "interface"), ("slab", "slab"),
                               ("gradient_downscaled", "gradient")):
                if oname not in oracle_jobs.results:
                    continue
                ref, odt, oupd = oracle_jobs.results[oname]
                for pname in ("f32", "f64"):
                    g = gpu_out[(oname, pname)]
                    err = {"trace_rel_l2": rel(g["trace"], ref["trace"]),
                           "dft_rel_l2": rel(g["dft"], ref["dft"])}
                    if oname == "gradient_downscaled":
                        plain[f"{key}_{pname}"]["error_vs_oracle_downscaled"] = err
                    else:
                        plain[f"{key}_{pname}"]["error_vs_oracle"] = err
                plain[f"{key}_f64"]["oracle"] = {
                    "value": oupd / odt, "unit": "cell-updates/s", "cores": 1,
                    "seconds": round(odt, 2),
                    "sample": ("full run" if oname != "gradient_downscaled" else
                               "the 2^14-cell, 2^12-step downscaled copy")}
            log("plain errors vs oracle: " + ", ".join(
                f"{k}: {v.get('error_vs_oracle', v.get('error_vs_oracle_downscaled', {})).get('trace_rel_l2', float('nan')):.2e}"
                for k, v in plain.items() if isinstance(v, dict) and "value" in v))

    # ------------------------------------------- transfer-matrix sweep (GPU)
    tmm = None
    if not args.no_tmm:
        stacks, omegas = W.tmm_crystals(args.seed, 4096, nomega=256)
        layers = sum(len(s.eps) for s in stacks)
        P.gfdtd_tmm(stacks[:8], omegas[:8])               # warm-up
        torch.cuda.synchronize()
        dt_call, dt_kernel = float("inf"), float("inf")
        for _ in range(3):                                 # best of three calls
            t0 = time.perf_counter()
            P.gfdtd_tmm(stacks, omegas)
            dt_call = min(dt_call, time.perf_counter() - t0)
            dt_kernel = min(dt_kernel, P.gfdtd_tmm_kernel_ms() / 1e3)
        evals = len(stacks) * len(omegas)
        tmm = {"stack_frequency_evals_per_s": evals / dt_call,
               "kernel_stack_frequency_evals_per_s": evals / dt_kernel,
               "layer_evals_per_s": layers * len(omegas) / dt_call,
               "kernel_layer_evals_per_s": layers * len(omegas) / dt_kernel,
               "call_ms": dt_call * 1e3, "kernel_ms": dt_kernel * 1e3,
               "stacks": len(stacks), "frequencies": len(omegas), "layers": layers,
               "note": "best of three synchronous gfdtd_tmm calls; call_ms includes "
                       "host packing, host-to-device upload and result copies, "
                       "kernel_ms is k_tmm alone (HIP events); FP64"}
        if not args.no_cpu:
            from oracle import analytic as A
            sub = stacks[:4]
            om = omegas[::32]
            c0 = time.perf_counter()
            for s in sub:
                for w in om:
                    A.transfer_matrix(w, list(s.eps), list(s.widths), s.beta)
            cdt = time.perf_counter() - c0
            tmm["cpu_oracle_stack_frequency_evals_per_s"] = len(sub) * len(om) / cdt
        log(f"transfer-matrix sweep: call {dt_call * 1e3:.2f} ms, kernel "
            f"{dt_kernel * 1e3:.3f} ms")

    # ------------------------------------------------------------- 2D path
    twod = None
    if not args.no_2d:
        twod = twod_leg(P, args)

    # ------------------- error and CPU baseline on a sample of the batch
    error = None
    cpu = None
    if not args.no_cpu:
        import oracle
        # runs of the batch at their full step counts, in batch order, each
        # at most 4e9 cell-updates (one host thread per run)
        sample_idx, acc = [], 0.0
        for k, q in enumerate(probs):
            if q.nz * q.steps <= 4e9:
                sample_idx.append(k)
                acc += q.nz * q.steps
                if acc >= args.cpu_sample_updates:
                    break
        sample = [probs[k].replace(precision=W.F64) for k in sample_idx]
        threads = min(16, os.cpu_count() or 1)
        log(f"oracle on {len(sample)} runs at full length ({acc:.3g} cell-updates), "
            f"{threads} threads")
        t0 = time.perf_counter()
        ref = oracle.solve_many(sample, threads=threads, fields=False)
        cdt = time.perf_counter() - t0
        errs = [rel(batch_out[k]["dft"], r["dft"]) for k, r in zip(sample_idx, ref)]
        error = {"dft_rel_l2_max": float(max(errs)),
                 "dft_rel_l2_median": float(np.median(errs)),
                 "vs": "FP64 oracle", "precision": args.precision,
                 "sample": f"{len(sample)} runs of the timed batch at their full "
                           "step counts (batch order, each <= 4e9 cell-updates)"}
        cpu = {"value": acc / cdt, "unit": "cell-updates/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{len(sample)} runs of the same seeded batch at full length "
                         f"({acc:.3g} cell-updates, {cdt:.1f} s), one run per thread"}
        log(f"cpu oracle: {cpu['value']:.4g} cell-updates/s on {threads} threads; "
            f"gpu DFT error max {error['dft_rel_l2_max']:.2e}")

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": f"batched moving bilayer crystals, {args.runs} runs, "
                        "nz log-uniform in [4096, 65536], steps = 4 nz, S = 0.5, "
                        "lambda0 = 40 cells",
            "runs": args.runs, "cell_updates_per_step": updates,
            "steps_cap": args.steps_cap or None,
            "seed": args.seed, "precision": args.precision,
            "parallelism": "single GPU, all runs in one launch per time block",
        },
        "roofline": roofline,
        "batched_f64": batched_f64,
        "serving": serving,
        "plain": plain,
        "batched_over_plain_slab": (value / plain[f"slab_{args.precision}"]["value"]
                                    if plain else None),
        "tmm_sweep": tmm,
        "twod": twod,
        "error": error,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
