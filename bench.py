"""Benchmark: batched generalized-FDTD solves on one MI355X.

A "step" is one pass of the whole hot path over one batch: every run of the
batched moving-bilayer-crystal workload (4096 runs, grid lengths
log-uniform in [4096, 65536], 4 nz time steps each) stepped from zero
fields to its last step, source, ends, probes and probe DFTs included.
Inputs (rest profiles, probes, frequencies) are resident in HBM before the
timed region.  `value` is total cell-updates (sum over runs of nz * steps)
per second of the timed passes.

Printed beside it, in the same JSON line:
  plain       -- the plain single-run form: the 65536-cell moving slab,
                 131072 steps, FP32 and FP64, one run per pass;
  error       -- relative L2 error against the FP64 oracle on a seeded
                 sample of the same workload;
  roofline    -- the stepping kernel (k_tiles) against the chip's vector
                 ALU peak, timed with HIP events on the library's stream;
  cpu_baseline-- the oracle on the host cores on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
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
# MI355X: 256 CUs x 64 lanes x 2 flops (FMA) x 2.4 GHz, without packed FP32
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


COUNTERS = os.path.join(ROOT, "profiles", "k_tiles_f32_crystals4096_hbm_counters.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2304_06586_amd", "csrc", "kernels.hip")


def measured_traffic_per_update(C, T):
    """HBM bytes per cell-update of k_tiles from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE counters (scaled by a plain copy), or None when
    the kernel source has changed since they were taken or they were taken
    at another tiling (cells per lane C, steps per launch T)."""
    import hashlib
    try:
        kv = {}
        for line in open(COUNTERS):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
        if kv.get("kernel_source_sha256") != sha:
            return None
        if int(kv["cells_per_lane"]) != C or int(kv["block_steps"]) != T:
            return None
        return float(kv["fetch_bytes_per_update"]) + float(kv["write_bytes_per_update"])
    except (OSError, KeyError, ValueError):
        return None


def gpu_pass_rate(P, problems, passes, warmup, tune=True, **exec_kw):
    import torch
    with P.Batch(problems, record_trace=False, fields=False, **exec_kw) as b:
        if tune:                      # outside the timed region
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
    return dt, st


def serve(P, stream, pool_bytes, max_slots, blocks_per_call=64, closed=False):
    """Drive the continuous-batching server with a request stream of
    (arrival time, problem).  closed=True submits everything at t = 0.
    Returns a dict: the seconds from the first arrival to the last
    completion, per-request latencies (s), total cell-updates, the
    (completion time, cell-updates) of every request, rejections, and the
    mean time a request waits for admission: by Little's law the time
    integral of the server's queue length divided by the requests that
    entered it."""
    lat = []
    done = []
    updates = 0
    rejected = 0
    queue_area = 0.0
    last_q, last_t = 0, 0.0
    accepted = 0
    with P.Server(pool_bytes=pool_bytes, max_slots=max_slots) as srv:
        pending = {}
        i = 0
        n = len(stream)
        t0 = time.perf_counter()
        while len(lat) + rejected < n:
            now = time.perf_counter() - t0
            while i < n and (closed or stream[i][0] <= now):
                arr = 0.0 if closed else stream[i][0]
                prob = stream[i][1]
                try:
                    rid = srv.submit(prob)
                except P.GfdtdError:
                    rejected += 1
                    i += 1
                    continue
                pending[rid] = (arr, prob.nz * prob.steps)
                updates += prob.nz * prob.steps
                accepted += 1
                i += 1
            if pending:
                now = time.perf_counter() - t0
                queue_area += last_q * (now - last_t)
                _, last_q = srv.progress(max_blocks=blocks_per_call)
                last_t = now
                for rid in list(pending):
                    if srv.ready(rid):
                        now = time.perf_counter() - t0
                        r = srv.poll(rid)
                        assert r["status"] == 0
                        arr, work = pending.pop(rid)
                        lat.append(now - arr)
                        done.append((now, work))
            elif i < n:
                time.sleep(max(0.0, min(0.01, stream[i][0] - now)))
        total = time.perf_counter() - t0
    return {"total_s": total, "latency_s": lat, "updates": updates,
            "done": sorted(done), "rejected": rejected,
            "queue_wait_mean_s": queue_area / max(1, accepted)}


def saturated_rate(done, lo=0.1, hi=0.7):
    """Cell-updates/s of a saturated server: the slope of completed work
    against time between lo and hi of the total work (the start, while the
    pipeline fills, and the drain, while the last long requests finish
    alone, are left out)."""
    t = np.array([d[0] for d in done])
    w = np.cumsum([d[1] for d in done])
    W = w[-1]
    i0 = int(np.searchsorted(w, lo * W))
    i1 = int(np.searchsorted(w, hi * W))
    if i1 <= i0 or t[i1] <= t[i0]:
        return W / t[-1]
    return float((w[i1] - w[i0]) / (t[i1] - t[i0]))


def cpu_baseline(sample, threads):
    import oracle
    t0 = time.perf_counter()
    outs = oracle.solve_many(sample, threads=threads, fields=False)
    dt = time.perf_counter() - t0
    upd = sum(p.nz * p.steps for p in sample)
    return upd / dt, dt, outs


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
    ap.add_argument("--cpu-sample-runs", type=int, default=384)
    ap.add_argument("--cpu-sample-steps", type=int, default=6000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default tiling instead of autotuning it")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-tmm", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=500)
    ap.add_argument("--serve-loads", default="0.25,0.5,0.75,0.9,1.1",
                    help="offered loads as fractions of the saturated request "
                         "rate, comma separated")
    ap.add_argument("--serve-nz-hi", type=float, default=1e5)
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
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
    dt, st = gpu_pass_rate(P, probs, args.steps, args.warmup, **exec_kw)
    value = updates * args.steps / dt
    ms_per_step = dt * 1e3 / args.steps
    log(f"batched: {value:.4g} cell-updates/s, {ms_per_step:.1f} ms per pass")

    # roofline of the stepping kernel from the library's HIP events (last pass)
    step_s = st["step_ms"] / 1e3
    avg_launch_ms = st["step_ms"] / max(1, st["launches"])
    k_rate = updates / step_s if step_s > 0 else 0.0
    achieved_tflops = k_rate * FLOPS_PER_UPDATE / 1e12
    hbm_equiv = k_rate * BYTES_PER_UPDATE[prec] / 1e9
    per_update = (measured_traffic_per_update(int(st["cells_per_lane"]),
                                              int(st["block_steps"]))
                  if prec == W.F32 else None)
    upd_per_launch = updates / max(1, st["launches"])
    traffic = per_update * upd_per_launch if per_update is not None else None
    roofline = {
        "kernel": "k_tiles",
        "bound": "alu",
        "achieved": round(achieved_tflops, 3),
        "peak": round(ALU_PEAK_TFLOPS, 1),
        "unit": "TFLOP/s",
        "frac": round(achieved_tflops / ALU_PEAK_TFLOPS, 4),
        "traffic": traffic,
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                        "copy-calibrated)",
        "measured_hbm_GBs": (round(traffic / (avg_launch_ms * 1e-3) / 1e9, 1)
                             if traffic is not None and avg_launch_ms > 0 else None),
        "algorithmic_bytes_per_launch": upd_per_launch * BYTES_PER_UPDATE[prec],
        "flops_per_update": FLOPS_PER_UPDATE,
        "launches_per_pass": int(st["launches"]),
        "avg_launch_ms": round(avg_launch_ms, 4),
        "cells_per_lane": int(st["cells_per_lane"]),
        "block_steps": int(st["block_steps"]),
        "single_step_hbm_equiv_GBs": round(hbm_equiv, 1),
        "single_step_hbm_frac": round(hbm_equiv / HBM_PEAK_GBS, 3),
    }

    # --------------------------------------------------- batched, other dtype
    batched_f64 = None
    if not args.no_f64 and prec == W.F32 and not args.steps_cap:
        probs64 = [q.replace(precision=W.F64) for q in probs]
        dt64, st64 = gpu_pass_rate(P, probs64, 1, 1, **exec_kw)
        batched_f64 = {"value": updates / dt64, "ms": dt64 * 1e3,
                       "cells_per_lane": int(st64["cells_per_lane"]),
                       "block_steps": int(st64["block_steps"]),
                       "hbm_equiv_frac": round(updates / dt64 * 32 / 8e12, 3)}
        log(f"batched f64: {batched_f64['value']:.4g} cell-updates/s")
        del probs64

    # ---------------------------------------------------------------- served
    serving = None
    if not args.no_serve:
        pool = int(args.serve_budget_gb * (1 << 30))
        stream = W.serving_stream(args.seed, args.serve_requests, 1.0,
                                  nz_hi=args.serve_nz_hi)
        sat = serve(P, stream, pool, 512, closed=True)
        cap = saturated_rate(sat["done"])
        mean_work = sat["updates"] / len(stream)
        cap_rps = cap / mean_work
        loads = []
        for frac in [float(x) for x in args.serve_loads.split(",") if x]:
            rate = frac * cap_rps
            st = W.serving_stream(args.seed + 1, args.serve_requests, rate,
                                  nz_hi=args.serve_nz_hi)
            res = serve(P, st, pool, 512)
            lat = np.array(res["latency_s"])
            loads.append({
                "offered_fraction": frac,
                "offered_requests_per_s": round(rate, 2),
                "cell_updates_per_s": res["updates"] / res["total_s"],
                "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
                "queue_wait_mean_ms": res["queue_wait_mean_s"] * 1e3,
                "rejected": res["rejected"],
            })
            log(f"serving at {frac:.2f} of capacity ({rate:.1f} req/s): "
                f"p50 {loads[-1]['p50_latency_ms']:.1f} ms p99 "
                f"{loads[-1]['p99_latency_ms']:.1f} ms, mean queueing "
                f"{loads[-1]['queue_wait_mean_ms']:.1f} ms")
        serving = {
            "saturated_cell_updates_per_s": cap,
            "saturated_requests_per_s": cap_rps,
            "saturated_note": "slope of completed work vs time between 10 % and "
                              "70 % of the total, all requests submitted at t = 0",
            "makespan_cell_updates_per_s": sat["updates"] / sat["total_s"],
            "loads": loads,
            "requests": len(stream),
            "mix": f"interface/slab/crystal/gradient, nz log-uniform in "
                   f"[1e3, {args.serve_nz_hi:.0e}], steps U[2,4] nz, "
                   "FP32 or FP64 with p = 1/2, Poisson arrivals",
            "budget_GB": args.serve_budget_gb,
        }
        log(f"serving: saturated {cap:.4g} cell-updates/s ({cap_rps:.1f} req/s)")

    # ------------------------------------------------------------------ plain
    plain = None
    if not args.no_plain:
        plain = {}
        for name, maker in (("interface", lambda pr: W.interface_run(args.seed, precision=pr)),
                            ("slab", lambda pr: W.slab_run(args.seed, precision=pr)),
                            ("gradient", lambda pr: W.gradient_run(args.seed,
                                                                  precision=pr))):
            for pname, pr in (("f32", W.F32), ("f64", W.F64)):
                p = maker(pr)
                pdt, pst = gpu_pass_rate(P, [p], 1, 1, tune=not args.no_tune)
                key = f"{name}_{pname}"
                plain[key] = {"value": p.nz * p.steps / pdt, "ms": pdt * 1e3,
                              "nz": p.nz, "steps": p.steps,
                              "cells_per_lane": int(pst["cells_per_lane"]),
                              "block_steps": int(pst["block_steps"]),
                              "graph": int(pst["graph"])}
                log(f"plain {key}: {plain[key]['value']:.4g} cell-updates/s "
                    f"(C={pst['cells_per_lane']}, T={pst['block_steps']})")

    # ------------------------------------------- transfer-matrix sweep (GPU)
    tmm = None
    if not args.no_tmm:
        stacks, omegas = W.tmm_crystals(args.seed, 4096, nomega=256)
        layers = sum(len(s.eps) for s in stacks)
        P.gfdtd_tmm(stacks[:8], omegas[:8])               # warm-up
        torch.cuda.synchronize()
        dt = float("inf")
        for _ in range(3):                                 # best of three calls
            t0 = time.perf_counter()
            Tg, Gg = P.gfdtd_tmm(stacks, omegas)
            dt = min(dt, time.perf_counter() - t0)
        evals = len(stacks) * len(omegas)
        tmm = {"stack_frequency_evals_per_s": evals / dt,
               "layer_evals_per_s": layers * len(omegas) / dt,
               "ms": dt * 1e3, "stacks": len(stacks), "frequencies": len(omegas),
               "layers": layers,
               "note": "one synchronous gfdtd_tmm call (best of three), host packing, "
                       "host-to-device upload of the stacks and result copies "
                       "included; FP64"}
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
        log(f"transfer-matrix sweep: {tmm['stack_frequency_evals_per_s']:.4g} "
            f"(stack, omega) evaluations/s, {tmm['layer_evals_per_s']:.4g} layers/s")

    # ---------------------------------------- error and CPU baseline (sample)
    sample = [q.replace(steps=min(q.steps, args.cpu_sample_steps))
              for q in W.crystal_runs(args.seed, count=args.cpu_sample_runs,
                                      precision=prec)]
    error = None
    cpu = None
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        log(f"oracle on {len(sample)} runs x <= {args.cpu_sample_steps} steps, "
            f"{threads} threads")
        rate, cdt, ref = cpu_baseline(sample, threads)
        got = P.gfdtd_solve_batch(sample, fields=False)
        errs = []
        for g, r in zip(got, ref):
            num = np.linalg.norm(g["trace"] - r["trace"])
            den = np.linalg.norm(r["trace"])
            errs.append(num / den if den > 0 else num)
        error = {"trace_rel_l2_max": float(max(errs)),
                 "trace_rel_l2_median": float(np.median(errs)),
                 "vs": "FP64 oracle", "sample": f"first {len(sample)} runs, "
                 f"steps capped at {args.cpu_sample_steps}"}
        cpu = {"value": rate, "unit": "cell-updates/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first {len(sample)} runs of the same seeded batch, "
                         f"each stepped min(4 nz, {args.cpu_sample_steps}) steps "
                         f"({sum(p.nz * p.steps for p in sample):.3g} "
                         f"cell-updates, {cdt:.1f} s)"}
        log(f"cpu oracle: {rate:.4g} cell-updates/s on {threads} threads; "
            f"gpu error max {error['trace_rel_l2_max']:.2e}")

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
        "error": error,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
