"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances (relative L2 over each output):
  FP64 path: 1e-12 -- the kernels use reciprocal coefficients and fused
             multiply-adds, so they differ from the oracle only in rounding;
  FP32 path: 1e-5 on the oracle-sized cases -- FP32 storage and stencil
             arithmetic; the error is printed per case.  Full-size FP32 runs
             are held to a bound from the arithmetic (fp32_bound below).
Final fields of a run whose pulse has left the grid are a residual far
below the pulse, so at full size they are compared by the largest
deviation relative to the largest field the run's probes recorded.
Bit-for-bit on the GPU side: results do not depend on the tiling, the
temporal block depth, graph capture or the batch they run in.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def rel(a, b):
    den = np.linalg.norm(np.ravel(b))
    num = np.linalg.norm(np.ravel(a) - np.ravel(b))
    return float(num / den) if den > 0 else float(num)


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2304_06586_amd as pkg
    pkg.load_library()
    return pkg


def compare(got, want, tol, label=""):
    errs = {}
    for key in ("trace", "dft", "d", "b"):
        if key not in got or key not in want:
            continue
        a, b = got[key], want[key]
        if key == "b":
            a, b = a[:-1], b[:-1]
        if np.size(b) == 0:
            continue
        errs[key] = rel(a, b)
    print(f"{label}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    for k, v in errs.items():
        assert v <= tol, (label, k, v)
    assert got["status"] == 0
    return errs


def fp32_bound(p):
    """Bound on the relative error of an FP32 run's probe trace and spectra
    against the FP64 oracle.  Coefficients rounded to FP32 (relative error
    u = 2^-24 each) change the local wave speed by at most u and unbalance
    the velocity terms by at most |beta| u, so a carrier at omega picks up
    a phase error of at most u (1 + |beta|) omega t after travelling for a
    time t (sum of k dz over the path = omega t, whatever the medium); the
    stencil's own roundings, about ten per cell and step, add a random walk
    of about u (10 N)^(1/2) over N steps.  Four times the sum."""
    u = 2.0 ** -24
    t = p.steps * p.courant
    return 4.0 * u * ((1.0 + abs(p.beta)) * p.pulse.omega * t + np.sqrt(10.0 * p.steps))


def field_dev(got, want, peak):
    """Largest deviation of a final field relative to the run's peak probe
    field."""
    return float(np.max(np.abs(np.asarray(got) - np.asarray(want))) / peak)


def run(P, p, **exec_kw):
    if not exec_kw:
        return P.gfdtd_solve(p)
    with P.Batch([p], **exec_kw) as b:
        b.run()
        return b.collect()[0]


# ---------------------------------------------------------------------------

def test_interface_config_fp64(P):
    """Moving interface, 2000 cells x 4000 steps, FP64 (full size)."""
    p = W.interface_run(0)
    compare(run(P, p), oracle.solve(p), TOL64, "interface f64")


def test_interface_config_fp32(P):
    p = W.interface_run(0, precision=W.F32)
    compare(run(P, p), oracle.solve(p), TOL32, "interface f32")


CASES = [
    # nz, steps, beta, kind, structure, abc
    (8, 1, 0.3, W.MODULATION, "random", W.ABC_MUR1),
    (9, 37, -0.2, W.MODULATION, "random", W.ABC_MUR1),
    (63, 100, 0.45, W.MODULATION, "slab", W.ABC_MUR1),
    (200, 333, 0.0, W.MODULATION, "random", W.ABC_MUR1),
    (1000, 517, -0.35, W.MODULATION, "crystal", W.ABC_MUR1),
    (3001, 1200, 0.3, W.MODULATION, "slab", W.ABC_PEC),
    (4099, 900, 0.25, W.MATTER, "random", W.ABC_MUR1),
    (2500, 700, -0.4, W.MATTER, "slab", W.ABC_MUR1),
    (777, 64, 0.6, W.MODULATION, "uniform", W.ABC_PEC),
]


@pytest.mark.parametrize("nz,steps,beta,kind,structure,abc", CASES)
@pytest.mark.parametrize("precision", [W.F64, W.F32])
def test_small_cases(P, nz, steps, beta, kind, structure, abc, precision):
    p = W.small_case(nz, steps, beta, kind=kind, structure=structure, abc=abc,
                     precision=precision, seed=nz + steps, nprobe=5)
    want = oracle.solve(p)
    tol = TOL64 if precision == W.F64 else TOL32
    compare(run(P, p), want, tol, f"{nz}x{steps} b={beta} k={kind} p={precision}")


@pytest.mark.parametrize("C,T", [(4, 1), (8, 1), (16, 1), (4, 7), (8, 16),
                                 (16, 16), (16, 33), (8, 32), (4, 15), (12, 1),
                                 (12, 24), (12, 37)])
@pytest.mark.parametrize("beta", [0.35, -0.3])
def test_tilings_agree_bitwise_and_match_oracle(P, C, T, beta):
    """Every (cells per lane, steps per launch) tiling gives the same bits,
    and they match the oracle."""
    p = W.small_case(2345, 301, beta, structure="crystal", seed=5, nprobe=5)
    ref = run(P, p, cells_per_lane=8, block_steps=1, use_graph=0)
    got = run(P, p, cells_per_lane=C, block_steps=T, use_graph=0)
    for k in ("trace", "dft", "d", "b"):
        assert np.array_equal(got[k], ref[k]), (C, T, k)
    compare(got, oracle.solve(p), TOL64, f"C={C} T={T}")


_TILING_ORACLE = {}


@pytest.mark.parametrize("C,T", [(12, 24), (12, 48), (16, 24), (16, 48), (4, 24), (8, 48)])
@pytest.mark.parametrize("beta", [0.35, -0.3])
@pytest.mark.parametrize("kind", [W.MODULATION, W.MATTER])
@pytest.mark.parametrize("precision", [W.F64, W.F32])
def test_one_wave_tilings_by_kind_and_precision(P, C, T, beta, kind, precision):
    """One-wave tiles at every cells-per-lane the tuner may pick, shallow
    and deep blocks, both kinds, both precisions and both signs of v: the
    same bits as one step per launch at 8 cells per lane, and the oracle."""
    p = W.small_case(4321, 500, beta, kind=kind, structure="crystal", seed=7, nprobe=5,
                     precision=precision)
    ref = run(P, p, cells_per_lane=8, block_steps=1, tile_waves=1, use_graph=0)
    got = run(P, p, cells_per_lane=C, block_steps=T, tile_waves=1, use_graph=0)
    for k in ("trace", "dft", "d", "b"):
        assert np.array_equal(got[k], ref[k]), (C, T, k)
    key = (kind, beta)
    if key not in _TILING_ORACLE:
        _TILING_ORACLE[key] = oracle.solve(p)
    tol = TOL64 if precision == W.F64 else TOL32
    compare(got, _TILING_ORACLE[key], tol, f"C={C} T={T} k={kind} b={beta} p={precision}")


def test_graph_capture_matches_plain_launches(P):
    p = W.small_case(1500, 800, 0.3, structure="slab", seed=9)
    a = run(P, p, use_graph=0)
    with P.Batch([p], use_graph=1) as b:
        assert b.stats()["graph"] == 1
        outs = []
        for _ in range(3):              # replays, with host work between
            b.run()
            outs.append(b.collect()[0])
    for o in outs:
        for k in ("trace", "dft", "d", "b"):
            assert np.array_equal(o[k], a[k]), k


def test_batch_equals_alone_bitwise(P):
    """Each run of a batch of mixed sizes, velocities, kinds and
    precisions gives the same bits as the run alone."""
    probs = [W.small_case(n, s, b, kind=k, precision=pr, structure=st, seed=i)
             for i, (n, s, b, k, pr, st) in enumerate([
                 (500, 200, 0.3, W.MODULATION, W.F64, "slab"),
                 (3000, 900, -0.2, W.MODULATION, W.F64, "crystal"),
                 (129, 1000, 0.5, W.MODULATION, W.F32, "random"),
                 (2049, 17, 0.1, W.MATTER, W.F64, "random"),
                 (900, 450, 0.4, W.MATTER, W.F32, "slab"),
                 (64, 64, -0.45, W.MODULATION, W.F32, "uniform"),
             ])]
    batch = P.gfdtd_solve_batch(probs)
    for p, got in zip(probs, batch):
        alone = P.gfdtd_solve(p)
        for k in ("trace", "dft", "d", "b"):
            assert np.array_equal(got[k], alone[k]), (p.label, k)
        tol = TOL64 if p.precision == W.F64 else TOL32
        compare(got, oracle.solve(p), tol, p.label)


def test_two_stream_batch_equals_alone_bitwise(P):
    """Groups of at least 4M cells are split into two halves whose launches
    go to two streams and overlap.  Each run of such a batch (two groups,
    runs of different lengths, so the halves end at different blocks) gives
    the same bits as the run alone, on one stream."""
    spec = [(700_001 + 37 * i, 120 + 41 * i, (-0.3, 0.2, 0.45)[i % 3]) for i in range(6)]
    probs = [W.small_case(n, s, b, kind=W.MODULATION, precision=W.F32,
                          structure="random", seed=10 + i)
             for i, (n, s, b) in enumerate(spec)]
    probs += [W.small_case(n, s + 7, -b, kind=W.MATTER, precision=W.F64,
                           structure="slab", seed=20 + i)
              for i, (n, s, b) in enumerate(spec)]
    assert sum(p.nz for p in probs[:6]) >= 4 << 20
    with P.Batch(probs) as b:
        b.run()
        got = b.collect()
        st = b.stats()
        # the tuner times both halves on their streams; the choice changes
        # only the tiling
        b.autotune(trial_blocks=2)
        b.run()
        tuned = b.collect()
        st_tuned = b.stats()
    assert st["streams"] == 2 and st["graph"] == 0, st
    assert st_tuned["streams"] == 2, st_tuned
    # a captured pass keeps every launch on one stream
    with P.Batch(probs, use_graph=1) as b:
        b.run()
        graphed = b.collect()
        st_graph = b.stats()
    assert st_graph["graph"] == 1 and st_graph["streams"] == 1, st_graph
    for i, p in enumerate(probs):
        alone = P.gfdtd_solve(p)
        for k in ("trace", "dft", "d", "b"):
            for name, res in (("split", got), ("tuned", tuned), ("graph", graphed)):
                assert np.array_equal(res[i][k], alone[k]), (p.label, name, k)


def test_zero_steps_and_no_probes(P):
    p = W.small_case(300, 0, 0.3, seed=2)
    got = P.gfdtd_solve(p)
    assert got["trace"].shape == (len(p.probes), 0)
    assert np.all(got["d"] == 0) and np.all(got["dft"] == 0)
    q = W.small_case(300, 50, 0.3, seed=2).replace(probes=np.zeros(0, np.int64),
                                                   omegas=np.zeros(0))
    got = P.gfdtd_solve(q)
    want = oracle.solve(q)
    assert rel(got["d"], want["d"]) < TOL64


def test_probes_and_source_at_the_edges(P):
    p = W.small_case(1111, 400, 0.3, seed=3, structure="random")
    p = p.replace(src_cell=1, probes=np.array([0, 1, 2, 1108, 1109, 1110]))
    compare(run(P, p), oracle.solve(p), TOL64, "edges src=1")
    q = p.replace(src_cell=1109, beta=-0.3)
    compare(run(P, q), oracle.solve(q), TOL64, "edges src=nz-2")


@pytest.mark.parametrize("kind", [W.MODULATION, W.MATTER])
@pytest.mark.parametrize("beta", [0.3, -0.3])
@pytest.mark.parametrize("precision", [W.F64, W.F32])
def test_many_probes_in_the_end_waves(P, kind, beta, precision):
    """Four probes in each end wave, on and next to the end nodes, with
    the source next to an end: narrow lanes (4 and 8 cells per lane) keep
    two probes as wave-uniform values and record the others by the general
    path; the same bits as 12 cells per lane, and the oracle."""
    nz = 1500
    p = W.small_case(nz, 600, beta, kind=kind, structure="random", seed=11,
                     precision=precision)
    p = p.replace(src_cell=2 if beta > 0 else nz - 3,
                  probes=np.array([0, 1, 2, 5, nz // 2, nz - 6, nz - 3, nz - 2, nz - 1]))
    ref = run(P, p, cells_per_lane=12, block_steps=16, tile_waves=1, use_graph=0)
    for C, T in ((4, 24), (8, 16), (4, 1)):
        got = run(P, p, cells_per_lane=C, block_steps=T, tile_waves=1, use_graph=0)
        for k in ("trace", "dft", "d", "b"):
            assert np.array_equal(got[k], ref[k]), (C, T, k)
    if precision == W.F64:
        compare(ref, oracle.solve(p), TOL64, f"many probes k={kind} b={beta}")


# ---------------------------------------------------------------------------
# Benchmark sizes, in the launch configuration the benchmark uses

def test_slab_full_grid_first_steps_fp64(P):
    """The 65536-cell moving slab at its full grid, stepped 3000 steps
    (oracle-checkable), default tiling."""
    p = W.slab_run(0).replace(steps=3000)
    compare(run(P, p), oracle.solve(p), TOL64, "slab 65536x3000 f64")


def test_gradient_downscaled_copy(P):
    """Moving-matter tanh gradient, 2^14 cells x 2^12 steps: FP64 and
    FP32 against the oracle."""
    p = W.gradient_run(0, precision=W.F64, downscaled=True)
    want = oracle.solve(p)
    compare(run(P, p), want, TOL64, "gradient small f64")
    compare(run(P, p.replace(precision=W.F32)), want, TOL32, "gradient small f32")


def test_crystal_batch_sample(P):
    """A seeded sample of the batched-crystal workload (first 8 runs,
    steps cut to 4000 so the oracle finishes in seconds), batched."""
    probs = [q.replace(steps=4000) for q in W.crystal_runs(0, count=8, precision=W.F64)]
    got = P.gfdtd_solve_batch(probs)
    for p, g in zip(probs, got):
        compare(g, oracle.solve(p), TOL64, p.label)


def test_autotune_keeps_results_bitwise(P):
    """The autotuner changes only the tiling: same bits before and after,
    with and without graph replay."""
    probs = [W.small_case(n, s, b, structure="crystal", seed=i, nprobe=3)
             for i, (n, s, b) in enumerate([(3000, 700, 0.3), (1500, 900, -0.25),
                                            (5000, 300, 0.1)])]
    for graph in (0, 1):
        with P.Batch(probs, use_graph=graph) as b:
            b.run()
            ref = b.collect()
            chosen = b.autotune(trial_blocks=3)
            assert chosen["cells_per_lane"] in (4, 8, 12, 16)
            assert chosen["block_steps"] in (8, 16, 24, 32, 48, 64)
            assert chosen["tile_waves"] in (1, 4)
            st = b.stats()
            assert (st["cells_per_lane"], st["block_steps"], st["tile_waves"]) == \
                (chosen["cells_per_lane"], chosen["block_steps"], chosen["tile_waves"])
            b.run()
            got = b.collect()
        for x, y in zip(got, ref):
            for k in ("trace", "dft", "d", "b"):
                assert np.array_equal(x[k], y[k]), k


def test_blowup_is_reported_per_run(P):
    """A run forced past the pre-flight (|beta| n > 1 with
    GFDTD_FLAG_ALLOW_UNSTABLE) overflows; the watchdog marks that run
    GFDTD_E_BLOWUP and its batch neighbour is unaffected."""
    bad = W.small_case(400, 2000, 0.3, seed=1, structure="uniform",
                       precision=W.F32)
    # vacuum, beta = 0.9 at S = 0.9: beyond S <= n/(1 + n beta); the
    # amplification factor is 4.4 per step
    bad = bad.replace(eps_rest=np.ones(400), mu_rest=np.ones(400), beta=0.9,
                      courant=0.9, flags=W.FLAG_ALLOW_UNSTABLE)
    good = W.small_case(400, 600, 0.3, seed=2, precision=W.F32)
    out = P.gfdtd_solve_batch([bad, good])
    assert out[0]["status"] == P.gfdtd.GFDTD_E_BLOWUP
    assert out[1]["status"] == 0
    alone = P.gfdtd_solve(good)
    assert np.array_equal(out[1]["trace"], alone["trace"])


def test_gradient_full_size_fp32_against_fp64(P):
    """Moving-matter gradient at full size (2^20 cells, 2^18 steps): the
    FP32 path (FP64 shifts, coefficients and DFT) against the FP64 path on
    the probe spectra and traces."""
    p64 = W.gradient_run(0, precision=W.F64)
    a = P.gfdtd_solve(p64, fields=False)
    b = P.gfdtd_solve(p64.replace(precision=W.F32), fields=False)
    e_dft = rel(b["dft"], a["dft"])
    e_tr = rel(b["trace"], a["trace"])
    print(f"gradient 2^20 x 2^18: FP32 vs FP64 dft {e_dft:.2e} trace {e_tr:.2e}")
    assert a["status"] == 0 and b["status"] == 0
    assert e_dft < 1e-3 and e_tr < 1e-3


def test_full_crystal_batch_in_benchmark_configuration(P):
    """The whole 4096-run FP32 crystal batch at full step counts, in the
    launch configuration the benchmark times (autotuned tiling): every run
    finishes with finite probes, and the probe spectra of the three
    smallest runs (4096+ cells, 16384+ steps each) match the oracle."""
    import oracle as O
    probs = W.crystal_runs(0, count=4096, precision=W.F32)
    with P.Batch(probs, record_trace=False, fields=False) as b:
        b.autotune(trial_blocks=4)
        b.run()
        got = b.collect()
        st = b.stats()
    assert all(g["status"] == 0 for g in got)
    order = np.argsort([p.nz for p in probs])[:3]
    for i in order:
        want = O.solve(probs[i], fields=False)
        e = rel(got[i]["dft"], want["dft"])
        print(f"run {i} nz={probs[i].nz} steps={probs[i].steps} C={st['cells_per_lane']} "
              f"T={st['block_steps']}: DFT rel err {e:.2e}", flush=True)
        assert e < TOL32


@pytest.fixture(scope="module")
def slab_reference():
    """The oracle on the full 65536-cell, 131072-step moving slab (8.6e9
    cell-updates), shared by the FP64 and FP32 checks."""
    p = W.slab_run(0)
    return p, oracle.solve(p)


def test_slab_full_size_fp64(P, slab_reference):
    """The 65536-cell moving slab for all 131072 steps in FP64 against the
    oracle.  The probe trace and spectra are held to the FP64 tolerance.  By
    the end the pulse has left through the absorbing ends and the final
    fields are a residual of about 1e-4 of the pulse, so they are compared
    by their largest deviation relative to the run's peak probe field, also
    at the FP64 tolerance."""
    p, want = slab_reference
    got = P.gfdtd_solve(p)
    peak = float(np.max(np.abs(want["trace"])))
    e_tr = rel(got["trace"], want["trace"])
    e_dft = rel(got["dft"], want["dft"])
    e_d = field_dev(got["d"], want["d"], peak)
    e_b = field_dev(got["b"][:-1], want["b"][:-1], peak)
    print(f"slab 65536x131072 f64: trace={e_tr:.2e} dft={e_dft:.2e} "
          f"max|dd|/peak={e_d:.2e} max|db|/peak={e_b:.2e}; "
          f"final |d| / peak probe = {np.max(np.abs(want['d'])) / peak:.1e}", flush=True)
    assert got["status"] == 0
    assert e_tr <= TOL64 and e_dft <= TOL64
    assert e_d <= TOL64 and e_b <= TOL64


def test_slab_full_size_fp32(P, slab_reference):
    """The same slab in FP32 (FP64 shifts, coefficients before rounding,
    source, probes and DFT) against the FP64 oracle, held to the
    arithmetic bound of the FP32 path."""
    p64, want = slab_reference
    p = p64.replace(precision=W.F32)
    got = P.gfdtd_solve(p)
    peak = float(np.max(np.abs(want["trace"])))
    e_tr = rel(got["trace"], want["trace"])
    e_dft = rel(got["dft"], want["dft"])
    e_d = field_dev(got["d"], want["d"], peak)
    bound = fp32_bound(p)
    print(f"slab 65536x131072 f32: trace={e_tr:.2e} dft={e_dft:.2e} "
          f"max|dd|/peak={e_d:.2e} (bound {bound:.2e})", flush=True)
    assert got["status"] == 0
    assert e_tr <= bound and e_dft <= bound and e_d <= bound


def test_crystal_batch_largest_runs_full_length(P):
    """The eight longest runs of the 4096-run crystal batch (nz near 65536,
    about 2.6e5 steps each, 1.3e11 cell-updates), batched in FP32 at their
    full step counts, against the FP64 oracle (one host thread per run)."""
    probs = W.crystal_runs(0, count=4096, precision=W.F32)
    order = np.argsort([-(q.nz * q.steps) for q in probs])[:8]
    sel = [probs[i] for i in order]
    got = P.gfdtd_solve_batch(sel, fields=False)
    threads = min(8, os.cpu_count() or 1)
    want = oracle.solve_many([q.replace(precision=W.F64) for q in sel], threads=threads)
    for i, q, g, r in zip(order, sel, got, want):
        e_tr = rel(g["trace"], r["trace"])
        e_dft = rel(g["dft"], r["dft"])
        bound = fp32_bound(q)
        print(f"crystal run {i}: nz={q.nz} steps={q.steps} beta={q.beta:.3f} f32: "
              f"trace={e_tr:.2e} dft={e_dft:.2e} (bound {bound:.2e})", flush=True)
        assert g["status"] == 0
        assert e_tr <= bound and e_dft <= bound
