"""Parity of the 2D HIP path (TE / TM) with the FP64 2D oracle, through
the C-ABI of include/gfdtd2d.h.

FP64 runs agree with the oracle to 1e-12 of the run's field scale (final
fields and probe traces; spectra to 1e-12 of their peak); FP32 runs within
max(1e-5, the arithmetic bound of the 1D tests), since each cell-update has
the same rounding profile.
Cases span several strips along z and several column chunks along x with
ragged tails, both signs of v and v = 0, all three z-end conditions and a
non-zero initial state; the execution options change nothing, bit for bit.
At the benchmark's full grid (4096 x 4096) a short run is compared with
the oracle element by element and the full-length run is checked through
properties that hold at any size: the x-structure the oblique source
imposes, FP32 against FP64, and finite spectra.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import stepper2d

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2304_06586_amd as pkg
    pkg.load_library()
    return pkg


def fp32_bound(p):
    u = 2.0 ** -24
    t = p.steps * p.courant
    return 4.0 * u * ((1.0 + abs(p.beta)) * p.pulse.omega * t + math.sqrt(10.0 * p.steps))


def peak(a):
    return max(float(np.max(np.abs(a))), 1e-300)


def compare(got, want, tol, what):
    """Largest deviation of every output: fields and traces relative to the
    run's field scale (the largest of the oracle's final fields and probe
    trace; a field that has nearly left the grid by the end is not its own
    scale), spectra relative to their peak."""
    scale = max(peak(want[k]) for k in ("d", "b", "c", "trace"))
    worst = {}
    for k in ("d", "b", "c", "trace"):
        worst[k] = float(np.max(np.abs(got[k] - want[k]))) / scale
    worst["dft"] = float(np.max(np.abs(got["dft"] - want["dft"]))) / peak(want["dft"])
    print(what, {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    for k, v in worst.items():
        assert v <= tol, (what, k, v)


CASES = [
    # nx, nz, steps, beta, abc
    (37, 700, 400, 0.35, W.ABC_MUR1),
    (37, 700, 400, -0.35, W.ABC_MUR1),
    (5, 301, 300, 0.0, W.ABC_MUR1),
    (64, 520, 360, 0.3, W.ABC_PEC),
    (19, 257, 333, -0.45, W.ABC_PERIODIC),
    (1, 130, 200, 0.2, W.ABC_MUR1),
]


@pytest.mark.parametrize("pol", [W.TE, W.TM])
@pytest.mark.parametrize("nx,nz,steps,beta,abc", CASES)
def test_small_cases_fp64(P, pol, nx, nz, steps, beta, abc):
    p = W.small_case_2d(nx, nz, steps, beta, pol=pol, abc=abc, seed=nx + nz,
                        m=1 if nx > 1 else 0, structure="random")
    print("case", pol, nx, nz, steps, beta, abc, flush=True)
    compare(P.gfdtd2d_solve(p), stepper2d.solve(p), TOL64, f"f64 {pol} {nx}x{nz}")


@pytest.mark.parametrize("pol", [W.TE, W.TM])
@pytest.mark.parametrize("nx,nz,steps,beta,abc", CASES[:2] + CASES[3:5])
def test_small_cases_fp32(P, pol, nx, nz, steps, beta, abc):
    p = W.small_case_2d(nx, nz, steps, beta, pol=pol, abc=abc, seed=nx + nz,
                        m=2, structure="slab", precision=W.F32)
    tol = max(TOL32, fp32_bound(p))
    print("case", pol, nx, nz, steps, beta, abc, "tol", tol, flush=True)
    compare(P.gfdtd2d_solve(p), stepper2d.solve(p), tol, f"f32 {pol} {nx}x{nz}")


@pytest.mark.parametrize("pol", [W.TE, W.TM])
@pytest.mark.parametrize("beta", [0.3, -0.3])
def test_initial_state_on_a_ring(P, pol, beta):
    rng = np.random.default_rng(7)
    p = W.small_case_2d(23, 400, 250, beta, pol=pol, abc=W.ABC_PERIODIC, seed=3)
    p.init_d = rng.normal(size=(23, 400))
    p.init_b = rng.normal(size=(23, 400))
    p.init_c = rng.normal(size=(23, 400))
    compare(P.gfdtd2d_solve(p), stepper2d.solve(p), TOL64, f"init ring {pol} {beta}")


@pytest.mark.parametrize("pol", [W.TE, W.TM])
@pytest.mark.parametrize("nz,abc", [(40, W.ABC_PERIODIC), (16, W.ABC_MUR1)])
def test_profile_moves_beyond_the_grid(P, pol, nz, abc):
    """Long runs on short grids: the profile shift m = rint(beta S tau)
    passes several grid lengths (wrapped on a ring, clamped off it)."""
    p = W.small_case_2d(7, nz, 1500, 0.5, pol=pol, abc=abc, seed=9, structure="random")
    m_end = round(p.beta * p.courant * (p.steps + 0.5))
    assert m_end > 4 * nz
    compare(P.gfdtd2d_solve(p), stepper2d.solve(p), TOL64, f"long shift {pol} {nz} {abc}")


def test_zero_steps_return_the_initial_state(P):
    rng = np.random.default_rng(1)
    p = W.small_case_2d(9, 80, 0, 0.2, pol=W.TM)
    p.init_d = rng.normal(size=(9, 80))
    p.init_c = rng.normal(size=(9, 80))
    got = P.gfdtd2d_solve(p)
    assert np.array_equal(got["d"], p.init_d)
    want_c = p.init_c.copy()
    want_c[:, -1] = 0.0                     # TM C has nz - 1 nodes
    assert np.array_equal(got["c"], want_c)
    assert not np.any(got["b"])


@pytest.mark.parametrize("precision,narrow,wide", [(W.F32, 4, 8), (W.F64, 2, 4)])
def test_execution_options_do_not_change_results(P, precision, narrow, wide):
    """Cells per lane, columns per wave and steps per launch change nothing,
    bit for bit (301 steps: the multi-step launches end with single
    steps); FP32 also at 2 cells per lane."""
    tilings = [(narrow, x, t) for t in (1, 2, 3, 4) for x in (1, 3, 16, 64)]
    tilings += [(wide, x, 1) for x in (1, 8)]
    if precision == W.F32:
        tilings += [(2, x, t) for t in (1, 3) for x in (5, 32)]
    for pol in (W.TE, W.TM):
        p = W.small_case_2d(41, 1500, 301, -0.3, pol=pol, precision=precision, seed=2,
                            m=3, structure="slab")
        ref = None
        for C, xch, T in tilings:
            with P.Run2D(p, cells_per_lane=C, columns_per_wave=xch, block_steps=T) as r:
                r.run()
                out = r.collect()
                st = r.stats()
            assert st["cells_per_lane"] == C and st["columns_per_wave"] == min(xch, 41)
            assert st["block_steps"] == T and st["launches"] == 301 // T + 301 % T
            if ref is None:
                ref = out
                continue
            for k in ("d", "b", "c", "trace"):
                diff = float(np.max(np.abs(out[k] - ref[k])))
                assert np.array_equal(out[k], ref[k]), (pol, C, xch, T, k, diff)


def test_multi_step_launches_near_the_grid_ends(P):
    """Short grids where the last strips hold the ends in their halo rows
    and the lattices end in different strips (nz = STRIDE + 1, + 2): four
    steps a launch against one, bit for bit, and against the oracle."""
    for precision, C in ((W.F32, 4), (W.F64, 2)):
        stride = 64 * C - 2 * 12
        for nz in (stride + 1, stride + 2, 2 * stride - 1):
            for pol in (W.TE, W.TM):
                for beta in (0.4, -0.4):
                    p = W.small_case_2d(6, nz, 120, beta, pol=pol, precision=precision,
                                        seed=nz, structure="random")
                    outs = []
                    for T in (1, 4):
                        with P.Run2D(p, block_steps=T) as r:
                            r.run()
                            outs.append(r.collect())
                    for k in ("d", "b", "c", "trace"):
                        assert np.array_equal(outs[0][k], outs[1][k]), (precision, nz, pol, beta, k)
                    if precision == W.F64:
                        compare(outs[1], stepper2d.solve(p), TOL64, f"ends {nz} {pol} {beta}")


def test_repeated_passes_are_identical(P):
    p = W.small_case_2d(33, 600, 300, 0.4, pol=W.TE, precision=W.F32, seed=4)
    with P.Run2D(p) as r:
        r.run()
        a = r.collect()
        r.run()
        b = r.collect()
    for k in ("d", "b", "c", "trace", "dft"):
        assert np.array_equal(a[k], b[k])


# ------------------------------------------------------- benchmark grid

def _bench(pol, precision, steps=None):
    p = W.slab_run_2d(0, pol=pol, precision=precision)
    if steps is not None:
        p = p.replace(steps=steps)
    return p


@pytest.mark.parametrize("pol,precision", [(W.TE, W.F32), (W.TM, W.F64)])
def test_benchmark_grid_short_run_elementwise(P, pol, precision):
    """The full 4096 x 4096 grid in the benchmark's launch configuration,
    for 40 steps (the oracle takes seconds there): every field element."""
    p = _bench(pol, precision, steps=40)
    p = p.replace(pulse=W.Pulse(amp=1.0, omega=p.pulse.omega, t0=5.0, tau=3.0,
                                phase=p.pulse.phase, t_off=10.0))
    with P.Run2D(p) as r:
        r.run()
        got = r.collect()
    want = stepper2d.solve(p)
    tol = TOL64 if precision == W.F64 else max(TOL32, fp32_bound(p))
    compare(got, want, tol, f"bench grid {pol} short")


@pytest.mark.parametrize("pol", [W.TE, W.TM])
def test_benchmark_grid_full_length_properties(P, pol):
    """Full benchmark run, both precisions: (1) the oblique source makes
    D(i, k) = cos(kx x_i) d(k) exactly (x_i = i for TE, i + 1/2 for TM), so
    every column is that multiple of one profile; (2) FP32 probes and final
    D agree with FP64 within the FP32 bound; (3) spectra are finite."""
    p64 = _bench(pol, W.F64)
    p32 = _bench(pol, W.F32)
    with P.Run2D(p64) as r:
        r.run()
        a = r.collect()
    with P.Run2D(p32) as r:
        r.run()
        b = r.collect()
    assert a["status"] == 0 and b["status"] == 0
    prof = p64.src_profile
    d = a["d"]
    j = int(np.argmax(np.abs(prof)))
    shape = np.outer(prof / prof[j], d[j])
    err = float(np.max(np.abs(d - shape))) / peak(d)
    print(f"x-structure {err:.2e}", flush=True)
    assert err < 1e-11
    tol = max(TOL32, fp32_bound(p32))
    tr = float(np.max(np.abs(a["trace"] - b["trace"]))) / peak(a["trace"])
    fd = float(np.max(np.abs(a["d"] - b["d"]))) / peak(a["d"])
    print(f"f32 vs f64: trace {tr:.2e} field {fd:.2e} tol {tol:.2e}", flush=True)
    assert tr <= tol and fd <= tol
    assert np.all(np.isfinite(a["dft"])) and np.all(np.isfinite(b["dft"]))
