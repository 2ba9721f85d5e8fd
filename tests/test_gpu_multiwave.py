"""GPU checks of multi-wave tiles: G waves step one tile side by side and
refresh the cells they share (xl + xr lanes between neighbours) through
LDS every K steps.  The tiling changes only which wave computes a cell,
never its arithmetic, so results must equal one-wave tiles bit for bit;
FP64 results are also held to the oracle (relative L2 1e-12, as in
test_gpu_parity).

Every run starts from seeded random fields, so all cells carry data from
the first step and a stale overlap shows in the final fields; probes are
spread over the whole grid, including cells that waves share."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


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


def _case(nz, steps, beta, kind=W.MODULATION, precision=W.F64, seed=0,
          structure="crystal", window=None):
    p = W.small_case(nz, steps, beta, kind=kind, precision=precision, seed=seed,
                     structure=structure)
    d, b = W.random_fields(nz, seed=seed + 1000)
    probes = np.unique(np.linspace(0, nz - 1, min(40, nz)).astype(np.int64))
    p = p.replace(init_d=d, init_b=b, probes=probes)
    if window is not None:
        p = p.replace(window=window)
    return p


def _batch():
    """Runs of many sizes (one wave or less up to several tiles, so some
    tiles hold waves past the grid end), both signs of beta, both kinds,
    step counts that end inside a block and shorter than a block."""
    out = []
    specs = [(100, 70, 0.3), (333, 131, -0.35), (777, 200, 0.45),
             (3001, 157, -0.25), (5000, 96, 0.3), (9000, 63, 0.2),
             (12345, 250, -0.4), (2049, 5, 0.3), (64, 1, -0.3)]
    for i, (nz, steps, beta) in enumerate(specs):
        out.append(_case(nz, steps, beta, seed=10 + i))
    out.append(_case(4000, 120, 0.3, kind=W.MATTER, seed=31, structure="slab"))
    out.append(_case(2500, 90, -0.3, kind=W.MATTER, seed=32, structure="random"))
    return out


def _run(P, probs, C, T, G, K):
    with P.Batch(probs, cells_per_lane=C, block_steps=T, tile_waves=G,
                 exchange_steps=K, use_graph=0) as bt:
        st = bt.stats()
        bt.run()
        res = bt.collect()
    return res, st


# (C, T, G, K): the production shapes and edge shapes (K = 1: a refresh
# after every step; K = T: none inside a block; 2 and 3 waves)
TILINGS = [(12, 64, 4, 8), (8, 64, 4, 16), (4, 24, 3, 1), (16, 100, 4, 16),
           (12, 7, 4, 3), (8, 32, 2, 5), (12, 48, 4, 48 // 4)]


@pytest.fixture(scope="module")
def reference(P):
    probs = _batch()
    ref, st = _run(P, probs, 8, 16, 1, 0)
    assert st["tile_waves"] == 1
    return probs, ref


@pytest.mark.parametrize("C,T,G,K", TILINGS)
def test_multiwave_tiles_bitwise_equal_one_wave(P, reference, C, T, G, K):
    probs, ref = reference
    out, st = _run(P, probs, C, T, G, K)
    assert st["tile_waves"] == G and st["exchange_steps"] == K
    assert st["cells_per_lane"] == C and st["block_steps"] == T
    for i, (a, b) in enumerate(zip(out, ref)):
        assert a["status"] == 0
        for k in ("trace", "dft", "d", "b"):
            assert np.array_equal(a[k], b[k]), (C, T, G, K, i, probs[i].nz, k)


def test_multiwave_tiles_against_oracle(P, reference):
    probs, _ = reference
    out, _ = _run(P, probs, 12, 64, 4, 8)
    for i in (0, 1, 3, 5, 7, 9):
        want = oracle.solve(probs[i])
        got = out[i]
        for k in ("trace", "dft", "d"):
            e = rel(got[k], want[k])
            assert e <= TOL64, (i, k, e)
        assert rel(got["b"][:-1], want["b"][:-1]) <= TOL64


@pytest.mark.parametrize("precision", [W.F32, W.F64])
def test_multiwave_windows_and_precisions(P, precision):
    """Finite-duration modulations (their own kernel) and FP32 runs."""
    probs = [_case(6000, 150, 0.3, precision=precision, seed=50,
                   window=W.TimeWindow(20.0, 55.5, 1.6, 1.0)),
             _case(2200, 140, -0.3, precision=precision, seed=51,
                   window=W.TimeWindow(-1e30, 30.25, 1.4, 1.0)),
             _case(7000, 133, 0.35, precision=precision, seed=52)]
    ref, _ = _run(P, probs, 8, 24, 1, 0)
    C = 12 if precision == W.F32 else 8
    out, _ = _run(P, probs, C, 64, 4, 8)
    for i, (a, b) in enumerate(zip(out, ref)):
        for k in ("trace", "dft", "d", "b"):
            assert np.array_equal(a[k], b[k]), (precision, i, k)


def test_rings_keep_one_wave_tiles(P):
    p = W.small_case(3000, 100, 0.3, seed=3, abc=W.ABC_PERIODIC)
    d, b = W.random_fields(3000, seed=4)
    p = p.replace(init_d=d, init_b=b)
    out, st = _run(P, [p], 12, 32, 4, 8)
    assert st["tile_waves"] == 1
    want = oracle.solve(p)
    assert rel(out[0]["d"], want["d"]) <= TOL64


def test_large_run_multiwave_matches_one_wave(P):
    """One long run spanning many tiles at the production shape, FP32."""
    p = _case(200000, 200, 0.3, precision=W.F32, seed=77)
    ref, _ = _run(P, [p], 12, 32, 1, 0)
    out, _ = _run(P, [p], 12, 64, 4, 8)
    for k in ("trace", "dft", "d", "b"):
        assert np.array_equal(out[0][k], ref[0][k]), k
