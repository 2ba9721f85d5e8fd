"""GPU checks of the halo bounds: probes on every cell of a band around the
edges of the owned regions (of one-wave tiles and of the waves of a
multi-wave tile), step counts that are whole blocks (so the final E sample
is taken after a full block), and cells per lane that divide 2T, where
the halo is exactly as wide as the reach it must cover.  Compared with
the FP64 oracle (relative L2 1e-12, as in test_gpu_parity), the final
trace sample included."""
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


def _case(beta, band, steps, seed):
    p = W.small_case(3000, steps, beta, structure="crystal", seed=seed)
    d, b = W.random_fields(3000, seed=seed + 1)
    return p.replace(init_d=d, init_b=b, probes=np.arange(band[0], band[1], dtype=np.int64))


# (beta, probe band, steps, C, T, G, K).  Bands cover the owned-region
# edges of the first tiles (and of the first waves of a 4-wave tile).
CASES = [
    (-0.3, (640, 704), 240, 12, 24, 1, 0),
    (0.3, (640, 704), 240, 12, 24, 1, 0),
    (-0.3, (420, 484), 256, 8, 32, 4, 8),
    (0.3, (420, 484), 256, 8, 32, 4, 8),
    (-0.3, (660, 724), 192, 12, 48, 4, 6),
    (0.3, (1340, 1404), 192, 12, 48, 4, 6),
]


@pytest.mark.parametrize("beta,band,steps,C,T,G,K", CASES)
def test_probe_bands_at_owned_edges(P, beta, band, steps, C, T, G, K):
    p = _case(beta, band, steps, seed=int(100 * abs(beta)) + C + T)
    with P.Batch([p], cells_per_lane=C, block_steps=T, tile_waves=G,
                 exchange_steps=K, use_graph=0) as bt:
        bt.run()
        got = bt.collect()[0]
    want = oracle.solve(p)
    # the whole trace, last sample (E after the final step) included
    assert rel(got["trace"], want["trace"]) <= TOL64
    assert rel(got["trace"][:, -1], want["trace"][:, -1]) <= TOL64
    assert rel(got["dft"], want["dft"]) <= TOL64
    assert rel(got["d"], want["d"]) <= TOL64
    assert rel(got["b"][:-1], want["b"][:-1]) <= TOL64


@pytest.mark.parametrize("beta", [-0.3, 0.3])
@pytest.mark.parametrize("C,T,G,K", [(12, 24, 1, 0), (8, 64, 4, 16), (8, 32, 4, 8)])
def test_grid_end_at_every_owned_position(P, beta, C, T, G, K):
    """Grids whose last node nz-1 falls on every lane position around the
    edges of the owned regions (a sweep of nz), so some run has it as the
    first owned cell of a tile or wave: the end condition there reads the
    cell to its left.  Runs that fit one tile take whole-grid tiles; the
    larger ones (from about 1340 cells) cross ordinary tile and wave edges."""
    probs = []
    for nz in (list(range(340, 470)) + list(range(650, 700)) + list(range(800, 830)) +
               list(range(1340, 1372)) + list(range(2036, 2056)) + list(range(2260, 2284))):
        p = W.small_case(nz, 2 * T, beta, structure="random", seed=nz)
        d, b = W.random_fields(nz, seed=nz + 3)
        probs.append(p.replace(init_d=d, init_b=b,
                               probes=np.array([nz - 3, nz - 2, nz - 1])))
    with P.Batch(probs, cells_per_lane=C, block_steps=T, tile_waves=G,
                 exchange_steps=K, use_graph=0) as bt:
        bt.run()
        res = bt.collect()
    for p, got in zip(probs, res):
        want = oracle.solve(p)
        for k in ("trace", "d"):
            assert rel(got[k], want[k]) <= TOL64, (p.nz, k)
        assert rel(got["b"][:-1], want["b"][:-1]) <= TOL64, p.nz


# One tile holding a whole open grid needs no field halo for its block
# depth; its upwind side holds the block's profile moves (ceil(|beta S| T)
# + 1 cells) plus two ghost cells, the other side one lane.  Here |beta S|
# = 0.15: one wave at C = 8, T = 256 holds (64 - 6 - 1) x 8 = 456 cells; a
# 4-wave tile at C = 12, K = 8, T = 256 holds (256 - 3 x 3 - 4 - 1) x 12 =
# 2904.  Past the whole-grid capacity at the given depth (496 cells for one
# wave at T = 24, 2940 for the 4-wave tile at T = 48) the usual halos apply.
@pytest.mark.parametrize("nz,C,G,T", [(456, 8, 1, 256), (497, 8, 1, 24), (300, 8, 1, 256),
                                      (2904, 12, 4, 256), (2941, 12, 4, 48),
                                      (2000, 12, 4, 200)])
@pytest.mark.parametrize("beta", [0.3, -0.3])
def test_whole_grid_tiles_any_block_depth(P, nz, C, G, T, beta):
    probs = []
    for i, (kind, abc, window) in enumerate([
            (W.MODULATION, W.ABC_MUR1, None),
            (W.MODULATION, W.ABC_PEC, None),
            (W.MATTER, W.ABC_MUR1, None),
            (W.MODULATION, W.ABC_MUR1, W.TimeWindow(30.0, 140.5, 1.5, 1.0))]):
        p = W.small_case(nz, 333, beta, kind=kind, structure="crystal", seed=nz + i,
                         abc=abc)
        d, b = W.random_fields(nz, seed=nz + 10 + i)
        p = p.replace(init_d=d, init_b=b,
                      probes=np.array([0, 1, 2, nz // 2, nz - 3, nz - 2, nz - 1]))
        if window is not None:
            p = p.replace(window=window)
        probs.append(p)

    def run(C_, T_, G_):
        with P.Batch(probs, cells_per_lane=C_, block_steps=T_, tile_waves=G_,
                     exchange_steps=8, use_graph=0) as bt:
            bt.run()
            return bt.collect()

    deep = run(C, T, G)
    ref = run(4, 16, 1)       # narrow tiles: no run fits one tile
    for i, (a, b) in enumerate(zip(deep, ref)):
        for k in ("trace", "dft", "d", "b"):
            assert np.array_equal(a[k], b[k]), (nz, i, k)
    for p, got in zip(probs[:2], deep[:2]):
        want = oracle.solve(p)
        assert rel(got["trace"], want["trace"]) <= TOL64
        assert rel(got["d"], want["d"]) <= TOL64



def test_whole_grid_tile_count(P):
    """A run that fits one tile is stepped as one tile per launch (C = 8,
    T = 24, |beta S| = 0.15: capacity 62 lanes x 8 = 496 cells); a larger
    one is split into ordinary tiles ((64 - 7 - 3) x 8 = 432 cells each)."""
    for nz, tiles in ((300, 1), (496, 1), (600, 2)):
        p = W.small_case(nz, 96, 0.3, structure="slab", seed=nz)
        with P.Batch([p], cells_per_lane=8, block_steps=24, tile_waves=1,
                     use_graph=0) as bt:
            st = bt.stats()
        assert st["launches"] == 4 and st["tiles"] == 4 * tiles, (nz, st)
