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
    cell to its left."""
    probs = []
    for nz in list(range(340, 470)) + list(range(650, 700)) + list(range(800, 830)):
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
