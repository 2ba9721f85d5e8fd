"""The dependency cone of the scheme, measured on the FP64 oracle: a single
perturbed D or B node spreads, per step, by at most 2 cells downstream (+1
in the first step) and 1 upstream for column a (v >= 0), and by 2 and 1
the other way for column b.  The tiled kernels size their halos from
exactly this reach (eq. (10) with the Table 1 terms): a cell of a tile
then depends on at most 2T + 1 cells on its upwind side and T on the
other after a block of T steps, and the halo adds one cell for the B
average a probe's E reads (and, for column b, the end condition at nz-1
reading nz-2).  Checked here on the method itself, independently of any
GPU code; the bound is attained."""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads as W


def _spread(beta, which, n):
    base = W.small_case(200, n, beta, structure="random", seed=1)
    base = base.replace(pulse=dataclasses.replace(base.pulse, amp=0.0))
    zero = np.zeros(200)
    pert = zero.copy()
    pert[100] = 1.0
    p = base.replace(init_d=pert if which == "d" else zero,
                     init_b=pert if which == "b" else zero)
    r = oracle.solve(p)
    cells = np.concatenate([np.nonzero(r["d"])[0], np.nonzero(r["b"][:-1])[0]])
    return int(cells.min()) - 100, int(cells.max()) - 100


@pytest.mark.parametrize("beta", [0.3, -0.3])
def test_dependency_cone_matches_halo_reach(beta):
    for n in (1, 2, 3, 5, 8, 13):
        lo = min(_spread(beta, w, n)[0] for w in ("d", "b"))
        hi = max(_spread(beta, w, n)[1] for w in ("d", "b"))
        if beta > 0:
            # a node influences 2n+1 cells downstream (so depends on 2n+1
            # upwind) and n upstream
            assert (lo, hi) == (-n, 2 * n + 1), (n, lo, hi)
        else:
            assert (lo, hi) == (-2 * n, n), (n, lo, hi)
