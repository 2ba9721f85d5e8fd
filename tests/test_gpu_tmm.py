"""GPU transfer-matrix sweeps (App. B.3) against the FP64 oracle's
transfer matrix (itself pinned to the closed forms of one interface and one
slab in test_oracle_physics), and the closed forms directly."""
import numpy as np
import pytest

import workloads as W
from oracle import analytic as A

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2304_06586_amd as pkg
    pkg.load_library()
    return pkg


def _oracle(stacks, omegas):
    T = np.zeros((len(stacks), len(omegas)), complex)
    G = np.zeros_like(T)
    for i, s in enumerate(stacks):
        for j, w in enumerate(omegas):
            T[i, j], G[i, j] = A.transfer_matrix(w, list(s.eps), list(s.widths), s.beta,
                                                 None if s.mu is None else list(s.mu))
    return T, G


def _close(got, want, tol):
    err = np.max(np.abs(got - want) / np.maximum(1.0, np.abs(want)))
    assert err < tol, err
    return err


def test_crystal_sweep_against_oracle(P):
    stacks, omegas = W.tmm_crystals(3, 48, nomega=24)
    T, G = P.gfdtd_tmm(stacks, omegas)
    Tw, Gw = _oracle(stacks, omegas)
    print("crystals: T err %.2e, Gamma err %.2e" % (_close(T, Tw, 1e-11), _close(G, Gw, 1e-11)))


def test_random_stacks_with_magnetic_layers_and_both_velocity_signs(P):
    rng = np.random.default_rng(11)
    stacks = []
    for k in range(40):
        N = int(rng.integers(2, 40))
        eps = rng.uniform(1.0, 6.0, size=N)
        mu = rng.uniform(0.5, 2.0, size=N)
        nmax = np.sqrt(np.max(eps * mu))
        beta = float(rng.uniform(-0.95, 0.95)) / nmax
        stacks.append(W.TmmStack(eps=eps, mu=mu, widths=rng.uniform(0.0, 80.0, size=N - 2),
                                 beta=beta))
    omegas = np.linspace(0.01, 1.2, 17)
    T, G = P.gfdtd_tmm(stacks, omegas)
    Tw, Gw = _oracle(stacks, omegas)
    _close(T, Tw, 1e-11)
    _close(G, Gw, 1e-11)


@pytest.mark.parametrize("beta", [0.3, -0.3, 0.0])
def test_single_interface_and_slab_closed_forms(P, beta):
    """Two layers: eq. (coef_interface); three layers: the slab formula."""
    T, G = P.gfdtd_tmm([W.TmmStack(eps=np.array([2.0, 4.0]), widths=np.zeros(0),
                                   beta=beta)], [0.3])
    t21, g121 = A.interface(2.0, 4.0, beta)
    assert abs(T[0, 0] - t21) < 1e-13 and abs(G[0, 0] - g121) < 1e-13
    omegas = np.linspace(0.05, 0.6, 9)
    T, G = P.gfdtd_tmm([W.TmmStack(eps=np.array([1.0, 4.0, 1.0]), widths=np.array([37.0]),
                                   beta=beta)], omegas)
    for j, w in enumerate(omegas):
        ts, gs = A.slab(w, 1.0, 4.0, beta, 37.0)
        assert abs(abs(T[0, j]) - abs(ts)) < 1e-12 and abs(abs(G[0, j]) - abs(gs)) < 1e-12


def test_kernel_time_is_reported(P):
    """gfdtd_tmm_kernel_ms gives the device time of the kernel alone: after
    a call it is positive and below the call's wall time."""
    import time
    stacks, omegas = W.tmm_crystals(5, 256, nomega=64)
    t0 = time.perf_counter()
    P.gfdtd_tmm(stacks, omegas)
    wall_ms = (time.perf_counter() - t0) * 1e3
    k = P.gfdtd_tmm_kernel_ms()
    print(f"transfer-matrix call {wall_ms:.3f} ms, kernel {k:.3f} ms")
    assert 0.0 < k < wall_ms
