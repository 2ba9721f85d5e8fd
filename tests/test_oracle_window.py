"""Finite-duration moving modulation in the oracle: a traveling-wave
structure that exists only for t_on <= t < t_off, the uniform background
before and after (the space-time slabs with temporal corners that the
footnote to the transfer-matrix method, App. B.3, says the FDTD scheme
handles and the transfer matrix cannot).  Pinned by reductions to runs
without a window, by the explicit step matrices (test_oracle_pins), and by
the closed form of a temporal interface: D and B continuous across the
switch (footnote to Section 2), which splits a wave of index n1 into a
forward and a backward wave of index n2 with E amplitudes
(r^2 + r)/2 and (r^2 - r)/2, r = n1/n2, for mu = 1."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _same(a, b):
    for k in ("trace", "dft", "d", "b"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("beta", [0.3, -0.25, 0.0])
def test_window_over_all_time_changes_nothing(beta):
    p = W.small_case(500, 700, beta, seed=3, structure="crystal")
    _same(oracle.solve(p), oracle.solve(p.replace(window=W.TimeWindow(-1e9, 1e9, 7.0, 2.0))))


@pytest.mark.parametrize("beta", [0.3, -0.25])
def test_window_closed_before_the_first_step_is_the_background(beta):
    """Off from t = S/4 on: every node time (>= S/2) sees the background,
    exactly as a uniform grid of the background medium."""
    p = W.small_case(400, 300, beta, seed=4, structure="slab")
    win = W.TimeWindow(-1e9, 0.25 * p.courant, 2.25, 1.1)
    bg = p.replace(eps_rest=np.full(400, 2.25), mu_rest=np.full(400, 1.1))
    _same(oracle.solve(p.replace(window=win)), oracle.solve(bg))


def _temporal_interface(n1, n2, lam=80.0, width=200.0, S=0.5, t0=100.0):
    """A forward wave packet (carrier lam cells, Gaussian envelope) in a
    uniform medium of index n1; at t0 the medium becomes n2.  Returns the
    peak |E| of the forward and backward packets once they have separated,
    for a packet of unit peak |E|."""
    Tp = 3.2 * width * n2 + 100.0
    nz = int(2 * (Tp / n2 + 4 * width) + t0 / n1 + 400)
    c0 = nz / 2 - t0 / n1 / 2
    k = np.arange(nz, dtype=float)
    th = 2 * math.pi / lam
    env = lambda z: np.exp(-((z - c0) / width) ** 2)
    e_half = env(k - 0.5 * S / n1) * np.cos(th * k - th / n1 * 0.5 * S)   # t = S/2
    e_zero = env(k + 0.5) * np.cos(th * (k + 0.5))                        # t = 0
    p = W.Problem(nz=nz, steps=int(round((t0 + Tp) / S)), eps_rest=np.full(nz, n1 ** 2),
                  mu_rest=np.ones(nz), courant=S, beta=0.0, src_cell=1,
                  pulse=W.Pulse(amp=0.0), init_d=n1 ** 2 * e_half, init_b=n1 * e_zero,
                  window=W.TimeWindow(-1e30, t0, n2 ** 2, 1.0))
    E = oracle.solve(p)["d"] / n2 ** 2
    T = p.steps * S
    zc = c0 + t0 / n1
    zf, zb = zc + (T - t0) / n2, zc - (T - t0) / n2
    w = int(2.5 * width)
    return (float(np.max(np.abs(E[int(zf) - w:int(zf) + w]))),
            float(np.max(np.abs(E[int(zb) - w:int(zb) + w]))))


@pytest.mark.parametrize("n1,n2", [(1.0, 2.0), (2.0, 1.0), (1.5, 2.5), (3.0, 1.2)])
def test_temporal_interface_amplitudes(n1, n2):
    r = n1 / n2
    fwd, bwd = _temporal_interface(n1, n2)
    assert abs(fwd / (0.5 * (r * r + r)) - 1) < 0.015
    assert abs(bwd / abs(0.5 * (r * r - r)) - 1) < 0.015


def test_temporal_interface_error_shrinks_with_resolution():
    r = 2.0
    coarse = abs(_temporal_interface(2.0, 1.0, lam=80.0)[0] / (0.5 * (r * r + r)) - 1)
    fine = abs(_temporal_interface(2.0, 1.0, lam=160.0, width=400.0)[0] / (0.5 * (r * r + r)) - 1)
    assert fine < 0.5 * coarse


def test_window_rejected_for_moving_matter():
    p = W.small_case(100, 10, 0.3, kind=W.MATTER, seed=1)
    with pytest.raises(ValueError):
        oracle.solve(p.replace(window=W.TimeWindow(0.0, 5.0, 1.0, 1.0)))
