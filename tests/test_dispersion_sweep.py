"""The stability / dispersion sweep on the CPU: plane waves on uniform
rings stepped by the FP64 oracle, with the amplification factors read off
the final fields by paper_2304_06586_amd.dispersion, against the von
Neumann matrix G (Section 5, App. A) and the values the paper prints for
its worked example (Section 5, the setting of Fig. 4)."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import stability as st
from paper_2304_06586_amd import dispersion as DS


def _oracle_growth(points, steps):
    res = [oracle.solve(r) for r in W.dispersion_runs(points, steps)]
    return DS.sweep_growth(points, res, steps)


def test_inputs_are_single_plane_waves():
    """Each point's two runs start from a cosine whose theta component is
    nz/2 in D (first run) or in B at the half-integer nodes (second run),
    and nothing at other wavenumbers of the ring."""
    pt = W.DispersionPoint(0.5, 0.3, 4.0, nz=24, m=5)
    rd, rb = W.dispersion_runs([pt], 7)
    assert rd.abc == rb.abc == W.ABC_PERIODIC and rd.pulse.amp == 0.0
    assert np.all(rd.init_b == 0) and np.all(rb.init_d == 0)
    spec = np.fft.fft(rd.init_d)
    assert abs(spec[5] - 12.0) < 1e-12 and abs(spec[19] - 12.0) < 1e-12
    spec[[5, 19]] = 0
    assert np.max(np.abs(spec)) < 1e-12
    k = np.arange(24)
    assert abs(rb.init_b @ np.exp(-1j * pt.theta * (k + 0.5)) - 12.0) < 1e-12


def test_sweep_recovers_the_amplification_factors():
    """Oracle-stepped rings give |zeta_+|, |zeta_-| of G to rounding, over
    the Fig. 4 setting and a seeded random sweep of (S, beta, eps, N_lambda)."""
    pts = W.fig4_points(max_nz=24) + W.dispersion_points(3, 40, max_nz=64)
    got = _oracle_growth(pts, 12)
    for p, (f, b) in zip(pts, got):
        zp, zm = st.zetas(p.theta, p.courant, p.beta, p.eps, p.mu, p.kind)
        assert abs(f - abs(zp)) < 1e-12 and abs(b - abs(zm)) < 1e-12, p


def test_worked_example_printed_values():
    """Section 5: S = 0.5, beta = 0.3, eps = 4, k_z dz = 2 pi / 5 gives
    |zeta_+| = 0.98 and |zeta_-| = 0.95 (the co-moving wave is less
    attenuated).  N_lambda = 5 on a ring of 10 cells, 40 steps."""
    pt = W.DispersionPoint(0.5, 0.3, 4.0, nz=10, m=2)
    (f, b), = _oracle_growth([pt], 40)
    assert round(f, 2) == 0.98 and round(b, 2) == 0.95
    alpha = DS.attenuation_rate([f, b], 0.5)
    assert alpha[0] > alpha[1] and np.all(alpha < 0)


@pytest.mark.parametrize("beta", [0.3, -0.3])
def test_co_moving_wave_is_less_attenuated(beta):
    """Fig. 4: for v > 0 the co-moving (forward) wave is attenuated less
    than the contra-moving one at every meshing density; for v < 0 the
    roles swap (the mirrored stencil, Table 1 column b)."""
    pts = [W.DispersionPoint(0.5, beta, 4.0, p.nz, p.m)
           for p in W.fig4_points(max_nz=20)]
    got = _oracle_growth(pts, 10)
    co = got[:, 0] if beta > 0 else got[:, 1]
    contra = got[:, 1] if beta > 0 else got[:, 0]
    assert np.all(co >= contra - 1e-12)
    # attenuation vanishes as the mesh is refined (consistency)
    fine = W.DispersionPoint(0.5, beta, 4.0, nz=400, m=1)
    (f, b), = _oracle_growth([fine], 10)
    assert 1.0 - min(f, b) < 1e-4
    assert max(f, b) <= 1.0 + 1e-12


def test_sweep_points_pass_the_preflight():
    """The random sweep's redraw rule keeps every point inside the stable
    region the library's pre-flight accepts."""
    import paper_2304_06586_amd as P
    P.load_library()
    for r in W.dispersion_runs(W.dispersion_points(11, 200), 4):
        g = P.gfdtd_check(r)
        assert g <= 1.0 + 1e-9 and math.isfinite(g)


def test_unresolvable_weak_mode_is_reported_not_guessed():
    """A point (v < 0) whose forward, contra-moving mode decays ~10x faster
    per step than the backward one: after 16 steps the modes differ by
    1e-16 and the weaker one is NaN; after 4 steps both are read
    correctly."""
    pt = W.DispersionPoint(0.9482223966030298, -0.47262393383077583,
                           3.532405267910378, nz=119, m=52)
    zp, zm = (abs(z) for z in st.zetas(pt.theta, pt.courant, pt.beta, pt.eps))
    (f16, b16), = _oracle_growth([pt], 16)
    assert np.isnan(f16) and abs(b16 - zm) < 1e-12
    (f4, b4), = _oracle_growth([pt], 4)
    assert abs(f4 - zp) < 1e-9 and abs(b4 - zm) < 1e-12
