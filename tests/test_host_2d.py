"""Host-side tests of the 2D C-ABI (no GPU): validation, workspace size and
the stability pre-flight.

The pre-flight evaluates, per medium, the one-step amplification matrix of
a plane wave on a 64 x 128 grid of (kx, kz) and reports the largest
eigenvalue modulus.  Here the same matrices are read off the FP64 oracle:
on a 128 x 128 doubly periodic grid in a uniform medium, one step from a
unit impulse in each of the three unknowns gives, after a 2D FFT, the
columns of G(kx, kz) for every grid mode at once.  Those modes are exactly
the pre-flight's sample points (kx = pi jx / 64, kz = pi jz / 64), so the
largest modulus must agree to rounding."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import stepper2d


@pytest.fixture(scope="module")
def P():
    import os
    import paper_2304_06586_amd as pkg
    from paper_2304_06586_amd import gfdtd
    if not os.path.exists(gfdtd.LIB_PATH):
        from paper_2304_06586_amd import build
        build.build()
    pkg.load_library()
    return pkg


def _oracle_growth(pol, eps, mu, S, beta, n=128):
    names = ("d", "b", "c")
    G = np.zeros((n, n, 3, 3), dtype=complex)
    for col, f in enumerate(names):
        init = {"init_" + g: np.zeros((n, n)) for g in names}
        init["init_" + f][0, 0] = 1.0
        p = W.Problem2D(pol=pol, nx=n, nz=n, steps=1, eps_rest=np.full(n, eps),
                        mu_rest=np.full(n, mu), courant=S, beta=beta,
                        pulse=W.Pulse(amp=0.0), abc=W.ABC_PERIODIC, **init)
        o = stepper2d.solve(p)
        for row, g in enumerate(names):
            # response to an impulse at the origin: G(k) = sum_r h(r) e^{-i k r}
            G[:, :, row, col] = np.fft.fft2(o[g])
    lam = np.linalg.eigvals(G.reshape(-1, 3, 3))
    return float(np.max(np.abs(lam)))


def _problem(pol, eps, mu, S, beta, **kw):
    nz = 64
    return W.Problem2D(pol=pol, nx=8, nz=nz, steps=10, eps_rest=np.full(nz, eps),
                       mu_rest=np.full(nz, mu), courant=S, beta=beta, src_row=20,
                       pulse=W.Pulse(amp=0.0), flags=W.FLAG_ALLOW_UNSTABLE, **kw)


@pytest.mark.parametrize("pol", [W.TE, W.TM])
@pytest.mark.parametrize("eps,mu,S,beta", [
    (1.0, 1.0, 0.5, 0.0),        # plain Yee, stable
    (1.0, 1.0, 0.75, 0.0),       # above the 2D Courant limit 1/sqrt(2)
    (2.25, 1.0, 0.5, 0.4),       # moving modulation, stable
    (4.0, 1.0, 0.5, -0.45),
    (1.0, 1.0, 0.6, 0.7),        # fast modulation in vacuum
    (2.0, 1.3, 0.7, 0.5),
])
def test_preflight_matches_oracle_amplification(P, pol, eps, mu, S, beta):
    want = _oracle_growth(pol, eps, mu, S, beta)
    got = P.gfdtd2d_check(_problem(pol, eps, mu, S, beta), steps=0)
    print(f"growth oracle {want:.15f} library {got:.15f}")
    assert abs(got - want) < 1e-10 * max(1.0, want)


def test_preflight_rejects_above_the_2d_courant_limit(P):
    p = _problem(W.TE, 1.0, 1.0, 0.75, 0.0)
    p.flags = 0
    with pytest.raises(P.GfdtdError) as e:
        P.gfdtd2d_check(p, steps=10)          # 2^10 > 10
    assert e.value.status == 2
    # the 1D scheme at the same S is stable
    q = W.Problem(nz=64, steps=10, eps_rest=np.ones(64), mu_rest=np.ones(64),
                  courant=0.75, src_cell=20, pulse=W.Pulse(amp=0.0))
    assert P.gfdtd_check(q) <= 1.0 + 1e-9


def test_run_growth_bound(P):
    """A moving modulation grows its worst oblique mode slightly every
    step: accepted while g^steps <= 10, rejected beyond."""
    p = _problem(W.TE, 1.0, 1.0, 0.5, 0.3)
    p.flags = 0
    g = P.gfdtd2d_check(p, steps=0)
    assert g > 1.0 + 1e-4
    n_ok = int(math.log(10.0) / math.log(g))
    P.gfdtd2d_check(p, steps=n_ok)
    with pytest.raises(P.GfdtdError) as e:
        P.gfdtd2d_check(p, steps=n_ok + 2)
    assert e.value.status == 2


def test_2d_workloads_pass_the_preflight(P):
    for pol in (W.TE, W.TM):
        for seed in range(6):
            p = W.slab_run_2d(seed, pol=pol)
            g = P.gfdtd2d_check(p)
            assert g ** p.steps <= 10.0
        for beta in (0.5, -0.5):
            P.gfdtd2d_check(W.small_case_2d(16, 300, 800, beta, pol=pol))


@pytest.mark.parametrize("field,value,msg", [
    ("pol", 7, "polarization"),
    ("nx", 0, "nx"),
    ("nz", 4, "nz"),
    ("src_row", 0, "src_row"),
    ("abc", 9, "end condition"),
    ("courant", -1.0, "Courant"),
    ("beta", 1.0, "beta"),
])
def test_validation(P, field, value, msg):
    p = W.small_case_2d(8, 64, 10, 0.2)
    setattr(p, field, value)
    with pytest.raises(P.GfdtdError) as e:
        P.gfdtd2d_check(p)
    assert e.value.status == 1 and msg in e.value.message


def test_probe_outside_grid_is_rejected(P):
    p = W.small_case_2d(8, 64, 10, 0.2)
    p.probe_x = np.array([8])
    p.probe_z = np.array([3])
    with pytest.raises(P.GfdtdError) as e:
        P.gfdtd2d_check(p)
    assert "outside the grid" in e.value.message


def test_time_window_flag_is_unsupported(P):
    p = W.small_case_2d(8, 64, 10, 0.2)
    p.flags = W.FLAG_RECORD_TRACE | 8
    with pytest.raises(P.GfdtdError) as e:
        P.gfdtd2d_check(p)
    assert e.value.status == 7


def test_workspace_bytes_scale_with_the_grid(P):
    a = P.gfdtd2d_workspace_bytes(W.small_case_2d(64, 1000, 100, 0.2, precision=W.F32))
    b = P.gfdtd2d_workspace_bytes(W.small_case_2d(64, 1000, 100, 0.2, precision=W.F64))
    # six field arrays of nx x ld (ld = nz rounded up to 64) dominate
    fa, fb = 6 * 64 * 1024 * 4, 6 * 64 * 1024 * 8
    assert fa < a < fa + 200_000
    assert fb < b < fb + 200_000


def test_execution_options_are_validated_before_the_device(P):
    """gfdtd2d_prepare checks its options before touching the device: a bad
    option is E_INVALID, a good one then fails on the missing workspace."""
    import ctypes as C
    from paper_2304_06586_amd import gfdtd as G
    lib = G.load_library()

    def prepare(p, cells=0, cols=0, steps_per_launch=0):
        m = G._Marshalled2D(p)
        e = G.gfdtd2d_exec()
        e.struct_size = C.sizeof(G.gfdtd2d_exec)
        e.cells_per_lane, e.columns_per_wave, e.block_steps = cells, cols, steps_per_launch
        h = C.c_void_p(None)
        return lib.gfdtd2d_prepare(C.byref(m.struct), m.steps, C.byref(e), None, 0, None,
                                   C.byref(h))
    p32 = W.small_case_2d(8, 64, 10, 0.2, precision=W.F32)
    p64 = W.small_case_2d(8, 64, 10, 0.2, precision=W.F64)
    ring = W.small_case_2d(8, 64, 10, 0.2, precision=W.F32, abc=W.ABC_PERIODIC)
    assert prepare(p32, steps_per_launch=5) == 1
    assert prepare(p32, cells=8, steps_per_launch=2) == 1     # wide lanes: one step
    assert prepare(p64, cells=4, steps_per_launch=4) == 1
    assert prepare(ring, steps_per_launch=2) == 1             # rings: one step
    assert prepare(p32, cells=3) == 1
    assert prepare(p64, cells=8) == 1
    for ok in ((p32, 4, 0, 4), (p32, 2, 0, 2), (p64, 2, 0, 2), (ring, 0, 0, 1), (p32, 8, 16, 1)):
        assert prepare(ok[0], ok[1], ok[2], ok[3]) == 3        # E_NOMEM: no workspace
