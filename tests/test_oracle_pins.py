"""Pins of the FP64 oracle against what the paper prints and what
mathematics fixes (no GPU).

Each test names the passage it rests on.  Together they are chosen so that
a dropped term, a wrong sign, a wrong offset or time level, or a swapped
Table 1 column in the oracle fails at least one of them.
"""
import cmath
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import stability as st

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    vals = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


def _ring(nz, eps, mu, beta, S=0.5, kind=W.MODULATION):
    return W.Problem(nz=nz, steps=0, eps_rest=np.full(nz, eps),
                     mu_rest=np.full(nz, mu), courant=S, beta=beta, kind=kind,
                     src_cell=1, pulse=W.Pulse(amp=0.0), abc=W.ABC_PERIODIC)


def _plane(nz, theta, Dhat, Bhat):
    k = np.arange(nz)
    return Dhat * np.exp(1j * theta * k), Bhat * np.exp(1j * theta * (k + 0.5))


def _complex_run(prob, steps, d0, b0):
    """Run the real oracle on the real and imaginary parts of complex
    initial data and recombine (the scheme is real-linear)."""
    re = oracle.solve(prob, steps=steps, init_d=d0.real, init_b=b0.real)
    im = oracle.solve(prob, steps=steps, init_d=d0.imag, init_b=b0.imag)
    return {k: re[k] + 1j * im[k] for k in ("d", "b", "es", "hs")}


# ---------------------------------------------------------------------------
# P1: the printed worked example of Section 5
# ---------------------------------------------------------------------------

def test_amplification_matrix_reproduces_printed_example():
    """Section 5, worked example after eq. (16): zeta_+ = 0.925 - 0.33 i,
    zeta_- = 0.917 + 0.23 i, |zeta_+| = 0.98, |zeta_-| = 0.95."""
    g = _golden("stability_example.txt")
    zp, zm = st.zetas(2 * math.pi * g["theta_over_2pi"], g["S"], g["beta"],
                      g["eps"], g["mu"])
    assert abs(zp.real - g["zeta_plus_re"]) < 5e-4
    assert abs(zp.imag - g["zeta_plus_im"]) < 5e-3
    assert abs(zm.real - g["zeta_minus_re"]) < 5e-4
    assert abs(zm.imag - g["zeta_minus_im"]) < 5e-3
    assert abs(abs(zp) - g["abs_zeta_plus"]) < 5e-3
    assert abs(abs(zm) - g["abs_zeta_minus"]) < 5e-3
    # forward (co-moving) wave is less attenuated, as the text says
    assert abs(zp) > abs(zm)


def _appendix_a_matrix(z, theta, S, beta, eps, mu):
    """The 4x4 homogeneous system of App. A (unknowns E*, H*, D, B) with
    A, B, C, D of eq. (ABCD), as printed."""
    s = math.sin(theta / 2.0)
    c = math.cos(theta / 2.0)
    A = 2j * cmath.sqrt(z) * S * s
    Bc = z - 1.0
    Cc = 2j * S * cmath.exp(-0.5j * theta) * s
    Dc = c / cmath.sqrt(z)
    return np.array([
        [A, 0, 0, Bc + beta * Cc],
        [0, A, Bc + beta * Cc, 0],
        [-eps, 0, 1, -eps * beta * Dc * cmath.exp(-1j * theta)],
        [0, -mu, -mu * beta * Dc, 1]], dtype=complex)


@pytest.mark.parametrize("S,beta,eps,mu,theta", [
    (0.5, 0.3, 4.0, 1.0, 2 * math.pi / 5),
    (0.2, 0.1, 2.0, 1.5, 0.7),
    (0.5, 0.45, 1.0, 1.0, 2.9),
])
def test_appendix_a_system_singular_at_eigenvalues(S, beta, eps, mu, theta):
    """App. A: det of the printed 4x4 system vanishes at both roots."""
    for z in np.linalg.eigvals(st.amplification_matrix(theta, S, beta, eps, mu)):
        M = _appendix_a_matrix(z, theta, S, beta, eps, mu)
        scale = np.prod(np.linalg.norm(M, axis=1))
        assert abs(np.linalg.det(M)) < 1e-12 * scale


@pytest.mark.parametrize("S,beta,eps", [(0.5, 0.3, 4.0), (0.2, 0.05, 9.0),
                                        (0.4, 0.6, 1.5)])
def test_printed_linear_coefficient_is_minus_trace(S, beta, eps):
    """App. A, eq. (zeta_polynom): the printed zeta^1 coefficient equals
    -trace G for v > 0 at every theta."""
    n2 = eps
    for theta in np.linspace(0.1, 3.0, 7):
        G = st.amplification_matrix(theta, S, beta, eps, 1.0)
        c1 = (4 * S * S - n2 * (4 - 3 * beta * S)
              - 4 * S * (S + n2 * beta) * math.cos(theta)) / (2 * n2) \
            + S * beta / 2 * (math.cos(2 * theta) + 2j * math.sin(theta)
                              - 1j * math.sin(2 * theta))
        assert abs(c1 + np.trace(G)) < 1e-13


@pytest.mark.parametrize("beta", [0.3, -0.3, 0.0, 0.55])
def test_determinant_closed_form(beta):
    """det G = [1 - 2 |beta| S sin^2(th/2)] [1 + 2 |beta| S e^{-+i th}
    sin^2(th/2)] (upper sign for v >= 0), independent of eps and mu: our
    reading of the garbled constant term of eq. (zeta_polynom); it is 1 at
    v = 0, as for the Yee scheme."""
    S = 0.5
    for eps, mu in ((4.0, 1.0), (1.7, 2.2)):
        for th in np.linspace(0.05, math.pi, 9):
            s2 = math.sin(th / 2) ** 2
            ph = cmath.exp(-1j * th) if beta >= 0 else cmath.exp(1j * th)
            b = abs(beta)
            want = (1 - 2 * b * S * s2) * (1 + 2 * b * S * ph * s2)
            got = np.linalg.det(st.amplification_matrix(th, S, beta, eps, mu))
            assert abs(got - want) < 1e-14


@pytest.mark.parametrize("which,steps", [(0, 200), (1, 40)])
def test_stepper_multiplies_eigenmode_by_zeta(which, steps):
    """P1 on the stepper itself: on a ring the eigenmode of G(2 pi/5) at
    the worked example's parameters is multiplied by zeta each step."""
    S, beta, eps, theta, nz = 0.5, 0.3, 4.0, 2 * math.pi / 5, 20
    z, v = st.eigenmode(theta, S, beta, eps, 1.0, which)
    d0, b0 = _plane(nz, theta, v[0], v[1])
    out = _complex_run(_ring(nz, eps, 1.0, beta, S), steps, d0, b0)
    want_d = z ** steps * d0
    want_b = z ** steps * b0
    scale = abs(z) ** steps
    assert np.max(np.abs(out["d"] - want_d)) < 1e-12 * scale
    assert np.max(np.abs(out["b"] - want_b)) < 1e-12 * scale


def test_stepper_matter_eigenmode():
    """Same for moving matter: the stepper's one-step map equals the
    amplification matrix built from the matter constitutive relations."""
    S, beta, eps, theta, nz = 0.5, 0.5, 6.0, 2 * math.pi * 3 / 16, 16
    for which in (0, 1):
        z, v = st.eigenmode(theta, S, beta, eps, 1.0, which, kind=W.MATTER)
        d0, b0 = _plane(nz, theta, v[0], v[1])
        out = _complex_run(_ring(nz, eps, 1.0, beta, S, W.MATTER), 30, d0, b0)
        assert np.max(np.abs(out["d"] - z ** 30 * d0)) < 1e-12


# ---------------------------------------------------------------------------
# P2: App. A test-field form of each update, one at a time
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("beta", [0.3, -0.35])
def test_single_updates_match_appendix_a(beta):
    """Eqs. (1_reorg)-(4_reorg) with the zeta powers read as explicit time
    levels, for one step from arbitrary (non-eigen) plane-wave data; the
    v < 0 forms follow the same steps with Table 1 column b (App. A says
    they are obtained similarly)."""
    S, eps, mu, nz = 0.4, 2.5, 1.3, 24
    theta = 2 * math.pi * 5 / nz
    rng = np.random.default_rng(1)
    Dh, Bh = rng.normal(size=2) + 1j * rng.normal(size=2)
    d0, b0 = _plane(nz, theta, Dh, Bh)
    prob = _ring(nz, eps, mu, beta, S)
    st0 = _complex_run(prob, 0, d0, b0)
    st1 = _complex_run(prob, 1, d0, b0)
    ph_e = np.exp(1j * theta * np.arange(nz))
    ph_h = np.exp(1j * theta * (np.arange(nz) + 0.5))
    E_half = st0["es"] / ph_e
    D_half = d0 / ph_e
    B_0 = b0 / ph_h
    B_1 = st1["b"] / ph_h
    H_1 = st1["hs"] / ph_h
    D_3h = st1["d"] / ph_e
    E_3h = st1["es"] / ph_e
    s, c = math.sin(theta / 2), math.cos(theta / 2)
    up = cmath.exp(-0.5j * theta) if beta >= 0 else cmath.exp(0.5j * theta)
    bb = cmath.exp(-1j * theta) if beta >= 0 else cmath.exp(1j * theta)
    tol = 1e-13 * (abs(Dh) + abs(Bh))
    # (1_reorg): Faraday
    r1 = E_half * 2j * S * s + B_1 - B_0 + beta * up * 2j * S * s * B_0
    # (2_reorg): Ampere
    r2 = D_3h - D_half + 2j * S * beta * up * s * D_half + H_1 * 2j * S * s
    # (3_reorg): E* constitutive relation (at n+1/2 and at the start)
    r3 = D_3h - eps * E_3h - eps * beta * B_1 * bb * c
    r3b = D_half - eps * E_half - eps * beta * B_0 * bb * c
    # (4_reorg): H* constitutive relation
    r4 = B_1 - mu * H_1 - mu * beta * D_half * c
    for r in (r1, r2, r3, r3b, r4):
        assert np.max(np.abs(r)) < tol


# ---------------------------------------------------------------------------
# P3: v = 0 is the standard Yee scheme
# ---------------------------------------------------------------------------

def _textbook_yee(p, steps):
    """Standard 1D Yee scheme (D/E at integer nodes, B/H between), written
    without any velocity terms, with the same source and first-order Mur
    ends."""
    nz, S = p.nz, p.courant
    eps, mu = p.eps_rest, p.mu_rest
    D = np.zeros(nz)
    B = np.zeros(nz - 1)
    E = D / eps
    trace = np.zeros((len(p.probes), steps))
    for n in range(1, steps + 1):
        B = B - S * (E[1:] - E[:-1])
        H = B / mu[:-1]
        Dn = D.copy()
        Dn[1:-1] = D[1:-1] - S * (H[1:] - H[:-1])
        t = n * S
        if t <= p.pulse.t_off:
            u = (t - p.pulse.t0) / p.pulse.tau
            Dn[p.src_cell] += p.pulse.amp * math.sin(
                p.pulse.omega * (t - p.pulse.t0) + p.pulse.phase) * math.exp(-u * u)
        nL = math.sqrt(eps[0] * mu[0])
        nR = math.sqrt(eps[-1] * mu[-2])
        cL = (S * (1.0 / nL) - 1.0) / (S * (1.0 / nL) + 1.0)
        cR = (S * (1.0 / nR) - 1.0) / (S * (1.0 / nR) + 1.0)
        Dn[0] = D[1] + cL * (Dn[1] - D[0])
        Dn[-1] = D[-2] + cR * (Dn[-2] - D[-1])
        D = Dn
        E = D / eps
        trace[:, n - 1] = E[p.probes]
    return D, B, trace


@pytest.mark.parametrize("structure", ["uniform", "random"])
def test_zero_velocity_is_standard_yee(structure):
    """Section 3: at v = 0 the boundary conditions reduce to the
    stationary ones and the scheme is the usual Yee scheme (Section 4,
    'discretized in the usual fashion').  Bitwise."""
    p = W.small_case(96, 300, 0.0, structure=structure, seed=3)
    if structure == "uniform":
        p = p.replace(mu_rest=np.ones(p.nz))
    out = oracle.solve(p)
    D, B, trace = _textbook_yee(p, p.steps)
    assert np.array_equal(out["d"], D)
    assert np.array_equal(out["b"][:-1], B)
    assert np.array_equal(out["trace"], trace)


@pytest.mark.parametrize("n", [1.0, 1.7, 3.0])
def test_zero_velocity_amplification_is_yee(n):
    """At v = 0 both roots are the textbook Yee factors, |zeta| = 1."""
    S = 0.5
    for th in np.linspace(0.1, math.pi, 6):
        zp, zm = st.zetas(th, S, 0.0, n * n, 1.0)
        want = st.yee_zeta(th, S, n)
        assert abs(zp - want) < 1e-13
        assert abs(zm - want.conjugate()) < 1e-13


# ---------------------------------------------------------------------------
# P4: the v < 0 column is the mirror image of the v > 0 column
# ---------------------------------------------------------------------------

def _mirror(p):
    nz = p.nz
    mu = p.mu_rest.copy()
    mu[:nz - 1] = p.mu_rest[nz - 2::-1]
    return p.replace(beta=-p.beta, eps_rest=p.eps_rest[::-1].copy(), mu_rest=mu,
                     src_cell=nz - 1 - p.src_cell,
                     probes=(nz - 1 - p.probes))


@pytest.mark.parametrize("beta,seed", [(0.3, 0), (0.25, 5), (0.5, 2)])
def test_negative_velocity_is_mirror_image(beta, seed):
    """App. A: the v < 0 scheme behaves identically to the v > 0 scheme
    (same characteristic polynomial).  On the grid: running at -v on the
    mirrored structure gives the mirrored fields, D(k) -> D(nz-1-k),
    B(j) -> -B(nz-2-j), bit for bit; the probes see the same E."""
    p = W.small_case(80, 260, beta, seed=seed, structure="random")
    q = _mirror(p)
    a = oracle.solve(p)
    b = oracle.solve(q)
    nz = p.nz
    assert np.array_equal(b["d"], a["d"][::-1])
    assert np.array_equal(b["b"][:nz - 1], -a["b"][nz - 2::-1])
    assert np.array_equal(b["trace"], a["trace"])


def test_stability_symmetric_in_velocity_sign():
    """App. A: the polynomial is the same for v < 0."""
    for beta in (0.1, 0.3, 0.6):
        for eps in (1.0, 2.0, 4.0):
            assert abs(st.max_growth(0.5, beta, eps) -
                       st.max_growth(0.5, -beta, eps)) < 1e-12


# ---------------------------------------------------------------------------
# P5: brute force -- the step as an explicit matrix
# ---------------------------------------------------------------------------

def _step_matrix(p, n):
    """Assemble one time step as an affine map x -> M x + s on the state
    x = (D[0..nz), B[0..nz-1)), reading the stencil of eq. (10) and Table 1
    as a list of (row, column, weight) entries."""
    nz, S, beta = p.nz, p.courant, p.beta
    nh = nz - 1
    bS = beta * S
    col_a = beta >= 0
    mE_prev = int(np.rint(bS * (n - 0.5)))
    mH = int(np.rint(bS * n))
    mE = int(np.rint(bS * (n + 0.5)))
    win = getattr(p, "window", None)

    def on(tau):             # the moving profile exists at time tau S
        return win is None or win.t_on <= tau * S < win.t_off

    eps_at = lambda k, m, tau: (p.eps_rest[min(max(k - m, 0), nz - 1)]
                                if on(tau) else win.eps_bg)
    mu_at = lambda j, m, tau: (p.mu_rest[min(max(j - m, 0), nz - 2)]
                               if on(tau) else win.mu_bg)
    N = nz + nh
    iD = lambda k: k
    iB = lambda j: nz + j

    def bbar_row(k):
        row = np.zeros(N)
        pair = (k - 1, k - 2) if col_a else (k + 1, k)
        for j in pair:       # off the grid: the edge value
            row[iB(min(max(j, 0), nh - 1))] += 0.5
        return row

    Es = np.zeros((nz, N))
    for k in range(nz):
        Es[k, iD(k)] = 1.0 / eps_at(k, mE_prev, n - 0.5)
        Es[k] -= beta * bbar_row(k)
    Bn = np.zeros((nh, N))
    for j in range(nh):
        Bn[j, iB(j)] += 1.0
        Bn[j] -= S * (Es[j + 1] - Es[j])
        if col_a:
            Bn[j, iB(j)] -= bS
            Bn[j, iB(max(j - 1, 0))] += bS
        else:
            Bn[j, iB(j)] += bS
            Bn[j, iB(min(j + 1, nh - 1))] -= bS
    Hs = np.zeros((nh, N))
    for j in range(nh):
        Hs[j] = Bn[j] / mu_at(j, mH, n)
        Hs[j, iD(j)] -= 0.5 * beta
        Hs[j, iD(j + 1)] -= 0.5 * beta
    Dn = np.zeros((nz, N))
    for k in range(1, nz - 1):
        Dn[k, iD(k)] += 1.0
        Dn[k] -= S * (Hs[k] - Hs[k - 1])
        if col_a:
            Dn[k, iD(k)] -= bS
            Dn[k, iD(k - 1)] += bS
        else:
            Dn[k, iD(k)] += bS
            Dn[k, iD(k + 1)] -= bS
    s = np.zeros(N)
    t = n * S
    if t <= p.pulse.t_off:
        u = (t - p.pulse.t0) / p.pulse.tau
        s[iD(p.src_cell)] = p.pulse.amp * math.sin(
            p.pulse.omega * (t - p.pulse.t0) + p.pulse.phase) * math.exp(-u * u)
    # first-order Mur rows (velocity ignored for a moving modulation)
    nL = math.sqrt(eps_at(0, mE, n + 0.5) * mu_at(0, mE, n + 0.5))
    nR = math.sqrt(eps_at(nz - 1, mE, n + 0.5) * mu_at(nz - 2, mE, n + 0.5))
    cL = (S / nL - 1) / (S / nL + 1)
    cR = (S / nR - 1) / (S / nR + 1)
    sL = s[iD(1)]
    sR = s[iD(nz - 2)]
    Dn[0] = cL * Dn[1]
    Dn[0, iD(1)] += 1.0
    Dn[0, iD(0)] -= cL
    Dn[nz - 1] = cR * Dn[nz - 2]
    Dn[nz - 1, iD(nz - 2)] += 1.0
    Dn[nz - 1, iD(nz - 1)] -= cR
    s[iD(0)] += cL * sL
    s[iD(nz - 1)] += cR * sR
    M = np.vstack([Dn, Bn])
    return M, s


@pytest.mark.parametrize("beta,nz,window", [
    (0.35, 12, None), (-0.4, 16, None), (0.0, 9, None),
    (0.35, 12, W.TimeWindow(3.1, 14.9, 2.5, 1.3)),
    (-0.4, 16, W.TimeWindow(-1.0, 7.25, 1.7, 1.0)),
    (0.3, 11, W.TimeWindow(12.0, 1e9, 3.0, 1.2))])
def test_brute_force_matrix(beta, nz, window):
    """The whole stepper (interior stencil, ghosts, source, Mur ends,
    moving profile, a modulation switched on and/or off in time) against
    explicit per-step matrices on tiny grids."""
    p = W.small_case(nz, 50, beta, seed=11, structure="random")
    p = p.replace(src_cell=nz // 2, pulse=W.Pulse(amp=1.0, omega=0.9, t0=4.0,
                                                   tau=3.0, phase=0.3,
                                                   t_off=20.0), window=window)
    rng = np.random.default_rng(7)
    d0 = rng.normal(size=nz)
    b0 = np.zeros(nz)
    b0[:nz - 1] = rng.normal(size=nz - 1)
    x = np.concatenate([d0, b0[:nz - 1]])
    for n in range(1, 51):
        M, s = _step_matrix(p, n)
        x = M @ x + s
        if n in (1, 2, 7, 50):
            out = oracle.solve(p, steps=n, init_d=d0, init_b=b0)
            got = np.concatenate([out["d"], out["b"][:nz - 1]])
            assert np.max(np.abs(got - x)) <= 1e-13 * max(1.0, np.max(np.abs(x)))


# ---------------------------------------------------------------------------
# P6: linearity
# ---------------------------------------------------------------------------

def test_linearity():
    """Maxwell's equations and the scheme are linear in the fields and the
    source: run(a s1 + b s2) = a run(s1) + b run(s2)."""
    p = W.small_case(200, 400, 0.3, seed=4, structure="random")
    rng = np.random.default_rng(0)
    d1, d2 = rng.normal(size=(2, p.nz))
    b1, b2 = rng.normal(size=(2, p.nz))
    a, b = 0.7, -1.3
    p1 = p.replace(pulse=W.Pulse(**{**p.pulse.__dict__, "amp": 1.0}))
    p2 = p.replace(pulse=W.Pulse(**{**p.pulse.__dict__, "amp": 0.0}))
    pab = p.replace(pulse=W.Pulse(**{**p.pulse.__dict__, "amp": a}))
    r1 = oracle.solve(p1, init_d=d1, init_b=b1)
    r2 = oracle.solve(p2, init_d=d2, init_b=b2)
    rab = oracle.solve(pab, init_d=a * d1 + b * d2, init_b=a * b1 + b * b2)
    for key in ("d", "b", "trace"):
        want = a * r1[key] + b * r2[key]
        assert np.max(np.abs(rab[key] - want)) < 1e-12 * np.max(np.abs(want))


# ---------------------------------------------------------------------------
# P11: stability thresholds used by the pre-flight
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1.2, 2.0, 3.46])
def test_luminal_threshold(n):
    """The scheme for a moving modulation is stable up to |beta| n = 1
    and unstable beyond (scan of the amplification matrix, Section 5)."""
    for S in (0.5, 0.2):
        for sgn in (1, -1):
            assert st.max_growth(S, sgn * 0.99 / n, n * n) <= 1 + 1e-12
            assert st.max_growth(S, sgn * 1.02 / n, n * n) > 1 + 1e-9


@pytest.mark.parametrize("n,beta", [(1.0, 0.3), (1.5, 0.2), (2.0, 0.4)])
def test_courant_threshold(n, beta):
    """The Courant-type limit S <= n / (1 + n |beta|)."""
    smax = n / (1 + n * beta)
    assert st.max_growth(0.99 * smax, beta, n * n) <= 1 + 1e-12
    assert st.max_growth(1.02 * smax, beta, n * n) > 1 + 1e-6


def test_stepper_bounded_inside_and_grows_outside():
    """The stepper itself: bounded for 2e4 steps at |beta| n = 0.99,
    growing at |beta| n = 1.3 (uniform ring, random initial data)."""
    nz, n = 64, 2.0
    rng = np.random.default_rng(2)
    d0 = rng.normal(size=nz)
    b0 = rng.normal(size=nz)
    inside = oracle.solve(_ring(nz, n * n, 1.0, 0.99 / n), steps=20000,
                          init_d=d0, init_b=b0)
    outside = oracle.solve(_ring(nz, n * n, 1.0, 1.3 / n), steps=20000,
                           init_d=d0, init_b=b0)
    assert np.max(np.abs(inside["d"])) < 10 * np.max(np.abs(d0))
    assert np.max(np.abs(outside["d"])) > 1e3 * np.max(np.abs(d0))


def test_matter_stable_where_modulation_is_not():
    """Moving matter with a ramp to eps' = 6 at beta = 0.5 (beta n' = 1.22)
    is stable with the matter constitutive relations."""
    for eps in (1.0, 2.0, 4.0, 6.0):
        assert st.max_growth(0.5, 0.5, eps, kind=W.MATTER) <= 1 + 1e-12
    assert st.max_growth(0.5, 0.5, 6.0, kind=W.MODULATION) > 1 + 1e-6
