"""Pins of the 2D oracle (TE and TM, stratified moving modulation; no GPU).

The paper discretizes the 1D problem only (Section 4); the 2D oracle reads
the mixed-field equations (6) with the star fields of eq. (2) for fields
independent of y and interfaces normal to v (Section 3, eq. (3)), putting
the Table 1 stencils on every z-difference of a velocity term and the Yee
differences on the curls.  Its pins:

1. Reduction to the 1D scheme.  With an x-uniform source and initial state
   every column carries the 1D pair of eq. (10): TE as (D_y, -B_x), TM as
   (D_x, B_y), and B_z / D_z stay zero.  The 2D fields and probe traces
   equal the (pinned) 1D oracle's bit for bit, for both signs of v, on open,
   PEC and ring ends.
2. v = 0 is the textbook 2D Yee scheme in (D, B) form, written here with
   whole-array numpy shifts and each node's material read from the rest
   cell that contains it: equal bit for bit on a stratified medium.
3. The discrete Yee plane-wave eigenmode (v = 0, uniform medium, doubly
   periodic) in closed form: every field after N steps equals the
   analytic one, with sin^2(w S/2) = S^2 (sin^2(kx/2) + sin^2(kz/2))/(eps
   mu), to 1e-12.  A wrong sign, index or staggering of any curl term, in
   x or z, fails it.
4. Divergence.  The discrete divergence of B (TE) or D (TM) obeys, exactly,
   div^{n} = div^{n-1} - beta S d_up(div^{n-1}), the Table 1 upwind
   difference along z (column a for v >= 0, b for v < 0), because the
   curls are divergence-free on the Yee lattice and the dynamic terms
   commute with the x-difference on a z-ring.  The oracle's divergence
   after N steps from a random state equals that closed form (FFT symbol)
   on a moving stratified medium.  A dropped or mis-directed dynamic term on
   either component, or a wrong x-neighbour in a curl, fails it.
5. Dispersion in a moving uniform modulation.  A moving modulation of a
   uniform medium is no modulation: the physical waves travel at 1/n in
   every direction.  The one-step amplification matrix of an oblique
   Fourier mode, read off the oracle, has the divergence eigenvalue of pin
   4 exactly and a physical pair whose phase speed converges to 1/n as the
   grid is refined at fixed physical wavevector.

Each pin also runs on variants of the oracle source with one planted
mistake, compiled here, and must fail there.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import build as obuild
from oracle import stepper, stepper2d

S = 0.5


# ------------------------------------------------------ 1. 1D reduction

def _pair(pol, beta, abc, seed, init):
    rng = np.random.default_rng(seed)
    nz, nx, steps = 160, 3, 260
    eps = rng.uniform(1.0, 3.0, size=nz)
    mu = rng.uniform(1.0, 1.4, size=nz)
    pulse = W.Pulse(amp=1.0, omega=2 * math.pi / 20.0, t0=40.0, tau=12.0,
                    phase=float(rng.uniform(0, 6.28)), t_off=80.0)
    probes = np.array([0, 7, 80, nz - 1])
    om = W.default_omegas(pulse.omega, 6)
    d0 = b0 = None
    if init:
        d0, b0 = W.random_fields(nz, seed + 1)
        if abc != W.ABC_PERIODIC:
            b0[-1] = 0.0
    p1 = W.Problem(nz=nz, steps=steps, eps_rest=eps, mu_rest=mu, courant=S,
                   beta=beta, src_cell=20, pulse=pulse, probes=probes,
                   omegas=om, abc=abc, init_d=d0, init_b=b0)
    sign = -1.0 if pol == W.TE else 1.0
    tile = (lambda a: None if a is None else np.tile(a, (nx, 1)))
    p2 = W.Problem2D(pol=pol, nx=nx, nz=nz, steps=steps, eps_rest=eps,
                     mu_rest=mu, courant=S, beta=beta, src_row=20,
                     src_profile=np.ones(nx), pulse=pulse,
                     probe_x=np.arange(len(probes)) % nx, probe_z=probes,
                     omegas=om, abc=abc, init_d=tile(d0),
                     init_b=None if b0 is None else sign * tile(b0))
    return p1, p2, sign


@pytest.mark.parametrize("pol", [W.TE, W.TM])
@pytest.mark.parametrize("beta", [0.35, -0.35, 0.0])
@pytest.mark.parametrize("abc,init", [(W.ABC_MUR1, False), (W.ABC_PEC, True),
                                      (W.ABC_PERIODIC, True)])
def test_x_uniform_runs_are_the_1d_scheme(pol, beta, abc, init):
    p1, p2, sign = _pair(pol, beta, abc, 3, init)
    o1 = stepper.solve(p1)
    o2 = stepper2d.solve(p2)
    nh = p1.nz if abc == W.ABC_PERIODIC else p1.nz - 1
    for i in range(p2.nx):
        assert np.array_equal(o2["d"][i], o1["d"])
        assert np.array_equal(o2["b"][i, :nh], sign * o1["b"][:nh])
    assert not np.any(o2["c"])
    assert np.array_equal(o2["trace"], o1["trace"])
    assert np.array_equal(o2["dft"], o1["dft"])


# ----------------------------------------------- 2. textbook Yee at v = 0

def _textbook_yee(p):
    """Plain 2D Yee in (D, B) form, x periodic, PEC z ends, soft source on
    D: arrays (nx, nz), shifts by np.roll / slicing.  Each node reads the
    rest cell containing it: eps cells [i-1/2, i+1/2), mu cells [i, i+1)."""
    nx, nz, S = p.nx, p.nz, p.courant
    eps, mu = p.eps_rest, p.mu_rest
    eps_e = eps                           # E-lattice node z = k
    mu_h = mu[:nz - 1]                    # H-lattice node z = j + 1/2
    mu_e = mu                             # z = k sits in mu cell k
    eps_h = eps[1:]                       # z = j + 1/2 sits in eps cell j + 1
    D = np.zeros((nx, nz))
    B = np.zeros((nx, nz - 1))
    C = np.zeros((nx, nz)) if p.pol == W.TE else np.zeros((nx, nz - 1))
    pl = p.pulse
    for n in range(1, p.steps + 1):
        E = D / eps_e
        if p.pol == W.TE:
            Ez = None
            B = B + S * (E[:, 1:] - E[:, :-1])
            C = C - S * (np.roll(E, -1, axis=0) - E)
            Hx = B / mu_h
            Hz = C / mu_e
            Dn = D.copy()
            Dn[:, 1:-1] = (D[:, 1:-1] + S * (Hx[:, 1:] - Hx[:, :-1])) \
                - S * (Hz - np.roll(Hz, 1, axis=0))[:, 1:-1]
        else:
            Ez = C / eps_h
            B = (B - S * (E[:, 1:] - E[:, :-1])) + S * (np.roll(Ez, -1, axis=0) - Ez)
            Hy = B / mu_h
            Dn = D.copy()
            Dn[:, 1:-1] = D[:, 1:-1] - S * (Hy[:, 1:] - Hy[:, :-1])
            C = C + S * (Hy - np.roll(Hy, 1, axis=0))
        t = n * S
        if t <= pl.t_off:
            u = (t - pl.t0) / pl.tau
            g = pl.amp * math.sin(pl.omega * (t - pl.t0) + pl.phase) * math.exp(-u * u)
            Dn[:, p.src_row] += p.src_profile * g
        Dn[:, 0] = 0.0
        Dn[:, -1] = 0.0
        D = Dn
    return D, B, C


@pytest.mark.parametrize("pol", [W.TE, W.TM])
def test_v0_is_textbook_yee(pol):
    p = W.small_case_2d(12, 90, 240, 0.0, pol=pol, seed=5, abc=W.ABC_PEC,
                        m=2, structure="random")
    o = stepper2d.solve(p)
    D, B, C = _textbook_yee(p)
    nc = p.nz if pol == W.TE else p.nz - 1
    assert np.array_equal(o["d"], D)
    assert np.array_equal(o["b"][:, :p.nz - 1], B)
    assert np.array_equal(o["c"][:, :nc], C)
    assert np.max(np.abs(D)) > 1e-3


# ------------------------------------------------ 3. Yee plane-wave eigenmode

def _eigenmode(pol, nx, nz, mx, mz, eps, mu, n):
    """Closed-form fields of the discrete Yee eigenmode at step n: D at
    (n + 1/2) S, B and C at n S (TE C = B_z at n S; TM C = D_z at
    (n + 1/2) S)."""
    kx, kz = 2 * math.pi * mx / nx, 2 * math.pi * mz / nz
    sw = S * math.sqrt((math.sin(kx / 2) ** 2 + math.sin(kz / 2) ** 2) / (eps * mu))
    w = 2.0 * math.asin(sw) / S
    i = np.arange(nx, dtype=np.float64)[:, None]
    k = np.arange(nz, dtype=np.float64)[None, :]
    td, tb = (n + 0.5) * S, n * S
    ph = lambda x, z, t: np.exp(1j * (kx * x + kz * z - w * t))
    if pol == W.TE:        # E_y amplitude 1
        bx = -S * math.sin(kz / 2) / math.sin(w * S / 2)
        bz = S * math.sin(kx / 2) / math.sin(w * S / 2)
        d = eps * ph(i, k, td)
        b = bx * ph(i, k + 0.5, tb)
        c = bz * ph(i + 0.5, k, tb)
    else:                  # H_y amplitude 1
        ex = S * math.sin(kz / 2) / (eps * math.sin(w * S / 2))
        ez = -S * math.sin(kx / 2) / (eps * math.sin(w * S / 2))
        b = mu * ph(i + 0.5, k + 0.5, tb)
        d = eps * ex * ph(i + 0.5, k, td)
        c = eps * ez * ph(i, k + 0.5, td)
    return d.real, b.real, c.real


def eigenmode_error(pol, lib=None, steps=200):
    nx, nz, eps, mu = 16, 24, 2.0, 1.3
    worst = 0.0
    for mx, mz in [(1, 2), (3, -5), (-2, 7), (5, 0), (0, 3)]:
        d0, b0, c0 = _eigenmode(pol, nx, nz, mx, mz, eps, mu, 0)
        p = W.Problem2D(pol=pol, nx=nx, nz=nz, steps=steps, eps_rest=np.full(nz, eps),
                        mu_rest=np.full(nz, mu), courant=S, beta=0.0,
                        pulse=W.Pulse(amp=0.0), abc=W.ABC_PERIODIC,
                        init_d=d0, init_b=b0, init_c=c0)
        o = _solve2d(p, lib)
        d, b, c = _eigenmode(pol, nx, nz, mx, mz, eps, mu, steps)
        scale = max(np.max(np.abs(d)), np.max(np.abs(b)), np.max(np.abs(c)))
        for got, want in ((o["d"], d), (o["b"], b), (o["c"], c)):
            worst = max(worst, float(np.max(np.abs(got - want))) / scale)
    return worst


EIG_TOL = 1e-12


@pytest.mark.parametrize("pol", [W.TE, W.TM])
def test_yee_eigenmode_closed_form(pol):
    err = eigenmode_error(pol)
    print(f"eigenmode error {err:.2e}")
    assert err < EIG_TOL


# ------------------------------------------------------------- 4. divergence

def _divergence(pol, o):
    """Discrete divergence on the Yee lattice of the field the curls keep
    divergence-free: TE div B at (i+1/2, j+1/2), TM div D at (i, k)."""
    if pol == W.TE:
        bx, bz = o["b"], o["c"]
        return (np.roll(bx, -1, axis=0) - bx) + (np.roll(bz, -1, axis=1) - bz)
    dx, dz = o["d"], o["c"]
    return (dx - np.roll(dx, 1, axis=0)) + (dz - np.roll(dz, 1, axis=1))


def _divergence_closed_form(div0, beta, steps):
    """div^N = (1 - beta S u(kz))^N div^0 per z-Fourier mode, u the symbol of
    the Table 1 upwind difference: 1 - e^{-i kz} (column a, v >= 0) or
    e^{i kz} - 1 (column b, v < 0)."""
    nz = div0.shape[1]
    kz = 2 * math.pi * np.fft.fftfreq(nz)
    u = (1 - np.exp(-1j * kz)) if beta >= 0 else (np.exp(1j * kz) - 1)
    g = (1 - beta * S * u) ** steps
    return np.fft.ifft(np.fft.fft(div0, axis=1) * g[None, :], axis=1).real


def divergence_error(pol, beta, lib=None, steps=150):
    rng = np.random.default_rng(11)
    nx, nz = 10, 48
    eps = rng.uniform(1.0, 2.5, size=nz)
    mu = rng.uniform(1.0, 1.3, size=nz)
    init = {k: rng.normal(size=(nx, nz)) for k in ("init_d", "init_b", "init_c")}
    pulse = W.Pulse(amp=1.0, omega=2 * math.pi / 12.0, t0=20.0, tau=6.0, t_off=40.0)
    p = W.Problem2D(pol=pol, nx=nx, nz=nz, steps=steps, eps_rest=eps, mu_rest=mu,
                    courant=S, beta=beta, src_row=9,
                    src_profile=W.oblique_profile(nx, 1, pol) if pol == W.TE
                    else np.ones(nx), pulse=pulse, abc=W.ABC_PERIODIC, **init)
    o0 = {"d": init["init_d"], "b": init["init_b"], "c": init["init_c"]}
    want = _divergence_closed_form(_divergence(pol, o0), beta, steps)
    got = _divergence(pol, _solve2d(p, lib))
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


DIV_TOL = 1e-12


@pytest.mark.parametrize("pol", [W.TE, W.TM])
@pytest.mark.parametrize("beta", [0.4, -0.3])
def test_divergence_follows_the_upwind_closed_form(pol, beta):
    err = divergence_error(pol, beta)
    print(f"divergence error {err:.2e}")
    assert err < DIV_TOL


# ----------------------------------------- 5. moving uniform modulation

def _one_step_matrix(pol, nx, nz, mx, mz, n_index, beta, lib=None):
    """3x3 amplification matrix of one step for the Fourier mode (mx, mz),
    from three one-step oracle runs starting from a cosine in one field.
    Real fields carry +-k; the +k coefficient maps by G(k)."""
    eps, mu = n_index ** 2, 1.0
    kx, kz = 2 * math.pi * mx / nx, 2 * math.pi * mz / nz
    i = np.arange(nx, dtype=np.float64)[:, None]
    k = np.arange(nz, dtype=np.float64)[None, :]
    # each field's own node positions (x offset, z offset)
    off = {W.TE: {"d": (0.0, 0.0), "b": (0.0, 0.5), "c": (0.5, 0.0)},
           W.TM: {"d": (0.5, 0.0), "b": (0.5, 0.5), "c": (0.0, 0.5)}}[pol]
    basis = {f: np.exp(1j * (kx * (i + ox) + kz * (k + oz))) for f, (ox, oz) in off.items()}
    G = np.zeros((3, 3), dtype=complex)
    names = ("d", "b", "c")
    for col, f in enumerate(names):
        init = {"init_" + g: (basis[g].real if g == f else np.zeros((nx, nz))) for g in names}
        p = W.Problem2D(pol=pol, nx=nx, nz=nz, steps=1, eps_rest=np.full(nz, eps),
                        mu_rest=np.full(nz, mu), courant=S, beta=beta,
                        pulse=W.Pulse(amp=0.0), abc=W.ABC_PERIODIC, **init)
        o = _solve2d(p, lib)
        for row, g in enumerate(names):
            G[row, col] = 2.0 * np.vdot(basis[g], o[g]) / (nx * nz)
    return G


def test_moving_uniform_modulation_dispersion():
    """beta = 0.4, n = 1.5, the mode (1, 1) on an (8 s) x (16 s) ring (wave
    vector at atan 2 from z; |k| h falls as 1/s): the divergence eigenvalue
    is 1 - beta S (1 - e^{-i kz}) exactly and the physical pair's phase
    speed tends to 1/n (error at least halving per grid halving, below 1 %
    on the finest grid)."""
    beta, n_index = 0.4, 1.5
    errs = []
    for scale in (1, 2, 4):
        nx, nz = 8 * scale, 16 * scale
        mx, mz = 1, 1
        G = _one_step_matrix(W.TE, nx, nz, mx, mz, n_index, beta)
        lam = np.linalg.eigvals(G)
        kx, kz = 2 * math.pi * mx / nx, 2 * math.pi * mz / nz
        div_lam = 1 - beta * S * (1 - np.exp(-1j * kz))
        j = int(np.argmin(np.abs(lam - div_lam)))
        assert abs(lam[j] - div_lam) < 1e-13
        phys = np.delete(lam, j)
        kabs = math.hypot(kx, kz)
        speeds = np.abs(np.angle(phys)) / S / kabs
        errs.append(float(np.max(np.abs(speeds * n_index - 1.0))))
        assert np.all(np.abs(phys) <= 1.0 + 1e-12)
    print("phase-speed errors", errs)
    assert errs[1] < errs[0] / 2 and errs[2] < errs[1] / 2
    assert errs[2] < 1e-2


# -------------------------------------------------------- planted mistakes

def _solve2d(p, lib):
    return stepper2d.solve(p, lib=lib)


def _variant(tmp_path, name, old, new, count=1):
    src = open(obuild.SRC2D).read()
    assert src.count(old) == count, old
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = str(tmp_path / f"lib{name}.so")
    obuild.compile_stepper(str(path), lib)
    return stepper2d.load(lib)


def test_planted_x_curl_sign_fails_the_eigenmode(tmp_path):
    lib = _variant(tmp_path, "bzsign", "Cn[i * nz + k] = Cf[i * nz + k] - S * (Es[ip * nz + k]",
                   "Cn[i * nz + k] = Cf[i * nz + k] + S * (Es[ip * nz + k]")
    assert eigenmode_error(W.TE, lib) > 1e3 * EIG_TOL


def test_planted_x_neighbour_fails_the_eigenmode(tmp_path):
    lib = _variant(tmp_path, "tmnb", "S * (Hs[i * nz + j] - Hs[im * nz + j])",
                   "S * (Hs[((i + 1) % nx) * nz + j] - Hs[i * nz + j])")
    assert eigenmode_error(W.TM, lib) > 1e3 * EIG_TOL


def test_planted_dropped_dynamic_term_fails_the_divergence(tmp_path):
    lib = _variant(tmp_path, "nodyn", "- S * (Es[ip * nz + k] - Es[i * nz + k])\n"
                   "                                     - bS * dC;",
                   "- S * (Es[ip * nz + k] - Es[i * nz + k]);")
    assert divergence_error(W.TE, 0.4, lib) > 1e3 * DIV_TOL


def test_planted_tm_dz_upwind_direction_fails_the_divergence(tmp_path):
    lib = _variant(tmp_path, "dzdir", "const double dC = dz_up(Cf, i, j, nz, nc, ring, col_a);",
                   "const double dC = dz_up(Cf, i, j, nz, nc, ring, !col_a);")
    assert divergence_error(W.TM, -0.3, lib) > 1e3 * DIV_TOL


def test_planted_ez_material_cell_fails_the_textbook(tmp_path):
    lib = _variant(tmp_path, "ezcell", "p->eps_rest[rest_cell(k + 1, mE, nz - 1, nz, ring)];",
                   "p->eps_rest[rest_cell(k, mE, nz - 1, nz, ring)];", count=2)
    p = W.small_case_2d(12, 90, 240, 0.0, pol=W.TM, seed=5, abc=W.ABC_PEC,
                        m=2, structure="random")
    assert not np.array_equal(_solve2d(p, lib)["c"][:, :p.nz - 1], _textbook_yee(p)[2])
