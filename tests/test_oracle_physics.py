"""Physics validation of the oracle against the exact solutions of App. B,
on the paper's illustrative set-ups (Section 6, Figs. 5-8), at the
paper's discretisation S = 0.2, dz = lambda0/150 (no GPU).

Missing caption parameters are read as: Fig. 6 eps1 = 2 (as Fig. 5),
Fig. 7 v = +0.3c, Fig. 8 eps 2 -> 4 and v = +0.3c.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import analytic as an

from physics_util import interface_experiment, ratio_experiment


def test_transfer_matrix_reduces_to_closed_forms():
    """App. B.3 self-checks: one interface gives eq. (coef_interface), a
    single layer gives the slab of App. B.2."""
    for beta in (0.3, -0.3, 0.0, 0.45):
        T, G = an.transfer_matrix(1.3, [2.0, 4.0], [], beta)
        T21, G121 = an.interface(2.0, 4.0, beta)
        assert abs(T - T21) < 1e-12 and abs(G - G121) < 1e-12
        for om in (0.04, 0.3, 1.1):
            T, G = an.transfer_matrix(om, [2.0, 4.0, 2.0], [37.0], beta)
            Ts, Gs = an.slab(om, 2.0, 4.0, beta, 37.0)
            assert abs(T - Ts) < 1e-12 and abs(G - Gs) < 1e-12


def test_interface_coefficients_printed_values():
    """eq. (coef_interface) and (comp_exp) at the Fig. 5 parameters."""
    T, G = an.interface(2.0, 4.0, -0.3)
    a_t, a_r = an.compression_factors(math.sqrt(2.0), 2.0, -0.3)
    assert abs(abs(G) - 0.4244) < 1e-4 and abs(T - 0.7374) < 1e-4
    assert abs(a_r - 2.4738) < 1e-4 and abs(a_t - 0.8902) < 1e-4


def test_moving_interface_fig5():
    """Fig. 5 (contra-moving interface, v = -0.3c, eps 2 | 4): reflected
    and transmitted pulse peaks and Doppler-shifted carriers against
    eq. (coef_interface)/(comp_exp); the error shrinks under refinement."""
    T, G = an.interface(2.0, 4.0, -0.3)
    a_t, a_r = an.compression_factors(math.sqrt(2.0), 2.0, -0.3)
    g150, t150, r150, q150 = interface_experiment(150.0)
    g75, t75, _, _ = interface_experiment(75.0)
    assert abs(g150 - abs(G)) < 0.03 * abs(G)
    assert abs(t150 - abs(T)) < 0.03 * abs(T)
    assert abs(r150 - a_r) < 0.005 * a_r
    assert abs(q150 - a_t) < 0.005 * a_t
    assert abs(g150 - abs(G)) < abs(g75 - abs(G))
    assert abs(t150 - abs(T)) < abs(t75 - abs(T))


def test_moving_slab_fig6():
    """Fig. 6 (co-moving space-time quarter-wave slab, v = 0.3c, eps2 =
    4 in eps1 = 2): |T(w)|, |Gamma(w)| from Fourier ratios against App.
    B.2 across the pulse band."""
    b, n1, n2 = 0.3, math.sqrt(2.0), 2.0
    ell = (1.0 / (4 * n2)) * (1 + n2 * b) / (1 - n1 * b)
    w, Tm, Tx, Gm, Gx = ratio_experiment([2.0, 4.0, 2.0], [ell], b, 150.0)
    assert np.max(np.abs(Tm - Tx)) < 0.02
    assert np.max(np.abs(Gm - Gx)) < 0.02


def test_moving_crystal_fig7():
    """Fig. 7 (co-moving bilayer crystal of 5 space-time quarter-wave
    cells, eps 1/4): Fourier-ratio coefficients against the transfer
    matrix; the stopband (|Gamma| ~ 0.54, |T| < 0.1 near 1.2 w0) is
    reproduced and the in-band error shrinks under refinement."""
    b = 0.3
    cell = [(1 + b) / (1 - 2 * b) / 4.0, (1 + 2 * b) / (1 - b) / 8.0]
    res = {}
    for lam in (75.0, 150.0):
        res[lam] = ratio_experiment([1.0] + [1.0, 4.0] * 5 + [1.0], cell * 5,
                                    b, lam)
    w, Tm, Tx, Gm, Gx = res[150.0]
    stop = (w > 1.17) & (w < 1.25)
    assert np.max(np.abs(Gm[stop] - Gx[stop])) < 0.03
    assert np.max(Tm[stop]) < 0.12
    rms = lambda a, b: float(np.sqrt(np.mean((a - b) ** 2)))
    assert rms(Tm, Tx) < 0.06 and rms(Gm, Gx) < 0.06
    w75, Tm75, Tx75, Gm75, Gx75 = res[75.0]
    assert rms(Tm, Tx) + rms(Gm, Gx) < rms(Tm75, Tx75) + rms(Gm75, Gx75)


def test_moving_gradient_fig8():
    """Fig. 8 (co-moving linear gradient eps 2 -> 4 over lambda0/2):
    Fourier-ratio coefficients against the transfer matrix with one layer
    per cell.  The transmitted wave is up-shifted by a_t = 1.44 and must be
    recorded far downstream (the probe has to stay ahead of the moving
    gradient), so the scheme's own attenuation (|zeta| < 1, Section 5)
    grows with frequency: the band is held to 0.75-1.05 w0."""
    b, lam = 0.3, 150.0
    L = int(lam / 2)
    layers = [2.0 + 2.0 * (i + 0.5) / L for i in range(L)]
    w, Tm, Tx, Gm, Gx = ratio_experiment([2.0] + layers + [4.0],
                                         [1.0 / lam] * L, b, lam,
                                         band=(0.75, 1.05), nband=31)
    assert np.max(np.abs(Tm - Tx)) < 0.03 * np.max(Tx)
    assert np.max(np.abs(Gm - Gx)) < 0.01


# ---------------------------------------------------------------------------
# P10: moving matter
# ---------------------------------------------------------------------------

def test_matter_constitutive_form_matches_tensors():
    """Footnote to eq. (5): with E = E* + v B and H = H* + v D (inverse of
    eq. (2) in 1D), the solved star form E* = g (mu' D - beta B),
    H* = g (eps' B - beta D), g = (1-beta^2)/(eps' mu' - beta^2), satisfies
    D = eps' alpha E + chi H and B = chi E + mu' alpha H."""
    rng = np.random.default_rng(0)
    for _ in range(50):
        eps, mu = rng.uniform(1, 6), rng.uniform(1, 2)
        beta = rng.uniform(-0.9, 0.9)
        if abs(1 - beta * beta * eps * mu) < 1e-3:
            continue
        D, B = rng.normal(size=2)
        g = (1 - beta * beta) / (eps * mu - beta * beta)
        Es = g * (mu * D - beta * B)
        Hs = g * (eps * B - beta * D)
        E, H = Es + beta * B, Hs + beta * D
        alpha, chi = an.matter_alpha_chi(eps, mu, beta)
        assert abs(eps * alpha * E + chi * H - D) < 1e-12 * (1 + abs(alpha))
        assert abs(chi * E + mu * alpha * H - B) < 1e-12 * (1 + abs(alpha))


def test_matter_at_rest_is_modulation_at_rest():
    """At v = 0 moving matter and moving modulation are the same medium."""
    p = W.small_case(120, 300, 0.0, seed=2, structure="random")
    p = p.replace(mu_rest=np.ones(p.nz))
    a = oracle.solve(p)
    b = oracle.solve(p.replace(kind=W.MATTER))
    assert np.max(np.abs(a["trace"] - b["trace"])) < 1e-13 * np.max(np.abs(a["trace"]))


def test_matter_speed_is_relativistic_addition():
    """Light in uniform matter of rest index 2 moving at +0.5c travels at
    (1/2 + 1/2)/(1 + 1/4) = 0.8 forward (velocity addition); in a uniform
    moving modulation of the same index it stays 1/2."""
    lam, S, nz = 160.0, 0.4, 6000
    tau = 1.5 * lam
    for kind, beta, want in ((W.MATTER, 0.5, an.matter_velocity(2.0, 0.5)[0]),
                             (W.MODULATION, 0.4, 0.5)):
        steps = int((8 * tau + 1.2 * 3000 / want) / S)
        p = W.Problem(nz=nz, steps=steps, eps_rest=np.full(nz, 4.0),
                      mu_rest=np.ones(nz), courant=S, beta=beta, kind=kind,
                      src_cell=500,
                      pulse=W.Pulse(1.0, 2 * math.pi / lam, 4 * tau, tau, 0.0,
                                    8 * tau),
                      probes=np.array([1500, 3500]))
        tr = oracle.solve(p, fields=False)["trace"]
        from physics_util import envelope
        e0, e1 = envelope(tr[0]), envelope(tr[1])
        ts = (np.arange(p.steps) + 1.5) * S
        c0 = np.sum(ts * e0 ** 2) / np.sum(e0 ** 2)
        c1 = np.sum(ts * e1 ** 2) / np.sum(e1 ** 2)
        speed = 2000.0 / (c1 - c0)
        assert abs(speed - want) < 0.01 * want


def test_transfer_matrix_conserves_energy_in_long_stationary_crystals():
    """At v = 0 a lossless stack between two vacuum half-spaces conserves
    energy, |Gamma|^2 + |T|^2 = 1, at every frequency -- also deep in the
    stopband of a long high-contrast crystal, where the entries of the
    total matrix grow by many orders of magnitude (the transmission comes
    from det M / M22 with det M carried factor by factor)."""
    from oracle import analytic as A
    rng = np.random.default_rng(5)
    for _ in range(6):
        e1, e2 = rng.uniform(1.0, 12.0, size=2)
        P = int(rng.integers(40, 100))
        eps = [1.0] + [e1, e2] * P + [1.0]
        widths = [13.0, 21.0] * P
        for w in np.linspace(0.05, 0.9, 23):
            T, G = A.transfer_matrix(w, eps, widths, 0.0)
            assert abs(abs(G) ** 2 + abs(T) ** 2 - 1.0) < 1e-9, (e1, e2, P, w)
