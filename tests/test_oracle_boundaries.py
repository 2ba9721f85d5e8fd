"""Pins of the oracle's probe spectrum and absorbing ends (no GPU).

Probe DFT.  In a v = 0 vacuum run the soft source's field at a probe a
distance d away is fixed by the discrete Green's function of the 1D Yee
update (the v = 0 limit of eq. (10a)-(10d), Section 4 "usual fashion"):
a source sample s^n added to D each step radiates, at angular frequency w,
    E(w) = s(w) exp(i kappa d) / (2 S cos(kappa/2)),
    sin(kappa/2) = sin(w S/2) / S         (textbook Yee dispersion),
in both directions, with the e^{-i w t} time dependence of the incident
wave of App. B.1.  The source spectrum s(w) is the closed-form spectrum of
the Gaussian-modulated sinusoid of App. B.1, the envelope
exp(-tau^2 (w - w_i)^2 / 4) (reading G3) together with its mirror term
at -w_i.  So the probe DFT X(w) = sum_n E_n S exp(+i w t_n),
t_n = (n + 1/2) S, must equal that product.  A flipped DFT sign, a time
offset of half a step or a wrong weight moves it far outside the bound.

Absorbing ends (first-order Mur on D, reading R3).  The reflection of an
end is measured as the largest difference at a probe near the end between
the run and a reference run whose end lies out of reach, relative to the
incident peak.  The ends absorb to below 1e-3 for vacuum, for a moving
modulation of either sign and, for moving matter, at the end the medium
moves towards (where the outgoing wave has the lab speed
(1/n + |beta|)/(1 + |beta|/n), relativistic addition) and at a vacuum end.
(The end that moving matter with n' > 1 moves away from reflects, about
0.7 at n' = 2^(1/2), beta = 0.5: stated in the design notes, not pinned.)

Each pin is also run on variants of the oracle source with one planted
mistake, compiled here, and must fail there.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import build as obuild
from oracle import stepper

S = 0.5


# ------------------------------------------------------------- probe DFT

def _pulse_spectrum(pulse, w):
    """Closed-form sum_n S g(n S) exp(+i w n S) of the App. B.1 pulse
    g(t) = A sin(w0 (t - t0) + phi) exp(-((t - t0)/tau)^2), as the
    integral: both Gaussian terms, exp(-tau^2 (w -+ w0)^2 / 4)."""
    A, w0, t0, tau, ph = pulse.amp, pulse.omega, pulse.t0, pulse.tau, pulse.phase
    plus = np.exp(1j * ph) * np.exp(-tau ** 2 * (w + w0) ** 2 / 4.0)
    minus = np.exp(-1j * ph) * np.exp(-tau ** 2 * (w - w0) ** 2 / 4.0)
    return A * np.exp(1j * w * t0) * math.sqrt(math.pi) * tau * (plus - minus) / 2j


def _yee_green(w, d):
    kappa = 2.0 * np.arcsin(np.sin(w * S / 2.0) / S)
    return np.exp(1j * kappa * d) / (2.0 * S * np.cos(kappa / 2.0))


def _dft_case():
    pulse = W.carrier_pulse(phase=0.7)
    nz, ks, d = 4000, 2000, 20
    steps = int((2 * pulse.t0 + d + 200) / S)
    om = pulse.omega * np.linspace(0.8, 1.2, 16)
    return W.Problem(nz=nz, steps=steps, eps_rest=np.ones(nz), mu_rest=np.ones(nz),
                     courant=S, beta=0.0, src_cell=ks, pulse=pulse,
                     probes=np.array([ks + d, ks - d]), omegas=om), d


def dft_error(lib=None):
    """Largest relative complex error of the oracle's probe DFTs (both
    probes, 16 frequencies across the band) against the closed form."""
    p, d = _dft_case()
    out = stepper.solve(p, fields=False, lib=lib)
    want = _yee_green(p.omegas, d) * _pulse_spectrum(p.pulse, p.omegas)
    return float(np.max(np.abs(out["dft"] / want[None, :] - 1.0)))


DFT_TOL = 2e-5     # source switched on at t = S and off at t = 2 t0 (envelope
                   # e^-16 there) and the 16-digit sums: measured 3e-6


def test_probe_dft_matches_closed_form_spectrum():
    e = dft_error()
    print(f"probe DFT vs closed form: max rel err {e:.2e}")
    assert e < DFT_TOL


def test_dft_is_the_sum_of_the_recorded_trace():
    """The running DFT equals sum_n E_n S exp(+i w (n + 1/2) S) over the
    returned trace (the accumulation, not only the end result)."""
    p, _ = _dft_case()
    out = stepper.solve(p, fields=False)
    t = (np.arange(1, p.steps + 1) + 0.5) * S
    X = out["trace"] @ (S * np.exp(1j * np.outer(t, p.omegas)))
    assert np.max(np.abs(X - out["dft"])) <= 1e-10 * np.max(np.abs(X))


def test_dft_pin_rejects_wrong_conventions():
    """The closed form tells the DFT conventions apart: the conjugate
    kernel exp(-i w t), times n S instead of (n + 1/2) S, or no weight S,
    all land far outside the bound."""
    p, d = _dft_case()
    out = stepper.solve(p, fields=False)
    want = _yee_green(p.omegas, d) * _pulse_spectrum(p.pulse, p.omegas)
    tr = out["trace"]
    n = np.arange(1, p.steps + 1)
    for label, t, wgt, sgn in (("conjugate kernel", (n + 0.5) * S, S, -1.0),
                               ("time n S", n * S, S, 1.0),
                               ("no weight", (n + 0.5) * S, 1.0, 1.0)):
        X = tr @ (wgt * np.exp(sgn * 1j * np.outer(t, p.omegas)))
        e = float(np.max(np.abs(X / want[None, :] - 1.0)))
        print(f"{label}: {e:.2e}")
        assert e > 100 * DFT_TOL, label


# ------------------------------------------------------------ Mur ends

LONG_PULSE = W.carrier_pulse(cycles=6, lambda0=160.0, phase=0.3)


def _speeds(eps, beta, kind):
    """Lab speeds of the right- and left-going waves of a uniform medium."""
    n = math.sqrt(eps)
    if kind == W.MATTER:
        return (1 / n + beta) / (1 + beta / n), (1 / n - beta) / (1 - beta / n)
    return 1 / n, 1 / n


def end_reflection(eps, beta, kind, side, lib=None, dsrc=150, margin=30):
    """Peak reflected / peak incident field at a probe `margin` cells inside
    the right (side = +1) or left (side = -1) end of a uniform medium."""
    ur, ul = _speeds(eps, beta, kind)
    u = ur if side > 0 else ul
    back = ul if side > 0 else ur
    nz = 2 * dsrc + 400
    ks = nz - 1 - dsrc if side > 0 else dsrc
    pr = nz - 1 - margin if side > 0 else margin
    t_end = dsrc / u + margin / back + 2 * LONG_PULSE.t0 + 50
    steps = int(t_end / S)
    far = int(t_end * max(ur, ul)) + 50

    def run(nz_, ks_, pr_):
        p = W.Problem(nz=nz_, steps=steps, eps_rest=np.full(nz_, float(eps)),
                      mu_rest=np.ones(nz_), courant=S, beta=beta, kind=kind,
                      src_cell=ks_, pulse=LONG_PULSE, probes=np.array([pr_]),
                      omegas=np.zeros(0))
        return stepper.solve(p, fields=False, lib=lib)["trace"][0]

    a = run(nz, ks, pr)
    off = far if side < 0 else 0
    b = run(nz + far, ks + off, pr + off)       # the tested end out of reach
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


MUR_TOL = 1e-3
ABSORBING = [
    # eps', beta, kind, side
    (1.0, 0.0, W.MODULATION, +1), (1.0, 0.0, W.MODULATION, -1),
    (4.0, 0.3, W.MODULATION, +1), (4.0, 0.3, W.MODULATION, -1),
    (4.0, -0.3, W.MODULATION, +1), (4.0, -0.3, W.MODULATION, -1),
    (2.0, 0.5, W.MATTER, +1), (2.0, -0.5, W.MATTER, -1),     # downstream ends
    (4.0, 0.3, W.MATTER, +1),
    (1.0, 0.5, W.MATTER, +1), (1.0, 0.5, W.MATTER, -1),       # vacuum, both
]


@pytest.mark.parametrize("eps,beta,kind,side", ABSORBING)
def test_mur_ends_absorb(eps, beta, kind, side):
    r = end_reflection(eps, beta, kind, side)
    print(f"eps'={eps} beta={beta} kind={kind} end={side:+d}: reflection {r:.2e}")
    assert r < MUR_TOL


# ------------------------------------------------- planted mistakes (CPU)

def _variant(tmp_path, name, old, new):
    """The oracle stepper with one source line changed, compiled and loaded."""
    src = open(obuild.SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = str(tmp_path / f"lib{name}.so")
    obuild.compile_stepper(str(path), lib)
    return stepper.load(lib)


def test_planted_dft_sign_fails_the_pin(tmp_path):
    lib = _variant(tmp_path, "dftsign", "sw[m] = sin(p->omegas[m] * tp);",
                   "sw[m] = -sin(p->omegas[m] * tp);")
    assert dft_error(lib) > 100 * DFT_TOL


def test_planted_dft_time_offset_fails_the_pin(tmp_path):
    lib = _variant(tmp_path, "dfttime", "const double tp = ((double)n + 0.5) * S;",
                   "const double tp = (double)n * S;")
    assert dft_error(lib) > 100 * DFT_TOL


def test_planted_mur_sign_fails_the_pin(tmp_path):
    lib = _variant(tmp_path, "mursign", "return (S * u - 1.0) / (S * u + 1.0);",
                   "return (1.0 - S * u) / (S * u + 1.0);")
    assert end_reflection(1.0, 0.0, W.MODULATION, +1, lib=lib) > 100 * MUR_TOL


def test_planted_nonrelativistic_exit_speed_fails_the_pin(tmp_path):
    """Moving matter's exit speed taken as 1/n (no velocity addition): the
    downstream end then reflects about 2e-2, against 3e-4."""
    lib = _variant(tmp_path, "exitspeed", "double b = dir * beta;",
                   "double b = 0.0 * dir * beta;")
    r = end_reflection(2.0, 0.5, W.MATTER, +1, lib=lib)
    print(f"non-relativistic exit speed: reflection {r:.2e}")
    assert r > 10 * MUR_TOL
