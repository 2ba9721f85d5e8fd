"""Helpers for the physics validations of Section 6: build the paper's
scattering set-ups on a grid, run the oracle, and read scattering
coefficients from probe traces the way the paper does (envelope peaks for
the interface, Fourier-transform ratios for the other structures, Fig. 5
caption)."""
import math

import numpy as np

import oracle
import workloads as W
from oracle import analytic as an


def envelope(x):
    """|analytic signal| of a real record (FFT Hilbert transform)."""
    n = len(x)
    X = np.fft.fft(x)
    h = np.zeros(n)
    h[0] = 1.0
    if n % 2 == 0:
        h[n // 2] = 1.0
        h[1:n // 2] = 2.0
    else:
        h[1:(n + 1) // 2] = 2.0
    return np.abs(np.fft.ifft(X * h))


def spectral_peak(x, S, mask):
    y = np.where(mask, x, 0.0)
    N = 1 << 22
    F = np.abs(np.fft.rfft(y, N))
    w = 2 * np.pi * np.fft.rfftfreq(N, S)
    return float(w[np.argmax(F)])


def interface_experiment(lam, S=0.2, beta=-0.3, eps1=2.0, eps2=4.0):
    """Fig. 5 set-up: medium 1 (left) and medium 2 (right) separated by an
    interface moving at beta; a modulated Gaussian incident from medium 1.
    Returns measured (|Gamma|, |T|, a_r, a_t)."""
    f = lam / 150.0
    nz, src, pin, pout, zi = (int(x * f) for x in (5000, 600, 1200, 3600, 3000))
    tau = 2.0 * lam
    t0 = 4.0 * tau
    steps = int(7300 * f / S)
    p = W.Problem(nz=nz, steps=steps,
                  eps_rest=W.interface_profile(nz, zi, eps1, eps2),
                  mu_rest=np.ones(nz), courant=S, beta=beta, src_cell=src,
                  pulse=W.Pulse(1.0, 2 * math.pi / lam, t0, tau, 0.0, 2 * t0),
                  probes=np.array([pin, pout]))
    tr = oracle.solve(p, fields=False)["trace"]
    ts = (np.arange(steps) + 1.5) * S
    # the incident pulse passes the input probe well before the reflected
    # one returns (kinematics of the set-up: ~2050 vs ~4400 at lam = 150)
    split = 0.5 * (2049.0 + 4402.0) * f
    e_in, e_out = envelope(tr[0]), envelope(tr[1])
    inc = e_in[ts < split].max()
    ref = e_in[ts >= split].max()
    tra = e_out.max()
    wi = spectral_peak(tr[0], S, ts < split)
    wr = spectral_peak(tr[0], S, ts >= split)
    wt = spectral_peak(tr[1], S, ts > 0)
    return ref / inc, tra / inc, wr / wi, wt / wi


def ratio_experiment(eps_layers, widths_in_lambda, beta, lam, S=0.2,
                     tau_periods=0.6, band=(0.75, 1.25), nband=41):
    """Structure of layers eps_layers[1:-1] (widths in units of lambda0,
    rounded to cells) between semi-infinite media eps_layers[0] (left)
    and eps_layers[-1] (right), all moving at beta; short pulse incident
    from the left.  Returns (w/w0, |T| measured, |T| TMM, |Gamma|
    measured, |Gamma| TMM) over the band, from Fourier-transform ratios:
    |T(w)| = a_t |X_t(a_t w)| / |X_i(w)|, |Gamma(w)| = a_r |X_r(a_r w)| /
    |X_i(w)| (each scattered wave is a Doppler-scaled copy, App. B.1)."""
    e_in, e_out = eps_layers[0], eps_layers[-1]
    n_in, n_out = math.sqrt(e_in), math.sqrt(e_out)
    widths = [int(round(w * lam)) for w in widths_in_lambda]
    L = int(sum(widths))
    tau = tau_periods * lam
    t0 = 5.0 * tau
    u = 1.0 / n_in
    src = int(5 * tau * u) + 20
    pin = src + int(2 * lam)
    z0 = pin + int(12 * tau * u) + 100
    tm = (z0 - src + u * t0) / (u - beta)       # pulse centre meets structure
    zm = z0 + beta * tm
    a_t, a_r = an.compression_factors(n_in, n_out, beta)
    t_ref = tm + (zm - pin) / u
    t_end = t_ref + 40 * tau / a_r
    for _ in range(20):   # output probe stays ahead of the moving structure
        pout = int(z0 + L + beta * t_end + lam)
        t_end = max(t_ref + 40 * tau / a_r,
                    tm + 2 * L * n_out + (pout - zm) * n_out + 40 * tau / a_t)
    nz = pout + int(40 * tau / a_t) + 200
    steps = int(t_end / S)
    eps = np.full(nz, float(e_in))
    eps[z0 + L:] = e_out
    a = z0
    for e, w in zip(eps_layers[1:-1], widths):
        eps[a:a + w] = e
        a += w
    p = W.Problem(nz=nz, steps=steps, eps_rest=eps, mu_rest=np.ones(nz),
                  courant=S, beta=beta, src_cell=src,
                  pulse=W.Pulse(1.0, 2 * math.pi / lam, t0, tau, 0.0, 2 * t0),
                  probes=np.array([pin, pout]))
    tr = oracle.solve(p, fields=False)["trace"]
    ts = (np.arange(steps) + 1.5) * S
    split = 0.5 * ((pin - src) / u + t0 + t_ref)
    inc = np.where(ts < split, tr[0], 0.0)
    ref = np.where(ts >= split, tr[0], 0.0)
    N = 1 << 22
    w = 2 * np.pi * np.fft.rfftfreq(N, S)
    Fi = np.abs(np.fft.rfft(inc, N))
    Fr = np.abs(np.fft.rfft(ref, N))
    Ft = np.abs(np.fft.rfft(tr[1], N))
    w0 = 2 * math.pi / lam
    om = np.linspace(band[0] * w0, band[1] * w0, nband)
    Ii = np.interp(om, w, Fi)
    Tm = a_t * np.interp(a_t * om, w, Ft) / Ii
    Gm = a_r * np.interp(a_r * om, w, Fr) / Ii
    Tx = np.empty(nband)
    Gx = np.empty(nband)
    for i, o in enumerate(om):
        T, G = an.transfer_matrix(o, eps_layers, widths, beta)
        Tx[i], Gx[i] = abs(T), abs(G)
    return om / w0, Tm, Tx, Gm, Gx
