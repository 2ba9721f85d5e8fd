"""Von Neumann analysis of the generalized scheme (Section 5, App. A).

TEST INFRASTRUCTURE: see oracle/__init__.py.

A plane-wave test field Psi_k^n = Psi0 xi^k zeta^n with xi = exp(i theta),
theta = k_z dz (eq. (14)), is pushed through one full time step of the
scheme -- (10c) E* from the state, (10a) Faraday, (10d) H*, (10b) Ampere,
each with the Table 1 dynamic terms -- which gives the 2x2 amplification
matrix G(theta) acting on the amplitudes (D, B).  Its eigenvalues are the
two roots zeta_+ (co-moving) and zeta_- (contra-moving) discussed in
Section 5; the closed forms printed for them (eq. (15)) and for the
characteristic polynomial (App. A) are not used here, only the matrix.
"""
from __future__ import annotations

import cmath
import math
from typing import Tuple

import numpy as np

MODULATION = 0
MATTER = 1


def _node_coefficients(eps: float, mu: float, beta: float, kind: int):
    """Constitutive coefficients of (10c)/(10d) for one medium:
    E* = aE D - bE Bbar, H* = aH B - bH Dbar."""
    if kind == MATTER:
        g = (1.0 - beta * beta) / (eps * mu - beta * beta)
        return g * mu, g * beta, g * eps, g * beta
    return 1.0 / eps, beta, 1.0 / mu, beta


def amplification_matrix(theta: float, S: float, beta: float, eps: float,
                         mu: float = 1.0, kind: int = MODULATION) -> np.ndarray:
    """G(theta) with (D^{n+1/2}, B^n) = G (D^{n-1/2}, B^{n-1}); D at node k,
    B at node k+1/2, both referred to their own node position."""
    col_a = beta >= 0.0
    aE, bE, aH, bH = _node_coefficients(eps, mu, beta, kind)
    ei = cmath.exp(1j * theta)
    half = cmath.exp(0.5j * theta)
    curl = half - 1.0 / half                     # e^{i th/2} - e^{-i th/2}
    if col_a:
        bbar = 0.5 * (1.0 / half + 1.0 / (half * ei))   # (Ba): k-1/2, k-3/2
        dB = 1.0 - 1.0 / ei                             # (dBa)
        dD = 1.0 - 1.0 / ei                             # (dDa)
    else:
        bbar = 0.5 * (half * ei + half)                 # (Bb): k+3/2, k+1/2
        dB = ei - 1.0                                   # (dBb)
        dD = ei - 1.0                                   # (dDb)
    dbar = 0.5 * (half + 1.0 / half)                    # (Da) = (Db)
    G = np.zeros((2, 2), dtype=complex)
    for col, (D, B) in enumerate(((1.0, 0.0), (0.0, 1.0))):
        Es = aE * D - bE * bbar * B                     # (10c) at n-1/2
        Bn = B - S * curl * Es - beta * S * dB * B      # (10a)
        Hs = aH * Bn - bH * dbar * D                    # (10d) at n
        Dn = D - S * curl * Hs - beta * S * dD * D      # (10b)
        G[0, col] = Dn
        G[1, col] = Bn
    return G


def zetas(theta: float, S: float, beta: float, eps: float, mu: float = 1.0,
          kind: int = MODULATION) -> Tuple[complex, complex]:
    """The two amplification factors at theta, ordered (zeta_+, zeta_-):
    zeta_+ is the root whose phase is negative (forward wave, eq. (16),
    upper sign), zeta_- the one with positive phase (backward wave)."""
    w = np.linalg.eigvals(amplification_matrix(theta, S, beta, eps, mu, kind))
    w = sorted(w, key=lambda z: np.angle(z))
    return complex(w[0]), complex(w[1])


def max_growth(S: float, beta: float, eps: float, mu: float = 1.0,
               kind: int = MODULATION, ntheta: int = 512) -> float:
    """max over theta in (0, pi] of the spectral radius of G(theta)."""
    best = 0.0
    for t in np.linspace(math.pi / ntheta, math.pi, ntheta):
        w = np.linalg.eigvals(amplification_matrix(t, S, beta, eps, mu, kind))
        best = max(best, float(np.max(np.abs(w))))
    return best


def eigenmode(theta: float, S: float, beta: float, eps: float, mu: float,
              which: int, kind: int = MODULATION):
    """(zeta, (D0, B0)) for eigenvalue index `which` (0: zeta_+, 1: zeta_-)."""
    G = amplification_matrix(theta, S, beta, eps, mu, kind)
    w, v = np.linalg.eig(G)
    order = np.argsort(np.angle(w))
    i = order[which]
    return complex(w[i]), v[:, i]


def yee_zeta(theta: float, S: float, n: float) -> complex:
    """Textbook 1D Yee amplification factor for a forward wave at v = 0:
    sin(w dt/2) = (S/n) sin(theta/2), |zeta| = 1 for S <= n."""
    s = (S / n) * math.sin(theta / 2.0)
    return cmath.exp(-2j * cmath.asin(s))
