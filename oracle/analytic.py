"""Exact frequency-domain solutions used to validate the time stepping
(App. B): Doppler compression factors, the moving interface, the moving
slab and a transfer-matrix method for piecewise-uniform moving profiles.

TEST INFRASTRUCTURE: see oracle/__init__.py.

Conventions: fields vary as exp(-i w t) (the incident pulse of App. B.1),
a forward wave in a medium of index n as exp(+i n w z).  In a moving
modulation the quantity w (1 -/+ n beta) is the same for every wave of one
scattering problem (forward/backward), which fixes all frequencies (App.
B.3, eq. for w_m^+-).  Continuity of the auxiliary fields E* and H* at a
moving interface (eq. (1a,b)) becomes ordinary Fresnel matching in the
"star" amplitudes A = a (1 - beta n) (forward) and B = b (1 + beta n)
(backward), where a and b are the E-field amplitudes.

Several printed formulas of App. B are typeset inconsistently; the forms
below are re-derived from eq. (1)-(2) and the readings are listed in the
design notes:
  * gamma_nmn's Doppler factor is (1 - n_n beta)/(1 + n_n beta);
  * the transfer matrix yields Gamma = -M21/M22, T = det M / M22;
  * the slab's round-trip term is Gamma_212 Gamma^-_212 = r*^2.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np


def index(eps: float, mu: float = 1.0) -> float:
    return math.sqrt(eps * mu)


def impedance(eps: float, mu: float = 1.0) -> float:
    return math.sqrt(mu / eps)


def compression_factors(n_in: float, n_out: float, beta: float
                        ) -> Tuple[float, float]:
    """(a_t, a_r) of eq. (comp_exp): transmitted and reflected frequency
    ratios for incidence in the medium of index n_in."""
    a_t = (1.0 - n_in * beta) / (1.0 - n_out * beta)
    a_r = (1.0 - n_in * beta) / (1.0 + n_in * beta)
    return a_t, a_r


def interface(eps1: float, eps2: float, beta: float, mu1: float = 1.0,
              mu2: float = 1.0) -> Tuple[float, float]:
    """(T21, Gamma121) of eq. (coef_interface): incidence from medium 1
    onto medium 2, the interface moving at beta."""
    n1, n2 = index(eps1, mu1), index(eps2, mu2)
    e1, e2 = impedance(eps1, mu1), impedance(eps2, mu2)
    T = 2.0 * e2 / (e1 + e2) * (1.0 - n1 * beta) / (1.0 - n2 * beta)
    G = (e2 - e1) / (e1 + e2) * (1.0 - n1 * beta) / (1.0 + n1 * beta)
    return T, G


def slab(omega: float, eps1: float, eps2: float, beta: float, length: float,
         mu1: float = 1.0, mu2: float = 1.0) -> Tuple[complex, complex]:
    """(T, Gamma) of a slab of medium 2 and lab-frame length `length` in
    background medium 1, moving at beta, for an incident wave of frequency
    omega from the left: multiple reflection (App. B.2), with forward and
    backward internal frequencies w2+ = w(1-n1 b)/(1-n2 b) and
    w2- = w(1-n1 b)/(1+n2 b)."""
    n1, n2 = index(eps1, mu1), index(eps2, mu2)
    e1, e2 = impedance(eps1, mu1), impedance(eps2, mu2)
    T21, G121 = interface(eps1, eps2, beta, mu1, mu2)
    T12, _ = interface(eps2, eps1, beta, mu2, mu1)
    rs = (e1 - e2) / (e1 + e2)                 # star reflection inside
    w2p = omega * (1.0 - n1 * beta) / (1.0 - n2 * beta)
    w2m = omega * (1.0 - n1 * beta) / (1.0 + n2 * beta)
    phi = n2 * (w2p + w2m) * length
    phip = n2 * w2p * length
    den = 1.0 - rs * rs * np.exp(1j * phi)
    T = T21 * T12 * np.exp(1j * phip) / den
    G = G121 * (1.0 - np.exp(1j * phi)) / den
    return complex(T), complex(G)


def transfer_matrix(omega: float, eps: Sequence[float], widths: Sequence[float],
                    beta: float, mu: Sequence[float] = None
                    ) -> Tuple[complex, complex]:
    """(T, Gamma) for layers 0..N-1 (layer 0 and N-1 are the semi-infinite
    outer media; `widths` gives the lab-frame widths of layers 1..N-2),
    all moving at beta, incident wave of frequency omega from layer 0.

    State vector: star amplitudes (A, B) of the forward and backward waves.
    Interface m|m+1: K_{m+1} u_{m+1} = K_m u_m with K = [[1, 1],
    [1/eta, -1/eta]] (continuity of E* and H*); layer m of width w:
    A -> A exp(i n w_m^+ w), B -> B exp(-i n w_m^- w).
    """
    N = len(eps)
    mu = [1.0] * N if mu is None else list(mu)
    assert len(widths) == N - 2
    n = [index(e, m) for e, m in zip(eps, mu)]
    eta = [impedance(e, m) for e, m in zip(eps, mu)]
    inv = omega * (1.0 - n[0] * beta)          # w (1 - n beta), invariant

    def K(m):
        return np.array([[1.0, 1.0], [1.0 / eta[m], -1.0 / eta[m]]], dtype=complex)

    # det M is carried as the product of the factors' determinants (det of
    # a product is the product of dets): forming it from the entries of M
    # cancels catastrophically when M grows, as in the stopband of a long
    # crystal.  det(K(m+1)^-1 K(m)) = eta_{m+1}/eta_m.
    M = np.eye(2, dtype=complex)
    det = 1.0 + 0.0j
    for m in range(N - 1):
        if m >= 1:
            wp = inv / (1.0 - n[m] * beta)
            wm = inv / (1.0 + n[m] * beta)
            P = np.diag([np.exp(1j * n[m] * wp * widths[m - 1]),
                         np.exp(-1j * n[m] * wm * widths[m - 1])])
            M = P @ M
            det *= P[0, 0] * P[1, 1]
        M = np.linalg.solve(K(m + 1), K(m)) @ M
        det *= eta[m + 1] / eta[m]
    r_star = -M[1, 0] / M[1, 1]
    t_star = det / M[1, 1]
    G = r_star * (1.0 - n[0] * beta) / (1.0 + n[0] * beta)
    T = t_star * (1.0 - n[0] * beta) / (1.0 - n[-1] * beta)
    return complex(T), complex(G)


# --------------------------------------------------------------------------
# Moving matter (footnote to eq. (5))
# --------------------------------------------------------------------------

def matter_alpha_chi(eps_r: float, mu_r: float, beta: float) -> Tuple[float, float]:
    """alpha and chi of the moving-matter tensors."""
    n2 = eps_r * mu_r
    den = 1.0 - beta * beta * n2
    return (1.0 - beta * beta) / den, beta * (1.0 - n2) / den


def matter_velocity(n_rest: float, beta: float) -> Tuple[float, float]:
    """Lab-frame phase speeds (forward, backward) of light in matter of rest
    index n moving at beta: relativistic velocity addition."""
    fwd = (1.0 / n_rest + beta) / (1.0 + beta / n_rest)
    bwd = (1.0 / n_rest - beta) / (1.0 - beta / n_rest)
    return fwd, bwd


# --------------------------------------------------------------------------
# Pulse spectra (App. B.1)
# --------------------------------------------------------------------------

def gaussian_spectrum_peak(omega_i: float, a: float) -> float:
    """Centre frequency of a scattered copy of a pulse with carrier
    omega_i compressed by the factor a (eq. (spectrum_scat_interface))."""
    return a * omega_i
