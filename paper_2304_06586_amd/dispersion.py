"""Amplification factors of the scheme read off simulated plane waves on
rings: the FDTD side of the stability figure (Section 5, Fig. 4).

Each sweep point (workloads.DispersionPoint) is simulated as two ring runs
(workloads.dispersion_runs) that start from a cosine in D or in B.  On a
uniform ring every spatial Fourier component evolves on its own, so after
N steps the theta = k_z dz components of the two final states are the
columns of the N-th power of the one-step 2x2 amplification matrix, in the
basis of D at nodes k and B at nodes k + 1/2 (the plane-wave test field of
eq. (14)).  Its eigenvalues are zeta^N.  The eigenvector whose B/D ratio is
positive is the forward (+z) wave, the co-moving one for beta > 0; the
other is the backward wave.  The attenuation rate Fig. 4 plots is
ln|zeta| / dt with dt = S.

Resolution: the smaller eigenvalue of G^N is known only to about the
field rounding times the larger one, so a point whose modes differ by
many orders of magnitude after N steps cannot give the weaker mode.  Such
a mode is reported as NaN (unresolved) when |lambda_min| / |lambda_max|
falls below `min_ratio` (1e-6 suits FP64 fields, 1e-2 FP32); the stronger
mode is always resolved.  Fewer steps resolve more strongly damped modes.

This is host post-processing of the fields the GPU returned: two dot
products of length nz and a 2x2 eigenproblem per point.
"""
from __future__ import annotations

from typing import Dict, Sequence, Tuple

import numpy as np


def step_matrix_power(point, res_d: Dict[str, np.ndarray],
                      res_b: Dict[str, np.ndarray]) -> np.ndarray:
    """G^N at the point's theta from the final fields of its two runs
    (D-cosine start, B-cosine start)."""
    nz = int(point.nz)
    th = float(point.theta)
    k = np.arange(nz, dtype=np.float64)
    ed = np.exp(-1j * th * k)
    eb = np.exp(-1j * th * (k + 0.5))
    scale = 2.0 / nz             # a cosine's theta component is nz / 2
    return scale * np.array([[res_d["d"] @ ed, res_b["d"] @ ed],
                             [res_d["b"] @ eb, res_b["b"] @ eb]])


def growth_factors(point, res_d: Dict[str, np.ndarray],
                   res_b: Dict[str, np.ndarray], steps: int,
                   min_ratio: float = 1e-6) -> Tuple[float, float]:
    """(|zeta_forward|, |zeta_backward|) per time step at one point; the
    weaker mode is NaN when unresolved (see the module notes)."""
    w, v = np.linalg.eig(step_matrix_power(point, res_d, res_b))
    sign = np.real(v[1] * np.conj(v[0]))      # sign of B/D per eigenvector
    f = int(np.argmax(sign))
    b = 1 - f
    a = np.abs(w)
    z = a ** (1.0 / steps)
    weak = int(np.argmin(a))
    if a[weak] < min_ratio * a[1 - weak]:
        z[weak] = np.nan
    return float(z[f]), float(z[b])


def sweep_growth(points: Sequence, results: Sequence[Dict[str, np.ndarray]],
                 steps: int, min_ratio: float = 1e-6) -> np.ndarray:
    """(len(points), 2) array of (|zeta_forward|, |zeta_backward|) from the
    results of workloads.dispersion_runs(points, steps), in order; NaN
    marks an unresolved weaker mode."""
    out = np.zeros((len(points), 2))
    for i, pt in enumerate(points):
        out[i] = growth_factors(pt, results[2 * i], results[2 * i + 1], steps,
                                min_ratio)
    return out


def attenuation_rate(zeta_abs, courant) -> np.ndarray:
    """alpha = ln|zeta| / dt, dt = S (negative: attenuation)."""
    return np.log(np.asarray(zeta_abs)) / np.asarray(courant)
