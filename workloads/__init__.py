"""Seeded synthetic inputs for the generalized-FDTD hot path.

This module only *describes* problems: grid size, rest-frame material
profile, velocity, source pulse, probes and step count.  It holds none of
the method's arithmetic, so both the FP64 oracle and the HIP path may take
their inputs from here without sharing any stepping code.

Units are normalised throughout: c = eps0 = mu0 = 1, the cell size is 1 and
time is measured in cell transit times, so the Courant number S is the time
step and beta = v/c.

The workload families follow the structures the paper illustrates in its
Fig. 1 (interface, slab, bilayer crystal, gradient) and validates in
Section 6 (Figs. 5-8), plus the plane waves on rings of the stability
analysis (Section 5, Fig. 4) and multilayer stacks for the transfer-matrix
method (App. B.3); each generator's docstring states its sizes and
distributions.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# Descriptor enumerations.  Their numeric values are the ones the C-ABI
# header and the oracle both accept.
MODULATION = 0      # moving perturbation: isotropic eps(z - vt), mu(z - vt)
MATTER = 1          # moving matter: bianisotropic in the lab frame
F32 = 0
F64 = 1
ABC_MUR1 = 0        # first-order absorbing ends
ABC_PEC = 1         # D = 0 at both end nodes
ABC_PERIODIC = 2    # ring grid: node nz-1 next to node 0

FLAG_RECORD_TRACE = 1
FLAG_ALLOW_UNSTABLE = 2

LAMBDA0 = 40.0      # free-space wavelength of the carrier, in cells
STEADY_COURANT = 0.5


@dataclasses.dataclass
class Pulse:
    """Gaussian-modulated sinusoid, the incident field shape of App. B.1
    (a carrier at omega_i under a Gaussian envelope of width tau_i).

    The sample injected at time t is amp*sin(omega*(t-t0)+phase)*
    exp(-((t-t0)/tau)**2) for t <= t_off and zero afterwards.
    """
    amp: float = 1.0
    omega: float = 2.0 * math.pi / LAMBDA0
    t0: float = 600.0
    tau: float = 150.0
    phase: float = 0.0
    t_off: float = 1200.0


def carrier_pulse(cycles: float = 30.0, lambda0: float = LAMBDA0,
                  phase: float = 0.0, amp: float = 1.0) -> Pulse:
    """A pulse spanning `cycles` carrier periods: centre at half the window,
    envelope width a quarter of that half-window, switched off at the end
    of the window (envelope there is exp(-16))."""
    period = lambda0                      # c = 1, cell = 1
    t0 = 0.5 * cycles * period
    return Pulse(amp=amp, omega=2.0 * math.pi / lambda0, t0=t0,
                 tau=t0 / 4.0, phase=phase, t_off=2.0 * t0)


def default_omegas(omega0: float, nfreq: int = 64,
                   lo: float = 0.5, hi: float = 2.5) -> np.ndarray:
    return omega0 * np.linspace(lo, hi, nfreq)


@dataclasses.dataclass(frozen=True)
class TimeWindow:
    """A moving modulation that exists only for t_on <= t < t_off: before
    and after, the whole grid is the uniform background (eps_bg, mu_bg).
    The switches are temporal interfaces, the corners of the space-time
    slab are where they meet the moving boundaries."""
    t_on: float
    t_off: float
    eps_bg: float = 1.0
    mu_bg: float = 1.0


@dataclasses.dataclass
class Problem:
    """One scattering solve: the quantities the paper's statement of the
    problem involves (Sections 3-4): a 1D grid, the permittivity and
    permeability of the medium at rest, its velocity and kind, a source
    pulse, probes and the number of time steps.

    eps_rest[i] is the rest permittivity of the cell centred on E node i;
    mu_rest[i] the rest permeability of the cell centred on H node i (at
    i + 1/2).  Both arrays have nz entries.
    """
    nz: int
    steps: int
    eps_rest: np.ndarray
    mu_rest: np.ndarray
    courant: float = STEADY_COURANT
    beta: float = 0.0
    kind: int = MODULATION
    precision: int = F64
    src_cell: int = 200
    pulse: Pulse = dataclasses.field(default_factory=Pulse)
    probes: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros(0, dtype=np.int64))
    omegas: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros(0, dtype=np.float64))
    abc: int = ABC_MUR1
    flags: int = 0
    label: str = ""
    # initial state: D at t = S/2 and B at t = 0 (nz values each; on a grid
    # with ends the last B entry is unused); None means zero
    init_d: Optional[np.ndarray] = None
    init_b: Optional[np.ndarray] = None
    # finite-duration modulation (moving modulation only), or None: always
    window: Optional[TimeWindow] = None

    def __post_init__(self):
        self.eps_rest = np.ascontiguousarray(self.eps_rest, dtype=np.float64)
        self.mu_rest = np.ascontiguousarray(self.mu_rest, dtype=np.float64)
        self.probes = np.ascontiguousarray(self.probes, dtype=np.int64)
        self.omegas = np.ascontiguousarray(self.omegas, dtype=np.float64)
        if self.init_d is not None:
            self.init_d = np.ascontiguousarray(self.init_d, dtype=np.float64)
        if self.init_b is not None:
            self.init_b = np.ascontiguousarray(self.init_b, dtype=np.float64)

    @property
    def cell_updates(self) -> int:
        return int(self.nz) * int(self.steps)

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# Profiles (rest frame)
# --------------------------------------------------------------------------

def uniform(nz: int, value: float = 1.0) -> np.ndarray:
    return np.full(nz, float(value))


def interface_profile(nz: int, at: int, eps_left: float,
                      eps_right: float) -> np.ndarray:
    eps = np.full(nz, float(eps_right))
    eps[:at] = eps_left
    return eps


def slab_profile(nz: int, start: int, length: int, eps_slab: float,
                 eps_bg: float = 1.0) -> np.ndarray:
    eps = np.full(nz, float(eps_bg))
    eps[max(0, start):max(0, min(nz, start + length))] = eps_slab
    return eps


def crystal_profile(nz: int, start: int, period: int, nper: int,
                    eps1: float, eps2: float, eps_bg: float = 1.0,
                    fill: Optional[int] = None) -> np.ndarray:
    """Bilayer crystal: layer 1 on the first `fill` cells of each period
    (half the period by default), layer 2 on the rest; clipped to the grid."""
    eps = np.full(nz, float(eps_bg))
    fill = period // 2 if fill is None else fill
    for q in range(nper):
        a = start + q * period
        if a >= nz:
            break
        eps[a:min(nz, a + fill)] = eps1
        eps[min(nz, a + fill):min(nz, a + period)] = eps2
    return eps


def tanh_ramp_profile(nz: int, centre: float, rise_cells: float,
                      eps_lo: float, eps_hi: float) -> np.ndarray:
    """eps(zeta) = eps_lo + (eps_hi-eps_lo)(1+tanh((zeta-centre)/w))/2,
    sampled at the rest cell centres, with w chosen so that the 10-90 %
    rise spans `rise_cells`."""
    w = rise_cells / (2.0 * math.atanh(0.8))
    z = np.arange(nz, dtype=np.float64)
    return eps_lo + (eps_hi - eps_lo) * 0.5 * (1.0 + np.tanh((z - centre) / w))


# --------------------------------------------------------------------------
# Stable-velocity draw
# --------------------------------------------------------------------------

LUMINAL_MARGIN = 0.98


def draw_beta(rng: np.random.Generator, lo: float, hi: float,
              n_max: float) -> float:
    """Draw beta ~ U[lo, hi], redrawing while |beta| * n_max exceeds the
    margin below the luminal limit |beta| n = 1, beyond which the scheme
    with moving modulation is unstable (see the von Neumann analysis of
    Section 5 and App. A; the threshold is checked in the tests)."""
    while True:
        b = float(rng.uniform(lo, hi))
        if abs(b) * n_max <= LUMINAL_MARGIN:
            return b


# --------------------------------------------------------------------------
# Benchmark configurations
# --------------------------------------------------------------------------

def interface_run(seed: int = 0, precision: int = F64) -> Problem:
    """Moving interface, 1D, plain: 2000 cells of lambda0/40, S = 0.5,
    4000 steps; eps 4 medium moving at +0.3c into vacuum, interface at
    cell 1000; source at 200, probes at 100 and 1900.  The seed only sets
    the pulse phase."""
    rng = np.random.default_rng(seed)
    nz = 2000
    pulse = carrier_pulse(phase=float(rng.uniform(0.0, 2.0 * math.pi)))
    return Problem(nz=nz, steps=4000,
                   eps_rest=interface_profile(nz, 1000, 4.0, 1.0),
                   mu_rest=uniform(nz), beta=0.3, precision=precision,
                   src_cell=200, pulse=pulse,
                   probes=np.array([100, 1900]),
                   omegas=default_omegas(pulse.omega), label="interface")


def slab_run(seed: int = 0, precision: int = F64, nz: int = 65536,
             steps: int = 131072, slab: int = 8192) -> Problem:
    """Moving slab, 1D, plain single run: eps_s ~ U[2,9], beta ~ U[-0.6,
    0.6] (stable draw), slab of `slab` cells centred on the grid."""
    rng = np.random.default_rng(seed)
    eps_s = float(rng.uniform(2.0, 9.0))
    beta = draw_beta(rng, -0.6, 0.6, math.sqrt(eps_s))
    phase = float(rng.uniform(0.0, 2.0 * math.pi))
    pulse = carrier_pulse(phase=phase)
    start = nz // 2 - slab // 2
    return Problem(nz=nz, steps=steps,
                   eps_rest=slab_profile(nz, start, slab, eps_s),
                   mu_rest=uniform(nz), beta=beta, precision=precision,
                   src_cell=200, pulse=pulse,
                   probes=np.array([100, nz - 100]),
                   omegas=default_omegas(pulse.omega), label="slab")


def crystal_runs(seed: int = 0, count: int = 4096, precision: int = F32,
                 nz_lo: int = 4096, nz_hi: int = 65536,
                 steps_per_cell: int = 4) -> List[Problem]:
    """Batched moving bilayer crystals: per run, in this draw order,
    nz log-uniform in [nz_lo, nz_hi]; period p ~ U{64..512}; eps1, eps2 ~
    U[1,12]; number of periods P ~ U{10..100}; modulation velocity beta ~
    U[0.1, 0.9] (stable draw); pulse phase.  Crystal starts at nz/4, layer
    1 fills the first half of each period; steps = 4 nz."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        nz = int(round(math.exp(rng.uniform(math.log(nz_lo), math.log(nz_hi)))))
        period = int(rng.integers(64, 513))
        eps1 = float(rng.uniform(1.0, 12.0))
        eps2 = float(rng.uniform(1.0, 12.0))
        nper = int(rng.integers(10, 101))
        beta = draw_beta(rng, 0.1, 0.9, math.sqrt(max(eps1, eps2)))
        phase = float(rng.uniform(0.0, 2.0 * math.pi))
        pulse = carrier_pulse(phase=phase)
        eps = crystal_profile(nz, nz // 4, period, nper, eps1, eps2)
        out.append(Problem(nz=nz, steps=steps_per_cell * nz, eps_rest=eps,
                           mu_rest=uniform(nz), beta=beta,
                           precision=precision, src_cell=200, pulse=pulse,
                           probes=np.array([100, nz - 100]),
                           omegas=default_omegas(pulse.omega, 32),
                           label=f"crystal{r}"))
    return out


def gradient_run(seed: int = 0, precision: int = F32,
                 downscaled: bool = False) -> Problem:
    """Moving gradient in moving matter: tanh permittivity ramp 1 -> 6
    (10-90 % over 2000 cells), beta = 0.5, 2^20 cells and 2^18 steps; the
    downscaled copy has 2^14 cells, 2^12 steps and the ramp scaled by 2^-6.
    256 DFT frequencies around the carrier."""
    rng = np.random.default_rng(seed)
    phase = float(rng.uniform(0.0, 2.0 * math.pi))
    if downscaled:
        nz, steps, centre, rise = 1 << 14, 1 << 12, 512.0, 2000.0 / 64.0
    else:
        nz, steps, centre, rise = 1 << 20, 1 << 18, 32768.0, 2000.0
    pulse = carrier_pulse(phase=phase)
    return Problem(nz=nz, steps=steps,
                   eps_rest=tanh_ramp_profile(nz, centre, rise, 1.0, 6.0),
                   mu_rest=uniform(nz), beta=0.5, kind=MATTER,
                   precision=precision, src_cell=200, pulse=pulse,
                   probes=np.array([100, nz - 100]),
                   omegas=default_omegas(pulse.omega, 256, 0.25, 3.0),
                   label="gradient" + ("_small" if downscaled else ""))


def serving_template(rng: np.random.Generator, nz: int, steps: int,
                     precision: int) -> Problem:
    """One request of the serving mix: a structure drawn uniformly from
    interface / slab / crystal / gradient, scaled to nz."""
    kind_draw = int(rng.integers(0, 4))
    phase = float(rng.uniform(0.0, 2.0 * math.pi))
    pulse = carrier_pulse(phase=phase)
    src = min(200, nz // 4)
    probes = np.array([min(100, src // 2), nz - min(100, src // 2) - 1])
    kind = MODULATION
    if kind_draw == 0:
        eps_in = float(rng.uniform(1.0, 4.0))
        beta = draw_beta(rng, -0.6, 0.6, math.sqrt(max(eps_in, 4.0)))
        eps = interface_profile(nz, nz // 2, 1.0, eps_in)
        label = "interface"
    elif kind_draw == 1:
        eps_s = float(rng.uniform(2.0, 9.0))
        beta = draw_beta(rng, -0.6, 0.6, math.sqrt(eps_s))
        ln = max(1, nz // 8)
        eps = slab_profile(nz, nz // 2 - ln // 2, ln, eps_s)
        label = "slab"
    elif kind_draw == 2:
        period = int(rng.integers(64, 513))
        eps1 = float(rng.uniform(1.0, 12.0))
        eps2 = float(rng.uniform(1.0, 12.0))
        nper = int(rng.integers(10, 101))
        beta = draw_beta(rng, 0.1, 0.9, math.sqrt(max(eps1, eps2)))
        eps = crystal_profile(nz, nz // 4, period, nper, eps1, eps2)
        label = "crystal"
    else:
        beta = 0.5
        kind = MATTER
        rise = max(1.0, 2000.0 * nz / float(1 << 20))
        eps = tanh_ramp_profile(nz, nz / 32.0, rise, 1.0, 6.0)
        label = "gradient"
    return Problem(nz=nz, steps=steps, eps_rest=eps, mu_rest=uniform(nz),
                   beta=beta, kind=kind, precision=precision, src_cell=src,
                   pulse=pulse, probes=probes,
                   omegas=default_omegas(pulse.omega, 32), label=label)


def serving_stream(seed: int, n_requests: int, rate_per_s: float,
                   nz_lo: float = 1e3, nz_hi: float = 1e6,
                   steps_lo: float = 2.0, steps_hi: float = 4.0
                   ) -> List[Tuple[float, Problem]]:
    """Poisson request stream: exponential inter-arrival gaps at
    `rate_per_s`; nz log-uniform in [nz_lo, nz_hi]; steps U[2,4] * nz;
    FP32 or FP64 with probability 1/2 each."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        nz = int(round(math.exp(rng.uniform(math.log(nz_lo), math.log(nz_hi)))))
        steps = int(round(rng.uniform(steps_lo, steps_hi) * nz))
        precision = F32 if rng.uniform() < 0.5 else F64
        out.append((t, serving_template(rng, nz, steps, precision)))
    return out


# --------------------------------------------------------------------------
# Small cases for parity tests
# --------------------------------------------------------------------------

def small_case(nz: int, steps: int, beta: float, kind: int = MODULATION,
               precision: int = F64, seed: int = 0, abc: int = ABC_MUR1,
               structure: str = "slab", nprobe: int = 2,
               nfreq: int = 16) -> Problem:
    """A short seeded run with a random structure, the source near the
    left end and probes spread over the grid; used to compare kernels with
    the oracle on grids that still span several tiles and a ragged tail."""
    rng = np.random.default_rng(seed)
    lam = 20.0
    pulse = Pulse(amp=1.0, omega=2.0 * math.pi / lam, t0=40.0, tau=12.0,
                  phase=float(rng.uniform(0, 2 * math.pi)), t_off=80.0)
    if structure == "slab":
        a = int(rng.integers(nz // 4, nz // 2))
        eps = slab_profile(nz, a, max(1, nz // 4), float(rng.uniform(2.0, 4.0)))
    elif structure == "random":
        eps = rng.uniform(1.0, 3.0, size=nz)
    elif structure == "crystal":
        eps = crystal_profile(nz, nz // 4, 16, max(1, nz // 32), 1.5, 3.5)
    else:
        eps = uniform(nz)
    mu = uniform(nz) if kind == MATTER else rng.uniform(1.0, 1.5, size=nz)
    nmax = math.sqrt(float(np.max(eps)) * float(np.max(mu)))
    if abs(beta) * nmax > LUMINAL_MARGIN:
        beta = math.copysign(LUMINAL_MARGIN / nmax * 0.95, beta)
    src = max(1, min(nz - 2, nz // 8))
    probes = np.unique(np.clip(
        np.array([0, src + 1, nz // 2, nz - 1, nz - 3][:max(1, nprobe)]),
        0, nz - 1))
    return Problem(nz=nz, steps=steps, eps_rest=eps, mu_rest=mu,
                   courant=0.5, beta=beta, kind=kind, precision=precision,
                   src_cell=src, pulse=pulse, probes=probes,
                   omegas=default_omegas(pulse.omega, nfreq), abc=abc,
                   label=f"small_{structure}")


def random_fields(nz: int, seed: int, scale: float = 1.0
                  ) -> Tuple[np.ndarray, np.ndarray]:
    """Seeded smooth random initial fields (D, B): a sum of a few long
    waves plus small white noise, for runs that start from a non-zero
    state."""
    rng = np.random.default_rng(seed)
    k = np.arange(nz, dtype=np.float64)
    d = np.zeros(nz)
    b = np.zeros(nz)
    for _ in range(4):
        kz = 2.0 * math.pi * rng.uniform(0.005, 0.2)
        d += rng.normal() * np.cos(kz * k + rng.uniform(0, 2 * math.pi))
        b += rng.normal() * np.cos(kz * (k + 0.5) + rng.uniform(0, 2 * math.pi))
    d += 0.05 * rng.normal(size=nz)
    b += 0.05 * rng.normal(size=nz)
    return scale * d, scale * b


# --------------------------------------------------------------------------
# Plane waves on rings: the stability / dispersion sweep (Section 5, Fig. 4)
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class DispersionPoint:
    """One point of the sweep: a uniform medium (eps' = eps, mu' = mu) on a
    ring of nz cells moving at beta, time step S, and the plane wave with
    m wavelengths around the ring, k_z dz = 2 pi m / nz, i.e. a meshing
    density N_lambda = nz / m cells per wavelength."""
    courant: float
    beta: float
    eps: float
    nz: int
    m: int
    mu: float = 1.0
    kind: int = MODULATION

    @property
    def theta(self) -> float:
        return 2.0 * math.pi * self.m / self.nz

    @property
    def n_lambda(self) -> float:
        return self.nz / self.m


def fig4_points(courant: float = 0.5, beta: float = 0.3, eps: float = 4.0,
                max_nz: int = 64) -> List[DispersionPoint]:
    """The setting of the paper's stability figure: S = 0.5, beta = 0.3,
    eps = 4, mu = 1, swept over meshing densities N_lambda = nz/m on rings
    of 8..max_nz cells (one point per distinct N_lambda, m < nz/2)."""
    seen = {}
    for nz in range(8, max_nz + 1):
        for m in range(1, (nz - 1) // 2 + 1):
            key = round(nz / m, 9)
            if key not in seen:
                seen[key] = DispersionPoint(courant, beta, eps, nz, m)
    return [seen[k] for k in sorted(seen)]


def dispersion_points(seed: int, count: int, max_nz: int = 256,
                      kinds=(MODULATION,)) -> List[DispersionPoint]:
    """Seeded random sweep points.  Drawn in order: S ~ U[0.05, 0.95],
    eps ~ U[1, 9], beta ~ U[-0.9, 0.9], nz ~ U{8..max_nz}, m ~
    U{1..(nz-1)//2}, kind uniform over `kinds`; a draw is repeated while
    |beta| n > 0.98 or S > 0.98 n / (1 + n |beta|) (n = sqrt(eps)), the
    luminal and Courant-type limits the stability analysis gives."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        S = float(rng.uniform(0.05, 0.95))
        eps = float(rng.uniform(1.0, 9.0))
        beta = float(rng.uniform(-0.9, 0.9))
        nz = int(rng.integers(8, max_nz + 1))
        m = int(rng.integers(1, (nz - 1) // 2 + 1))
        kind = int(kinds[int(rng.integers(0, len(kinds)))])
        n = math.sqrt(eps)
        if abs(beta) * n > LUMINAL_MARGIN or S > LUMINAL_MARGIN * n / (1.0 + n * abs(beta)):
            continue
        out.append(DispersionPoint(S, beta, eps, nz, m, 1.0, kind))
    return out


def dispersion_runs(points, steps: int, precision: int = F64) -> List[Problem]:
    """Two ring runs per point, no source, no probes, starting from a
    cosine in one field: D_k = cos(theta k), B = 0, and D = 0,
    B_j = cos(theta (j + 1/2)) (B lives at j + 1/2).  After `steps` steps
    the theta components of (D, B) of the two runs are the columns of the
    steps-th power of the one-step amplification matrix."""
    runs = []
    for i, pt in enumerate(points):
        k = np.arange(pt.nz, dtype=np.float64)
        cd = np.cos(pt.theta * k)
        cb = np.cos(pt.theta * (k + 0.5))
        zero = np.zeros(pt.nz)
        base = dict(nz=pt.nz, steps=steps, eps_rest=np.full(pt.nz, pt.eps),
                    mu_rest=np.full(pt.nz, pt.mu), courant=pt.courant,
                    beta=pt.beta, kind=pt.kind, precision=precision,
                    src_cell=0, pulse=Pulse(amp=0.0), abc=ABC_PERIODIC)
        runs.append(Problem(**base, init_d=cd, init_b=zero, label=f"disp{i}_d"))
        runs.append(Problem(**base, init_d=zero, init_b=cb, label=f"disp{i}_b"))
    return runs


# --------------------------------------------------------------------------
# Transfer-matrix sweeps (App. B.3): uniform moving multilayers in the
# frequency domain
# --------------------------------------------------------------------------

@dataclasses.dataclass
class TmmStack:
    """Layers 0..N-1 moving at beta (0 and N-1 semi-infinite); widths of
    the inner layers in cells (lab frame)."""
    eps: np.ndarray
    widths: np.ndarray
    beta: float
    mu: Optional[np.ndarray] = None


def tmm_crystals(seed: int, count: int, nomega: int = 256
                 ) -> Tuple[List[TmmStack], np.ndarray]:
    """Seeded bilayer crystals in vacuum, drawn like the batched FDTD
    crystals: eps1, eps2 ~ U[1, 12], period p ~ U{16..128} cells split in
    half, P ~ U{5..100} periods, beta ~ U[-0.9, 0.9] redrawn while
    |beta| sqrt(max eps) > 0.98; and nomega angular frequencies spread over
    [0.2, 3] omega0 (omega0 = 2 pi / 40)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        e1, e2 = (float(x) for x in rng.uniform(1.0, 12.0, size=2))
        p = int(rng.integers(16, 129))
        P = int(rng.integers(5, 101))
        beta = float(rng.uniform(-0.9, 0.9))
        nmax = math.sqrt(max(e1, e2))
        while abs(beta) * nmax > LUMINAL_MARGIN:
            beta = float(rng.uniform(-0.9, 0.9))
        eps = np.array([1.0] + [e1, e2] * P + [1.0])
        widths = np.array([p // 2, p - p // 2] * P, dtype=np.float64)
        out.append(TmmStack(eps=eps, widths=widths, beta=beta))
    omega0 = 2.0 * math.pi / LAMBDA0
    return out, np.linspace(0.2 * omega0, 3.0 * omega0, nomega)


# --------------------------------------------------------------------------
# 2D runs: TE / TM in the (x, z) plane, motion along z, a stratified
# moving modulation (interfaces normal to the velocity, as Section 3
# assumes), x periodic
# --------------------------------------------------------------------------

TE = 0              # E_y, H_x, H_z
TM = 1              # H_y, E_x, E_z


@dataclasses.dataclass
class Problem2D:
    """One 2D solve.  Columns i = 0..nx-1 along x (periodic), z nodes as in
    the 1D grid.  The modulation is stratified: eps_rest and mu_rest hold
    one value per rest cell along z (nz entries each, the same cells as in
    1D).  The source is a line along x at z node src_row: src_profile[i] times
    the pulse, added to the D component of the 1D pair (D_y for TE, D_x for
    TM).  Probes sit at (probe_x[q], probe_z[q]).

    Field arrays (init_* and results) are (nx, nz), row i = column i of the
    grid:  TE  D = D_y(i, k),  B = B_x(i, k+1/2),  C = B_z(i+1/2, k);
           TM  D = D_x(i+1/2, k),  B = B_y(i+1/2, k+1/2),  C = D_z(i, k+1/2).
    On a grid with ends the last entry of each row of B (and of C for TM)
    is unused."""
    pol: int
    nx: int
    nz: int
    steps: int
    eps_rest: np.ndarray
    mu_rest: np.ndarray
    courant: float = STEADY_COURANT
    beta: float = 0.0
    precision: int = F64
    src_row: int = 200
    src_profile: Optional[np.ndarray] = None
    pulse: Pulse = dataclasses.field(default_factory=Pulse)
    probe_x: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros(0, dtype=np.int64))
    probe_z: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros(0, dtype=np.int64))
    omegas: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros(0, dtype=np.float64))
    abc: int = ABC_MUR1
    flags: int = 0
    label: str = ""
    init_d: Optional[np.ndarray] = None
    init_b: Optional[np.ndarray] = None
    init_c: Optional[np.ndarray] = None

    def __post_init__(self):
        self.eps_rest = np.ascontiguousarray(self.eps_rest, dtype=np.float64)
        self.mu_rest = np.ascontiguousarray(self.mu_rest, dtype=np.float64)
        if self.src_profile is None:
            self.src_profile = np.ones(self.nx)
        self.src_profile = np.ascontiguousarray(self.src_profile, dtype=np.float64)
        self.probe_x = np.ascontiguousarray(self.probe_x, dtype=np.int64)
        self.probe_z = np.ascontiguousarray(self.probe_z, dtype=np.int64)
        self.omegas = np.ascontiguousarray(self.omegas, dtype=np.float64)
        for k in ("init_d", "init_b", "init_c"):
            a = getattr(self, k)
            if a is not None:
                setattr(self, k, np.ascontiguousarray(
                    np.reshape(a, (self.nx, self.nz)), dtype=np.float64))

    @property
    def cell_updates(self) -> int:
        return int(self.nx) * int(self.nz) * int(self.steps)

    def replace(self, **kw) -> "Problem2D":
        return dataclasses.replace(self, **kw)


def oblique_profile(nx: int, m: int, pol: int, phase: float = 0.0) -> np.ndarray:
    """Line-source profile cos(2 pi m x / nx + phase) sampled where the
    sourced component lives: x = i (TE, D_y) or x = i + 1/2 (TM, D_x).  It
    launches the +-k_x pair of waves at sin(theta) = k_x / (n omega) with
    k_x = 2 pi m / nx."""
    x = np.arange(nx, dtype=np.float64) + (0.5 if pol == TM else 0.0)
    return np.cos(2.0 * math.pi * m * x / nx + phase)


COURANT_2D = 0.25


def slab_run_2d(seed: int = 0, pol: int = TE, precision: int = F32,
                nx: int = 4096, nz: int = 4096, steps: int = 4096,
                slab: int = 1024) -> Problem2D:
    """Moving slab in 2D: nx x nz cells (x periodic), S = 0.25, eps_s ~
    U[2, 9], beta ~ U[-0.6, 0.6] (stable draw), a slab of `slab` cells
    starting at nz/4 - 256 along z; a 10-cycle carrier pulse (lambda0 = 40
    cells) from a line source at z node 200 with an oblique profile of
    m ~ U{1..nx/64} periods across x (up to 0.63 of the carrier's free-space
    wavenumber), probes at z = 100 and nz - 100 on four columns each.  The
    duration (steps S = 1024 at the defaults) carries the pulse across the
    slab."""
    rng = np.random.default_rng(seed)
    eps_s = float(rng.uniform(2.0, 9.0))
    beta = draw_beta(rng, -0.6, 0.6, math.sqrt(eps_s))
    phase = float(rng.uniform(0.0, 2.0 * math.pi))
    m = int(rng.integers(1, max(2, nx // 64) + 1))
    pulse = carrier_pulse(cycles=10.0, phase=phase)
    start = max(0, nz // 4 - 256)
    px = np.array([0, nx // 4, nx // 2, 3 * nx // 4] * 2, dtype=np.int64)
    pz = np.array([100] * 4 + [nz - 100] * 4, dtype=np.int64)
    return Problem2D(pol=pol, nx=nx, nz=nz, steps=steps,
                     eps_rest=slab_profile(nz, start, slab, eps_s),
                     mu_rest=uniform(nz), courant=COURANT_2D, beta=beta,
                     precision=precision, src_row=200,
                     src_profile=oblique_profile(nx, m, pol),
                     pulse=pulse, probe_x=px, probe_z=pz,
                     omegas=default_omegas(pulse.omega, 32),
                     label=f"slab2d_{'te' if pol == TE else 'tm'}")


def small_case_2d(nx: int, nz: int, steps: int, beta: float, pol: int = TE,
                  precision: int = F64, seed: int = 0, abc: int = ABC_MUR1,
                  m: int = 1, structure: str = "slab",
                  nfreq: int = 8) -> Problem2D:
    """A short seeded 2D run for parity tests: S = 0.25, random stratified
    eps (slab or random cells) and mu ~ U[1, 1.5] per cell, an oblique line
    source near the lower z end, probes spread over both axes."""
    rng = np.random.default_rng(seed)
    lam = 20.0
    pulse = Pulse(amp=1.0, omega=2.0 * math.pi / lam, t0=40.0, tau=12.0,
                  phase=float(rng.uniform(0, 2 * math.pi)), t_off=80.0)
    if structure == "slab":
        a = int(rng.integers(nz // 4, nz // 2))
        eps = slab_profile(nz, a, max(1, nz // 4), float(rng.uniform(2.0, 4.0)))
    elif structure == "random":
        eps = rng.uniform(1.0, 3.0, size=nz)
    else:
        eps = uniform(nz)
    mu = rng.uniform(1.0, 1.5, size=nz)
    nmax = math.sqrt(float(np.max(eps)) * float(np.max(mu)))
    if abs(beta) * nmax > LUMINAL_MARGIN:
        beta = math.copysign(LUMINAL_MARGIN / nmax * 0.95, beta)
    src = max(1, min(nz - 2, nz // 8))
    pz = np.clip(np.array([0, src + 1, nz // 2, nz - 1, nz - 3]), 0, nz - 1)
    px = np.array([0, nx - 1, nx // 2, 1 % nx, nx // 3])
    return Problem2D(pol=pol, nx=nx, nz=nz, steps=steps, eps_rest=eps,
                     mu_rest=mu, courant=COURANT_2D, beta=beta, precision=precision,
                     src_row=src, src_profile=oblique_profile(nx, m, pol),
                     pulse=pulse, probe_x=px, probe_z=pz,
                     omegas=default_omegas(pulse.omega, nfreq), abc=abc,
                     label=f"small2d_{structure}")
