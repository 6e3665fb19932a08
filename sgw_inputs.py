"""Seeded synthetic workloads shared by the GPU library's tests/benchmark and the oracle.

This module holds problem *descriptions* only (sizes, domains, coefficients,
seeds) and no arithmetic of the method: each side turns a ``Problem`` into its
own structures and evaluates the initial condition itself.

Workloads (all analytic, as in the paper's Sec. 3; no dataset is involved):

* ``c1_advection_2d``  2D linear advection u_t+u_x+u_y=0 on [0,2]^2, u0=sin(pi(x+y)), T=1,
  root 4x4, finest level 3 (32x32), CFL 0.5.
* ``c2_burgers_2d``    2D Burgers on [-1,1]^2, u0=0.3+0.7 sin(pi(x+y)), T=0.5/pi^2 or 1.5/pi^2,
  root 8x8, finest level 5 (256x256), CFL 0.5.
* ``c3_advection_3d``  3D linear advection on [0,2]^3, u0=sin(pi(x+y+z)), T=1, root 8^3, level 5.
* ``c4_vlasov_4d``     4D phase-space Vlasov with the fixed field E=0.01(sin(x1/2), sin(x2/2)),
  x in [0,4pi]^2, v in [-6,6]^2 (periodic), f0 = Maxwellian (1+0.01 cos(x1/2) cos(x2/2)),
  root 8^4, level 4, CFL 0.4, T=1.
* the paper's Example 1 (2D advection, linear scheme, dt = dx^(5/3)) and Example 3(a)
  (2D Burgers, dt = dx^(5/3)) for the pins.
* ``serving_stream``   a seeded Poisson-arrival stream of mixed solves.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

FLUX_ADVECTION = 0
FLUX_BURGERS = 1
FLUX_VLASOV = 2
FLUX_VLASOV_HARMONIC = 3
FLUX_VLASOV_MAXWELL = 4

IC_SINE = 0
IC_MAXWELL_COS = 1
IC_VB = 2
IC_VM = 3

DT_CFL = 0
DT_POW53 = 1

PROLONG_WENO5 = 0
PROLONG_LAGRANGE5 = 1

PREC_FP64 = 0
PREC_FP32 = 1

BC_PERIODIC = 0
BC_ZERO = 1


@dataclasses.dataclass
class Problem:
    """One sparse-grid solve: PDE, initial condition, grids and time-stepping."""
    d: int
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]
    flux: int
    flux_params: Tuple[float, ...]
    ic: int
    ic_params: Tuple[float, ...]
    nr: int
    nl: int
    T: float
    cfl: float = 0.5
    dt_mode: int = DT_CFL
    prolong: int = PROLONG_WENO5
    linear: bool = False
    precision: int = PREC_FP64
    # epsilon of the flux and interpolation weights, eqs. (2.6) and (eqnlnwe); the paper's
    # printed WENO errors (Tables ex3aweno, ex3-baweno) are reproduced with 1e-3 in both.
    eps_flux: float = 1e-3
    eps_interp: float = 1e-3
    name: str = ""
    # boundary condition per direction: 0 periodic, 1 zero values beyond both ends
    bc: Tuple[int, ...] = ()
    # relaxation source (mu_inf(v) rho(x) - f) / tau of the Vlasov-Boltzmann model (off at tau 0)
    # and the kinetic temperature theta of mu_inf
    relax_tau: float = 0.0
    relax_theta: float = 1.0

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)

    @property
    def n_fine(self) -> int:
        return self.nr << self.nl


def _pad4(v, fill=0.0):
    v = list(v)
    return tuple(v + [fill] * (4 - len(v)))


def c1_advection_2d(nr: int = 4, nl: int = 3, precision: int = PREC_FP64) -> Problem:
    return Problem(d=2, lo=(0.0, 0.0), hi=(2.0, 2.0), flux=FLUX_ADVECTION, flux_params=(1.0, 1.0),
                   ic=IC_SINE, ic_params=(0.0, 1.0, math.pi, 0.0), nr=nr, nl=nl, T=1.0, cfl=0.5,
                   precision=precision, name="c1_advection_2d")


def c2_burgers_2d(nr: int = 8, nl: int = 5, T: float = 1.5 / math.pi ** 2,
                  precision: int = PREC_FP32) -> Problem:
    return Problem(d=2, lo=(-1.0, -1.0), hi=(1.0, 1.0), flux=FLUX_BURGERS, flux_params=(),
                   ic=IC_SINE, ic_params=(0.3, 0.7, math.pi, 0.0), nr=nr, nl=nl, T=T, cfl=0.5,
                   precision=precision, name="c2_burgers_2d")


def c3_advection_3d(nr: int = 8, nl: int = 5, precision: int = PREC_FP64, T: float = 1.0) -> Problem:
    return Problem(d=3, lo=(0.0,) * 3, hi=(2.0,) * 3, flux=FLUX_ADVECTION, flux_params=(1.0, 1.0, 1.0),
                   ic=IC_SINE, ic_params=(0.0, 1.0, math.pi, 0.0), nr=nr, nl=nl, T=T, cfl=0.5,
                   precision=precision, name="c3_advection_3d")


def c4_vlasov_4d(nr: int = 8, nl: int = 4, precision: int = PREC_FP32, T: float = 1.0) -> Problem:
    four_pi = 4.0 * math.pi
    return Problem(d=4, lo=(0.0, 0.0, -6.0, -6.0), hi=(four_pi, four_pi, 6.0, 6.0), flux=FLUX_VLASOV,
                   flux_params=(0.01, 0.5), ic=IC_MAXWELL_COS, ic_params=(0.01, 0.5, 0.0, 0.0),
                   nr=nr, nl=nl, T=T, cfl=0.4, precision=precision, name="c4_vlasov_4d")


def paper_example1(n_h: int, nr: Optional[int] = None, nl: int = 0) -> Problem:
    """Example 1 of Sec. 3.1: u_t+u_x+u_y=0, u0=0.3+0.7 sin(pi/2 (x+y)) on [0,4]^2, T=0.5,
    linear scheme, dt = dx^(5/3).  Single grid: nr = n_h, nl = 0."""
    if nr is None:
        nr = n_h >> nl
    return Problem(d=2, lo=(0.0, 0.0), hi=(4.0, 4.0), flux=FLUX_ADVECTION, flux_params=(1.0, 1.0),
                   ic=IC_SINE, ic_params=(0.3, 0.7, math.pi / 2, 0.0), nr=nr, nl=nl, T=0.5,
                   dt_mode=DT_POW53, linear=True, prolong=PROLONG_LAGRANGE5, name="paper_example1")


def paper_example3a(n_h: int, nr: Optional[int] = None, nl: int = 0, linear: bool = False,
                    prolong: int = PROLONG_WENO5) -> Problem:
    """Example 3(a) of Sec. 3.2: 2D Burgers, u0 = 1 + sin(x+y)/2 on [0,2pi]^2, T=0.3, dt = dx^(5/3)."""
    if nr is None:
        nr = n_h >> nl
    two_pi = 2.0 * math.pi
    return Problem(d=2, lo=(0.0, 0.0), hi=(two_pi, two_pi), flux=FLUX_BURGERS, flux_params=(),
                   ic=IC_SINE, ic_params=(1.0, 0.5, 1.0, 0.0), nr=nr, nl=nl, T=0.3, dt_mode=DT_POW53,
                   linear=linear, prolong=prolong, name="paper_example3a")


def paper_example3b(n_h: int, nr: Optional[int] = None, nl: int = 0, linear: bool = False,
                    prolong: int = PROLONG_WENO5) -> Problem:
    """Example 3(b): 3D Burgers, u0 = 1 + sin(x+y+z)/2 on [0,2pi]^3, T=0.1, dt = dx^(5/3)."""
    if nr is None:
        nr = n_h >> nl
    two_pi = 2.0 * math.pi
    return Problem(d=3, lo=(0.0,) * 3, hi=(two_pi,) * 3, flux=FLUX_BURGERS, flux_params=(),
                   ic=IC_SINE, ic_params=(1.0, 0.5, 1.0, 0.0), nr=nr, nl=nl, T=0.1, dt_mode=DT_POW53,
                   linear=linear, prolong=prolong, name="paper_example3b")


def _simpson(f, a: float, b: float, n: int = 1 << 20) -> float:
    x = np.linspace(a, b, n + 1)
    w = np.ones(n + 1)
    w[1:-1:2] = 4.0
    w[2:-1:2] = 2.0
    return float((b - a) / (3.0 * n) * np.dot(w, f(x)))


def vb_normalisation(d: int, lo: float = -5.0, hi: float = 5.0) -> float:
    """The constant s of the Vlasov-Boltzmann initial condition: the integral over the domain of
    sin(x_1^2/2)^2 [cos(x_2^2/2)^2] exp(-(|x|^2+|v|^2)/2), a product of one-dimensional integrals
    taken by composite Simpson on 2^20 intervals."""
    ix1 = _simpson(lambda x: np.sin(0.5 * x * x) ** 2 * np.exp(-0.5 * x * x), lo, hi)
    ix2 = _simpson(lambda x: np.cos(0.5 * x * x) ** 2 * np.exp(-0.5 * x * x), lo, hi)
    iv = math.sqrt(2.0 * math.pi) * math.erf(hi / math.sqrt(2.0))
    return ix1 * iv if d == 2 else ix1 * ix2 * iv * iv


def paper_example5(d: int = 2, nr: Optional[int] = None, nl: int = 3, T: float = 0.5,
                   precision: int = PREC_FP64) -> Problem:
    """Example 5 of Sec. 3.4, the Vlasov-Boltzmann transport equation with E = -x and the linear
    relaxation source, theta = tau = 1, on [-5,5]^d with zero boundary values, CFL 0.4:
    (a) d = 2 on a 40^2 root grid, (b) d = 4 on a 10^4 root grid, finest level 3."""
    if nr is None:
        nr = 40 if d == 2 else 10
    return Problem(d=d, lo=(-5.0,) * d, hi=(5.0,) * d, flux=FLUX_VLASOV_HARMONIC, flux_params=(),
                   ic=IC_VB, ic_params=(1.0 / vb_normalisation(d),), nr=nr, nl=nl, T=T, cfl=0.4,
                   precision=precision, bc=(BC_ZERO,) * d, relax_tau=1.0, relax_theta=1.0,
                   name=f"paper_example5_{d}d")


def paper_example6(nr: int = 20, nl: int = 3, T: float = 10.0, precision: int = PREC_FP64,
                   beta: float = 0.01, b: float = 0.001, delta: float = 0.5, v01: float = 0.3, v02: float = 0.3,
                   k0: float = 0.2) -> Problem:
    """Example 6 of Sec. 3.4, the 3D Vlasov-Maxwell system in (x_2, xi_1, xi_2) on
    [0, 2 pi/k0] x [-1.2, 1.2]^2, periodic, CFL 0.4: 20^3 root grid, finest level 3 (160^3)."""
    return Problem(d=3, lo=(0.0, -1.2, -1.2), hi=(2.0 * math.pi / k0, 1.2, 1.2), flux=FLUX_VLASOV_MAXWELL,
                   flux_params=(), ic=IC_VM, ic_params=(beta, b, delta, v01, v02, k0), nr=nr, nl=nl, T=T,
                   cfl=0.4, precision=precision, name="paper_example6")


FAMILIES = {
    1: c1_advection_2d,
    2: c2_burgers_2d,
    3: c3_advection_3d,
    4: c4_vlasov_4d,
}


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    problem: Problem
    family: int


def randomized(family: int, nl: int, rng: np.random.Generator, precision: int = PREC_FP32) -> Problem:
    """A member of workload family 1-4 at finest level nl with a seeded phase/amplitude."""
    phi = float(rng.uniform(0.0, 2.0 * math.pi))
    if family == 1:
        A = float(rng.uniform(0.5, 1.5))
        return c1_advection_2d(nl=nl, precision=precision).replace(ic_params=(0.0, A, math.pi, phi))
    if family == 2:
        A = float(rng.uniform(0.5, 0.9))
        T = 0.5 / math.pi ** 2 if rng.uniform() < 0.5 else 1.5 / math.pi ** 2
        return c2_burgers_2d(nl=nl, precision=precision, T=T).replace(ic_params=(0.3, A, math.pi, phi))
    if family == 3:
        A = float(rng.uniform(0.5, 1.5))
        return c3_advection_3d(nl=nl, precision=precision).replace(ic_params=(0.0, A, math.pi, phi))
    amp = float(rng.uniform(0.005, 0.02))
    phi2 = float(rng.uniform(0.0, 2.0 * math.pi))
    return c4_vlasov_4d(nl=nl, precision=precision).replace(ic_params=(amp, 0.5, phi, phi2))


def serving_stream(n: int = 512, rate_hz: float = 100.0, seed: int = 2007_10196,
                   levels=(2, 3, 4, 5), families=(1, 2, 3, 4), precision: int = PREC_FP32,
                   max_level_by_family=None) -> List[Request]:
    """Poisson arrivals (exponential gaps, rate ``rate_hz``) of solves drawn uniformly from the
    families and levels; request i has its own generator seeded ``seed + 1 + i``."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate_hz))
        fam = int(rng.choice(families))
        nl = int(rng.choice(levels))
        if max_level_by_family and fam in max_level_by_family:
            nl = min(nl, max_level_by_family[fam])
        r = np.random.default_rng(seed + 1 + i)
        out.append(Request(rid=i, arrival_s=t, problem=randomized(fam, nl, r, precision), family=fam))
    return out



def component_noise(total_nodes: int, seed: int = 2007_10196) -> np.ndarray:
    """Seeded uniform values in [0, 1) for every component-grid node (grids back to back in plan
    order): caller-set data that stresses the nonlinear interpolation weights."""
    return np.random.default_rng(seed).random(total_nodes)
