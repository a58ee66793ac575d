"""Seeded synthetic inputs for the as-S_N explicit step.

This module only *describes problems*: grids, per-cell material fields, the
initial angular flux and random states.  It holds none of the method's
arithmetic (no quadrature, no scattering kernel, no time step, no update).
Both the FP64 oracle tests and the HIP path take their inputs from here, so
the two sides see bit-identical FP32 inputs and nothing else in common.

Problems (paper, Section 4):
  * line source (Section 4.1): isotropic narrow Gaussian pulse
    psi0 = max(1e-4, exp(-|x|^2 / (4 delta)) / (4 pi delta)), delta = 0.03^2,
    on [-1.5, 1.5]^2 with sigma_s = sigma_t = 1;
  * lattice / checkerboard (Section 4.2, material table): 7 x 7 cm domain of
    1 x 1 blocks; absorbers sigma_a = 10, scatterers sigma_s = 1, and a unit
    isotropic source in the centre block, vacuum boundaries, t_end = 3.2.
    The layout figure is not available; blocks (I, J) with I + J even are
    absorbers, the centre block (3, 3) is absorber + source.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

LINE_SOURCE_DELTA = 0.03 ** 2
LINE_SOURCE_FLOOR = 1.0e-4


@dataclasses.dataclass
class Problem:
    """One as-S_N solve: uniform grid, product quadrature order, fields, IC."""

    name: str
    nx: int
    ny: int
    x_min: float
    x_max: float
    y_min: float
    y_max: float
    n_polar: int
    n_azim: int
    sigma_s: np.ndarray          # float32 [ny, nx]
    sigma_a: np.ndarray          # float32 [ny, nx]
    sigma_as: np.ndarray         # float32 [ny, nx]
    source: np.ndarray           # float32 [ny, nx], isotropic per-steradian q
    psi0_cell: np.ndarray        # float32 [ny, nx], isotropic initial psi
    beta: float = 4.5            # kernel width constant, eps = beta / Q
    t_final: float = 1.0
    cfl: float = 0.95
    ico_order: int = 0           # > 0: icosahedron quadrature of this order instead

    @property
    def q(self) -> int:
        if self.ico_order:
            return 10 * (self.ico_order - 1) ** 2 + 2
        return self.n_polar * self.n_azim

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def psi0(self) -> np.ndarray:
        """Full initial state float32 [Q, ny, nx] (same value for every ordinate)."""
        return np.broadcast_to(self.psi0_cell, (self.q, self.ny, self.nx)).astype(np.float32)


def _cell_centres(n_lo: float, n_hi: float, n: int) -> np.ndarray:
    h = (n_hi - n_lo) / n
    return n_lo + (np.arange(n, dtype=np.float64) + 0.5) * h


def line_source(n: int, n_polar: int = 8, n_azim: Optional[int] = None,
                sigma_as: float = 1.0, sigma_s: float = 1.0, sigma_a: float = 0.0,
                t_final: float = 1.0, beta: float = 4.5, cfl: float = 0.95,
                half_width: float = 1.5, delta: float = LINE_SOURCE_DELTA,
                floor: float = LINE_SOURCE_FLOOR) -> Problem:
    """Line-source problem on [-half_width, half_width]^2 with n x n cells.

    The initial pulse is point-sampled at cell centres (paper Section 4.1).
    """
    n_azim = 2 * n_polar if n_azim is None else n_azim
    xc = _cell_centres(-half_width, half_width, n)
    r2 = xc[None, :] ** 2 + xc[:, None] ** 2
    pulse = np.exp(-r2 / (4.0 * delta)) / (4.0 * math.pi * delta)
    psi0 = np.maximum(floor, pulse).astype(np.float32)
    full = lambda v: np.full((n, n), v, dtype=np.float32)
    return Problem(name=f"line_source_{n}_q{n_polar * n_azim}", nx=n, ny=n,
                   x_min=-half_width, x_max=half_width, y_min=-half_width, y_max=half_width,
                   n_polar=n_polar, n_azim=n_azim,
                   sigma_s=full(sigma_s), sigma_a=full(sigma_a), sigma_as=full(sigma_as),
                   source=full(0.0), psi0_cell=psi0, beta=beta, t_final=t_final, cfl=cfl)


def checkerboard(n: int, n_polar: int = 24, n_azim: Optional[int] = None,
                 sigma_as: float = 5.0, t_final: float = 3.2, beta: float = 4.5,
                 cfl: float = 0.95, source_total: float = 1.0) -> Problem:
    """Lattice problem on [0, 7]^2 with n x n cells; each cell takes its centre's block.

    The total isotropic emission rate per unit area in the centre block is
    ``source_total``; the per-steradian source is that over 4 pi.
    """
    n_azim = 2 * n_polar if n_azim is None else n_azim
    xc = _cell_centres(0.0, 7.0, n)
    bi = np.floor(xc).astype(np.int64)
    I = bi[None, :]
    J = bi[:, None]
    absorber = ((I + J) % 2 == 0)
    centre = (I == 3) & (J == 3)
    sig_a = np.where(absorber, 10.0, 0.0).astype(np.float32)
    sig_s = np.where(absorber, 0.0, 1.0).astype(np.float32)
    src = np.where(centre, source_total / (4.0 * math.pi), 0.0).astype(np.float32)
    return Problem(name=f"checkerboard_{n}_q{n_polar * n_azim}", nx=n, ny=n,
                   x_min=0.0, x_max=7.0, y_min=0.0, y_max=7.0,
                   n_polar=n_polar, n_azim=n_azim,
                   sigma_s=sig_s, sigma_a=sig_a,
                   sigma_as=np.full((n, n), sigma_as, dtype=np.float32),
                   source=src, psi0_cell=np.zeros((n, n), dtype=np.float32),
                   beta=beta, t_final=t_final, cfl=cfl)


def random_problem(seed: int, nx: int, ny: int, n_polar: int = 2, n_azim: int = 4,
                   t_final: float = 0.1, beta: float = 1.5, cfl: float = 0.9,
                   sigma_max: float = 3.0) -> Problem:
    """Random non-negative per-cell fields on a rectangular (possibly ragged) grid."""
    rng = np.random.default_rng(seed)
    f = lambda: (rng.random((ny, nx)) * sigma_max).astype(np.float32)
    return Problem(name=f"random_{nx}x{ny}_s{seed}", nx=nx, ny=ny,
                   x_min=-0.7, x_max=0.5, y_min=0.1, y_max=0.1 + 1.3 * ny / nx,
                   n_polar=n_polar, n_azim=n_azim,
                   sigma_s=f(), sigma_a=f(), sigma_as=f(),
                   source=(rng.random((ny, nx)) * 0.5).astype(np.float32),
                   psi0_cell=rng.random((ny, nx)).astype(np.float32),
                   beta=beta, t_final=t_final, cfl=cfl)


def random_state(seed: int, q: int, ny: int, nx: int, anisotropic: bool = True) -> np.ndarray:
    """Random positive float32 angular flux [q, ny, nx] with a smooth mean and noise."""
    rng = np.random.default_rng(seed)
    base = rng.random((1, ny, nx)) + 0.5
    if not anisotropic:
        return np.broadcast_to(base, (q, ny, nx)).astype(np.float32)
    return (base * (0.5 + rng.random((q, ny, nx)))).astype(np.float32)


@dataclasses.dataclass
class Request:
    """One serving request: a problem and its arrival time (seconds)."""

    rid: int
    kind: str
    n: int
    n_polar: int
    sigma_as: float
    t_final: float
    arrival: float

    def problem(self) -> Problem:
        if self.kind == "line":
            return line_source(self.n, n_polar=self.n_polar, sigma_as=self.sigma_as,
                               t_final=self.t_final)
        return checkerboard(self.n, n_polar=self.n_polar, sigma_as=self.sigma_as,
                            t_final=self.t_final)


def serving_requests(seed: int = 0, count: int = 512, rate: float = 10.0,
                     n_range=(64, 512), polar_orders=(8, 12, 16, 24),
                     sigma_as_range=(0.0, 5.0), t_range=(0.5, 3.2)) -> List[Request]:
    """Seeded request stream: uniform kinds/sizes/orders/strengths, Poisson arrivals."""
    rng = np.random.default_rng(seed)
    arrivals = np.random.default_rng([seed, 1])     # separate stream: same requests at any rate
    reqs = []
    t = 0.0
    for rid in range(count):
        t += arrivals.exponential(1.0 / rate) if rate > 0 else 0.0
        kind = "line" if rng.random() < 0.5 else "checker"
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        n_p = int(polar_orders[int(rng.integers(0, len(polar_orders)))])
        s_as = float(rng.uniform(*sigma_as_range))
        tf = float(rng.uniform(*t_range))
        reqs.append(Request(rid=rid, kind=kind, n=n, n_polar=n_p, sigma_as=s_as,
                            t_final=tf, arrival=t))
    return reqs
