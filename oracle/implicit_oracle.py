"""Plain FP64 reference for the implicit as-S_N scheme (TEST INFRASTRUCTURE ONLY).

Imported by the tests and nothing else.  It follows Camminady, Frank, Hauck and
Kusch (arXiv:1911.08801), Section 3.4 (implicit Euler, moving the artificial
scattering into the sweep, eq. KrylovFixedPoint), Section 3.5 (second-order
upwind flux without limiter, source iteration = Algorithm 1, the linear system
A phi = b with its left-hand side = Algorithm 2, the Sweeping-Krylov time loop =
Algorithm 3) and Appendix B (L2 stability of the implicit flux).

One implicit step solves, per ordinate q and cell,
    L psi - sigma_s (Phi / W) - sigma_as (K psi)_q = q_src + psi_old / dt,
    L psi = xi d_x psi + eta d_y psi + (sigma_a + sigma_s + sigma_as + 1/dt) psi,
with the x-flux through the face right of cell i equal to 3/2 psi_i - 1/2 psi_{i-1}
for xi > 0 and 3/2 psi_{i+1} - 1/2 psi_{i+2} for xi < 0 (likewise along y), and
two zero ghost cells outside every boundary (vacuum).  Physical scattering is
isotropic, so its moment expansion needs the scalar flux only: M psi = Phi =
sum_q w_q psi_q, and sigma_s O Sigma phi = sigma_s phi / W for every ordinate.

Readings (also listed in the design notes):
  * the source iteration of Algorithm 1 stops once ||psi^(l+1) - psi^(l)||_2 <
    eps c~ with c~ = (1 - T)/T, the absolute test as printed: the a-posteriori
    estimate T/(1-T) ||psi^(l+1) - psi^(l)||_2 of the distance to the fixed point
    is below eps (Section 4.1 sets that estimated error to 1e-4).  The 2-norm is the
    plain Euclidean norm over all ordinates and cells.  The Lipschitz estimate T
    is the a-priori contraction bound max_c sigma_as / (sigma_a + sigma_s +
    sigma_as + 1/dt).  A test relative to the iterate, ... < eps c~
    ||psi^(l+1)||_2, is available as an option (relative=True) for right-hand
    sides whose scale is far from one; it is not the paper's form;
  * the loop is capped at 500 sweeps (the paper states no cap) and then returns
    its last iterate;
  * the final sweep of Algorithm 3 keeps the source q beside psi_old / dt
    (the printed line drops it; the right-hand side b of the same step has it);
  * GMRES stops at a relative residual of its tolerance, restarted every 30
    vectors, initial guess the previous step's scalar flux.
"""
from __future__ import annotations

import math
from typing import Callable, Dict, Optional, Tuple

import numpy as np

from . import asn_oracle as o

FLUX_A = 1.5      # coefficient of the upwind cell in the implicit face flux
FLUX_B = -0.5     # coefficient of the cell two upwind


def total_rate(st: o.Setup, dt: float) -> np.ndarray:
    """sigma_t of L: sigma_a + sigma_s + sigma_as + 1/dt per cell."""
    return st.sigma_a + st.sigma_s + st.sigma_as + 1.0 / dt


def sweep(R: np.ndarray, st: o.Setup, dt: float) -> np.ndarray:
    """Solve L_Delta psi = R for every ordinate (the transport sweep).

    Per ordinate the grid is mirrored so that the flow points to increasing
    indices; cell (i, j) then depends on (i-1, j), (i-2, j), (i, j-1), (i, j-2)
    only, and the cells of one anti-diagonal i + j = d are solved together.
    """
    Q, ny, nx = R.shape
    sig = total_rate(st, dt)
    out = np.empty_like(R, dtype=np.float64)
    for q in range(Q):
        xi, eta = st.omega[q, 0], st.omega[q, 1]
        r, s = np.asarray(R[q], np.float64), sig
        if xi < 0:
            r, s = r[:, ::-1], s[:, ::-1]
        if eta < 0:
            r, s = r[::-1, :], s[::-1, :]
        ax, ay = abs(xi) / st.dx, abs(eta) / st.dy
        p = np.zeros((ny + 2, nx + 2))           # two zero ghost rows / columns in front
        diag = FLUX_A * (ax + ay) + s
        for d in range(nx + ny - 1):
            j = np.arange(max(0, d - nx + 1), min(ny, d + 1))
            i = d - j
            # L psi_ij = ax (a psi_ij + (b - a) psi_{i-1,j} - b psi_{i-2,j}) + ay (...) + s psi_ij
            rhs = (r[j, i] - ax * ((FLUX_B - FLUX_A) * p[j + 2, i + 1] - FLUX_B * p[j + 2, i])
                   - ay * ((FLUX_B - FLUX_A) * p[j + 1, i + 2] - FLUX_B * p[j, i + 2]))
            p[j + 2, i + 2] = rhs / diag[j, i]
        v = p[2:, 2:]
        if eta < 0:
            v = v[::-1, :]
        if xi < 0:
            v = v[:, ::-1]
        out[q] = v
    return out


def lipschitz_estimate(st: o.Setup, dt: float) -> float:
    """A-priori contraction bound of the source iteration: max sigma_as / sigma_t."""
    return float(np.max(st.sigma_as / total_rate(st, dt)))


def source_iteration(psi0: np.ndarray, R: np.ndarray, st: o.Setup, dt: float,
                     eps: float = 1e-4, max_iter: int = 500,
                     relative: bool = False) -> Tuple[np.ndarray, int]:
    """Algorithm 1: psi^(l+1) = L^-1 (sigma_as K psi^(l) + R) until the estimated
    error T/(1-T) ||psi^(l+1) - psi^(l)||_2 falls below eps (times ||psi^(l+1)||_2
    when relative).  Returns (last iterate, sweeps)."""
    T = lipschitz_estimate(st, dt)
    c = math.inf if T == 0.0 else (1.0 - T) / T
    prev = np.asarray(psi0, np.float64)
    new = sweep(st.sigma_as[None] * o.as_in_scattering(prev, st.K) + R, st, dt)
    it = 1

    def threshold(v):
        return eps * c * (np.linalg.norm(v) if relative else 1.0)

    while np.linalg.norm(new - prev) >= threshold(new) and it < max_iter:
        prev = new
        new = sweep(st.sigma_as[None] * o.as_in_scattering(prev, st.K) + R, st, dt)
        it += 1
    return new, it


def gmres(matvec: Callable[[np.ndarray], np.ndarray], b: np.ndarray, x0: np.ndarray,
          tol: float, restart: int = 30, max_iter: int = 300) -> Tuple[np.ndarray, int]:
    """Restarted GMRES (Arnoldi with modified Gram-Schmidt, Givens rotations).
    Stops when ||b - A x|| <= tol ||b||; returns (x, matrix-vector products)."""
    x = np.asarray(x0, np.float64).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(x), 0
    n_mv = 0
    while n_mv < max_iter:
        r = b - matvec(x)
        n_mv += 1
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            return x, n_mv
        V = [r / beta]
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        k_done = 0
        for k in range(restart):
            w = matvec(V[k])
            n_mv += 1
            for i in range(k + 1):
                H[i, k] = np.dot(w, V[i])
                w = w - H[i, k] * V[i]
            h_next = np.linalg.norm(w)
            H[k + 1, k] = h_next
            for i in range(k):            # previous rotations
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            den = math.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            k_done = k + 1
            if abs(g[k + 1]) <= tol * bnorm or h_next == 0.0 or n_mv >= max_iter:
                break
            V.append(w / h_next)
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        x = x + sum(y[i] * V[i] for i in range(k_done))
        if abs(g[k_done]) <= tol * bnorm:
            return x, n_mv
    return x, n_mv


def implicit_step(psi_old: np.ndarray, st: o.Setup, dt: float, phi_old: Optional[np.ndarray] = None,
                  gmres_tol: float = 1.5e-8, si_eps: float = 1e-4,
                  stats: Optional[Dict[str, int]] = None, si_relative: bool = False):
    """Algorithm 3, one time step: returns (psi_new, phi_new), where phi_new is the
    GMRES solution of A phi = b and psi_new the final source iteration driven by it.
    The scalar flux of the new state is M psi_new; it equals phi_new only when every
    source iteration has converged (their difference is the iteration error)."""
    psi_old = np.asarray(psi_old, np.float64)
    src = st.source[None] + psi_old / dt                 # q~ = q + psi_old / dt
    if phi_old is None:
        phi_old = o.scalar_flux(psi_old, st.w)
    psi_b, n_b = source_iteration(psi_old, np.broadcast_to(src, psi_old.shape), st, dt, si_eps,
                                  relative=si_relative)
    b = o.scalar_flux(psi_b, st.w)
    counts = {"si_sweeps": n_b}

    def lhs(phi):                                         # Algorithm 2
        R = np.broadcast_to((st.sigma_s * phi / st.W)[None], psi_old.shape)
        psi_t, n = source_iteration(psi_old, R, st, dt, si_eps, relative=si_relative)
        counts["si_sweeps"] += n
        return phi - o.scalar_flux(psi_t, st.w)

    shape = phi_old.shape
    x, n_mv = gmres(lambda v: lhs(v.reshape(shape)).ravel(), b.ravel(), phi_old.ravel(), gmres_tol)
    phi_new = x.reshape(shape)
    psi_new, n_f = source_iteration(psi_old, (st.sigma_s * phi_new / st.W)[None] + src, st, dt,
                                    si_eps, relative=si_relative)
    counts["si_sweeps"] += n_f
    counts["gmres_matvecs"] = n_mv
    if stats is not None:
        stats.update(counts)
    return psi_new, phi_new


def implicit_budget(psi_old: np.ndarray, psi_new: np.ndarray, st: o.Setup, dt: float) -> Dict[str, float]:
    """Particle balance of one implicit step, every term at the new level:
    M^{n+1} - M^n = dt (-A - O + S + D) when the system is solved exactly."""
    area = st.dx * st.dy
    phi = o.scalar_flux(psi_new, st.w)
    Q = psi_new.shape[0]
    out = 0.0
    for q in range(Q):
        xi, eta = st.omega[q, 0], st.omega[q, 1]
        p = psi_new[q]
        if xi > 0:
            face = FLUX_A * p[:, -1] + FLUX_B * (p[:, -2] if p.shape[1] > 1 else 0.0)
            out += st.w[q] * st.dy * xi * face.sum()
        elif xi < 0:
            face = FLUX_A * p[:, 0] + FLUX_B * (p[:, 1] if p.shape[1] > 1 else 0.0)
            out += st.w[q] * st.dy * -xi * face.sum()
        if eta > 0:
            face = FLUX_A * p[-1, :] + FLUX_B * (p[-2, :] if p.shape[0] > 1 else 0.0)
            out += st.w[q] * st.dx * eta * face.sum()
        elif eta < 0:
            face = FLUX_A * p[0, :] + FLUX_B * (p[1, :] if p.shape[0] > 1 else 0.0)
            out += st.w[q] * st.dx * -eta * face.sum()
    Y = o.as_in_scattering(psi_new, st.K)
    wq = st.w[:, None, None]
    return {"mass": area * float(o.scalar_flux(psi_old, st.w).sum()),
            "mass_next": area * float(phi.sum()),
            "absorption": area * float(np.sum(st.sigma_a * phi)),
            "outflow": out,
            "source": area * st.W * float(st.source.sum()),
            "as_defect": area * float(np.sum(st.sigma_as * np.sum(wq * (Y - psi_new), axis=0)))}


def run_implicit(problem, dt: float, n_steps: int, mode: str = "sym", gmres_tol: float = 1.5e-8,
                 si_eps: float = 1e-4, psi0: Optional[np.ndarray] = None,
                 si_relative: bool = False):
    """Advance a problem n_steps implicit steps of size dt; returns (psi, setup)."""
    st = o.setup(problem, mode, dt=dt)
    psi = (problem.psi0() if psi0 is None else psi0).astype(np.float64)
    phi = o.scalar_flux(psi, st.w)
    for _ in range(n_steps):
        psi, phi = implicit_step(psi, st, dt, phi, gmres_tol, si_eps, si_relative=si_relative)
    return psi, st
