"""Plain FP64 reference for the explicit artificial-scattering S_N (as-S_N) step.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It is deliberately
slow and literal: every function follows one passage of Camminady, Frank,
Hauck and Kusch, "Ray effect mitigation for the discrete ordinates method
using artificial scattering" (arXiv:1911.08801), cited by section/equation.

Readings of points the paper leaves open (each also listed in the design notes):
  * time stepping is forward Euler with first-order donor-cell (upwind) fluxes
    on a uniform Cartesian grid; the paper's own explicit scheme, Heun with a
    minmod limiter (described only by reference, Section 3.1), is heun_step,
    with the textbook reading stated where it is defined;
  * the CFL number bounds dt * max_q(|xi_q|/dx + |eta_q|/dy), the stable
    reading for an unsplit 2-D upwind update (Section 4.1 states it as dt/dx);
  * the quadrature is a product Gauss-Legendre (polar) x uniform azimuth set
    with offset 1/2, ordinate q = i * n_azim + k, projected onto x-y (Section 4);
  * the artificial kernel's eq. (5) prefactor cancels under normalisation;
  * normalisation: "row" is the paper's c_q^(eps) (Section 3.2, eq. asSNeq);
    "sym" is a symmetric Sinkhorn scaling whose rows AND w-weighted columns
    sum to one, so the discrete operator conserves particles, the property the
    paper states for the continuous operator (Section 2.3, item 2);
  * physical isotropic scattering uses sigma_s * Phi / W with W = sum_q w_q;
  * vacuum boundaries: zero incoming flux through every boundary face.

Parity status: every function here is pinned by tests/test_oracle_*.py.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np


# ---------------------------------------------------------------------------
# Quadrature (Section 3.1: S_N ordinates and weights; Section 4: 2-D projection)
# ---------------------------------------------------------------------------

def gauss_legendre(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """Gauss-Legendre nodes/weights on [-1, 1] by Golub-Welsch plus Newton polish.

    Nodes are the eigenvalues of the Jacobi matrix of the Legendre three-term
    recurrence; two Newton steps on P_n refine them and the weights follow
    from w = 2 / ((1 - x^2) P_n'(x)^2).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    if n == 1:
        return np.array([0.0]), np.array([2.0])
    k = np.arange(1, n, dtype=np.float64)
    off = k / np.sqrt(4.0 * k * k - 1.0)
    jac = np.diag(off, 1) + np.diag(off, -1)
    x = np.linalg.eigvalsh(jac)
    for _ in range(2):
        p, dp = _legendre_and_derivative(n, x)
        x = x - p / dp
    _, dp = _legendre_and_derivative(n, x)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    return x, w


def _legendre_and_derivative(n: int, x: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    p0 = np.ones_like(x)
    p1 = x.copy()
    for j in range(2, n + 1):
        p0, p1 = p1, ((2 * j - 1) * x * p1 - (j - 1) * p0) / j
    dp = n * (x * p1 - p0) / (x * x - 1.0)
    return p1, dp


def product_quadrature(n_polar: int, n_azim: int) -> Tuple[np.ndarray, np.ndarray]:
    """Ordinates Omega[Q, 3] = (xi, eta, mu) and weights w[Q] summing to 4 pi.

    mu_i are Gauss-Legendre nodes (z axis normal to the grid plane), azimuths
    phi_k = (k + 1/2) 2 pi / n_azim, ordinate index q = i * n_azim + k.
    """
    mu, g = gauss_legendre(n_polar)
    phi = (np.arange(n_azim, dtype=np.float64) + 0.5) * (2.0 * math.pi / n_azim)
    omega = np.zeros((n_polar * n_azim, 3))
    w = np.zeros(n_polar * n_azim)
    for i in range(n_polar):
        s = math.sqrt(1.0 - mu[i] * mu[i])
        for k in range(n_azim):
            q = i * n_azim + k
            omega[q] = (s * math.cos(phi[k]), s * math.sin(phi[k]), mu[i])
            w[q] = g[i] * 2.0 * math.pi / n_azim
    return omega, w


def icosahedron_vertices() -> Tuple[np.ndarray, List[Tuple[int, int, int]]]:
    """Regular icosahedron with a vertex at (0, 0, 1) (Section 3.3) and its 20 faces.

    Vertices: the poles, an upper ring at z = 1/sqrt(5) with azimuths 2 pi k / 5 and a
    lower ring at z = -1/sqrt(5) turned by pi / 5.
    """
    z = 1.0 / math.sqrt(5.0)
    r = 2.0 / math.sqrt(5.0)
    v = [(0.0, 0.0, 1.0)]
    v += [(r * math.cos(2 * math.pi * k / 5), r * math.sin(2 * math.pi * k / 5), z)
          for k in range(5)]
    v += [(r * math.cos(2 * math.pi * k / 5 + math.pi / 5),
           r * math.sin(2 * math.pi * k / 5 + math.pi / 5), -z) for k in range(5)]
    v += [(0.0, 0.0, -1.0)]
    up = lambda k: 1 + k % 5
    lo = lambda k: 6 + k % 5
    faces = []
    for k in range(5):
        faces.append((0, up(k), up(k + 1)))
        faces.append((up(k), lo(k), up(k + 1)))
        faces.append((up(k + 1), lo(k), lo(k + 1)))
        faces.append((11, lo(k + 1), lo(k)))
    return np.array(v), faces


def _spherical_triangle_area(a: np.ndarray, b: np.ndarray, c: np.ndarray) -> float:
    """Area of the spherical triangle a, b, c on the unit sphere (Van Oosterom-Strackee)."""
    num = abs(float(np.dot(a, np.cross(b, c))))
    den = 1.0 + float(np.dot(a, b) + np.dot(b, c) + np.dot(c, a))
    return 2.0 * math.atan2(num, den)


def icosahedron_quadrature(order: int) -> Tuple[np.ndarray, np.ndarray]:
    """Icosahedron quadrature of the given order (Section 3.3), N_q = 10 (order-1)^2 + 2.

    Every face is split into (order-1)^2 triangles by equidistant points on its edges
    and the corresponding interior points; the nodes are projected onto the sphere.
    A node's weight is the area of the spherical polygon that joins the centres
    (normalised vertex means) of the triangles around it.  Ordinates are sorted by
    decreasing z, then by increasing azimuth in [0, 2 pi).
    """
    if order < 2:
        raise ValueError("order must be >= 2")
    m = order - 1
    verts, faces = icosahedron_vertices()
    key = lambda p: tuple(np.round(p, 12))
    nodes: Dict[tuple, int] = {}
    pts: List[np.ndarray] = []

    def node(p):
        p = p / np.linalg.norm(p)
        k = key(p)
        if k not in nodes:
            nodes[k] = len(pts)
            pts.append(p)
        return nodes[k]

    tris = []
    for (ia, ib, ic) in faces:
        A, B, C = verts[ia], verts[ib], verts[ic]
        idx = {}
        for a in range(m + 1):
            for b in range(m + 1 - a):
                idx[(a, b)] = node(A + (a / m) * (B - A) + (b / m) * (C - A))
        for a in range(m):
            for b in range(m - a):
                tris.append((idx[(a, b)], idx[(a + 1, b)], idx[(a, b + 1)]))
                if a + b <= m - 2:
                    tris.append((idx[(a + 1, b)], idx[(a + 1, b + 1)], idx[(a, b + 1)]))
    P = np.array(pts)
    around: List[List[np.ndarray]] = [[] for _ in range(len(P))]
    for t in tris:
        c = P[list(t)].sum(axis=0)
        c /= np.linalg.norm(c)
        for v in t:
            around[v].append(c)
    w = np.zeros(len(P))
    for v in range(len(P)):
        p = P[v]
        # order the surrounding centres by angle in the tangent plane of p
        e1 = np.cross(p, [0.0, 0.0, 1.0]) if abs(p[2]) < 0.9 else np.cross(p, [1.0, 0.0, 0.0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(p, e1)
        cs = sorted(around[v], key=lambda c: math.atan2(np.dot(c, e2), np.dot(c, e1)))
        w[v] = sum(_spherical_triangle_area(p, cs[i], cs[(i + 1) % len(cs)])
                   for i in range(len(cs)))
    az = np.mod(np.arctan2(P[:, 1], P[:, 0]), 2 * math.pi)
    order_idx = np.lexsort((np.round(az, 9), -np.round(P[:, 2], 9)))
    return P[order_idx], w[order_idx]


# ---------------------------------------------------------------------------
# Artificial scattering kernel (Section 2.3 eq. (5); Section 3.2 eq. asSNeq)
# ---------------------------------------------------------------------------

def s_eps(mu: np.ndarray, eps: float) -> np.ndarray:
    """The paper's Dirac-like kernel, eq. (5), including its normalising prefactor."""
    pref = 2.0 / (math.sqrt(math.pi) * eps * math.erf(2.0 / eps))
    return pref * np.exp(-((1.0 - np.asarray(mu, dtype=np.float64)) / eps) ** 2)


def transport_coefficient(i: int, eps: float) -> float:
    """p_{eps,i} = int_{-1}^{1} (1 - mu)^i s_eps(mu) dmu in closed form (Section 2.5).

    With y = (1 - mu)/eps the integral is eps^i * gamma_lower((i+1)/2, 4/eps^2)
    / (sqrt(pi) * Erf(2/eps)); the printed form drops a factor 1/2 and one eps,
    which this restores (it gives p_{eps,0} = 1 as the normalisation demands).
    """
    from scipy.special import gamma, gammainc
    a = 0.5 * (i + 1)
    lower = gammainc(a, 4.0 / eps ** 2) * gamma(a)
    return eps ** i * lower / (math.sqrt(math.pi) * math.erf(2.0 / eps))


def kernel_width(q: int, beta: float) -> float:
    """eps = beta / N_q (Section 2.3, item 1)."""
    return beta / q


def as_kernel_unnormalised(omega: np.ndarray, eps: float) -> np.ndarray:
    """S_qp = exp(-((1 - Omega_q . Omega_p)/eps)^2), eq. (5) without its prefactor."""
    c = omega @ omega.T
    return np.exp(-((1.0 - c) / eps) ** 2)


def as_kernel_matrix(omega: np.ndarray, w: np.ndarray, eps: float, mode: str = "sym",
                     tol: float = 1e-14, max_iter: int = 10000) -> np.ndarray:
    """Discrete normalised artificial in-scattering matrix K (Q x Q).

    (K psi)_q approximates the normalised integral of s_eps(Omega_q . Omega') psi(Omega').
    mode "row": K_qp = w_p c_q s_qp with c_q = 1 / sum_p w_p s_qp (eq. asSNeq).
    mode "sym": K = diag(d) S diag(w d) with d > 0 chosen so every row sums to one;
      because S is symmetric the w-weighted column sums are then one as well.
      d is found by the symmetric Sinkhorn iteration d <- d / sqrt(d * (S (w d))).
    """
    s = as_kernel_unnormalised(omega, eps)
    if mode == "row":
        return (s * w[None, :]) / (s @ w)[:, None]
    if mode != "sym":
        raise ValueError(f"unknown normalisation {mode!r}")
    d = 1.0 / np.sqrt(s @ w)
    for _ in range(max_iter):
        rows = d * (s @ (w * d))
        if np.max(np.abs(rows - 1.0)) <= tol:
            break
        d = d / np.sqrt(rows)
    else:
        raise RuntimeError("symmetric Sinkhorn scaling did not converge")
    return d[:, None] * s * (w * d)[None, :]


# ---------------------------------------------------------------------------
# Grid, time step and set-up
# ---------------------------------------------------------------------------

def cfl_time_step(omega: np.ndarray, dx: float, dy: float, cfl: float,
                  t_final: float) -> Tuple[float, int]:
    """dt = t_final / n with n = ceil(t_final / dt_max), dt_max = cfl / max_q(|xi|/dx + |eta|/dy)."""
    rate = float(np.max(np.abs(omega[:, 0]) / dx + np.abs(omega[:, 1]) / dy))
    dt_max = cfl / rate
    n = max(1, int(math.ceil(t_final / dt_max * (1.0 - 1e-12))))
    return t_final / n, n


def stability_number(omega: np.ndarray, K: np.ndarray, dx: float, dy: float, dt: float,
                     sigma_s: np.ndarray, sigma_a: np.ndarray, sigma_as: np.ndarray) -> float:
    """z = dt [2 max_q r_q + max_c (sigma_a + sigma_s + 2 (1 - min_q K_qq) sigma_as)],
    r_q = |xi_q|/dx + |eta_q|/dy.

    In a region of uniform material a state that alternates in sign from cell to
    cell is moved by the donor-cell fluxes at rate 2 r_q (each face passes the
    neighbour's opposite value), and collisions act on its ordinate vector with
    (sigma_a + sigma_s + sigma_as) I - sigma_as K - sigma_s (isotropic
    projection).  Scaled by the square roots of the weights the whole rate
    matrix is symmetric for the symmetric K, so its eigenvalues are real and, by
    Weyl's inequality, at most the bracket: Gershgorin's theorem puts every
    eigenvalue of K (rows summing to one) at or above 2 min_q K_qq - 1, and the
    isotropic projection only removes particles.  Forward Euler and Heun damp a
    real mode only while dt times its rate is in [0, 2].
    """
    r = float(np.max(np.abs(omega[:, 0]) / dx + np.abs(omega[:, 1]) / dy))
    g = 2.0 * (1.0 - float(np.min(np.diag(K))))
    m = float(np.max(np.asarray(sigma_a, np.float64) + np.asarray(sigma_s, np.float64)
                     + g * np.asarray(sigma_as, np.float64)))
    return dt * (2.0 * r + m)


def stiff_time_step(omega: np.ndarray, K: np.ndarray, dx: float, dy: float, cfl: float,
                    t_final: float, sigma_s, sigma_a, sigma_as) -> Tuple[float, int]:
    """cfl_time_step with dt_max also limited so that stability_number <= 2 cfl."""
    rate = float(np.max(np.abs(omega[:, 0]) / dx + np.abs(omega[:, 1]) / dy))
    z1 = stability_number(omega, K, dx, dy, 1.0, sigma_s, sigma_a, sigma_as)
    dt_max = min(cfl / rate, 2.0 * cfl / z1)
    n = max(1, int(math.ceil(t_final / dt_max * (1.0 - 1e-12))))
    return t_final / n, n


@dataclasses.dataclass
class Setup:
    omega: np.ndarray
    w: np.ndarray
    W: float
    K: np.ndarray
    eps: float
    dx: float
    dy: float
    dt: float
    n_steps: int
    sigma_s: np.ndarray      # float64 [ny, nx]
    sigma_a: np.ndarray
    sigma_as: np.ndarray
    source: np.ndarray

    @property
    def q(self) -> int:
        return self.w.size


def setup(problem, mode: str = "sym", eps: Optional[float] = None,
          cfl: Optional[float] = None, omega: Optional[np.ndarray] = None,
          w: Optional[np.ndarray] = None, dt: Optional[float] = None,
          dt_rule: str = "streaming") -> Setup:
    """Build quadrature, K and dt for a workloads.Problem (all FP64).

    dt_rule "streaming" is the CFL rule on the streaming alone; "stiff" also keeps
    stability_number <= 2 cfl."""
    if omega is None:
        if getattr(problem, "ico_order", 0):
            omega, w = icosahedron_quadrature(problem.ico_order)
        else:
            omega, w = product_quadrature(problem.n_polar, problem.n_azim)
    q = w.size
    eps = kernel_width(q, problem.beta) if eps is None else eps
    K = as_kernel_matrix(omega, w, eps, mode)
    dx = (problem.x_max - problem.x_min) / problem.nx
    dy = (problem.y_max - problem.y_min) / problem.ny
    c = problem.cfl if cfl is None else cfl
    if dt is None and dt_rule == "stiff":
        dt, n = stiff_time_step(omega, K, dx, dy, c, problem.t_final, problem.sigma_s,
                                problem.sigma_a, problem.sigma_as)
    elif dt is None:
        dt, n = cfl_time_step(omega, dx, dy, c, problem.t_final)
    else:
        n = max(1, int(round(problem.t_final / dt)))
    f64 = lambda a: np.asarray(a, dtype=np.float64)
    return Setup(omega=omega, w=w, W=float(np.sum(w)), K=K, eps=eps, dx=dx, dy=dy, dt=dt,
                 n_steps=n, sigma_s=f64(problem.sigma_s), sigma_a=f64(problem.sigma_a),
                 sigma_as=f64(problem.sigma_as), source=f64(problem.source))


# ---------------------------------------------------------------------------
# The explicit step (Section 3.2, eq. asSNeq, discretised in space and time)
# ---------------------------------------------------------------------------

def scalar_flux(psi: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Phi = sum_q w_q psi_q (Section 2.2 definition of the scalar flux)."""
    return np.tensordot(w, psi, axes=(0, 0))


def upwind_face_fluxes(psi: np.ndarray, xi: np.ndarray, eta: np.ndarray):
    """Donor-cell face fluxes with zero (vacuum) ghost values.

    Fx[q, j, f] is the x-flux through the face at x_min + f dx (f = 0..nx);
    it carries xi_q times the value of the cell upstream of the face.
    Fy[q, f, i] likewise for the faces at y_min + f dy.
    """
    Q, ny, nx = psi.shape
    Fx = np.zeros((Q, ny, nx + 1))
    Fy = np.zeros((Q, ny + 1, nx))
    for q in range(Q):
        if xi[q] > 0:
            Fx[q, :, 1:] = xi[q] * psi[q]
        elif xi[q] < 0:
            Fx[q, :, :-1] = xi[q] * psi[q]
        if eta[q] > 0:
            Fy[q, 1:, :] = eta[q] * psi[q]
        elif eta[q] < 0:
            Fy[q, :-1, :] = eta[q] * psi[q]
    return Fx, Fy


def as_in_scattering(psi: np.ndarray, K: np.ndarray) -> np.ndarray:
    """Y_q = sum_p K_qp psi_p in every cell (the sigma_as in-scattering sum of eq. asSNeq)."""
    Q = psi.shape[0]
    return (K @ psi.reshape(Q, -1)).reshape(psi.shape)


def step(psi: np.ndarray, st: Setup, Y: Optional[np.ndarray] = None,
         want_budget: bool = True):
    """One forward-Euler as-S_N step; returns (psi_new, budget dict).

    psi_new = psi - dt * div(F_upwind)
              - dt (sigma_a + sigma_s + sigma_as) psi
              + dt sigma_s Phi / W + dt sigma_as Y + dt q,
    every right-hand-side term evaluated at the old level.  ``Y`` may be
    supplied (e.g. by the low-precision emulation); otherwise Y = K psi.
    """
    xi, eta = st.omega[:, 0], st.omega[:, 1]
    phi = scalar_flux(psi, st.w)
    if Y is None:
        Y = as_in_scattering(psi, st.K)
    Fx, Fy = upwind_face_fluxes(psi, xi, eta)
    div = (Fx[:, :, 1:] - Fx[:, :, :-1]) / st.dx + (Fy[:, 1:, :] - Fy[:, :-1, :]) / st.dy
    sig_t = st.sigma_a + st.sigma_s + st.sigma_as
    rhs = (-div - sig_t[None] * psi + (st.sigma_s * phi / st.W)[None]
           + st.sigma_as[None] * Y + st.source[None])
    psi_new = psi + st.dt * rhs
    if not want_budget:
        return psi_new, None
    area = st.dx * st.dy
    wq = st.w[:, None, None]
    outflow = (st.dy * np.sum(st.w * (Fx[:, :, -1].sum(1) - Fx[:, :, 0].sum(1)))
               + st.dx * np.sum(st.w * (Fy[:, -1, :].sum(1) - Fy[:, 0, :].sum(1))))
    budget = {
        "mass": area * phi.sum(),
        "absorption": area * np.sum(st.sigma_a * phi),
        "outflow": outflow,
        "source": area * st.W * st.source.sum(),
        "as_defect": area * np.sum(st.sigma_as * np.sum(wq * (Y - psi), axis=0)),
    }
    return psi_new, budget


def mass(psi: np.ndarray, st: Setup) -> float:
    return st.dx * st.dy * float(scalar_flux(psi, st.w).sum())


def budget_residual(b: Dict[str, float], mass_next: float, dt: float) -> float:
    """M^{n+1} - [M^n + dt (-A - O + S + D)] for one step's budget record."""
    return mass_next - (b["mass"] + dt * (-b["absorption"] - b["outflow"] + b["source"]
                                          + b["as_defect"]))


def run(problem, n_steps: Optional[int] = None, st: Optional[Setup] = None,
        psi0: Optional[np.ndarray] = None, mode: str = "sym", budget: bool = False):
    """Advance a problem; returns (psi, setup, list of per-step budget records)."""
    st = setup(problem, mode) if st is None else st
    psi = (problem.psi0() if psi0 is None else psi0).astype(np.float64)
    n = st.n_steps if n_steps is None else n_steps
    hist: List[Dict[str, float]] = []
    for _ in range(n):
        psi, b = step(psi, st, want_budget=budget)
        if budget:
            b["mass_next"] = mass(psi, st)
            hist.append(b)
    return psi, st, hist


def step_entries(psi: np.ndarray, st: Setup, qs: np.ndarray, js: np.ndarray,
                 iis: np.ndarray, phi: Optional[np.ndarray] = None) -> np.ndarray:
    """psi^{n+1} at the listed (q, j, i) only, evaluated entry by entry.

    Used for parity at sizes where a full oracle step is too slow.  ``phi``
    (the scalar flux of ``psi``) may be passed to avoid recomputing it.
    """
    Q, ny, nx = psi.shape
    if phi is None:
        phi = np.zeros((ny, nx))
        for q in range(Q):
            phi += st.w[q] * psi[q].astype(np.float64)
    out = np.empty(len(qs))
    for n, (q, j, i) in enumerate(zip(qs, js, iis)):
        xi, eta = st.omega[q, 0], st.omega[q, 1]
        v = lambda jj, ii: float(psi[q, jj, ii]) if (0 <= jj < ny and 0 <= ii < nx) else 0.0
        c = v(j, i)
        if xi > 0:
            dfx = xi * (c - v(j, i - 1))
        elif xi < 0:
            dfx = xi * (v(j, i + 1) - c)
        else:
            dfx = 0.0
        if eta > 0:
            dfy = eta * (c - v(j - 1, i))
        elif eta < 0:
            dfy = eta * (v(j + 1, i) - c)
        else:
            dfy = 0.0
        y = float(np.dot(st.K[q], psi[:, j, i].astype(np.float64)))
        s_s, s_a, s_as = st.sigma_s[j, i], st.sigma_a[j, i], st.sigma_as[j, i]
        rhs = (-dfx / st.dx - dfy / st.dy - (s_a + s_s + s_as) * c
               + s_s * phi[j, i] / st.W + s_as * y + st.source[j, i])
        out[n] = c + st.dt * rhs
    return out


def run_entries(psi: np.ndarray, st: Setup, n_steps: int, qs: np.ndarray, js: np.ndarray,
                iis: np.ndarray) -> np.ndarray:
    """psi after n_steps forward-Euler steps (step above) at the listed (q, j, i) only.

    Information moves at most one cell per step, so a cell's value after n steps
    depends only on the old state within n cells along each axis.  Each distinct
    cell is advanced on the (2n + 1)^2 window around it, all ordinates, with the
    cells outside the grid at the ghost value 0; cells of the window beyond the
    grid stay 0 after every step, and values near the window's own edge, which
    lack their outer neighbours, never reach its centre within n steps.
    """
    Q, ny, nx = psi.shape
    h = n_steps
    w = 2 * h + 1

    def window(a, j, i):
        """a[..., j - h .. j + h, i - h .. i + h] in FP64, zero outside the grid."""
        out = np.zeros(a.shape[:-2] + (w, w))
        j0, j1, i0, i1 = max(j - h, 0), min(j + h + 1, ny), max(i - h, 0), min(i + h + 1, nx)
        out[..., j0 - (j - h):j1 - (j - h), i0 - (i - h):i1 - (i - h)] = a[..., j0:j1, i0:i1]
        return out

    cache: Dict[Tuple[int, int], np.ndarray] = {}
    out = np.empty(len(qs))
    for n, (q, j, i) in enumerate(zip(qs, js, iis)):
        key = (int(j), int(i))
        if key not in cache:
            j, i = key
            sub = dataclasses.replace(st, **{k: window(getattr(st, k), j, i)
                                             for k in ("sigma_s", "sigma_a", "sigma_as", "source")})
            mask = window(np.ones((ny, nx)), j, i)[None]
            p = window(psi, j, i)
            for _ in range(n_steps):
                p, _ = step(p, sub, want_budget=False)
                p = p * mask
            cache[key] = p[:, h, h]
        out[n] = cache[key][q]
    return out


# ---------------------------------------------------------------------------
# The paper's own explicit scheme (Section 3.1): Heun's method in time with
# minmod-limited second-order upwind fluxes in space.  The paper defers the
# details to earlier work; the reading used here is the textbook one:
#   * per ordinate and per axis, a linear reconstruction in every cell with the
#     limited slope s_i = minmod(psi_i - psi_{i-1}, psi_{i+1} - psi_i);
#   * the flux through a face takes the value reconstructed on its upwind side,
#     psi_i + s_i / 2 (from the left cell) or psi_{i+1} - s_{i+1} / 2 (right);
#   * two zero ghost cells outside every boundary (vacuum: the ghost slope is
#     minmod(0, .) = 0, so no particles enter);
#   * Heun: psi1 = psi + dt R(psi), psi^{n+1} = (psi + psi1 + dt R(psi1)) / 2,
#     with R every right-hand-side term of eq. asSNeq (streaming, collisions,
#     physical and artificial scattering, source) at the stage's own level.
# ---------------------------------------------------------------------------

def minmod(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """The argument of smaller magnitude when a and b share a sign, else 0."""
    return np.where(a * b > 0.0, np.where(np.abs(a) <= np.abs(b), a, b), 0.0)


def muscl_face_fluxes(psi: np.ndarray, xi: np.ndarray, eta: np.ndarray):
    """Limited second-order upwind face fluxes with two zero ghost cells per side.

    Same face indexing as upwind_face_fluxes: Fx[q, j, f] crosses x_min + f dx.
    """
    Q, ny, nx = psi.shape
    Fx = np.zeros((Q, ny, nx + 1))
    Fy = np.zeros((Q, ny + 1, nx))
    for q in range(Q):
        g = np.zeros((ny + 4, nx + 4))
        g[2:-2, 2:-2] = psi[q]
        # x: cells -1 .. nx of the row (padded columns 1 .. nx + 2), their slopes,
        # and the values reconstructed at their right and left faces
        c = g[2:-2, 1:nx + 3]
        s = minmod(c - g[2:-2, 0:nx + 2], g[2:-2, 2:nx + 4] - c)
        if xi[q] > 0:
            Fx[q] = xi[q] * (c + 0.5 * s)[:, 0:nx + 1]      # face f from cell f - 1
        elif xi[q] < 0:
            Fx[q] = xi[q] * (c - 0.5 * s)[:, 1:nx + 2]      # face f from cell f
        c = g[1:ny + 3, 2:-2]
        s = minmod(c - g[0:ny + 2, 2:-2], g[2:ny + 4, 2:-2] - c)
        if eta[q] > 0:
            Fy[q] = eta[q] * (c + 0.5 * s)[0:ny + 1, :]
        elif eta[q] < 0:
            Fy[q] = eta[q] * (c - 0.5 * s)[1:ny + 2, :]
    return Fx, Fy


def heun_rhs(psi: np.ndarray, st: Setup):
    """R(psi) of eq. asSNeq with the limited fluxes; returns (R, stage budget terms)."""
    xi, eta = st.omega[:, 0], st.omega[:, 1]
    phi = scalar_flux(psi, st.w)
    Y = as_in_scattering(psi, st.K)
    Fx, Fy = muscl_face_fluxes(psi, xi, eta)
    div = (Fx[:, :, 1:] - Fx[:, :, :-1]) / st.dx + (Fy[:, 1:, :] - Fy[:, :-1, :]) / st.dy
    sig_t = st.sigma_a + st.sigma_s + st.sigma_as
    R = (-div - sig_t[None] * psi + (st.sigma_s * phi / st.W)[None]
         + st.sigma_as[None] * Y + st.source[None])
    area = st.dx * st.dy
    wq = st.w[:, None, None]
    terms = {
        "mass": area * phi.sum(),
        "absorption": area * np.sum(st.sigma_a * phi),
        "outflow": (st.dy * np.sum(st.w * (Fx[:, :, -1].sum(1) - Fx[:, :, 0].sum(1)))
                    + st.dx * np.sum(st.w * (Fy[:, -1, :].sum(1) - Fy[:, 0, :].sum(1)))),
        "source": area * st.W * st.source.sum(),
        "as_defect": area * np.sum(st.sigma_as * np.sum(wq * (Y - psi), axis=0)),
    }
    return R, terms


def heun_step(psi: np.ndarray, st: Setup, want_budget: bool = True):
    """One Heun step with limited fluxes; returns (psi_new, budget dict).

    The budget holds M^n and the stage averages of absorption, outflow, source
    and defect, so that M^{n+1} = M^n + dt (-A - O + S + D) exactly, as for
    the Euler step (budget_residual applies unchanged).
    """
    R0, b0 = heun_rhs(psi, st)
    psi1 = psi + st.dt * R0
    R1, b1 = heun_rhs(psi1, st)
    psi_new = 0.5 * (psi + (psi1 + st.dt * R1))
    if not want_budget:
        return psi_new, None
    budget = {k: 0.5 * (b0[k] + b1[k]) for k in b0}
    budget["mass"] = b0["mass"]
    return psi_new, budget


def run_heun(problem, n_steps: Optional[int] = None, st: Optional[Setup] = None,
             psi0: Optional[np.ndarray] = None, mode: str = "sym", budget: bool = False):
    """Advance a problem with heun_step; returns (psi, setup, budget records)."""
    st = setup(problem, mode) if st is None else st
    psi = (problem.psi0() if psi0 is None else psi0).astype(np.float64)
    n = st.n_steps if n_steps is None else n_steps
    hist: List[Dict[str, float]] = []
    for _ in range(n):
        psi, b = heun_step(psi, st, want_budget=budget)
        if budget:
            b["mass_next"] = mass(psi, st)
            hist.append(b)
    return psi, st, hist


def heun_step_entries(psi: np.ndarray, st: Setup, qs: np.ndarray, js: np.ndarray,
                      iis: np.ndarray) -> np.ndarray:
    """heun_step's psi^{n+1} at the listed (q, j, i) only.

    A cell's new value depends on the old state within four cells along each
    axis (two per stage), so each entry is computed on the 9 x 9 window around
    it, all ordinates, with the cells outside the grid held at the ghost value 0.
    """
    Q, ny, nx = psi.shape
    h = 4
    pad = lambda a: np.pad(np.asarray(a, dtype=np.float64), [(0, 0)] * (a.ndim - 2) + [(h, h), (h, h)])
    P = pad(psi)
    inside = pad(np.ones((ny, nx)))
    fields = {k: pad(getattr(st, k)) for k in ("sigma_s", "sigma_a", "sigma_as", "source")}
    out = np.empty(len(qs))
    for n, (q, j, i) in enumerate(zip(qs, js, iis)):
        win = (slice(j, j + 2 * h + 1), slice(i, i + 2 * h + 1))
        sub = dataclasses.replace(st, **{k: v[win] for k, v in fields.items()})
        mask = inside[win][None]
        p0 = P[(slice(None),) + win]
        R0, _ = heun_rhs(p0, sub)
        p1 = (p0 + st.dt * R0) * mask
        R1, _ = heun_rhs(p1, sub)
        out[n] = 0.5 * (p0 + p1 + st.dt * R1)[q, h, h]
    return out


# ---------------------------------------------------------------------------
# Reduced-precision emulation of the in-scattering contraction
# ---------------------------------------------------------------------------
# The GPU path may evaluate Y = K psi with BF16 or FP16 operands and FP32
# accumulation.  The recipe (fixed by the design, not by the paper) is:
#   iso_c  = fp32(Phi_c / W)                        isotropic part, exact for K
#   dev_qc = fp32(psi_qc - iso_c)                    only the deviation is rounded
#   e_b    = frexp exponent of max_{q, c in b} |psi_qc| over blocks b of n cells
#            of the flattened grid (n = 256 unless chosen: a power of two 64..4096),
#            at least -100 (0 for an all-zero block)
#   s_qc   = dev_qc * 2^(E - e_b), E = 14            power-of-two block scale
#   x_qc   = T(s_qc) for FP16;  for BF16 two terms   RNE throughout
#            x = hi + lo, hi = T(s), lo = T(s - hi)  (8 more significant bits)
#   Y_qc   = iso_c + 2^(e_b - E) sum_p T(K)_qp x_pc + r_q dev_qc
#            with r_q = 1 - sum_p T(K)_qp             quantised row-sum defect
#   Y_qc  -= (sum_q w_q Y_qc - Phi_c) / W              per-cell particle fix
# Here the contraction is accumulated in FP64 so the emulation isolates the
# effect of the operand rounding.

SCALE_BLOCK = 256
SCALE_EXP = 14
SCALE_EXP_MIN = -100


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even), returned as float32."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def round_f16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to IEEE half (numpy's conversion is round-to-nearest-even)."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


def quantise(x: np.ndarray, dtype: str) -> np.ndarray:
    """Round float32 values to the operand type; "f32" keeps them (recipe without rounding)."""
    if dtype == "f32":
        return np.asarray(x, dtype=np.float32)
    if dtype == "bf16":
        return round_bf16(x)
    if dtype == "f16":
        return round_f16(x)
    raise ValueError(dtype)


def operand_terms(s32: np.ndarray, dtype: str) -> np.ndarray:
    """The rounded contraction operand as float64: one term for FP16 (and the
    unrounded "f32" recipe), hi + lo for BF16 (s - hi is exact in FP32)."""
    if dtype != "bf16":
        return quantise(s32, dtype).astype(np.float64)
    hi = round_bf16(s32)
    lo = round_bf16((s32 - hi).astype(np.float32))
    return hi.astype(np.float64) + lo.astype(np.float64)


def lowprec_kernel(K: np.ndarray, dtype: str) -> Tuple[np.ndarray, np.ndarray]:
    """(T(fp32(K)) as float64, row defect r = fp32(1 - row sums)) for the emulation."""
    kq = quantise(K.astype(np.float32), dtype).astype(np.float64)
    r = (1.0 - kq.sum(axis=1)).astype(np.float32).astype(np.float64)
    return kq, r


def block_exponents(psi32: np.ndarray, block: int = SCALE_BLOCK) -> np.ndarray:
    """Per-cell exponent e_b of the block max |psi| (flattened cells, blocks of `block`)."""
    Q = psi32.shape[0]
    flat = np.abs(psi32.reshape(Q, -1)).max(axis=0)
    C = flat.size
    nb = (C + block - 1) // block
    padded = np.zeros(nb * block, dtype=np.float32)
    padded[:C] = flat
    bmax = padded.reshape(nb, block).max(axis=1)
    _, e = np.frexp(bmax.astype(np.float64))
    e = np.where(bmax > 0, e, 0)
    e = np.maximum(e, SCALE_EXP_MIN)     # keeps 2^(E - e) finite in FP32
    return np.repeat(e, block)[:C]


def _weighted_ordinate_sum(w: np.ndarray, x: np.ndarray) -> np.ndarray:
    """sum_q w_q x_q in a fixed order (row by row), independent of memory layout."""
    acc = np.zeros(x.shape[1:], dtype=np.float64)
    for q in range(x.shape[0]):
        acc += w[q] * x[q]
    return acc


def lowprec_in_scattering(psi32: np.ndarray, st: Setup, dtype: str,
                          kq: Optional[np.ndarray] = None,
                          r: Optional[np.ndarray] = None,
                          block: int = SCALE_BLOCK,
                          e: Optional[np.ndarray] = None) -> np.ndarray:
    """Y by the reduced-precision recipe above, for a float32 state [Q, ny, nx], with
    scale blocks of `block` cells (or the per-cell block exponents `e`, given when the
    state passed is part of the grid)."""
    if kq is None:
        kq, r = lowprec_kernel(st.K, dtype)
    Q = psi32.shape[0]
    p = np.asarray(psi32, dtype=np.float32).reshape(Q, -1)
    phi = _weighted_ordinate_sum(st.w, p.astype(np.float64))
    iso = (phi / st.W).astype(np.float32)
    dev = (p - iso[None, :]).astype(np.float32)
    if e is None:
        e = block_exponents(p, block)
    s_in = np.ldexp(np.float32(1.0), (SCALE_EXP - e)).astype(np.float32)
    x = operand_terms((dev * s_in[None, :]).astype(np.float32), dtype)
    acc = kq @ x
    Y = iso[None, :].astype(np.float64) + np.ldexp(acc, (e - SCALE_EXP)[None, :]) \
        + r[:, None] * dev.astype(np.float64)
    m = _weighted_ordinate_sum(st.w, Y) - phi
    Y = Y - (m / st.W)[None, :]
    return Y.reshape(psi32.shape)


def lowprec_step(psi32: np.ndarray, st: Setup, dtype: str, kq=None, r=None,
                 block: int = SCALE_BLOCK):
    """One step with the reduced-precision Y; the rest of the step stays FP64."""
    Y = lowprec_in_scattering(psi32, st, dtype, kq, r, block)
    return step(np.asarray(psi32, dtype=np.float64), st, Y=Y)


def lowprec_step_entries(psi32: np.ndarray, st: Setup, dtype: str, qs: np.ndarray,
                         js: np.ndarray, iis: np.ndarray, kq=None, r=None,
                         block: int = SCALE_BLOCK) -> np.ndarray:
    """psi^{n+1} of lowprec_step at the listed (q, j, i) only, for grids where a full
    emulated step is too slow.

    The recipe is per cell apart from the block exponent: each distinct cell's column
    of Y is formed from its own ordinates with the exponent of its whole scale block,
    and the step is taken on the 3 x 3 window around the cell (zero outside the grid),
    whose centre needs the old values of its four neighbours and its own Y only.
    """
    if kq is None:
        kq, r = lowprec_kernel(st.K, dtype)
    Q, ny, nx = psi32.shape
    flat = np.asarray(psi32, dtype=np.float32).reshape(Q, -1)
    C = ny * nx

    def window(a, j, i):
        """a[..., j - 1 .. j + 1, i - 1 .. i + 1] in FP64, zero outside the grid."""
        out = np.zeros(a.shape[:-2] + (3, 3))
        j0, j1, i0, i1 = max(j - 1, 0), min(j + 2, ny), max(i - 1, 0), min(i + 2, nx)
        out[..., j0 - (j - 1):j1 - (j - 1), i0 - (i - 1):i1 - (i - 1)] = a[..., j0:j1, i0:i1]
        return out

    cache: Dict[Tuple[int, int], np.ndarray] = {}
    out = np.empty(len(qs))
    for n, (q, j, i) in enumerate(zip(qs, js, iis)):
        key = (int(j), int(i))
        if key not in cache:
            j, i = key
            b0 = ((j * nx + i) // block) * block
            eb = block_exponents(flat[:, b0:min(b0 + block, C)], block)[:1]
            Yc = lowprec_in_scattering(psi32[:, j:j + 1, i:i + 1], st, dtype, kq, r, block, e=eb)
            sub = dataclasses.replace(st, **{k: window(getattr(st, k), j, i)
                                             for k in ("sigma_s", "sigma_a", "sigma_as", "source")})
            p = window(psi32, j, i)
            Y = np.zeros_like(p)
            Y[:, 1, 1] = Yc[:, 0, 0]
            new, _ = step(p, sub, Y=Y, want_budget=False)
            cache[key] = new[:, 1, 1]
        out[n] = cache[key][q]
    return out
