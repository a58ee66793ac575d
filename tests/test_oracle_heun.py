"""Pins for the oracle's Heun + minmod scheme (the paper's explicit scheme, Section
3.1, read as textbook MUSCL with a minmod limiter and Heun's method).

Each pin is fixed by mathematics, not by re-running the oracle's formulas:
exactness on linear data, second-order convergence against the exact solution,
the maximum principle of the limited scheme, the Heun polynomial on the pure
collision ODE, the particle budget identity, symmetries of the line source, and
the paper's twelve-ordinate artificial-scattering error ratio."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import asn_oracle as o
from oracle import linesource_ref as L


def _one_ordinate(nx, ny, xi, eta, cfl=0.5, t=0.1, sigma_a=0.0):
    f = lambda v: np.full((ny, nx), v, dtype=np.float32)
    prob = wl.Problem(name="one", nx=nx, ny=ny, x_min=0.0, x_max=1.0, y_min=0.0,
                      y_max=ny / nx, n_polar=1, n_azim=1, sigma_s=f(0.0), sigma_a=f(sigma_a),
                      sigma_as=f(0.0), source=f(0.0), psi0_cell=f(0.0), t_final=t, cfl=cfl)
    om = np.array([[xi, eta, math.sqrt(max(0.0, 1.0 - xi * xi - eta * eta))]])
    return prob, o.setup(prob, omega=om, w=np.array([4 * math.pi]))


def test_minmod_values():
    a = np.array([1.0, -1.0, 1.0, 0.0, 2.0, -4.0, 3.0])
    b = np.array([2.0, -3.0, -1.0, 5.0, 2.0, -0.5, 0.0])
    assert np.array_equal(o.minmod(a, b), [1.0, -1.0, 0.0, 0.0, 2.0, -0.5, 0.0])


@pytest.mark.parametrize("xi,eta", [(0.6, 0.3), (-0.5, 0.4), (0.2, -0.7), (-0.45, -0.45)])
def test_linear_data_is_translated_exactly(xi, eta):
    # A linear profile is reconstructed exactly, so both stages translate it by
    # dt (xi, eta) with no error, away from the boundaries.
    prob, st = _one_ordinate(24, 20, xi, eta)
    x = prob.x_min + (np.arange(24) + 0.5) * st.dx
    y = prob.y_min + (np.arange(20) + 0.5) * st.dy
    lin = lambda xx, yy: 5.0 + 2.0 * xx[None, :] - 3.0 * yy[:, None]
    psi = lin(x, y)[None]
    new, _ = o.heun_step(psi, st, want_budget=False)
    exact = lin(x - xi * st.dt, y - eta * st.dt)
    assert np.max(np.abs(new[0, 4:-4, 4:-4] - exact[4:-4, 4:-4])) < 1e-12


def _gaussian_l1_error(step, n):
    prob, st = _one_ordinate(n, 1, 0.6, 0.0, cfl=0.5, t=0.3)
    x = (np.arange(n) + 0.5) / n
    g = lambda xx: np.exp(-((xx - 0.35) / 0.08) ** 2)
    psi = g(x)[None, None, :]
    for _ in range(st.n_steps):
        psi, _ = step(psi, st, want_budget=False)
    return float(np.abs(psi[0, 0] - g(x - 0.6 * st.dt * st.n_steps)).sum() / n)


def test_second_order_convergence_on_a_smooth_pulse():
    # Exact solution: the pulse translated by xi t.  Halving dx (and dt) cuts the L1
    # error by about 4 (minmod clips the peak, so a little less); the donor-cell
    # Euler step halves it.
    e = [_gaussian_l1_error(o.heun_step, n) for n in (100, 200, 400)]
    assert e[0] / e[1] > 2.6 and e[1] / e[2] > 3.0
    d = [_gaussian_l1_error(o.step, n) for n in (100, 200)]
    assert 1.7 < d[0] / d[1] < 2.2
    assert e[1] < 0.25 * d[1]


def test_limited_scheme_keeps_a_step_within_its_bounds():
    # With dt |xi| / dx <= 2/3 each Euler stage of the limited scheme is a convex
    # combination of old values, so a unit step stays in [0, 1]; an unlimited
    # (central) slope overshoots by more than 10 % here.
    prob, st = _one_ordinate(100, 1, 0.6, 0.0, cfl=0.66, t=0.3)
    x = (np.arange(100) + 0.5) / 100
    psi = (x < 0.3).astype(np.float64)[None, None, :]
    for _ in range(st.n_steps):
        psi, _ = o.heun_step(psi, st, want_budget=False)
    assert psi.min() >= 0.0 and psi.max() <= 1.0
    assert psi.max() > 0.99 and psi[0, 0, 60:].max() < 1e-3 and psi[0, 0, 30:40].min() > 0.1


def test_collisions_follow_the_heun_polynomial():
    # Ordinates along +-z do not stream; with absorption and artificial scattering
    # the state obeys psi' = A psi, and Heun's method advances it by
    # I + dt A + (dt A)^2 / 2 per step.
    f = lambda v: np.full((3, 2), v, dtype=np.float32)
    prob = wl.Problem(name="ode", nx=2, ny=3, x_min=0.0, x_max=1.0, y_min=0.0, y_max=1.5,
                      n_polar=1, n_azim=2, sigma_s=f(0.75), sigma_a=f(0.5), sigma_as=f(2.0),
                      source=f(0.0), psi0_cell=f(0.0), t_final=1.0, cfl=0.5, beta=4.5)
    om = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    w = np.array([2 * math.pi, 2 * math.pi])
    st = o.setup(prob, omega=om, w=w, eps=4.0, dt=0.1)
    A = -(0.5 + 0.75 + 2.0) * np.eye(2) + 0.75 * np.outer(np.ones(2), w) / w.sum() + 2.0 * st.K
    step_matrix = np.eye(2) + st.dt * A + 0.5 * (st.dt * A) @ (st.dt * A)
    psi0 = np.array([1.0, 0.25])
    psi = np.broadcast_to(psi0[:, None, None], (2, 3, 2)).copy()
    for _ in range(5):
        psi, _ = o.heun_step(psi, st, want_budget=False)
    expect = np.linalg.matrix_power(step_matrix, 5) @ psi0
    assert np.max(np.abs(psi - expect[:, None, None])) < 1e-14
    assert abs(st.K[0, 1]) > 1e-3        # the kernel really couples the two ordinates


@pytest.mark.parametrize("mode", ["sym", "row"])
def test_particle_budget_closes_every_step(mode):
    spec = wl.random_problem(11, 23, 17, n_polar=2, n_azim=8, beta=4.5, t_final=0.2)
    psi0 = wl.random_state(2, spec.q, 17, 23)
    _, st, hist = o.run_heun(spec, budget=True, psi0=psi0, mode=mode)
    for b in hist:
        assert abs(o.budget_residual(b, b["mass_next"], st.dt)) <= 1e-13 * b["mass"]
        assert b["outflow"] > 0.0
    if mode == "sym":
        assert max(abs(b["as_defect"]) for b in hist) <= 1e-13 * hist[0]["mass"]


def test_isotropic_state_preserved_in_interior():
    spec = wl.random_problem(4, 30, 26, n_polar=2, n_azim=8, beta=4.5)
    spec.sigma_a[:] = 0.0
    spec.source[:] = 0.0
    psi = np.full((spec.q, 26, 30), 2.5)
    st = o.setup(spec)
    for _ in range(2):
        psi, _ = o.heun_step(psi, st, want_budget=False)
    assert np.max(np.abs(psi[:, 8:-8, 8:-8] - 2.5)) < 1e-13


def test_line_source_symmetries_of_the_product_set():
    # The product set with n_azim a multiple of 4 and offset 1/2 is invariant under
    # both mirrors and the swap of x and y, and so is the discrete flux.
    spec = wl.line_source(30, n_polar=2, sigma_as=1.0, t_final=0.3)
    psi, st, _ = o.run_heun(spec)
    phi = o.scalar_flux(psi, st.w)
    s = np.abs(phi).max()
    for other in (phi[:, ::-1], phi[::-1, :], phi.T):
        assert np.max(np.abs(phi - other)) < 1e-13 * s


def test_sampled_entries_match_the_full_step():
    spec = wl.random_problem(7, 15, 11, n_polar=2, n_azim=4, beta=4.5)
    psi0 = wl.random_state(3, spec.q, 11, 15).astype(np.float64)
    st = o.setup(spec)
    full, _ = o.heun_step(psi0, st, want_budget=False)
    rng = np.random.default_rng(0)
    qs = rng.integers(0, spec.q, 40)
    js = np.concatenate([[0, 0, 10, 10, 5, 1], rng.integers(0, 11, 34)])
    iis = np.concatenate([[0, 14, 0, 14, 7, 13], rng.integers(0, 15, 34)])
    got = o.heun_step_entries(psi0, st, qs, js, iis)
    assert np.max(np.abs(got - full[qs, js, iis])) < 1e-13 * np.abs(full).max()


def test_twelve_ordinate_artificial_scattering_ratio_near_the_paper():
    # Section 4.1 parameter study: 12 icosahedron ordinates, 50^2 cells, Heun +
    # minmod; beta = 4.5, sigma_as = 5 reaches 37.8 % of the sigma_as = 0 error of
    # Phi.  (The paper's 12-point table is not a regular icosahedron and its
    # reference solution and CFL reading may differ, so the band is wide.)
    ref = 4 * math.pi * L.line_source_on_grid(50, 1.0, wl.LINE_SOURCE_DELTA, n_k=800, n_tau=1200)
    err = {}
    for s_as in (0.0, 5.0):
        spec = wl.line_source(50, sigma_as=s_as, beta=4.5)
        spec.ico_order = 2
        psi, st, _ = o.run_heun(spec)
        phi = o.scalar_flux(psi, st.w)
        err[s_as] = np.linalg.norm(phi - ref) / np.linalg.norm(ref)
    assert 0.3 < err[5.0] / err[0.0] < 0.5
