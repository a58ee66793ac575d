"""Pins for the oracle's explicit step: P3 closed-form streaming, P4 brute-force
dense step matrix, P5 homogeneous interior, P6 isotropic preservation, P7 mass
budget, P9 instability of the literal dt/dx CFL reading.
"""
import math

import numpy as np
import pytest
from scipy.special import factorial

import workloads as wl
from oracle import asn_oracle as o


def _blank(nx, ny, n_polar=2, n_azim=4, sigma=(0.0, 0.0, 0.0), src=0.0, x=(0.0, 1.0),
           y=(0.0, 1.0), t_final=1.0, beta=1.5, cfl=0.9):
    f = lambda v: np.full((ny, nx), v, dtype=np.float32)
    return wl.Problem(name="blank", nx=nx, ny=ny, x_min=x[0], x_max=x[1], y_min=y[0], y_max=y[1],
                      n_polar=n_polar, n_azim=n_azim, sigma_s=f(sigma[0]), sigma_a=f(sigma[1]),
                      sigma_as=f(sigma[2]), source=f(src), psi0_cell=f(0.0), beta=beta,
                      t_final=t_final, cfl=cfl)


# ---------------------------------------------------------------- P3 closed form

@pytest.mark.parametrize("sx,sy", [(1, 1), (-1, 1), (1, -1), (-1, -1)])
def test_single_ordinate_delta_is_multinomial(sx, sy):
    # One ordinate (so K = [1] and the scattering gain equals its loss), a unit
    # delta far from the boundary: after n steps the donor-cell update spreads it as
    # n!/(a! b! c!) (1 - nu_x - nu_y - dt sigma_a)^a nu_x^b nu_y^c along (sx, sy).
    nx = ny = 21
    n = 6
    dx = 1.0 / nx
    xi, eta = 0.6 * sx, 0.48 * sy
    mu = math.sqrt(1 - xi * xi - eta * eta)
    om = np.array([[xi, eta, mu]])
    w = np.array([4 * math.pi])
    sig_a = float(np.float32(0.7))   # the fields are stored in float32
    prob = _blank(nx, ny, sigma=(1.3, sig_a, 2.1))
    dt = 0.5 * dx
    st = o.setup(prob, mode="row", omega=om, w=w, dt=dt)
    psi = np.zeros((1, ny, nx))
    j0 = i0 = 10
    psi[0, j0, i0] = 1.0
    for _ in range(n):
        psi, _ = o.step(psi, st, want_budget=False)
    nu_x, nu_y = dt * abs(xi) / dx, dt * abs(eta) / dx
    stay = 1 - nu_x - nu_y - dt * sig_a
    expect = np.zeros((ny, nx))
    for b in range(n + 1):
        for c in range(n + 1 - b):
            a = n - b - c
            coef = factorial(n, exact=True) // (factorial(a, exact=True) * factorial(b, exact=True)
                                                * factorial(c, exact=True))
            expect[j0 + sy * c, i0 + sx * b] = coef * stay ** a * nu_x ** b * nu_y ** c
    assert np.max(np.abs(psi[0] - expect)) < 1e-15


def test_axis_ordinate_at_unit_courant_shifts_exactly_and_outflow_balances():
    nx, ny = 7, 3
    om = np.array([[1.0, 0.0, 0.0]])
    w = np.array([4 * math.pi])
    prob = _blank(nx, ny)
    st = o.setup(prob, mode="row", omega=om, w=w, dt=1.0 / nx)
    psi = np.zeros((1, ny, nx))
    psi[0, 1, 2] = 5.0
    total_out = 0.0
    for k in range(7):
        m0 = o.mass(psi, st)
        psi_new, b = o.step(psi, st)
        assert o.budget_residual(b, o.mass(psi_new, st), st.dt) == pytest.approx(0.0, abs=1e-14)
        total_out += st.dt * b["outflow"]
        psi = psi_new
        if 2 + k + 1 < nx:
            assert psi[0, 1, 2 + k + 1] == 5.0 and np.count_nonzero(psi) == 1
    assert np.count_nonzero(psi) == 0
    assert total_out == pytest.approx(5.0 * 4 * math.pi * st.dx * st.dy, rel=1e-15)


# ---------------------------------------------------------------- P4 brute force

def _assemble_step_matrix(st, nx, ny):
    """The full one-step map psi_new = A psi + b, assembled entry by entry."""
    Q = st.w.size
    idx = lambda q, j, i: (q * ny + j) * nx + i
    N = Q * ny * nx
    A = np.zeros((N, N))
    b = np.zeros(N)
    for q in range(Q):
        xi, eta = st.omega[q, 0], st.omega[q, 1]
        for j in range(ny):
            for i in range(nx):
                r = idx(q, j, i)
                s_s, s_a, s_as = st.sigma_s[j, i], st.sigma_a[j, i], st.sigma_as[j, i]
                A[r, r] += 1.0 - st.dt * (s_s + s_a + s_as)
                A[r, r] -= st.dt * (abs(xi) / st.dx + abs(eta) / st.dy)
                up_i = i - 1 if xi > 0 else i + 1
                up_j = j - 1 if eta > 0 else j + 1
                if 0 <= up_i < nx:
                    A[r, idx(q, j, up_i)] += st.dt * abs(xi) / st.dx
                if 0 <= up_j < ny:
                    A[r, idx(q, up_j, i)] += st.dt * abs(eta) / st.dy
                for p in range(Q):
                    A[r, idx(p, j, i)] += st.dt * (s_s * st.w[p] / st.W + s_as * st.K[q, p])
                b[r] = st.dt * st.source[j, i]
    return A, b


@pytest.mark.parametrize("mode", ["sym", "row"])
def test_step_equals_brute_force_dense_matrix(mode):
    nx, ny = 5, 4
    prob = wl.random_problem(3, nx, ny, n_polar=2, n_azim=4)
    st = o.setup(prob, mode=mode)
    A, b = _assemble_step_matrix(st, nx, ny)
    psi = wl.random_state(11, st.q, ny, nx).astype(np.float64)
    new, _ = o.step(psi, st)
    assert np.max(np.abs(new.ravel() - (A @ psi.ravel() + b))) < 1e-14
    if mode == "sym":
        # Weighted column sums: 1 - dt sigma_a - (share of the ordinate leaving the domain).
        Q = st.q
        wv = np.repeat(st.w, ny * nx)
        col = (wv @ A) / wv
        expect = np.zeros((Q, ny, nx))
        for p in range(Q):
            xi, eta = st.omega[p, 0], st.omega[p, 1]
            e = 1.0 - st.dt * st.sigma_a
            if xi > 0:
                e[:, -1] -= st.dt * xi / st.dx
            else:
                e[:, 0] -= st.dt * -xi / st.dx
            if eta > 0:
                e[-1, :] -= st.dt * eta / st.dy
            else:
                e[0, :] -= st.dt * -eta / st.dy
            expect[p] = e
        assert np.max(np.abs(col - expect.ravel())) < 1e-14


def test_brute_force_with_custom_quadrature_not_summing_to_four_pi():
    # The isotropic gain is sigma_s sum_p w_p psi_p / sum_p w_p (c_q of eq. asSNeq for a
    # constant kernel), whatever the weights sum to.
    nx, ny = 4, 3
    rng = np.random.default_rng(12)
    om = rng.standard_normal((6, 3))
    om /= np.linalg.norm(om, axis=1)[:, None]
    w = rng.random(6) + 0.2
    prob = wl.random_problem(8, nx, ny)
    st = o.setup(prob, mode="row", omega=om, w=w)
    assert abs(st.W - 4 * np.pi) > 0.1
    A, b = _assemble_step_matrix(st, nx, ny)
    psi = wl.random_state(1, 6, ny, nx).astype(np.float64)
    new, _ = o.step(psi, st)
    assert np.max(np.abs(new.ravel() - (A @ psi.ravel() + b))) < 1e-14


def test_step_entries_agree_with_full_step():
    prob = wl.random_problem(5, 9, 7, n_polar=2, n_azim=8)
    st = o.setup(prob)
    psi = wl.random_state(2, st.q, 7, 9).astype(np.float64)
    full, _ = o.step(psi, st)
    rng = np.random.default_rng(0)
    qs, js, iis = rng.integers(0, st.q, 40), rng.integers(0, 7, 40), rng.integers(0, 9, 40)
    qs[:4], js[:4], iis[:4] = [0, 1, 2, 3], [0, 6, 0, 6], [0, 8, 8, 0]
    got = o.step_entries(psi, st, qs, js, iis)
    assert np.max(np.abs(got - full[qs, js, iis])) < 1e-14


# ---------------------------------------------------------------- P5 homogeneous interior

@pytest.mark.parametrize("mode", ["sym", "row"])
def test_homogeneous_interior_is_angular_matrix_power(mode):
    n = 5
    side = 2 * n + 3
    prob = _blank(side, side, n_polar=4, n_azim=8, sigma=(0.75, 0.25, 2.5), t_final=0.2)
    st = o.setup(prob, mode=mode)
    xi, mu = st.omega[:, 0], st.omega[:, 2]
    f0 = 1.0 + xi + 2.0 * mu * mu
    psi = np.broadcast_to(f0[:, None, None], (st.q, side, side)).copy()
    for _ in range(n):
        psi, _ = o.step(psi, st, want_budget=False)
    Q = st.q
    M = np.eye(Q) + st.dt * (-(0.75 + 0.25 + 2.5) * np.eye(Q)
                             + 0.75 * np.outer(np.ones(Q), st.w) / st.W + 2.5 * st.K)
    expect = np.linalg.matrix_power(M, n) @ f0
    c = side // 2
    for j in range(n, side - n):
        for i in range(n, side - n):
            assert np.max(np.abs(psi[:, j, i] - expect)) < 1e-13
    # Near the boundary the vacuum inflow must have changed the solution.
    assert np.max(np.abs(psi[:, 0, c] - expect)) > 1e-3


# ---------------------------------------------------------------- P6 isotropic states

@pytest.mark.parametrize("mode", ["sym", "row"])
def test_isotropic_state_preserved_away_from_boundary(mode):
    n = 4
    nx, ny = 2 * n + 4, 2 * n + 3
    prob = wl.random_problem(7, nx, ny, n_polar=3, n_azim=6)
    prob.sigma_a[:] = 0.0
    prob.source[:] = 0.0
    st = o.setup(prob, mode=mode)
    psi = np.full((st.q, ny, nx), 2.75)
    for _ in range(n):
        psi, _ = o.step(psi, st, want_budget=False)
    inner = psi[:, n:ny - n, n:nx - n]
    assert np.max(np.abs(inner - 2.75)) <= 4e-15 * 2.75


# ---------------------------------------------------------------- P7 mass budget

@pytest.mark.parametrize("mode", ["sym", "row"])
def test_mass_budget_identity(mode):
    prob = wl.random_problem(9, 11, 8, n_polar=3, n_azim=6, t_final=0.2, beta=4.5)
    st = o.setup(prob, mode=mode)
    psi0 = wl.random_state(4, st.q, 8, 11).astype(np.float64)
    psi, _, hist = o.run(prob, n_steps=15, st=st, psi0=psi0, budget=True)
    m0 = hist[0]["mass"]
    cum = 0.0
    for b in hist:
        res = o.budget_residual(b, b["mass_next"], st.dt)
        assert abs(res) <= 1e-13 * m0
        cum += res
    assert abs(cum) <= 1e-12 * m0
    b = hist[0]
    area = st.dx * st.dy
    if mode == "sym":
        assert abs(b["as_defect"]) <= 1e-13 * m0
    else:
        # Row mode conserves rows but not weighted columns: the defect is
        # sum_c sigma_as sum_p psi_p (col_p - w_p), col = w^T K.
        col = st.w @ st.K
        pred = area * np.sum(st.sigma_as * np.tensordot(col - st.w, psi0, axes=(0, 0)))
        assert b["as_defect"] == pytest.approx(pred, rel=1e-12, abs=1e-14 * m0)
        assert abs(b["as_defect"]) > 1e-6 * m0


def test_line_source_budget_closes_over_full_run():
    prob = wl.line_source(30, n_polar=4, sigma_as=1.0)
    psi, st, hist = o.run(prob, budget=True)
    m0 = hist[0]["mass"]
    assert max(abs(o.budget_residual(b, b["mass_next"], st.dt)) for b in hist) <= 1e-13 * m0
    # Nothing absorbs (sigma_a = 0): all mass lost left through the boundary.
    lost = sum(st.dt * b["outflow"] for b in hist)
    assert hist[-1]["mass_next"] == pytest.approx(m0 - lost, rel=1e-12)


# ---------------------------------------------------------------- P9 literal CFL

def test_literal_dt_over_dx_reading_is_unstable_and_proposed_reading_is_not():
    prob = wl.line_source(50, n_polar=8, sigma_as=1.0)
    st = o.setup(prob)
    dx = st.dx
    assert st.dt * np.max(np.abs(st.omega[:, 0]) / dx + np.abs(st.omega[:, 1]) / dx) <= 0.95 + 1e-12
    psi0 = prob.psi0().astype(np.float64)
    lit = o.setup(prob, dt=0.95 * dx)
    psi = psi0.copy()
    for _ in range(40):
        psi, _ = o.step(psi, lit, want_budget=False)
    assert np.max(np.abs(psi)) > 1e3 * np.max(psi0)
    psi = psi0.copy()
    for _ in range(40):
        psi, _ = o.step(psi, st, want_budget=False)
    assert np.max(np.abs(psi)) <= np.max(psi0)


def test_cfl_rule_values_for_the_workloads():
    # (grid, polar order) -> steps and dt from dt_max = 0.95 / max(|xi|/dx + |eta|/dy).
    cases = [(50, 8, 1.0, 3.0, 24), (400, 16, 1.0, 3.0, 197), (700, 24, 3.2, 7.0, 475),
             (1024, 32, 1.0, 3.0, 507)]
    for n, n_polar, tf, L, steps in cases:
        om, w = o.product_quadrature(n_polar, 2 * n_polar)
        dt, k = o.cfl_time_step(om, L / n, L / n, 0.95, tf)
        assert k == steps and dt == pytest.approx(tf / steps, rel=1e-15)


def test_windowed_entries_equal_the_full_run():
    # run_entries advances each sampled cell on its own (2n + 1)^2 window; every entry
    # (corners, edges, interior) must equal the full-grid run
    spec = wl.random_problem(21, 13, 9, n_polar=2, n_azim=4, beta=4.5)
    st = o.setup(spec)
    psi0 = wl.random_state(5, spec.q, 9, 13).astype(np.float64)
    n = 3
    full, _, _ = o.run(spec, n_steps=n, st=st, psi0=psi0)
    qs, js, iis = np.meshgrid(np.arange(spec.q), np.arange(9), np.arange(13), indexing="ij")
    got = o.run_entries(psi0, st, n, qs.ravel(), js.ravel(), iis.ravel())
    assert np.max(np.abs(got - full.ravel())) <= 1e-13 * np.abs(full).max()
