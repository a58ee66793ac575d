"""Pins for the stability number of the explicit schemes and the stiff time-step
rule.  The number is exact for the modes it is built from: a cell-to-cell
sawtooth of one ordinate, and of two ordinates with the same projection that
alternate in sign across them.  Its growth factor per step is 1 - z (forward
Euler) and 1 - z + z^2/2 (Heun; the limiter takes every sawtooth slope to 0)."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import asn_oracle as o


def _uniform(nx, ny, sigma_s, sigma_a, sigma_as, omega, w, eps=0.5, dt=None, cfl=0.95):
    f = lambda v: np.full((ny, nx), v, dtype=np.float32)
    prob = wl.Problem(name="u", nx=nx, ny=ny, x_min=0.0, x_max=1.0, y_min=0.0, y_max=ny / nx,
                      n_polar=1, n_azim=1, sigma_s=f(sigma_s), sigma_a=f(sigma_a),
                      sigma_as=f(sigma_as), source=f(0.0), psi0_cell=f(0.0), t_final=1.0,
                      cfl=cfl)
    return prob, o.setup(prob, omega=omega, w=w, eps=eps, dt=dt)


def _z(st):
    return o.stability_number(st.omega, st.K, st.dx, st.dy, st.dt, st.sigma_s, st.sigma_a,
                              st.sigma_as)


def _saw(ny, nx):
    j, i = np.mgrid[0:ny, 0:nx]
    return np.where((i + j) % 2 == 0, 1.0, -1.0)


@pytest.mark.parametrize("scheme", ["euler", "heun"])
@pytest.mark.parametrize("sigma_a,dt", [(0.5, 0.02), (40.0, 0.025), (10.0, 0.04)])
def test_single_ordinate_sawtooth_grows_by_the_predicted_factor(scheme, sigma_a, dt):
    om = np.array([[0.6, -0.48, math.sqrt(1 - 0.36 - 0.2304)]])
    prob, st = _uniform(40, 40, 0.0, sigma_a, 0.0, om, np.array([4 * math.pi]), dt=dt)
    z = _z(st)
    assert z == pytest.approx(dt * (2 * (0.6 + 0.48) * 40 + sigma_a), rel=1e-14)
    g = 1 - z if scheme == "euler" else 1 - z + 0.5 * z * z
    step = o.step if scheme == "euler" else o.heun_step
    psi = _saw(40, 40)[None]
    for _ in range(3):
        psi, _ = step(psi, st, want_budget=False)
    inner = psi[0, 14:26, 14:26] / _saw(40, 40)[14:26, 14:26]
    assert np.max(np.abs(inner - g ** 3)) < 1e-12 * max(1.0, abs(g) ** 3)


@pytest.mark.parametrize("scheme", ["euler", "heun"])
def test_two_mirrored_ordinates_attain_the_bound(scheme):
    # Same projection (xi, eta), opposite mu, equal weights: a sawtooth of opposite
    # sign on the two ordinates has no scalar flux, and K maps it to (2 K_11 - 1)
    # times itself, so its decay rate is sigma_a + sigma_s + 2 (1 - K_11) sigma_as,
    # the bracket of the stability number.
    mu = 0.5
    s = math.sqrt(1 - mu * mu)
    om = np.array([[s * math.cos(0.3), s * math.sin(0.3), mu],
                   [s * math.cos(0.3), s * math.sin(0.3), -mu]])
    w = np.array([2 * math.pi, 2 * math.pi])
    prob, st = _uniform(30, 30, 0.75, 0.375, 6.0, om, w, eps=0.8, dt=0.03)
    assert 0.5 < st.K[0, 0] < 0.99
    z = _z(st)
    rate = 2 * 30 * (abs(om[0, 0]) + abs(om[0, 1])) + 0.375 + 0.75 + 2 * (1 - st.K[0, 0]) * 6.0
    assert z == pytest.approx(0.03 * rate, rel=1e-13)
    g = 1 - z if scheme == "euler" else 1 - z + 0.5 * z * z
    step = o.step if scheme == "euler" else o.heun_step
    saw = _saw(30, 30)
    psi = np.stack([saw, -saw])
    for _ in range(2):
        psi, _ = step(psi, st, want_budget=False)
    ratio = psi[:, 10:20, 10:20] / np.stack([saw, -saw])[:, 10:20, 10:20]
    assert np.max(np.abs(ratio - g ** 2)) < 1e-12


def test_bound_covers_every_sawtooth_mode_of_a_product_set():
    # Exact rate matrix of the sawtooth in a uniform medium, all ordinates coupled:
    # its largest eigenvalue never exceeds the stability number's rate.
    om, w = o.product_quadrature(4, 8)
    for beta, (s_s, s_a, s_as) in [(4.5, (1.0, 0.0, 5.0)), (1.5, (0.3, 2.0, 1.0)),
                                   (40.0, (0.0, 10.0, 5.0))]:
        K = o.as_kernel_matrix(om, w, beta / w.size, "sym")
        dx = dy = 0.01
        r = np.abs(om[:, 0]) / dx + np.abs(om[:, 1]) / dy
        A = (np.diag(2 * r) + (s_a + s_s + s_as) * np.eye(w.size) - s_as * K
             - s_s * np.outer(np.ones(w.size), w) / w.sum())
        lam = np.linalg.eigvals(A)
        assert np.max(np.abs(lam.imag)) < 1e-9 * np.max(np.abs(lam))
        rate = o.stability_number(om, K, dx, dy, 1.0, np.array([s_s]), np.array([s_a]),
                                  np.array([s_as]))
        assert lam.real.max() <= rate * (1 + 1e-12)


def test_stiff_rule_keeps_the_coarse_lattice_stable():
    # 70^2 cells, 32 ordinates, sigma_a = 10: the streaming rule's dt is outside the
    # explicit stability interval and the discrete solution grows without bound;
    # the stiff rule's dt is inside and the run stays non-negative and bounded by
    # the source-over-absorption level.
    spec = wl.checkerboard(70, n_polar=4, sigma_as=5.0, t_final=3.2)
    st = o.setup(spec)
    stiff = o.setup(spec, dt_rule="stiff")
    assert _z(st) > 2.5 and _z(stiff) <= 2 * spec.cfl * (1 + 1e-12)
    assert stiff.dt * np.max(np.abs(stiff.omega[:, 0]) / stiff.dx
                             + np.abs(stiff.omega[:, 1]) / stiff.dy) <= spec.cfl
    assert stiff.n_steps * stiff.dt == pytest.approx(3.2, rel=1e-14)
    psi, _, _ = o.run(spec, st=stiff)
    assert psi.min() >= 0.0 and psi.max() < 0.01
    psi_bad = spec.psi0().astype(np.float64)
    for _ in range(st.n_steps):
        psi_bad, _ = o.step(psi_bad, st, want_budget=False)
    assert np.abs(psi_bad).max() > 100 * psi.max()


def test_stiff_rule_matches_streaming_rule_where_streaming_dominates():
    spec = wl.line_source(40, n_polar=2, sigma_as=0.0, sigma_s=0.0)
    st, stiff = o.setup(spec), o.setup(spec, dt_rule="stiff")
    # no collisions: rate 2 r_max, 2 cfl / (2 r_max) = cfl / r_max
    assert stiff.n_steps == st.n_steps and stiff.dt == st.dt
