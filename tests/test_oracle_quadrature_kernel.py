"""Pins for the oracle's quadrature (P1) and artificial-scattering kernel (P2).

Each check compares against something other than the oracle itself: a library
routine, an exact moment, a closed form, or a structural invariant that a
dropped term, a wrong sign or a transposed operand would break.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import eval_legendre

from oracle import asn_oracle as o


# ---------------------------------------------------------------- P1 quadrature

@pytest.mark.parametrize("n", [1, 2, 3, 8, 12, 16, 24, 32])
def test_gauss_legendre_matches_library(n):
    x, w = o.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(x - xr)) < 1e-14
    assert np.max(np.abs(w - wr)) < 1e-14


@pytest.mark.parametrize("n_polar,n_azim", [(2, 4), (8, 16), (16, 32), (24, 48), (32, 64)])
def test_product_quadrature_exact_moments(n_polar, n_azim):
    om, w = o.product_quadrature(n_polar, n_azim)
    xi, eta, mu = om.T
    assert w.size == n_polar * n_azim
    assert np.all(w > 0)
    assert np.allclose(np.linalg.norm(om, axis=1), 1.0, atol=1e-15)
    four_pi = 4.0 * math.pi
    assert abs(w.sum() - four_pi) < 1e-13
    for v in (xi, eta, mu):
        assert abs(np.dot(w, v)) < 1e-14
    for v in (xi, eta, mu):
        assert abs(np.dot(w, v * v) - four_pi / 3.0) < 1e-13
    assert abs(np.dot(w, xi * eta)) < 1e-14
    # Gauss-Legendre integrates mu^(2k) exactly up to degree 2 n_polar - 1.
    for k in range(0, n_polar):
        assert abs(np.dot(w, mu ** (2 * k)) - four_pi / (2 * k + 1)) < 1e-13
    # Uniform azimuths integrate cos(m phi), sin(m phi) exactly for 0 < m < n_azim.
    phi = np.arctan2(eta, xi)
    for m in range(1, n_azim):
        assert abs(np.dot(w, np.cos(m * phi))) < 1e-12
        assert abs(np.dot(w, np.sin(m * phi))) < 1e-12


def test_product_quadrature_ordering_and_offset():
    om, w = o.product_quadrature(3, 8)
    mu = om[:, 2].reshape(3, 8)
    assert np.all(mu == mu[:, :1])                       # polar-major: q = i * n_azim + k
    assert np.all(np.diff(mu[:, 0]) > 0)
    phi = np.mod(np.arctan2(om[:8, 1], om[:8, 0]), 2 * math.pi)
    assert np.allclose(phi, (np.arange(8) + 0.5) * 2 * math.pi / 8, atol=1e-14)
    assert np.all(np.abs(om[:, 0]) > 1e-3) and np.all(np.abs(om[:, 1]) > 1e-3)


# ---------------------------------------------------------------- P2 kernel

@pytest.mark.parametrize("eps", [0.5, 0.1, 0.02, 0.0088])
def test_s_eps_is_normalised_dirac_sequence(eps):
    # int_{-1}^{1} s_eps(mu) dmu = 1 (Section 2.3), by adaptive library quadrature.
    val, err = integrate.quad(lambda m: o.s_eps(m, eps), -1.0, 1.0, points=[1.0 - 3 * eps],
                              epsabs=1e-14, epsrel=1e-13, limit=200)
    assert abs(val - 1.0) < 1e-11


@pytest.mark.parametrize("i", [0, 1, 2, 3])
@pytest.mark.parametrize("eps", [1.5, 0.3, 0.05])
def test_transport_coefficient_closed_form(i, eps):
    val, _ = integrate.quad(lambda m: (1 - m) ** i * o.s_eps(m, eps), -1.0, 1.0,
                            epsabs=1e-15, epsrel=1e-12, limit=200)
    assert abs(o.transport_coefficient(i, eps) - val) <= 1e-10 * max(1.0, abs(val))


def test_transport_coefficient_order_eps():
    # p_{eps,i} = O(eps^i): the ratio p / eps^i tends to Gamma((i+1)/2)/sqrt(pi).
    from scipy.special import gamma
    for i in (1, 2, 3):
        lim = gamma(0.5 * (i + 1)) / math.sqrt(math.pi)
        assert abs(o.transport_coefficient(i, 0.01) / 0.01 ** i - lim) < 1e-12


def test_kernel_width_rule():
    assert o.kernel_width(92, 4.5) == pytest.approx(4.5 / 92)
    assert o.kernel_width(2048, 4.5) == pytest.approx(4.5 / 2048)


@pytest.mark.parametrize("mode", ["sym", "row"])
@pytest.mark.parametrize("n_polar", [2, 8, 16])
def test_kernel_rows_sum_to_one_and_nonnegative(mode, n_polar):
    om, w = o.product_quadrature(n_polar, 2 * n_polar)
    K = o.as_kernel_matrix(om, w, o.kernel_width(w.size, 4.5), mode)
    assert np.all(K >= 0)
    assert np.max(np.abs(K.sum(axis=1) - 1.0)) < 1e-14
    # An isotropic state is a fixed point of K in both modes.
    assert np.max(np.abs(K @ np.full(w.size, 3.25) - 3.25)) < 1e-13


@pytest.mark.parametrize("n_polar", [2, 8, 16, 24])
def test_sym_kernel_conserves_particles_and_is_self_adjoint(n_polar):
    om, w = o.product_quadrature(n_polar, 2 * n_polar)
    Q = w.size
    K = o.as_kernel_matrix(om, w, o.kernel_width(Q, 4.5), "sym")
    # w-weighted column sums equal w: sum_q w_q (K psi)_q = sum_p w_p psi_p.
    assert np.max(np.abs(w @ K - w) / w) < 1e-13
    sw = np.sqrt(w)
    A = sw[:, None] * K / sw[None, :]
    assert np.max(np.abs(A - A.T)) < 1e-14
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.max() == pytest.approx(1.0, abs=1e-13)
    assert ev.min() >= -1.0 - 1e-13


def test_row_kernel_is_paper_normalisation():
    # K_qp = w_p c_q s(Omega_q . Omega_p), c_q = 1 / sum_p w_p s_qp, from the dot products.
    om, w = o.product_quadrature(4, 8)
    eps = 0.3
    Q = w.size
    ref = np.zeros((Q, Q))
    for q in range(Q):
        s = np.array([o.s_eps(np.dot(om[q], om[p]), eps) for p in range(Q)])
        ref[q] = w * s / np.dot(w, s)
    K = o.as_kernel_matrix(om, w, eps, "row")
    assert np.max(np.abs(K - ref)) < 1e-15


def _legendre_eigenvalue(n, eps):
    num, _ = integrate.quad(lambda m: o.s_eps(m, eps) * eval_legendre(n, m), -1, 1,
                            epsabs=1e-15, epsrel=1e-13, limit=400)
    den, _ = integrate.quad(lambda m: o.s_eps(m, eps), -1, 1, epsabs=1e-15, epsrel=1e-13)
    return num / den


@pytest.mark.parametrize("mode", ["sym", "row"])
def test_funk_hecke_on_fine_quadrature(mode):
    # For a wide kernel on a fine product set, K acting on P_n(Omega . e) returns
    # lambda_n P_n(Omega . e) with lambda_n = int s_eps P_n / int s_eps (Funk-Hecke);
    # for n = 1, lambda_1 = 1 - p_{eps,1} (Section 2.5 transport coefficient).
    eps = 0.3
    om, w = o.product_quadrature(32, 64)
    K = o.as_kernel_matrix(om, w, eps, mode)
    lam1 = 1.0 - o.transport_coefficient(1, eps)
    assert _legendre_eigenvalue(1, eps) == pytest.approx(lam1, abs=1e-12)
    for axis in (np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0]),
                 np.array([0.6, 0.0, 0.8])):
        c = om @ axis
        for n in (1, 2, 3):
            f = eval_legendre(n, c)
            lam = _legendre_eigenvalue(n, eps)
            assert np.max(np.abs(K @ f - lam * f)) < 1e-12, (n, axis)


def test_kernel_sharpens_with_more_ordinates():
    # eps = beta / N_q shrinks, so the forward peak (diagonal weight) grows with Q.
    diag = []
    for n_polar in (4, 8, 16):
        om, w = o.product_quadrature(n_polar, 2 * n_polar)
        K = o.as_kernel_matrix(om, w, o.kernel_width(w.size, 4.5), "sym")
        diag.append(np.dot(w, K.diagonal()) / w.sum())
    assert diag[0] < diag[1] < diag[2]
