"""Continuous-angle line-source references (TEST INFRASTRUCTURE ONLY).

The paper compares against a semi-analytic solution of the full transport
problem (Section 4.1) that it does not print.  This module derives its own:

* uncollided flux of a unit line source pulse (no scattering in flight): the
  3-D point-source shell projected along z gives, for rho < t,
      Phi_un(rho, t) = exp(-sigma_t t) / (2 pi t sqrt(t^2 - rho^2));
* the full flux with isotropic scattering: in 2-D Fourier space the scalar
  flux obeys, for every wave number k, the Volterra equation
      F(k, t) = e^{-sigma_t t} j0(k t) F0(k)
                + sigma_s int_0^t e^{-sigma_t tau} j0(k tau) F(k, t - tau) dtau,
  j0(x) = sin(x)/x (the Fourier transform of the unit shell), and
      Phi(rho, t) = (1 / 2 pi) int_0^inf k J0(k rho) F(k, t) dk.
  A Gaussian initial pulse of unit mass and variance parameter delta has
  F0(k) = exp(-delta k^2).  The Volterra equation is solved by the trapezoidal
  rule in tau and the Hankel transform by Gauss-Legendre in k.

The flux returned is for unit total initial mass; the paper's initial state
psi0 = exp(-r^2/(4 delta))/(4 pi delta) per steradian carries 4 pi.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import j0 as bessel_j0


def uncollided_line_source(rho: np.ndarray, t: float, sigma_t: float = 1.0) -> np.ndarray:
    rho = np.asarray(rho, dtype=np.float64)
    out = np.zeros_like(rho)
    inside = rho < t
    out[inside] = math.exp(-sigma_t * t) / (2.0 * math.pi * t * np.sqrt(t * t - rho[inside] ** 2))
    return out


def _sinc(x: np.ndarray) -> np.ndarray:
    return np.sinc(x / math.pi)


def fourier_flux(k: np.ndarray, t: float, delta: float, sigma_s: float = 1.0,
                 sigma_t: float = 1.0, n_tau: int = 2000) -> np.ndarray:
    """F(k, t) for every k by the trapezoidal rule on the Volterra equation above."""
    k = np.asarray(k, dtype=np.float64)
    tau = np.linspace(0.0, t, n_tau + 1)
    h = tau[1] - tau[0]
    f0 = np.exp(-delta * k * k)
    g = sigma_s * np.exp(-sigma_t * tau)[:, None] * _sinc(np.outer(tau, k))   # [n_tau+1, nk]
    src = np.exp(-sigma_t * tau)[:, None] * _sinc(np.outer(tau, k)) * f0[None, :]
    F = np.zeros((n_tau + 1, k.size))
    F[0] = f0
    for n in range(1, n_tau + 1):
        # F_n = src_n + h [ g_0 F_n / 2 + sum_{m=1}^{n-1} g_m F_{n-m} + g_n F_0 / 2 ]
        acc = 0.5 * g[n] * F[0]
        if n > 1:
            acc = acc + np.einsum("mk,mk->k", g[1:n], F[n - 1:0:-1])
        F[n] = (src[n] + h * acc) / (1.0 - 0.5 * h * g[0])
    return F[-1]


def line_source_flux(rho: np.ndarray, t: float, delta: float, sigma_s: float = 1.0,
                     sigma_t: float = 1.0, k_max: float = None, n_k: int = 1500,
                     n_tau: int = 2000) -> np.ndarray:
    """Scalar flux at radii rho for a unit-mass Gaussian pulse (Hankel inversion)."""
    if k_max is None:
        k_max = math.sqrt(40.0 / delta)
    x, wq = np.polynomial.legendre.leggauss(n_k)
    k = 0.5 * k_max * (x + 1.0)
    wk = 0.5 * k_max * wq
    F = fourier_flux(k, t, delta, sigma_s, sigma_t, n_tau)
    rho = np.asarray(rho, dtype=np.float64)
    J = bessel_j0(np.outer(rho.ravel(), k))
    out = (J * (wk * k * F)[None, :]).sum(axis=1) / (2.0 * math.pi)
    return out.reshape(rho.shape)


def line_source_on_grid(n: int, t: float, delta: float, half_width: float = 1.5,
                        sigma_s: float = 1.0, sigma_t: float = 1.0, n_rho: int = 600,
                        **kw) -> np.ndarray:
    """Reference flux at the n x n cell centres of [-half_width, half_width]^2."""
    h = 2.0 * half_width / n
    xc = -half_width + (np.arange(n) + 0.5) * h
    r = np.sqrt(xc[None, :] ** 2 + xc[:, None] ** 2)
    radii = np.linspace(0.0, r.max() * 1.0001, n_rho)
    prof = line_source_flux(radii, t, delta, sigma_s, sigma_t, **kw)
    return np.interp(r, radii, prof)
