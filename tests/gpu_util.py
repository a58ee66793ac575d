"""Helpers shared by the GPU tests: run a problem through the C ABI and through
the oracle on identical seeded inputs."""
from __future__ import annotations

import math

import numpy as np

import workloads as wl
from oracle import asn_oracle as o


def gpu_run(asn, spec, n_steps, psi0=None, dtype="f32", norm="sym", eps_override=0.0,
            scheme="euler", dt=0.0, unfused=False, form=None, scale_block=256):
    """Advance ``spec`` on the GPU; returns (state, phi, budget, info).  The kernel
    form is ``form`` if given, else fused (unfused False) or separate (True)."""
    p = asn.from_spec(spec, dtype=dtype, norm=norm, eps_override=eps_override,
                      set_initial_state=psi0 is None, scheme=scheme, dt_override=dt,
                      unfused=unfused, form=form, scale_block=scale_block)
    if form is not None:
        assert asn.asn_step_form(p) == (form if form != "auto" else asn.asn_step_form(p))
    try:
        if psi0 is not None:
            asn.asn_set_state(p, psi0)
        asn.asn_step(p, n_steps)
        return (asn.asn_get_state(p), asn.asn_scalar_flux(p), asn.asn_mass_budget(p),
                asn.asn_info(p))
    finally:
        p.close()


def oracle_run(spec, n_steps, psi0=None, norm="sym", eps=None, scheme="euler", dt=None):
    st = o.setup(spec, mode=norm, eps=eps, dt=dt)
    psi = (spec.psi0() if psi0 is None else psi0).astype(np.float64)
    step = o.heun_step if scheme == "heun" else o.step
    for _ in range(n_steps):
        psi, _ = step(psi, st, want_budget=False)
    return psi, o.scalar_flux(psi, st.w), st


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def fp32_budget_floor(state, w):
    """Relative size of the FP32 storage rounding of the mass: 2^-24 ||w psi||_2 / ||w psi||_1."""
    wp = np.abs(state.astype(np.float64) * w[:, None, None])
    return 2.0 ** -24 * math.sqrt(float(np.sum(wp * wp))) / float(np.sum(wp))


def structured_state(spec, rng):
    """A full-size anisotropic state psi0 = a1_q * cell + a2_q * mean(cell) (FP32
    products, then FP32 sums), built in place."""
    Q, ny, nx = spec.q, spec.ny, spec.nx
    a1 = (0.5 + rng.random(Q)).astype(np.float32)
    a2 = rng.standard_normal(Q).astype(np.float32) * np.float32(0.3)
    psi0 = np.empty((Q, ny, nx), dtype=np.float32)
    np.multiply(a1[:, None, None], spec.psi0_cell[None], out=psi0)
    psi0 += (a2 * np.float32(spec.psi0_cell.mean()))[:, None, None]
    return psi0


def sampled_entries(rng, Q, ny, nx, n_samples, n_centre=0):
    """(q, j, i) sample: uniform entries plus every corner / edge-midpoint class at
    four ordinates (first, two interior, last), and n_centre more entries within six
    cells of the grid's centre (where a centred pulse is large)."""
    qs = rng.integers(0, Q, n_samples)
    js = rng.integers(0, ny, n_samples)
    iis = rng.integers(0, nx, n_samples)
    edge = np.array([[0, 0], [0, nx - 1], [ny - 1, 0], [ny - 1, nx - 1], [0, nx // 2],
                     [ny // 2, 0], [ny - 1, nx // 2], [ny // 2, nx - 1]])
    k = len(edge) * 4
    js[:k] = np.repeat(edge[:, 0], 4)
    iis[:k] = np.repeat(edge[:, 1], 4)
    qs[:k] = np.tile([0, Q // 4 + 1, Q // 2 + 3, Q - 1], len(edge))
    if n_centre:
        qs = np.concatenate([qs, rng.integers(0, Q, n_centre)])
        js = np.concatenate([js, np.clip(ny // 2 + rng.integers(-6, 7, n_centre), 0, ny - 1)])
        iis = np.concatenate([iis, np.clip(nx // 2 + rng.integers(-6, 7, n_centre), 0, nx - 1)])
    return qs, js, iis


def sampled_phi(psi0, w, js, iis):
    """The scalar flux of psi0 (FP64) at the sampled cells; zero elsewhere."""
    phi = np.zeros(psi0.shape[1:])
    phi[js, iis] = w @ psi0[:, js, iis].astype(np.float64)
    return phi
