"""Pins for the oracle's reduced-precision emulation of the in-scattering sum."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import asn_oracle as o


def _floats(seed, n=20000):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal(n) * np.exp2(rng.integers(-30, 30, n))).astype(np.float32)
    # Exact ties for bf16 (low 16 bits 0x8000) and neighbours of them.
    b = x[:2000].view(np.uint32) & np.uint32(0xFFFF0000)
    ties = (b | np.uint32(0x8000)).view(np.float32)
    return np.concatenate([x, ties, np.nextafter(ties, np.float32(np.inf))])


def test_bf16_rounding_matches_library():
    x = _floats(1)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(o.round_bf16(x), ref)


def test_f16_rounding_matches_library():
    rng = np.random.default_rng(2)
    x = (rng.standard_normal(50000) * np.exp2(rng.integers(-26, 16, 50000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float16).to(torch.float32).numpy()
    assert np.array_equal(o.round_f16(x), ref)


def _setup(n_polar=4, nx=37, ny=9, seed=3):
    prob = wl.random_problem(seed, nx, ny, n_polar=n_polar, n_azim=2 * n_polar, beta=4.5)
    return o.setup(prob), prob


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_isotropic_state_exact(dtype):
    st, _ = _setup()
    psi = np.broadcast_to(wl.random_state(5, 1, 9, 37), (st.q, 9, 37)).astype(np.float32)
    Y = o.lowprec_in_scattering(psi, st, dtype)
    assert np.array_equal(Y, psi.astype(np.float64))


@pytest.mark.parametrize("dtype", ["bf16", "f16", "f32"])
def test_particle_fix_and_accuracy(dtype):
    st, _ = _setup()
    psi = wl.random_state(6, st.q, 9, 37)
    Y = o.lowprec_in_scattering(psi, st, dtype)
    Yx = o.as_in_scattering(psi.astype(np.float64), st.K)
    phi = o.scalar_flux(psi.astype(np.float64), st.w)
    # The fix makes sum_q w_q Y_q equal Phi in every cell.
    assert np.max(np.abs(o.scalar_flux(Y, st.w) - phi) / phi) < 1e-14
    dev = np.abs(psi - phi / st.W).max()
    bound = {"bf16": 2.0 ** -7, "f16": 2.0 ** -10, "f32": 2.0 ** -21}[dtype]
    err = np.abs(Y - Yx).max()
    assert err < bound * dev
    if dtype != "f32":
        assert err > 2.0 ** -16 * dev          # the rounding is really applied


@pytest.mark.parametrize("block", [64, 256, 4096])
def test_block_exponents_bound_block_maximum(block):
    # 23 x 211 = 4853 cells: a ragged last block at every size
    rng = np.random.default_rng(7)
    psi = (rng.random((3, 23, 211)) * np.exp2(rng.integers(-20, 20, (1, 23, 211)))).astype(np.float32)
    e = o.block_exponents(psi, block)
    flat = np.abs(psi.reshape(3, -1)).max(axis=0)
    for b in range(0, flat.size, block):
        m = flat[b:b + block].max()
        eb = e[b]
        assert np.all(e[b:b + block] == eb)
        assert 2.0 ** (eb - 1) <= m < 2.0 ** eb


def _banded_magnitude_state(st, seed, ratio_exp):
    """A 32 x 128 state whose rows 0-15 are 2^ratio_exp times smaller than rows 16-31:
    blocks of 64 cells (half a row) never mix the two bands, blocks of 4096 do."""
    psi = wl.random_state(seed, st.q, 32, 128)
    psi[:, :16] *= np.float32(2.0 ** ratio_exp)
    return psi


def test_scale_block_leaves_bf16_unchanged_and_sets_f16_subnormal_range():
    # Scaling by a power of two commutes with rounding while the scaled operand stays a
    # normal number: the two-term BF16 operand (8 exponent bits) gives the same Y for
    # every block size.  FP16 (5 exponent bits) does not: with one scale for both bands
    # the small band's operands fall below 2^-14 and lose bits to the subnormal spacing,
    # with blocks of 64 each band keeps 11 significant bits.
    prob = wl.random_problem(11, 128, 32, n_polar=4, n_azim=8, beta=4.5)
    st = o.setup(prob)
    psi = _banded_magnitude_state(st, 12, -30)
    Yx = o.as_in_scattering(psi.astype(np.float64), st.K)
    small = (slice(None), slice(0, 16))
    phi = o.scalar_flux(psi.astype(np.float64), st.w)
    dev_small = np.abs(psi[small] - (phi / st.W)[:16]).max()
    y64 = o.lowprec_in_scattering(psi, st, "bf16", block=64)
    y4k = o.lowprec_in_scattering(psi, st, "bf16", block=4096)
    assert np.array_equal(y64, y4k)
    f64 = o.lowprec_in_scattering(psi, st, "f16", block=64)
    f4k = o.lowprec_in_scattering(psi, st, "f16", block=4096)
    e64 = np.abs(f64[small] - Yx[small]).max()
    e4k = np.abs(f4k[small] - Yx[small]).max()
    assert e64 < 2.0 ** -10 * dev_small
    assert e4k > 8 * e64


def test_scaled_operands_fit_half_range():
    # |psi - iso| <= 2 max|psi| < 2^(e+1), so scaled operands stay below 2^15.
    st, _ = _setup()
    psi = (wl.random_state(8, st.q, 9, 37) * np.float32(3e4)).astype(np.float32)
    p = psi.reshape(st.q, -1)
    iso = (o.scalar_flux(psi.astype(np.float64), st.w).ravel() / st.W).astype(np.float32)
    dev = p - iso[None]
    e = o.block_exponents(p)
    assert np.abs(dev * np.exp2(o.SCALE_EXP - e)[None]).max() <= 2.0 ** 15


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_lowprec_step_is_close_to_exact_step(dtype):
    st, prob = _setup(n_polar=4, nx=23, ny=17, seed=4)
    psi32 = wl.random_state(9, st.q, 17, 23)
    new, b = o.lowprec_step(psi32, st, dtype)
    ref, _ = o.step(psi32.astype(np.float64), st)
    rel = np.linalg.norm(new - ref) / np.linalg.norm(ref)
    assert rel < {"bf16": 2e-3, "f16": 3e-4}[dtype]
    assert abs(b["as_defect"]) < 1e-12 * b["mass"]


def test_row_defect_correction_removes_row_sum_bias():
    # With a smooth deviation that is exactly representable in bf16 the operand
    # rounding vanishes; the only error left is from the rounded kernel.  Adding
    # r_q dev_q makes the effective rows sum to one, so the error shrinks to the
    # kernel's local variation instead of r_q dev_q.
    prob = wl.random_problem(3, 16, 16, n_polar=16, n_azim=32, beta=4.5)
    st = o.setup(prob)
    d = o.round_bf16((0.25 * st.omega[:, 0]).astype(np.float32))
    psi = np.broadcast_to((1.0 + d)[:, None, None], (st.q, 16, 16)).astype(np.float32)
    kq, r = o.lowprec_kernel(st.K, "bf16")
    Yx = o.as_in_scattering(psi.astype(np.float64), st.K)
    with_r = np.abs(o.lowprec_in_scattering(psi, st, "bf16", kq, r) - Yx).max()
    without = np.abs(o.lowprec_in_scattering(psi, st, "bf16", kq, 0.0 * r) - Yx).max()
    assert with_r < 0.5 * without


def test_block_exponent_is_clamped_for_tiny_blocks():
    psi = np.full((2, 1, 300), 1e-40, dtype=np.float32)
    psi[:, 0, 256:] = 3.0
    e = o.block_exponents(psi)
    assert e[0] == o.SCALE_EXP_MIN and e[299] == 2
    assert np.isfinite(np.ldexp(np.float32(1.0), o.SCALE_EXP - e[0]))


def test_bf16_operand_split_carries_sixteen_bits():
    rng = np.random.default_rng(11)
    s = (rng.standard_normal(100000) * np.exp2(rng.integers(-20, 14, 100000))).astype(np.float32)
    x = o.operand_terms(s, "bf16")
    assert np.all(np.abs(x - s) <= 2.0 ** -16 * np.abs(s))
    hi = o.round_bf16(s)
    assert np.array_equal(o.round_bf16(hi), hi)                # both terms are bf16 values
    assert np.abs(x - s).max() < np.abs(hi - s).max() / 100


@pytest.mark.slow
def test_bf16_recipe_meets_bound_on_lattice_where_single_term_would_not():
    # Quasi-steady regions of the lattice problem round the same operand values the
    # same way every step, so single-term BF16 operands bias the solution (3.6e-3
    # here); the two-term operand keeps the scalar flux within 2e-3 of the exact step.
    spec = wl.checkerboard(70, n_polar=8, sigma_as=5.0)
    st = o.setup(spec)
    kq, r = o.lowprec_kernel(st.K, "bf16")
    ex = spec.psi0().astype(np.float64)
    lp = spec.psi0().astype(np.float32)
    for _ in range(st.n_steps):
        ex, _ = o.step(ex, st, want_budget=False)
        lp = o.lowprec_step(lp, st, "bf16", kq, r)[0].astype(np.float32)
    phi_ex = o.scalar_flux(ex, st.w)
    err = np.linalg.norm(o.scalar_flux(lp.astype(np.float64), st.w) - phi_ex) / np.linalg.norm(phi_ex)
    assert err < 2e-3


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_entrywise_step_equals_full_emulated_step(dtype):
    # the sampled evaluator used at full size: the same recipe per cell, the exponent of
    # each cell's whole scale block (blocks of 64 on a ragged 23 x 11 grid: 4 blocks, the
    # last partial), the step on the cell's window; entries on the edges and corners too
    prob = wl.random_problem(11, 23, 11, n_polar=4, n_azim=8, beta=4.5)
    st = o.setup(prob)
    psi = wl.random_state(12, st.q, 11, 23)
    psi[:, :3] *= np.float32(2.0 ** -20)        # blocks of very different scale
    full, _ = o.lowprec_step(psi, st, dtype, block=64)
    rng = np.random.default_rng(13)
    qs = rng.integers(0, st.q, 60)
    js = np.concatenate([[0, 10, 0, 10], rng.integers(0, 11, 56)])
    iis = np.concatenate([[0, 0, 22, 22], rng.integers(0, 23, 56)])
    got = o.lowprec_step_entries(psi, st, dtype, qs, js, iis, block=64)
    ref = full[qs, js, iis]
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.abs(full).max()
