"""GPU parity of the banded reduced-precision step (BF16 / FP16 operands on MFMA, FP32
accumulate, product sets of 32, 48 or 64 azimuths): each level pair's circulant block of
the stored K multiplies the rounded partner level, the update follows the fused
reduced-precision form (pending per-cell particle correction).  Checked against the
oracle's emulation of the rounding recipe element by element on ragged grids (one
step <= 2e-6 of max|psi|), against the fused form, against the exact FP64 oracle over
several steps, with the particle budget, operand scale blocks of 64 and 4096 cells,
and batches."""
import numpy as np
import pytest

import workloads as wl
from oracle import asn_oracle as o
from gpu_util import fp32_budget_floor, gpu_run, oracle_run, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_1911_08801_amd import asn  # noqa: E402

GRIDS = [(1, 1), (9, 1), (1, 7), (33, 2), (65, 17), (130, 67), (200, 3)]
# (n_polar, n_azim, beta): every azimuth count; reach of the BF16 / FP16 K: 1/0, 2/1,
# 3/2, 0/0, 2/1, 1/1, 2/1, -
QUADS = [(4, 32, 4.5), (16, 32, 4.5), (16, 32, 12.0), (2, 64, 4.5), (16, 64, 9.0), (12, 64, 6.0),
         (24, 48, 4.5), (4, 48, 4.5)]


def _emulated(spec, n, psi0, dtype, block=o.SCALE_BLOCK):
    st = o.setup(spec)
    kq, r = o.lowprec_kernel(st.K, dtype)
    psi = psi0.astype(np.float32)
    for _ in range(n):
        new, _ = o.lowprec_step(psi, st, dtype, kq, r, block)
        psi = new.astype(np.float32)
    return psi, st


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
@pytest.mark.parametrize("nx,ny", GRIDS)
@pytest.mark.parametrize("n_polar,n_azim,beta", QUADS)
def test_one_step_matches_emulation(dtype, nx, ny, n_polar, n_azim, beta):
    spec = wl.random_problem(nx * 7 + ny + n_azim, nx, ny, n_polar=n_polar, n_azim=n_azim, beta=beta)
    psi0 = wl.random_state(nx + 3 * ny + n_polar, spec.q, ny, nx)
    print(f"banded {dtype} one step {nx}x{ny}, {n_polar}x{n_azim}, beta {beta}", flush=True)
    state, phi, bud, _ = gpu_run(asn, spec, 1, psi0=psi0, dtype=dtype, form="banded")
    ref, st = _emulated(spec, 1, psi0, dtype)
    assert np.max(np.abs(state - ref)) <= 2e-6 * np.abs(ref).max()
    # the fused form rounds the same operands; its FP32 sums run in another order
    fused, phi_f, _, _ = gpu_run(asn, spec, 1, psi0=psi0, dtype=dtype, form="fused")
    assert np.max(np.abs(state - fused)) <= 1e-6 * np.abs(fused).max()
    assert np.max(np.abs(phi - phi_f)) <= 1e-6 * np.abs(phi_f).max()


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
@pytest.mark.parametrize("n_polar,n_azim", [(8, 32), (4, 64)])
def test_multi_step_budget_and_exact_oracle(dtype, n_polar, n_azim):
    spec = wl.random_problem(3 + n_polar, 70, 33, n_polar=n_polar, n_azim=n_azim, beta=4.5,
                             t_final=0.3)
    psi0 = wl.random_state(9, spec.q, 33, 70)
    state, phi, bud, _ = gpu_run(asn, spec, 8, psi0=psi0, dtype=dtype, form="banded")
    ref, st = _emulated(spec, 8, psi0, dtype)
    assert rel_l2(state, ref) <= 1e-5
    exact, phi_ref, _ = oracle_run(spec, 8, psi0=psi0)
    assert rel_l2(phi, phi_ref) <= 2e-3
    assert bud["steps"] == 8
    assert bud["max_residual"] <= max(1e-10, 64 * fp32_budget_floor(state, st.w))


def test_line_source_full_run_against_exact_oracle():
    spec = wl.line_source(40, n_polar=16, sigma_as=5.0)   # 32 azimuths
    n = 24
    for dtype in ("bf16", "f16"):
        state, phi, bud, _ = gpu_run(asn, spec, n, dtype=dtype, form="banded")
        _, phi_ref, st = oracle_run(spec, n)
        assert rel_l2(phi, phi_ref) <= 2e-3
        assert bud["max_residual"] <= max(1e-10, 64 * fp32_budget_floor(state, st.w))


@pytest.mark.parametrize("block", [64, 4096])
@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_scale_block_matches_emulation(block, dtype):
    nx, ny = 128, 70
    spec = wl.random_problem(29, nx, ny, n_polar=4, n_azim=32, beta=4.5)
    spec.source[:] = 0.0
    psi0 = wl.random_state(30, spec.q, ny, nx)
    psi0[:, :16] *= np.float32(2.0 ** -50)
    state, _, _, _ = gpu_run(asn, spec, 1, psi0=psi0, dtype=dtype, form="banded", scale_block=block)
    ref, _ = _emulated(spec, 1, psi0, dtype, block)
    assert np.max(np.abs(state - ref)) <= 2e-6 * np.abs(ref).max()
    band = (slice(None), slice(0, 12))
    assert np.max(np.abs(state[band] - ref[band])) <= 2e-6 * np.abs(ref[band]).max()


def test_automatic_form_and_batch_equals_alone():
    # problems of different reach in one batch: the kernel takes the largest
    specs = [wl.random_problem(s, nx, ny, n_polar=np_, n_azim=32, beta=b)
             for s, nx, ny, np_, b in ((1, 40, 30, 8, 4.5), (2, 17, 5, 4, 4.5), (3, 64, 64, 16, 12.0))]
    states = [wl.random_state(10 + i, sp.q, sp.ny, sp.nx) for i, sp in enumerate(specs)]
    for dtype in ("bf16", "f16"):
        p = asn.from_spec(specs[0], dtype=dtype)
        assert asn.asn_step_form(p) == "banded"
        p.close()
        alone = []
        for sp, s0 in zip(specs, states):
            a1, _, _, _ = gpu_run(asn, sp, 4, psi0=s0, dtype=dtype, form="banded")
            a2, _, _, _ = gpu_run(asn, sp, 4, psi0=s0, dtype=dtype, form="banded")
            assert np.array_equal(a1, a2)
            alone.append(a1)
        probs = [asn.from_spec(sp, dtype=dtype, set_initial_state=False, form="banded") for sp in specs]
        try:
            for p, s0 in zip(probs, states):
                asn.asn_set_state(p, s0)
            asn.asn_step_batch(probs, 4)
            for p, ref in zip(probs, alone):
                assert np.array_equal(asn.asn_get_state(p), ref)
        finally:
            for p in probs:
                p.close()


def test_refused_without_an_instance():
    spec = wl.random_problem(1, 10, 10, n_polar=4, n_azim=16, beta=4.5)   # FP32 only
    with pytest.raises(asn.AsnError) as e:
        asn.from_spec(spec, form="banded", dtype="f16")
    assert e.value.status == asn.ASN_E_UNSUPPORTED
    p = asn.from_spec(spec, dtype="f16")    # the automatic form falls back to fused
    assert asn.asn_step_form(p) == "fused"
    p.close()


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_contraction_work_counts_whole_circulant_blocks(dtype):
    # every coupled level pair's n_az x n_az block of the 16-bit K is multiplied
    spec = wl.line_source(16, n_polar=16, sigma_as=5.0)
    p = asn.from_spec(spec, dtype=dtype, form="banded")
    work = asn.asn_contraction_work(p)
    p.close()
    om, w = asn.asn_build_quadrature(16, 32)
    K = asn.asn_build_kernel(om, w, spec.beta / 512)
    bits, _ = asn.asn_build_kernel_lowp(K, dtype)
    pairs = ((bits & 0x7FFF) != 0).reshape(16, 32, 16, 32).any(axis=(1, 3)).sum()
    assert work["tile_flops"] == 2.0 * pairs * 32 * 32 * 256
    assert work["nonzero_flops"] == 2.0 * np.count_nonzero(bits & 0x7FFF) * 256
