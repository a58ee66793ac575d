"""CPU checks of the C-ABI library: it loads, exports every declared symbol, its
host-side builder agrees with the oracle, and invalid arguments are rejected
before any device work.  No GPU compute is called here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import asn_oracle as o

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
asn = pytest.importorskip("paper_1911_08801_amd.asn", reason="libasn.so not built")


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "asn.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(asn_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = _declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(asn.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing
    assert set(names) <= set(asn.EXPORTED)


@pytest.mark.parametrize("n_polar,n_azim", [(1, 4), (2, 4), (8, 16), (16, 32), (24, 48), (32, 64),
                                            (5, 7)])
def test_host_quadrature_matches_oracle(n_polar, n_azim):
    om, w = asn.asn_build_quadrature(n_polar, n_azim)
    om_o, w_o = o.product_quadrature(n_polar, n_azim)
    assert np.max(np.abs(om - om_o)) < 1e-14
    assert np.max(np.abs(w - w_o)) < 1e-14


@pytest.mark.parametrize("norm", ["sym", "row"])
@pytest.mark.parametrize("n_polar,beta", [(2, 1.5), (8, 4.5), (16, 4.5), (24, 4.5), (4, 40.0)])
def test_host_kernel_matches_oracle(norm, n_polar, beta):
    om, w = o.product_quadrature(n_polar, 2 * n_polar)
    eps = beta / w.size
    K = asn.asn_build_kernel(om, w, eps, norm)
    K_o = o.as_kernel_matrix(om, w, eps, norm)
    # Two independent scaling loops each stop within 1e-14 of unit row sums.
    assert np.max(np.abs(K - K_o)) < 1e-13
    assert np.max(np.abs(K.sum(axis=1) - 1)) < 1e-14
    if norm == "sym":
        assert np.max(np.abs(w @ K - w) / w) < 1e-13


def test_host_kernel_on_custom_ordinates():
    rng = np.random.default_rng(3)
    om = rng.standard_normal((10, 3))
    om /= np.linalg.norm(om, axis=1)[:, None]
    w = rng.random(10) + 0.1
    for norm in ("sym", "row"):
        assert np.max(np.abs(asn.asn_build_kernel(om, w, 0.7, norm)
                             - o.as_kernel_matrix(om, w, 0.7, norm))) < 1e-14


@pytest.mark.parametrize("n,n_polar,tf,L", [(50, 8, 1.0, 3.0), (400, 16, 1.0, 3.0),
                                            (700, 24, 3.2, 7.0), (1024, 32, 1.0, 3.0),
                                            (37, 3, 0.37, 1.1)])
def test_host_time_step_matches_oracle(n, n_polar, tf, L):
    om, _ = o.product_quadrature(n_polar, 2 * n_polar)
    g = asn.make_grid(n, n + 3, 0.0, L, -1.0, -1.0 + L * (n + 3) / n)
    dt, k = asn.asn_time_step(g, om, 0.95, tf)
    dt_o, k_o = o.cfl_time_step(om, L / n, L / n, 0.95, tf)
    assert k == k_o and dt == pytest.approx(dt_o, rel=1e-15)


def test_time_step_rejects_cfl_above_one():
    om, _ = o.product_quadrature(2, 4)
    with pytest.raises(asn.AsnError) as e:
        asn.asn_time_step(asn.make_grid(4, 4, 0, 1, 0, 1), om, 1.3, 1.0)
    assert e.value.status == asn.ASN_E_UNSTABLE


@pytest.mark.parametrize("order", [2, 3, 4, 5, 9, 16])
def test_host_icosahedron_matches_oracle(order):
    om, w = asn.asn_build_icosahedron(order)
    om_o, w_o = o.icosahedron_quadrature(order)
    assert w.size == 10 * (order - 1) ** 2 + 2
    # Same ordering (decreasing z, then azimuth) and the same dual-cell areas,
    # from two separate constructions.
    assert np.max(np.abs(om - om_o)) < 1e-13
    assert np.max(np.abs(w - w_o)) < 1e-13


def test_icosahedron_workspace_and_rejects():
    opt = asn.make_options()
    g = asn.make_grid(20, 20, -1.5, 1.5, -1.5, 1.5)
    ico = asn.asn_workspace_size(g, asn.asn_quadrature(0, 0, 0, None, None, 4), opt)
    prod = asn.asn_workspace_size(g, asn.asn_quadrature(4, 23, 0, None, None, 0), opt)
    assert ico == prod                     # 92 ordinates either way
    for order in (1, 42, -3):
        with pytest.raises(asn.AsnError) as e:
            asn.asn_build_icosahedron(order) if order > 1 else asn._check(
                asn._lib.asn_build_icosahedron(order, None, None), "ico")
        assert e.value.status == asn.ASN_E_INVALID
    st, _ = _raw_create(ico=1)
    assert st == asn.ASN_E_INVALID


def test_builders_reject_bad_arguments():
    with pytest.raises(asn.AsnError) as e:
        asn.asn_build_kernel(np.zeros((0, 3)), np.zeros(0), 0.1)
    assert e.value.status == asn.ASN_E_INVALID
    om, w = o.product_quadrature(2, 4)
    with pytest.raises(asn.AsnError):
        asn.asn_build_kernel(om, w, -1.0)


def _raw_create(nx=4, ny=3, n_polar=2, n_azim=4, cfl=0.95, sig=None, beta=4.5, t_final=1.0,
                grid=None, ico=0):
    lib = asn._lib
    g = grid or asn.make_grid(nx, ny, 0.0, 1.0, 0.0, 1.0)
    q = asn.asn_quadrature(n_polar, n_azim, 0, None, None, ico)
    opt = asn.make_options(cfl=cfl)
    f = np.zeros(max(nx * ny, 1), dtype=np.float32) if sig is None else sig
    h = ctypes.c_void_p()
    st = lib.asn_create(ctypes.byref(g), ctypes.byref(q), asn._fptr(f), asn._fptr(f), asn._fptr(f),
                        None, beta, t_final, ctypes.byref(opt), None, None, 0, ctypes.byref(h))
    return st, h


def test_create_validates_before_touching_the_device():
    assert _raw_create(nx=0)[0] == asn.ASN_E_INVALID
    assert _raw_create(n_polar=0)[0] == asn.ASN_E_INVALID
    assert _raw_create(cfl=1.2)[0] == asn.ASN_E_UNSTABLE
    assert _raw_create(cfl=0.0)[0] == asn.ASN_E_INVALID
    assert _raw_create(beta=0.0)[0] == asn.ASN_E_INVALID
    assert _raw_create(t_final=-1.0)[0] == asn.ASN_E_INVALID
    bad = np.zeros(12, dtype=np.float32)
    bad[5] = -1.0
    assert _raw_create(sig=bad)[0] == asn.ASN_E_INVALID
    bad[5] = np.nan
    assert _raw_create(sig=bad)[0] == asn.ASN_E_INVALID
    assert _raw_create(grid=asn.make_grid(4, 3, 1.0, 1.0, 0.0, 1.0))[0] == asn.ASN_E_INVALID


def test_create_rejects_unknown_scheme():
    lib = asn._lib
    g = asn.make_grid(4, 3, 0.0, 1.0, 0.0, 1.0)
    q = asn.asn_quadrature(2, 4, 0, None, None, 0)
    f = np.zeros(12, dtype=np.float32)
    for scheme, want in ((7, asn.ASN_E_INVALID), (-1, asn.ASN_E_INVALID)):
        opt = asn.make_options()
        opt.scheme = scheme
        h = ctypes.c_void_p()
        st = lib.asn_create(ctypes.byref(g), ctypes.byref(q), asn._fptr(f), asn._fptr(f),
                            asn._fptr(f), None, 4.5, 1.0, ctypes.byref(opt), None, None, 0,
                            ctypes.byref(h))
        assert st == want and not h.value
    # both schemes keep two state buffers: the Heun stages need no more memory; the
    # fused FP32 Euler step keeps the contraction output in registers (no Y buffer)
    g2 = asn.make_grid(200, 120, 0.0, 1.0, 0.0, 1.0)
    q2 = asn.asn_quadrature(4, 8, 0, None, None, 0)
    e = asn.asn_workspace_size(g2, q2, asn.make_options(scheme="euler", unfused=True))
    h = asn.asn_workspace_size(g2, q2, asn.make_options(scheme="heun"))
    f = asn.asn_workspace_size(g2, q2, asn.make_options(scheme="euler"))
    plane = 32 * ((200 * 120 + 255) // 256 * 256) * 4
    assert abs(h - e) < 0.05 * e
    assert e - f > 0.95 * plane


def test_step_form_choice_by_size_and_operand_type():
    # the automatic form: FP32 forward Euler on a product set takes the banded step when
    # K has that form (known once K is built), else, like every other case: FP32 from
    # 2^25 cell-ordinates runs separate kernels (its workspace holds the contraction
    # output Y), smaller problems, 16-bit operands and grids wider than the flat stencil
    # fuse.  The automatic workspace size covers both candidates; explicit forms are
    # taken as asked.
    def ws(nx, ny, n_polar, dtype="f32", unfused=None, form=None):
        g = asn.make_grid(nx, ny, 0.0, 1.0, 0.0, 1.0)
        q = asn.asn_quadrature(n_polar, 2 * n_polar, 0, None, None, 0)
        return asn.asn_workspace_size(g, q, asn.make_options(dtype=dtype, unfused=unfused, form=form))
    for nx, ny, npol, dtype, sep in ((400, 400, 16, "f32", True), (128, 128, 16, "f32", False),
                                     (400, 400, 16, "bf16", False), (5000, 20, 16, "f32", False),
                                     (256, 256, 16, "f32", True), (255, 256, 16, "f32", False)):
        auto = ws(nx, ny, npol, dtype)
        fallback = ws(nx, ny, npol, dtype, unfused=sep)
        if dtype == "f32":
            assert auto == max(fallback, ws(nx, ny, npol, dtype, form="banded"))
        else:
            assert auto == fallback
        assert fallback != ws(nx, ny, npol, dtype, unfused=not sep)
    # the banded layout has no Y buffer and one Phi partial per cell
    plane = 512 * 400 * 400 * 4
    assert ws(400, 400, 16, form="separate") - ws(400, 400, 16, form="banded") > 0.99 * plane
    opt = asn.make_options()
    opt.step_form = 4
    g = asn.make_grid(8, 8, 0.0, 1.0, 0.0, 1.0)
    q = asn.asn_quadrature(2, 4, 0, None, None, 0)
    with pytest.raises(asn.AsnError):
        asn.asn_workspace_size(g, q, opt)


def test_scale_block_choices_checked():
    g = asn.make_grid(40, 30, 0.0, 1.0, 0.0, 1.0)
    q = asn.asn_quadrature(2, 4, 0, None, None, 0)
    for dtype in ("f32", "bf16"):
        sizes = [asn.asn_workspace_size(g, q, asn.make_options(dtype=dtype, scale_block=sb))
                 for sb in (0, 64, 128, 256, 1024, 4096)]
        assert len(set(sizes)) == 1          # block maxima are sized for the smallest block
        for sb in (-64, 1, 32, 96, 100, 8192):
            with pytest.raises(asn.AsnError):
                asn.asn_workspace_size(g, q, asn.make_options(dtype=dtype, scale_block=sb))
    assert asn.asn_options_default().scale_block == 256


def test_destroy_accepts_null_and_status_strings():
    assert asn._lib.asn_destroy(None) == asn.ASN_OK
    for s in range(-6, 1):
        assert asn._lib.asn_status_string(s)


def test_workspace_size_grows_with_problem():
    q = asn.asn_quadrature(8, 16, 0, None, None)
    opt = asn.make_options()
    a = asn.asn_workspace_size(asn.make_grid(50, 50, -1.5, 1.5, -1.5, 1.5), q, opt)
    b = asn.asn_workspace_size(asn.make_grid(100, 50, -1.5, 1.5, -1.5, 1.5), q, opt)
    assert b > a > 2 * 128 * 2500 * 4          # two state copies (fused step: no Y buffer)


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
@pytest.mark.parametrize("n_polar", [2, 8, 16])
def test_host_lowp_kernel_matches_oracle_rounding(dtype, n_polar):
    om, w = o.product_quadrature(n_polar, 2 * n_polar)
    K = o.as_kernel_matrix(om, w, 4.5 / w.size, "sym")
    bits, r = asn.asn_build_kernel_lowp(K, dtype)
    kq = o.quantise(K.astype(np.float32), dtype)
    ref = (kq.view(np.uint32) >> 16).astype(np.uint16) if dtype == "bf16" \
        else kq.astype(np.float16).view(np.uint16)
    assert np.array_equal(bits, ref)
    _, r_o = o.lowprec_kernel(K, dtype)
    assert np.allclose(r.astype(np.float64), r_o, rtol=2.5e-7, atol=1e-13)
    assert np.abs(r).max() > 0


def test_binding_shares_torchs_hip_runtime():
    # Exactly one HIP runtime may be mapped in the process (torch's), or device
    # pointers from torch would be foreign to the library.
    maps = {l.split()[-1] for l in open("/proc/self/maps") if "libamdhip64" in l}
    assert len(maps) == 1


@pytest.mark.parametrize("n_polar,beta", [(4, 4.5), (8, 4.5), (12, 4.5), (16, 4.5), (24, 4.5),
                                          (32, 4.5), (8, 2.0), (16, 9.0)])
def test_banded_form_rebuilds_the_stored_kernel(n_polar, beta):
    # The banded step applies K as per-level-pair rows of coefficients over azimuth
    # offsets; expanded back they must give fp32(K) of the oracle entry for entry.
    n_azim = 2 * n_polar
    om, w = o.product_quadrature(n_polar, n_azim)
    K = o.as_kernel_matrix(om, w, beta / w.size, "sym")
    got, reach = asn.asn_band_expand(n_polar, n_azim, K)
    assert np.array_equal(got, K.astype(np.float32))
    lv = np.arange(w.size) // n_azim
    nz = K.astype(np.float32) != 0
    assert reach == np.max(np.abs(lv[:, None] - lv[None, :])[nz])


def test_banded_form_refuses_kernels_without_it():
    # an icosahedron set has no azimuthal rotation symmetry; a row-shuffled product
    # K is no longer circulant; an odd azimuth count is refused
    om, w = o.product_quadrature(4, 8)
    K = o.as_kernel_matrix(om, w, 4.5 / 32, "sym")
    perm = np.random.default_rng(0).permutation(32)
    with pytest.raises(asn.AsnError) as e:
        asn.asn_band_expand(4, 8, K[perm][:, perm])
    assert e.value.status == asn.ASN_E_UNSUPPORTED
    om, w = o.product_quadrature(3, 7)
    K = o.as_kernel_matrix(om, w, 4.5 / 21, "sym")
    with pytest.raises(asn.AsnError) as e:
        asn.asn_band_expand(3, 7, K)
    assert e.value.status == asn.ASN_E_UNSUPPORTED
    # a wide kernel couples levels more than three apart
    om, w = o.product_quadrature(16, 32)
    K = o.as_kernel_matrix(om, w, 0.5, "sym")
    with pytest.raises(asn.AsnError) as e:
        asn.asn_band_expand(16, 32, K)
    assert e.value.status == asn.ASN_E_UNSUPPORTED


def test_banded_form_size_and_scheme_limits():
    # the banded kernels address a polar level's planes (n_azim * P floats) with 32-bit
    # byte offsets: an explicit request beyond that, for Heun or an icosahedron set, or in
    # BF16 / FP16 at an azimuth count without a reduced-precision instance, is refused;
    # the automatic form falls back to the MFMA forms without error
    q = asn.asn_quadrature(32, 64, 0, None, None, 0)
    q40 = asn.asn_quadrature(20, 40, 0, None, None, 0)
    small = asn.make_grid(1024, 1024, -1.5, 1.5, -1.5, 1.5)
    big = asn.make_grid(2900, 2900, -1.5, 1.5, -1.5, 1.5)      # 64 x P x 4 >= 2^31
    assert asn.asn_workspace_size(small, q, asn.make_options(form="banded")) > 0
    for dt in ("bf16", "f16"):
        assert asn.asn_workspace_size(small, q, asn.make_options(form="banded", dtype=dt)) > 0
    for grid, quad, opts in ((big, q, dict(form="banded")), (small, q40, dict(form="banded", dtype="bf16")),
                             (small, q40, dict(form="banded", dtype="f16")),
                             (small, q, dict(form="banded", scheme="heun"))):
        with pytest.raises(asn.AsnError) as e:
            asn.asn_workspace_size(grid, quad, asn.make_options(**opts))
        assert e.value.status == asn.ASN_E_UNSUPPORTED
    assert asn.asn_workspace_size(big, q, asn.make_options(form="auto")) > 0
    ico = asn.asn_quadrature(0, 0, 0, None, None, 3)
    with pytest.raises(asn.AsnError) as e:
        asn.asn_workspace_size(small, ico, asn.make_options(form="banded"))
    assert e.value.status == asn.ASN_E_UNSUPPORTED
