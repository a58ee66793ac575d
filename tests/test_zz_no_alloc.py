"""asn_step_batch_noalloc (batch tables in a static device array, no allocation)
against asn_step_batch on the same problems: bitwise equal states, scalar fluxes and
budgets, on two calls in a row, the second with a smaller input."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_1911_08801_amd import asn  # noqa: E402


def _pair(specs, form, dtype="f32"):
    """Two identical sets of problems (same inputs, seeded anisotropic states)."""
    sets = []
    for _ in range(2):
        probs = []
        for k, s in enumerate(specs):
            p = asn.from_spec(s, set_initial_state=False, form=form, dtype=dtype)
            asn.asn_set_state(p, wl.random_state(100 + k, s.q, s.ny, s.nx))
            probs.append(p)
        sets.append(probs)
    return sets


def _same(a, b):
    for p, q in zip(a, b):
        assert np.array_equal(asn.asn_get_state(p), asn.asn_get_state(q))
        assert np.array_equal(asn.asn_scalar_flux(p), asn.asn_scalar_flux(q))
        assert asn.asn_mass_budget(p) == asn.asn_mass_budget(q)
        assert asn.asn_info(p)["steps_done"] == asn.asn_info(q)["steps_done"]


@pytest.mark.parametrize("form,dtype,naz", [("fused", "f32", 16), ("banded", "f32", 16),
                                            ("fused", "bf16", 16), ("banded", "bf16", 32),
                                            ("banded", "f16", 32)])
def test_noalloc_batch_equals_allocating_batch(form, dtype, naz):
    # (the reduced-precision banded step takes 32, 48 or 64 azimuths; its problems here
    # differ in reach, so the batch runs the largest)
    big = [wl.random_problem(1, 70, 45, n_polar=4, n_azim=naz, beta=4.5),
           wl.random_problem(2, 33, 90, n_polar=8, n_azim=naz, beta=4.5),
           wl.random_problem(3, 128, 64, n_polar=6, n_azim=naz, beta=12.0 if naz == 32 else 4.5)]
    small = [wl.random_problem(4, 9, 7, n_polar=2, n_azim=naz, beta=4.5)]
    ref, got = _pair(big, form, dtype)
    asn.asn_step_batch(ref, 5)
    asn.asn_step_batch_noalloc(got, 5)
    _same(ref, got)
    # a second call in a row with a smaller input: one small problem, fewer steps
    ref2, got2 = _pair(small, form, dtype)
    asn.asn_step_batch(ref2, 3)
    asn.asn_step_batch_noalloc(got2, 3)
    _same(ref2, got2)
    # and the first set again, continuing from where it stopped
    asn.asn_step_batch(ref, 2)
    asn.asn_step_batch_noalloc(got, 2)
    _same(ref, got)
    for p in ref + got + ref2 + got2:
        p.close()


def test_noalloc_batch_rejects_what_a_batch_rejects():
    s = wl.random_problem(5, 20, 10, n_polar=2, n_azim=4, beta=4.5)
    p1 = asn.from_spec(s, dtype="f32")
    p2 = asn.from_spec(s, dtype="bf16")
    try:
        with pytest.raises(asn.AsnError):
            asn.asn_step_batch_noalloc([p1, p2], 1)
        with pytest.raises(asn.AsnError):
            asn.asn_step_batch_noalloc([p1, p1], 1)
        with pytest.raises(asn.AsnError):
            asn.asn_step_batch_noalloc([p1], -1)
    finally:
        p1.close()
        p2.close()
