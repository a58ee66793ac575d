"""Continuous batching on the GPU: requests arriving while others run are admitted,
share fused launches, and each result equals the same request run alone."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_1911_08801_amd import asn  # noqa: E402
from paper_1911_08801_amd.serve import GpuBackend, Job, Server  # noqa: E402


def _jobs(seed, n, mixed_dtypes):
    reqs = wl.serving_requests(seed, n, rate=400.0, n_range=(24, 80), polar_orders=(2, 4, 8),
                               t_range=(0.1, 0.4))
    jobs = []
    for r in reqs:
        dt = ("bf16" if r.rid % 3 == 0 else "f32") if mixed_dtypes else "f32"
        scheme = ("heun" if r.rid % 4 == 1 else "euler") if mixed_dtypes else "euler"
        jobs.append(Job(rid=r.rid, spec=r.problem(), arrival=r.arrival, dtype=dt, scheme=scheme))
    return jobs


@pytest.mark.parametrize("mixed", [False, True])
def test_each_result_equals_the_request_alone(mixed):
    jobs = _jobs(11, 10, mixed)
    srv = Server(GpuBackend(), hbm_budget=2 * 1024 ** 3, max_slots=6, chunk=4)
    rep = srv.serve(jobs)
    s = rep.summary()
    assert s["done"] == 10 and s["p99_s"] is not None and s["aggregate_updates_per_s"] > 0
    assert rep.batch_builds >= 2                  # the batch changed as requests came and went
    for j in rep.jobs:
        p = asn.from_spec(j.spec, dtype=j.dtype, scheme=j.scheme, dt_rule="stiff",
                          form=None if j.scheme == "heun" else j.form)
        assert asn.asn_stability(p) <= 2 * j.spec.cfl * (1 + 1e-12)
        asn.asn_step(p, j.steps_total)
        alone = asn.asn_scalar_flux(p)
        p.close()
        assert np.array_equal(j.phi, alone), j.rid
        assert j.budget["steps"] == j.steps_total


def test_large_and_small_requests_share_the_fused_form():
    # asked for the fused form, requests of every size and azimuth count share one batch
    big = [wl.line_source(256, n_polar=16, sigma_as=5.0, t_final=0.02) for _ in range(2)]
    small = [wl.line_source(48, n_polar=8, sigma_as=5.0, t_final=0.05) for _ in range(3)]
    jobs = [Job(rid=k, spec=s, arrival=0.0) for k, s in enumerate(big + small)]
    rep = Server(GpuBackend(form="fused"), hbm_budget=4 * 1024 ** 3, max_slots=8,
                 chunk=4).serve(jobs)
    assert all(j.status == "done" for j in rep.jobs)
    assert [j.form for j in rep.jobs] == ["fused"] * 5
    for j in rep.jobs:
        p = asn.from_spec(j.spec, dt_rule="stiff", unfused=False)
        asn.asn_step(p, j.steps_total)
        alone = asn.asn_scalar_flux(p)
        p.close()
        assert np.array_equal(j.phi, alone), j.rid


def test_unstable_request_fails_alone_and_others_finish():
    jobs = _jobs(12, 5, False)
    # a NaN source makes one request blow up; the library rejects NaN fields, so
    # poison its initial state instead
    bad = jobs[2]
    bad.spec.psi0_cell[3, 4] = np.inf
    srv = Server(GpuBackend(), hbm_budget=2 * 1024 ** 3, max_slots=5, chunk=4)
    rep = srv.serve(jobs)
    st = {j.rid: j.status for j in rep.jobs}
    assert st[bad.rid] == "failed"
    assert sum(v == "done" for v in st.values()) == 4


def test_banded_requests_batch_by_azimuth_count():
    # the automatic form: FP32 product sets take the banded step; requests of one
    # azimuth count share a batch, and each result equals the request alone
    specs = [wl.line_source(40 + 8 * k, n_polar=(4, 8)[k % 2], sigma_as=3.0, t_final=0.1)
             for k in range(6)]
    jobs = [Job(rid=k, spec=s, arrival=0.0) for k, s in enumerate(specs)]
    rep = Server(GpuBackend(), hbm_budget=2 * 1024 ** 3, max_slots=8, chunk=4).serve(jobs)
    assert all(j.status == "done" for j in rep.jobs)
    assert {j.form for j in rep.jobs} == {"banded"}
    for j in rep.jobs:
        p = asn.from_spec(j.spec, dt_rule="stiff")
        asn.asn_step(p, j.steps_total)
        alone = asn.asn_scalar_flux(p)
        p.close()
        assert np.array_equal(j.phi, alone), j.rid
