"""The serving scheduler on a CPU stand-in backend: admission by memory budget and
slots, continuous batching, per-request step counts, failure isolation and
cancellation.  (The GPU backend is exercised by tests/test_gpu_serve.py.)"""
import numpy as np
import pytest

import workloads as wl
from paper_1911_08801_amd.serve import Job, Server


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


class FakeHandle:
    def __init__(self, spec, steps):
        self.spec, self.total, self.steps, self.released = spec, steps, 0, False


class FakeBackend:
    def __init__(self, clock, free=10 ** 9, poison=()):
        self.clock, self.free, self.poison = clock, free, set(poison)
        self.used = self.peak = 0
        self.max_batch = 0
        self.batches_seen = []
        self.created = []
        self.kinds = {}

    def bytes_needed(self, spec, dtype, scheme="euler"):
        return spec.nx * spec.ny * spec.n_polar * spec.n_azim * 12

    def free_bytes(self):
        return self.free

    def create(self, spec, dtype, scheme="euler"):
        self.used += self.bytes_needed(spec, dtype)
        self.peak = max(self.peak, self.used)
        self.created.append((dtype, scheme))
        h = FakeHandle(spec, max(1, int(round(spec.t_final * 20))))
        self.kinds[id(h)] = (dtype, scheme, self.form(h))
        return h, h.total

    def form(self, h):
        # stands in for the library's size rule
        return "separate" if h.spec.nx * h.spec.ny >= 300 else "fused"

    def make_batch(self, handles):
        assert len({self.kinds.get(id(h)) for h in handles}) == 1
        self.max_batch = max(self.max_batch, len(handles))
        self.batches_seen.append([id(h) for h in handles])
        return list(handles)

    def step(self, batch, k, limits):
        for h, l in zip(batch, limits):
            assert not h.released
            h.steps += min(k, l)
        self.clock.t += 0.01 * k

    def wait(self):
        pass

    def finish(self, h):
        if h.spec.name in self.poison:
            raise FloatingPointError("scalar flux is not finite")
        return np.full((h.spec.ny, h.spec.nx), float(h.steps)), {"mass": 1.0}

    def drop_batch(self, b):
        pass

    def release(self, h):
        h.released = True
        self.used -= self.bytes_needed(h.spec, "f32")


def _jobs(n=20, seed=0, rate=5.0):
    reqs = wl.serving_requests(seed, n, rate=rate, n_range=(8, 24), polar_orders=(2, 4))
    jobs = []
    for r in reqs:
        spec = r.problem()
        spec.name = f"r{r.rid}"
        jobs.append(Job(rid=r.rid, spec=spec, arrival=r.arrival))
    return jobs


def test_every_request_completes_with_its_own_step_count():
    clk = Clock()
    be = FakeBackend(clk)
    rep = Server(be, hbm_budget=10 ** 9, chunk=4, clock=clk, sleep=clk.sleep).serve(_jobs())
    assert all(j.status == "done" for j in rep.jobs)
    for j in rep.jobs:
        assert j.phi[0, 0] == j.steps_total and j.latency >= 0
        assert j.t_done >= j.arrival
    s = rep.summary()
    assert s["done"] == 20 and s["p50_s"] <= s["p99_s"]


def test_memory_budget_and_slots_are_respected():
    clk = Clock()
    be = FakeBackend(clk)
    jobs = _jobs(30, seed=1, rate=50.0)
    budget = 3 * max(be.bytes_needed(j.spec, "f32") for j in jobs)
    rep = Server(be, hbm_budget=budget, max_slots=4, chunk=4, clock=clk, sleep=clk.sleep).serve(jobs)
    assert all(j.status == "done" for j in rep.jobs)
    assert be.peak <= budget and be.max_batch <= 4 and be.used == 0


def test_requests_join_while_others_run():
    clk = Clock()
    be = FakeBackend(clk)
    jobs = _jobs(12, seed=2, rate=20.0)
    Server(be, hbm_budget=10 ** 9, chunk=2, clock=clk, sleep=clk.sleep).serve(jobs)
    # some batch mixed a request admitted in an earlier round with a newer one
    assert be.max_batch >= 2
    assert len(be.batches_seen) > 2


def test_oversized_request_is_rejected_up_front_and_others_finish():
    clk = Clock()
    be = FakeBackend(clk)
    jobs = _jobs(8, seed=3)
    big = wl.line_source(200, n_polar=8)
    big.name = "big"
    jobs.append(Job(rid=99, spec=big, arrival=0.05))
    small = max(be.bytes_needed(j.spec, "f32") for j in jobs[:-1])
    rep = Server(be, hbm_budget=4 * small, chunk=4, clock=clk, sleep=clk.sleep).serve(jobs)
    st = {j.rid: j.status for j in rep.jobs}
    assert st[99] == "rejected"
    assert all(v == "done" for k, v in st.items() if k != 99)


def test_failing_request_is_isolated():
    clk = Clock()
    jobs = _jobs(10, seed=4)
    be = FakeBackend(clk, poison={"r3"})
    rep = Server(be, hbm_budget=10 ** 9, chunk=4, clock=clk, sleep=clk.sleep).serve(jobs)
    st = {j.rid: j.status for j in rep.jobs}
    assert st[3] == "failed" and sum(v == "done" for v in st.values()) == 9
    assert be.used == 0


def test_cancellation_releases_the_request():
    clk = Clock()
    be = FakeBackend(clk)
    jobs = _jobs(6, seed=5, rate=100.0)
    srv = Server(be, hbm_budget=10 ** 9, chunk=1, clock=clk, sleep=clk.sleep)
    fired = []

    def cancel_first(s):
        if not fired:
            s.cancel(jobs[0].rid)
            fired.append(1)

    rep = srv.serve(jobs, on_chunk=cancel_first)
    st = {j.rid: j.status for j in rep.jobs}
    assert st[jobs[0].rid] == "cancelled" and be.used == 0
    assert sum(v == "done" for v in st.values()) == 5


def test_batches_never_mix_kernel_forms():
    clk = Clock()
    be = FakeBackend(clk)
    jobs = _jobs(24, seed=5, rate=100.0)
    forms = {be.form(FakeHandle(j.spec, 1)) for j in jobs}
    assert forms == {"fused", "separate"}          # the stream holds both kinds
    rep = Server(be, hbm_budget=10 ** 9, chunk=4, clock=clk, sleep=clk.sleep).serve(jobs)
    assert all(j.status == "done" for j in rep.jobs)
    assert {j.form for j in rep.jobs} == {"fused", "separate"}


def test_batches_never_mix_operand_types_or_schemes():
    clk = Clock()
    be = FakeBackend(clk)
    jobs = _jobs(24, seed=3, rate=100.0)
    for k, j in enumerate(jobs):
        j.dtype = ("f32", "bf16")[k % 2]
        j.scheme = ("euler", "heun")[(k // 2) % 2]
    rep = Server(be, hbm_budget=10 ** 9, chunk=4, clock=clk, sleep=clk.sleep).serve(jobs)
    assert all(j.status == "done" for j in rep.jobs)
    assert set(be.created) == {("f32", "euler"), ("bf16", "euler"), ("f32", "heun"), ("bf16", "heun")}
