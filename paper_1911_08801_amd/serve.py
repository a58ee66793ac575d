"""Continuous-batching server for as-S_N solves on one GPU.

Requests (a problem description plus an arrival time) are admitted while a slot
and device memory are free, keep their angular flux resident on the GPU, and
advance together: every chunk of `chunk` steps is one fused launch per kernel
per step over all active requests (asn_batch_step, captured once per batch
composition into a HIP graph).  Each request stops at its own step count; when
it finishes, its scalar flux is copied to the host, its memory is released and
waiting requests are admitted at the next chunk boundary.  Latency runs from
arrival to the scalar flux on the host.

The scheduler only talks to a backend object (GpuBackend here); tests drive
the same scheduler with a CPU stand-in to check admission and failure handling.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Any, Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Job:
    rid: int
    spec: Any
    arrival: float
    dtype: str = "f32"
    scheme: str = "euler"           # "euler" (donor cell) or "heun" (Heun + minmod)
    form: str = ""                  # kernel form the library chose ("banded" / "fused" / ...)
    status: str = "queued"          # queued, active, done, failed, rejected, cancelled
    bytes: int = 0
    steps_total: int = 0
    steps_left: int = 0
    updates: float = 0.0            # cells * ordinates * steps
    handle: Any = None
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    phi: Optional[np.ndarray] = None
    budget: Optional[dict] = None
    error: Optional[str] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.arrival


class GpuBackend:
    """The as-S_N library on the current GPU, all work on one dedicated stream.

    Requests get the stiff time-step rule by default: arbitrary requests include
    coarse, strongly absorbing problems for which the streaming CFL step alone
    is outside the explicit schemes' stability interval.

    form: kernel form of forward-Euler requests.  "auto" (default) lets the library
    choose per request (the banded step for FP32 product sets, whose batches group
    requests of one azimuth count); "fused" puts every Euler request in the fused
    GEMM form, so that all of them share one batch."""

    def __init__(self, stream=None, dt_rule: str = "stiff", form: str = "auto"):
        import torch

        from . import asn
        self.torch = torch
        self.asn = asn
        self.dt_rule = dt_rule
        self.form_asked = form
        self.stream = stream if stream is not None else torch.cuda.Stream()

    def _form(self, scheme: str):
        return self.form_asked if scheme == "euler" else None

    def bytes_needed(self, spec, dtype: str, scheme: str = "euler") -> int:
        a = self.asn
        grid = a.make_grid(spec.nx, spec.ny, spec.x_min, spec.x_max, spec.y_min, spec.y_max)
        quad = a.asn_quadrature(spec.n_polar, spec.n_azim, 0, None, None,
                                getattr(spec, "ico_order", 0))
        return a.asn_workspace_size(grid, quad, a.make_options(dtype, cfl=spec.cfl, scheme=scheme,
                                                               form=self._form(scheme)))

    def free_bytes(self) -> int:
        return int(self.torch.cuda.mem_get_info()[0])

    def create(self, spec, dtype: str, scheme: str = "euler"):
        with self.torch.cuda.stream(self.stream):
            p = self.asn.from_spec(spec, dtype=dtype, scheme=scheme, dt_rule=self.dt_rule,
                                   form=self._form(scheme))
        return p, self.asn.asn_info(p)["steps_to_tfinal"]

    def form(self, handle) -> str:
        """Kernel form the library chose for the request (batches group by it)."""
        return self.asn.asn_step_form(handle)

    def make_batch(self, handles):
        with self.torch.cuda.stream(self.stream):
            return self.asn.asn_batch_create(handles)

    def step(self, batch, n_steps: int, limits: Sequence[int]) -> None:
        self.asn.asn_batch_step(batch, n_steps, list(limits))

    def wait(self) -> None:
        self.stream.synchronize()

    def finish(self, handle):
        """(scalar flux on the host, particle budget); raises if the solve blew up."""
        phi = self.asn.asn_scalar_flux(handle)
        bud = self.asn.asn_mass_budget(handle)
        if not np.all(np.isfinite(phi)):
            raise FloatingPointError("scalar flux is not finite")
        return phi, bud

    def drop_batch(self, batch) -> None:
        batch.close()

    def release(self, handle) -> None:
        handle.close()


@dataclasses.dataclass
class Report:
    jobs: List[Job]
    makespan: float
    chunks: int
    batch_builds: int

    def done(self) -> List[Job]:
        return [j for j in self.jobs if j.status == "done"]

    def summary(self) -> Dict[str, Any]:
        done = self.done()
        lat = np.array([j.latency for j in done]) if done else np.zeros(0)
        upd = float(sum(j.updates for j in done))
        pct = (lambda q: float(np.percentile(lat, q)) if lat.size else None)
        return {"requests": len(self.jobs), "done": len(done),
                "failed": sum(j.status == "failed" for j in self.jobs),
                "rejected": sum(j.status == "rejected" for j in self.jobs),
                "p50_s": pct(50), "p99_s": pct(99), "p999_s": pct(99.9),
                "mean_s": float(lat.mean()) if lat.size else None,
                "updates": upd, "makespan_s": self.makespan,
                "aggregate_updates_per_s": upd / self.makespan if self.makespan > 0 else None,
                "chunks": self.chunks, "batch_builds": self.batch_builds}


class Server:
    """Admission by device-memory budget and slot count, continuous batching."""

    def __init__(self, backend, hbm_budget: Optional[int] = None, budget_fraction: float = 0.75,
                 max_slots: int = 64, chunk: int = 16,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.b = backend
        self.sleep = sleep
        self.max_slots = min(max_slots, 64)
        self.chunk = chunk
        self.clock = clock
        self.budget = hbm_budget if hbm_budget is not None else \
            int(budget_fraction * backend.free_bytes())
        self._cancel: set = set()

    def cancel(self, rid: int) -> None:
        """Cancel a request: dropped if queued, released at the next chunk if active."""
        self._cancel.add(rid)

    def serve(self, jobs: List[Job], on_chunk: Optional[Callable[["Server"], None]] = None
              ) -> Report:
        jobs = sorted(jobs, key=lambda j: j.arrival)
        pending = list(jobs)
        waiting: List[Job] = []
        active: List[Job] = []
        used = 0
        batches: Dict[Any, Any] = {}
        batch_members: Dict[Any, List[int]] = {}
        chunks = builds = 0
        t0 = self.clock()
        now = lambda: self.clock() - t0

        while pending or waiting or active:
            t = now()
            while pending and pending[0].arrival <= t:
                waiting.append(pending.pop(0))
            for j in list(waiting):                       # cancelled while queued
                if j.rid in self._cancel:
                    j.status = "cancelled"
                    waiting.remove(j)
            # admission, first come first served; a request that can never fit is rejected
            while waiting and len(active) < self.max_slots:
                j = waiting[0]
                if not j.bytes:
                    j.bytes = self.b.bytes_needed(j.spec, j.dtype, j.scheme)
                if j.bytes > self.budget:
                    j.status, j.error = "rejected", "larger than the whole device budget"
                    waiting.pop(0)
                    continue
                if used + j.bytes > self.budget:
                    break
                waiting.pop(0)
                try:
                    j.handle, j.steps_total = self.b.create(j.spec, j.dtype, j.scheme)
                except Exception as e:  # noqa: BLE001 - any set-up failure fails this job only
                    j.status, j.error = "failed", f"create: {e}"
                    continue
                j.form = self.b.form(j.handle)
                j.steps_left = j.steps_total
                j.updates = float(j.spec.nx * j.spec.ny * j.spec.q
                                  * j.steps_total)
                j.t_admit = now()
                j.status = "active"
                used += j.bytes
                active.append(j)
            if not active:
                if pending:
                    self.sleep(max(0.0, min(pending[0].arrival - now(), 0.05)))
                continue

            # one batch per operand type, time scheme and kernel form (banded: and azimuth
            # count); rebuilt when its members change
            groups: Dict[Any, List[Job]] = {}
            for j in active:
                az = j.spec.n_azim if j.form == "banded" else 0
                groups.setdefault((j.dtype, j.scheme, j.form, az), []).append(j)
            for dt in list(batches):
                if dt not in groups:
                    self.b.drop_batch(batches.pop(dt))
                    batch_members.pop(dt, None)
            for dt, members in groups.items():
                ids = [j.rid for j in members]
                if batch_members.get(dt) != ids:
                    if dt in batches:
                        self.b.drop_batch(batches.pop(dt))
                    batches[dt] = self.b.make_batch([j.handle for j in members])
                    batch_members[dt] = ids
                    builds += 1
                self.b.step(batches[dt], self.chunk, [j.steps_left for j in members])
            chunks += 1
            for j in active:
                j.steps_left = max(0, j.steps_left - self.chunk)
            self.b.wait()
            if on_chunk is not None:
                on_chunk(self)

            finished = [j for j in active if j.steps_left == 0 or j.rid in self._cancel]
            for j in finished:
                if j.rid in self._cancel and j.steps_left > 0:
                    j.status = "cancelled"
                else:
                    try:
                        j.phi, j.budget = self.b.finish(j.handle)
                        j.status = "done"
                    except Exception as e:  # noqa: BLE001 - isolate the failing request
                        j.status, j.error = "failed", str(e)
                j.t_done = now()
                active.remove(j)
                used -= j.bytes
            if finished:
                # drop the batches before releasing their members' memory
                for dt in list(batches):
                    self.b.drop_batch(batches.pop(dt))
                    batch_members.pop(dt, None)
                for j in finished:
                    self.b.release(j.handle)
                    j.handle = None
        for dt in list(batches):
            self.b.drop_batch(batches.pop(dt))
        return Report(jobs=jobs, makespan=now(), chunks=chunks, batch_builds=builds)


def jobs_from_requests(requests, dtype: str = "f32", scheme: str = "euler") -> List[Job]:
    """Jobs from objects with rid, arrival and problem() (a problem description)."""
    return [Job(rid=r.rid, spec=r.problem(), arrival=r.arrival, dtype=dtype, scheme=scheme)
            for r in requests]


def poisson_rate_for(load: float, capacity_updates_per_s: float, mean_updates: float) -> float:
    """Arrival rate that offers `load` times the measured capacity."""
    return load * capacity_updates_per_s / max(mean_updates, 1.0)


def percentile(xs: Sequence[float], q: float) -> float:
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else math.nan
