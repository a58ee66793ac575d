"""Benchmark of the explicit as-S_N step on one MI355X.

One "step" is one pass of the whole per-step hot path over the workload: the
ordinate contraction Y = K Psi, stream + collide, moment finalize and budget
fold (for FP32 product sets one banded kernel does the contraction and the
stencil).  Headline workload: the line source on 1024 x 1024 cells of
[-1.5, 1.5]^2 with 32 x 64 = 2048 product ordinates, sigma_s = 1, sigma_as = 5,
beta = 4.5, CFL 0.95 (507 steps to t = 1), FP32; the same step with the BF16 and
FP16 contraction, the 400 x 400 x 512 line source, the Heun + minmod and implicit
schemes, the serving stream and the FP64 oracle are reported beside it.  Inputs
are resident on the GPU before timing.

Prints ONE JSON line (rank 0, N = 1).
"""
from __future__ import annotations

import argparse
import math
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-ordinate updates/s per as-S_N step (FP32 vs BF16-GEMM) + p99 solve latency"
PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP32_VALU_TFLOPS = 78.6     # FMA on 16 lanes per SIMD, no packed FP32 (not used here)
PEAK_LP_MFMA_TFLOPS = 2500.0     # dense BF16 / FP16 MFMA
BYTES_PER_UPDATE = 8.0           # read psi^n and write psi^{n+1} once, FP32
BAND_WIDE_ROW_CELLS = 1024       # rows from this width on take the banded kernel's wide-row instance


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=5,
                    help="the timed steps are split into this many chunks (eager), and a "
                         "graph of one chunk is replayed as often; medians are reported")
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--n-polar", type=int, default=32)
    ap.add_argument("--sigma-as", type=float, default=5.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lowp", action="store_true", help="skip the BF16 / FP16 lines")
    ap.add_argument("--no-separate", action="store_true",
                    help="skip the headline workload with separate FP32 kernels")
    ap.add_argument("--cpu-rows", type=int, default=64,
                    help="rows of the headline grid (through the pulse) the oracle steps")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 400 x 400 x 512 line (all FP32 forms, precision vs oracle)")
    ap.add_argument("--no-heun", action="store_true", help="skip the Heun + minmod line")
    ap.add_argument("--no-implicit", action="store_true", help="skip the implicit-scheme line")
    ap.add_argument("--sweep", choices=["lattice700", "line1024", "line400"], default=None,
                    help="precision sweep to t_final on a configured workload (one JSON line)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one elementwise copy of 1 GiB (read 1 GiB, write 1 GiB) so "
                         "hardware byte counters can be scaled against known traffic")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-nmax", type=int, default=512)
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="offered load as a fraction of the measured batch capacity")
    return ap.parse_args()


def oracle_slab(spec, rows):
    """`rows` rows of the workload's grid through its centre (same dx, dy, dt, fields)."""
    import dataclasses
    r0 = max(0, spec.ny // 2 - rows // 2)
    dy = (spec.y_max - spec.y_min) / spec.ny
    cut = lambda a: a[r0:r0 + rows].copy()
    return dataclasses.replace(spec, name=f"{spec.name}_rows{r0}-{r0 + rows}", ny=rows,
                               y_min=spec.y_min + r0 * dy, y_max=spec.y_min + (r0 + rows) * dy,
                               sigma_s=cut(spec.sigma_s), sigma_a=cut(spec.sigma_a),
                               sigma_as=cut(spec.sigma_as), source=cut(spec.source),
                               psi0_cell=cut(spec.psi0_cell))


def cpu_baseline(spec, rows, steps):
    """The FP64 oracle, as it stands, on a bounded sample of the workload: `rows` full
    rows of its grid (same spacing, ordinates, K and dt), `steps` steps after one untimed."""
    import numpy as np
    from oracle import asn_oracle as o
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    slab = oracle_slab(spec, rows)
    st = o.setup(slab)
    psi = slab.psi0().astype(np.float64)
    psi, _ = o.step(psi, st, want_budget=False)          # first touch outside the timing
    t0 = time.perf_counter()
    for _ in range(steps):
        psi, _ = o.step(psi, st, want_budget=False)
    dt = time.perf_counter() - t0
    ups = slab.cells * slab.q * steps / dt
    return {"value": ups, "unit": "cell-ordinate updates/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{steps} FP64 oracle steps on {rows} rows ({slab.nx}x{rows} cells, "
                      f"Q={slab.q}, dt={st.dt:.6g}) of the {spec.nx}x{spec.ny} line-source "
                      f"workload ({dt:.1f} s, {platform.processor() or 'host cpu'})"}


def measure(asn, spec, dtype, steps, warmup, reps, scheme="euler", form=None, graph=True):
    """Time `steps` steps as the library runs them, bracketed by synchronisations; the
    steps go in `reps` chunks with events between them on the problem's stream (median
    chunk rate).  Then a HIP graph of one chunk (a batch of this one problem) is
    replayed `reps` times (median rate), and one more pass records events between the
    kernels of each step (per-kernel durations; the markers add a few us per kernel
    boundary, so the throughput is not taken from that pass).  Runs on a side stream,
    which the library captures into graphs."""
    import torch
    side = torch.cuda.Stream()
    cq = spec.cells * spec.q
    with torch.cuda.stream(side):
        p = asn.from_spec(spec, dtype=dtype, scheme=scheme, form=form)
        info = asn.asn_info(p)
        work = asn.asn_contraction_work(p)
        step_form = asn.asn_step_form(p)
        asn.asn_step(p, warmup)
        chunk = max(1, steps // reps)
        sizes = [chunk] * (reps - 1) + [steps - chunk * (reps - 1)]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r, n in enumerate(sizes):
            ev[r].record(side)
            asn.asn_step(p, n)
        ev[reps].record(side)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        eager = [cq * n / (ev[r].elapsed_time(ev[r + 1]) * 1e-3) for r, n in enumerate(sizes)]
        graph_rates = []
        if graph and scheme == "euler" and chunk >= 2:
            b = asn.asn_batch_create([p])
            asn.asn_batch_step(b, chunk)                # capture + first replay
            torch.cuda.synchronize()
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(side)
                asn.asn_batch_step(b, chunk)
                e1.record(side)
                torch.cuda.synchronize()
                graph_rates.append(cq * chunk / (e0.elapsed_time(e1) * 1e-3))
            b.close()
        kms = asn.asn_step_timed(p, chunk)
        torch.cuda.synchronize()
        bud = asn.asn_mass_budget(p)
        p.close()
    torch.cuda.synchronize()
    return {"wall": wall, "kms": kms, "info": info, "work": work, "budget": bud,
            "scheme": scheme, "form": step_form, "eager_chunk_rates": eager,
            "graph_chunk_rates": graph_rates, "chunk": chunk, "steps": steps}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_line_source_1024_q2048.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1911_08801_amd", "csrc", "asn_kernels.hip")


def kernel_source_hash(path=KERNEL_SOURCE):
    """sha256 of the kernel source with its comments and blank space removed, so that a
    change of comments alone keeps a traffic record valid and any code change voids it."""
    import hashlib
    import re
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = " ".join(src.split())
    return hashlib.sha256(src.encode()).hexdigest()


def measured_traffic(kernel, spec):
    """HBM bytes per dispatch (read + write) from the committed counter summary, or None
    if the kernels changed since it was taken or the workload is not the one measured.
    A name ending in ", R>" stands for the instance of any reach R."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_code_sha256") != kernel_source_hash() or \
            [spec.nx, spec.ny, spec.q] != rec.get("workload_nx_ny_q"):
        return None
    k = rec["kernels"].get(kernel)
    if k is None and kernel.endswith(", R>"):
        k = next((v for n, v in rec["kernels"].items() if n.startswith(kernel[:-2])), None)
    return None if k is None else k["fetch_bytes"] + k["write_bytes"]


# the dominant kernel of each kernel form (its event slot in asn_step_timed)
def dominant_kernel(res, spec, dtype):
    form = res["form"]
    lp = {"f32": 0, "bf16": 1, "f16": 2}[dtype]
    if form == "banded" and lp:   # instantiated per reach of K
        return f"banded_lp_kernel<{spec.n_azim}, {lp}, R>", "contraction"
    if form == "banded":
        wide = "true" if spec.nx >= BAND_WIDE_ROW_CELLS else "false"
        return f"banded_euler_kernel<{spec.n_azim}, {wide}>", "contraction"
    if form == "fused":
        name = "gemm_f32_kernel<true>" if lp == 0 else f"gemm_lp_kernel<{lp}, true>"
        return name, "contraction"
    kms = res["kms"]
    if kms["contraction"] >= kms["stream_collide"]:
        return ("gemm_f32_kernel<false>" if lp == 0 else f"gemm_lp_kernel<{lp}, false>"), "contraction"
    return ("stream_collide_flat_kernel<false>" if lp == 0 else
            "stream_collide_flat_kernel<true>"), "stream_collide"


def roofline(res, spec, dtype):
    """Roofline of the step's dominant kernel on the method's own work.  Bytes: each
    update reads psi^n and writes psi^{n+1} once (8 B in FP32) -- the binding roof, since
    the contraction's own arithmetic, 2 nnz(K) flop per cell over the stored nonzeros,
    stays below the compute ridge.  Separate-kernel forms move Y through memory as well
    (their contraction and stencil each reported against the same 8 B/update)."""
    name, slot = dominant_kernel(res, spec, dtype)
    t = res["kms"][slot] * 1e-3
    cq = spec.cells * spec.q
    bytes_ = BYTES_PER_UPDATE * cq
    ach = bytes_ / t / 1e9
    nz = res["work"]["nonzero_flops"]
    executed = res["work"]["tile_flops"]
    compute_peak = (PEAK_FP32_VALU_TFLOPS if res["form"] == "banded" and dtype == "f32" else
                    PEAK_FP32_MFMA_TFLOPS if dtype == "f32" else PEAK_LP_MFMA_TFLOPS)
    traffic = measured_traffic(name, spec)
    return {"bound": "hbm", "kernel": name, "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": traffic,
            "algorithmic": f"{BYTES_PER_UPDATE:g} B x Q x C = {bytes_:.4g} B per step "
                           f"(Q={spec.q}, C={spec.cells}); kernel {t * 1e3:.4g} ms (HIP events, "
                           f"mean of {res['chunk']} steps)",
            "kernel_ms": t * 1e3,
            "method_flops": nz,
            "method_TFLOPs": nz / t / 1e12,
            "compute_peak_TFLOPs": compute_peak,
            "method_compute_frac": nz / t / 1e12 / compute_peak,
            "intensity_flop_per_byte": nz / bytes_,
            "ridge_flop_per_byte": compute_peak * 1e12 / (PEAK_HBM_GBS * 1e9),
            "executed_over_nonzero": executed / nz,
            "dense_equivalent_TFLOPs": res["work"]["dense_flops"] / t / 1e12,
            "traffic_over_algorithmic": None if traffic is None else traffic / bytes_,
            "kernels": per_kernel_rooflines(res, spec, dtype)}


def per_kernel_rooflines(res, spec, dtype):
    """Each kernel of the step against its own roof: a separate stencil against HBM on
    its algorithmic bytes (psi^n and Y read, psi^{n+1} written: 12 B per update in FP32),
    a contraction against its MFMA peak on the products it executes (the multiplied
    blocks) and on the nonzeros of K."""
    kms = res["kms"]
    cq = spec.cells * spec.q
    out = {}
    if res["form"] == "separate" and kms.get("stream_collide", 0) > 0:
        t = kms["stream_collide"] * 1e-3
        out["stream_collide"] = {"bound": "hbm", "algorithmic_bytes": 12.0 * cq,
                                 "achieved_GBs": 12.0 * cq / t / 1e9,
                                 "frac": 12.0 * cq / t / 1e9 / PEAK_HBM_GBS}
    if res["form"] in ("separate", "fused") and kms.get("contraction", 0) > 0:
        t = kms["contraction"] * 1e-3
        peak = PEAK_FP32_MFMA_TFLOPS if dtype == "f32" else PEAK_LP_MFMA_TFLOPS
        ex = res["work"]["tile_flops"] / t / 1e12
        nz = res["work"]["nonzero_flops"] / t / 1e12
        out["contraction"] = {"bound": "mfma", "peak_TFLOPs": peak,
                              "executed_TFLOPs": ex, "executed_frac": ex / peak,
                              "nonzero_TFLOPs": nz, "nonzero_frac": nz / peak}
    return out


def summary(res, spec, dtype="f32"):
    cq = spec.cells * spec.q
    steps = res["steps"]
    out = {"value": cq * steps / res["wall"], "ms_per_step": 1e3 * res["wall"] / steps,
           "form": res["form"], "dtype": dtype,
           "eager_chunk_median_updates_per_s": statistics.median(res["eager_chunk_rates"]),
           "eager_chunk_rates": res["eager_chunk_rates"],
           "chunk_steps": res["chunk"],
           "kernels_ms": res["kms"],
           "budget_max_residual": res["budget"]["max_residual"]}
    if res["graph_chunk_rates"]:
        out["graph_chunk_median_updates_per_s"] = statistics.median(res["graph_chunk_rates"])
        out["graph_chunk_rates"] = res["graph_chunk_rates"]
    return out


def serving_run(args):
    """Seeded Poisson request stream through the continuous-batching server.

    Requests: line source or lattice (p = 1/2), N x N cells with N uniform in
    [64, serve_nmax], polar order in {8, 12, 16, 24} (2x azimuths), sigma_as in
    [0, 5], t_final in [0.5, 3.2]; FP32 contraction.  The arrival rate offers
    `serve_load` times the throughput the same server reaches when all requests
    are queued at once (measured first, on the first 16 requests).
    """
    import numpy as np

    import workloads as wl
    from paper_1911_08801_amd import asn
    from paper_1911_08801_amd.serve import GpuBackend, Job, Server

    def updates(r):
        spec = r.problem()
        om, _ = asn.asn_build_quadrature(spec.n_polar, spec.n_azim)
        g = asn.make_grid(spec.nx, spec.ny, spec.x_min, spec.x_max, spec.y_min, spec.y_max)
        _, n = asn.asn_time_step(g, om, spec.cfl, spec.t_final)
        return spec.cells * spec.q * n

    base = wl.serving_requests(0, args.serve_requests, rate=0.0, n_range=(64, args.serve_nmax))
    mean_upd = float(np.mean([updates(r) for r in base]))
    backend = GpuBackend()
    # capacity: a burst of 16 requests all present at t = 0
    burst = [Job(rid=r.rid, spec=r.problem(), arrival=0.0) for r in base[:16]]
    cap = Server(backend, chunk=16).serve(burst).summary()["aggregate_updates_per_s"]
    rate = args.serve_load * cap / mean_upd
    reqs = wl.serving_requests(0, args.serve_requests, rate=rate, n_range=(64, args.serve_nmax))
    last = [time.perf_counter()]

    def progress(srv):            # a line every 20 s so long runs show they are alive
        if time.perf_counter() - last[0] > 20.0:
            last[0] = time.perf_counter()
            print(f"# serving: chunk done at {time.strftime('%H:%M:%S')}", file=sys.stderr,
                  flush=True)
    rep = Server(backend, chunk=16).serve([Job(rid=r.rid, spec=r.problem(), arrival=r.arrival)
                                           for r in reqs], on_chunk=progress)
    out = rep.summary()
    out.update({"arrival_rate_per_s": rate, "burst_capacity_updates_per_s": cap,
                "mean_updates_per_request": mean_upd,
                "workload": f"{args.serve_requests} seeded requests (seed 0), N in [64, "
                            f"{args.serve_nmax}], Q in {{128, 288, 512, 1152}}, FP32, Poisson "
                            f"arrivals at {args.serve_load} x measured capacity"})
    return out


def implicit_run(steps=3):
    """The paper's implicit line-source configuration: 200 x 200 cells, the 92-ordinate
    icosahedron set (S4), sigma_as = 7, beta = 4, dt = 2 dx, FP64 sweeps + GMRES with
    the paper's tolerances (1.5e-8 GMRES, 1e-4 source iteration)."""
    import torch

    import workloads as wl
    from paper_1911_08801_amd import asn
    spec = wl.line_source(200, sigma_as=7.0, beta=4.0)
    spec.ico_order = 4
    n_tot = int(math.ceil(1.0 / (2 * 3.0 / 200)))
    dt = 1.0 / n_tot
    p = asn.from_spec(spec, scheme="implicit", dt_override=dt)
    asn.asn_step(p, 1)                      # warm-up step
    torch.cuda.synchronize()
    c0 = asn.asn_iteration_counts(p)
    t0 = time.perf_counter()
    asn.asn_step(p, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    c1 = asn.asn_iteration_counts(p)
    p.close()
    sweeps = (c1["sweeps"] - c0["sweeps"]) / steps
    mv = (c1["matvecs"] - c0["matvecs"]) / steps
    return {"workload": f"line source 200x200, icosahedron S4 (92 ordinates), sigma_as=7, beta=4, "
                        f"dt=2dx ({n_tot} steps to t=1), FP64",
            "ms_per_step": 1e3 * wall / steps, "sweeps_per_step": sweeps,
            "gmres_matvecs_per_step": mv,
            "cell_ordinate_sweeps_per_s": spec.cells * spec.q * sweeps * steps / wall,
            "steps_timed": steps}


GOLDEN_400 = os.path.join(ROOT, "tests", "golden", "line_source_400_q512_phi.npz")


def precision_sweep(name):
    """Full runs to t_final with FP32, BF16 and FP16 contractions on one workload:
    updates/s per form and each result's scalar-flux error against the FP32 run and,
    for the 400 x 400 line source, against the FP64 oracle's stored flux."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_1911_08801_amd import asn
    oracle_phi = None
    if name == "lattice700":
        spec = wl.checkerboard(700, n_polar=24, sigma_as=5.0)
    elif name == "line400":
        spec = wl.line_source(400, n_polar=16, sigma_as=5.0)
        oracle_phi = np.load(GOLDEN_400)["phi_as5"].astype(np.float64)
    else:
        spec = wl.line_source(1024, n_polar=32, sigma_as=5.0)
    forms = ("f32", "bf16", "f16")
    out = {"workload": spec.name, "cells": spec.cells, "ordinates": spec.q, "forms": {}}
    ref = None
    for dt in forms:
        p = asn.from_spec(spec, dtype=dt)
        n = asn.asn_info(p)["steps_to_tfinal"]
        form = asn.asn_step_form(p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        asn.asn_step(p, n)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        phi = asn.asn_scalar_flux(p)
        bud = asn.asn_mass_budget(p)
        p.close()
        rec = {"form": form, "steps": n, "seconds": wall,
               "updates_per_s": spec.cells * spec.q * n / wall,
               "budget_max_residual": bud["max_residual"],
               "defect_over_mass": bud["defect"] / max(bud["mass"], bud["mass0"], 1e-300)}
        if ref is None:
            ref = phi
        else:
            rec["phi_rel_l2_vs_f32"] = float(np.linalg.norm(phi - ref) / np.linalg.norm(ref))
        if oracle_phi is not None:
            rec["phi_rel_l2_vs_fp64_oracle"] = float(np.linalg.norm(phi - oracle_phi) /
                                                     np.linalg.norm(oracle_phi))
        out["forms"][dt] = rec
        print(f"# {name} {dt}: {rec}", file=sys.stderr, flush=True)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only (no collectives, no "
                                   "multi-GPU path); run with --gpus 1"}), flush=True)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.sweep:
        print(json.dumps({"sweep": precision_sweep(args.sweep)}), flush=True)
        return

    import workloads as wl
    from paper_1911_08801_amd import asn

    def log(msg):
        print(f"# {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)

    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)                 # 1 GiB read + 1 GiB written
        torch.cuda.synchronize()
        del x, y
    spec = wl.line_source(args.n, n_polar=args.n_polar, sigma_as=args.sigma_as)
    C, Q = spec.cells, spec.q
    log(f"headline: {args.n}^2 x {Q}, FP32, {args.steps} steps")
    res = measure(asn, spec, "f32", args.steps, args.warmup, args.reps)
    head = summary(res, spec)
    out = {
        "metric": METRIC, "value": head["value"], "unit": "cell-ordinate updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"line source {args.n}x{args.n} on [-1.5,1.5]^2, "
                               f"{args.n_polar}x{2 * args.n_polar}={Q} ordinates, sigma_s=1, "
                               f"sigma_as={args.sigma_as}, beta=4.5, CFL 0.95, FP32",
                   "cells": C, "ordinates": Q, "dt": res["info"]["dt"],
                   "steps_to_tfinal": res["info"]["steps_to_tfinal"],
                   "kernel_form": head["form"]},
        "f32": head,
        "roofline": roofline(res, spec, "f32"),
    }
    if not args.no_lowp:
        for dt in ("bf16", "f16"):
            log(f"headline workload, {dt}")
            r = measure(asn, spec, dt, args.steps, args.warmup, args.reps)
            out[dt] = summary(r, spec, dt)
            out[dt]["roofline"] = roofline(r, spec, dt)
    if not args.no_separate:
        # the same workload with the FP32 contraction and the stencil as separate kernels:
        # the stencil against HBM and the contraction against MFMA at this size
        log("headline workload, FP32 separate kernels")
        r = measure(asn, spec, "f32", args.steps, args.warmup, args.reps, form="separate")
        out["f32_separate"] = summary(r, spec)
        out["f32_separate"]["roofline"] = roofline(r, spec, "f32")
    if not args.no_small:
        # the 400 x 400 x 512 line source: every FP32 kernel form, and each precision's
        # full run to t = 1 against the FP64 oracle's stored flux
        small = wl.line_source(400, n_polar=16, sigma_as=5.0)
        out["line400"] = {}
        for form in ("auto", "separate", "fused"):
            log(f"400^2 x 512, FP32 {form}")
            r = measure(asn, small, "f32", 40, args.warmup, args.reps, form=form)
            out["line400"][r["form"]] = summary(r, small)
            out["line400"][r["form"]]["roofline"] = roofline(r, small, "f32")
        log("400^2 x 512 precision vs oracle")
        out["line400"]["precision_vs_oracle"] = precision_sweep("line400")["forms"]
    if not args.no_heun:
        # the paper's own explicit scheme (Heun + minmod), 400 x 400 x 512
        small = wl.line_source(400, n_polar=16, sigma_as=5.0)
        log("Heun + minmod 400^2 x 512")
        r = measure(asn, small, "f32", 20, args.warmup, args.reps, scheme="heun", graph=False)
        out["heun_f32_line400"] = summary(r, small)
    if not args.no_implicit:
        log("implicit")
        out["implicit"] = implicit_run()
    if not args.no_serving:
        log(f"serving {args.serve_requests} requests")
        out["serving"] = serving_run(args)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_rows, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
