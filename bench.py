"""Benchmark of the explicit as-S_N step on one MI355X.

One "step" is one pass of the whole per-step hot path over the workload: the
ordinate contraction Y = K Psi, stream + collide, moment finalize and budget
fold.  Workload: line source on 400 x 400 cells of [-1.5, 1.5]^2 with 16 x 32 =
512 product ordinates, sigma_s = 1, sigma_as = 5, beta = 4.5, CFL 0.95 (197 steps
to t = 1), FP32 contraction.  Inputs are resident on the GPU before timing.

Prints ONE JSON line (rank 0, N = 1).
"""
from __future__ import annotations

import argparse
import math
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-ordinate updates/s per as-S_N step (FP32 vs BF16-GEMM) + p99 solve latency"
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=400)
    ap.add_argument("--n-polar", type=int, default=16)
    ap.add_argument("--sigma-as", type=float, default=5.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lowp", action="store_true", help="skip the BF16 / FP16 lines")
    ap.add_argument("--cpu-steps", type=int, default=15)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-heun", action="store_true", help="skip the Heun + minmod line")
    ap.add_argument("--no-separate", action="store_true",
                    help="skip the FP32 Euler line in the other kernel form (fused or separate) "
                         "than the one the library chooses")
    ap.add_argument("--no-implicit", action="store_true", help="skip the implicit-scheme line")
    ap.add_argument("--sweep", choices=["lattice700", "line1024"], default=None,
                    help="precision sweep to t_final on a configured workload (one JSON line)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one elementwise copy of 1 GiB (read 1 GiB, write 1 GiB) so "
                         "hardware byte counters can be scaled against known traffic")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-nmax", type=int, default=256)
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="offered load as a fraction of the measured batch capacity")
    return ap.parse_args()


def cpu_baseline(spec, steps):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload."""
    import numpy as np
    from oracle import asn_oracle as o
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    st = o.setup(spec)
    psi = spec.psi0().astype(np.float64)
    psi, _ = o.step(psi, st, want_budget=False)          # first touch outside the timing
    t0 = time.perf_counter()
    for _ in range(steps):
        psi, _ = o.step(psi, st, want_budget=False)
    dt = time.perf_counter() - t0
    ups = spec.cells * spec.q * steps / dt
    return {"value": ups, "unit": "cell-ordinate updates/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{steps} FP64 oracle steps of the same {spec.nx}x{spec.ny}, Q={spec.q} "
                      f"line-source workload ({dt:.1f} s, {platform.processor() or 'host cpu'})"}


PEAK_LP_MFMA_TFLOPS = 2500.0     # dense BF16 / FP16 MFMA


def timed_run(asn, spec, dtype, steps, warmup, scheme="euler", unfused=None):
    """Warm up, time `steps` steps as the library runs them (no timing events between
    the kernels), then run `steps` more with HIP events recorded on the problem's stream
    between the kernels for the per-kernel durations.  The event markers themselves add
    a few microseconds per kernel boundary, so the throughput comes from the first pass."""
    import torch
    p = asn.from_spec(spec, dtype=dtype, scheme=scheme, unfused=unfused)
    info = asn.asn_info(p)
    work = asn.asn_contraction_work(p)
    asn.asn_step(p, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    asn.asn_step(p, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t1 = time.perf_counter()
    kms = asn.asn_step_timed(p, steps)
    torch.cuda.synchronize()
    wall_events = time.perf_counter() - t1
    bud = asn.asn_mass_budget(p)
    p.close()
    return {"wall": wall, "wall_events": wall_events, "kms": kms, "info": info, "work": work,
            "budget": bud, "scheme": scheme}


# Stencil bytes per update per step: Euler reads psi and Y and writes psi^{n+1}; a Heun
# step is two passes, the second also reading psi^n.
STENCIL_BYTES = {"euler": 12.0, "heun": 28.0}
# widest grid whose separate stencil runs over flat 2048-cell chunks (three staged
# rounds of 2048 floats hold the chunk and its neighbour rows); column strips beyond
FLAT_MAX_NX = {"euler": 3 * 2048 - 2048 - 8, "heun": (3 * 2048 - 2048 - 8) // 3}
PASSES = {"euler": 1, "heun": 2}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_line_source_400_q512.json")
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
    if the kernels changed since it was taken or the workload is not the one measured."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_code_sha256") != kernel_source_hash() or (spec.nx, spec.q) != (400, 512):
        return None
    total = 0.0
    for name in kernel if isinstance(kernel, (list, tuple)) else [kernel]:
        k = rec["kernels"].get(name)
        if k is None:
            return None
        total += k["fetch_bytes"] + k["write_bytes"]
    return total


def contraction_roofline(res, spec, dtype):
    """MFMA roofline of the contraction kernel (fused or separate) of a run."""
    kms = res["kms"]
    scheme = res.get("scheme", "euler")
    t_gemm = kms["contraction"] * 1e-3
    fused = fused_run(res, dtype)
    flops = PASSES[scheme] * res["work"]["tile_flops"]
    peak = PEAK_FP32_MFMA_TFLOPS if dtype == "f32" else PEAK_LP_MFMA_TFLOPS
    ach = flops / t_gemm / 1e12
    if dtype == "f32":
        prof = "gemm_f32_kernel<true>" if fused else "gemm_f32_kernel<false>"
    else:
        prof = f"gemm_lp_kernel<{1 if dtype == 'bf16' else 2}, {'true' if fused else 'false'}>"
    traffic = measured_traffic(prof, spec)
    return {"bound": "mfma", "kernel": prof + (" (contraction + stream/collide)" if fused else ""),
            "achieved": ach, "peak": peak, "unit": "TFLOP/s",
            "frac": ach / peak,
            "traffic": None if traffic is None else PASSES[scheme] * traffic,
            "algorithmic": f"2*C*(K entries in the multiplied sub-blocks) = {flops:.4g} flop per "
                           f"step (dense 2*Q*Q*C = {res['work']['dense_flops']:.4g} per launch)",
            "dense_equivalent_TFLOPs": PASSES[scheme] * res["work"]["dense_flops"] / t_gemm / 1e12}


def stencil_roofline(res, spec, dtype):
    """HBM roofline of the separate stencil kernel(s) of a run (None when fused)."""
    if fused_run(res, dtype):
        return None
    C, Q = spec.cells, spec.q
    scheme = res.get("scheme", "euler")
    t_sc = res["kms"]["stream_collide"] * 1e-3
    sc_bytes = STENCIL_BYTES[scheme] * Q * C
    ach = sc_bytes / t_sc / 1e9
    lp = "false" if dtype == "f32" else "true"
    flat = "_flat" if spec.nx <= FLAT_MAX_NX[scheme] else ""
    prof = [f"stream_collide{flat}_kernel<{lp}>"] if scheme == "euler" else \
        [f"muscl{flat}_kernel<{lp}, 1>", f"muscl{flat}_kernel<{lp}, 2>"]
    return {"bound": "hbm", "kernel": " + ".join(prof), "achieved": ach,
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
            "traffic": measured_traffic(prof, spec),
            "algorithmic": f"{STENCIL_BYTES[scheme]:g}*Q*C = {sc_bytes:.4g} bytes per step"}


def roofline(res, spec, dtype):
    """Roofline entry of the kernel with the largest share of the step."""
    kms = res["kms"]
    if kms["contraction"] >= kms["stream_collide"]:
        return contraction_roofline(res, spec, dtype)
    return stencil_roofline(res, spec, dtype)


def rooflines(res, spec, dtype):
    """Both rooflines of a run: MFMA for the contraction, HBM for a separate stencil."""
    out = {"contraction": contraction_roofline(res, spec, dtype)}
    st = stencil_roofline(res, spec, dtype)
    if st is not None:
        out["stencil"] = st
    return out


def fused_run(res, dtype):
    """True when the stencil ran inside the contraction (forward Euler)."""
    kms = res["kms"]
    return res.get("scheme", "euler") == "euler" and \
        kms["stream_collide"] < 0.05 * kms["contraction"]


def summary(res, spec, steps, dtype="f32"):
    C, Q = spec.cells, spec.q
    kms = res["kms"]
    scheme = res.get("scheme", "euler")
    sc_bytes = STENCIL_BYTES[scheme] * Q * C
    fused = fused_run(res, dtype)
    return {"value": C * Q * steps / res["wall"], "ms_per_step": 1e3 * res["wall"] / steps,
            "ms_per_step_with_kernel_events": 1e3 * res["wall_events"] / steps,
            "kernels_ms": kms,
            "contraction_TFLOPs": PASSES[scheme] * res["work"]["tile_flops"]
            / (kms["contraction"] * 1e-3) / 1e12,
            "stream_collide_GBs": None if fused else sc_bytes / (kms["stream_collide"] * 1e-3) / 1e9,
            "fused_step": fused,
            "budget_max_residual": res["budget"]["max_residual"]}


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


def precision_sweep(name):
    """Full runs to t_final with FP32, BF16 and FP16 contractions on one workload;
    updates/s per form and each reduced form's scalar-flux error against FP32."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_1911_08801_amd import asn
    if name == "lattice700":
        spec = wl.checkerboard(700, n_polar=24, sigma_as=5.0)
        forms = ("f32", "bf16")
    else:
        spec = wl.line_source(1024, n_polar=32, sigma_as=5.0)
        forms = ("f32", "bf16", "f16")
    out = {"workload": spec.name, "cells": spec.cells, "ordinates": spec.q, "forms": {}}
    ref = None
    for dt in forms:
        p = asn.from_spec(spec, dtype=dt)
        n = asn.asn_info(p)["steps_to_tfinal"]
        work = asn.asn_contraction_work(p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        asn.asn_step(p, n)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        phi = asn.asn_scalar_flux(p)
        bud = asn.asn_mass_budget(p)
        p.close()
        rec = {"steps": n, "seconds": wall, "updates_per_s": spec.cells * spec.q * n / wall,
               "tile_flops_per_step": work["tile_flops"], "budget_max_residual": bud["max_residual"],
               "defect_over_mass": bud["defect"] / max(bud["mass"], bud["mass0"], 1e-300)}
        if ref is None:
            ref = phi
        else:
            rec["phi_rel_l2_vs_f32"] = float(np.linalg.norm(phi - ref) / np.linalg.norm(ref))
        out["forms"][dt] = rec
        print(f"# {name} {dt}: {rec}", file=sys.stderr, flush=True)
    return out


def main():
    args = parse()
    if args.sweep:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"sweep": precision_sweep(args.sweep)}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import workloads as wl
    from paper_1911_08801_amd import asn

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)                 # 1 GiB read + 1 GiB written
        torch.cuda.synchronize()
        del x, y
    spec = wl.line_source(args.n, n_polar=args.n_polar, sigma_as=args.sigma_as)
    C, Q = spec.cells, spec.q
    res = timed_run(asn, spec, "f32", args.steps, args.warmup)
    head = summary(res, spec, args.steps)
    out = {
        "metric": METRIC, "value": head["value"], "unit": "cell-ordinate updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"line source {args.n}x{args.n} on [-1.5,1.5]^2, "
                               f"{args.n_polar}x{2 * args.n_polar}={Q} ordinates, sigma_s=1, "
                               f"sigma_as={args.sigma_as}, beta=4.5, CFL 0.95, FP32 contraction",
                   "cells": C, "ordinates": Q, "dt": res["info"]["dt"],
                   "steps_to_tfinal": res["info"]["steps_to_tfinal"]},
        "f32": head,
        "roofline": roofline(res, spec, "f32"),
    }
    out["f32"]["rooflines"] = rooflines(res, spec, "f32")
    if not args.no_separate:
        # the same FP32 Euler step in the other kernel form than the library chose
        # (separate: Y through memory and the stencil's own HBM roofline; fused: the
        # stencil in the contraction's epilogue)
        sep = head["fused_step"]
        r = timed_run(asn, spec, "f32", args.steps, args.warmup, unfused=sep)
        key = "f32_separate" if sep else "f32_fused"
        out[key] = summary(r, spec, args.steps)
        out[key]["rooflines"] = rooflines(r, spec, "f32")
    if not args.no_lowp:
        for dt in ("bf16", "f16"):
            r = timed_run(asn, spec, dt, args.steps, args.warmup)
            out[dt] = summary(r, spec, args.steps, dt)
            out[dt]["roofline"] = roofline(r, spec, dt)
            out[dt]["rooflines"] = rooflines(r, spec, dt)
    if not args.no_heun:
        # the paper's own explicit scheme (Heun + minmod), same workload, FP32 contraction
        r = timed_run(asn, spec, "f32", args.steps, args.warmup, scheme="heun")
        out["heun_f32"] = summary(r, spec, args.steps)
        out["heun_f32"]["roofline"] = roofline(r, spec, "f32")
        out["heun_f32"]["rooflines"] = rooflines(r, spec, "f32")
    if not args.no_implicit:
        out["implicit"] = implicit_run()
    if not args.no_serving:
        out["serving"] = serving_run(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
