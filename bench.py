"""Benchmark: periodic FFT stencil solve (StencilFFT-P) on one MI355X.

Workload: 2-D periodic 5-point Jacobi stencil (centre and four neighbours 0.2)
on an 8192 x 8192 grid, T = 4096 steps, initial grid U[0,1) from seed 2.  One
step = one whole solve (all passes: R2C rows, column sub-transforms, the fused
symbol-power middle pass, inverse columns, C2R rows) over the grid resident in
HBM, in place.  The FP32 path is the headline (FP32 FFT passes with the FP64
symbol power); the FP64 path is timed in the same run and reported beside it.

Metric: effective cell-updates/s = N * T / time.  Also reported: per-step
latency p50 / p99, the HBM roofline of the dominant kernel from HIP events on
the launch stream, and the FP64 loop oracle timed on the host cores on a
bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2105_06676_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, launches_per_step: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        if d.get("source_hash") != kernel_source_hash():
            return None
        k = d.get("kernels", {}).get(kernel)
        return None if k is None else float(k["bytes_per_launch"])
    except Exception:
        return None


def time_path(sfft, torch, w, dtype: str, steps: int, warmup: int):
    """Three passes of `steps` solves each, after `warmup` untimed ones:
    (1) the timed region: back-to-back solves bracketed by synchronisations (wall
        clock and one event pair) -> throughput; no instrumentation inside;
    (2) per-solve event pairs -> latency percentiles;
    (3) the library's per-kernel HIP events on the launch stream -> per-kernel
        durations for the roofline (events between kernels add gaps, so this
        pass is not the one timed for throughput)."""
    td = torch.float32 if dtype == "f32" else torch.float64
    grid = torch.from_numpy(w.grid()).to(device="cuda:0", dtype=td)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        sfft.periodic(grid, w.coeffs, w.T)
    # (1) timed region
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record(stream)
    for _ in range(steps):
        sfft.periodic(grid, w.coeffs, w.T)
    b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = a.elapsed_time(b)
    # (2) latency
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for i in range(steps):
        ev[i][0].record(stream)
        sfft.periodic(grid, w.coeffs, w.T)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    lat = np.array([x.elapsed_time(y) for x, y in ev])
    # (3) per-kernel durations
    sfft.profile_start()
    for _ in range(steps):
        sfft.periodic(grid, w.coeffs, w.T)
    torch.cuda.synchronize()
    prof = sfft.profile_read()
    sfft.profile_stop()
    ok = bool(torch.isfinite(grid).all().item())
    del grid
    torch.cuda.empty_cache()
    return wall, gpu_ms, lat, prof["kernels"], ok


def serving_run(sfft, torch, reqs, rate=None, window=None, chunk=128, seed=5):
    """Drive the continuous-batching server with the request list.  rate=None:
    closed loop (keep `window` requests outstanding); else open-loop Poisson
    arrivals at `rate` requests/s (the list's arrival times rescaled).  Grids are
    filled on the device from seeded torch generators, a chunk ahead of use."""
    import time as _t
    srv = sfft.Server(0, 32 << 30, 64)
    gen = torch.Generator(device="cuda")
    ready = []
    nxt = 0

    def refill():
        nonlocal nxt
        out = []
        for r in reqs[nxt:nxt + chunk]:
            gen.manual_seed(seed * 1000003 + r.rid)
            td = torch.float32 if r.dtype == "f32" else torch.float64
            out.append((r, torch.rand(r.dims, generator=gen, device="cuda", dtype=td)))
        nxt += len(out)
        torch.cuda.synchronize()
        ready.extend(out)

    scale = None
    if rate is not None:
        scale = (len(reqs) / rate) / max(reqs[-1].arrival_s, 1e-9)
    pending = {}
    lat, cells_T, failed = [], 0.0, 0
    t0 = _t.perf_counter()
    i = 0
    while i < len(reqs) or pending:
        now = _t.perf_counter() - t0
        while i < len(reqs):
            if rate is not None and reqs[i].arrival_s * scale > now:
                break
            if rate is None and len(pending) >= window:
                break
            if not ready:
                refill()
            r, g = ready.pop(0)
            i += 1
            try:
                t = srv.submit(g, r.coeffs, r.T)
            except sfft.SfftError:
                failed += 1
                continue
            pending[t] = (r, g)
        for t in list(pending):
            try:
                done = srv.poll(t)
            except sfft.SfftError:
                failed += 1
                del pending[t]
                continue
            if done:
                a, b = srv.times(t)
                lat.append(b - a)
                cells_T += float(pending[t][0].cells) * pending[t][0].T
                del pending[t]
        _t.sleep(20e-6)
    wall = _t.perf_counter() - t0
    st = srv.stats()
    srv.close()
    lat = np.array(lat) * 1e3
    return {"requests": len(reqs), "completed": len(lat), "failed": failed, "wall_s": wall,
            "req_per_s": len(lat) / wall,
            "cell_updates_per_s": cells_T / wall, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "batches": st["batches"], "max_batch": st["max_batch"],
            "peak_workspace_bytes": st["peak_bytes"]}


def serving_bench(sfft, torch, count):
    import workloads as wl
    reqs = wl.serving_mix(count)
    # warm the plan cache with a short closed-loop pass over every distinct shape
    closed = serving_run(sfft, torch, reqs, rate=None, window=256)
    mu = closed["req_per_s"]
    openl = serving_run(sfft, torch, reqs, rate=0.7 * mu)
    return {"workload": f"Poisson stream of {count} periodic requests: d ~ U{{1,2,3}}, cells log-uniform "
                        "2^10..2^24 (7-smooth extents), r ~ U{1,2}, T log-uniform 1..1e5, FP32/FP64 50/50",
            "closed_loop": closed, "open_loop_rate_req_s": 0.7 * mu, "open_loop": openl}


def time_solve(sfft, torch, w, dtype, reps=5, warmup=1):
    """Median device time of one solve of workload w (inputs resident in HBM)."""
    td = torch.float32 if dtype == "f32" else torch.float64
    grid0 = torch.from_numpy(w.grid()).to(device="cuda:0", dtype=td)
    grid = grid0.clone()
    if w.implicit_q is not None:
        def fn(g, c, T):
            return sfft.periodic_implicit(g, w.implicit_q, c, T)
    else:
        fn = sfft.aperiodic if w.aperiodic else (sfft.periodic_fields if w.fields > 1 else sfft.periodic)
    for _ in range(warmup):
        fn(grid, w.coeffs, w.T)
    ts = []
    for _ in range(reps):
        grid.copy_(grid0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn(grid, w.coeffs, w.T)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ms = float(np.median(ts))
    cells = int(np.prod(w.dims))
    del grid, grid0
    torch.cuda.empty_cache()
    return {"ms": ms, "cell_updates_per_s": cells * w.T / (ms * 1e-3)}


def other_workloads(sfft, torch, only=None):
    """The other workloads of the method, timed the same way (context for the headline);
    `only`: a set of "<workload>_<dtype>" keys to restrict the list to."""
    import workloads as wl
    out = {}
    for name, dts in (("heat1d_65536", ("f64",)), ("star3d_512", ("f32",)),
                      ("box2d_aperiodic_4096", ("f64", "f32")), ("upwind2d_aperiodic_4096", ("f64", "f32")),
                      ("wave2d_leapfrog_4096", ("f32", "f64")),
                      ("heat2d_backward_euler_4096", ("f32", "f64")), ("jacobi2d_6300x6720_smooth", ("f32",)),
                      ("jacobi2d_8191_prime", ("f32",))):
        w = wl.config(name)
        for dt in dts:
            if only is not None and f"{name}_{dt}" not in only:
                continue
            out[f"{name}_{dt}"] = dict(time_solve(sfft, torch, w, dt), dims=list(w.dims), T=w.T,
                                       aperiodic=w.aperiodic, fields=w.fields, implicit=w.implicit_q is not None)
    return out


def copy_reference(torch, nbytes: int, reps: int = 10):
    """Device-to-device copy bandwidth (read + write bytes / time) of a plain
    elementwise copy of `nbytes`, the practical HBM ceiling the passes are
    compared with."""
    n = nbytes // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes": 2 * nbytes, "avg_us": ms * 1e3, "GBps": 2 * nbytes / (ms * 1e-3) / 1e9}


def cpu_baseline(w, budget_s: float = 12.0):
    """The FP64 loop oracle on the full-size grid for a bounded number of steps."""
    import oracle
    a0 = w.grid()
    nthr = oracle.threads()
    t0 = time.perf_counter()
    oracle.periodic(a0, w.coeffs, 1, nthreads=nthr)
    t1 = time.perf_counter() - t0
    steps = int(max(1, min(64, budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    oracle.periodic(a0, w.coeffs, steps, nthreads=nthr)
    dt = time.perf_counter() - t0
    cells = int(np.prod(w.dims))
    return {"value": cells * steps / dt, "unit": "cell-updates/s", "cores": nthr, "kind": "oracle",
            "sample": f"full {w.dims[0]}x{w.dims[1]} grid, {steps} of the {w.T} steps "
                      f"(FP64 nested loop, OpenMP, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 path")
    ap.add_argument("--serving", type=int, default=10000, help="serving-mix requests (0 = skip)")
    ap.add_argument("--no-copy", action="store_true", help="skip the device-copy bandwidth reference")
    ap.add_argument("--no-others", action="store_true", help="skip the other workloads")
    ap.add_argument("--others", default=None,
                    help="comma-separated <workload>_<dtype> keys: time only these other workloads")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(a single periodic solve would need two all-to-alls per solve across GPUs, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2105_06676_amd as sfft
    import workloads as wl

    w = wl.config("jacobi2d_8192")
    N = int(np.prod(w.dims))
    wall32, gms32, lat32, k32, ok32 = time_path(sfft, torch, w, "f32", args.steps, args.warmup)
    ms32 = wall32 * 1e3 / args.steps
    res64 = None
    if not args.no_f64:
        wall64, gms64, lat64, k64, ok64 = time_path(sfft, torch, w, "f64", args.steps, args.warmup)
        ms64 = wall64 * 1e3 / args.steps
        res64 = {"value": N * w.T / (ms64 / 1e3), "ms_per_step": ms64,
                 "p50_ms": float(np.percentile(lat64, 50)), "p99_ms": float(np.percentile(lat64, 99)),
                 "finite": ok64,
                 "kernels": {k: {"avg_us": v["ms"] * 1e3 / v["launches"],
                                 "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9}
                             for k, v in k64.items()}}

    # dominant kernel of the headline path
    dom = max(k32.items(), key=lambda kv: kv[1]["ms"])
    name, kd = dom
    avg_s = kd["ms"] * 1e-3 / kd["launches"]
    bytes_per_launch = kd["bytes"] / kd["launches"]
    achieved = bytes_per_launch / avg_s / 1e9
    total_bytes = sum(v["bytes"] for v in k32.values()) / args.steps  # per solve (pass 3 ran `steps` solves)
    traffic = measured_traffic(name, kd["launches"] // args.steps)

    out = {
        "metric": "cell-updates/s (N*T/time)",
        "value": N * w.T / (ms32 / 1e3),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2-D periodic 5-point Jacobi stencil, 8192x8192 grid, T=4096, "
                               "FP32 FFT passes with FP64 symbol power (seeded U[0,1) grid)",
                   "dims": list(w.dims), "T": w.T, "radius": 1},
        "gpu_ms_per_step": gms32 / args.steps,
        "p50_ms": float(np.percentile(lat32, 50)),
        "p99_ms": float(np.percentile(lat32, 99)),
        "fft_hbm_roofline_frac_end_to_end": total_bytes / (ms32 * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "finite": ok32,
        "roofline": {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": avg_s * 1e6},
        "kernels_f32": {k: {"avg_us": v["ms"] * 1e3 / v["launches"], "launches": v["launches"],
                            "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9} for k, v in k32.items()},
        "f64": res64,
        "copy_reference": None if args.no_copy else copy_reference(torch, N * 4 * 2),
        "other_workloads": None if args.no_others else other_workloads(
            sfft, torch, None if args.others is None else set(args.others.split(","))),
        "cpu_baseline": None if args.no_cpu else cpu_baseline(w),
        "serving": serving_bench(sfft, torch, args.serving) if args.serving > 0 else None,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
