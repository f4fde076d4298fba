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
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def kernel_source_files() -> list:
    """The sources that decide what the pass kernels do: every .hip file, the
    headers they include (transitively), and the planner and table code that set
    their launch shapes and tables.  Host-only files (entry points, server, tuner,
    verification) are left out, so changing them keeps counter summaries valid."""
    csrc = os.path.join(ROOT, "paper_2105_06676_amd", "csrc")
    names = {n for n in os.listdir(csrc) if n.endswith(".hip")}
    names |= {"sfft_plan.cpp", "sfft_plan.h", "sfft_runtime.cpp"}
    todo = sorted(names)
    while todo:
        n = todo.pop()
        with open(os.path.join(csrc, n)) as f:
            for inc in re.findall(r'#include "([^"/]+)"', f.read()):
                if inc not in names and os.path.exists(os.path.join(csrc, inc)):
                    names.add(inc)
                    todo.append(inc)
    return sorted(names)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2105_06676_amd", "csrc")
    for name in kernel_source_files():
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
    # (2) latency (at least 200 samples, so that p99 is not just the largest of a few)
    nlat = max(steps, 200)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nlat)]
    for i in range(nlat):
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


def _request_grid(torch, r, gen, seed=5):
    """The request's initial grid, filled on the device from a torch generator
    seeded by the request id (the same grid every time it is drawn)."""
    gen.manual_seed(seed * 1000003 + r.rid)
    td = torch.float32 if r.dtype == "f32" else torch.float64
    return torch.rand(r.dims, generator=gen, device="cuda", dtype=td)


def _digest(torch, g):
    """Two wrapping int64 sums over the bit patterns of a result (plain and
    position-weighted): equal digests mean bit-identical results barring a
    collision."""
    v = g.reshape(-1).view(torch.int32 if g.dtype == torch.float32 else torch.int64).to(torch.int64)
    w = torch.arange(v.numel(), device=v.device, dtype=torch.int64) * 2 + 1
    return int(v.sum().item()), int((v * w).sum().item())


def serving_run(sfft, torch, reqs, rate=None, window=None, chunk=128, seed=5, on_done=None):
    """Drive the continuous-batching server with the request list.  rate=None:
    closed loop (keep `window` requests outstanding); else open-loop Poisson
    arrivals at `rate` requests/s (the list's arrival times rescaled).  Grids are
    filled on the device from seeded torch generators, a chunk ahead of use.
    on_done(request, grid) is called for each finished request (verification
    runs only: it is not part of a timed run)."""
    import time as _t
    srv = sfft.Server(0, 32 << 30, 64)
    gen = torch.Generator(device="cuda")
    ready = []
    nxt = 0

    def refill():
        nonlocal nxt
        out = []
        for r in reqs[nxt:nxt + chunk]:
            out.append((r, _request_grid(torch, r, gen, seed)))
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
                if on_done is not None:
                    on_done(*pending[t])
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
            "peak_workspace_bytes": st["peak_bytes"], "device": st.get("device")}


def serving_verify(sfft, torch, reqs, oracle_budget=4e9, per_stratum=9, seed=5):
    """Correctness of the served mix: (1) every request's served result (closed
    loop, as in the timed run) against the same request solved alone, bit for bit
    (by digest); (2) a stratified sample -- up to `per_stratum` requests of each
    (d, r, dtype) class among those whose loop-oracle cost N*T*(2r+1)^d is at most
    5e7, spread over T -- against the FP64 loop oracle (rel-L2 and max-abs)."""
    import oracle
    strata = {}
    for r in reqs:
        if r.cells * r.T * (2 * r.radius + 1) ** r.ndim <= 5e7:
            strata.setdefault((r.ndim, r.radius, r.dtype), []).append(r)
    sample = set()
    for key, lst in strata.items():
        lst = sorted(lst, key=lambda q: q.T)
        k = min(per_stratum, len(lst))
        for j in range(k):
            sample.add(lst[(j * (len(lst) - 1)) // max(1, k - 1)].rid)
    mixed, kept = {}, {}

    def on_done(r, g):
        mixed[r.rid] = _digest(torch, g)
        if r.rid in sample:
            kept[r.rid] = g.cpu().numpy().astype(np.float64)

    serving_run(sfft, torch, reqs, rate=None, window=256, seed=seed, on_done=on_done)
    gen = torch.Generator(device="cuda")
    mismatched = []
    for r in reqs:
        g = _request_grid(torch, r, gen, seed)
        sfft.periodic(g, r.coeffs, r.T)
        if _digest(torch, g) != mixed.get(r.rid):
            mismatched.append(r.rid)
    nthr = oracle.threads()
    errs = {"f32": [], "f64": []}
    spent = 0.0
    t0 = time.perf_counter()
    for rid in sorted(sample, key=lambda i: reqs[i].cells * reqs[i].T):
        r = reqs[rid]
        cost = r.cells * r.T * (2 * r.radius + 1) ** r.ndim
        if spent + cost > oracle_budget:
            continue
        spent += cost
        a0 = _request_grid(torch, r, gen, seed).cpu().numpy().astype(np.float64)
        ref = oracle.periodic(a0, r.coeffs, r.T, nthreads=nthr)
        e = _errors(kept[rid], ref)
        e.update(rid=rid, dims=list(r.dims), radius=r.radius, T=r.T)
        errs[r.dtype].append(e)
    tol = {"f32": 1e-5, "f64": 1e-12}
    summary = {}
    for dt, lst in errs.items():
        summary[dt] = {"checked": len(lst),
                       "max_rel_l2": max((e["rel_l2"] for e in lst), default=None),
                       "max_max_abs_rel": max((e["max_abs_rel"] for e in lst), default=None),
                       "within_tolerance": all(e["rel_l2"] <= tol[dt] and e["max_abs_rel"] <= tol[dt] for e in lst),
                       "strata": sorted({(e["dims"].__len__(), e["radius"]) for e in lst})}
    return {"alone_vs_mix": {"requests": len(reqs), "bit_identical": len(reqs) - len(mismatched),
                             "mismatched_ids": mismatched[:20]},
            "oracle_sample": dict(summary, sample_size=sum(len(v) for v in errs.values()),
                                  selection="up to 9 per (d, r, dtype) class with N*T*(2r+1)^d <= 5e7, spread over T",
                                  oracle_s=time.perf_counter() - t0)}


def serving_bench(sfft, torch, count, verify=True):
    import workloads as wl
    reqs = wl.serving_mix(count)
    # warm the plan cache with a short closed-loop pass over every distinct shape
    closed = serving_run(sfft, torch, reqs, rate=None, window=256)
    mu = closed["req_per_s"]
    openl = serving_run(sfft, torch, reqs, rate=0.7 * mu)
    out = {"workload": f"Poisson stream of {count} periodic requests: d ~ U{{1,2,3}}, cells log-uniform "
                       "2^10..2^24 (7-smooth extents), r ~ U{1,2}, T log-uniform 1..1e5, FP32/FP64 50/50",
           "closed_loop": closed, "open_loop_rate_req_s": 0.7 * mu, "open_loop": openl}
    if verify:
        out["verification"] = serving_verify(sfft, torch, reqs)
    # the same distribution at exact extents (rounded to the nearest integer, not
    # to a 7-smooth one): requests with a prime factor above 7 in an extent take
    # the chirp-z path, each solved on its own inside its arena block
    exact = wl.serving_mix(count // 5, smooth=False)
    out["exact_extents"] = dict(serving_run(sfft, torch, exact, rate=None, window=256),
                                workload=f"{count // 5} requests of the same distribution with extents rounded to "
                                         "the nearest integer")
    return out


def time_solve(sfft, torch, w, dtype, reps=5, warmup=1):
    """Median device time of one solve of workload w (inputs resident in HBM)."""
    td = torch.float32 if dtype == "f32" else torch.float64
    grid0 = torch.from_numpy(w.grid()).to(device="cuda:0", dtype=td)
    grid = grid0.clone()
    if w.implicit_q is not None:
        def fn(g, c, T):
            return sfft.periodic_implicit(g, w.implicit_q, c, T)
    else:
        if w.aperiodic:
            def fn(g, c, T):
                return sfft.aperiodic(g, c, T, bc=w.bc)
        else:
            fn = sfft.periodic_fields if w.fields > 1 else sfft.periodic
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


def other_workloads(sfft, torch, only=None, reps=5, warmup=1):
    """The other workloads of the method, timed the same way (context for the headline);
    `only`: a set of "<workload>_<dtype>" keys to restrict the list to."""
    import workloads as wl
    out = {}
    for name, dts in (("heat1d_65536", ("f64",)), ("star3d_512", ("f32",)),
                      ("box2d_aperiodic_4096", ("f64", "f32")), ("box2d_reflect_4096", ("f64", "f32")),
                      ("upwind2d_aperiodic_4096", ("f64", "f32")),
                      ("wave2d_leapfrog_4096", ("f32", "f64")),
                      ("heat2d_backward_euler_4096", ("f32", "f64")), ("jacobi2d_6300x6720_smooth", ("f32",)),
                      ("jacobi2d_8000_smooth", ("f32", "f64")), ("heat3d_800_smooth", ("f32",)),
                      ("jacobi2d_8191_prime", ("f32",))):
        w = wl.config(name)
        for dt in dts:
            if only is not None and f"{name}_{dt}" not in only:
                continue
            out[f"{name}_{dt}"] = dict(time_solve(sfft, torch, w, dt, reps=reps, warmup=warmup), dims=list(w.dims), T=w.T,
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
    """The FP64 loop oracle on the full-size grid for a bounded number of steps.
    The grid is the FP32-rounded initial grid (exact in both dtypes), so the
    oracle's output also serves as the expected value of both GPU paths at that
    step count.  Returns (baseline record, rounded input, steps, oracle output)."""
    import oracle
    a0 = w.grid().astype(np.float32).astype(np.float64)
    nthr = oracle.threads()
    t0 = time.perf_counter()
    oracle.periodic(a0, w.coeffs, 1, nthreads=nthr)
    t1 = time.perf_counter() - t0
    steps = int(max(1, min(64, budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    ref = oracle.periodic(a0, w.coeffs, steps, nthreads=nthr)
    dt = time.perf_counter() - t0
    cells = int(np.prod(w.dims))
    rec = {"value": cells * steps / dt, "unit": "cell-updates/s", "cores": nthr, "kind": "oracle",
           "sample": f"full {'x'.join(map(str, w.dims))} grid, {steps} of the {w.T} steps "
                     f"(FP64 nested loop, OpenMP, {dt:.1f} s)"}
    # one thread on a shortened problem (the first rows of the grid, periodic on
    # that crop), and the host it ran on
    inner = int(np.prod(w.dims[1:])) if len(w.dims) > 1 else 1
    rows = max(1, min(w.dims[0], (1 << 23) // inner))
    crop = np.ascontiguousarray(a0[:rows])
    t0 = time.perf_counter()
    oracle.periodic(crop, w.coeffs, 1, nthreads=1)
    t1 = time.perf_counter() - t0
    s1 = int(max(1, min(16, 3.0 / max(t1, 1e-3))))
    t0 = time.perf_counter()
    oracle.periodic(crop, w.coeffs, s1, nthreads=1)
    dt1 = time.perf_counter() - t0
    one = crop.size * s1 / dt1
    rec["one_thread"] = {"value": one, "unit": "cell-updates/s",
                         "sample": f"{'x'.join(map(str, crop.shape))} crop, {s1} steps ({dt1:.1f} s)",
                         "parallel_speedup": rec["value"] / one}
    rec["host"] = host_info()
    return rec, a0, steps, ref


def host_info() -> dict:
    """CPU model name and core counts of the host the oracle ran on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def _errors(y: np.ndarray, ref: np.ndarray) -> dict:
    """rel-L2 = |y - y*|_2 / |y*|_2, max-abs = max |y - y*|, and max-abs / max |y*|."""
    d = np.abs(y - ref)
    den = float(np.linalg.norm(ref))
    mref = float(np.max(np.abs(ref)))
    ma = float(np.max(d))
    return {"rel_l2": float(np.linalg.norm(y - ref)) / den if den > 0 else float(np.linalg.norm(y - ref)),
            "max_abs": ma, "max_abs_rel": ma / mref if mref > 0 else ma}


def _gpu_solve(sfft, torch, a0, coeffs, T, dtype, aperiodic=False):
    td = torch.float32 if dtype == "f32" else torch.float64
    g = torch.from_numpy(np.ascontiguousarray(a0)).to(device="cuda:0", dtype=td)
    (sfft.aperiodic if aperiodic else sfft.periodic)(g, coeffs, T)
    torch.cuda.synchronize()
    out = g.cpu().numpy().astype(np.float64)
    del g
    return out


def result_errors(sfft, torch, w, full=None):
    """Errors of GPU results against the FP64 loop oracle (the oracle of an FP32
    result runs on the FP32-rounded input), per result:
      * the 2-D Jacobi workload's 256 x 256 periodic instance (same stencil and
        T = 4096, initial data the top-left crop of the seeded grid), FP32 and FP64;
      * the full 8192 x 8192 grid at the step count of the CPU baseline's oracle
        run (`full` = (rounded input, steps, oracle output)), FP32 and FP64;
      * the full 8192 x 8192 FP32 result at T = 4096 against the FP64 GPU path
        (the oracle cannot run 2.7e11 cell updates within the bench);
      * the 1-D heat workload in full (N = 65536, T = 1024, FP64);
      * a 256 x 256 instance of the aperiodic 9-point box workload (same
        coefficients, T = 64, frame and interior from its seed), FP64 and FP32."""
    import oracle
    import workloads as wl
    nthr = oracle.threads()
    out = {"tolerance": {"f32": 1e-5, "f64": 1e-12}}
    crop = wl.crop_grid(w, 256)
    for dt in ("f32", "f64"):
        a0 = crop.astype(np.float32).astype(np.float64) if dt == "f32" else crop
        ref = oracle.periodic(a0, w.coeffs, w.T, nthreads=nthr)
        out[f"jacobi2d_256x256_instance_T{w.T}_{dt}"] = _errors(_gpu_solve(sfft, torch, a0, w.coeffs, w.T, dt), ref)
    if full is not None:
        a0, steps, ref = full
        for dt in ("f32", "f64"):
            out[f"jacobi2d_8192x8192_T{steps}_{dt}"] = _errors(_gpu_solve(sfft, torch, a0, w.coeffs, steps, dt), ref)
    a0 = w.grid().astype(np.float32).astype(np.float64)
    y32 = _gpu_solve(sfft, torch, a0, w.coeffs, w.T, "f32")
    y64 = _gpu_solve(sfft, torch, a0, w.coeffs, w.T, "f64")
    out[f"jacobi2d_8192x8192_T{w.T}_f32_vs_gpu_f64"] = _errors(y32, y64)
    del y32, y64, a0
    w1 = wl.config("heat1d_65536")
    ref = oracle.periodic(w1.grid(), w1.coeffs, w1.T, nthreads=nthr)
    out[f"heat1d_65536_T{w1.T}_f64"] = _errors(_gpu_solve(sfft, torch, w1.grid(), w1.coeffs, w1.T, "f64"), ref)
    w4 = wl.config("box2d_aperiodic_4096")
    ap = wl.crop_grid(w4, 258)
    for dt in ("f64", "f32"):
        a0 = ap.astype(np.float32).astype(np.float64) if dt == "f32" else ap
        ref = oracle.aperiodic(a0, w4.coeffs, 64, nthreads=nthr)
        out[f"box2d_aperiodic_256x256_instance_T64_{dt}"] = _errors(
            _gpu_solve(sfft, torch, a0, w4.coeffs, 64, dt, aperiodic=True), ref)
    out["max_rel_l2_vs_oracle"] = {dt: max(v["rel_l2"] for k, v in out.items() if k.endswith("_" + dt) and "_vs_" not in k
                                           and isinstance(v, dict) and "rel_l2" in v) for dt in ("f32", "f64")}
    return out


def mfma_probe(torch, n: int = 1 << 21, reps: int = 32):
    """One measurement of a DFT stage as a matrix product on the matrix cores
    against the butterflies the pass kernels use (paper_2105_06676_amd/probes):
    n 16-point FP32 complex vectors, each transformed `reps` times in registers."""
    import ctypes
    path = os.path.join(ROOT, "paper_2105_06676_amd", "libsfft_probe.so")
    lib = ctypes.CDLL(path)
    f = lib.sfft_probe_dft16
    f.restype = ctypes.c_float
    f.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
    gen = torch.Generator(device="cpu").manual_seed(5)
    x = torch.rand(n, 16, 2, generator=gen, dtype=torch.float32).to("cuda")
    outs, res = [], {}
    st = torch.cuda.current_stream().cuda_stream
    for variant, name in ((0, "butterfly"), (1, "mfma")):
        y = torch.empty_like(x)
        f(variant, x.data_ptr(), y.data_ptr(), n, 1, st)  # warm-up
        ms = min(f(variant, x.data_ptr(), y.data_ptr(), n, reps, st) for _ in range(3))
        ms1 = min(f(variant, x.data_ptr(), y.data_ptr(), n, 1, st) for _ in range(3))
        f(variant, x.data_ptr(), y.data_ptr(), n, reps, st)
        torch.cuda.synchronize()
        outs.append(y.double())
        # arithmetic of one application: (reps-time - one-application time) / (reps - 1)
        per = max(ms - ms1, 1e-9) / (reps - 1)
        res[name] = {"ms_reps": ms, "ms_one": ms1, "dft16_per_s": n / (per * 1e-3)}
    ref = outs[0]
    err = float((outs[1] - ref).norm() / ref.norm())
    res["mfma_vs_butterfly_rel_l2"] = err
    res["speedup_mfma_over_butterfly"] = res["mfma"]["dft16_per_s"] / res["butterfly"]["dft16_per_s"]
    res["config"] = {"vectors": n, "reps": reps, "dtype": "f32", "points": 16}
    return res


def strip_probe(torch, pitch: int = 4112, cols: int = 4097, reps: int = 20):
    """The memory side of a one-pass strided 8192-point transform
    (paper_2105_06676_amd/probes/strip_probe.hip): W = 1 or 2 columns of the
    8192^2 workload's half spectrum per workgroup (8 or 16 bytes per row and wave
    access), one LDS exchange, no arithmetic; against a plain device copy of the
    same bytes."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2105_06676_amd", "libsfft_probe.so"))
    f = lib.sfft_probe_strip
    f.restype = ctypes.c_float
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                  ctypes.c_int, ctypes.c_void_p]
    gen = torch.Generator(device="cpu").manual_seed(6)
    x = torch.rand(8192, pitch, 2, generator=gen, dtype=torch.float32).to("cuda")
    y = torch.zeros_like(x)
    st = torch.cuda.current_stream().cuda_stream
    nbytes = 2 * 8192 * cols * 8
    res = {"config": {"rows": 8192, "pitch": pitch, "columns": cols, "dtype": "f32 complex",
                      "bytes_per_launch": nbytes}}
    for W in (1, 2):
        for remap in (0, 1):
            if f(W, remap, x.data_ptr(), y.data_ptr(), pitch, cols, 2, st) < 0:
                raise RuntimeError("strip probe launch failed")
            ms = min(f(W, remap, x.data_ptr(), y.data_ptr(), pitch, cols, reps, st) for _ in range(3))
            torch.cuda.synchronize()
            ok = bool(torch.equal(y[:, :cols], x[:, :cols]))
            res[f"W{W}_remap{remap}"] = {"us": ms * 1e3, "GBps": nbytes / (ms * 1e-3) / 1e9, "exact_copy": ok}
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        y.copy_(x)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    res["device_copy"] = {"us": ms * 1e3, "GBps": 2 * x.numel() * 4 / (ms * 1e-3) / 1e9}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 path")
    ap.add_argument("--no-errors", action="store_true", help="skip the per-result errors against the oracle")
    ap.add_argument("--no-tune", action="store_true", help="plan with the default heuristics (no autotuning)")
    ap.add_argument("--serving", type=int, default=10000, help="serving-mix requests (0 = skip)")
    ap.add_argument("--no-copy", action="store_true", help="skip the device-copy bandwidth reference")
    ap.add_argument("--no-others", action="store_true", help="skip the other workloads")
    ap.add_argument("--others", default=None,
                    help="comma-separated <workload>_<dtype> keys: time only these other workloads")
    ap.add_argument("--only-others", action="store_true",
                    help="profiling runs: time only the other workloads (prints their JSON, no headline line)")
    ap.add_argument("--strip-probe", action="store_true",
                    help="measure the memory side of a one-pass strided 8192-point transform (prints its JSON only)")
    ap.add_argument("--mfma-probe", action="store_true",
                    help="measure a DFT stage on the matrix cores against butterflies (prints its JSON only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(a single periodic solve would need two all-to-alls per solve across GPUs, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2105_06676_amd as sfft
    import workloads as wl

    if args.mfma_probe:
        print(json.dumps({"mfma_probe": mfma_probe(torch)}))
        return
    if args.strip_probe:
        print(json.dumps({"strip_probe": strip_probe(torch)}))
        return

    if args.only_others:
        print(json.dumps({"other_workloads": other_workloads(
            sfft, torch, None if args.others is None else set(args.others.split(",")), reps=args.steps,
            warmup=args.warmup)}))
        return

    w = wl.config("jacobi2d_8192")
    N = int(np.prod(w.dims))
    # plan selection by the library's autotuner, outside the timed regions
    tuning = {}
    if not args.no_tune:
        for dt in ("f32",) + (() if args.no_f64 else ("f64",)):
            t0 = time.perf_counter()
            rep = sfft.tune(w.dims, dt, reps=5)
            tuning[dt] = {"seconds": time.perf_counter() - t0,
                          "axes": [{"n": a["n"], "chosen": a["chosen"], "chosen_us": a["chosen_us"],
                                    "default_us": a["default_us"]} for a in rep["axes"]],
                          "plan": sfft.plan_describe(w.dims, dt)["levels"]}
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

    cpu_rec, cpu_full = None, None
    if not args.no_cpu:
        cpu_rec, a0r, steps_r, ref_r = cpu_baseline(w)
        cpu_full = (a0r, steps_r, ref_r)

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
        "autotune": tuning or None,
        "copy_reference": None if args.no_copy else copy_reference(torch, N * 4 * 2),
        "other_workloads": None if args.no_others else other_workloads(
            sfft, torch, None if args.others is None else set(args.others.split(","))),
        "cpu_baseline": cpu_rec,
        "errors": None if args.no_errors else result_errors(sfft, torch, w, cpu_full),
        "serving": serving_bench(sfft, torch, args.serving, verify=not args.no_errors) if args.serving > 0 else None,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
