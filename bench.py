#!/usr/bin/env python3
"""Decompose + recompose throughput of the multigrid refactoring on one MI355X.

A step is one full decomposition followed by one full recomposition of the
workload (every level, every kernel of the path), inputs resident in HBM.
Prints one JSON line:
  value        refactoring throughput, the paper's unit (Sec. IV-D): bytes of
               field decomposed plus bytes recomposed per second,
               2 * n * sizeof(dtype) / (t_decompose + t_recompose), in GB/s;
  roofline     the dominant kernel's algorithmic bytes per launch / its mean
               launch time from HIP events recorded on the launch stream over
               the timed region, against the 8 TB/s HBM peak;
  cpu_baseline the FP64 CPU oracle on the same workload (one step), GB/s in
               the same unit, with the number of threads it used.
Extra keys: the algorithmic-byte rate of the whole step, `hbm_measured` (the
rocprofv3 HBM bytes of every kernel of one step, from the committed PMC
summary of the same kernel code, over the step time, and their ratio to the
algorithmic bytes), per-kernel totals,
the FP32 mode on the same grid, the round-trip error of the timed data,
`progressive`: the time and relative L2 error of recomposing from the k
coarsest coefficient classes, k = 0..nlevels, and
`batched`: 64 mixed 2-D/3-D FP32/FP64 fields decomposed and recomposed one
field per call, with the batched entry points, and with the batch replayed
from a HIP graph (p50/p99 ms per batch, GB/s, and whether the batched results
are bitwise those of the single calls), and
`service`: Poisson streams of mixed-size decompose/recompose requests served
under an HBM budget (p50/p99 latency, GB/s) next to the plain path, and
`spatiotemporal`: T = 1..16 time steps of a 400^3 FP64 field refactored
together as one 4-D field.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCE = os.path.join(ROOT, "paper_2105_12764_amd", "csrc", "mgr_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")


def code_sha256(path: str) -> str:
    """sha256 of a C++/HIP source with its // comments, trailing blanks and
    blank lines removed: it changes when the code changes, not its comments."""
    import hashlib
    import re

    lines = []
    for line in open(path, encoding="utf-8"):
        line = re.sub(r"//.*$", "", line.rstrip("\n")).rstrip()
        if line.strip():
            lines.append(line)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def traffic_record(kernel: str):
    """The committed rocprofv3 PMC record (profiles/*.md, a line
    '<!-- traffic: {json} -->') whose dominant kernel is `kernel`: HBM bytes
    per launch of that kernel and of the whole profiled step.  None when
    there is none or the kernel code changed since the counters were taken."""
    import glob
    import json as _json

    sha = code_sha256(KERNEL_SOURCE)
    for path in sorted(glob.glob(os.path.join(PROFILES, "*.md"))):
        for line in open(path):
            line = line.strip()
            if line.startswith("<!-- traffic:") and line.endswith("-->"):
                rec = _json.loads(line[len("<!-- traffic:"):-3])
                if rec.get("kernel") == kernel and rec.get("code_sha256") == sha:
                    return rec
    return None
METRIC = "decompose+recompose GB/s at 513^3 FP64/FP32 (% HBM peak); batched p50/p99 ms"


def _log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def run_gpu(name: str, steps: int, warmup: int, graph_steps: int = 0, tune: bool = True,
            progressive_on: bool = True, keep_output: bool = False):
    """One workload: warm-up, autotuning, the timed steps (events at the
    decompose/recompose boundaries), the same steps with per-launch events
    (per-kernel totals and the roofline), optional graph replay and the
    partial recompositions.  With keep_output, the host copy of the GPU's
    decomposition of the input is returned too (for the errors against the
    oracle, computed in the CPU-baseline leg)."""
    import torch

    from paper_2105_12764_amd import mgr
    from paper_2105_12764_amd.synth import WORKLOADS, make_input

    shape, seed, nonuni, dtype, nlev = WORKLOADS[name]
    _log(f"[bench] {name}: generating {shape} {np.dtype(dtype).name}")
    u, coords = make_input(shape, seed, nonuniform=nonuni, dtype=dtype)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(u).to(dev)
    d = torch.empty_like(x)
    r = torch.empty_like(x)
    ws = mgr.alloc_workspace(shape, x.dtype, nlev, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        mgr.decompose(x, coords, nlev, out=d, workspace=ws, stream=stream)
        if ev is not None:
            ev.record(stream)
        mgr.recompose(d, coords, nlev, out=r, workspace=ws, stream=stream)

    _log(f"[bench] {name}: warmup {warmup}")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()

    untuned = None
    report = None
    if tune:
        # the built-in launch shapes first, then the autotuned ones (the plan
        # keeps them; the timed regions below use them)
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        n0 = max(3, steps // 2)
        a0.record(stream)
        for _ in range(n0):
            step()
        a1.record(stream)
        torch.cuda.synchronize()
        untuned = a0.elapsed_time(a1) / n0
        report = mgr.autotune(x, coords, nlev, out=r, workspace=ws)
        for _ in range(max(1, warmup)):
            step()
        torch.cuda.synchronize()
        _log(f"[bench] {name}: untuned {untuned:.3f} ms/step; autotuned")

    # timed region 1: the throughput (events only at decompose/recompose boundaries)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    mids = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record(stream)
        step(mids[i])
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_dec = sum(starts[i].elapsed_time(mids[i]) for i in range(steps)) / steps
    t_rec = sum(mids[i].elapsed_time(ends[i]) for i in range(steps)) / steps
    _log(f"[bench] {name}: {steps} steps, dec {t_dec:.3f} ms, rec {t_rec:.3f} ms")

    # timed region 2: the same steps with every kernel launch bracketed by HIP
    # events on its stream (per-kernel times for the roofline)
    mgr.timing_reset()
    mgr.timing_enable(True)
    torch.cuda.synchronize()
    for i in range(steps):
        step()
    torch.cuda.synchronize()
    mgr.timing_enable(False)
    totals = mgr.timing_totals()

    graph = None
    if graph_steps:
        # the same step captured once into a HIP graph and replayed: the
        # library's launches become graph nodes (no per-launch host overhead)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step()  # warm the plan cache outside the capture
            with torch.cuda.graph(g, stream=side):
                mgr.decompose(x, coords, nlev, out=d, workspace=ws, stream=side)
                mgr.recompose(d, coords, nlev, out=r, workspace=ws, stream=side)
        torch.cuda.synchronize()
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record()
        for _ in range(graph_steps):
            g.replay()
        g1.record()
        torch.cuda.synchronize()
        gms = g0.elapsed_time(g1) / graph_steps
        graph = {"ms_per_step": gms, "value": 2.0 * int(np.prod(shape)) * np.dtype(dtype).itemsize / (gms * 1e-3) / 1e9}
        _log(f"[bench] {name}: graph replay {gms:.3f} ms/step")

    rt_err = float((r.double() - x.double()).abs().max() / x.double().abs().max())
    mgr.decompose(x, coords, nlev, out=d, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    dec_host = d.cpu().numpy() if keep_output else None

    # progressive recomposition: error and time with the nkeep coarsest classes
    progressive = []
    xn = float(x.double().norm())
    for nkeep in range(nlev + 1 if progressive_on else 0):
        mgr.recompose_partial(d, nkeep, coords, nlev, out=r, workspace=ws, stream=stream)
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record(stream)
        for _ in range(3):
            mgr.recompose_partial(d, nkeep, coords, nlev, out=r, workspace=ws, stream=stream)
        p1.record(stream)
        torch.cuda.synchronize()
        progressive.append({"classes_kept": nkeep, "ms": round(p0.elapsed_time(p1) / 3, 4),
                            "rel_l2_error": float((r.double() - x.double()).norm()) / xn})
    n = int(np.prod(shape))
    esz = np.dtype(dtype).itemsize
    ms_step = wall * 1e3 / steps
    value = 2.0 * n * esz / ((t_dec + t_rec) * 1e-3) / 1e9
    alg_bytes_step = sum(b for (_, _, b) in totals.values()) / steps
    kernels = {k: {"launches_per_step": v[0] / steps, "ms_per_step": v[1] / steps,
                   "alg_GBps": (v[2] / (v[1] * 1e-3) / 1e9) if v[1] > 0 else None}
               for k, v in sorted(totals.items(), key=lambda kv: -kv[1][1])}
    dom_name, (dom_n, dom_ms, dom_b) = max(totals.items(), key=lambda kv: kv[1][1])
    achieved = dom_b / (dom_ms * 1e-3) / 1e9
    rec = traffic_record(dom_name)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": rec["bytes_per_launch"] if rec else None,
                "kernel": dom_name,
                "alg_bytes_per_launch": dom_b / dom_n, "mean_launch_us": dom_ms * 1e3 / dom_n}
    # measured HBM bytes of the whole step (rocprofv3 FETCH_SIZE + WRITE_SIZE over
    # every dispatch of one decompose + recompose) over the step's event time
    hbm_measured = None
    if rec and rec.get("step_bytes"):
        sb = float(rec["step_bytes"])
        gbps = sb / ((t_dec + t_rec) * 1e-3) / 1e9
        hbm_measured = {"bytes_per_step": int(sb), "GBps": round(gbps, 1),
                        "pct_hbm_peak": round(100.0 * gbps / HBM_PEAK_GBS, 2),
                        "amplification_over_alg": round(sb / alg_bytes_step, 3)}
    res = {
        "workload": name, "shape": list(shape), "dtype": np.dtype(dtype).name, "nlevels": nlev,
        "t_dec_ms": t_dec, "t_rec_ms": t_rec, "ms_per_step": ms_step, "value": value,
        "alg_GB_per_step": alg_bytes_step / 1e9,
        "alg_GBps": alg_bytes_step / ((t_dec + t_rec) * 1e-3) / 1e9,
        "roundtrip_max_rel_err": rt_err, "kernels": kernels, "roofline": roofline,
        "hbm_measured": hbm_measured,
        "graph": graph,
        "progressive": progressive,
        "autotune": None if not tune else {
            "untuned_ms_per_step": round(untuned, 4),
            "untuned_value": round(2.0 * n * esz / (untuned * 1e-3) / 1e9, 2),
            "report": report.strip().splitlines()},
    }
    del x, d, r, ws
    torch.cuda.empty_cache()
    return res, u, coords, nlev, dec_host


def _pct(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, int(round(q * (len(v) - 1))))]


def run_batched(reps: int = 10, warmup: int = 2, nfields: int = 64):
    """The mixed batch (synth.batch_specs): one field per call vs. the batched
    entry points with grouped launches (one grid per kernel and level step
    across the fields) and with per-field chains on internal streams, each
    also replayed from a HIP graph."""
    import torch

    from paper_2105_12764_amd import mgr
    from paper_2105_12764_amd.synth import batch_specs, make_input

    specs = batch_specs(nfields)
    dev = torch.device("cuda:0")
    _log(f"[bench] batch: generating {nfields} fields")
    xs = []
    for shape, dtype, seed in specs:
        u, _ = make_input(shape, seed, nonuniform=False, dtype=dtype)
        xs.append(torch.from_numpy(u).to(dev))
        del u
    nbytes = sum(2 * x.numel() * x.element_size() for x in xs)
    nlev = [mgr.max_levels(tuple(x.shape)) for x in xs]
    d1 = [torch.empty_like(x) for x in xs]
    r1 = [torch.empty_like(x) for x in xs]
    d2 = [torch.empty_like(x) for x in xs]
    r2 = [torch.empty_like(x) for x in xs]
    ws1 = torch.empty(max(mgr.workspace_size(tuple(x.shape), x.dtype, n) for x, n in zip(xs, nlev)) + 1,
                      dtype=torch.uint8, device=dev)
    bd = mgr.Batch([(x, y, None, n) for x, y, n in zip(xs, d2, nlev)])
    br = mgr.Batch([(y, z, None, n) for y, z, n in zip(d2, r2, nlev)])
    ws2 = bd.alloc_workspace(dev)
    stream = torch.cuda.current_stream(dev)

    for x, y, n in zip(xs, d1, nlev):  # autotuned launch shapes for every field's plan
        mgr.autotune(x, None, n, out=y, workspace=ws1, stream=stream)
    torch.cuda.synchronize()

    def serial():
        for x, y, z, n in zip(xs, d1, r1, nlev):
            mgr.decompose(x, None, n, out=y, workspace=ws1, stream=stream)
            mgr.recompose(y, None, n, out=z, workspace=ws1, stream=stream)

    def batched(st=None, per_field=False):
        mgr.decompose_batch(bd, ws2, stream=st or stream, per_field=per_field)
        mgr.recompose_batch(br, ws2, stream=st or stream, per_field=per_field)

    def per_field(st=None):
        batched(st, per_field=True)

    def timed(fn, n):
        out = []
        for _ in range(n):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            out.append(a.elapsed_time(b))
        return out

    for _ in range(warmup):
        serial()
        per_field()
        batched()
    torch.cuda.synchronize()
    t_serial = timed(serial, reps)
    t_pf = timed(per_field, reps)
    t_batch = timed(batched, reps)

    def graph_of(fn):
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                fn(side)
        torch.cuda.synchronize()
        for _ in range(warmup):
            g.replay()
        torch.cuda.synchronize()
        return g

    g_pf = graph_of(per_field)
    t_pf_graph = timed(g_pf.replay, reps)
    g = graph_of(batched)
    t_graph = timed(g.replay, reps)  # the grouped batch's results stay in d2, r2
    same = all(torch.equal(a, b) for a, b in zip(d1, d2)) and all(torch.equal(a, b) for a, b in zip(r1, r2))
    err = max(float((z.double() - x.double()).abs().max() / x.double().abs().max()) for x, z in zip(xs, r2))
    # kernel launches per batch in each mode (every launch of the library is timed)
    launches = {}
    for name, fn in (("one_field_per_call", serial), ("per_field", per_field), ("grouped", batched)):
        mgr.timing_reset()
        mgr.timing_enable(True)
        fn()
        torch.cuda.synchronize()
        mgr.timing_enable(False)
        launches[name] = int(sum(v[0] for v in mgr.timing_totals().values()))

    def stats(v):
        return {"p50": round(_pct(v, 0.5), 4), "p99": round(_pct(v, 0.99), 4),
                "GBps": round(nbytes / (_pct(v, 0.5) * 1e-3) / 1e9, 1)}

    res = {"fields": nfields, "shapes": "2-D sides 257..2049 and 3-D sides 33..257, log-uniform; "
                                         "FP32/FP64 mixed; all levels; seeds 4000+i; autotuned",
           "n_2d": sum(1 for s in specs if len(s[0]) == 2),
           "n_fp64": sum(1 for s in specs if s[1] == np.float64),
           "bytes_per_batch": nbytes, "reps": reps,
           "one_field_per_call_ms": stats(t_serial),
           "per_field_streams_ms": stats(t_pf), "per_field_streams_graph_ms": stats(t_pf_graph),
           "grouped_ms": stats(t_batch), "grouped_graph_ms": stats(t_graph),
           "launches_per_batch": launches,
           "speedup_grouped_graph_vs_one_field_per_call": round(_pct(t_serial, 0.5) / _pct(t_graph, 0.5), 3),
           "speedup_grouped_graph_vs_per_field_graph": round(_pct(t_pf_graph, 0.5) / _pct(t_graph, 0.5), 3),
           "bitwise_equal_to_single_calls": bool(same), "roundtrip_max_rel_err": err}
    _log(f"[bench] batch: one field per call {res['one_field_per_call_ms']['p50']:.3f} ms, per-field streams "
         f"{res['per_field_streams_ms']['p50']:.3f} ms (graph {res['per_field_streams_graph_ms']['p50']:.3f}), "
         f"grouped {res['grouped_ms']['p50']:.3f} ms (graph {res['grouped_graph_ms']['p50']:.3f}); "
         f"launches {launches}")
    del xs, d1, r1, d2, r2, ws1, ws2, g, g_pf
    torch.cuda.empty_cache()
    return res


def run_latency(name: str = "cube65_f64", reps: int = 100, warmup: int = 10):
    """Latency of one small workload (65^3 FP64, 5 levels: launch-bound):
    per repetition the device time of the decomposition and of the
    recomposition (HIP events on the stream) and the host wall time of the
    whole step (both calls, then a stream synchronisation); medians in
    microseconds."""
    import torch

    from paper_2105_12764_amd import mgr
    from paper_2105_12764_amd.synth import WORKLOADS, make_input

    shape, seed, nonuni, dtype, nlev = WORKLOADS[name]
    u, coords = make_input(shape, seed, nonuniform=nonuni, dtype=dtype)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(u).to(dev)
    d, r = torch.empty_like(x), torch.empty_like(x)
    ws = mgr.alloc_workspace(shape, x.dtype, nlev, device=dev)
    stream = torch.cuda.current_stream(dev)
    for _ in range(warmup):
        mgr.decompose(x, coords, nlev, out=d, workspace=ws, stream=stream)
        mgr.recompose(d, coords, nlev, out=r, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    t_dec, t_rec, wall = [], [], []
    for _ in range(reps):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        h0 = time.perf_counter()
        e0.record(stream)
        mgr.decompose(x, coords, nlev, out=d, workspace=ws, stream=stream)
        e1.record(stream)
        mgr.recompose(d, coords, nlev, out=r, workspace=ws, stream=stream)
        e2.record(stream)
        stream.synchronize()
        wall.append((time.perf_counter() - h0) * 1e6)
        t_dec.append(e0.elapsed_time(e1) * 1e3)
        t_rec.append(e1.elapsed_time(e2) * 1e3)
    err = float((r - x).abs().max() / x.abs().max())
    both = [a + b for a, b in zip(t_dec, t_rec)]
    res = {"workload": f"{name}: {'x'.join(map(str, shape))} {np.dtype(dtype).name}, {nlev} levels",
           "reps": reps, "decompose_us_p50": round(_pct(t_dec, 0.5), 1),
           "recompose_us_p50": round(_pct(t_rec, 0.5), 1), "device_step_us_p50": round(_pct(both, 0.5), 1),
           "device_step_us_p99": round(_pct(both, 0.99), 1), "host_wall_step_us_p50": round(_pct(wall, 0.5), 1),
           "host_wall_step_us_p99": round(_pct(wall, 0.99), 1),
           "GBps_at_p50": round(2.0 * x.numel() * x.element_size() / (_pct(both, 0.5) * 1e-6) / 1e9, 1),
           "roundtrip_max_rel_err": err}
    _log(f"[bench] latency {name}: device {res['device_step_us_p50']} us, host wall {res['host_wall_step_us_p50']} us")
    del x, d, r, ws
    torch.cuda.empty_cache()
    return res


def run_service(nreq: int = 5000, rates=(50, 100, 200, 500, 1000, 2000, 4000, 8000, 16000),
                max_secs: float = 10.0, budget_gb: float = 64.0, nstreams: int = 4, slots: int = 32,
                tight_gb: float = 4.0):
    """The refactoring service (mgr_service_*) under Poisson arrivals.

    Requests come from synth.service_requests (3-D cubes, integer side
    log-uniform over [17, 513], FP32:FP64 = 3:1, decompose:recompose = 1:1,
    seed 5000).  A request's input is the leading side^3 elements of one
    seeded random pool per dtype (time does not depend on values); its output
    is one of `slots` buffers sized for the largest request, used in turn (a
    buffer is reused only after its previous request is done).  Latency is
    submit -> completion seen by the service's waiter thread.  Also timed:
    the plain path (the requests back to back, one call per request on one
    stream) and the service with every request submitted at once, under the
    stated budget and under a tight one.  Each Poisson rate serves the first
    min(nreq, rate x max_secs) requests of the stream."""
    import torch

    from paper_2105_12764_amd import mgr
    from paper_2105_12764_amd.synth import SERVICE_SIDE_MAX, service_requests

    dev = torch.device("cuda:0")
    reqs = service_requests(nreq)
    gen = torch.Generator(device=dev)
    gen.manual_seed(5000)
    nmax = SERVICE_SIDE_MAX ** 3
    pool = {dt: torch.randn(nmax, dtype=dt, device=dev, generator=gen) for dt in (torch.float32, torch.float64)}
    outbuf = [torch.empty(nmax * 8, dtype=torch.uint8, device=dev) for _ in range(slots)]
    tdt = [torch.float32 if r[1] == np.float32 else torch.float64 for r in reqs]

    def io(i):
        side, dt = reqs[i][0], tdt[i]
        n = side ** 3
        esz = 4 if dt == torch.float32 else 8
        return (pool[dt][:n].view(side, side, side),
                outbuf[i % slots][:n * esz].view(dt).view(side, side, side))

    def nbytes_of(k):
        return sum(2 * (reqs[i][0] ** 3) * (4 if tdt[i] == torch.float32 else 8) for i in range(k))

    stream = torch.cuda.current_stream(dev)
    ws = torch.empty(mgr.workspace_size((SERVICE_SIDE_MAX,) * 3, torch.float64,
                                        mgr.max_levels((SERVICE_SIDE_MAX,) * 3)) + 1, dtype=torch.uint8, device=dev)

    def plain():
        for i, r in enumerate(reqs):
            x, y = io(i)
            (mgr.recompose if r[2] else mgr.decompose)(x, None, None, out=y, workspace=ws, stream=stream)

    nbytes = nbytes_of(nreq)
    _log(f"[bench] service: {nreq} requests, {len({r[0] for r in reqs})} distinct sides, "
         f"{nbytes / 1e9:.1f} GB moved per pass")
    plain()  # builds every plan
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    plain()
    b.record(stream)
    b.synchronize()
    t_plain = a.elapsed_time(b)

    def serve(rate, budget, k):
        svc = mgr.Service(int(budget), nstreams=nstreams)
        last = {}
        tickets, t_sub, lags = [], [], []
        t0 = time.perf_counter()
        t_arr = 0.0
        for i in range(k):
            r = reqs[i]
            if rate:
                t_arr += r[3] / rate
                while True:
                    wait = t0 + t_arr - time.perf_counter()
                    if wait <= 0:
                        break
                    if wait > 2e-4:
                        time.sleep(wait - 1e-4)
            slot = i % slots
            prev = last.get(slot)
            while prev is not None and not svc.result(prev)[0]:
                time.sleep(5e-5)  # that output buffer's previous request is still running
            ts = time.perf_counter()
            lags.append(ts - (t0 + t_arr) if rate else 0.0)
            x, y = io(i)
            t = svc.submit(bool(r[2]), x, y, None, None)
            last[slot] = t
            tickets.append(t)
            t_sub.append(ts)
        svc.wait_all()
        res = [svc.result(t) for t in tickets]
        svc.close()
        bad = sum(1 for q in res if not q[0] or q[1] != mgr.MGR_OK)
        lat = [q[3] for q in res]
        que = [q[2] for q in res]
        span = max(ts + q[3] * 1e-3 for ts, q in zip(t_sub, res)) - min(t_sub)
        nb = nbytes_of(k)
        out = {"requests": k, "latency_ms": {"p50": round(_pct(lat, 0.5), 4), "p99": round(_pct(lat, 0.99), 4),
                                             "max": round(max(lat), 4)},
               "queue_ms": {"p50": round(_pct(que, 0.5), 4), "p99": round(_pct(que, 0.99), 4)},
               "GBps": round(nb / span / 1e9, 1), "span_s": round(span, 4), "failed": bad}
        if rate:
            out["offered_GBps"] = round(nb * rate / sum(reqs[i][3] for i in range(k)) / 1e9, 1)
            out["arrival_lag_ms_p99"] = round(1e3 * _pct(lags, 0.99), 4)
        return out

    budget = budget_gb * 1e9
    sat = serve(None, budget, nreq)
    _log(f"[bench] service: plain path {nbytes / (t_plain * 1e-3) / 1e9:.1f} GB/s, service all-at-once "
         f"{sat['GBps']} GB/s, p99 {sat['latency_ms']['p99']} ms")
    tight = serve(None, tight_gb * 1e9, nreq)
    per_rate = {}
    for rate in rates:
        k = int(min(nreq, max(50, rate * max_secs)))
        per_rate[str(rate)] = serve(rate, budget, k)
        _log(f"[bench] service: {rate}/s x {k}: p50 {per_rate[str(rate)]['latency_ms']['p50']} ms, "
             f"p99 {per_rate[str(rate)]['latency_ms']['p99']} ms, {per_rate[str(rate)]['GBps']} GB/s")
    res = {"requests": nreq, "seed": 5000,
           "mix": "3-D cubes, integer side log-uniform over [17, 513], FP32:FP64 = 3:1, "
                  "decompose:recompose = 1:1, all levels, built-in launch shapes",
           "distinct_sides": len({r[0] for r in reqs}),
           "bytes_per_pass": nbytes, "budget_GB": budget_gb, "streams": nstreams, "output_slots": slots,
           "per_rate_requests": f"min({nreq}, rate x {max_secs:g} s)",
           "plain_one_call_per_request": {"ms": round(t_plain, 3),
                                          "GBps": round(nbytes / (t_plain * 1e-3) / 1e9, 1)},
           "all_at_once": sat, f"all_at_once_budget_{tight_gb:g}GB": tight, "poisson": per_rate,
           "mean_request_bytes": nbytes / nreq / 2}
    del pool, outbuf, ws
    torch.cuda.empty_cache()
    return res


def run_spatiotemporal(side: int = 400, steps=(1, 2, 4, 8, 16), reps: int = 3):
    """4-D refactoring (time as a fourth dimension, Sec. III-D, IV-F): T time
    steps of a side^3 FP64 field (512 MB per step at side 400) refactored
    together as one (T, side, side, side) field, all levels; T = 1 is the
    3-D path on one step.  GB/s = 2 x bytes / (t_dec + t_rec), best of reps;
    per-kernel totals of one T = max(steps) pass."""
    import torch

    from paper_2105_12764_amd import mgr

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(6000)
    tmax = max(steps)
    full = torch.randn((tmax, side, side, side), dtype=torch.float64, device=dev, generator=gen)
    out = {}
    kern = None
    for T in steps:
        x = full[0] if T == 1 else full[:T]
        shape = tuple(x.shape)
        nlev = mgr.max_levels(shape)
        d = torch.empty_like(x)
        r = torch.empty_like(x)
        ws = mgr.alloc_workspace(shape, x.dtype, nlev, device=dev)
        mgr.decompose(x, None, nlev, out=d, workspace=ws, stream=stream)
        mgr.recompose(d, None, nlev, out=r, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record(stream)
            mgr.decompose(x, None, nlev, out=d, workspace=ws, stream=stream)
            e1.record(stream)
            mgr.recompose(d, None, nlev, out=r, workspace=ws, stream=stream)
            e2.record(stream)
            torch.cuda.synchronize()
            t = (e0.elapsed_time(e1), e1.elapsed_time(e2))
            if best is None or sum(t) < sum(best):
                best = t
        if T == tmax:
            mgr.timing_reset()
            mgr.timing_enable(True)
            mgr.decompose(x, None, nlev, out=d, workspace=ws, stream=stream)
            mgr.recompose(d, None, nlev, out=r, workspace=ws, stream=stream)
            torch.cuda.synchronize()
            mgr.timing_enable(False)
            kern = {k: {"launches": v[0], "ms": round(v[1], 4),
                        "alg_GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
                    for k, v in sorted(mgr.timing_totals().items(), key=lambda kv: -kv[1][1])[:10]}
        err = float((r - x).abs().max() / x.abs().max())
        nbytes = x.numel() * 8
        out[str(T)] = {"shape": list(shape), "nlevels": nlev, "t_dec_ms": round(best[0], 3),
                       "t_rec_ms": round(best[1], 3),
                       "GBps": round(2.0 * nbytes / (sum(best) * 1e-3) / 1e9, 1), "roundtrip_max_rel_err": err}
        _log(f"[bench] spatiotemporal T={T}: dec {best[0]:.2f} ms rec {best[1]:.2f} ms "
             f"{out[str(T)]['GBps']} GB/s")
        del d, r, ws
    del full
    torch.cuda.empty_cache()
    return {"space": f"{side}^3 FP64 per time step ({side ** 3 * 8 / 2 ** 20:.0f} MiB)",
            "data": "torch.randn, seed 6000 (time does not depend on values)", "per_T": out,
            "kernels_at_max_T": kern}


def probe_bandwidth(nbytes: int = 1 << 30, reps: int = 10):
    """Achievable single-pass bandwidth: the library's streaming copy probe
    (one read + one write of every byte), 2 * bytes / time."""
    import torch

    from paper_2105_12764_amd import mgr

    dev = torch.device("cuda:0")
    a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream(dev)
    for _ in range(3):
        mgr.probe_copy(a, b, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        mgr.probe_copy(a, b, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(a, b))
    del a, b
    torch.cuda.empty_cache()
    return {"bytes": nbytes, "ms": ms, "GBps": 2.0 * nbytes / (ms * 1e-3) / 1e9, "verified": ok}


def _drop_level(n: int, nlev: int) -> np.ndarray:
    """Level at which each position of a dimension of n nodes leaves the
    hierarchy (nlev for the coarsest grid's positions): along a dimension of
    m >= 3 level nodes the coarser grid keeps the even positions and the last."""
    out = np.full(n, nlev, dtype=np.int8)
    pos = np.arange(n)
    for s in range(nlev):
        m = len(pos)
        keep = np.ones(m, bool) if m < 3 else ((np.arange(m) % 2 == 0) | (np.arange(m) == m - 1))
        out[pos[~keep]] = s
        pos = pos[keep]
    return out


def errors_vs_oracle(got, ref, nlev):
    """The GPU's decomposition against the oracle's: max |g - o| / max |o| and
    relative L2 over the whole nodal array, and per coefficient class (the
    nodes leaving the hierarchy at one level; the last class is the coarsest
    grid) the class's max error and L2 error relative to that class."""
    shape = ref.shape
    cls = None
    for k, n in enumerate(shape):
        sh = [1] * len(shape)
        sh[k] = n
        lv = _drop_level(n, nlev).reshape(sh)
        cls = lv if cls is None else np.minimum(cls, lv)
    cls = np.broadcast_to(cls, shape)
    diff = got.astype(np.float64) - ref
    out = {"max_rel": float(np.max(np.abs(diff)) / np.max(np.abs(ref))),
           "l2_rel": float(np.linalg.norm(diff) / np.linalg.norm(ref)), "per_class": []}
    for c in range(nlev + 1):
        m = cls == c
        if not m.any():
            continue
        dc, rc = diff[m], ref[m]
        rmax, rl2 = float(np.max(np.abs(rc))), float(np.linalg.norm(rc))
        out["per_class"].append({"class": c, "nodes": int(m.sum()),
                                 "max_rel": float(np.max(np.abs(dc))) / rmax if rmax > 0 else None,
                                 "l2_rel": float(np.linalg.norm(dc)) / rl2 if rl2 > 0 else None})
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(kept, batch_fields: int = 64, service_reqs=None, service_GBps=None):
    """The FP64 CPU oracle, as it stands, timed on this host: built for it
    (gcc -O2 -march=native, same arithmetic) and run with all cores
    (OMP_NUM_THREADS, else every CPU) and with one.  `kept` maps a workload
    name to (field, coords, nlevels, GPU decomposition); for each the oracle's
    decomposition and recomposition are timed (median of 3 where a run takes
    under a few seconds, else one run) and the GPU's decomposition is
    compared with the oracle's.  The headline value is the full 513^3 FP64
    workload on all cores; the one-core figure uses a 257^3 sample of the
    same recipe (the full workload takes about half a minute on one core).
    Also timed: the 64-field batch on all cores, and the request rate the
    oracle could sustain on the service stream (from its 513^3 rate)."""
    import oracle
    from paper_2105_12764_amd.synth import batch_specs, make_input

    nat = oracle.Native()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1

    def timed(u, coords, nlev, nthreads, reps, recompose=True):
        nat.threads(nthreads)
        u64 = np.ascontiguousarray(u, dtype=np.float64)
        runs, dref = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            dref = nat.decompose(u64, coords, nlev)
            t1 = time.perf_counter()
            if recompose:
                nat.recompose(dref, coords, nlev)
            t2 = time.perf_counter()
            runs.append((t1 - t0, t2 - t1))
        runs.sort(key=lambda t: t[0] + t[1])
        td, tr = runs[len(runs) // 2]
        nb = u.size * u.dtype.itemsize
        rec = {"threads": nat.max_threads(), "runs": reps, "dec_s": round(td, 4)}
        if recompose:
            rec.update({"rec_s": round(tr, 4), "GBps": round(2.0 * nb / (td + tr) / 1e9, 4)})
        else:
            rec["GBps_decompose"] = round(nb / td / 1e9, 4)
        return dref, rec

    per, errors = {}, {}
    for name, (u, coords, nlev, got) in kept.items():
        big = u.size > 50_000_000
        _log(f"[bench] cpu baseline: oracle on {name}, {threads} threads")
        recompose = not (big and u.dtype == np.float32)  # the FP32 513^3 run is only for the errors
        dref, rec_all = timed(u, coords, nlev, threads, 1 if big else 3, recompose=recompose)
        per[name] = {"all_cores": rec_all}
        if got is not None:
            errors[name] = errors_vs_oracle(got, dref, nlev)
            _log(f"[bench] {name}: GPU vs oracle max {errors[name]['max_rel']:.2e}, L2 {errors[name]['l2_rel']:.2e}")
        del dref
        if not big:
            _, per[name]["one_core"] = timed(u, coords, nlev, 1, 3 if u.size < 1_000_000 else 1)
    # one core on a 257^3 sample of the 513^3 FP64 workload's recipe
    us, cs = make_input((257, 257, 257), 1002)
    _log("[bench] cpu baseline: one core on a 257^3 sample")
    _, one = timed(us, cs, 8, 1, 1)
    one["sample"] = "257^3 FP64, 8 levels, same generator recipe as the 513^3 workload (seed 1002)"
    del us
    head = per.get("cube513_f64", {}).get("all_cores")
    res = {"value": head["GBps"] if head else None, "unit": "GB/s", "cores": head["threads"] if head else threads,
           "kind": "oracle",
           "sample": (f"one decompose+recompose of the full 513x513x513 FP64 workload "
                      f"({head['dec_s'] + head['rec_s']:.1f} s)") if head else None,
           "single_core": one, "nproc": os.cpu_count(), "cpu_model": _cpu_model(), "build": nat.flags,
           "per_config": per}
    if batch_fields:
        specs = batch_specs(batch_fields)
        nat.threads(threads)
        tot, nb = 0.0, 0
        for shape, dtype, seed in specs:
            u, _ = make_input(shape, seed, nonuniform=False, dtype=dtype)
            nl = oracle.max_levels(shape)
            u64 = u.astype(np.float64)
            t0 = time.perf_counter()
            d = nat.decompose(u64, None, nl)
            nat.recompose(d, None, nl)
            tot += time.perf_counter() - t0
            nb += 2 * u.size * u.dtype.itemsize
        res["batch"] = {"fields": batch_fields, "threads": nat.max_threads(), "s": round(tot, 3),
                        "GBps": round(nb / tot / 1e9, 4)}
        _log(f"[bench] cpu baseline: 64-field batch {tot:.2f} s")
    if service_reqs and head:
        # per direction the oracle moves a request's bytes at about its 513^3 rate
        t_mean = float(np.mean([(r[0] ** 3) * (4 if r[1] == np.float32 else 8) / (head["GBps"] * 1e9)
                                for r in service_reqs]))
        res["service_sustainable_req_per_s"] = round(1.0 / t_mean, 3)
        res["service_note"] = ("estimated: each request's bytes at the oracle's all-core 513^3 rate "
                               "(per direction), averaged over the request stream")
    return res, errors


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cube513_f64")
    ap.add_argument("--fp32-workload", default="cube513_f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="also time this many replays of the step captured as a HIP graph")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-field batch")
    ap.add_argument("--no-service", action="store_true", help="skip the service sweep")
    ap.add_argument("--no-4d", action="store_true", help="skip the spatiotemporal (4-D) sweep")
    ap.add_argument("--no-progressive", action="store_true",
                    help="skip the partial recompositions (the timed step's kernels are then the last ones)")
    ap.add_argument("--no-box", action="store_true", help="skip the 400x300x250 FP32 non-uniform workload")
    ap.add_argument("--no-latency", action="store_true", help="skip the 65^3 latency measurement")
    ap.add_argument("--service-requests", type=int, default=5000,
                    help="requests in the service stream (each Poisson rate serves at most 10 s of it)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(this refactoring path runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    want_cpu = not args.no_cpu_baseline
    probe = probe_bandwidth()
    _log(f"[bench] copy probe: {probe['GBps']:.0f} GB/s")
    kept = {}
    res, u, coords, nlev, dh = run_gpu(args.workload, args.steps, args.warmup, args.graph_steps,
                                       progressive_on=not args.no_progressive, keep_output=want_cpu)
    kept[args.workload] = (u, coords, nlev, dh)
    fp32 = None
    if not args.no_fp32 and args.fp32_workload:
        r32, u32, c32, n32, d32 = run_gpu(args.fp32_workload, args.steps, args.warmup,
                                          progressive_on=not args.no_progressive, keep_output=want_cpu)
        kept[args.fp32_workload] = (u32, c32, n32, d32)
        fp32 = {k: r32[k] for k in ("workload", "value", "t_dec_ms", "t_rec_ms", "alg_GBps",
                                     "roundtrip_max_rel_err", "roofline")}
        fp32["untuned_value"] = r32["autotune"]["untuned_value"] if r32.get("autotune") else None
    box = None
    if not args.no_box:
        rb, ub, cb, nb, db = run_gpu("box400x300x250_f32", args.steps, args.warmup, progressive_on=False,
                                     keep_output=want_cpu)
        kept["box400x300x250_f32"] = (ub, cb, nb, db)
        box = {k: rb[k] for k in ("workload", "shape", "nlevels", "value", "t_dec_ms", "t_rec_ms", "alg_GBps",
                                   "roundtrip_max_rel_err", "roofline")}
        box["data"] = "non-uniform coordinates (spacing U[0.5, 1.5]), seed 1003"
    latency = None
    if not args.no_latency:
        latency = run_latency("cube65_f64")
        if want_cpu:
            from paper_2105_12764_amd.synth import WORKLOADS, make_input
            sh, sd, nu, dt, nl = WORKLOADS["cube65_f64"]
            u65, c65 = make_input(sh, sd, nonuniform=nu, dtype=dt)
            import torch
            from paper_2105_12764_amd import mgr
            d65 = mgr.decompose(torch.from_numpy(u65).cuda(), c65, nl)
            torch.cuda.synchronize()
            kept["cube65_f64"] = (u65, c65, nl, d65.cpu().numpy())
    batched = None if args.no_batch else run_batched()
    service = None if args.no_service else run_service(args.service_requests)
    spatiotemporal = None if args.no_4d else run_spatiotemporal()
    cpu, errors = None, None
    if want_cpu:
        from paper_2105_12764_amd.synth import service_requests
        cpu, errors = cpu_baseline(kept, batch_fields=0 if args.no_batch else 64,
                                   service_reqs=service_requests(args.service_requests))
        if fp32 is not None:
            fp32["errors_vs_oracle"] = errors.get(args.fp32_workload)
        if box is not None:
            box["errors_vs_oracle"] = errors.get("box400x300x250_f32")
        if latency is not None:
            latency["errors_vs_oracle"] = errors.get("cube65_f64")

    line = {
        "metric": METRIC,
        "value": round(res["value"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if res["dtype"] == "float64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{res['workload']}: {'x'.join(map(str, res['shape']))} "
                               f"{res['dtype']}, {res['nlevels']} levels, one decompose + one "
                               "recompose per step, autotuned launch shapes",
                   "shape": res["shape"], "nlevels": res["nlevels"]},
        "t_dec_ms": round(res["t_dec_ms"], 4),
        "t_rec_ms": round(res["t_rec_ms"], 4),
        "alg_GBps": round(res["alg_GBps"], 1),
        "pct_hbm_peak": round(100.0 * res["alg_GBps"] / HBM_PEAK_GBS, 2),
        "copy_probe_GBps": round(probe["GBps"], 1),
        "pct_of_copy_probe": round(100.0 * res["alg_GBps"] / probe["GBps"], 2),
        "roundtrip_max_rel_err": res["roundtrip_max_rel_err"],
        "errors_vs_oracle": errors.get(args.workload) if errors else None,
        "roofline": res["roofline"],
        "hbm_measured": res["hbm_measured"],
        "cpu_baseline": cpu,
        "kernels": res["kernels"],
        "fp32": fp32,
        "box400x300x250_f32": box,
        "latency_65": latency,
        "graph": res["graph"],
        "autotune": res["autotune"],
        "progressive": res["progressive"],
        "batched": batched,
        "service": service,
        "spatiotemporal": spatiotemporal,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
