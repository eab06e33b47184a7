"""Throughput of the fused five-equation phase-field EHD lattice Boltzmann
sweep on one MI355X.

A step is one pass of the whole method over the grid (all five LB equations
per cell, one fused Poisson update).  Default workload: the 2048 x 2048
droplet case (radius 320, W = 5) in FP32, state resident in HBM.

Prints one JSON line with the throughput (MLUPS), the HBM roofline of the
sweep kernel measured live with HIP events, and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (all 5 LB eqs/cell) at 2048² vs HBM roofline; sweep solves/hr; p99 latency"
HBM_PEAK_GBS = 8000.0
PMC_FILE = os.path.join(ROOT, "profiles", "sweep_hbm_traffic.json")
# the device code of the sweep; the launch shape is recorded beside the counts
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2501_04920_amd", "csrc", f)
                  for f in ("lbm_ehd_device.hpp", "lbm_ehd_kernels.hpp")]


def kernel_hash() -> str:
    """Hash of the sweep's device code, comments and blank lines left out."""
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f) as fh:
            src = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in src.splitlines():
            code = line.split("//", 1)[0].strip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(workload: str, waves: int, tile_rows: int):
    """HBM bytes per sweep launch from the committed rocprofv3 counter runs,
    or None if they were taken on another version of the kernel or in
    another launch shape."""
    try:
        with open(PMC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    ent = rec.get("workloads", {}).get(workload)
    if ent is None or (ent.get("waves"), ent.get("tile_rows")) != (waves, tile_rows):
        return None
    return ent.get("bytes_per_launch")


def _omp_threads(n: int):
    """Set the OpenMP thread count of the oracle's runtime (libgomp, already
    loaded by the oracle); returns the previous count."""
    import ctypes

    gomp = ctypes.CDLL("libgomp.so.1")
    prev = gomp.omp_get_max_threads()
    gomp.omp_set_num_threads(int(n))
    return prev


def cpu_baseline(params, drop, steps: int, steps_1t: int):
    """The CPU oracle (plain FP64 C, OpenMP) on the same grid, few steps, on
    the host's threads and on one thread."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # in-place streaming is a storage pattern of the GPU state, not another
    # method: the oracle steps the same lattice with its own layout
    o = oracle.Oracle({k: v for k, v in params.items() if k != "inplace"})
    o.init_droplet(drop["xc"], drop["yc"], drop["radius"], drop["noise"], drop["seed"])
    o.step(1)                       # first touch of the state
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    cells = params["nx"] * params["ny"]
    out = {"value": cells * steps / dt / 1e6, "unit": "MLUPS", "cores": threads,
           "kind": "oracle",
           "sample": "%dx%d droplet case, %d steps after 1 warm-up step, FP64, %.1f s"
                     % (params["nx"], params["ny"], steps, dt)}
    if steps_1t > 0:
        prev = _omp_threads(1)
        t0 = time.perf_counter()
        o.step(steps_1t)
        dt1 = time.perf_counter() - t0
        _omp_threads(prev)
        out["one_core"] = {"value": cells * steps_1t / dt1 / 1e6, "unit": "MLUPS", "cores": 1,
                           "sample": "%d further steps on one thread, %.1f s" % (steps_1t, dt1)}
    return out


def copy_calibration(gib: float, reps: int, width: int):
    """A plain device-to-device copy of known size with the library's copy
    kernel (same buffer instructions as the sweep): its bandwidth is the
    attainable HBM rate, and its FETCH_SIZE / WRITE_SIZE counters calibrate
    the counter runs of the sweep."""
    import torch

    from paper_2501_04920_amd import lbm_ehd

    n = int(gib * (1 << 30)) // 16 * 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()

    def run():
        lbm_ehd.lbm_ehd_stream_copy(a.data_ptr(), b.data_ptr(), 4 * n, st.cuda_stream, width)

    for _ in range(3):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        run()
    e1.record(st)
    torch.cuda.synchronize()
    assert bool((b == 1).all())
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * 4 * n
    print(json.dumps({"copy_bytes_per_launch": nbytes, "read_bytes": 4 * n,
                      "write_bytes": 4 * n, "width": width, "ms": round(ms, 5),
                      "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1)}), flush=True)


def summarize_pmc(paths, workload: str, waves: int, tile_rows: int):
    """Turn four rocprofv3 --pmc CSVs (sweep FETCH_SIZE, sweep WRITE_SIZE, copy
    FETCH_SIZE, copy WRITE_SIZE; KiB per dispatch) into HBM bytes per sweep
    launch, each counter scaled by what it reads for the copy kernel of known
    size, and record them in the traffic file with the kernel source hash."""
    import csv

    def mean(path, kname, counter):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                if kname in r["Kernel_Name"] and r["Counter_Name"] == counter]
        if not vals:
            raise SystemExit("no %s rows for %s in %s" % (counter, kname, path))
        return sum(vals) / len(vals) * 1024.0

    sf, sw, cf, cw = paths
    copy_read = copy_write = float(1 << 30)   # --copy-gib 1
    kf = copy_read / mean(cf, "k_copy<4>", "FETCH_SIZE")
    kw = copy_write / mean(cw, "k_copy<4>", "WRITE_SIZE")
    fetch = mean(sf, "k_sweep", "FETCH_SIZE") * kf
    write = mean(sw, "k_sweep", "WRITE_SIZE") * kw
    try:
        rec = json.load(open(PMC_FILE))
    except (OSError, ValueError):
        rec = {}
    if rec.get("kernel_hash") != kernel_hash():
        rec = {"kernel_hash": kernel_hash(), "workloads": {}}
    rec["workloads"][workload] = {
        "waves": waves, "tile_rows": tile_rows,
        "fetch_bytes": round(fetch), "write_bytes": round(write),
        "bytes_per_launch": round(fetch + write),
        "fetch_scale": round(kf, 4), "write_scale": round(kw, 4)}
    with open(PMC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec["workloads"][workload]))


def _alone_D(m, precision, steps):
    """Deformation of one member run alone (its own launches) and the wall
    time of that run."""
    import torch

    from paper_2501_04920_amd import lbm_ehd

    p, d = m["params"], m["droplet"]
    sim = lbm_ehd.Simulation(dict(p, precision=precision), device="cuda:0")
    sim.init_droplet(d["xc"], d["yc"], d["radius"], d["noise"], d["seed"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    dt = time.perf_counter() - t0
    D = sim.diagnostics()["D"]
    sim.close()
    return D, dt


def bench_batched(args):
    """64 droplets of uneven sizes (128^2-1024^2) in one batch, FP16 storage,
    autotuned launch shape, 10k steps each: sweep solves per hour.  Baseline:
    the same 64 runs one after the other in plain FP32 (timed on a sample of
    steps and scaled); error: D of sampled members against the member run
    alone in plain FP32."""
    import torch

    from paper_2501_04920_amd import lbm_ehd, workloads

    members = workloads.config4_members(count=args.members, steps=args.batch_steps)
    steps = args.batch_steps
    sims = []
    for m in members:
        p, d = m["params"], m["droplet"]
        s = lbm_ehd.Simulation(dict(p, precision="fp16"), device="cuda:0")
        s.init_droplet(d["xc"], d["yc"], d["radius"], d["noise"], d["seed"])
        sims.append(s)
    torch.cuda.synchronize()
    b = lbm_ehd.Batch(sims)
    t0 = time.perf_counter()
    waves, rows, taken = b.autotune(10)
    b.run(steps - taken)
    b.synchronize()
    wall = time.perf_counter() - t0
    cells = sum(m["params"]["nx"] * m["params"]["ny"] for m in members)
    D_batch = [s.diagnostics()["D"] for s in sims]
    b.close()
    for s in sims:
        s.close()
    print("batch of %d done in %.1f s" % (len(members), wall), file=sys.stderr, flush=True)
    # baseline: each member alone in FP32, timed over a few steps, scaled
    seq = 0.0
    for m in members:
        _, dt = _alone_D(m, "fp32", args.seq_steps)
        seq += dt * steps / args.seq_steps
    # error of the FP16 batch against FP32 alone, on every 8th member
    errs = []
    for k in range(0, len(members), 8):
        D32, _ = _alone_D(members[k], "fp32", steps)
        errs.append(abs(D_batch[k] - D32))
    line = {
        "metric": "sweep solves/hr", "value": round(len(members) * 3600.0 / wall, 1),
        "unit": "solves/hr", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": round(wall / steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched-%d-droplets-128-1024" % len(members),
                   "cells": cells, "storage": "fp16", "waves": waves, "tile_rows": rows,
                   "autotune_steps": taken},
        "aggregate_glups": round(cells * steps / wall / 1e9, 3),
        "sequential_fp32_s": round(seq, 2), "speedup_vs_sequential_fp32": round(seq / wall, 2),
        "D_err_vs_fp32_alone_max": max(errs), "D_err_members": list(range(0, len(members), 8)),
    }
    print(json.dumps(line), flush=True)


def batched_summary(members=64, steps=10000):
    """The batched form as timed in the default run: the 64 droplets of
    128^2-1024^2 (seeded Latin hypercube), FP16 storage, autotuned launch
    shape, `steps` steps each, from created members to the last step."""
    import torch

    from paper_2501_04920_amd import lbm_ehd, workloads

    ms = workloads.config4_members(count=members, steps=steps)
    sims = []
    for m in ms:
        p, d = m["params"], m["droplet"]
        s = lbm_ehd.Simulation(dict(p, precision="fp16"), device="cuda:0")
        s.init_droplet(d["xc"], d["yc"], d["radius"], d["noise"], d["seed"])
        sims.append(s)
    torch.cuda.synchronize()
    b = lbm_ehd.Batch(sims)
    t0 = time.perf_counter()
    waves, rows, taken = b.autotune(10)
    b.run(steps - taken)
    b.synchronize()
    wall = time.perf_counter() - t0
    cells = sum(m["params"]["nx"] * m["params"]["ny"] for m in ms)
    bad = sum(s.diagnostics()["nonfinite"] for s in sims)
    b.close()
    for s in sims:
        s.close()
    return {"metric": "sweep solves/hr", "value": round(len(ms) * 3600.0 / wall, 1),
            "unit": "solves/hr", "wall_s": round(wall, 3),
            "workload": "batched-%d-droplets-128-1024-%dsteps" % (len(ms), steps),
            "storage": "fp16", "cells": cells, "aggregate_glups": round(cells * steps / wall / 1e9, 3),
            "waves": waves, "tile_rows": rows, "autotune_steps": taken, "nonfinite": int(bad)}


def serving_summary(requests=64, rate=20.0, budget_gib=64.0, block=256):
    """The serving form as timed in the default run: the first `requests`
    requests of the seeded trace (Poisson arrivals at `rate` per second,
    grids 64^2-2048^2, 2k-50k steps), replayed in real time through the
    request server (HBM admission, continuous batching, FP16 storage)."""
    import numpy as np

    from paper_2501_04920_amd import lbm_ehd, workloads

    trace = workloads.config5_trace(count=requests, rate=rate)
    done, span, maxrun = _serve_trace(trace, int(budget_gib * (1 << 30)), block)
    lat = np.array([v[0] for v in done.values()])
    work = sum(v[1] for v in done.values())
    failed = sum(1 for v in done.values() if v[2] != lbm_ehd.REQ_DONE)
    return {"metric": "p99 latency", "value": round(float(np.percentile(lat, 99)), 3), "unit": "s",
            "p50_s": round(float(np.percentile(lat, 50)), 3),
            "throughput_req_per_s": round(len(trace) / span, 3),
            "aggregate_glups": round(work / span / 1e9, 3), "makespan_s": round(span, 2),
            "workload": "serving-%d-requests-64-2048-rate%g" % (len(trace), rate),
            "storage": "fp16", "hbm_budget_gib": budget_gib, "max_running": maxrun,
            "failed": failed}


ENCLOSURE_STUDY = (
    [("eps_r", e) for e in (0.5, 1.0, 2.0, 5.0, 10.0, 50.0)]
    + [("mu_r", m) for m in (0.25, 0.5, 1.0, 2.0, 10.0)]
    + [("d_mm", 0.5), ("d_mm", 1.0), ("d_mm", 4.0), ("kv", 0.5), ("kv", 0.25)])


def bench_enclosure(args):
    """The paper's parameter study of Sec. 6 as one batched job: the enclosure
    (256^2, side walls, Sec. 6 defaults) at each point of an eps_r scan, a
    mu_r scan and five further conduction numbers W0 (gap d and voltage),
    advanced to the steady droplet (160 000 steps) in one launch per step:
    study solves per hour, and the steady deformation factor and charge
    observables of every point."""
    import numpy as np
    import torch

    from paper_2501_04920_amd import lbm_ehd, workloads

    cases = [workloads.enclosure(args.enclosure_n, **{k: v}) for k, v in ENCLOSURE_STUDY]
    steps = args.study_steps or cases[0]["steps"]
    # each point is set up and pre-solved on a stream of its own (default
    # priority): its 2 x 30 000 small g-only launches overlap with the others'
    sims, streams = [], []
    t_init = time.perf_counter()
    for c in cases:
        p, d = c["params"], c["droplet"]
        st = torch.cuda.Stream(device="cuda:0")
        with torch.cuda.stream(st):
            s = lbm_ehd.Simulation(dict(p, precision=args.precision), device="cuda:0")
            s.init_droplet(d["xc"], d["yc"], d["radius"], d["noise"], d["seed"],
                           presolve=c["presolve"])
        sims.append(s)
        streams.append(st)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t_init
    b = lbm_ehd.Batch(sims)
    t0 = time.perf_counter()
    waves, rows, taken = b.autotune(10)
    left, done = steps - taken, taken
    while left > 0:
        k = min(left, 40000)
        b.run(k)
        b.synchronize()
        left -= k
        done += k
        print("enclosure study: %d of %d steps (%.1f s)" % (done, steps, time.perf_counter() - t0),
              file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    cells = sum(c["params"]["nx"] * c["params"]["ny"] for c in cases)
    D = [s.diagnostics()["D"] for s in sims]
    bad = sum(s.diagnostics()["nonfinite"] for s in sims)
    # charge observables of Sec. 6, in units of q c0: rows from the anode to
    # where rho_e at column 8 falls to 1/e of its wall value (heterocharge
    # layer), and the mean |rho_e| within half the droplet radius (zero in
    # the ohmic state's electroneutral core)
    layer, core = [], []
    for c, s in zip(cases, sims):
        p, d = c["params"], c["droplet"]
        r = s.fields(("rhoe",))["rhoe"] / (p["q"] * p["c0"])
        col = r[:, 8]
        layer.append(int(np.argmax(np.abs(col) < abs(col[0]) / np.e)))
        yy, xx = np.mgrid[0:p["ny"], 0:p["nx"]]
        core.append(float(np.abs(r[np.hypot(xx - d["xc"], yy - d["yc"]) < d["radius"] / 2]).mean()))
    b.close()
    for s in sims:
        s.close()
    line = {
        "metric": "sweep solves/hr", "value": round(len(cases) * 3600.0 / wall, 1),
        "unit": "solves/hr", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": round(wall / steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32f64": "f64", "fp16": "f32",
                  "bf16": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "enclosure-study-%d-points-%d" % (len(cases), args.enclosure_n),
                   "cells": cells, "storage": args.precision, "waves": waves,
                   "tile_rows": rows, "autotune_steps": taken,
                   "presolve_sweeps": cases[0]["presolve"]},
        "aggregate_glups": round(cells * steps / wall / 1e9, 3),
        "init_and_presolve_s": round(t_init, 2),
        "steady_D": {"%s=%g" % kv: round(x, 5) for kv, x in zip(ENCLOSURE_STUDY, D)},
        "heterocharge_rows": {"%s=%g" % kv: x for kv, x in zip(ENCLOSURE_STUDY, layer)},
        "core_charge": {"%s=%g" % kv: float("%.3g" % x) for kv, x in zip(ENCLOSURE_STUDY, core)},
        "nonfinite": int(bad),
    }
    print(json.dumps(line), flush=True)


def _serve_trace(trace, budget, block, precision="fp16", inplace=0):
    """Replay a trace in real time through the request server; returns
    per-request (latency s, cells x steps) and the makespan."""
    from paper_2501_04920_amd import lbm_ehd

    srv = lbm_ehd.Server(budget, block_steps=block)
    pending = sorted(trace, key=lambda r: r["arrival"])
    ids = {}
    done = {}
    t0 = time.perf_counter()
    k = 0
    max_running = 0
    while len(done) < len(trace):
        now = time.perf_counter() - t0
        while k < len(pending) and pending[k]["arrival"] <= now:
            r = pending[k]
            d = r["droplet"]
            rid = srv.submit(dict(r["params"], precision=precision, inplace=inplace), d["xc"],
                             d["yc"], d["radius"], d["noise"], d["seed"], r["steps"])
            ids[rid] = r
            k += 1
        running, queued = srv.advance()
        max_running = max(max_running, running)
        for rid in list(ids):
            inf = srv.info(rid)
            if inf["state"] >= lbm_ehd.REQ_DONE:
                r = ids.pop(rid)
                done[r["name"]] = (inf["t_done"] - inf["t_submit"],
                                   r["params"]["nx"] * r["params"]["ny"] * r["steps"],
                                   inf["state"], inf["diag"]["D"])
                srv.release(rid)
                if len(done) % 32 == 0:
                    print("served %d/%d requests" % (len(done), len(trace)), file=sys.stderr,
                          flush=True)
        if running == 0 and queued == 0 and k < len(pending):
            time.sleep(max(0.0, pending[k]["arrival"] - (time.perf_counter() - t0)))
    makespan = time.perf_counter() - t0
    srv.close()
    return done, makespan, max_running


def bench_serving(args):
    """Poisson arrivals (20 per second, seeded) of droplet requests 64^2-2048^2
    with 2k-50k steps, served with HBM-footprint admission and continuous
    batching (FP16 storage by default): p50 / p99 completion latency and
    throughput; then the same requests at a rate giving ~70 % load."""
    import numpy as np

    from paper_2501_04920_amd import lbm_ehd, workloads

    trace = workloads.config5_trace(count=args.requests, rate=args.rate)
    budget = int(args.budget_gib * (1 << 30))
    prec, ip = args.serve_precision, int(args.serve_inplace)
    done, span, maxrun = _serve_trace(trace, budget, args.block, prec, ip)
    lat = np.array([v[0] for v in done.values()])
    work = sum(v[1] for v in done.values())
    glups = work / span / 1e9
    failed = sum(1 for v in done.values() if v[2] != lbm_ehd.REQ_DONE)
    # error of the served FP16 results against the same request run alone in
    # plain FP32, on every 32nd request
    errs = []
    for r in trace[::32]:
        D32, _ = _alone_D(r, "fp32", r["steps"])
        errs.append(abs(done[r["name"]][3] - D32))
    print("checked %d served results against FP32 alone" % len(errs), file=sys.stderr, flush=True)
    # a sub-saturation trace: the same requests, arrival rate for ~70 % load
    mean_work = work / len(trace)
    rate_sub = 0.7 * glups * 1e9 / mean_work
    sub = None
    if args.sub:
        trace2 = workloads.config5_trace(count=args.requests, rate=rate_sub)
        done2, span2, _ = _serve_trace(trace2, budget, args.block, prec, ip)
        lat2 = np.array([v[0] for v in done2.values()])
        sub = {"rate_per_s": round(rate_sub, 3), "p50_s": round(float(np.percentile(lat2, 50)), 3),
               "p99_s": round(float(np.percentile(lat2, 99)), 3),
               "makespan_s": round(span2, 2)}
    line = {
        "metric": "p99 latency", "value": round(float(np.percentile(lat, 99)), 3), "unit": "s",
        "n_gpus": 1, "steps": int(sum(r["steps"] for r in trace)), "warmup": 0,
        "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving-%d-requests-64-2048-rate%g" % (len(trace), args.rate)
                   + ("-inplace" if ip else ""),
                   "storage": prec, "inplace": ip, "hbm_budget_gib": args.budget_gib,
                   "block_steps": args.block},
        "p50_s": round(float(np.percentile(lat, 50)), 3),
        "throughput_req_per_s": round(len(trace) / span, 3), "aggregate_glups": round(glups, 3),
        "makespan_s": round(span, 2), "max_running": maxrun, "failed": failed,
        "D_err_vs_fp32_alone_max": max(errs), "D_err_requests": len(errs),
        "sub_saturation": sub,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp32",
                    choices=["fp64", "fp32", "fp32f64", "fp16", "bf16"])
    ap.add_argument("--n", type=int, default=2048,
                    help="grid n x n (radius n / 6.4, W = 5; 128: the 128^2 parity case, W = 4)")
    ap.add_argument("--cpu-steps", type=int, default=64)
    ap.add_argument("--cpu-steps-1t", type=int, default=4,
                    help="further oracle steps on one thread (0: skip)")
    ap.add_argument("--inplace", action="store_true",
                    help="in-place streaming (one population buffer, AA pattern)")
    ap.add_argument("--ion-q9", action="store_true",
                    help="the ion LBEs on D2Q9 instead of D2Q5")
    ap.add_argument("--no-forms", action="store_true",
                    help="leave out the batched and serving sub-objects of the default line")
    ap.add_argument("--form-requests", type=int, default=64,
                    help="requests of the serving sub-object (first of the seeded trace)")
    ap.add_argument("--waves", type=int, default=0,
                    help="wavefronts per sweep workgroup (1, 2, 4, 8; 0 = library default)")
    ap.add_argument("--tile-rows", type=int, default=0,
                    help="rows per sweep band (0 = library default)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="only run the copy-kernel calibration of this size")
    ap.add_argument("--copy-width", type=int, default=4, choices=[4, 16])
    ap.add_argument("--summarize-pmc", nargs=4, metavar="CSV",
                    help="sweep FETCH, sweep WRITE, copy FETCH, copy WRITE counter files")
    ap.add_argument("--form", default="single",
                    choices=["single", "batched", "serving", "enclosure"],
                    help="single simulation (default), batched sweep, request server, or "
                         "the paper's enclosure parameter study as one batch")
    ap.add_argument("--enclosure-n", type=int, default=256)
    ap.add_argument("--study-steps", type=int, default=0,
                    help="steps of the enclosure study (0: to the steady droplet, 160 000)")
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=10000)
    ap.add_argument("--seq-steps", type=int, default=100)
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--serve-precision", default="fp16", choices=["fp16", "bf16", "fp32", "fp64"],
                    help="storage of the served requests (--form serving)")
    ap.add_argument("--serve-inplace", action="store_true",
                    help="serve with in-place streaming (one population buffer per request)")
    ap.add_argument("--sub", type=int, default=1, help="also run the ~70 %% load trace")
    args = ap.parse_args()
    if args.summarize_pmc:
        if not (args.waves and args.tile_rows):
            sys.exit("--summarize-pmc needs the --waves and --tile-rows of the counter runs")
        summarize_pmc(args.summarize_pmc, "droplet-%d-%s" % (args.n, args.precision),
                      args.waves, args.tile_rows)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.copy_gib > 0:
        copy_calibration(args.copy_gib, max(args.steps, 1), args.copy_width)
        return
    if args.form == "batched":
        bench_batched(args)
        return
    if args.form == "serving":
        bench_serving(args)
        return
    if args.form == "enclosure":
        bench_enclosure(args)
        return

    import torch

    from paper_2501_04920_amd import lbm_ehd, workloads

    n = args.n
    if n == 2048:
        cfg = workloads.config3()
    elif n == 128:
        cfg = workloads.config1()       # the 128^2 parity case (W = 4)
    else:
        cfg = workloads.scaled(n, W=5.0)
    params, drop = cfg["params"], cfg["droplet"]
    workload = "droplet-%d-%s" % (n, args.precision) + ("-inplace" if args.inplace else "") \
        + ("-ions-d2q9" if args.ion_q9 else "")
    if args.inplace:
        params = dict(params, inplace=1)
    if args.ion_q9:
        params = dict(params, ion_q9=1)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sim = lbm_ehd.Simulation(dict(params, precision=args.precision), device=dev)
    sim.init_droplet(drop["xc"], drop["yc"], drop["radius"], drop["noise"], drop["seed"])
    if args.waves or args.tile_rows:
        w0, r0 = sim.launch
        sim.set_launch(args.waves or w0, args.tile_rows or r0)
    waves, tile_rows = sim.launch
    stream = sim.stream
    sim.step(args.warmup)
    sim.synchronize()
    torch.cuda.synchronize()

    # per-launch duration of the sweep kernel: one launch per step, the K
    # launches back to back between two events on the stream the library
    # launches on (events between the launches would add their own gaps to
    # the timed region)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    sim.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = e0.elapsed_time(e1) / args.steps

    cells = params["nx"] * params["ny"]
    mlups = cells * args.steps / wall / 1e6
    # algorithmic bytes per lattice update: the 33 populations read and
    # written once in the storage type, plus (phi u)(t-1) read and written
    # (FP32; FP64 in the FP64 forms); the layout's own count (FP64 rest
    # populations, reference lines) is reported beside it
    s_bytes = {"fp64": 8, "fp32": 4, "fp32f64": 4, "fp16": 2, "bf16": 2}[args.precision]
    j_bytes = 8 if args.precision in ("fp64", "fp32f64") else 4
    npop = 41 if args.ion_q9 else 33    # the ions on D2Q9 add 2 x 4 diagonals
    alg = 2 * npop * s_bytes + 2 * 2 * j_bytes
    design = lbm_ehd.lbm_ehd_bytes_per_lup(args.precision) + (2 * 8 * s_bytes if args.ion_q9 else 0)
    achieved = alg * cells / (kern_ms * 1e-3) / 1e9
    diag = sim.diagnostics()
    traffic = measured_traffic(workload, waves, tile_rows)
    line = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32f64": "f64", "fp16": "f32",
                  "bf16": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": workload, "nx": params["nx"], "ny": params["ny"],
                   "radius": drop["radius"], "W": params["W"], "storage": args.precision,
                   "poisson_sweeps_per_step": 1 + params["poisson_iters"],
                   "bytes_per_lup": alg, "layout_bytes_per_lup": design, "waves": waves,
                   "tile_rows": tile_rows},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     # in place a step is the edge pre-pass and the sweep
                     "kernel": "k_aa_hood + k_sweep_aa" if args.inplace else "k_sweep_batch",
                     "kernel_ms": round(kern_ms, 5),
                     "layout_frac": round(design * cells / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "check": {"sum_phi": diag["sum_phi"], "nonfinite": diag["nonfinite"]},
    }
    sim.close()
    print("single: %.1f MLUPS, kernel %.4f ms" % (mlups, kern_ms), file=sys.stderr, flush=True)
    if not args.no_forms:
        line["batched"] = batched_summary()
        print("batched: %s solves/hr" % line["batched"]["value"], file=sys.stderr, flush=True)
        line["serving"] = serving_summary(requests=args.form_requests)
        print("serving: p99 %s s" % line["serving"]["value"], file=sys.stderr, flush=True)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(params, drop, args.cpu_steps, args.cpu_steps_1t)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
