"""Benchmark: particle binning throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload hotspot|gmm|uniform|nd3|batched|served|insitu|multi]

hotspot / gmm / uniform: one step = one bin_particles call over the whole
particle set (init, bin, finalize), inputs resident in HBM.  Prints one JSON
line with throughput (Gparticles/s), the roofline position of the dominant
kernel measured with HIP events recorded by the library around that kernel,
and the CPU oracle timed on a bounded sample of the same workload.

batched: 256 independent requests (particle counts log-uniform in [1e3, 1e7],
square grids of side 32..1024, 1-4 attributes, random op sets); one step =
the whole batch, as a captured graph, as one batched call, and as 256
one-at-a-time calls, all timed on the same stream.

served: Poisson arrival streams of requests drawn from the batched set,
served by the continuous-batching server (64 GB budget) and, for
comparison, one request at a time; p50/p99 latency and throughput per rate.

multi: nine coordinate systems over one ten-column table (16M particles,
256x256 grids), one fused call against nine separate calls.

insitu: a synthetic solver and the binning of its particles on one GPU:
solver alone, lockstep zero-copy binning, and the asynchronous deep-copy
mode on a second stream (solver slowdown, apparent in situ time).
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gparticles/s binned + % HBM roofline; p50/p99 request latency (served)"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the sources that decide what a single call launches: the
    device code, its headers and the planner (host-side batching, serving,
    tuning and API files, and their host-only headers, are left out)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2310_02926_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if (f.endswith((".hip", ".h")) and f not in ("internal.h", "server_admit.h", "batch_classes.h")) or f == "plan.cpp":
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def make_workload(name: str, scale: int):
    from paper_2310_02926_amd import synth
    if name == "hotspot":
        n = (1 << 27) >> scale
        return synth.hotspot_f32(n=n, seed=0, side=2048), {
            "workload": "hotspot_128M_2048sq", "n": n, "grid": "2048x2048", "attrs": "1 x f32 (mass ~ lognormal(0,2))",
            "coords": "2 x f32", "hot": "90% of particles in 1% of bins", "ops": "count,sum,min,max,avg"}
    if name == "gmm":
        n = (1 << 24) >> scale
        return synth.gmm_f32(n=n, seed=0, nx=1024, ny=1024, k=4), {
            "workload": "gmm_16M_1024sq_k4", "n": n, "grid": "1024x1024", "attrs": "4 x f32", "coords": "2 x f32",
            "ops": "count,sum,min,max,avg"}
    if name == "uniform":
        n = 65536 >> scale
        return synth.uniform_f64(n, seed=0), {"workload": "uniform_64K_64sq_f64", "n": n, "grid": "64x64",
                                               "attrs": "1 x f64", "coords": "2 x f64", "ops": "count,sum,min,max,avg"}
    if name == "nd3":
        n = (1 << 26) >> scale
        return synth.halos3d_f32(n=n, seed=0, side=128), {
            "workload": "halos3d_64M_128cube", "n": n, "grid": "128x128x128 (axes x, y, z)",
            "attrs": "1 x f32 (mass ~ lognormal(0,1))", "coords": "3 x f32",
            "clustered": "80% of particles in 64 Gaussian halos", "ops": "count,sum,min,max,avg"}
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(ws):
    naxes = len(ws.meta["nd"][0]) if "nd" in ws.meta else 2
    ins = sum(c.itemsize * c.size for c in ws.coords[:naxes]) + sum(a.itemsize * a.size for a in ws.attrs)
    nb = ws.nx * ws.ny
    a64 = bool(ws.attrs) and ws.attrs[0].dtype == np.float64
    per_attr = (8 + 8 + 8 + 8) if a64 else (8 + 4 + 4 + 8)  # sum, min, max, avg (default precision)
    outs = nb * (4 + per_attr * len(ws.attrs))
    return ins, outs


def host_cpu():
    """CPU model and logical CPU count of the host the benchmark runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def _oracle_call(ws, lo, hi):
    from oracle import binning_oracle as orc
    if "nd" in ws.meta:
        axes, bounds, dims = ws.meta["nd"]
        return orc.bin_particles_nd([c[lo:hi] for c in ws.coords], [a[lo:hi] for a in ws.attrs], axes, bounds, dims)
    return orc.bin_particles([c[lo:hi] for c in ws.coords], [a[lo:hi] for a in ws.attrs], ws.axes, ws.bounds,
                             ws.nx, ws.ny)


def cpu_baseline_1core(ws, target_s: float = 12.0):
    """The oracle as it stands, one NumPy thread, on a prefix sample of the
    same particles: grow the sample until one run takes about target_s
    seconds (or the whole workload is used)."""
    n = ws.n
    m = min(n, 1 << 20)
    while True:
        t0 = time.perf_counter()
        _oracle_call(ws, 0, m)
        dt = time.perf_counter() - t0
        if dt >= 0.5 * target_s or m >= n:
            break
        m = int(min(n, m * max(2.0, min(16.0, target_s / max(dt, 1e-3)))))
    return {"value": round(m / dt / 1e9, 6), "unit": "Gparticles/s", "cores": 1, "kind": "oracle",
            "sample": f"first {m} of {n} particles of the same workload (same grid, ops), one NumPy thread, "
                      f"{dt:.1f} s"}


_NCORE = {}


def _ncore_worker(w):
    """Oracle on slice w of the sample; writes count, sum, |a| sum, min and
    max into this worker's rows of the shared result arrays."""
    ws, m, W, sh = _NCORE["ws"], _NCORE["m"], _NCORE["W"], _NCORE["sh"]
    lo, hi = w * m // W, (w + 1) * m // W
    r = _oracle_call(ws, lo, hi)
    sh["count"][w] = r["count"].ravel()
    for j in range(len(ws.attrs)):
        for key in ("sum", "abs_sum", "min", "max"):
            sh[key][w, j] = r[key][j].ravel()
    return r["inside"]


def cpu_baseline_ncore(ws, m: int, workers: int):
    """The same oracle on N processes: the first m particles split into N
    slices, each binned by the oracle in its own process (forked, results
    written to shared memory), the partial grids combined by the oracle's
    merge law (counts and sums add, min of mins, max of maxes)."""
    import multiprocessing as mp
    from multiprocessing import shared_memory
    from oracle import binning_oracle as orc
    nb = int(np.prod(ws.meta["nd"][2])) if "nd" in ws.meta else ws.nx * ws.ny
    k = len(ws.attrs)
    W = workers
    blocks, sh = [], {}
    for key, shape in (("count", (W, nb)), ("sum", (W, k, nb)), ("abs_sum", (W, k, nb)), ("min", (W, k, nb)),
                       ("max", (W, k, nb))):
        dt = np.int64 if key == "count" else np.float64
        shm = shared_memory.SharedMemory(create=True, size=max(8, int(np.prod(shape)) * 8))
        blocks.append(shm)
        sh[key] = np.ndarray(shape, dtype=dt, buffer=shm.buf)
    _NCORE.update(ws=ws, m=m, W=W, sh=sh)
    try:
        t0 = time.perf_counter()
        with mp.get_context("fork").Pool(W) as pool:
            inside = pool.map(_ncore_worker, range(W), chunksize=1)
        parts = [{"count": sh["count"][w], "inside": inside[w],
                  **{key: [sh[key][w, j] for j in range(k)] for key in ("sum", "abs_sum", "min", "max")}}
                 for w in range(W)]
        orc.merge(parts)
        dt = time.perf_counter() - t0
    finally:
        _NCORE.clear()
        for shm in blocks:
            shm.close()
            shm.unlink()
    return {"value": round(m / dt / 1e9, 6), "unit": "Gparticles/s", "cores": W, "kind": "oracle",
            "sample": f"first {m} of {ws.n} particles of the same workload in {W} slices, one process per "
                      f"slice, partial grids combined by the merge law, {dt:.1f} s"}


def kernel_algorithmic_bytes(name: str, ws) -> int:
    """Bytes per launch that the binning definition itself requires of this
    kernel: the particle columns it must read, or the result grid it must
    write.  Intermediate records, counts and partials are not counted."""
    ins, outs = algorithmic_bytes(ws)
    if name == "fold_axes_kernel":  # axes 1 and 2 in, the composite column out
        return 3 * ws.coords[1].itemsize * ws.n
    if name in ("part_scatter_kernel", "bin_global_kernel", "bin_lds_kernel"):
        if "nd" in ws.meta:  # axis 0, the composite column and the attributes
            return ins - ws.coords[2].itemsize * ws.n
        return ins
    if name in ("part_bin_kernel", "part_merge_kernel", "lds_merge_kernel", "bin_finalize_kernel"):
        return outs
    return 0


def load_traffic(kernel_hash: str, workload: str):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(workload)
    except Exception:
        return None
    if not rec or rec.get("kernel_hash") != kernel_hash:
        return None
    return rec


def _gen_instance(spec):
    from paper_2310_02926_amd import synth
    return synth.instance(spec)


def batch_workloads(count: int, seed: int, scale: int, workers: int = 16):
    """The batched request set (synth.batch_specs), generated by a pool of
    processes forked before any GPU use."""
    import multiprocessing as mp
    from paper_2310_02926_amd import synth
    specs = synth.batch_specs(count, seed=seed, n_hi=1e7 / (1 << scale))
    workers = max(1, min(workers, os.cpu_count() or 1))
    with mp.get_context("fork").Pool(workers) as pool:
        wss = pool.map(_gen_instance, specs, chunksize=1)
    return specs, wss


def _upload(wss, dev):
    import torch
    from paper_2310_02926_amd import binding as B
    reqs = []
    for ws in wss:
        coords = [torch.from_numpy(c).to(dev) for c in ws.coords]
        attrs = [torch.from_numpy(a).to(dev) for a in ws.attrs]
        out = B.alloc_outputs(attrs, ws.nx, ws.ny, ws.ops, dev)
        reqs.append(dict(coords=coords, attrs=attrs, n=ws.n, axes=ws.axes, bounds=ws.bounds, nx=ws.nx, ny=ws.ny,
                         ops=ws.ops, out=out))
    return reqs


def _timed(stream, steps, fn):
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        fn()
    ev1.record(stream)
    stream.synchronize()
    return ev0.elapsed_time(ev1) / steps


def _same_results(reqs, snap):
    """Counts equal and sums within 1e-9 relative of a snapshot."""
    import torch
    for r, s in zip(reqs, snap):
        for key, val in s.items():
            cur = r["out"][key]
            if key == "count":
                if not torch.equal(cur, val):
                    return False
            else:
                for x, y in zip(cur, val):
                    if not torch.allclose(x, y, rtol=1e-9, atol=1e-9, equal_nan=True):
                        return False
    return True


def _snapshot(reqs):
    snap = []
    for r in reqs:
        d = {}
        for key, val in r["out"].items():
            d[key] = val.clone() if key == "count" else [t.clone() for t in val]
        snap.append(d)
    return snap


def run_batched(args):
    t0 = time.time()
    specs, wss = batch_workloads(256, 0, args.scale)
    total_n = sum(ws.n for ws in wss)
    in_bytes = sum(sum(c.nbytes for c in ws.coords) + sum(a.nbytes for a in ws.attrs) for ws in wss)
    log(f"generated 256 batched instances, {total_n} particles, {in_bytes / 1e9:.2f} GB in {time.time() - t0:.1f}s")
    import torch
    from paper_2310_02926_amd import binding as B
    dev = torch.device("cuda:0")
    reqs = _upload(wss, dev)
    del wss
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    t0 = time.time()
    if not args.no_autotune:
        B.bin_autotune(reqs)
        log(f"autotune {time.time() - t0:.1f}s")
    batch = B.Batch(reqs)

    def one_at_a_time():
        for i in range(batch.n):
            batch.launch_one(i, stream)

    # reference results: one request at a time
    one_at_a_time()
    stream.synchronize()
    ref = _snapshot(reqs)
    for _ in range(args.warmup):
        batch.launch(stream)
    stream.synchronize()
    ok_batched = _same_results(reqs, ref)
    graph = B.BinGraph(reqs)
    for _ in range(args.warmup):
        graph.launch(stream)
    stream.synchronize()
    ok_graph = _same_results(reqs, ref)
    for _ in range(args.warmup):
        one_at_a_time()
    ms_one = _timed(stream, args.steps, one_at_a_time)
    ms_batch = _timed(stream, args.steps, lambda: batch.launch(stream))
    ms_graph = _timed(stream, args.steps, lambda: graph.launch(stream))
    graph.destroy()
    log(f"one-at-a-time {ms_one:.3f} ms, batched {ms_batch:.3f} ms, graph {ms_graph:.3f} ms per batch")
    gp = lambda ms: round(total_n / (ms / 1e3) / 1e9, 3)
    best = min(ms_graph, ms_batch)
    rec = {
        "metric": METRIC, "value": gp(best), "unit": "Gparticles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(best, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched_256_requests", "n_total": total_n, "input_bytes": in_bytes,
                   "requests": "n log-uniform [1e3,1e7], square side in {32..1024}, 1-4 f32 attrs, random ops",
                   "tuning": ("the tuning cache or planner defaults" if args.no_autotune
                              else "bin_autotune over the request shapes")},
        "batched": {"graph_ms": round(ms_graph, 4), "batched_call_ms": round(ms_batch, 4),
                    "one_at_a_time_ms": round(ms_one, 4), "graph_Gps": gp(ms_graph),
                    "batched_call_Gps": gp(ms_batch), "one_at_a_time_Gps": gp(ms_one),
                    "speedup_vs_one_at_a_time": round(ms_one / best, 3),
                    "results_equal_one_at_a_time": bool(ok_batched and ok_graph),
                    "input_GBs": round(in_bytes / (best / 1e3) / 1e9, 1)},
        "cpu_baseline": None,
    }
    print(json.dumps(rec), flush=True)


def _percentiles(lat_ms):
    a = np.sort(np.asarray(lat_ms))
    return round(float(np.percentile(a, 50)), 3), round(float(np.percentile(a, 99)), 3)


def run_served(args):
    import threading
    t0 = time.time()
    specs, wss = batch_workloads(256, 0, args.scale)
    log(f"generated request pool in {time.time() - t0:.1f}s")
    import torch
    from paper_2310_02926_amd import binding as B
    from paper_2310_02926_amd import synth
    dev = torch.device("cuda:0")
    pool = _upload(wss, dev)
    del wss
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    B.bin_autotune(pool)
    batch = B.Batch(pool)
    # the configured sweep (100-5000 req/s), then past what one-at-a-time
    # launches sustain
    rates = [100, 200, 500, 1000, 2000, 5000, 10000, 20000, 40000]
    rows = []
    for rate in rates:
        count = int(min(5000, max(1000, 2 * rate)))
        arr = synth.poisson_arrivals(rate, count, seed=rate)
        pick = np.random.default_rng(rate).integers(0, len(pool), count)
        n_total = int(sum(pool[i]["n"] for i in pick))
        # served: one submitter thread at the arrival times, the main thread waits
        srv = B.Server(budget_bytes=64 << 30, n_slots=4, max_batch=64)
        # untimed: every request shape once, so the server's grid pool holds
        # blocks as the one-at-a-time path holds its preallocated outputs
        warm = [srv.submit(r["coords"], r["attrs"], r["n"], r["axes"], r["bounds"], r["nx"], r["ny"], r["ops"])
                for r in pool]
        for t in warm:
            srv.wait(t, timeout_s=120)
            srv.release(t)
        warm_batches = int(srv.stats()["batches"])
        tickets = [None] * count
        sub_t = [0.0] * count
        # each pool request marshalled once, as a simulation that submits the
        # same columns every step would: the submitter thread only submits
        preps = [srv.prepare(r["coords"], r["attrs"], r["n"], r["axes"], r["bounds"], r["nx"], r["ny"], r["ops"])
                 for r in pool]

        def submitter():
            start = time.perf_counter()
            for j in range(count):
                while time.perf_counter() - start < arr[j]:
                    d = arr[j] - (time.perf_counter() - start)
                    if d > 2e-4:
                        time.sleep(d - 1e-4)
                sub_t[j] = time.perf_counter()
                tickets[j] = srv.submit_prepared(preps[pick[j]])

        th = threading.Thread(target=submitter)
        t_start = time.perf_counter()
        th.start()
        lat = []
        t_end = t_start
        for j in range(count):
            while tickets[j] is None:
                time.sleep(5e-5)
            res = srv.wait(tickets[j], timeout_s=120)
            if res.status != B.BIN_OK:
                raise SystemExit(f"served request failed: {B.status_string(res.status)}")
            lat.append(res.submit_to_done_ms)
            t_end = max(t_end, sub_t[j] + res.submit_to_done_ms / 1e3)
            srv.release(tickets[j])
        th.join()
        submit_span = sub_t[-1] - sub_t[0] if count > 1 else 0.0
        stats = srv.stats()
        srv.destroy()
        p50, p99 = _percentiles(lat)
        span = t_end - t_start
        # one at a time: same arrivals, each request enqueued alone and waited for
        lat1 = []
        start = time.perf_counter()
        t_end1 = start
        for j in range(count):
            now = time.perf_counter() - start
            if now < arr[j]:
                time.sleep(arr[j] - now)
            batch.launch_one(int(pick[j]), stream)
            stream.synchronize()
            done = time.perf_counter()
            lat1.append((done - start - arr[j]) * 1e3)
            t_end1 = done
        q50, q99 = _percentiles(lat1)
        span1 = t_end1 - start
        row = {"rate_req_s": rate, "requests": count, "particles": n_total,
               "submitted_req_s": round((count - 1) / submit_span, 1) if submit_span > 0 else None,
               "served": {"Gps": round(n_total / span / 1e9, 3), "p50_ms": p50, "p99_ms": p99,
                          "batches": int(stats["batches"]) - warm_batches, "peak_bytes": int(stats["peak_bytes"])},
               "one_at_a_time": {"Gps": round(n_total / span1 / 1e9, 3), "p50_ms": q50, "p99_ms": q99}}
        log(f"rate {rate}: {row}")
        rows.append(row)
    top = rows[-1]
    rec = {
        "metric": METRIC, "value": top["served"]["Gps"], "unit": "Gparticles/s", "n_gpus": 1,
        "steps": len(rates), "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "served_poisson_batched_pool", "budget_bytes": 64 << 30, "slots": 4,
                   "max_batch": 64, "rates_req_s": rates, "warm_up": "each request shape once, untimed, per rate",
                   "latency": "submit to completion event (served); "
                   "arrival to completion after a stream sync (one at a time)",
                   "requests": "drawn uniformly from the 256-request batched set"},
        "served": rows, "p50_ms": top["served"]["p50_ms"], "p99_ms": top["served"]["p99_ms"],
        "cpu_baseline": None,
    }
    print(json.dumps(rec), flush=True)


def run_multi(args):
    """Several coordinate systems over one particle table (the paper's in situ
    load: ten variables binned on nine planes every step): one
    bin_particles_multi call (one fused pass over the table, then the tile
    binning of every grid) against the nine grids binned one call each."""
    import torch
    from paper_2310_02926_amd import binding as B
    from paper_2310_02926_amd import synth
    n = (1 << 24) >> args.scale
    side = 256
    t0 = time.time()
    tab = synth.insitu_table(n, seed=0)
    log(f"generated the ten-column table, n={n}, in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    cols = [torch.from_numpy(c).to(dev) for c in tab.columns]
    grids = []
    for (a, b), bd in zip(tab.planes, tab.bounds):
        grids.append(dict(axes=(a, b), bounds=bd, nx=side, ny=side, ops=31,
                          out=B.alloc_outputs(cols, side, side, 31, dev)))
    stream = torch.cuda.Stream()

    # both sides marshalled once, as a simulation binning every step would
    multi = B.Multi(cols, cols, n, grids)
    alone = B.Batch([dict(coords=cols, attrs=cols, n=n, axes=g["axes"], bounds=g["bounds"], nx=side, ny=side,
                          ops=31, out=g["out"]) for g in grids])

    def fused():
        multi.launch(stream)

    def separate():
        for i in range(alone.n):
            alone.launch_one(i, stream)
    graph = B.BinGraph.multi(cols, cols, n, grids)  # the per-step replay of the same call
    for _ in range(args.warmup):
        fused()
        separate()
        graph.launch(stream)
    stream.synchronize()
    ms_fused = time_region(fused, stream, args.steps) / args.steps
    ms_sep = time_region(separate, stream, args.steps) / args.steps
    ms_graph = time_region(lambda: graph.launch(stream), stream, args.steps) / args.steps
    graph.destroy()
    B.bin_timing_enable(True)
    fused()
    stream.synchronize()
    B.bin_timing_enable(False)
    rep = B.bin_timing_report()
    k_ms = {k: round(v[1] / max(v[0], 1), 5) for k, v in rep.items()}
    log(f"fused {ms_fused:.3f} ms, graph replay {ms_graph:.3f} ms, nine separate calls {ms_sep:.3f} ms; "
        f"kernels {k_ms}")
    table_bytes = sum(c.nbytes for c in tab.columns)
    rec = {
        "metric": METRIC, "value": round(n / (ms_fused / 1e3) / 1e9, 3), "unit": "Gparticles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_fused, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "multi_9planes_10vars_16M_256sq", "n": n, "grids": "9 planes x 256x256",
                   "variables": "10 x f32 (position, velocity, acceleration, mass)", "ops": "count,sum,min,max,avg"},
        "multi": {"fused_ms": round(ms_fused, 4), "graph_replay_ms": round(ms_graph, 4),
                  "separate_calls_ms": round(ms_sep, 4),
                  "speedup": round(ms_sep / ms_fused, 3), "table_bytes": table_bytes,
                  "fused_scatter_ms": k_ms.get("part_scatter_multi_kernel"), "kernels_ms": k_ms},
        "cpu_baseline": None,
    }
    print(json.dumps(rec), flush=True)


def run_insitu(args):
    """Same-device in situ coupling: a synthetic solver (particle push plus a
    chain of bf16 matrix products standing in for the force computation) and
    the binning of its particles every step, three ways: solver alone,
    lockstep zero-copy binning on the solver's stream, and the asynchronous
    mode (deep copy on the solver's stream, binning on a second stream)."""
    import torch
    from paper_2310_02926_amd import binding as B
    from paper_2310_02926_amd import synth
    n = (1 << 24) >> args.scale
    side = 1024
    ws = synth.gmm_f32(n=n, seed=3, nx=side, ny=side, k=1)
    dev = torch.device("cuda:0")
    x, y = (torch.from_numpy(c).to(dev) for c in ws.coords)
    m = torch.from_numpy(ws.attrs[0]).to(dev)
    g = torch.Generator(device="cpu").manual_seed(3)
    vx = (torch.randn(n, generator=g) * 1e-3).to(dev)
    vy = (torch.randn(n, generator=g) * 1e-3).to(dev)
    h = torch.randn(4096, 4096, generator=g).to(dev, torch.bfloat16)
    w = (torch.randn(4096, 4096, generator=g) / 64).to(dev, torch.bfloat16)
    outs = B.alloc_outputs([m], side, side, 31, dev)
    src, bs = torch.cuda.Stream(), torch.cuda.Stream()
    bounds = (0.0, 1.0, 0.0, 1.0)

    def solver():
        nonlocal h
        x.add_(vx).remainder_(1.0)
        y.add_(vy).remainder_(1.0)
        for _ in range(4):
            h = torch.mm(h, w)

    def step_solver():
        with torch.cuda.stream(src):
            solver()

    def step_lockstep():
        with torch.cuda.stream(src):
            solver()
            B.bin_particles([x, y], [m], n, (0, 1), bounds, side, side, 31, outs, stream=src)

    def step_async():
        with torch.cuda.stream(src):
            solver()
            B.bin_particles_async([x, y], [m], n, (0, 1), bounds, side, side, 31, outs, src_stream=src,
                                  bin_stream=bs)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e_src, e_bs = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(src)
        bs.wait_event(e0)
        for _ in range(args.steps):
            fn()
        e_src.record(src)
        e_bs.record(bs)
        torch.cuda.synchronize()
        return e0.elapsed_time(e_src) / args.steps, max(e0.elapsed_time(e_src), e0.elapsed_time(e_bs)) / args.steps

    def bin_alone():
        B.bin_particles([x, y], [m], n, (0, 1), bounds, side, side, 31, outs, stream=src)

    t_bin, _ = timed(bin_alone)
    t_solver, _ = timed(step_solver)
    t_lock, _ = timed(step_lockstep)
    t_async_solver, t_async = timed(step_async)
    rec = {
        "metric": METRIC, "value": round(n / (t_bin / 1e3) / 1e9, 3), "unit": "Gparticles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_async, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "insitu_same_device_16M_1024sq", "n": n, "grid": f"{side}x{side}",
                   "solver": "particle push + 4 bf16 4096^3 matrix products per step"},
        "insitu": {"bin_alone_ms": round(t_bin, 4), "solver_alone_ms": round(t_solver, 4),
                   "lockstep_step_ms": round(t_lock, 4), "async_step_ms": round(t_async, 4),
                   "async_solver_stream_ms": round(t_async_solver, 4),
                   "lockstep_insitu_ms": round(t_lock - t_solver, 4),
                   "async_apparent_insitu_ms": round(t_async - t_solver, 4),
                   "async_solver_slowdown": round(t_async_solver / t_solver, 4)},
        "cpu_baseline": None,
    }
    print(json.dumps(rec), flush=True)


def time_region(call, stream, steps):
    """Milliseconds of `steps` back-to-back calls: one event pair on the
    launch stream around all of them, the device synchronised on both sides."""
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    h0 = time.perf_counter()
    for _ in range(steps):
        call()
    e1.record(stream)
    # host time to enqueue the region: a region whose device time exceeds
    # the sum of its calls' own times by far while this is small waited on
    # the device; one where this is close to the device time was host-bound
    time_region.host_ms = (time.perf_counter() - h0) * 1e3
    stream.synchronize()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def time_each(call, stream, steps):
    """Milliseconds of each of `steps` calls (an event pair around each)."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        call()
        b.record(stream)
    stream.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def stream_copy_GBs(dev, stream, nbytes=1 << 30, reps=10):
    """Measured device-to-device copy bandwidth (bytes read + written per
    second) of a plain 1 GiB copy: the practical streaming ceiling."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        dst.copy_(src)
        ms = time_region(lambda: dst.copy_(src), stream, reps)
    del src, dst
    return 2 * nbytes * reps / (ms / 1e3) / 1e9


def _bits(a):
    return a.view(np.int64 if a.dtype == np.float64 else np.int32)


def precision_study(ws, coords, attrs, stream, steps):
    """Each precision mode on the whole workload against the binary64 oracle:
    count/min/max mismatches (bins), and per op the largest and the 99th
    percentile error over non-empty bins - |sum - ref| / sum|a| and
    |avg - ref| / (sum|a| / count) - plus plain relative error |x - ref| / |ref|
    where the sum does not cancel (|ref| >= sum|a| / 1000); and each mode's
    time per call."""
    import torch
    from oracle import binning_oracle as orc
    from paper_2310_02926_amd import binding as B
    t0 = time.perf_counter()
    ref = orc.bin_particles(ws.coords, ws.attrs, ws.axes, ws.bounds, ws.nx, ws.ny)
    log(f"precision study: oracle on all {ws.n} particles in {time.perf_counter() - t0:.1f}s")
    cnt = ref["count"].ravel()
    full = cnt > 0
    out = {}
    for name, flag in (("default", 0), ("comp", B.PREC_COMP), ("plain", B.PREC_PLAIN), ("f64", B.PREC_F64)):
        ops = B.OPS_ALL | flag
        o = B.alloc_outputs(attrs, ws.nx, ws.ny, ops, coords[0].device)

        def call():
            B.bin_particles(coords, attrs, ws.n, ws.axes, ws.bounds, ws.nx, ws.ny, ops, o, stream=stream)
        for _ in range(3):
            call()
        ms = time_region(call, stream, steps) / steps
        g = {"count": o["count"].cpu().numpy().view(np.uint32).astype(np.int64).ravel()}
        row = {"ms_per_step": round(ms, 5), "Gparticles_s": round(ws.n / (ms / 1e3) / 1e9, 3),
               "count_mismatches": int(np.sum(g["count"] != cnt))}
        for j in range(len(ws.attrs)):
            asum = ref["abs_sum"][j].ravel()
            for key in ("min", "max"):
                got = o[key][j].cpu().numpy().ravel()
                row[f"{key}_mismatches"] = row.get(f"{key}_mismatches", 0) + int(
                    np.sum(_bits(got) != _bits(ref[key][j].ravel().astype(got.dtype))))
            for key in ("sum", "avg"):
                got = o[key][j].cpu().numpy().ravel().astype(np.float64)
                r = ref[key][j].ravel()
                err = np.abs(got[full] - r[full])
                scale = asum[full] if key == "sum" else asum[full] / cnt[full]
                norm = err / scale
                well = np.abs(r[full]) * 1e3 >= scale
                rel = err[well] / np.abs(r[full][well])
                row[f"{key}_err_norm_max"] = float(norm.max()) if norm.size else 0.0
                row[f"{key}_err_norm_p99"] = float(np.percentile(norm, 99)) if norm.size else 0.0
                row[f"{key}_err_rel_max"] = float(rel.max()) if rel.size else 0.0
                row[f"{key}_err_rel_p99"] = float(np.percentile(rel, 99)) if rel.size else 0.0
        out[name] = row
        log(f"precision {name}: {row}")
        del o
        torch.cuda.synchronize()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="hotspot",
                    choices=["hotspot", "gmm", "uniform", "nd3", "batched", "served", "insitu", "multi"])
    ap.add_argument("--prec", default="default", choices=["default", "comp", "plain", "f64"])
    ap.add_argument("--scale", type=int, default=0, help="shrink n by 2^scale (quick runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-studies", action="store_true",
                    help="skip the precision study and the bounds-from-data leg of the headline")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched: skip bin_autotune (plans come from the BIN_TUNE_CACHE file, else the planner)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of known size (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "served":
        return run_served(args)
    if args.workload == "insitu":
        return run_insitu(args)
    if args.workload == "multi":
        return run_multi(args)

    import torch
    from paper_2310_02926_amd import binding as B

    t0 = time.time()
    ws, cfg = make_workload(args.workload, args.scale)
    log(f"generated {cfg['workload']} n={ws.n} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    coords = [torch.from_numpy(c).to(dev) for c in ws.coords]
    attrs = [torch.from_numpy(a).to(dev) for a in ws.attrs]
    flag = {"default": 0, "comp": B.PREC_COMP, "plain": B.PREC_PLAIN, "f64": B.PREC_F64}[args.prec]
    ops = B.OPS_ALL | flag
    stream = torch.cuda.Stream()
    if "nd" in ws.meta:
        nd_axes, nd_bounds, nd_dims = ws.meta["nd"]
        out = B.alloc_outputs_nd(attrs, nd_dims, ops, dev)

        def call():
            B.bin_particles_nd(coords, attrs, ws.n, nd_axes, nd_bounds, nd_dims, ops, out, stream=stream)
    else:
        out = B.alloc_outputs(attrs, ws.nx, ws.ny, ops, dev)
        prepared = B.Call(coords, attrs, ws.n, ws.axes, ws.bounds, ws.nx, ws.ny, ops, out)

        def call():
            prepared.launch(stream)
    torch.cuda.synchronize()

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB device-to-device copy done")
        del src, dst

    # (for three axes: the plan of the folded two-axis mesh nx by ny * nz)
    req, keep = B.request(coords, attrs, ws.n, ws.axes, ws.bounds, ws.nx, ws.ny, ops,
                          {k: (v.view(-1) if not isinstance(v, list) else [t.view(-1) for t in v])
                           for k, v in out.items()})
    plan = B.bin_describe_plan(req)
    log(f"plan: {plan}")
    for _ in range(args.warmup):
        call()
    stream.synchronize()
    log(f"warmup {args.warmup} done")

    # Timed region 1: exactly `steps` whole calls, bracketed by events on the
    # launch stream with the device synchronised on both sides.
    ms_step = time_region(call, stream, args.steps) / args.steps
    host_ms_step = time_region.host_ms / args.steps
    # Region 2: the same calls one by one (an event pair around each), for
    # the distribution of the time per call.
    each = np.asarray(time_each(call, stream, args.steps))
    # Region 3: the same calls with the library's per-kernel event pairs.
    B.bin_timing_enable(True)
    for _ in range(args.steps):
        call()
    stream.synchronize()
    B.bin_timing_enable(False)
    rep = B.bin_timing_report()
    dominant = max(rep, key=lambda k: rep[k][1])
    launches, kern_ms = rep[dominant]
    log(f"timed {args.steps} steps: {ms_step:.4f} ms/step (median {np.median(each):.4f}, host enqueue "
        f"{host_ms_step:.4f} ms/step); kernels (avg ms): "
        + ", ".join(f"{k}={v[1] / max(v[0], 1):.4f}" for k, v in sorted(rep.items(), key=lambda kv: -kv[1][1])))
    copy_gbs = stream_copy_GBs(dev, stream)
    log(f"stream copy {copy_gbs:.0f} GB/s")

    ins, outs = algorithmic_bytes(ws)
    kern_avg_s = kern_ms / max(launches, 1) / 1e3
    kbytes = kernel_algorithmic_bytes(dominant, ws)
    achieved = kbytes / kern_avg_s / 1e9
    khash = kernel_source_hash()
    value = ws.n / (ms_step / 1e3) / 1e9
    whole_gbs = (ins + outs) / (ms_step / 1e3) / 1e9
    # HBM bytes per launch of the dominant kernel from the committed counter
    # runs (FETCH_SIZE + WRITE_SIZE, copy-calibrated), only while the kernel
    # sources are the ones those counters were taken on
    tr = load_traffic(khash, cfg["workload"])
    traffic_bytes, traffic_detail = None, None
    if tr and tr.get("kernel") == dominant:
        b = tr["bytes_per_launch"]
        traffic_bytes = int(b["fetch"] + b["write"])
        traffic_detail = {"fetch": b["fetch"], "write": b["write"], "source": tr.get("source")}
    rec = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gparticles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.workload == "uniform" else "f32",
        "data": "synthetic",
        "config": dict(cfg, precision={"default": "f32 inputs, fp64 per-bin accumulation in LDS, fp64 sum/avg out",
                                       "comp": "fp32 compensated (TwoSum) sums, fp64 merge",
                                       "plain": "fp32 sums", "f64": "fp64 sums"}[args.prec], plan=plan),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_bytes,
            "traffic_detail": traffic_detail,
            "kernel": dominant,
            "algorithmic_bytes_per_launch": kbytes,
            "kernel_ms_avg": round(kern_avg_s * 1e3, 5),
        },
        "per_call_ms": {"median": round(float(np.median(each)), 5), "p10": round(float(np.percentile(each, 10)), 5),
                        "p90": round(float(np.percentile(each, 90)), 5), "calls": int(each.size)},
        "host_enqueue_ms_per_step": round(host_ms_step, 5),
        "kernels_ms_avg": {k: round(v[1] / max(v[0], 1), 5) for k, v in rep.items()},
        "whole_call": {
            "algorithmic_bytes": ins + outs,
            "achieved_GBs": round(whole_gbs, 1),
            "frac_of_hbm_peak": round(whole_gbs / HBM_PEAK_GBS, 4),
            "stream_copy_GBs": round(copy_gbs, 1),
            "frac_of_stream_copy": round(whole_gbs / copy_gbs, 4),
        },
        "kernel_source_hash": khash,
        "host_cpu": host_cpu(),
    }
    if args.workload == "hotspot" and args.prec == "default" and not args.no_studies and "nd" not in ws.meta:
        # Bounds from the data: the same call with bounds = NULL (a min/max
        # pass over the two coordinate columns first).
        oa = B.alloc_outputs(attrs, ws.nx, ws.ny, ops, dev)

        def call_auto():
            B.bin_particles(coords, attrs, ws.n, ws.axes, None, ws.nx, ws.ny, ops, oa, stream=stream)
        for _ in range(3):
            call_auto()
        ms_auto = time_region(call_auto, stream, args.steps) / args.steps
        B.bin_timing_enable(True)
        for _ in range(args.steps):
            call_auto()
        stream.synchronize()
        B.bin_timing_enable(False)
        ra = B.bin_timing_report()
        bk = ra.get("bounds_reduce_kernel", (1, 0.0))
        b_ms = bk[1] / max(bk[0], 1)
        b_bytes = sum(c.itemsize * c.size for c in ws.coords[:2])
        rec["bounds_from_data"] = {
            "ms_per_step": round(ms_auto, 5), "Gparticles_s": round(ws.n / (ms_auto / 1e3) / 1e9, 3),
            "bounds_reduce_kernel_ms": round(b_ms, 5),
            "bounds_pass_GBs": round(b_bytes / (b_ms / 1e3) / 1e9, 1) if b_ms > 0 else None,
            "bounds_pass_frac_of_hbm_peak": round(b_bytes / (b_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if b_ms > 0 else None,
            "floor_bytes_per_particle": 2 * ws.coords[0].itemsize}
        log(f"bounds from the data: {rec['bounds_from_data']}")
        del oa
        rec["precision_study"] = precision_study(ws, coords, attrs, stream, max(10, args.steps // 2))
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample (one process)")
        one = cpu_baseline_1core(ws)
        m = int(one["sample"].split()[1])
        workers = max(1, min(16, os.cpu_count() or 1))
        log(f"timing the CPU oracle on {workers} processes")
        rec["cpu_baseline"] = cpu_baseline_ncore(ws, m, workers)
        rec["cpu_baseline_1core"] = one
    else:
        rec["cpu_baseline"] = None
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
