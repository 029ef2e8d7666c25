"""Batched launches and HIP graphs: each request's result equals the oracle
and its own plain bin_particles result (alone vs in the mix)."""
import sys

import numpy as np
import pytest

from paper_2310_02926_amd import synth
from tests import gpu_check as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _to_np(out):
    res = {}
    if "count" in out:
        res["count"] = out["count"].cpu().numpy().view(np.uint32).astype(np.int64)
    for key in ("sum", "min", "max", "avg"):
        if key in out:
            res[key] = [t.cpu().numpy() for t in out[key]]
    return res


def _mix(count, seed, n_hi=300_000, sides=(32, 64, 128, 256, 512, 1024)):
    specs = synth.batch_specs(count, seed=seed, n_lo=1e3, n_hi=n_hi, sides=sides)
    wss = [synth.instance(s) for s in specs]
    return specs, wss


def _requests(wss, flags=0):
    from paper_2310_02926_amd import binding as B
    reqs, dev = [], torch.device("cuda")
    for ws in wss:
        coords, attrs = G.to_device(ws)
        ops = ws.ops | flags
        out = B.alloc_outputs(attrs, ws.nx, ws.ny, ops, dev)
        reqs.append(dict(coords=coords, attrs=attrs, n=ws.n, axes=ws.axes, bounds=ws.bounds, nx=ws.nx, ny=ws.ny,
                         ops=ops, out=out))
    return reqs


def _check_vs_oracle(reqs, wss, what):
    for i, (r, ws) in enumerate(zip(reqs, wss)):
        G.assert_parity(_to_np(r["out"]), G.oracle(ws), ws.ops, what=f"{what} request {i} (n={ws.n}, {ws.nx}^2)")


def _same_as_alone(reqs, wss, what):
    """Each batched result equals the plain call's: count/min/max exactly,
    sums/avgs within rounding of binary64 accumulation order."""
    from paper_2310_02926_amd import binding as B
    for i, (r, ws) in enumerate(zip(reqs, wss)):
        out = B.alloc_outputs(r["attrs"], ws.nx, ws.ny, r["ops"], r["coords"][0].device)
        B.bin_particles(r["coords"], r["attrs"], r["n"], r["axes"], r["bounds"], ws.nx, ws.ny, r["ops"], out)
        torch.cuda.synchronize()
        a, b = _to_np(out), _to_np(r["out"])
        if "count" in a:
            assert np.array_equal(a["count"], b["count"]), (what, i)
        for key in ("min", "max"):
            for x, y in zip(a.get(key, []), b.get(key, [])):
                assert np.array_equal(x.view(np.int32), y.view(np.int32)), (what, i, key)
        for key in ("sum", "avg"):
            for x, y in zip(a.get(key, []), b.get(key, [])):
                assert np.allclose(x, y, rtol=1e-12, atol=1e-12, equal_nan=True), (what, i, key)


@pytest.mark.parametrize("seed", [0, 1])
def test_batched_mix_matches_oracle_and_plain(seed):
    from paper_2310_02926_amd import binding as B
    _case(f"batched mix of 40 requests seed={seed}")
    specs, wss = _mix(40, seed)
    reqs = _requests(wss)
    B.bin_particles_batched(reqs)
    torch.cuda.synchronize()
    _check_vs_oracle(reqs, wss, "batched")
    _same_as_alone(reqs, wss, "batched")


@pytest.mark.parametrize("prec", ["comp", "plain", "f64"])
def test_batched_precisions(prec):
    from paper_2310_02926_amd import binding as B
    _case(f"batched precision {prec}")
    flag = {"comp": B.PREC_COMP, "plain": B.PREC_PLAIN, "f64": B.PREC_F64}[prec]
    specs, wss = _mix(12, 7)
    reqs = _requests(wss, flag)
    B.bin_particles_batched(reqs)
    torch.cuda.synchronize()
    for i, (r, ws) in enumerate(zip(reqs, wss)):
        G.assert_parity(_to_np(r["out"]), G.oracle(ws), ws.ops, plain=(prec == "plain"), what=f"{prec} req {i}")


def test_batched_mixed_dtypes_and_strategies():
    """f64 coordinates, f64 attributes and a forced global-atomic request in
    one batch: several groups plus the one-by-one fallback."""
    from paper_2310_02926_amd import binding as B
    _case("batched mixed dtypes")
    rng = np.random.default_rng(3)
    wss = []
    for (n, side, cdt, adt) in [(50_000, 48, np.float64, np.float32), (80_000, 700, np.float64, np.float64),
                                (20_000, 16, np.float32, np.float64), (120_000, 900, np.float32, np.float32)]:
        wss.append(synth.Workload([rng.random(n).astype(cdt), rng.random(n).astype(cdt)],
                                  [rng.standard_normal(n).astype(adt) for _ in range(2)], nx=side, ny=side))
    reqs = _requests(wss)
    B.bin_particles_batched(reqs)
    torch.cuda.synchronize()
    _check_vs_oracle(reqs, wss, "mixed")
    B.bin_set_plan_override(0, 0, 0)  # every request through the global-atomic fallback
    try:
        reqs = _requests(wss)
        B.bin_particles_batched(reqs)
        torch.cuda.synchronize()
    finally:
        B.bin_set_plan_override(-1, 0, 0)
    _check_vs_oracle(reqs, wss, "global fallback")


def test_batched_lds_classes():
    """Members whose tiles (tile binning: up to an eighth, a quarter, a half
    and more of a CU's LDS) or whole grids (LDS strategy: up to a quarter, a
    half and more) fall in different classes run as separate launches of
    their own workgroup size; every result equals the oracle and the same
    request run alone."""
    import re
    from paper_2310_02926_amd import binding as B
    _case("batched LDS classes")
    A = B.OPS_ALL
    specs = [synth.InstanceSpec(200_000, 1024, 4, A, 11), synth.InstanceSpec(150_000, 1024, 2, A, 12),
             synth.InstanceSpec(300_000, 512, 4, A, 18),
             synth.InstanceSpec(300_000, 256, 2, A, 13), synth.InstanceSpec(300_000, 256, 1, A, 14),
             synth.InstanceSpec(80_000, 32, 1, A, 15), synth.InstanceSpec(100_000, 64, 1, A, 16),
             synth.InstanceSpec(80_000, 48, 3, A, 17),
             # a whole grid its own plan bins in two slices
             synth.InstanceSpec(20_000, 32, 2, A, 19)]
    wss = [synth.instance(sp) for sp in specs]
    reqs = _requests(wss)
    arr, keep = B.request_array(reqs)
    props = torch.cuda.get_device_properties(0)
    cu_lds = getattr(props, "shared_memory_per_multiprocessor", 0) or 163840
    seen = {"partition": set(), "lds": set()}
    for i in range(len(reqs)):
        d = B.bin_describe_plan(arr[i])
        kind = d.split()[0]
        size = int(re.search(r"bin_lds=(\d+)" if kind == "partition" else r"\blds=(\d+)", d).group(1))
        shares = (8, 4, 2) if kind == "partition" else (4, 2)
        seen[kind].add(next((c for c, f in enumerate(shares) if f * size <= cu_lds), len(shares)))
    assert seen == {"partition": {0, 1, 2, 3}, "lds": {0, 1, 2}}, seen
    B.bin_particles_batched(reqs)
    torch.cuda.synchronize()
    _check_vs_oracle(reqs, wss, "classes")
    _same_as_alone(reqs, wss, "classes")


def test_batched_edge_requests():
    from paper_2310_02926_amd import binding as B
    _case("batched edge requests")
    rng = np.random.default_rng(4)
    wss = [synth.Workload([np.zeros(0, np.float32), np.zeros(0, np.float32)], [np.zeros(0, np.float32)], nx=300, ny=300),
           synth.Workload([np.full(100, 5.0, np.float32), np.full(100, 5.0, np.float32)], [np.ones(100, np.float32)],
                          nx=2000, ny=3),
           synth.Workload([rng.random(1, dtype=np.float32), rng.random(1, dtype=np.float32)], [np.ones(1, np.float32)],
                          nx=1, ny=1)]
    reqs = _requests(wss)
    B.bin_particles_batched(reqs)
    torch.cuda.synchronize()
    _check_vs_oracle(reqs, wss, "edge")
    B.bin_particles_batched([])  # empty batch is a no-op


def test_batched_rejects_bad_request_by_index():
    from paper_2310_02926_amd import binding as B
    specs, wss = _mix(3, 9)
    reqs = _requests(wss)
    reqs[2]["nx"] = 0
    with pytest.raises(B.BinError) as ei:
        B.bin_particles_batched(reqs)
    assert ei.value.status == B.BIN_ERR_INVALID_ARG and "request 2" in str(ei.value)


def test_graph_replays_match_eager():
    """A captured batch replayed several times, with eager work and syncs in
    between, gives the eager result every time (inputs refilled between
    replays are picked up)."""
    from paper_2310_02926_amd import binding as B
    _case("graph replays")
    specs, wss = _mix(16, 5)
    reqs = _requests(wss)
    g = B.BinGraph(reqs)
    s = torch.cuda.Stream()
    try:
        for rep in range(3):
            for r in reqs:  # scribble over the outputs: replays must overwrite them
                if "count" in r["out"]:
                    r["out"]["count"].fill_(7)
                for key in ("sum", "min", "max", "avg"):
                    for t in r["out"].get(key, []):
                        t.fill_(-3.0)
            torch.cuda.synchronize()
            g.launch(s)
            s.synchronize()
            _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
            _check_vs_oracle(reqs, wss, f"graph replay {rep}")
        # refill the inputs of request 0 in place; the next replay must see them
        ws0 = wss[0]
        new_x = np.random.default_rng(99).random(ws0.n).astype(np.float32)
        reqs[0]["coords"][0].copy_(torch.from_numpy(new_x))
        ws0.coords[0] = new_x
        torch.cuda.synchronize()
        g.launch(s)
        s.synchronize()
        _check_vs_oracle(reqs[:1], wss[:1], "graph after refill")
    finally:
        g.destroy()


def test_autotune_then_bin(tmp_path, monkeypatch):
    """The autotuner picks a configuration per shape class; results stay
    exact/within tolerance with the tuned configuration."""
    from paper_2310_02926_amd import binding as B
    import json
    _case("autotune")
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("BIN_TUNE_CACHE", str(cache))
    specs, wss = _mix(3, 11, n_hi=200_000, sides=(48, 600))
    reqs = _requests(wss)
    B.bin_autotune(reqs)
    # the batch policy was timed on the whole set and filed under this device
    pols = json.loads(cache.read_text())["batch"]
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert list(pols) == [f"{arch}:{cus}"], pols
    assert next(iter(pols.values()))["strategy"] in (0, 1, 2), pols
    B.bin_particles_batched(reqs)
    torch.cuda.synchronize()
    _check_vs_oracle(reqs, wss, "after autotune")
    for r, ws in zip(reqs, wss):
        out = B.alloc_outputs(r["attrs"], ws.nx, ws.ny, r["ops"], r["coords"][0].device)
        B.bin_particles(r["coords"], r["attrs"], r["n"], r["axes"], r["bounds"], ws.nx, ws.ny, r["ops"], out)
        torch.cuda.synchronize()
        G.assert_parity(_to_np(out), G.oracle(ws), ws.ops, what="plain after autotune")


def test_multi_grid_nine_planes_ten_variables():
    """bin_particles_multi: nine coordinate systems over one ten-column table,
    every variable reduced on every plane; each grid equals the oracle and
    the same grid binned alone."""
    from paper_2310_02926_amd import binding as B
    _case("multi-grid: 9 planes x 10 variables")
    tab = synth.insitu_table(300_001, seed=4)
    cols = [torch.from_numpy(c).cuda() for c in tab.columns]
    sides = [64, 128, 32, 256, 64, 100, 48, 64, 512]
    grids = []
    for (a, b), bd, side in zip(tab.planes, tab.bounds, sides):
        out = B.alloc_outputs(cols, side, side // 2 + 1, 31, "cuda")
        grids.append(dict(axes=(a, b), bounds=bd, nx=side, ny=side // 2 + 1, ops=31, out=out))
    B.bin_timing_enable(True)
    B.bin_particles_multi(cols, cols, tab.n, grids)
    torch.cuda.synchronize()
    B.bin_timing_enable(False)
    rep = B.bin_timing_report()
    assert rep.get("part_scatter_multi_kernel", (0, 0))[0] == 1, rep  # one fused pass over the table
    assert "part_scatter_kernel" not in rep, rep
    for g, grid in enumerate(grids):
        ws = synth.Workload(tab.columns, tab.columns, axes=grid["axes"], bounds=grid["bounds"], nx=grid["nx"],
                            ny=grid["ny"], ops=31)
        got = _to_np(grid["out"])
        G.assert_parity(got, G.oracle(ws), 31, what=f"multi grid {g}")
        alone = B.alloc_outputs(cols, grid["nx"], grid["ny"], 31, "cuda")
        B.bin_particles(cols, cols, tab.n, grid["axes"], grid["bounds"], grid["nx"], grid["ny"], 31, alone)
        torch.cuda.synchronize()
        a = _to_np(alone)
        assert np.array_equal(got["count"], a["count"]), g
        for key in ("min", "max"):
            for x, y in zip(got[key], a[key]):
                assert np.array_equal(x.view(np.int32), y.view(np.int32)), (g, key)
        for key in ("sum", "avg"):
            for x, y in zip(got[key], a[key]):
                assert np.allclose(x, y, rtol=1e-12, atol=1e-9, equal_nan=True), (g, key)
    # the same call marshalled once (binding.Multi) and enqueued twice
    before = [_to_np(grid["out"]) for grid in grids]
    for grid in grids:
        for key, val in grid["out"].items():
            for t in (val if isinstance(val, list) else [val]):
                t.fill_(7)
    m = B.Multi(cols, cols, tab.n, grids)
    m.launch()
    m.launch()
    torch.cuda.synchronize()
    for g, (grid, b) in enumerate(zip(grids, before)):
        got = _to_np(grid["out"])
        assert np.array_equal(got["count"], b["count"]), g
        for key in ("min", "max"):
            for x, y in zip(got[key], b[key]):
                assert np.array_equal(x.view(np.int32), y.view(np.int32)), (g, key)


_TUNE_CHILD = r'''
import json, sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
from paper_2310_02926_amd import binding as B
from paper_2310_02926_amd import synth
from tests import gpu_check as G
ws = synth.gmm_f32(n=200_000, seed=9, nx=256, ny=256, k=1)
c, a = G.to_device(ws)
out = B.alloc_outputs(a, ws.nx, ws.ny, ws.ops, "cuda")
req, keep = B.request(c, a, ws.n, ws.axes, ws.bounds, ws.nx, ws.ny, ws.ops, out)
before = B.bin_describe_plan(req)
if sys.argv[2] == "tune":
    B.bin_autotune([dict(coords=c, attrs=a, n=ws.n, axes=ws.axes, bounds=ws.bounds, nx=ws.nx, ny=ws.ny,
                         ops=ws.ops, out=out)])
print(json.dumps({"before": before, "after": B.bin_describe_plan(req),
                  "arch": torch.cuda.get_device_properties(0).gcnArchName.split(":")[0],
                  "cus": torch.cuda.get_device_properties(0).multi_processor_count}))
'''


def test_multi_grid_graph_replays_each_step():
    """bin_graph_create_multi: the nine-plane, ten-variable load captured
    once (the fused scatter included) and replayed as a simulation would
    every step - the table rewritten in place between replays, eager work
    and synchronisations in between, outputs scribbled over - each replay
    equal to the oracle on that step's table."""
    from paper_2310_02926_amd import binding as B
    _case("multi-grid graph: 9 planes x 10 variables, 3 steps")
    n = 200_003
    tab = synth.insitu_table(n, seed=8)
    cols = [torch.from_numpy(c).cuda() for c in tab.columns]
    sides = [64, 128, 32, 256, 64, 100, 48, 64, 512]
    grids = []
    for (a, b), bd, side in zip(tab.planes, tab.bounds, sides):
        out = B.alloc_outputs(cols, side, side // 2 + 1, 31, "cuda")
        grids.append(dict(axes=(a, b), bounds=bd, nx=side, ny=side // 2 + 1, ops=31, out=out))
    torch.cuda.synchronize()
    g = B.BinGraph.multi(cols, cols, n, grids)
    s = torch.cuda.Stream()
    try:
        for step in range(3):
            if step:  # the simulation moves on: a new table in the same columns
                nxt = synth.insitu_table(n, seed=8 + step)
                for c, h in zip(cols, nxt.columns):
                    c.copy_(torch.from_numpy(h))
                tab = nxt
            for grid in grids:
                for key, val in grid["out"].items():
                    for t in (val if isinstance(val, list) else [val]):
                        t.fill_(7)
            torch.cuda.synchronize()
            g.launch(s)
            s.synchronize()
            _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
            for gi, grid in enumerate(grids):
                ws = synth.Workload(tab.columns, tab.columns, axes=grid["axes"], bounds=grid["bounds"],
                                    nx=grid["nx"], ny=grid["ny"], ops=31)
                G.assert_parity(_to_np(grid["out"]), G.oracle(ws), 31, what=f"step {step} grid {gi}")
    finally:
        g.destroy()


_POLICY_CHILD = r'''
import json, sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
from paper_2310_02926_amd import binding as B
from paper_2310_02926_amd import synth
from tests import gpu_check as G
specs = synth.batch_specs(12, seed=5, n_hi=300_000)
wss = [synth.instance(sp) for sp in specs]
reqs = []
for ws in wss:
    c, a = G.to_device(ws)
    reqs.append(dict(coords=c, attrs=a, n=ws.n, axes=ws.axes, bounds=ws.bounds, nx=ws.nx, ny=ws.ny, ops=ws.ops,
                     out=B.alloc_outputs(a, ws.nx, ws.ny, ws.ops, "cuda")))
B.bin_particles_batched(reqs)
torch.cuda.synchronize()
for r, ws in zip(reqs, wss):
    got = {"count": r["out"]["count"].cpu().numpy().view(np.uint32).astype(np.int64)} if "count" in r["out"] else {}
    for key in ("sum", "min", "max", "avg"):
        if key in r["out"]:
            got[key] = [t.cpu().numpy() for t in r["out"][key]]
    G.assert_parity(got, G.oracle(ws), ws.ops, what=f"policy {sys.argv[2]}")
print("ok")
'''


@pytest.mark.parametrize("policy", [(0, 0, 0), (2, 1024, 4), (2, 512, 8), (2, 1024, 16)],
                         ids=["rules", "shape1024x4", "shape512x8", "shape1024x16"])
def test_batch_policy_from_the_tuning_cache(tmp_path, policy):
    """Every batch policy the autotuner can file - the planner's rules, or
    one shared scatter shape (a shape a request cannot take falls back to
    its own) - gives the oracle's results; the policy is read from the
    BIN_TUNE_CACHE file in a fresh process."""
    import json
    import os
    import subprocess
    import sys as _sys
    _case(f"batch policy {policy}")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    mode, nt, ppt = policy
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({"version": 1, "entries": {}, "batch": {
        f"{arch}:{cus}": {"strategy": mode, "scatter_threads": nt, "scatter_ppt": ppt}}}))
    script = tmp_path / "child.py"
    script.write_text(_POLICY_CHILD)
    p = subprocess.run([_sys.executable, str(script), root, str(policy)], capture_output=True, text=True,
                       env=dict(os.environ, BIN_TUNE_CACHE=str(cache)), timeout=300, cwd=root)
    assert p.returncode == 0 and p.stdout.strip().endswith("ok"), p.stderr[-3000:]


def test_autotune_cache_is_json_keyed_by_device(tmp_path):
    """BIN_TUNE_CACHE: the autotuner writes JSON entries keyed by the
    device's architecture and compute units, with every hint (quads
    included); a fresh process reads them back and plans with them; entries
    for another device are ignored."""
    import json
    import os
    import subprocess
    import sys as _sys
    _case("autotune cache")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = tmp_path / "child.py"
    script.write_text(_TUNE_CHILD)
    cache = tmp_path / "tune.json"
    env = dict(os.environ, BIN_TUNE_CACHE=str(cache))

    def child(mode):
        p = subprocess.run([_sys.executable, str(script), root, mode], capture_output=True, text=True, env=env,
                           timeout=300, cwd=root)
        assert p.returncode == 0, p.stderr[-2000:]
        return json.loads(p.stdout.strip().splitlines()[-1])

    tuned = child("tune")
    doc = json.loads(cache.read_text())
    assert doc["version"] == 1 and doc["entries"]
    prefix = f"{tuned['arch']}:{tuned['cus']}|"
    for key, e in doc["entries"].items():
        assert key.startswith(prefix), key
        assert set(e) == {"strategy", "block", "grid", "part_wg", "scatter_ppt", "scatter_threads", "tile_shift",
                          "split_len", "quads"}, e
    again = child("plan")
    assert again["before"] == tuned["after"]  # the fresh process plans with the cached entry
    # the same entries filed under another device are not used here
    doc["entries"] = {"gfx000:1|" + k.split("|", 1)[1]: v for k, v in doc["entries"].items()}
    cache.write_text(json.dumps(doc))
    other = child("plan")
    assert other["before"] == tuned["before"]
