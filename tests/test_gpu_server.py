"""The request server: continuous batching under a memory budget.  Each
result equals the oracle and the same request run alone; admission waits for
released memory; errors come back per request."""
import sys
import threading

import numpy as np
import pytest

from paper_2310_02926_amd import synth
from tests import gpu_check as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(wss):
    return [G.to_device(ws) for ws in wss]


def _alone(coords, attrs, ws):
    from paper_2310_02926_amd import binding as B
    out = B.alloc_outputs(attrs, ws.nx, ws.ny, ws.ops, coords[0].device)
    B.bin_particles(coords, attrs, ws.n, ws.axes, ws.bounds, ws.nx, ws.ny, ws.ops, out)
    torch.cuda.synchronize()
    res = {}
    if "count" in out:
        res["count"] = out["count"].cpu().numpy().view(np.uint32).astype(np.int64)
    for key in ("sum", "min", "max", "avg"):
        if key in out:
            res[key] = [t.cpu().numpy() for t in out[key]]
    return res


def test_server_results_equal_alone_and_oracle():
    from paper_2310_02926_amd import binding as B
    _case("server: 48 requests from 2 threads")
    specs = synth.batch_specs(48, seed=21, n_lo=1e3, n_hi=2e5)
    wss = [synth.instance(s) for s in specs]
    dev = _dev(wss)
    srv = B.Server(budget_bytes=4 << 30, n_slots=2, max_batch=16)
    tickets = [None] * len(wss)

    def submitter(idx):
        for i in idx:
            c, a = dev[i]
            ws = wss[i]
            tickets[i] = srv.submit(c, a, ws.n, ws.axes, ws.bounds, ws.nx, ws.ny, ws.ops)

    th = [threading.Thread(target=submitter, args=(range(r, len(wss), 2),)) for r in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    try:
        for i, ws in enumerate(wss):
            res = srv.wait(tickets[i], timeout_s=60)
            assert res.status == B.BIN_OK
            assert res.submit_to_done_ms >= res.queue_ms >= 0
            got = srv.fetch(tickets[i], res)
            G.assert_parity(got, G.oracle(ws), ws.ops, what=f"served {i}")
            alone = _alone(*dev[i], ws)
            if "count" in got:
                assert np.array_equal(got["count"], alone["count"])
            for key in ("min", "max"):
                for x, y in zip(got.get(key, []), alone.get(key, [])):
                    assert np.array_equal(x.view(np.int32), y.view(np.int32))
            for key in ("sum", "avg"):
                for x, y in zip(got.get(key, []), alone.get(key, [])):
                    assert np.allclose(x, y, rtol=1e-12, atol=1e-12, equal_nan=True)
            srv.release(tickets[i])
        st = srv.stats()
        assert st["submitted"] == st["completed"] == st["released"] == len(wss)
        assert st["failed"] == 0 and st["batches"] >= 1
    finally:
        srv.destroy()


def test_server_prepared_requests_submitted_again():
    """A request marshalled once (Server.prepare) and submitted three times
    gives three results equal to the oracle's."""
    from paper_2310_02926_amd import binding as B
    _case("server: one prepared request submitted three times")
    ws = synth.instance(synth.batch_specs(1, seed=33, n_lo=5e4, n_hi=2e5)[0])
    c, a = G.to_device(ws)
    srv = B.Server(budget_bytes=1 << 30, n_slots=2, max_batch=8)
    try:
        prep = srv.prepare(c, a, ws.n, ws.axes, ws.bounds, ws.nx, ws.ny, ws.ops)
        tickets = [srv.submit_prepared(prep) for _ in range(3)]
        ref = G.oracle(ws)
        for t in tickets:
            res = srv.wait(t, timeout_s=60)
            assert res.status == B.BIN_OK
            G.assert_parity(srv.fetch(t, res), ref, ws.ops, what=f"prepared ticket {t}")
            srv.release(t)
    finally:
        srv.destroy()


def test_server_budget_admission_and_errors():
    from paper_2310_02926_amd import binding as B
    _case("server: tight budget")
    rng = np.random.default_rng(5)
    n, side = 200_000, 1024  # grids: count + 4 ops x 1 attr ~ 25 MiB per request
    wss = [synth.Workload([rng.random(n, dtype=np.float32), rng.random(n, dtype=np.float32)],
                          [rng.standard_normal(n).astype(np.float32)], nx=side, ny=side) for _ in range(4)]
    dev = _dev(wss)
    srv = B.Server(budget_bytes=80 << 20, n_slots=2, max_batch=4)
    try:
        # a request that can never fit is rejected at submission
        c, a = dev[0]
        with pytest.raises(B.BinError) as ei:
            srv.submit(c, a, n, (0, 1), (0.0, 1.0, 0.0, 1.0), 8192, 4096, 31)
        assert ei.value.status == B.BIN_ERR_ADMISSION
        t = [srv.submit(*dev[i], n, (0, 1), (0.0, 1.0, 0.0, 1.0), side, side, 31) for i in range(4)]
        r0 = srv.wait(t[0], timeout_s=60)
        assert r0.status == B.BIN_OK
        # the budget holds only a couple of resident results: the last waits
        with pytest.raises(B.BinError) as ei:
            srv.wait(t[3], timeout_s=0.2)
        assert ei.value.status == B.BIN_ERR_TIMEOUT
        for i in range(3):
            r = srv.wait(t[i], timeout_s=60)
            G.assert_parity(srv.fetch(t[i], r), G.oracle(wss[i]), 31, what=f"budget {i}")
            srv.release(t[i])
        r = srv.wait(t[3], timeout_s=60)  # admitted once memory was released
        G.assert_parity(srv.fetch(t[3], r), G.oracle(wss[3]), 31, what="budget 3")
        srv.release(t[3])
        with pytest.raises(B.BinError) as ei:
            srv.release(t[3])
        assert ei.value.status == B.BIN_ERR_NOT_FOUND
        with pytest.raises(B.BinError) as ei:
            srv.submit(*dev[0], n, (0, 1), (0.0, 1.0, 0.0, 1.0), 0, 4, 31)
        assert ei.value.status == B.BIN_ERR_INVALID_ARG
        assert srv.stats()["peak_bytes"] <= 80 << 20
    finally:
        srv.destroy()
    h = srv._h
    assert h is None


def test_server_reads_inputs_after_the_producer_stream():
    """A simulation enqueues the writes of its particle columns on its own
    stream behind long-running work and submits at once (no host sync): the
    server orders its kernels after the producer stream's event, so the
    result is the oracle's on the written values."""
    from paper_2310_02926_amd import binding as B
    _case("server: producer stream")
    rng = np.random.default_rng(17)
    n, side = 1_000_003, 256
    ws = synth.Workload([rng.random(n, dtype=np.float32), rng.random(n, dtype=np.float32)],
                        [rng.lognormal(0, 1, n).astype(np.float32)], nx=side, ny=side)
    src_c, src_a = G.to_device(ws)
    coords = [torch.zeros(n, device="cuda") for _ in range(2)]  # all in bin 0 until written
    attrs = [torch.zeros(n, device="cuda")]
    h = torch.randn(4096, 4096, device="cuda", dtype=torch.bfloat16)
    w = (torch.randn(4096, 4096, device="cuda", dtype=torch.bfloat16) / 64).contiguous()
    torch.cuda.synchronize()
    prod = torch.cuda.Stream()
    srv = B.Server(budget_bytes=2 << 30, n_slots=2, max_batch=8)
    try:
        with torch.cuda.stream(prod):
            for _ in range(24):  # a few ms of work ahead of the writes
                h = torch.mm(h, w)
            for d, s in zip(coords + attrs, src_c + src_a):
                d.copy_(s)
        t = srv.submit(coords, attrs, n, (0, 1), ws.bounds, side, side, 31, producer_stream=prod)
        r = srv.wait(t, timeout_s=60)
        G.assert_parity(srv.fetch(t, r), G.oracle(ws), 31, what="producer stream")
        srv.release(t)
    finally:
        srv.destroy()
        torch.cuda.synchronize()


_FAIL_CHILD = r'''
import json, sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
from paper_2310_02926_amd import binding as B
from paper_2310_02926_amd import synth
from tests import gpu_check as G
rng = np.random.default_rng(3)
srv = B.Server(budget_bytes=4 << 30, n_slots=1, max_batch=4)
out = []
for i, (n, side) in enumerate([(30_000, 64), (60_000, 128), (90_000, 256), (120_000, 512), (150_000, 1024)]):
    ws = synth.Workload([rng.random(n, dtype=np.float32), rng.random(n, dtype=np.float32)],
                        [rng.standard_normal(n).astype(np.float32)], nx=side, ny=side)
    c, a = G.to_device(ws)
    t = srv.submit(c, a, n, (0, 1), ws.bounds, side, side, 31)
    try:
        r = srv.wait(t, timeout_s=60)
        G.assert_parity(srv.fetch(t, r), G.oracle(ws), 31, what=f"request {i}")
        out.append("ok")
    except B.BinError as e:
        out.append(B.status_string(e.status))
    srv.release(t)
st = srv.stats()
srv.destroy()
print(json.dumps({"results": out, "failed": int(st["failed"]), "completed": int(st["completed"])}))
'''


@pytest.mark.parametrize("at", [1, 3, 5])
def test_server_failed_allocation_fails_only_its_request(at, tmp_path):
    """With the library's allocation hook set (BIN_FAIL_ALLOC_AT=k: the k-th
    device allocation of the process fails), exactly one request - the one
    whose grid or scratch allocation failed - comes back BIN_ERR_OOM, and
    every other request of the same server equals the oracle."""
    import json
    import os
    import subprocess
    _case(f"server: allocation failure at {at}")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = tmp_path / "child.py"
    script.write_text(_FAIL_CHILD)
    env = dict(os.environ, BIN_FAIL_ALLOC_AT=str(at))
    p = subprocess.run([sys.executable, str(script), root], capture_output=True, text=True, env=env, timeout=240,
                       cwd=root)
    assert p.returncode == 0, p.stderr[-2000:]
    rec = json.loads(p.stdout.strip().splitlines()[-1])
    assert rec["results"].count("BIN_ERR_OOM") == 1, rec
    assert rec["results"].count("ok") == len(rec["results"]) - 1, rec
    assert rec["failed"] == 1 and rec["completed"] == len(rec["results"]) - 1


def test_server_calls_racing_destroy():
    """Threads keep submitting and waiting while the main thread destroys
    the server: each call either finishes (results equal the oracle) or
    fails with BIN_ERR_INVALID_ARG; nothing crashes or hangs."""
    from paper_2310_02926_amd import binding as B
    _case("server: destroy while in use")
    rng = np.random.default_rng(23)
    n, side = 50_000, 128
    ws = synth.Workload([rng.random(n, dtype=np.float32), rng.random(n, dtype=np.float32)],
                        [rng.standard_normal(n).astype(np.float32)], nx=side, ny=side)
    c, a = G.to_device(ws)
    ref = G.oracle(ws)
    srv = B.Server(budget_bytes=1 << 30, n_slots=2, max_batch=8)
    h = srv._h
    stats = {"ok": 0, "dead": 0, "other": []}
    lock = threading.Lock()
    stop = threading.Event()

    def client():
        L = B.lib()
        cc, ck = B.columns(c)
        aa, ak = B.columns(a)
        while not stop.is_set():
            req = B.ServerRequest(cc, aa, n, (B.c_int32 * 2)(0, 1), (B.c_double * 4)(*ws.bounds), side, side, 31,
                                  None)
            t = B.c_uint64()
            st = L.binsrv_submit(h, B.ctypes.byref(req), B.ctypes.byref(t))
            if st != B.BIN_OK:
                with lock:
                    (stats.__setitem__("dead", stats["dead"] + 1) if st == B.BIN_ERR_INVALID_ARG
                     else stats["other"].append(st))
                return
            res = B.Result()
            st = L.binsrv_wait(h, t.value, 60 * 10**9, B.ctypes.byref(res))
            if st == B.BIN_OK:
                cnt = B.copy_to_host(res.count, 4 * side * side, np.uint32, (side, side)).astype(np.int64)
                mn = B.copy_to_host(res.min[0], 4 * side * side, np.float32, (side, side))
                assert np.array_equal(cnt, ref["count"])
                assert np.array_equal(mn.view(np.int32), ref["min"][0].astype(np.float32).view(np.int32))
                L.binsrv_release(h, t.value)
                with lock:
                    stats["ok"] += 1
            elif st == B.BIN_ERR_INVALID_ARG:
                with lock:
                    stats["dead"] += 1
                return
            else:
                with lock:
                    stats["other"].append(st)
                return

    th = [threading.Thread(target=client) for _ in range(4)]
    for t in th:
        t.start()
    import time
    time.sleep(0.5)
    srv.destroy()
    stop.set()
    for t in th:
        t.join(timeout=60)
    assert not any(t.is_alive() for t in th)
    assert stats["other"] == [] and stats["ok"] > 0, stats
