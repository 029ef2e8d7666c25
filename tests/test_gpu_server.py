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
