"""GPU parity at the benchmark's full sizes, on the benchmark's own inputs
(same generators and seeds) and in its launch configuration (automatic plan,
a side stream, all five operations): hotspot 2^27 particles on 2048^2,
Gaussian mixture 2^24 with four attributes on 1024^2, 64 halos 2^26 on a
128^3 mesh, the batch of 256 requests (2.7e8 particles) after the
autotuner, as one batched call and as a graph, and nine 256^2 planes over one
2^24-particle table of ten variables in one multi-grid call.  The oracle bins the whole
set in seconds, so every bin is compared (for the batch: every bin of a
seeded sample of 40 requests, the largest and smallest among them): count/min/max bit-exact, sum/avg within 1e-5 * sum|a| (the plain
FP32 mode within its sequential error bound).  The largest relative sum error
of each precision mode is printed beside the check."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import binning_oracle as orc
from paper_2310_02926_amd import synth
from tests import gpu_check as G

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
torch = pytest.importorskip("torch")

PRECS = ["default", "comp", "plain", "f64"]


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _flag(prec):
    from paper_2310_02926_amd import binding as B
    return {"default": 0, "comp": B.PREC_COMP, "plain": B.PREC_PLAIN, "f64": B.PREC_F64}[prec]


@pytest.fixture(autouse=True)
def _auto_plan():
    from paper_2310_02926_amd import binding as B
    B.bin_set_plan_override(-1, 0, 0)
    yield


class _Loaded:
    def __init__(self, ws):
        self.ws = ws
        dev = torch.device("cuda:0")
        self.coords = [torch.from_numpy(np.ascontiguousarray(c)).to(dev) for c in ws.coords]
        self.attrs = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in ws.attrs]
        nd = ws.meta.get("nd") if ws.meta else None
        if nd:
            self.ref = orc.bin_particles_nd(ws.coords, ws.attrs, *nd)
        else:
            self.ref = G.oracle(ws)

    def run(self, ops):
        """One call as the benchmark times it; results as numpy arrays."""
        from paper_2310_02926_amd import binding as B
        ws, dev = self.ws, torch.device("cuda:0")
        stream = torch.cuda.Stream()
        nd = ws.meta.get("nd") if ws.meta else None
        if nd:
            out = B.alloc_outputs_nd(self.attrs, nd[2], ops, dev)
            torch.cuda.synchronize()
            B.bin_particles_nd(self.coords, self.attrs, ws.n, nd[0], nd[1], nd[2], ops, out, stream=stream)
        else:
            out = B.alloc_outputs(self.attrs, ws.nx, ws.ny, ops, dev)
            torch.cuda.synchronize()
            B.bin_particles(self.coords, self.attrs, ws.n, ws.axes, ws.bounds, ws.nx, ws.ny, ops, out,
                            stream=stream)
        stream.synchronize()
        res = {"count": out["count"].cpu().numpy().view(np.uint32).astype(np.int64)}
        for key in ("sum", "min", "max", "avg"):
            res[key] = [t.cpu().numpy() for t in out[key]]
        return res


_CACHE = {}


def _workload(name):
    """Generated and binned by the oracle once per process (tens of seconds
    for the largest)."""
    if name not in _CACHE:
        _CACHE.clear()
        _case(f"generating {name} and binning it with the oracle")
        ws = {"hotspot": lambda: synth.hotspot_f32(n=1 << 27, seed=0, side=2048),
              "gmm": lambda: synth.gmm_f32(n=1 << 24, seed=0, nx=1024, ny=1024, k=4),
              "nd3": lambda: synth.halos3d_f32(n=1 << 26, seed=0, side=128)}[name]()
        _CACHE[name] = _Loaded(ws)
    return _CACHE[name]


def _max_rel_sum_error(got, ref):
    worst = 0.0
    for j in range(len(ref["sum"])):
        s = ref["abs_sum"][j]
        nz = s > 0
        err = np.abs(got["sum"][j].astype(np.float64) - ref["sum"][j])
        if nz.any():
            worst = max(worst, float(np.max(err[nz] / s[nz])))
    return worst


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["hotspot", "gmm", "nd3"])
def test_full_size_workload(name, prec):
    from paper_2310_02926_amd import binding as B
    w = _workload(name)
    _case(f"full size {name} n={w.ws.n} prec={prec}")
    got = w.run(B.OPS_ALL | _flag(prec))
    ref = w.ref
    assert got["count"].shape == ref["count"].shape
    assert int(got["count"].sum()) == int(ref["count"].sum())
    G.assert_parity(got, ref, B.OPS_ALL, plain=(prec == "plain"), what=f"{name} {prec}")
    print(f"[error] {name} {prec}: largest |sum - oracle| / sum|a| = {_max_rel_sum_error(got, ref):.3e}",
          flush=True)


def _to_np(out):
    res = {}
    if "count" in out:
        res["count"] = out["count"].cpu().numpy().view(np.uint32).astype(np.int64)
    for key in ("sum", "min", "max", "avg"):
        if key in out:
            res[key] = [t.cpu().numpy() for t in out[key]]
    return res


class _Batch:
    """The 256-request set, uploaded and tuned as the benchmark does; the
    oracle's results for a seeded sample of it."""

    def __init__(self):
        from paper_2310_02926_amd import binding as B
        specs = synth.batch_specs(256, seed=0, n_hi=1e7)
        with ThreadPoolExecutor(8) as ex:  # each instance has its own generator
            self.wss = list(ex.map(synth.instance, specs))
        dev = torch.device("cuda:0")
        self.reqs = []
        for ws in self.wss:
            coords, attrs = G.to_device(ws)
            out = B.alloc_outputs(attrs, ws.nx, ws.ny, ws.ops, dev)
            self.reqs.append(dict(coords=coords, attrs=attrs, n=ws.n, axes=ws.axes, bounds=ws.bounds, nx=ws.nx,
                                  ny=ws.ny, ops=ws.ops, out=out))
        torch.cuda.synchronize()
        B.bin_autotune(self.reqs)
        ns = np.array([ws.n for ws in self.wss])
        rng = np.random.default_rng(7)
        pick = set(rng.choice(len(ns), 38, replace=False).tolist()) | {int(ns.argmax()), int(ns.argmin())}
        self.sample = sorted(pick)
        self.refs = {i: G.oracle(self.wss[i]) for i in self.sample}

    def clear_outputs(self):
        for r in self.reqs:
            for key, val in r["out"].items():
                for t in (val if isinstance(val, list) else [val]):
                    t.fill_(7)
        torch.cuda.synchronize()


def _batch():
    if "batch" not in _CACHE:
        _CACHE.clear()
        _case("generating the 256-request batch, autotuning, binning a sample with the oracle")
        _CACHE["batch"] = _Batch()
    return _CACHE["batch"]


@pytest.mark.parametrize("mode", ["batched", "graph"])
def test_full_size_batch(mode):
    from paper_2310_02926_amd import binding as B
    w = _batch()
    total = sum(r["n"] for r in w.reqs)
    _case(f"full batch of {len(w.reqs)} requests, {total} particles, {mode}")
    w.clear_outputs()
    stream = torch.cuda.Stream()
    if mode == "batched":
        batch = B.Batch(w.reqs)
        for _ in range(2):
            batch.launch(stream)
    else:
        graph = B.BinGraph(w.reqs)
        try:
            for _ in range(2):
                graph.launch(stream)
            stream.synchronize()
        finally:
            graph.destroy()
    stream.synchronize()
    for i in w.sample:
        ws = w.wss[i]
        G.assert_parity(_to_np(w.reqs[i]["out"]), w.refs[i], ws.ops,
                        what=f"{mode} request {i} (n={ws.n}, {ws.nx}^2, k={ws.k})")


def test_full_size_multi():
    """The benchmark's multi-grid workload: nine planes of 256^2 bins over one
    2^24-particle table of ten f32 variables, every variable reduced on every
    plane, in one bin_particles_multi call (one fused pass over the table),
    called twice on the same outputs; every bin of every grid against the
    oracle."""
    from paper_2310_02926_amd import binding as B
    _case("full size multi-grid: n=2^24, 9 planes of 256^2, 10 variables")
    n, side = 1 << 24, 256
    tab = synth.insitu_table(n, seed=0)
    dev = torch.device("cuda:0")
    cols = [torch.from_numpy(c).to(dev) for c in tab.columns]
    grids = []
    for (a, b), bd in zip(tab.planes, tab.bounds):
        grids.append(dict(axes=(a, b), bounds=bd, nx=side, ny=side, ops=31,
                          out=B.alloc_outputs(cols, side, side, 31, dev)))
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    B.bin_timing_enable(True)
    for _ in range(2):
        B.bin_particles_multi(cols, cols, n, grids, stream=stream)
    stream.synchronize()
    B.bin_timing_enable(False)
    rep = B.bin_timing_report()
    assert rep.get("part_scatter_multi_kernel", (0, 0))[0] == 2, rep
    assert "part_scatter_kernel" not in rep, rep

    def ref(g):
        ws = synth.Workload(tab.columns, tab.columns, axes=g["axes"], bounds=g["bounds"], nx=side, ny=side, ops=31)
        return G.oracle(ws)
    with ThreadPoolExecutor(3) as ex:
        refs = list(ex.map(ref, grids))
    for gi, (g, r) in enumerate(zip(grids, refs)):
        got = _to_np(g["out"])
        assert int(got["count"].sum()) == int(r["count"].sum()), gi
        G.assert_parity(got, r, 31, what=f"multi grid {gi}")
