"""GPU parity at the benchmark's full sizes, on the benchmark's own inputs
(same generators and seeds) and in its launch configuration (automatic plan,
a side stream, all five operations): hotspot 2^27 particles on 2048^2,
Gaussian mixture 2^24 with four attributes on 1024^2, 64 halos 2^26 on a
128^3 mesh.  The oracle bins the whole set in seconds, so every bin is
compared: count/min/max bit-exact, sum/avg within 1e-5 * sum|a| (the plain
FP32 mode within its sequential error bound).  The largest relative sum error
of each precision mode is printed beside the check."""
import sys

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
