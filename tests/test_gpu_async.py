"""Asynchronous in situ binning (bin_particles_async): the library bins a
deep copy taken in the simulation stream's order, so the simulation may
overwrite its columns at once.  The binning stream is held back behind a
long matrix product so that every later solver step has already rewritten
the columns when the binning runs; each step's grids must still equal the
oracle on that step's values."""
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
    res = {"count": out["count"].cpu().numpy().view(np.uint32).astype(np.int64)}
    for key in ("sum", "min", "max", "avg"):
        res[key] = [t.cpu().numpy() for t in out[key]]
    return res


def _solver_step_host(x, y, m):
    return (np.float32(1) - x).astype(np.float32), (y * np.float32(0.5) + np.float32(0.25)).astype(np.float32), \
        (m * np.float32(2)).astype(np.float32)


def _solver_step_dev(x, y, m):
    x.neg_().add_(1.0)
    y.mul_(0.5).add_(0.25)
    m.mul_(2.0)


@pytest.mark.parametrize("same_stream", [False, True])
@pytest.mark.parametrize("side,bounds", [(64, (0.0, 1.0, 0.0, 1.0)), (1024, (0.0, 1.0, 0.0, 1.0)), (256, None)])
def test_async_bins_the_copy_taken_at_call_time(side, bounds, same_stream):
    from paper_2310_02926_amd import binding as B
    _case(f"async side={side} bounds={'auto' if bounds is None else 'explicit'} same_stream={same_stream}")
    rng = np.random.default_rng(side)
    n = 1_500_001
    hx = rng.uniform(-0.1, 1.1, n).astype(np.float32)
    hy = rng.uniform(-0.1, 1.1, n).astype(np.float32)
    hm = rng.lognormal(0, 1, n).astype(np.float32)
    x, y, m = (torch.from_numpy(a).cuda() for a in (hx, hy, hm))
    src = torch.cuda.Stream()
    bs = src if same_stream else torch.cuda.Stream()
    a = torch.randn(4096, 4096, device="cuda")
    torch.cuda.synchronize()
    if not same_stream:
        with torch.cuda.stream(bs):  # hold the binning stream back
            for _ in range(12):
                a = (a @ a).clamp_(-1.0, 1.0)
    steps, outs, expect = 4, [], []
    with torch.cuda.stream(src):
        for _ in range(steps):
            _solver_step_dev(x, y, m)
            hx, hy, hm = _solver_step_host(hx, hy, hm)
            out = B.alloc_outputs([m], side, side, 31, "cuda")
            B.bin_particles_async([x, y], [m], n, (0, 1), bounds, side, side, 31, out, src_stream=src,
                                  bin_stream=bs)
            outs.append(out)
            expect.append(synth.Workload([hx.copy(), hy.copy()], [hm.copy()], bounds=bounds, nx=side, ny=side))
    torch.cuda.synchronize()
    for i, (out, ws) in enumerate(zip(outs, expect)):
        G.assert_parity(_to_np(out), G.oracle(ws), 31, what=f"async step {i}")
