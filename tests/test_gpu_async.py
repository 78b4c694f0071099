"""randqlp_factor_async: the method enqueued without host synchronisation,
so that it can be captured into a HIP graph.  Checked against randqlp_factor
(bitwise: the same kernels on the fast path), inside a captured graph
replayed several times with eager work and synchronisations between the
replays, and for the device status words on a panel that breaks down."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import log, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rq():
    import paper_2110_01011_amd as rq
    rq.lib()
    return rq


def _same(a, b):
    return all(np.array_equal(to_np(x), to_np(y)) for x, y in zip(a, b))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_async_matches_factor(rq, dtype):
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    A, U, s, V = W.poly_decay(1500, 1200, 1.0, seed=71)
    Ad = to_dev(A, tdt)
    ref = rq.factor(Ad, 40, 10, 2, 5)
    Q, L, P, st = rq.factor_async(Ad, 40, 10, 2, 5)
    torch.cuda.synchronize()
    log(f"  async {dtype}: status {to_np(st).astype(int).tolist()}")
    assert int(st[0].item()) == 0
    assert _same((Q, L, P), ref)


def test_async_in_a_captured_graph(rq):
    import torch
    A, U, s, V = W.poly_decay(2000, 1600, 1.2, seed=72)
    Ad = to_dev(A)
    ref = rq.factor(Ad, 60, 10, 2, 9)
    af = rq.AsyncFactor(Ad, 60, 10, 2, 9)
    af.launch()                      # eager first call (one-time set-up)
    torch.cuda.synchronize()
    assert _same(af.launch()[:3], ref)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        af.launch()
    x = torch.randn(512, 512, device="cuda", dtype=torch.float64)
    for r in range(3):
        for t in (af.Q, af.L, af.P):
            t.zero_()
        af.status.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        log(f"  replay {r}: status {to_np(af.status).astype(int).tolist()}")
        assert int(af.status[0].item()) == 0
        assert _same((af.Q, af.L, af.P), ref)
        x = x @ x.T / 512.0          # eager work between the replays
        torch.cuda.synchronize()
    # the graph reads A's current values: 2 A gives 2 L and the same Q, P
    Ad.mul_(2.0)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    ref2 = rq.factor(Ad, 60, 10, 2, 9)
    assert _same((af.Q, af.L, af.P), ref2)
    assert np.array_equal(to_np(af.L), 2.0 * to_np(ref[1]))


def test_async_reports_a_breakdown(rq):
    """A zero matrix on the fast path: the pivot test fires and status[0]
    says so (factor() would rerun with the robust panels)."""
    import torch
    Z = np.zeros((120, 90))
    Q, L, P, st = rq.factor_async(to_dev(Z), 10, 2, 1, 0)
    torch.cuda.synchronize()
    log(f"  zero matrix: status {to_np(st).astype(int).tolist()}")
    assert int(st[0].item()) & 1
