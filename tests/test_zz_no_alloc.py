"""The plan-free entry point (bls_search_device_noalloc) on the GPU.

It allocates nothing and works in the library's fixed per-GPU scratch array;
its results must equal bls_search_device's on the same batch (and so the
FP64 oracle's, by the acceptance rule).  Two calls in a row on one stream,
the second with a smaller batch, are checked; the first batch has more
curves than one descriptor launch carries and weights, the second unit
weights.  Limits are rejected on the host.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.parity import check_curve

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bls():
    import paper_1112_1701_amd as bls
    bls._lib.load()
    return bls


def _nres(b):
    return int(b.p_off[-1]) if b.p_off is not None else \
        b.ncurves * b.periods.size


def _device(b):
    import torch
    dev = torch.device("cuda:0")
    m = _nres(b)
    ins = dict(t=torch.tensor(b.t, device=dev), x=torch.tensor(b.x, device=dev),
               w=None if b.w is None else torch.tensor(b.w, device=dev),
               per=torch.tensor(b.periods, device=dev))
    outs = [torch.full((m,), -7.0, device=dev, dtype=torch.float32),
            torch.full((m,), -7.0, device=dev, dtype=torch.float32),
            torch.full((m,), -9, device=dev, dtype=torch.int32),
            torch.full((m,), -9, device=dev, dtype=torch.int32),
            torch.full((b.ncurves,), -9, device=dev, dtype=torch.int64)]
    return ins, outs


def _with_plan(bls, b):
    """The same batch through bls_search_device (untuned tile table)."""
    ins, outs = _device(b)
    with bls.Plan(max_curves=b.ncurves, max_points=b.total_points(),
                  max_periods=_nres(b), flags=bls.BLS_NO_AUTOTUNE) as p:
        bls.bls_search_device(p.handle, b.n_off, ins["t"], ins["x"], ins["w"],
                              ins["per"], b.p_off, b.nbins, b.qmin, b.qmax,
                              *outs)
        bls.bls_synchronize(p.handle)
    return [o.cpu().numpy() for o in outs]


def test_noalloc_equals_device_call_twice(bls):
    import torch
    big = synth.uneven_batch(20, 91, n_range=(100, 20000), np_range=(200, 1500),
                             nbins_range=(64, 600))
    small = synth.uniform_batch(5, 800, 300, 200, seed=92)
    assert big.ncurves > 16 and big.total_points() <= bls.BLS_NOALLOC_MAX_POINTS
    assert small.total_points() < big.total_points()
    dev = [_device(b) for b in (big, small)]
    s = torch.cuda.Stream()
    _say("noalloc: two calls on one stream, %d then %d points"
         % (big.total_points(), small.total_points()))
    with torch.cuda.stream(s):
        for b, (ins, outs) in zip((big, small), dev):
            bls.bls_search_device_noalloc(
                b.n_off, ins["t"], ins["x"], ins["w"], ins["per"], b.p_off,
                b.nbins, b.qmin, b.qmax, *outs, stream=s)
    s.synchronize()
    got = [[o.cpu().numpy() for o in outs] for _, outs in dev]
    for k, b in enumerate((big, small)):
        _say("noalloc: plan call for batch", k)
        ref = _with_plan(bls, b)
        for name, g, r in zip(("sr", "depth", "jstart", "kwidth", "best"),
                              got[k], ref):
            assert np.array_equal(g, r, equal_nan=True), \
                "batch %d: %s differs from bls_search_device" % (k, name)
        sr, dp, js, ks, bi = got[k]
        for c in (0, b.ncurves // 2, b.ncurves - 1):
            lc = b.curve(c)
            a = int(b.p_off[c]) if b.p_off is not None else c * b.periods.size
            e = a + lc.periods.size
            o = oracle.search(lc.t, lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                              lc.qmax)
            check_curve(lc, dict(sr=sr[a:e], depth=dp[a:e], jstart=js[a:e],
                                 kwidth=ks[a:e], best_index=bi[c]), o,
                        label="noalloc batch %d curve %d" % (k, c))


def test_noalloc_limits(bls):
    import torch
    _say("noalloc: limits")
    b = synth.uniform_batch(bls.BLS_NOALLOC_MAX_CURVES + 1, 50, 10, 64, seed=93)
    ins, outs = _device(b)
    with pytest.raises(bls.BlsError) as e:
        bls.bls_search_device_noalloc(b.n_off, ins["t"], ins["x"], ins["w"],
                                      ins["per"], b.p_off, b.nbins, b.qmin,
                                      b.qmax, *outs)
    assert e.value.status == bls.BLS_ERR_CAPACITY
    with pytest.raises(bls.BlsError) as e:
        bls.bls_search_device_noalloc(b.n_off[:3], ins["t"], ins["x"], None,
                                      ins["per"], None, 64, 0.01, 0.1, *outs,
                                      flags=bls.BLS_NO_GRAPH)
    assert e.value.status == bls.BLS_ERR_INVALID_ARG
    torch.cuda.synchronize()
    # nothing was queued: the outputs keep their fill values
    assert float(outs[0][0].item()) == -7.0
