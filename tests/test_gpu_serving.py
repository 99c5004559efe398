"""Serving loop (continuous batching) on the GPU, through the C ABI.

The key property: a request's results are the same alone (bls_search) and
in the mix of concurrently admitted requests, and match the FP64 oracle.
"""
import sys
import time

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


def _requests(nreq, seed, n_range=(200, 4000), np_range=(100, 1500),
              nbins_range=(100, 600), weighted_every=0):
    out = []
    for k, (_, lc) in enumerate(synth.serving_requests(
            nreq, 1000.0, seed=seed, n_range=n_range, np_range=np_range,
            nbins_range=nbins_range)):
        if weighted_every and k % weighted_every == 1:
            w = np.random.default_rng(k).uniform(0.5, 2.0, lc.n)
            lc = synth.LightCurve(lc.t, lc.x, w, lc.periods, lc.nbins,
                                  lc.qmin, lc.qmax, lc.truth)
        out.append(lc)
    return out


def _submit(bls, srv, lc):
    return bls.bls_server_submit(srv, lc.t, lc.x, lc.w, lc.periods, lc.nbins,
                                 lc.qmin, lc.qmax)


def test_mix_equals_alone_and_oracle(bls):
    reqs = _requests(24, 5151, weighted_every=4)
    _say("serving mix", len(reqs))
    srv = bls.bls_server_create(max_slots=16, arena_bytes=256 << 20,
                                tick_cost=2e7)
    try:
        tickets = [_submit(bls, srv, lc) for lc in reqs]
        res = [bls.bls_server_wait(srv, tk, 60.0) for tk in tickets]
        st = bls.bls_server_get_stats(srv)
    finally:
        bls.bls_server_destroy(srv)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["ticks"] > 1 and st["p99_ms"] >= st["p50_ms"] > 0
    with bls.Plan(max_points=1 << 16, max_periods=1 << 16) as p:
        for k, (lc, r) in enumerate(zip(reqs, res)):
            assert r["status"] == bls.BLS_OK
            alone = bls.bls_search(p.handle, lc.t, lc.x, lc.w, lc.periods,
                                   lc.nbins, lc.qmin, lc.qmax)
            # same kernel, same exact binning: bit-identical alone and in the mix
            assert np.array_equal(alone["sr"].astype(np.float32), r["sr"]), k
            assert np.array_equal(alone["jstart"], r["jstart"]), k
            assert np.array_equal(alone["kwidth"], r["kwidth"]), k
            assert alone["best_index"] == r["best_index"], k
            if k % 3 == 0:
                o = oracle.search(lc.t, lc.x, lc.w, lc.periods, lc.nbins,
                                  lc.qmin, lc.qmax)
                check_curve(lc, r, o, label="served %d" % k)


def _bytes(lc):
    up = lambda v: -(-v // 64) * 64
    return 40 * up(lc.n) + 24 * up(lc.periods.size)


def test_arena_takes_any_mix_of_shapes(bls):
    """Point-heavy and period-heavy requests share one byte budget: requests
    of 20000 points and 300 periods, then of 600 points and 30000 periods,
    each kind fitting only because neither region has a fixed share."""
    heavy_pts = [synth.small_curve(60 + k, 20000, nperiods=300, nbins=200,
                                   qmin=0.01, qmax=0.1) for k in range(4)]
    heavy_per = [synth.small_curve(70 + k, 600, nperiods=30000, nbins=200,
                                   qmin=0.01, qmax=0.1) for k in range(4)]
    arena = int(2.5 * max(_bytes(lc) for lc in heavy_pts + heavy_per))
    _say("arena mix", arena)
    srv = bls.bls_server_create(max_slots=8, arena_bytes=max(arena, 1 << 20))
    try:
        tickets = [_submit(bls, srv, lc) for lc in heavy_pts + heavy_per]
        res = [bls.bls_server_wait(srv, tk, 60.0) for tk in tickets]
        st = bls.bls_server_get_stats(srv)
    finally:
        bls.bls_server_destroy(srv)
    assert all(r["status"] == bls.BLS_OK for r in res)
    assert st["completed"] == len(tickets)
    assert st["device_bytes_peak"] <= max(arena, 1 << 20)
    for lc, r in zip([heavy_pts[0], heavy_per[-1]], [res[0], res[-1]]):
        o = oracle.search(lc.t, lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                          lc.qmax)
        check_curve(lc, r, o, label="arena mix")


def test_small_arena_queues_instead_of_failing(bls):
    reqs = _requests(10, 5252, n_range=(3000, 6000), np_range=(6000, 9000))
    # a resident request holds 40 B per point and 24 B per period; the arena
    # holds about two of the largest
    need = max(_bytes(lc) for lc in reqs)
    arena = max(int(need * 2.2), 1 << 20)   # the server's smallest arena
    assert arena < 4 * need
    _say("small arena", arena)
    srv = bls.bls_server_create(max_slots=8, arena_bytes=arena)
    try:
        tickets = [_submit(bls, srv, lc) for lc in reqs]
        st0 = bls.bls_server_get_stats(srv)
        assert st0["submitted"] == len(reqs)
        res = [bls.bls_server_wait(srv, tk, 60.0) for tk in tickets]
        st = bls.bls_server_get_stats(srv)
    finally:
        bls.bls_server_destroy(srv)
    assert all(r["status"] == bls.BLS_OK for r in res)
    assert st["completed"] == len(reqs)
    # admission never exceeded the arena
    assert st["device_bytes_peak"] <= arena


def test_errors_isolated(bls):
    reqs = _requests(4, 5353)
    _say("errors")
    srv = bls.bls_server_create(max_slots=4, arena_bytes=64 << 20,
                                max_request_points=5000)
    try:
        good = [_submit(bls, srv, lc) for lc in reqs if lc.n <= 5000]
        big = synth.small_curve(1, 6000, nperiods=10, nbins=100)
        with pytest.raises(bls.BlsError) as ei:
            _submit(bls, srv, big)
        assert ei.value.status == bls.BLS_ERR_CAPACITY
        bad = reqs[0]
        x = bad.x.copy()
        x[3] = np.inf
        with pytest.raises(bls.BlsError) as ei:
            bls.bls_server_submit(srv, bad.t, x, None, bad.periods, bad.nbins,
                                  bad.qmin, bad.qmax)
        assert ei.value.status == bls.BLS_ERR_INVALID_ARG
        with pytest.raises(bls.BlsError):
            bls.bls_server_poll(srv, 987654321)
        for tk in good:
            r = bls.bls_server_wait(srv, tk, 60.0)
            assert r["status"] == bls.BLS_OK
            assert bls.bls_server_poll(srv, tk) is not None
            bls.bls_server_release(srv, tk)
            with pytest.raises(bls.BlsError):
                bls.bls_server_poll(srv, tk)
        bls.bls_server_drain(srv, 10.0)
    finally:
        bls.bls_server_destroy(srv)


def test_open_loop_stream_reports_latency(bls):
    """Requests arrive on a Poisson clock while others run; all complete and
    the latency percentiles are reported."""
    reqs = list(synth.serving_requests(40, 400.0, seed=5454,
                                       n_range=(500, 5000),
                                       np_range=(2000, 20000),
                                       nbins_range=(200, 1000)))
    _say("open loop", len(reqs))
    srv = bls.bls_server_create(max_slots=64, arena_bytes=1 << 30)
    try:
        t0 = time.perf_counter()
        tickets = []
        for (t_arr, lc) in reqs:
            while time.perf_counter() - t0 < t_arr:
                time.sleep(0.0002)
            tickets.append(_submit(bls, srv, lc))
        bls.bls_server_drain(srv, 120.0)
        st = bls.bls_server_get_stats(srv)
        res = [bls.bls_server_poll(srv, tk) for tk in tickets]
    finally:
        bls.bls_server_destroy(srv)
    _say("stats", {k: st[k] for k in ("completed", "ticks", "p50_ms",
                                      "p99_ms", "busy_s", "wall_s")})
    assert st["completed"] == len(reqs)
    assert all(r is not None and r["status"] == 0 for r in res)
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    assert st["trial_points"] == pytest.approx(
        sum(lc.n * lc.periods.size for _, lc in reqs))


def test_result_pool_reuse_and_fallback(bls):
    """Finished requests hold blocks of the pinned result pool (half the
    arena) until released; a request finding no room gets its results
    copied into pageable memory instead.  With a 1 MiB arena the 512 KiB pool
    holds one of these requests' results at a time, so in each wave of three
    the first lands in the pool and the other two take the pageable path;
    releasing between waves lets the pool be reused.  Every result must be
    bit-identical to the same request searched alone."""
    reqs = _requests(9, 5353, n_range=(300, 800), np_range=(18000, 21000),
                     nbins_range=(100, 200), weighted_every=4)
    assert all(16 * lc.periods.size + 16 > (1 << 20) // 4 for lc in reqs)
    _say("result pool", len(reqs))
    srv = bls.bls_server_create(max_slots=4, arena_bytes=1 << 20)
    res = []
    try:
        for w in range(0, len(reqs), 3):
            tickets = [_submit(bls, srv, lc) for lc in reqs[w:w + 3]]
            res += [bls.bls_server_wait(srv, tk, 60.0) for tk in tickets]
            for tk in tickets:
                bls.bls_server_release(srv, tk)
        st = bls.bls_server_get_stats(srv)
    finally:
        bls.bls_server_destroy(srv)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    with bls.Plan(max_points=1 << 12, max_periods=1 << 15) as p:
        for k, (lc, r) in enumerate(zip(reqs, res)):
            assert r["status"] == bls.BLS_OK, k
            alone = bls.bls_search(p.handle, lc.t, lc.x, lc.w, lc.periods,
                                   lc.nbins, lc.qmin, lc.qmax)
            assert np.array_equal(alone["sr"].astype(np.float32), r["sr"]), k
            assert np.array_equal(alone["depth"].astype(np.float32),
                                  r["depth"], equal_nan=True), k
            assert np.array_equal(alone["jstart"], r["jstart"]), k
            assert np.array_equal(alone["kwidth"], r["kwidth"]), k
            assert alone["best_index"] == r["best_index"], k
