"""GPU tests of the MSM server (msm_server_*): admission by workspace
footprint, overlap on several streams, and results that are the same alone
and in the mix (bit for bit, and equal to the oracle's closed form)."""

import numpy as np
import pytest
import torch

from oracle import msm
from paper_2502_11660_amd import api, inputs, serve
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _dev(a):
    return api.to_device(a)


def _pool(pts):
    xyu, status = api.points_prepare(_dev(H.soa(pts, 2)), len(pts))
    assert int(api.to_host(status)[0]) == 0
    return xyu


def _requests(xyu_pool, npool, sizes, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs, meta = [], []
    for j, n in enumerate(sizes):
        n = int(n)
        off = int(rng.integers(0, npool - n + 1))
        sc = [inputs.words_to_int(r) for r in inputs.scalars_mod_r(seed + j, n)]
        jobs.append((xyu_pool[off * 36:(off + n) * 36], _dev(H.scalar_words(sc)),
                     api.words(api.MSM_RESULT_WORDS), n, 0))
        meta.append((off, sc))
    return jobs, meta


def test_server_queues_by_footprint_and_matches_alone(oracle_pool):
    ks, pts = oracle_pool
    xyu_pool = _pool(pts)
    sizes = [2048, 1000, 17, 1500, 300, 2048, 5, 800, 1200, 64] * 3
    jobs, meta = _requests(xyu_pool, len(pts), sizes, 9100)
    # a budget of about two large workspaces forces most requests to wait
    big = api.workspace_bytes(2048, api.default_window(2048))
    srv = api.Server(int(2.2 * big), streams=4)
    tickets = [srv.submit(*j) for j in jobs]
    assert tickets == list(range(1, len(jobs) + 1))
    inflight, queued, used = srv.stats()
    assert queued > 0 and used <= int(2.2 * big)
    srv.drain()
    done = srv.progress()
    assert sorted(done) == tickets
    assert srv.stats()[:2] == (0, 0)
    for (xyu, st, res, n, c), (off, sc) in zip(jobs, meta):
        alone = api.msm_run(xyu, st, n, c)
        assert np.array_equal(api.to_host(alone), api.to_host(res))
        assert api.decode_result(api.to_host(res)) == (msm.closed_form(sc, ks[off:off + n]), 0)
    # a request larger than the whole budget is refused, nothing queued
    with pytest.raises(api.MSMError):
        srv.submit(*jobs[0][:3], 2048, 16)
    assert srv.stats()[:2] == (0, 0)
    srv.destroy()


def test_served_trace_equals_plain_replay(oracle_pool):
    """A Poisson trace replayed through the server (overlapping requests) and
    by the plain path one at a time gives identical result words."""
    ks, pts = oracle_pool
    xyu_pool = _pool(pts)
    arrivals = inputs.poisson_arrivals(77, 3000.0, 0.02)
    nreq = len(arrivals)
    sizes = inputs.log_uniform_sizes(78, nreq, 4, 11)
    jobs, meta = _requests(xyu_pool, len(pts), sizes, 9300)
    srv = api.Server(1 << 30, streams=4)
    lat_s, wall_s = serve.replay_served(srv, arrivals, jobs)
    served = [api.to_host(j[2]).copy() for j in jobs]
    srv.destroy()
    for j in jobs:
        j[2].zero_()
    lat_p, wall_p = serve.replay_plain(arrivals, jobs)
    for k, ((xyu, st, res, n, c), (off, sc)) in enumerate(zip(jobs, meta)):
        assert np.array_equal(served[k], api.to_host(res)), k
        if k % 7 == 0:
            assert api.decode_result(served[k])[0] == msm.closed_form(sc, ks[off:off + n])
    assert np.all(np.isfinite(lat_s)) and np.all(lat_s > 0)
    s = serve.summarize(lat_s, wall_s, np.ones(nreq, dtype=bool))
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_server_request_waits_for_the_producer_stream(oracle_pool):
    """Inputs written on the caller's stream just before submission (behind
    other queued work, with no synchronisation) are what the request reads."""
    ks, pts = oracle_pool
    xyu_pool = _pool(pts)
    n = 1500
    sc = [inputs.words_to_int(r) for r in inputs.scalars_mod_r(9400, n)]
    src = _dev(H.scalar_words(sc))
    dst = torch.zeros_like(src)
    res = api.words(api.MSM_RESULT_WORDS)
    res.fill_(-1)
    busy = _dev(H.scalar_words([inputs.words_to_int(r) for r in inputs.scalars_mod_r(9401, 2048)]))
    torch.cuda.synchronize()
    srv = api.Server(1 << 28, streams=2)
    for _ in range(4):                      # work ahead of the producer's writes
        api.msm_run(xyu_pool[:2048 * 36], busy, 2048, 0)
    dst.copy_(src)
    srv.submit(xyu_pool[:n * 36], dst, res, n, 0)
    srv.drain()
    assert srv.progress() == [1]
    assert api.decode_result(api.to_host(res)) == (msm.closed_form(sc, ks[:n]), 0)
    srv.destroy()
