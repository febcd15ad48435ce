"""The allocation-free MSM entry point (msm_run_noalloc) against msm_run on
the same inputs: consecutive calls, each later one smaller than the one
before (the scratch keeps the previous call's contents), every result equal
bit for bit to msm_run's and to the oracle's closed form; requests larger
than the scratch are refused."""

import numpy as np
import pytest

from oracle import msm
from paper_2502_11660_amd import api, inputs
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _prepared(pts, endo):
    xyu, status = api.points_prepare(api.to_device(H.soa(pts, 2)), len(pts), endo=endo)
    assert int(api.to_host(status)[0]) == 0
    return xyu


@pytest.mark.parametrize("enc", [api.MSM_DIGITS_SIGNED, api.MSM_DIGITS_UNSIGNED,
                                 api.MSM_DIGITS_GLV])
def test_noalloc_equals_msm_run(oracle_pool, enc):
    ks, pts = oracle_pool
    npool = len(pts)
    rec = 2 if enc == api.MSM_DIGITS_GLV else 1
    xyu = _prepared(pts, enc == api.MSM_DIGITS_GLV)
    reps = (1 << 16) // npool
    big = xyu.repeat(reps)                      # 2^16 points: the pool tiled
    res = api.words(api.MSM_RESULT_WORDS)
    for t, (n, c) in enumerate(((1 << 16, 0), (1500, 9), (300, 5))):
        sw = inputs.scalars_mod_r(9500 + enc, n, stream=t)
        sd = api.to_device(sw)
        x = big[:rec * n * 36]
        want = api.msm_run(x, sd, n, c, enc)
        got = api.msm_run_noalloc(x, sd, n, c, enc, result=res)
        assert np.array_equal(api.to_host(want), api.to_host(got)), (n, c)
        kk = [ks[i % npool] for i in range(n)]
        ss = [inputs.words_to_int(r) for r in sw]
        assert api.decode_result(api.to_host(got)) == (msm.closed_form(ss, kk), 0)


def test_noalloc_refuses_more_than_the_scratch(oracle_pool):
    ks, pts = oracle_pool
    xyu = _prepared(pts, False).repeat(1 << 8)   # 2^19 points
    n = 1 << 19
    assert api.workspace_bytes(n, 16) > api._lib.MSM_NOALLOC_SCRATCH_BYTES
    sd = api.to_device(inputs.scalars_mod_r(9600, n))
    with pytest.raises(api.MSMError):
        api.msm_run_noalloc(xyu, sd, n, 16)


def test_noalloc_under_graph_capture(oracle_pool):
    """The callers the entry point is for include code under HIP graph
    capture: msm_run_noalloc recorded once in a graph (torch.cuda.graph) and
    replayed three times, new scalars copied into the captured scalar buffer
    before each replay and the program's own work and synchronisation between
    replays; every replay's result equals the closed form of its scalars and
    msm_run's result for them."""
    import torch
    ks, pts = oracle_pool
    npool = len(pts)
    n, c, enc = 1 << 14, 0, api.MSM_DIGITS_SIGNED
    xyu = _prepared(pts, False).repeat(n // npool)
    sd = api.to_device(inputs.scalars_mod_r(9700, n))
    res = api.words(api.MSM_RESULT_WORDS)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # first call on this GPU outside the capture
        api.msm_run_noalloc(xyu, sd, n, c, enc, result=res)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        api.msm_run_noalloc(xyu, sd, n, c, enc, result=res)
    kk = [ks[i % npool] for i in range(n)]
    for rep in range(3):
        sw = inputs.scalars_mod_r(9710 + rep, n)
        sd.copy_(api.to_device(sw))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ss = [inputs.words_to_int(r) for r in sw]
        assert api.decode_result(api.to_host(res)) == (msm.closed_form(ss, kk), 0), rep
        want = api.msm_run(xyu, sd, n, c, enc)
        torch.cuda.synchronize()
        assert np.array_equal(api.to_host(want), api.to_host(res)), rep
