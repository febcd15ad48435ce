"""GPU parity of the endomorphism split (MSM_DIGITS_GLV): prepared images
phi(P) against the oracle's map, buckets of the split MSM against their
definition, and MSM results against the closed form and the naive sum."""

import numpy as np
import pytest
import torch

from oracle import curve, glv, msm, te
from oracle.field import R_ORDER
from paper_2502_11660_amd import api, inputs
from tests import helpers as H

pytestmark = pytest.mark.gpu
GLV = api.MSM_DIGITS_GLV


def _dev(a):
    return api.to_device(a)


def _prepared_endo(pts):
    xy = H.soa([(0, 0) if p is None else p for p in pts], 2)
    inf = np.array([1 if p is None else 0 for p in pts], dtype=np.uint32)
    xyu, status = api.points_prepare(_dev(xy), len(pts), inf=_dev(inf), endo=True)
    assert int(api.to_host(status)[0]) == 0
    return xyu


def _run(xyu, scalars, c):
    res = api.msm_run(xyu, _dev(H.scalar_words(scalars)), len(scalars), c, GLV)
    return api.decode_result(api.to_host(res))


def test_prepare_endo_records(oracle_pool):
    ks, pts = oracle_pool
    sel = pts[:100] + [curve.INF]
    n = len(sel)
    recs = H.unaos(api.to_host(_prepared_endo(sel)), 3, 2 * n)
    plain = H.unaos(api.to_host(api.points_prepare(_dev(H.soa([(0, 0) if p is None else p
                                                               for p in sel], 2)), n,
                                                   inf=_dev(np.array([p is None for p in sel],
                                                                     dtype=np.uint32)))[0]), 3, n)
    for i, pt in enumerate(sel):
        assert recs[2 * i] == plain[i]
        assert recs[2 * i + 1] == H.te_prepared_mont(te.w_to_te(glv.phi(pt))), i


@pytest.mark.parametrize("c", [2, 5, 8, 13, 16])
def test_glv_msm_widths(oracle_pool, c):
    ks, pts = oracle_pool
    n = 150 + 41 * c
    sc = [inputs.words_to_int(r) for r in inputs.scalars_mod_r(3000 + c, n)]
    got, flags = _run(_prepared_endo(pts[:n]), sc, c)
    assert flags == 0 and got == msm.closed_form(sc, ks[:n])


def test_glv_msm_degenerate_and_naive(oracle_pool):
    ks, pts = oracle_pool
    L = glv.LAMBDA
    edge = [0, 1, L - 1, L, L + 1, 2 * L, L * L, R_ORDER - 1, (1 << 253) - 1,
            (L + 1) * L, (L + 1) * L + L - 1]
    n = len(edge)
    got, _ = _run(_prepared_endo(pts[:n]), edge, 8)
    assert got == msm.msm_naive(edge, pts[:n])
    got, _ = _run(_prepared_endo(pts[:40]), [0] * 40, 7)
    assert got is None
    # identity points and a cancelling pair
    sel = [pts[0], curve.INF, pts[0]]
    got, _ = _run(_prepared_endo(sel), [5, 9, R_ORDER - 5], 4)
    assert got is None


def test_glv_buckets_match_definition(oracle_pool):
    ks, pts = oracle_pool
    n, c = 300, 6
    sc = [inputs.words_to_int(r) for r in inputs.scalars_mod_r(3100, n)]
    xyu = _prepared_endo(pts[:n])
    buckets, ws = api.bucket_accumulate(xyu, _dev(H.scalar_words(sc)), n, c, GLV)
    sc2, pts2 = glv.msm_split(sc, pts[:n])   # interleaved like the records
    W = msm.num_signed_windows(c, glv.SPLIT_BITS)
    B = 1 << (c - 1)
    assert W == api.num_windows(c, GLV)
    want = msm.signed_buckets(sc2, pts2, c, glv.SPLIT_BITS)
    got = H.unaos(api.to_host(buckets), 4, W * B)
    for w in range(W):
        for m in range(B):
            assert H.normalize_extended_mont(got[w * B + m]) == te.w_to_te(want[w][m]), (w, m)


def test_glv_batch_and_server(oracle_pool):
    ks, pts = oracle_pool
    sizes = [1, 33, 500, 2000, 700]
    offs = [5, 0, 1000, 0, 1300]
    pool = _prepared_endo(pts[:2048])
    jobs, meta = [], []
    for j, (n, o) in enumerate(zip(sizes, offs)):
        # slices of the interleaved records are the records of the slice
        xyu = pool[2 * o * 36:2 * (o + n) * 36]
        sc = [inputs.words_to_int(r) for r in inputs.scalars_mod_r(3200 + j, n)]
        jobs.append((xyu, _dev(H.scalar_words(sc)), api.words(api.MSM_RESULT_WORDS), n, 0))
        meta.append((o, sc))
    b = api.Batch(jobs, api.MSM_DIGITS_GLV, use_graph=True)
    b.run()
    torch.cuda.synchronize()
    for (x, s, r, n, c), (o, sc) in zip(jobs, meta):
        assert api.decode_result(api.to_host(r)) == (msm.closed_form(sc, ks[o:o + n]), 0), n
    b.destroy()
    srv = api.Server(1 << 30, streams=2, encoding=GLV)
    for job in jobs:
        job[2].zero_()
        srv.submit(*job)
    srv.drain()
    for (x, s, r, n, c), (o, sc) in zip(jobs, meta):
        assert api.decode_result(api.to_host(r)) == (msm.closed_form(sc, ks[o:o + n]), 0), n
    srv.destroy()


@pytest.mark.parametrize("c", [16])
def test_glv_full_size_closed_form(c):
    n = 1 << 20
    seed = inputs.config_seed(3)
    kw = inputs.nonzero_scalars_mod_r(seed, n, stream=1)
    sw = inputs.scalars_mod_r(seed, n, stream=2)
    xy, inf = api.gen_points(_dev(kw), n)
    xyu, status = api.points_prepare(xy, n, inf=inf, endo=True)
    res = api.msm_run(xyu, _dev(sw), n, c, GLV)
    got, flags = api.decode_result(api.to_host(res))
    assert flags == 0 and int(api.to_host(status)[0]) == 0
    ks = [inputs.words_to_int(r) for r in kw]
    ss = [inputs.words_to_int(r) for r in sw]
    assert got == msm.closed_form(ss, ks)


def test_glv_sparse_top_window_large_partitions():
    """n = 2^15 with c = 10: the top window keeps 8 digit bits, so its 2^16
    entries crowd about 120 of 512 buckets and each of its first sort
    partitions (32 buckets) holds ~16k entries, above the LDS stage of the sort (7168 entries):
    the many-block path (several items per partition, many buckets) runs."""
    n = 1 << 15
    seed = inputs.config_seed(4)
    kw = inputs.nonzero_scalars_mod_r(seed, n, stream=5)
    sw = inputs.scalars_mod_r(seed, n, stream=6)
    xy, inf = api.gen_points(_dev(kw), n)
    xyu, status = api.points_prepare(xy, n, inf=inf, endo=True)
    res = api.msm_run(xyu, _dev(sw), n, 10, GLV)
    got, flags = api.decode_result(api.to_host(res))
    assert flags == 0 and int(api.to_host(status)[0]) == 0
    ks = [inputs.words_to_int(r) for r in kw]
    ss = [inputs.words_to_int(r) for r in sw]
    assert got == msm.closed_form(ss, ks)
