"""GPU parity of bucket accumulation and the full MSM against the oracle.

Inputs are seeded; points P_i = k_i G.  Expected values come from the oracle:
bucket sums by their definition, and the MSM either by the naive sum or by
the closed form ((sum s_i k_i) mod r) G (both pinned in test_oracle.py).
"""

import random

import numpy as np
import pytest
import torch

from oracle import curve, msm, te
from oracle.field import R_ORDER
from paper_2502_11660_amd import api, inputs
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _dev(a):
    return api.to_device(a)


def _prepared(pts):
    xy = H.soa([(0, 0) if p is None else p for p in pts], 2)
    inf = np.array([1 if p is None else 0 for p in pts], dtype=np.uint32)
    xyu, status = api.points_prepare(_dev(xy), len(pts), inf=_dev(inf))
    assert int(api.to_host(status)[0]) == 0
    return xyu


SIGNED, UNSIGNED = api.MSM_DIGITS_SIGNED, api.MSM_DIGITS_UNSIGNED


def _run(xyu, scalars, c, encoding=SIGNED):
    n = len(scalars)
    res = api.msm_run(xyu, _dev(H.scalar_words(scalars)), n, c, encoding)
    pt, flags = api.decode_result(api.to_host(res))
    return pt, flags


def test_bucket_accumulate_config1_unsigned(oracle_pool):
    """n = 1024, c = 8, plain slices: every bucket B[w][b] equals its definition."""
    ks, pts = oracle_pool
    n, c = 1024, 8
    sc = [inputs.words_to_int(r) for r in inputs.scalars_mod_r(inputs.config_seed(1), n)]
    xyu = _prepared(pts[:n])
    buckets, ws = api.bucket_accumulate(xyu, _dev(H.scalar_words(sc)), n, c, UNSIGNED)
    W = msm.num_windows(c)
    got = H.unaos(api.to_host(buckets), 4, W << c)
    want = msm.buckets(sc, pts[:n], c)
    for w in range(W):
        for b in range(1 << c):
            assert H.normalize_extended_mont(got[(w << c) + b]) == te.w_to_te(want[w][b]), (w, b)
    assert int(api.to_host(ws[:1])[0]) == 0


def test_bucket_accumulate_config1_signed(oracle_pool):
    """n = 1024, c = 8, signed digits: B[w][m] = signed sum of its points."""
    ks, pts = oracle_pool
    n, c = 1024, 8
    sc = [inputs.words_to_int(r) for r in inputs.scalars_mod_r(inputs.config_seed(1), n)]
    xyu = _prepared(pts[:n])
    buckets, ws = api.bucket_accumulate(xyu, _dev(H.scalar_words(sc)), n, c, SIGNED)
    W = msm.num_signed_windows(c)
    B = 1 << (c - 1)
    got = H.unaos(api.to_host(buckets), 4, W * B)
    want = msm.signed_buckets(sc, pts[:n], c)
    for w in range(W):
        for m in range(B):
            assert H.normalize_extended_mont(got[w * B + m]) == te.w_to_te(want[w][m]), (w, m)
    assert int(api.to_host(ws[:1])[0]) == 0


def test_msm_config1_closed_form_and_naive(oracle_pool):
    ks, pts = oracle_pool
    n, c = 1024, 8
    sc = [inputs.words_to_int(r) for r in inputs.scalars_mod_r(inputs.config_seed(1), n)]
    xyu = _prepared(pts[:n])
    for enc in (SIGNED, UNSIGNED):
        got, flags = _run(xyu, sc, c, enc)
        assert flags == 0
        assert got == msm.closed_form(sc, ks[:n])
        # direct definition on a prefix
        m = 48
        got_m, _ = _run(_prepared(pts[:m]), sc[:m], c, enc)
        assert got_m == msm.msm_naive(sc[:m], pts[:m])


@pytest.mark.parametrize("c", [1, 2, 3, 5, 7, 10, 11, 12, 13, 16, 17])
def test_msm_window_widths(oracle_pool, c):
    ks, pts = oracle_pool
    n = 200 + 37 * c
    sc = [inputs.words_to_int(r) for r in inputs.scalars_mod_r(1000 + c, n)]
    xyu = _prepared(pts[:n])
    for enc in ((UNSIGNED,) if c == 1 else (SIGNED, UNSIGNED)):
        got, flags = _run(xyu, sc, c, enc)
        assert flags == 0
        assert got == msm.closed_form(sc, ks[:n]), enc


@pytest.mark.parametrize("n", [1, 2, 31, 32, 33, 65, 1000])
def test_msm_ragged_sizes(oracle_pool, n):
    ks, pts = oracle_pool
    sc = [inputs.words_to_int(r) for r in inputs.scalars_mod_r(77 + n, n)]
    got, _ = _run(_prepared(pts[:n]), sc, 8)
    assert got == msm.closed_form(sc, ks[:n])


def test_msm_degenerate_scalars(oracle_pool):
    ks, pts = oracle_pool
    n = 300
    xyu = _prepared(pts[:n])
    # all zero -> point at infinity
    got, _ = _run(xyu, [0] * n, 8)
    assert got is None
    # every slice at its maximum: signed recoding carries through all windows;
    # at c = 2 the top window reaches the largest digit 2^(c-1)
    top = (1 << 253) - 1
    for c in (11, 2):
        got, _ = _run(xyu, [top] * n, c)
        assert got == msm.closed_form([top] * n, ks[:n]), c
    # slices at exactly 2^(c-1), the recoding boundary
    half = sum(1 << (w * 8 + 7) for w in range(31))
    got, _ = _run(xyu, [half] * n, 8)
    assert got == msm.closed_form([half] * n, ks[:n])
    # all equal: every point in the same bucket of every window (skew)
    s = 0x1234567890ABCDEF1234567890ABCDEF1234567890ABCDEF1234567890ABCDE % R_ORDER
    got, _ = _run(xyu, [s] * n, 8)
    assert got == msm.closed_form([s] * n, ks[:n])
    # extremes: r - 1, 2^253 - 1 (>= r, still valid input), 1
    sc = [R_ORDER - 1, (1 << 253) - 1, 1] * (n // 3)
    got, flags = _run(xyu, sc, 8)
    assert flags == 0
    assert got == msm.closed_form(sc, ks[:n])
    # cancellation: s and r - s on the same point -> infinity
    sc2 = [5, R_ORDER - 5]
    got, _ = _run(_prepared([pts[0], pts[0]]), sc2, 4)
    assert got is None


def test_msm_scalar_out_of_range_flagged(oracle_pool):
    ks, pts = oracle_pool
    n = 16
    sc = [random.Random(i).randrange(R_ORDER) for i in range(n)]
    sc[3] |= 1 << 254
    got, flags = _run(_prepared(pts[:n]), sc, 8)
    assert flags & api.MSM_FLAG_RANGE
    trunc = [s & ((1 << 253) - 1) for s in sc]
    assert got == msm.closed_form(trunc, ks[:n])


def test_msm_with_identity_points(oracle_pool):
    ks, pts = oracle_pool
    sel = [pts[0], curve.INF, pts[1], curve.INF]
    sc = [3, 5, 7, 11]
    got, _ = _run(_prepared(sel), sc, 3)
    assert got == msm.msm_naive(sc, sel)


def test_msm_point_order_and_repeat_invariance(oracle_pool):
    ks, pts = oracle_pool
    n = 513
    sc = [inputs.words_to_int(r) for r in inputs.scalars_mod_r(4242, n)]
    perm = list(range(n))
    random.Random(1).shuffle(perm)
    a, _ = _run(_prepared(pts[:n]), sc, 9)
    b, _ = _run(_prepared([pts[i] for i in perm]), [sc[i] for i in perm], 9)
    c2, _ = _run(_prepared(pts[:n]), sc, 9)
    assert a == b == c2 == msm.closed_form(sc, ks[:n])


@pytest.mark.parametrize("c", [16, 17])
def test_msm_full_size_closed_form(c):
    """n = 2^20 GPU-generated points (checked on a sample), closed form."""
    n = 1 << 20
    seed = inputs.config_seed(3)
    kw = inputs.nonzero_scalars_mod_r(seed, n, stream=1)
    sw = inputs.scalars_mod_r(seed, n, stream=2)
    xy, inf = api.gen_points(_dev(kw), n)
    xyu, status = api.points_prepare(xy, n, inf=inf)
    res = api.msm_run(xyu, _dev(sw), n, c)
    torch.cuda.synchronize()
    got, flags = api.decode_result(api.to_host(res))
    assert flags == 0 and int(api.to_host(status)[0]) == 0
    ks = [inputs.words_to_int(r) for r in kw]
    ss = [inputs.words_to_int(r) for r in sw]
    assert got == msm.closed_form(ss, ks)
    # sample of the generated points against the oracle
    from oracle import points
    rows = H.unsoa(api.to_host(xy).reshape(24, n)[:, :64].reshape(-1), 2, 64)
    for i in range(0, 64, 8):
        assert rows[i] == points.fixed_base_mul(ks[i])


def test_msm_run_on_two_streams_at_once(oracle_pool):
    """msm_run is reentrant given distinct workspaces: two MSMs of different
    sizes and encodings, each on its own stream with its own workspace,
    enqueued back to back with no synchronisation between them, both equal
    to the closed form (and to the same calls made one at a time)."""
    ks, pts = oracle_pool
    npool = len(pts)
    xs = _prepared(pts)
    jobs = []
    for t, (n, c, enc) in enumerate(((1 << 16, 13, SIGNED), (3 << 14, 11, UNSIGNED))):
        sc = [inputs.words_to_int(r) for r in inputs.scalars_mod_r(8800 + t, n)]
        jobs.append((n, c, enc, sc, xs.repeat(n // npool), _dev(H.scalar_words(sc)),
                     api.workspace(n, c, enc), api.words(api.MSM_RESULT_WORDS)))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for _ in range(3):
        for st, (n, c, enc, sc, x, sd, ws, res) in zip(streams, jobs):
            with torch.cuda.stream(st):
                api.msm_run(x, sd, n, c, enc, result=res, ws=ws)
    torch.cuda.synchronize()
    for (n, c, enc, sc, x, sd, ws, res) in jobs:
        sel_k = [ks[i % npool] for i in range(n)]
        got, flags = api.decode_result(api.to_host(res))
        assert flags == 0 and got == msm.closed_form(sc, sel_k), (n, c, enc)
        alone = api.msm_run(x, sd, n, c, enc)
        assert np.array_equal(api.to_host(alone), api.to_host(res)), (n, c, enc)


@pytest.mark.parametrize("n,c,enc", [
    ((1 << 21) + 777, 16, api.MSM_DIGITS_GLV),
    ((1 << 22), 16, api.MSM_DIGITS_GLV),
    ((1 << 23), 20, SIGNED),
    ((1 << 26) - 1, 16, api.MSM_DIGITS_GLV),
])
def test_msm_large_jobs(n, c, enc):
    """Jobs whose sort takes groups of tiles (one pass-1 histogram per group).
    On a 256-CU device: n = 2^21 + 777 with the endomorphism split at c' = 16,
    2^11 partitions a window and groups of 16 tiles, the last group of each
    window holding only 1554 entries; n = 2^22 with the split at c' = 16,
    groups of 16 tiles and 2^11 partitions of ~4096 entries (LDS path);
    n = 2^23 with signed digits at c = 20, groups of 16 tiles over 13 windows;
    n = 2^26 - 1, the largest job the interface takes, with the split at
    c' = 16: 2^30 - 16 digit slots (entry positions, keys and indices are
    32-bit words), groups of 32 tiles, 2^12 partitions of ~32 K entries per
    window, all on the many-block sort, and 5464-entry accumulation chunks
    (device memory: about 50 GB).  k_i and s_i are drawn
    uniformly below 2^252 with numpy (no rejection step, which would take a
    minute at this size); the result is checked against the closed form,
    summed exactly with float64 digit products (oracle.msm.dot_mod_r)."""
    rng = np.random.default_rng(inputs.config_seed(3) + n % 1000 + c)
    kw = rng.integers(0, 1 << 32, size=(n, 8), dtype=np.uint32)
    kw[:, 7] &= 0x0FFFFFFF
    kw[:, 0] |= 1
    sw = rng.integers(0, 1 << 32, size=(n, 8), dtype=np.uint32)
    sw[:, 7] &= 0x0FFFFFFF
    k_dev = _dev(kw)
    xy, inf = api.gen_points(k_dev, n)
    del k_dev
    xyu, status = api.points_prepare(xy, n, inf=inf, endo=enc == api.MSM_DIGITS_GLV)
    del xy, inf
    s_dev = _dev(sw)
    res = api.msm_run(xyu, s_dev, n, c, enc)
    got, flags = api.decode_result(api.to_host(res))
    ok_status = int(api.to_host(status)[0]) == 0
    del xyu, s_dev
    torch.cuda.empty_cache()
    assert flags == 0 and ok_status
    assert got == msm.closed_form_words(sw, kw)


def test_msm_skewed_partition_larger_than_lds_stage(oracle_pool):
    """All scalars equal at n = 20000: one bucket per window holds every entry,
    so the sort's partition exceeds its LDS stage and the accumulation's
    split-bucket tree runs (spans of hundreds of chunks)."""
    ks, pts = oracle_pool
    n = 20000
    sel_k = [ks[i % len(ks)] for i in range(n)]
    sel_p = [pts[i % len(pts)] for i in range(n)]
    s = 0x0123456789ABCDEF0123456789ABCDEF0123456789ABCDEF0123456789ABCDE % R_ORDER
    xyu = _prepared(sel_p)
    for c, enc in ((8, SIGNED), (13, SIGNED), (8, UNSIGNED)):
        got, _ = _run(xyu, [s] * n, c, enc)
        assert got == msm.closed_form([s] * n, sel_k), c
    # half the scalars equal, half random: mixed bucket sizes
    sc = [s if i % 2 else inputs.words_to_int(r)
          for i, r in enumerate(inputs.scalars_mod_r(99, n))]
    got, _ = _run(xyu, sc, 11)
    assert got == msm.closed_form(sc, sel_k)


def test_msm_partition_at_the_lds_stage_boundary(oracle_pool):
    """Equal scalars put all n entries of a window into one bucket and one sort
    partition: n = 5120 is the largest partition of the short register form
    of pass 2 and 5121 the smallest of the long one; n = 10240 fills the
    pass-2 LDS stage exactly (the one-block path), n = 10241 is one entry over
    it (the many-block path)."""
    ks, pts = oracle_pool
    s = 0x0123456789ABCDEF0123456789ABCDEF0123456789ABCDEF0123456789ABCDE % R_ORDER
    for n in (5120, 5121, 10240, 10241):
        sel_k = [ks[i % len(ks)] for i in range(n)]
        xyu = _prepared([pts[i % len(pts)] for i in range(n)])
        for c, enc in ((8, UNSIGNED), (9, SIGNED)):
            got, flags = _run(xyu, [s] * n, c, enc)
            assert flags == 0 and got == msm.closed_form([s] * n, sel_k), (n, c)


@pytest.mark.parametrize("c", [10, 13])
def test_msm_quarter_million_closed_form(c):
    """n = 2^18 GPU-generated points; c = 10 / 13 split digits into 6+4 / 6+7 bits."""
    n = 1 << 18
    seed = inputs.config_seed(3) + c
    kw = inputs.nonzero_scalars_mod_r(seed, n, stream=3)
    sw = inputs.scalars_mod_r(seed, n, stream=4)
    xy, inf = api.gen_points(_dev(kw), n)
    xyu, status = api.points_prepare(xy, n, inf=inf)
    res = api.msm_run(xyu, _dev(sw), n, c)
    got, flags = api.decode_result(api.to_host(res))
    assert flags == 0 and int(api.to_host(status)[0]) == 0
    ks = [inputs.words_to_int(r) for r in kw]
    ss = [inputs.words_to_int(r) for r in sw]
    assert got == msm.closed_form(ss, ks)
