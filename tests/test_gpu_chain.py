"""GPU parity of the paper's two PADD workloads outside an MSM: the dependent
addition chain (latency) and independent accumulation streams (throughput).
Expected values: the oracle's Edwards/Weierstrass sums of the same points,
and the closed form (sum k_i) G for points P_i = k_i G."""

import random

import numpy as np
import pytest

from oracle import curve, te
from oracle.field import P as FP, R_ORDER
from paper_2502_11660_amd import api
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _xytz_records(pts, seed):
    rng = random.Random(seed)
    recs = [H.te_extended_mont(te.w_to_te(p), rng.randrange(1, FP)) for p in pts]
    return api.to_device(H.aos(recs, 4))


def _sum_w(points):
    acc = curve.INF
    for p in points:
        acc = curve.add(acc, p)
    return acc


@pytest.mark.parametrize("unit", [api.MSM_UNIT_WIDE, api.MSM_UNIT_QUAD, api.MSM_UNIT_LANE])
def test_padd_chain_sum_and_edge_chains(oracle_pool, unit):
    ks, pts = oracle_pool
    n = 257
    out = api.padd_chain(_xytz_records(pts[:n], 11), n, unit)
    got = H.normalize_extended_mont(H.unaos(api.to_host(out), 4, 1)[0])
    want = curve.smul(sum(ks[:n]) % R_ORDER, curve.G)
    assert got == te.w_to_te(want)
    # one point; a point and its negative; the same point twice (doubling)
    p0, p1 = pts[0], pts[1]
    for chain in ([p0], [p0, curve.neg(p0)], [p1, p1, p0], [p0, curve.neg(p0), p1]):
        out = api.padd_chain(_xytz_records(chain, 5), len(chain), unit)
        got = H.normalize_extended_mont(H.unaos(api.to_host(out), 4, 1)[0])
        assert got == te.w_to_te(_sum_w(chain)), (unit, len(chain))


def test_padd_chain_rejects_bad_unit(oracle_pool):
    ks, pts = oracle_pool
    with pytest.raises(api.MSMError):
        api.padd_chain(_xytz_records(pts[:2], 1), 2, 7)


@pytest.mark.parametrize("n,A", [(1000, 37), (1000, 10), (64, 100), (2048, 1024), (2048, 1500),
                                 (1100, 2000)])
def test_accumulate_stream(oracle_pool, n, A):
    ks, pts = oracle_pool
    xy = H.soa(pts[:n], 2)
    xyu, status = api.points_prepare(api.to_device(xy), n)
    out = api.accumulate_stream(xyu, n, A)
    recs = H.unaos(api.to_host(out), 4, A)
    total = curve.INF
    for a in range(A):
        mine = [pts[i] for i in range(a, n, A)]
        got = H.normalize_extended_mont(recs[a])
        assert got == te.w_to_te(_sum_w(mine)), a
        total = curve.add(total, _sum_w(mine))
    assert total == curve.smul(sum(ks[:n]) % R_ORDER, curve.G)
