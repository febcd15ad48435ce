"""GPU parity of the field-multiplication cores compared in the benchmark
(Montgomery, Barrett, Karatsuba-Montgomery, lane-parallel Montgomery and the
carry-free 28-bit Montgomery core) against plain modular arithmetic: chained
products out = a b^rounds (times R^-rounds for the Montgomery forms, with
R = 2^384, or 2^392 for the 28-bit core)."""

import random

import numpy as np
import pytest

from oracle.field import P
from paper_2502_11660_amd import api
from tests import helpers as H

pytestmark = pytest.mark.gpu

R_INV = pow(1 << 384, -1, P)
R28_INV = pow(1 << 392, -1, P)


def _expected(variant, a, b, rounds):
    v = a * pow(b, rounds, P) % P
    if variant in (api.MSM_MUL_MONT, api.MSM_MUL_KARATSUBA, api.MSM_MUL_WIDE):
        v = v * pow(R_INV, rounds, P) % P
    if variant == api.MSM_MUL_F28:
        v = v * pow(R28_INV, rounds, P) % P
    return v


@pytest.mark.parametrize("variant", [api.MSM_MUL_MONT, api.MSM_MUL_BARRETT,
                                     api.MSM_MUL_KARATSUBA, api.MSM_MUL_WIDE, api.MSM_MUL_F28])
@pytest.mark.parametrize("rounds", [1, 7])
def test_fe_mul_chain_variants(variant, rounds):
    rng = random.Random(100 + variant * 10 + rounds)
    edge = [(0, 5), (1, 1), (P - 1, P - 1), (P - 1, 1), ((1 << 376) + 3, P - 2),
            (P - 1, (1 << 384) % P)]
    pairs = edge + [(rng.randrange(P), rng.randrange(P)) for _ in range(333 - len(edge))]
    n = len(pairs)
    a = api.to_device(H.soa([(x,) for x, _ in pairs], 1))
    b = api.to_device(H.soa([(y,) for _, y in pairs], 1))
    out = api.fe_mul_chain(a, b, n, variant, rounds)
    got = [v[0] for v in H.unsoa(api.to_host(out), 1, n)]
    for i, (x, y) in enumerate(pairs):
        assert got[i] == _expected(variant, x, y, rounds), (i, variant, rounds)


def test_fe_mul_chain_rejects_bad_arguments():
    a = api.to_device(np.zeros(12, dtype=np.uint32))
    with pytest.raises(api.MSMError):
        api.fe_mul_chain(a, a, 1, 9, 1)
    with pytest.raises(api.MSMError):
        api.fe_mul_chain(a, a, 1, api.MSM_MUL_MONT, 0)
