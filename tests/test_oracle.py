"""Pins for the CPU oracle: what the mathematics and the curve definition fix.

Each check is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, a swapped operand, a wrong constant) fails at least one of them.
None of them re-types the formula it checks.
"""

import random

import numpy as np
import pytest

from oracle import curve, field, glv, msm, points, te
from oracle.field import P, R_ORDER
from paper_2502_11660_amd import inputs
from tests.golden.fixtures import read_kv

RNG = random.Random(1234)


def is_probable_prime(n, rounds=32):
    if n < 2:
        return False
    for q in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29):
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    rng = random.Random(n & 0xFFFF)
    for _ in range(rounds):
        a = rng.randrange(2, n - 2)
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def random_curve_point(rng=RNG):
    """A point on y^2 = x^3 + 1 found by trying random x (not necessarily in G1)."""
    while True:
        x = rng.randrange(P)
        rhs = (x ** 3 + 1) % P
        if field.is_square(rhs):
            y = field.fsqrt(rhs)
            if rng.random() < 0.5:
                y = (-y) % P
            return (x, y)


def random_g1_point(rng=RNG):
    return points.fixed_base_mul(rng.randrange(1, R_ORDER))


# --------------------------------------------------------------------------
# constants
# --------------------------------------------------------------------------

def test_constants_match_published_curve():
    g = read_kv("bls12_377_g1.txt")
    assert field.X0 == g["x0"]
    assert P == g["p"]
    assert R_ORDER == g["r"]
    assert field.COFACTOR == g["h"]
    assert (field.A_W, field.B_W) == (g["a"], g["b"])
    assert (field.G_X, field.G_Y) == (g["gx"], g["gy"])


def test_field_orders_prime_and_sized():
    assert is_probable_prime(P)
    assert is_probable_prime(R_ORDER)
    assert P.bit_length() == 377
    assert R_ORDER.bit_length() == 253
    assert field.COFACTOR * R_ORDER == P + 1 - field.TRACE


def test_two_adicity_and_montgomery_word_factor():
    # p = 1 (mod 2^46) makes the low word of p equal to 1 and n' = -1 mod 2^32.
    v, q = 0, P - 1
    while q % 2 == 0:
        q //= 2
        v += 1
    assert v == 46
    assert field.to_limbs(P)[0] == 1
    assert field.N_PRIME_32 == 0xFFFFFFFF
    assert (P * field.N_PRIME_32 + 1) % (1 << 32) == 0


def test_montgomery_constants():
    assert field.R_MONT == 1 << 384
    assert field.R_MONT * field.R_MONT_INV % P == 1
    assert field.R2_MONT == pow(2, 768, P)
    assert (1 << 384) // P == 152


def test_generator_on_curve_and_order_r():
    assert curve.on_curve(curve.G)
    assert curve.smul(R_ORDER, curve.G) is curve.INF
    assert curve.smul(R_ORDER - 1, curve.G) == curve.neg(curve.G)


def test_group_order_kills_random_point():
    q = random_curve_point(random.Random(7))
    assert curve.smul(field.COFACTOR * R_ORDER, q) is curve.INF
    # a random curve point lies outside G1 (h > 1), and the subgroup test sees it
    assert not curve.in_subgroup(q)
    # cofactor clearing lands in G1, at a point other than the identity
    g1 = curve.smul(field.COFACTOR, q)
    assert g1 is not curve.INF
    assert curve.in_subgroup(g1)


def test_inputs_module_bounds_are_the_curve_orders():
    assert inputs.SCALAR_FIELD_ORDER == R_ORDER
    assert inputs.BASE_FIELD_ORDER == P


# --------------------------------------------------------------------------
# field
# --------------------------------------------------------------------------

def test_sqrt_and_inverse():
    for _ in range(20):
        a = RNG.randrange(1, P)
        s = field.fsqrt(a * a)
        assert s * s % P == a * a % P
        assert s <= P - s
        assert field.finv(a) * a % P == 1
        # Fermat's little theorem gives the same inverse
        assert field.finv(a) == pow(a, P - 2, P)
    for a in (1, 2, P - 1, (P + 1) // 2, 1 << 376):
        assert field.finv(a) == pow(a, P - 2, P)
    with pytest.raises(ZeroDivisionError):
        field.finv(0)
    # 3 is a square (needed by the twisted-Edwards map)
    assert field.is_square(3)


def test_limbs_roundtrip():
    for _ in range(50):
        a = RNG.randrange(1 << 384)
        assert field.from_limbs(field.to_limbs(a)) == a


def test_redc_congruence_and_lazy_bound():
    edge = [0, 1, 2, P - 1, P, P + 1, 2 * P - 1, 6 * P - 1, 12 * P - 1]
    vals = edge + [RNG.randrange(12 * P) for _ in range(200)]
    for a in vals:
        for b in (RNG.choice(vals), RNG.randrange(12 * P)):
            u = field.mont_mul(a, b)
            assert u < 2 * P
            assert (u * field.R_MONT - a * b) % P == 0
    # the bound that makes lazily reduced operands safe: a, b < 12p => a b < R p
    assert 144 * P < field.R_MONT
    # to/from Montgomery form
    for _ in range(50):
        a = RNG.randrange(P)
        m = field.to_mont(a)
        assert field.from_mont(m) == a
        assert field.from_mont(field.mont_mul(m, field.to_mont(7))) == 7 * a % P


def test_redc_rejects_out_of_range_input():
    with pytest.raises(AssertionError):
        field.redc(field.R_MONT * P)


# --------------------------------------------------------------------------
# Weierstrass group law
# --------------------------------------------------------------------------

def test_group_laws_on_random_points():
    for _ in range(10):
        a, b, c = (random_curve_point() for _ in range(3))
        s = curve.add(a, b)
        assert curve.on_curve(s)
        assert s == curve.add(b, a)                              # commutative
        assert curve.add(curve.add(a, b), c) == curve.add(a, curve.add(b, c))  # associative
        assert curve.add(a, curve.INF) == a and curve.add(curve.INF, a) == a
        assert curve.add(a, curve.neg(a)) is curve.INF
        d = curve.add(a, a)                                       # tangent case
        assert curve.on_curve(d)
        assert curve.add(d, a) == curve.add(a, d)
        assert curve.add(curve.add(d, a), curve.neg(a)) == d


def test_doubling_consistent_with_chord():
    # 2P computed by the tangent equals (P + Q) + (P - Q) computed by chords only
    for _ in range(5):
        p1, q1 = random_curve_point(), random_curve_point()
        lhs = curve.add(p1, p1)
        rhs = curve.add(curve.add(p1, q1), curve.add(p1, curve.neg(q1)))
        assert lhs == rhs


def test_scalar_mul_linearity_and_brute_force():
    pt = random_g1_point()
    acc = curve.INF
    for k in range(0, 20):
        assert curve.smul(k, pt) == acc
        acc = curve.add(acc, pt)
    for _ in range(5):
        a, b = RNG.randrange(R_ORDER), RNG.randrange(R_ORDER)
        assert curve.smul(a + b, pt) == curve.add(curve.smul(a, pt), curve.smul(b, pt))
        assert curve.smul(a, curve.smul(b, pt)) == curve.smul(a * b % R_ORDER, pt)
    assert curve.smul(R_ORDER, pt) is curve.INF


def test_fixed_base_generator_matches_double_and_add():
    for k in [1, 2, 3, R_ORDER - 1] + [RNG.randrange(1, R_ORDER) for _ in range(5)]:
        assert points.fixed_base_mul(k) == curve.smul(k, curve.G)


# --------------------------------------------------------------------------
# MSM and Pippenger decomposition
# --------------------------------------------------------------------------

def test_msm_brute_force_tiny():
    for n in range(1, 5):
        pts = [random_g1_point() for _ in range(n)]
        sc = [RNG.randrange(16) for _ in range(n)]
        acc = curve.INF
        for s, pt in zip(sc, pts):
            for _ in range(s):
                acc = curve.add(acc, pt)
        assert msm.msm_naive(sc, pts) == acc


def test_msm_linearity_and_closed_form():
    n = 6
    ks = [RNG.randrange(1, R_ORDER) for _ in range(n)]
    pts = [points.fixed_base_mul(k) for k in ks]
    s1 = [RNG.randrange(R_ORDER) for _ in range(n)]
    s2 = [RNG.randrange(R_ORDER) for _ in range(n)]
    m1, m2 = msm.msm_naive(s1, pts), msm.msm_naive(s2, pts)
    m12 = msm.msm_naive([a + b for a, b in zip(s1, s2)], pts)
    assert curve.add(m1, m2) == m12
    assert m1 == msm.closed_form(s1, ks)
    assert msm.msm_naive([0] * n, pts) is curve.INF


def test_dot_mod_r_equals_plain_sum():
    """The digit-matrix form of sum s_i k_i mod r against the plain integer
    sum: random values, the largest 253- and 256-bit words, a block boundary
    (2^20 + 3 rows, so two blocks are summed) and an empty tail."""
    rng = np.random.default_rng(5)
    for n in (1, 7, 1000):
        s = rng.integers(0, 2**32, size=(n, 8), dtype=np.uint32)
        k = rng.integers(0, 2**32, size=(n, 8), dtype=np.uint32)
        si = [inputs.words_to_int(r) for r in s]
        ki = [inputs.words_to_int(r) for r in k]
        assert msm.dot_mod_r(s, k) == sum(a * b for a, b in zip(si, ki)) % R_ORDER
    n = (1 << 20) + 3
    s = np.full((n, 8), 0xFFFFFFFF, dtype=np.uint32)
    k = np.full((n, 8), 0xFFFFFFFF, dtype=np.uint32)
    assert msm.dot_mod_r(s, k) == n * ((1 << 256) - 1) ** 2 % R_ORDER
    s[:, 7] = 0x1FFFFFFF
    k[:, 7] = 0x1FFFFFFF
    assert msm.dot_mod_r(s, k) == n * ((1 << 253) - 1) ** 2 % R_ORDER
    sw = inputs.scalars_mod_r(11, 50)
    kw = inputs.nonzero_scalars_mod_r(12, 50)
    si = [inputs.words_to_int(r) for r in sw]
    ki = [inputs.words_to_int(r) for r in kw]
    assert msm.closed_form_words(sw, kw) == msm.closed_form(si, ki)


@pytest.mark.parametrize("c", [1, 4, 8, 13])
def test_pippenger_decomposition_equals_definition(c):
    n = 5 if c > 1 else 2
    ks = [RNG.randrange(1, R_ORDER) for _ in range(n)]
    pts = [points.fixed_base_mul(k) for k in ks]
    sc = [RNG.randrange(R_ORDER) for _ in range(n)]
    if c == 13:
        sc[0] = sc[1]          # two points in every shared bucket
    assert msm.msm_pippenger(sc, pts, c) == msm.closed_form(sc, ks)


def test_digits_recombine():
    for c in (1, 7, 8, 10, 16, 20):
        W = msm.num_windows(c)
        assert W * c >= 253 > (W - 1) * c
        for _ in range(20):
            s = RNG.randrange(1 << 253)
            assert sum(msm.digit(s, w, c) << (w * c) for w in range(W)) == s


def test_signed_digits_worked_example():
    """c = 4, s = 0x878, worked by hand: slices 8, 7, 8, 0 become
    8 -> -8 (carry), 7+1 -> -8 (carry), 8+1 -> -7 (carry), 0+1 -> 1."""
    d = msm.signed_digits(0x878, 4)
    assert d[:4] == [-8, -8, -7, 1] and not any(d[4:])
    assert len(d) == 64                     # ceil(254 / 4)


def test_signed_digits_recombine_and_ranges():
    cases = [0, 1, R_ORDER - 1, (1 << 253) - 1, int("10" * 126, 2)]
    cases += [RNG.randrange(1 << 253) for _ in range(40)]
    for c in (2, 3, 4, 7, 8, 11, 13, 16, 17, 20):
        W = msm.num_signed_windows(c)
        assert W * c >= 254 > (W - 1) * c
        half = 1 << (c - 1)
        for s in cases:
            d = msm.signed_digits(s, c)
            assert len(d) == W
            assert sum(x << (w * c) if x >= 0 else -((-x) << (w * c))
                       for w, x in enumerate(d)) == s
            assert all(-half <= x < half for x in d[:-1]), (c, s)
            assert 0 <= d[-1] <= half
    # exhaustive on small scalars
    for c in (2, 3, 5):
        half = 1 << (c - 1)
        for s in range(1 << 11):
            d = msm.signed_digits(s, c)
            assert sum(x * (1 << (w * c)) for w, x in enumerate(d)) == s
            assert all(-half <= x < half for x in d[:-1])


@pytest.mark.parametrize("c", [2, 3, 6, 13])
def test_signed_pippenger_equals_definition(c):
    n = 4
    ks = [RNG.randrange(1, R_ORDER) for _ in range(n)]
    pts = [points.fixed_base_mul(k) for k in ks]
    sc = [RNG.randrange(R_ORDER) for _ in range(n)]
    sc[1] = sc[0]            # shared buckets in every window
    sc[2] = R_ORDER - 1      # mostly negative digits
    assert msm.msm_pippenger_signed(sc, pts, c) == msm.msm_naive(sc, pts)
    # bucket contents by their definition: the signed digit sum of each bucket
    B = msm.signed_buckets(sc, pts, c)
    w = 1
    for m in range(1 << (c - 1)):
        coeff = sum((1 if x > 0 else -1) * k for s, k in zip(sc, ks)
                    for x in [msm.signed_digits(s, c)[w]] if abs(x) == m + 1)
        assert B[w][m] == curve.smul(coeff % R_ORDER, curve.G)


def test_endomorphism_constants():
    # lambda^2 + lambda + 1 equals r as integers (BLS12 family identity)
    assert glv.LAMBDA ** 2 + glv.LAMBDA + 1 == R_ORDER
    assert glv.LAMBDA.bit_length() == 127
    w = glv.OMEGA
    assert w != 1 and pow(w, 3, P) == 1 and (w * w + w + 1) % P == 0


def test_endomorphism_acts_as_lambda_on_g1():
    for _ in range(3):
        pt = random_g1_point()
        ph = glv.phi(pt)
        assert curve.on_curve(ph)
        assert ph == curve.smul(glv.LAMBDA, pt)
        # phi^3 = identity and P + phi(P) + phi^2(P) = O
        assert glv.phi(glv.phi(ph)) == pt
        assert curve.add(curve.add(pt, ph), glv.phi(ph)) is curve.INF
    assert glv.phi(curve.INF) is curve.INF


def test_scalar_split_recombines_and_is_short():
    cases = [0, 1, glv.LAMBDA - 1, glv.LAMBDA, glv.LAMBDA + 1, R_ORDER - 1,
             (1 << 253) - 1] + [RNG.randrange(1 << 253) for _ in range(200)]
    for s in cases:
        s0, s1 = glv.split(s)
        assert s1 * glv.LAMBDA + s0 == s
        assert 0 <= s0 < glv.LAMBDA and 0 <= s1 < (1 << glv.SPLIT_BITS)


def test_split_msm_equals_naive():
    n = 4
    ks = [RNG.randrange(1, R_ORDER) for _ in range(n)]
    pts = [points.fixed_base_mul(k) for k in ks]
    sc = [RNG.randrange(R_ORDER) for _ in range(n - 1)] + [(1 << 253) - 1]
    sc2, pts2 = glv.msm_split(sc, pts)
    assert len(pts2) == 2 * n and max(sc2).bit_length() <= glv.SPLIT_BITS
    assert msm.msm_naive(sc2, pts2) == msm.msm_naive(sc, pts) == msm.closed_form(sc, ks)


# --------------------------------------------------------------------------
# twisted Edwards
# --------------------------------------------------------------------------

def test_te_parameters():
    assert te.ALPHA * te.ALPHA % P == 3
    assert te.A_TE == P - 1                                    # a = -1
    assert te.K_TE == 2 * te.D_TE % P                          # k / 2 = d
    assert te.BETA * te.BETA % P == te.B_MONT * pow(te.ALPHA, 3, P) % P
    assert te.D_TE not in (0, 1, P - 1)


def test_te_map_is_homomorphism():
    for _ in range(8):
        a, b = random_g1_point(), random_g1_point()
        ea, eb = te.w_to_te(a), te.w_to_te(b)
        assert te.on_te(ea) and te.on_te(eb)
        assert te.te_to_w(ea) == a
        assert te.w_to_te(curve.add(a, b)) == te.te_add(ea, eb)
        assert te.w_to_te(curve.add(a, a)) == te.te_add(ea, ea)
        assert te.te_add(ea, te.te_neg(ea)) == te.IDENTITY
        assert te.w_to_te(curve.neg(a)) == te.te_neg(ea)
        assert te.te_add(ea, te.IDENTITY) == ea
    assert te.w_to_te(curve.INF) == te.IDENTITY
    assert te.te_to_w(te.IDENTITY) is curve.INF


def test_extended_coordinates():
    for _ in range(10):
        pt = te.w_to_te(random_g1_point())
        lam = RNG.randrange(1, P)
        X, Y, T, Z = te.to_extended(pt, lam)
        assert te.from_extended(X, Y, T, Z) == pt
        assert (T * Z - X * Y) % P == 0
        with pytest.raises(ValueError):
            te.from_extended(X, Y, (T + 1) % P, Z)
        x, y, u = te.to_prepared(pt)
        assert u == te.K_TE * x * y % P


# --------------------------------------------------------------------------
# seeded generators
# --------------------------------------------------------------------------

def test_scalar_generator_range_and_determinism():
    a = inputs.scalars_mod_r(7, 1000)
    b = inputs.scalars_mod_r(7, 1000)
    assert np.array_equal(a, b)
    vals = [inputs.words_to_int(r) for r in a]
    assert all(0 <= v < R_ORDER for v in vals)
    assert max(vals) > R_ORDER // 2        # uses the full range
    e = inputs.base_field_elements(3, 200)
    assert all(0 < inputs.words_to_int(r) < P for r in e)


def test_gen_points_equals_scalar_multiples():
    """The generator of the workload points, with and without its process
    pool, gives k G as double-and-add computes it."""
    rng = random.Random(77)
    ks = [0, 1, 2, R_ORDER - 1] + [rng.randrange(R_ORDER) for _ in range(68)]
    want = [curve.smul(k, curve.G) for k in ks]
    assert points.gen_points(ks) == want
    assert points.gen_points(ks, processes=2) == want
