"""Endomorphism split of scalar multiplication on BLS12-377 G1 (test oracle).

Test infrastructure: imported only by tests, the smoke check and the CPU
baseline of the benchmark.

This is not in the paper: it is an optional way to run the same MSM with
half-length scalars.  The curve y^2 = x^3 + 1 has the automorphism
phi(x, y) = (omega x, y) for a primitive cube root of unity omega in GF(p);
on the prime-order subgroup it acts as multiplication by a root lambda of
lambda^2 + lambda + 1 = 0 (mod r).  For the BLS12 family,
lambda = x0^2 - 1 satisfies lambda^2 + lambda + 1 = r exactly (as integers),
so every s < 2^253 splits as s = s1 lambda + s0 with s0 = s mod lambda and
s1 = s div lambda, both below 2^127, and

    s P = s0 P + s1 phi(P).

An MSM over n points with 253-bit scalars is therefore an MSM over the 2n
points P_i, phi(P_i) with 127-bit scalars.  omega is the cube root for
which phi(G) = lambda G (the other root gives lambda^2).
"""

from . import curve
from .field import P, R_ORDER, X0, fsqrt

LAMBDA = X0 * X0 - 1
SPLIT_BITS = 127


def _cube_roots_of_unity():
    # roots of w^2 + w + 1 = 0: w = (-1 +- sqrt(-3)) / 2
    s = fsqrt((-3) % P)
    inv2 = pow(2, P - 2, P)
    return sorted(((-1 + s) * inv2 % P, (-1 - s) * inv2 % P))


def _pick_omega():
    for w in _cube_roots_of_unity():
        if (w * curve.G[0] % P, curve.G[1]) == curve.smul(LAMBDA, curve.G):
            return w
    raise AssertionError("no cube root of unity matches lambda")


OMEGA = _pick_omega()


def phi(pt):
    """The endomorphism (x, y) -> (omega x, y); O -> O."""
    if pt is curve.INF:
        return curve.INF
    return (OMEGA * pt[0] % P, pt[1])


def split(s):
    """(s0, s1) with s = s1 * LAMBDA + s0, 0 <= s0 < LAMBDA."""
    return s % LAMBDA, s // LAMBDA


def msm_split(scalars, points):
    """The 2n-point MSM with half-length scalars that equals the original
    (point i followed by its image, scalar halves s0, s1 likewise)."""
    pts, sc = [], []
    for s, pt in zip(scalars, points):
        s0, s1 = split(s)
        pts += [pt, phi(pt)]
        sc += [s0, s1]
    return sc, pts
