"""Twisted-Edwards form of BLS12-377 G1 and its extended coordinates (oracle).

Test infrastructure: imported only by tests, the smoke check and the CPU
baseline of the benchmark.

Sec. II-D converts the Weierstrass curve into the twisted-Edwards curve
-x^2 + y^2 = 1 + (k/2) x^2 y^2 and represents points in extended projective
coordinates (X, Y, T, Z) with X = x Z, Y = y Z, T = X Y / Z; inputs to the
mixed addition carry U = k T instead of T, with Z = 1.  The paper prints
neither k nor the map, so they are derived here:

1. y^2 = x^3 + 1 has the 2-torsion point (-1, 0).  Put x = alpha u - 1 and
   y = beta v with alpha^2 = 3.  Dividing by alpha^3 gives the Montgomery
   curve  B v^2 = u^3 + A u^2 + u  with  A = -alpha,  B = beta^2 / alpha^3.
2. The Montgomery curve maps to a x^2 + y^2 = 1 + d x^2 y^2 with
   a = (A + 2) / B,  d = (A - 2) / B  via  x_e = u / v,  y_e = (u-1)/(u+1).
   Requiring a = -1 fixes B = -(A + 2) = alpha - 2, hence
   beta^2 = (alpha - 2) alpha^3  and  d = (alpha + 2) / (2 - alpha).
3. The paper's coefficient k/2 is this d, so k = 2 d.

Both square roots are chosen as the smaller of the two representatives in
[0, p).  The sign choice changes twisted-Edwards coordinates but never a
Weierstrass-level result.

Affine twisted-Edwards addition with a = -1 is the textbook unified law
    x3 = (x1 y2 + y1 x2) / (1 + d x1 x2 y1 y2)
    y3 = (y1 y2 + x1 x2) / (1 - d x1 x2 y1 y2)
with identity (0, 1) and negation (x, y) -> (-x, y).
"""

from .field import P, finv, fsqrt, is_square
from . import curve

ALPHA = fsqrt(3)
_beta_sq = (ALPHA - 2) * pow(ALPHA, 3, P) % P
assert is_square(_beta_sq), "beta^2 must be a square for the chosen alpha"
BETA = fsqrt(_beta_sq)
A_MONT = (-ALPHA) % P
B_MONT = (ALPHA - 2) % P
A_TE = (A_MONT + 2) * finv(B_MONT) % P          # equals p - 1, i.e. a = -1
D_TE = (A_MONT - 2) * finv(B_MONT) % P
K_TE = 2 * D_TE % P                              # the paper's k (U = k T)

IDENTITY = (0, 1)


def on_te(pt):
    x, y = pt
    return (A_TE * x * x + y * y - 1 - D_TE * x * x * y * y) % P == 0


def te_neg(pt):
    x, y = pt
    return ((-x) % P, y)


def te_add(p1, p2):
    x1, y1 = p1
    x2, y2 = p2
    t = D_TE * x1 % P * x2 % P * y1 % P * y2 % P
    x3 = (x1 * y2 + y1 * x2) * finv(1 + t) % P
    y3 = (y1 * y2 - A_TE * x1 * x2) * finv(1 - t) % P
    return (x3, y3)


def w_to_te(pt):
    """Weierstrass affine point (or None = O) -> twisted-Edwards affine."""
    if pt is curve.INF:
        return IDENTITY
    x, y = pt
    u = (x + 1) * finv(ALPHA) % P
    v = y * finv(BETA) % P
    if v == 0 or (u + 1) % P == 0:
        raise ValueError("point is exceptional for the birational map")
    return (u * finv(v) % P, (u - 1) * finv(u + 1) % P)


def te_to_w(pt):
    """Twisted-Edwards affine -> Weierstrass affine (identity -> None)."""
    xe, ye = pt
    if (xe, ye) == IDENTITY:
        return curve.INF
    if xe == 0 or ye == 1:
        raise ValueError("point is exceptional for the birational map")
    u = (1 + ye) * finv(1 - ye) % P
    v = u * finv(xe) % P
    return ((ALPHA * u - 1) % P, BETA * v % P)


# ---------------------------------------------------------------------------
# Extended coordinates (X, Y, T, Z) and the prepared form (X, Y, U), Z = 1
# ---------------------------------------------------------------------------

def to_extended(pt, lam=1):
    """Affine (x, y) -> (X, Y, T, Z) = (lam x, lam y, lam x y, lam)."""
    x, y = pt
    lam %= P
    assert lam != 0
    return (lam * x % P, lam * y % P, lam * x % P * y % P, lam)


def to_prepared(pt):
    """Affine (x, y) -> (X, Y, U) with Z = 1 and U = k x y."""
    x, y = pt
    return (x, y, K_TE * x % P * y % P)


def from_extended(X, Y, T, Z):
    """(X, Y, T, Z) -> affine (x, y), checking T Z = X Y and Z != 0."""
    X, Y, T, Z = (v % P for v in (X, Y, T, Z))
    if Z == 0:
        raise ValueError("Z = 0")
    if (T * Z - X * Y) % P != 0:
        raise ValueError("extended-coordinate invariant T Z = X Y fails")
    zi = finv(Z)
    return (X * zi % P, Y * zi % P)
