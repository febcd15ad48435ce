"""Short-Weierstrass affine arithmetic on BLS12-377 G1 (test oracle).

Test infrastructure: imported only by tests, the smoke check and the CPU
baseline of the benchmark.

The curve is y^2 = x^3 + a x + b over GF(p) (Sec. II-D) with a = 0, b = 1.
A point is a pair (x, y) of canonical integers, or ``None`` for the point at
infinity O.  Addition is the textbook chord-and-tangent law; scalar
multiplication is most-significant-bit-first double-and-add.
"""

from .field import P, A_W, B_W, G_X, G_Y, R_ORDER, finv

INF = None
G = (G_X, G_Y)


def on_curve(pt):
    if pt is INF:
        return True
    x, y = pt
    return 0 <= x < P and 0 <= y < P and (y * y - (x * x * x + A_W * x + B_W)) % P == 0


def neg(pt):
    if pt is INF:
        return INF
    x, y = pt
    return (x, (-y) % P)


def add(p1, p2):
    """Affine point addition P1 + P2 (chord, tangent, and the O cases)."""
    if p1 is INF:
        return p2
    if p2 is INF:
        return p1
    x1, y1 = p1
    x2, y2 = p2
    if x1 == x2:
        if (y1 + y2) % P == 0:
            return INF                      # P + (-P) = O (covers y = 0 doubling)
        lam = (3 * x1 * x1 + A_W) * finv(2 * y1) % P   # tangent
    else:
        lam = (y2 - y1) * finv(x2 - x1) % P            # chord
    x3 = (lam * lam - x1 - x2) % P
    y3 = (lam * (x1 - x3) - y1) % P
    return (x3, y3)


def double(pt):
    return add(pt, pt)


def smul(k, pt):
    """k * pt by MSB-first double-and-add; k >= 0 (0 * pt = O)."""
    if k < 0:
        return smul(-k, neg(pt))
    acc = INF
    for bit in bin(k)[2:] if k else "":
        acc = add(acc, acc)
        if bit == "1":
            acc = add(acc, pt)
    return acc


def in_subgroup(pt):
    return on_curve(pt) and smul(R_ORDER, pt) is INF
