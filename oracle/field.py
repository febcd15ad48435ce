"""Base field, scalar field and Montgomery form for BLS12-377 (test oracle).

Test infrastructure: imported only by tests, the smoke check and the CPU
baseline of the benchmark.

The paper targets the BLS12-377 curve over a 377-bit prime field (Abstract;
Sec. II-D) but prints none of its parameters.  They follow from the BLS12
family parameterisation with the curve's published seed x0:

    r = x0^4 - x0^2 + 1            (prime order of G1, 253 bits)
    p = (x0 - 1)^2 * r / 3 + x0    (base-field prime, 377 bits)
    t = x0 + 1                     (trace of Frobenius)
    #E(F_p) = p + 1 - t = h * r

The only value taken as given is the generator G (the conventional G1
generator of BLS12-377); tests check that it lies on y^2 = x^3 + 1 and has
order r.

Montgomery form uses R = 2^384 (twelve 32-bit words).  The paper names
Montgomery representation as the way to cut exact carry propagation
(Sec. V-C); ``redc`` below is the textbook word-serial reduction, kept here so
the lazy-reduction bounds the GPU design relies on can be pinned on the CPU.
"""

X0 = 0x8508C00000000001

R_ORDER = X0**4 - X0**2 + 1
_num = (X0 - 1) ** 2 * R_ORDER
assert _num % 3 == 0
P = _num // 3 + X0
TRACE = X0 + 1
N_POINTS = P + 1 - TRACE
assert N_POINTS % R_ORDER == 0
COFACTOR = N_POINTS // R_ORDER

# Short-Weierstrass coefficients of BLS12-377 G1: y^2 = x^3 + A x + B.
A_W = 0
B_W = 1

# Conventional G1 generator of BLS12-377 (given, not derived).
G_X = 0x008848DEFE740A67C8FC6225BF87FF5485951E2CAA9D41BB188282C8BD37CB5CD5481512FFCD394EEAB9B16EB21BE9EF
G_Y = 0x01914A69C5102EFF1F674F5D30AFEEC4BD7FB348CA3E52D96D182AD44FB82305C2FE3D3634A9591AFD82DE55559C8EA6

# Montgomery radix: twelve 32-bit words.
LIMB_BITS = 32
N_LIMBS = 12
R_MONT = 1 << (LIMB_BITS * N_LIMBS)
R_MONT_INV = pow(R_MONT, -1, P)
R2_MONT = R_MONT * R_MONT % P
# n' = -p^{-1} mod 2^32, the per-word Montgomery factor.
N_PRIME_32 = (-pow(P, -1, 1 << 32)) % (1 << 32)


def fadd(a, b):
    return (a + b) % P


def fsub(a, b):
    return (a - b) % P


def fmul(a, b):
    return (a * b) % P


def finv(a):
    """The inverse a^-1 mod p (a must be non-zero mod p), by Python's built-in
    modular inverse (extended Euclid).  It equals a^(p-2) mod p (Fermat), the
    form the tests pin it against; the built-in is used because it is some
    fifty times faster, which keeps the full-size result checks short."""
    a %= P
    if a == 0:
        raise ZeroDivisionError("inverse of 0 in F_p")
    return pow(a, -1, P)


def fneg(a):
    return (-a) % P


def is_square(a):
    """Euler's criterion."""
    a %= P
    return a == 0 or pow(a, (P - 1) // 2, P) == 1


def fsqrt(a):
    """Tonelli-Shanks square root in F_p; returns the root r with r <= p - r.

    Raises ValueError if a is not a square.
    """
    a %= P
    if a == 0:
        return 0
    if not is_square(a):
        raise ValueError("not a square")
    # p - 1 = q * 2^s with q odd
    q, s = P - 1, 0
    while q % 2 == 0:
        q //= 2
        s += 1
    z = 2
    while is_square(z):
        z += 1
    m, c, t, root = s, pow(z, q, P), pow(a, q, P), pow(a, (q + 1) // 2, P)
    while t != 1:
        i, t2 = 0, t
        while t2 != 1:
            t2 = t2 * t2 % P
            i += 1
        b = pow(c, 1 << (m - i - 1), P)
        m, c = i, b * b % P
        t = t * c % P
        root = root * b % P
    assert root * root % P == a
    return min(root, P - root)


# ---------------------------------------------------------------------------
# Montgomery form (R = 2^384) and word layout
# ---------------------------------------------------------------------------

def to_mont(a):
    """a -> a R mod p (canonical)."""
    return a * R_MONT % P


def from_mont(a):
    """a R -> a (canonical); accepts any non-negative representative."""
    return a * R_MONT_INV % P


def to_limbs(a, n=N_LIMBS):
    """Little-endian 32-bit words of a non-negative integer."""
    assert 0 <= a < (1 << (32 * n))
    return [(a >> (32 * i)) & 0xFFFFFFFF for i in range(n)]


def from_limbs(words):
    return sum(int(w) << (32 * i) for i, w in enumerate(words))


def redc(t):
    """Word-serial Montgomery reduction of 0 <= t < R p.

    Returns u with u = t R^{-1} (mod p) and u < 2p, without a final
    conditional subtraction.  Each step picks m = t_0 n' mod 2^32 so the low
    word of t + m p vanishes, then drops that word.
    """
    assert 0 <= t < R_MONT * P
    for _ in range(N_LIMBS):
        m = (t & 0xFFFFFFFF) * N_PRIME_32 & 0xFFFFFFFF
        t = (t + m * P) >> 32
    assert t < 2 * P
    return t


def mont_mul(a, b):
    """Montgomery product a b R^{-1} (mod p), lazily reduced (< 2p).

    Valid whenever a b < R p, e.g. a, b < 12 p because 144 p < R.
    """
    return redc(a * b)
