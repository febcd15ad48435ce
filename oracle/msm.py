"""Multi-scalar multiplication and Pippenger's decomposition (test oracle).

Test infrastructure: imported only by tests, the smoke check and the CPU
baseline of the benchmark.

MSM is the sum of scalar-point products sum_i s_i P_i over G1 (Abstract;
Sec. II-C).  Pippenger's algorithm (Sec. II-C) cuts k-bit scalars into w-bit
windows, giving k/w groups; inside each group the points go to buckets by
their sliced scalar value and are summed (bucket accumulation); the buckets
are then combined (bucket aggregation); and the groups are combined into the
result (group aggregation).  Reading of the slicing: unsigned c-bit digits,
digit 0 contributes nothing, the top window holds the remaining
253 mod c bits.

A signed-digit encoding of the same windows is also given (it is not in the
paper; it gives the same MSM with half as many buckets): every scalar is
rewritten as s = sum_w d_w 2^(w c) with d_w in [-2^(c-1), 2^(c-1)], and a
point with a negative digit is subtracted from bucket |d_w|.

Everything here is the plain definition, on Weierstrass affine points, so the
functions below are independent of the twisted-Edwards machinery in ``te``.
"""

from .curve import INF, G, add, neg, smul
from .field import R_ORDER

SCALAR_BITS = 253


def msm_naive(scalars, points):
    """sum_i s_i P_i by independent double-and-add products."""
    acc = INF
    for s, pt in zip(scalars, points):
        acc = add(acc, smul(s, pt))
    return acc


def num_windows(c, bits=SCALAR_BITS):
    return -(-bits // c)


def digit(s, w, c):
    """The w-th c-bit slice of scalar s (window w covers bits [w c, w c + c))."""
    return (s >> (w * c)) & ((1 << c) - 1)


def buckets(scalars, points, c):
    """B[w][b] = sum of P_i whose w-th digit equals b (bucket accumulation)."""
    W = num_windows(c)
    B = [[INF] * (1 << c) for _ in range(W)]
    for s, pt in zip(scalars, points):
        for w in range(W):
            d = digit(s, w, c)
            if d:
                B[w][d] = add(B[w][d], pt)
    return B


def window_sum(bucket_row):
    """S = sum_b b * B[b] (bucket aggregation, written as the definition)."""
    acc = INF
    for b, pt in enumerate(bucket_row):
        if b and pt is not INF:
            acc = add(acc, smul(b, pt))
    return acc


def group_aggregate(window_sums, c):
    """Q = sum_w 2^(w c) S_w (group aggregation, written as the definition)."""
    acc = INF
    for w, s in enumerate(window_sums):
        acc = add(acc, smul(1 << (w * c), s))
    return acc


def msm_pippenger(scalars, points, c):
    """The three Pippenger steps composed; equals msm_naive for any c >= 1."""
    B = buckets(scalars, points, c)
    return group_aggregate([window_sum(row) for row in B], c)


def num_signed_windows(c, bits=SCALAR_BITS):
    """Windows of the signed encoding: one more bit than the scalar, so the
    top window never needs a carry out."""
    return -(-(bits + 1) // c)


def signed_digits(s, c, bits=SCALAR_BITS):
    """Digits d_0..d_{W-1} with s = sum_w d_w 2^(w c) for s < 2^bits, written
    from the definition: walking up from the lowest window, v = slice +
    carry; when v >= 2^(c-1) (and this is not the top window) the digit is
    v - 2^c and a carry of one moves up, otherwise the digit is v and no
    carry moves."""
    W = num_signed_windows(c, bits)
    half, full = 1 << (c - 1), 1 << c
    out, carry = [], 0
    for w in range(W):
        v = digit(s, w, c) + carry
        if v >= half and w + 1 < W:
            out.append(v - full)
            carry = 1
        else:
            out.append(v)
            carry = 0
    return out


def signed_buckets(scalars, points, c, bits=SCALAR_BITS):
    """B[w][m] = sum over i with |d_w(s_i)| = m + 1 of sign(d_w(s_i)) P_i."""
    W = num_signed_windows(c, bits)
    B = [[INF] * (1 << (c - 1)) for _ in range(W)]
    for s, pt in zip(scalars, points):
        for w, d in enumerate(signed_digits(s, c, bits)):
            if d > 0:
                B[w][d - 1] = add(B[w][d - 1], pt)
            elif d < 0:
                B[w][-d - 1] = add(B[w][-d - 1], neg(pt))
    return B


def signed_window_sum(bucket_row):
    """S = sum_m (m + 1) * B[m] (bucket m holds digit magnitude m + 1)."""
    acc = INF
    for m, pt in enumerate(bucket_row):
        if pt is not INF:
            acc = add(acc, smul(m + 1, pt))
    return acc


def msm_pippenger_signed(scalars, points, c):
    """Pippenger with signed digits; equals msm_naive for any c >= 2."""
    B = signed_buckets(scalars, points, c)
    return group_aggregate([signed_window_sum(row) for row in B], c)


def closed_form(scalars, ks):
    """For P_i = k_i G:  sum_i s_i P_i = ((sum_i s_i k_i) mod r) G."""
    tot = sum(s * k for s, k in zip(scalars, ks)) % R_ORDER
    return smul(tot, G)


def dot_mod_r(s_words, k_words):
    """(sum_i s_i k_i) mod r for scalars given as (n, 8) arrays of
    little-endian 32-bit words, computed exactly and fast for large n.

    Every value is cut into sixteen 16-bit digits, so
    sum_i s_i k_i = sum_{a,b} 2^(16 (a+b)) D[a][b] with
    D[a][b] = sum_i s_i[a] k_i[b].  Each digit product is below 2^32, so a
    sum of at most 2^20 of them stays below 2^52 and the 16 x 16 sums D are
    exact as float64 matrix products of the digit columns (every partial sum
    is an integer below 2^53); longer inputs are summed in blocks of 2^20."""
    import numpy as np
    s = np.ascontiguousarray(s_words, dtype=np.uint32).reshape(-1, 8)
    k = np.ascontiguousarray(k_words, dtype=np.uint32).reshape(-1, 8)
    assert s.shape == k.shape

    def digits(w):
        out = np.empty((w.shape[0], 16), dtype=np.float64)
        out[:, 0::2] = w & 0xFFFF
        out[:, 1::2] = w >> 16
        return out

    tot = 0
    for lo in range(0, s.shape[0], 1 << 20):
        D = digits(s[lo:lo + (1 << 20)]).T @ digits(k[lo:lo + (1 << 20)])
        for a in range(16):
            for b in range(16):
                tot += int(D[a, b]) << (16 * (a + b))
    return tot % R_ORDER


def closed_form_words(s_words, k_words):
    """closed_form for scalars and point multipliers given as word arrays."""
    return smul(dot_mod_r(s_words, k_words), G)
