"""Seeded synthetic workload generators shared by the GPU path and the tests.

This module draws random numbers and nothing else: it holds none of the
MSM's arithmetic.  Both sides receive what it draws as plain inputs -- the
scalar multipliers k_i of the point pools P_i = k_i G, the MSM scalars s_i,
the projective scale factors lambda, job sizes and arrival times.  The points
themselves are computed separately by each side (the CPU oracle in tests, the
GPU generator in the benchmark).

All draws use numpy's PCG64 with an explicit seed.  Multi-word integers are
returned as little-endian uint32 word arrays, one row per value.

The two bounds below are the orders of BLS12-377's scalar field (r) and base
field (p); they only bound the uniform draws.
"""

import numpy as np

SCALAR_FIELD_ORDER = 0x12AB655E9A2CA55660B44D1E5C37B00159AA76FED00000010A11800000000001
BASE_FIELD_ORDER = 0x01AE3A4617C510EAC63B05C06CA1493B1A22D9F300F5138F1EF3622FBA094800170B5D44300000008508C00000000001

SEED_BASE = 20250217


def config_seed(config_no):
    """Seed of a workload configuration: a fixed base plus its number."""
    return SEED_BASE + int(config_no)


def _words64(value, nwords):
    return [(value >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(nwords)]


def _uniform_below(rng, n, bound, bits):
    """n uniform integers in [0, bound) by rejection from `bits`-bit draws.

    Returns an (n, ceil(bits/64)) uint64 array of little-endian 64-bit words.
    """
    nw = -(-bits // 64)
    top_bits = bits - 64 * (nw - 1)
    top_mask = np.uint64((1 << top_bits) - 1)
    bw = _words64(bound, nw)
    out = np.empty((0, nw), dtype=np.uint64)
    while out.shape[0] < n:
        m = int((n - out.shape[0]) * 1.8) + 16
        cand = rng.integers(0, 2**64, size=(m, nw), dtype=np.uint64, endpoint=False)
        cand[:, nw - 1] &= top_mask
        # lexicographic cand < bound, most significant word first
        lt = np.zeros(m, dtype=bool)
        eq = np.ones(m, dtype=bool)
        for j in range(nw - 1, -1, -1):
            b = np.uint64(bw[j])
            lt |= eq & (cand[:, j] < b)
            eq &= cand[:, j] == b
        out = np.concatenate([out, cand[lt]], axis=0)
    return out[:n]


def _to_u32_words(w64, n32):
    lo = (w64 & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    hi = (w64 >> np.uint64(32)).astype(np.uint32)
    inter = np.empty((w64.shape[0], 2 * w64.shape[1]), dtype=np.uint32)
    inter[:, 0::2] = lo
    inter[:, 1::2] = hi
    return np.ascontiguousarray(inter[:, :n32])


def scalars_mod_r(seed, n, stream=0):
    """n scalars uniform in [0, r), as an (n, 8) uint32 array (little-endian)."""
    rng = np.random.Generator(np.random.PCG64([int(seed), int(stream)]))
    w = _uniform_below(rng, n, SCALAR_FIELD_ORDER, 253)
    return _to_u32_words(w, 8)


def nonzero_scalars_mod_r(seed, n, stream=0):
    """n scalars uniform in [1, r) (point multipliers k_i must be non-zero)."""
    s = scalars_mod_r(seed, n + 64, stream)
    nz = s.any(axis=1)
    s = s[nz][:n]
    assert s.shape[0] == n
    return s


def base_field_elements(seed, n, stream=0, nonzero=True):
    """n elements uniform in [0, p) (or [1, p)), as (n, 12) uint32 words."""
    rng = np.random.Generator(np.random.PCG64([int(seed), int(stream)]))
    w = _uniform_below(rng, n + 64, BASE_FIELD_ORDER, 377)
    e = _to_u32_words(w, 12)
    if nonzero:
        e = e[e.any(axis=1)]
    return np.ascontiguousarray(e[:n])


def log_uniform_sizes(seed, count, lo_exp, hi_exp, stream=0):
    """count sizes n_j = floor(2^u), u ~ U[lo_exp, hi_exp]."""
    rng = np.random.Generator(np.random.PCG64([int(seed), int(stream)]))
    u = rng.uniform(lo_exp, hi_exp, size=count)
    return np.floor(np.exp2(u)).astype(np.int64)


def poisson_arrivals(seed, rate_per_s, duration_s, stream=0):
    """Arrival times (s) of a Poisson process with the given mean rate."""
    rng = np.random.Generator(np.random.PCG64([int(seed), int(stream)]))
    n_guess = int(rate_per_s * duration_s * 1.5) + 32
    gaps = rng.exponential(1.0 / rate_per_s, size=n_guess)
    t = np.cumsum(gaps)
    while t[-1] < duration_s:
        more = np.cumsum(rng.exponential(1.0 / rate_per_s, size=n_guess)) + t[-1]
        t = np.concatenate([t, more])
    return t[t < duration_s]


def words_to_int(row):
    """Little-endian uint32 words -> Python int."""
    return sum(int(w) << (32 * i) for i, w in enumerate(row))


def ints_to_words(values, nwords):
    """Python ints -> (len, nwords) uint32 array of little-endian words."""
    out = np.zeros((len(values), nwords), dtype=np.uint32)
    for i, v in enumerate(values):
        v = int(v)
        for j in range(nwords):
            out[i, j] = (v >> (32 * j)) & 0xFFFFFFFF
    return out
