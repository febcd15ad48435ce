"""Synthetic point pools P_i = k_i G for tests (oracle side).

Test infrastructure: imported only by tests, the smoke check and the CPU
baseline of the benchmark.

The scalars k_i come from the shared seeded generators; the points are
computed here with plain affine arithmetic.  To keep test fixtures fast the
fixed base G uses a table of its doublings 2^j G (each entry is an ordinary
affine doubling of the previous one), so k G is the sum of the table entries
selected by the bits of k -- the same value double-and-add gives.
"""

from functools import lru_cache

from .curve import INF, G, add


@lru_cache(maxsize=1)
def _doublings(bits=256):
    tab = [G]
    for _ in range(bits - 1):
        tab.append(add(tab[-1], tab[-1]))
    return tab


def fixed_base_mul(k):
    """k G via the table of doublings of G (k >= 0, k < 2^256)."""
    tab = _doublings()
    acc = INF
    j = 0
    while k:
        if k & 1:
            acc = add(acc, tab[j])
        k >>= 1
        j += 1
    return acc


def gen_points(ks, processes=None):
    """[k G for k in ks], optionally in a process pool."""
    ks = [int(k) for k in ks]
    if processes and len(ks) > 64:
        import multiprocessing as mp
        _doublings()
        ctx = mp.get_context("fork")
        with ctx.Pool(processes) as pool:
            return pool.map(fixed_base_mul, ks, chunksize=max(1, len(ks) // (4 * processes)))
    return [fixed_base_mul(k) for k in ks]
