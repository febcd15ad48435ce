"""Host-side counts that bench.py reports beside its timings, checked against
the oracle's own digit definitions (CPU only).

The headline rate divides the additions the MSM performs by its time, and
the accumulation's share of them is one mixed addition per non-zero digit
(Sec. II-C): bench.py counts those digits with vectorised numpy over the
scalar words.  Here the count is rebuilt scalar by scalar from the oracle's
unsigned digit, signed digit and endomorphism split, so that a wrong window
count, carry rule, split constant or word order in the bench's counter fails.
"""

import random

import numpy as np
import pytest

import bench
from oracle import glv, msm
from oracle.field import R_ORDER
from paper_2502_11660_amd import inputs

RNG = random.Random(20250220)
EDGE = [0, 1, 2, R_ORDER - 1, R_ORDER - 2, (1 << 252) - 1, 1 << 252, glv.LAMBDA,
        glv.LAMBDA - 1, glv.LAMBDA + 1, (1 << 127) - 1, 1 << 127, 0x5555 << 200]
SCALARS = EDGE + [RNG.randrange(R_ORDER) for _ in range(48)]


def oracle_count(scalars, c, encoding):
    """Non-zero digits of every scalar at width c, from the oracle."""
    if encoding == "unsigned":
        W = msm.num_windows(c)
        return sum(1 for s in scalars for w in range(W) if msm.digit(s, w, c))
    if encoding == "signed":
        return sum(1 for s in scalars for d in msm.signed_digits(s, c) if d)
    # the split halves are below 2^127; their signed digits take 128 bits
    return sum(1 for s in scalars for h in glv.split(s)
               for d in msm.signed_digits(h, c, bits=127) if d)


@pytest.mark.parametrize("encoding,c", [
    ("unsigned", 5), ("unsigned", 8), ("unsigned", 11), ("unsigned", 16),
    ("signed", 5), ("signed", 8), ("signed", 13), ("signed", 16), ("signed", 17),
    ("glv", 8), ("glv", 13), ("glv", 16), ("glv", 19),
])
def test_nonzero_digit_entries_match_oracle_digits(encoding, c):
    words = np.asarray(inputs.ints_to_words(SCALARS, 8), dtype=np.uint32)
    assert bench.window_bits(c, encoding) == c  # widths that run as requested
    assert bench.nonzero_digit_entries(words, c, encoding) == oracle_count(SCALARS, c, encoding)


def test_window_counts_match_oracle():
    for c in range(2, 21):
        assert bench.num_windows(c, "unsigned") == msm.num_windows(c)
        assert bench.num_windows(c, "signed") == msm.num_signed_windows(c)
        assert bench.num_windows(c, "glv") == msm.num_signed_windows(c, bits=127)


def test_glv_halves_match_oracle_split():
    words = np.asarray(inputs.ints_to_words(SCALARS, 8), dtype=np.uint32)
    halves = bench.glv_halves(words).reshape(-1, 2, 8)
    for s, (h0, h1) in zip(SCALARS, halves):
        assert (inputs.words_to_int(h0), inputs.words_to_int(h1)) == glv.split(s)
