"""Test-side helpers: word layouts and oracle-side conversions.

Everything that turns oracle integers into the library's word layouts (and
back) lives here, computed with the oracle's own Montgomery conversion, so no
expected value ever passes through the GPU library.
"""

import numpy as np

from oracle import field, te
from oracle.field import P

W = 12


def int_words(v, n=W):
    return [(v >> (32 * i)) & 0xFFFFFFFF for i in range(n)]


def words_int(ws):
    return sum(int(w) << (32 * i) for i, w in enumerate(ws))


def soa(rows, ncoord):
    """rows: list of ncoord-tuples of ints -> flat SoA uint32 array."""
    cnt = len(rows)
    out = np.zeros((ncoord * W, cnt), dtype=np.uint32)
    for i, row in enumerate(rows):
        for c in range(ncoord):
            v = int(row[c])
            for l in range(W):
                out[c * W + l, i] = (v >> (32 * l)) & 0xFFFFFFFF
    return out.reshape(-1)


def unsoa(flat, ncoord, cnt):
    a = np.asarray(flat, dtype=np.uint32).reshape(ncoord * W, cnt)
    rows = []
    for i in range(cnt):
        rows.append(tuple(words_int(a[c * W:(c + 1) * W, i]) for c in range(ncoord)))
    return rows


def aos(rows, ncoord):
    out = np.zeros((len(rows), ncoord * W), dtype=np.uint32)
    for i, row in enumerate(rows):
        for c in range(ncoord):
            out[i, c * W:(c + 1) * W] = int_words(int(row[c]))
    return out.reshape(-1)


def unaos(flat, ncoord, cnt):
    a = np.asarray(flat, dtype=np.uint32).reshape(cnt, ncoord * W)
    return [tuple(words_int(a[i, c * W:(c + 1) * W]) for c in range(ncoord)) for i in range(cnt)]


def scalar_words(values):
    out = np.zeros((len(values), 8), dtype=np.uint32)
    for i, v in enumerate(values):
        out[i] = int_words(int(v), 8)
    return out.reshape(-1)


# --- Montgomery-form Edwards records (oracle side) --------------------------

def mont(v):
    return field.to_mont(v % P)


def unmont(v):
    return field.from_mont(v)


def te_extended_mont(pt_te, lam):
    """TE affine point -> extended (X, Y, T, Z) scaled by lam, Montgomery form."""
    return tuple(mont(v) for v in te.to_extended(pt_te, lam))


def te_prepared_mont(pt_te):
    return tuple(mont(v) for v in te.to_prepared(pt_te))


def normalize_extended_mont(rec):
    """(X, Y, T, Z) in Montgomery form (any lazily reduced representative)
    -> TE affine point, checking T Z = X Y."""
    X, Y, T, Z = (unmont(v) for v in rec)
    return te.from_extended(X, Y, T, Z)
