"""Readers for the text fixtures in this folder."""

import os

HERE = os.path.dirname(os.path.abspath(__file__))


def read_kv(name):
    vals = {}
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = (s.strip() for s in line.split("=", 1))
            vals[k] = int(v, 0)
    return vals
