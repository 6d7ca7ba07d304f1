"""Readers for the small text fixtures in this folder."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def read_kv(name):
    out = {}
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, val = (x.strip() for x in line.split("=", 1))
            rows = [np.array([float(t) for t in r.split()]) for r in val.split(";")]
            out[key] = rows[0] if len(rows) == 1 else np.stack(rows)
    return out
