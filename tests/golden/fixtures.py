"""Readers for the text fixtures in this folder."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def read_sections(name):
    """Parse a fixture: '[key]' headers followed by whitespace-separated rows.
    Returns {key: list of token lists}; '#' lines are comments."""
    out, key = {}, None
    with open(os.path.join(HERE, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("[") and line.endswith("]"):
                key = line[1:-1]
                out[key] = []
                continue
            out[key].append(line.split())
    return out


def printed_values(tokens):
    """Values and the half-unit-of-last-digit tolerance of each printed number."""
    vals, tols = [], []
    for t in tokens:
        vals.append(float(t))
        dec = len(t.split(".")[1]) if "." in t else 0
        tols.append(0.5 * 10.0 ** (-dec))
    return np.array(vals), np.array(tols)


def worked_example():
    s = read_sections("worked_example.txt")
    A = np.array([[float(v) for v in row] for row in s["A"]])
    d = dict(A=A)
    d["f"] = np.array([float(v) for v in s["f"][0]])
    d["part_ptr"] = np.array([int(v) for v in s["part_ptr"][0]], dtype=np.int64)
    d["c"] = np.array([int(v) for v in s["c"][0]], dtype=np.int64)
    for k in ("g", "zhat", "x"):
        d[k] = printed_values(s[k][0])
    rows = [printed_values(r) for r in s["G"]]
    d["G"] = (np.array([r[0] for r in rows]), np.array([r[1] for r in rows]))
    return d
