"""Loaders for the paper's printed fixtures under tests/golden/ (CPU only)."""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def paper_matrices() -> dict:
    """The ABCD matrices printed in Secs. 5 and 6 (four decimals, unprojected)."""
    out, cur = {}, None
    with open(os.path.join(GOLDEN, "paper_matrices.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line[0].isalpha():
                cur = line
                out[cur] = []
                continue
            out[cur].append([float(v) for v in line.split()])
    return {k: np.array(v) for k, v in out.items()}


def printed_values() -> dict:
    vals = {}
    with open(os.path.join(GOLDEN, "printed_values.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if "=" in line:
                k, v = line.split("=")
                vals[k.strip()] = float(v)
    return vals
