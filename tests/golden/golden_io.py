"""Reader of the whole-solve goldens ``pcg_<case>.txt`` (written by
make_pcg_goldens.py from the oracle).  It holds no arithmetic of the method
and imports nothing of the oracle, so the benchmark can quote the stored
values."""

from __future__ import annotations

import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def golden_path(name: str) -> str:
    return os.path.join(HERE, f"pcg_{name}.txt")


def load_golden(name: str) -> dict:
    """key = value lines as strings; the sample lines (x y z u) as an array [n][4]."""
    kv, rows = {}, []
    with open(golden_path(name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if "=" in line:
                key, val = line.split("=", 1)
                kv[key.strip()] = val.strip()
            else:
                rows.append([float(v) for v in line.split()])
    kv["samples"] = np.array(rows)
    return kv
