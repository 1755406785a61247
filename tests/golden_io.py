"""Reader of the stored oracle values under tests/golden/ (written by make_golden.py)."""
import hashlib
import os

import numpy as np

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def sha(A) -> str:
    return hashlib.sha256(W.colmajor(A).tobytes()).hexdigest()


def load(tag: str):
    """(header dict, (4, n) limb array) of tests/golden/<tag>_eigs.txt."""
    hdr, rows = {}, []
    with open(os.path.join(GOLDEN, tag.replace(":", "_") + "_eigs.txt")) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                if ":" in line:
                    k, v = line[1:].split(":", 1)
                    hdr[k.strip()] = v.strip()
                continue
            rows.append([float.fromhex(x) for x in line.split()])
    return hdr, np.array(rows).T.copy()


def exists(tag: str) -> bool:
    return os.path.exists(os.path.join(GOLDEN, tag.replace(":", "_") + "_eigs.txt"))
