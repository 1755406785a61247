"""Write stored oracle eigenvalues for the named workloads.

Calls only ``oracle`` (the MPFR Jacobi solver) and ``workloads`` (the seeded
generators); no value here comes from the HIP path.  Each output file holds a
header (workload, seed, SHA-256 of the column-major complex128 matrix bytes,
oracle precision/sweeps) and one line per ascending eigenvalue with its four
binary64 limbs in hex-float form (exact).

usage: python tests/golden/make_golden.py c1 | c3 | c2:<index> | c4:<n>:<index> [--threads T]
"""
import argparse
import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def matrix_sha256(A: np.ndarray) -> str:
    return hashlib.sha256(W.colmajor(A).tobytes()).hexdigest()


def golden_path(tag: str) -> str:
    return os.path.join(HERE, tag.replace(":", "_") + "_eigs.txt")


def load_golden(tag: str):
    """(header dict, (4, n) limb array) of a stored golden file."""
    hdr = {}
    rows = []
    with open(golden_path(tag)) as f:
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


def build_matrix(tag: str):
    parts = tag.split(":")
    cfg = int(parts[0][1:])
    if cfg in (1, 3):
        wl = W.workload(cfg)
    elif cfg == 2:
        wl = W.workload(2, index=int(parts[1]))
    elif cfg == 4:
        wl = W.workload(4, index=int(parts[2]), n=int(parts[1]))
    elif cfg == 5:
        wl = W.workload(5, index=int(parts[2]), n=int(parts[1]))
    else:
        raise ValueError(tag)
    return wl


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("tag")
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    wl = build_matrix(args.tag)
    A = wl["A"]
    t0 = time.time()
    r = oracle.heev([A], want_vectors=False, nthreads=args.threads or None)
    dt = time.time() - t0
    with open(golden_path(args.tag) + ".tmp", "w") as f:
        f.write(f"# workload: {args.tag}\n")
        f.write(f"# n: {A.shape[0]}\n")
        f.write(f"# seed: {wl['seed']}\n")
        f.write(f"# sha256: {matrix_sha256(A)}\n")
        f.write(f"# oracle: MPFR cyclic Jacobi, {oracle.DEFAULT_PREC} bits, sweeps {r.sweeps}, "
                f"off/||A||_F {r.off_rel:.3e}, {dt:.1f} s\n")
        f.write("# columns: four binary64 limbs of each ascending eigenvalue (hex float)\n")
        for k in range(A.shape[0]):
            f.write(" ".join(float(x).hex() for x in r.w_limbs[:, k]) + "\n")
    os.replace(golden_path(args.tag) + ".tmp", golden_path(args.tag))
    print(f"{args.tag}: n={A.shape[0]} sweeps={r.sweeps} {dt:.1f}s -> {golden_path(args.tag)}")


if __name__ == "__main__":
    main()
