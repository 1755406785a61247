"""Host planning of the all-pairs refinement (csrc/ap_host.h), built with g++.

The blocks must be exactly the finest partition of the sorted positions into
runs such that no coupled pair straddles a boundary (checked by brute force
over explicit random coupling graphs), and the order of the Rayleigh quotients
must sort double-double values exactly and stably.
"""
import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "ap_shim.cpp")
# one library per process: parallel test workers must not load a file another is still writing
LIB = os.path.join(HERE, "host", f"libap_shim.{os.getpid()}.so")


@pytest.fixture(scope="module")
def lib():
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", SRC, "-o", LIB])
    l = ctypes.CDLL(LIB)
    os.unlink(LIB)
    P = ctypes.c_void_p
    l.t_ap_runs.argtypes = [P, ctypes.c_int, P, P]
    l.t_ap_runs.restype = ctypes.c_int
    l.t_ap_sorted_order.argtypes = [P, ctypes.c_int, P]
    return l


def _runs(lib, reach):
    n = len(reach)
    r = np.ascontiguousarray(reach, dtype=np.int32)
    s = np.zeros(n, np.int32)
    e = np.zeros(n, np.int32)
    k = lib.t_ap_runs(r.ctypes.data, n, s.ctypes.data, e.ctypes.data)
    return list(zip(s[:k].tolist(), e[:k].tolist()))


@pytest.mark.parametrize("seed", range(40))
def test_runs_are_the_finest_non_straddled_partition(lib, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    m = int(rng.integers(0, 2 * n))
    pairs = set()
    for _ in range(m):
        a, b = sorted(rng.integers(0, n, 2).tolist())
        if a < b and rng.random() < 0.7:
            b = min(n - 1, a + int(rng.integers(1, 4)))   # mostly short-range, as near eigenvalues couple
        if a < b:
            pairs.add((a, b))
    reach = list(range(n))
    for a, b in pairs:
        reach[b] = min(reach[b], a)
    runs = _runs(lib, reach)
    # a partition of 0..n-1 into consecutive runs
    assert runs[0][0] == 0 and runs[-1][1] == n
    assert all(runs[k][1] == runs[k + 1][0] for k in range(len(runs) - 1))
    bounds = {s for s, _ in runs[1:]}
    for p in range(1, n):
        straddled = any(a < p <= b for a, b in pairs)
        assert (p in bounds) == (not straddled), (p, straddled)


def test_runs_special_cases(lib):
    assert _runs(lib, [0]) == [(0, 1)]
    assert _runs(lib, [0, 1, 2, 3]) == [(0, 1), (1, 2), (2, 3), (3, 4)]
    assert _runs(lib, [0, 0, 0, 0]) == [(0, 4)]
    # a long-range coupling merges everything in between
    assert _runs(lib, [0, 1, 2, 0, 4]) == [(0, 4), (4, 5)]


def test_sorted_order_double_double(lib):
    rng = np.random.default_rng(3)
    n = 200
    hi = np.round(rng.standard_normal(n), 2)          # many equal leading parts
    lo = rng.standard_normal(n) * 1e-20 * np.abs(hi)
    lo[::7] = 0.0
    hi[::11] = 0.5
    lo[::11] = 0.0                                     # exact ties
    th = np.ascontiguousarray(np.concatenate([hi, lo]))
    out = np.zeros(n, np.int32)
    lib.t_ap_sorted_order(th.ctypes.data, n, out.ctypes.data)
    vals = [Fraction(float(hi[i])) + Fraction(float(lo[i])) for i in range(n)]
    ref = sorted(range(n), key=lambda i: (vals[i], i))   # stable on exact value
    assert out.tolist() == ref
