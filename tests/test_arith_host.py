"""Host build of the multi-limb arithmetic (csrc/mp.h) against exact rationals.

Error-free transforms must be exact; double-double operations must stay within
small multiples of u^2 (u = 2^-53) relative error (Joldes, Muller, Popescu
2017 bounds: add <= 3u^2, mul <= 4u^2); quad-double within small multiples of
u^4.  Operands include heavy cancellation and wide exponent spread.
"""
import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "arith_shim.cpp")
LIB = os.path.join(HERE, "host", "libarith_shim.so")

U = Fraction(1, 2 ** 53)


@pytest.fixture(scope="module")
def lib():
    subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", SRC, "-o", LIB])
    l = ctypes.CDLL(LIB)
    P, D = ctypes.c_void_p, ctypes.c_double
    for name in ("t_dd_add", "t_dd_mul", "t_dd_div", "t_qd_add", "t_qd_mul", "t_qd_div"):
        getattr(l, name).argtypes = [P, P, P]
    for name in ("t_dd_sqrt", "t_qd_sqrt", "t_qd_renorm16"):
        getattr(l, name).argtypes = [P, P]
    l.t_two_sum.argtypes = [D, D, P, P]
    l.t_two_prod.argtypes = [D, D, P, P]
    return l


def F(x):
    return sum((Fraction(float(v)) for v in np.atleast_1d(x)), Fraction(0))


def split(x: Fraction, L: int):
    out = []
    r = x
    for _ in range(L):
        f = float(r)
        out.append(f)
        r -= Fraction(f)
    return np.array(out)


def rand_mp(rng, L, spread=60):
    e = int(rng.integers(-spread, spread))
    x = Fraction(int(rng.integers(-2 ** 62, 2 ** 62))) * Fraction(2) ** (e - 62)
    x += Fraction(int(rng.integers(-2 ** 62, 2 ** 62))) * Fraction(2) ** (e - 62 - 64)
    x += Fraction(int(rng.integers(-2 ** 62, 2 ** 62))) * Fraction(2) ** (e - 62 - 128)
    x += Fraction(int(rng.integers(-2 ** 62, 2 ** 62))) * Fraction(2) ** (e - 62 - 192)
    return split(x, L)


def call2(f, a, b, L):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    r = np.zeros(L)
    f(a.ctypes.data, b.ctypes.data, r.ctypes.data)
    return r


def test_eft_exact(lib):
    rng = np.random.Generator(np.random.PCG64(1))
    s, e = ctypes.c_double(), ctypes.c_double()
    for _ in range(2000):
        a = float(rng.standard_normal() * 2.0 ** int(rng.integers(-60, 60)))
        b = float(rng.standard_normal() * 2.0 ** int(rng.integers(-60, 60)))
        lib.t_two_sum(ctypes.c_double(a), ctypes.c_double(b), ctypes.byref(s), ctypes.byref(e))
        assert Fraction(s.value) + Fraction(e.value) == Fraction(a) + Fraction(b)
        lib.t_two_prod(ctypes.c_double(a), ctypes.c_double(b), ctypes.byref(s), ctypes.byref(e))
        assert Fraction(s.value) + Fraction(e.value) == Fraction(a) * Fraction(b)


@pytest.mark.parametrize("L,op", [(2, "add"), (2, "mul"), (2, "div"), (4, "add"), (4, "mul"), (4, "div")])
def test_binary_ops(lib, L, op):
    rng = np.random.Generator(np.random.PCG64(10 + L))
    f = getattr(lib, f"t_{'dd' if L == 2 else 'qd'}_{op}")
    bound = {2: {"add": 4, "mul": 6, "div": 16}, 4: {"add": 16, "mul": 32, "div": 64}}[L][op]
    ul = U ** L
    worst = 0.0
    for it in range(1500):
        a = rand_mp(rng, L)
        b = rand_mp(rng, L)
        if op == "add" and it % 3 == 0:
            # heavy cancellation: b close to -a
            b = split(-F(a) + F(rand_mp(rng, L, 5)) * Fraction(2) ** (-int(rng.integers(40, 150))), L)
        if op == "div" and F(b) == 0:
            continue
        r = call2(f, a, b, L)
        exact = {"add": F(a) + F(b), "mul": F(a) * F(b), "div": F(a) / F(b) if F(b) != 0 else 0}[op]
        got = F(r)
        if exact == 0:
            assert got == 0
            continue
        rel = abs(got - exact) / abs(exact)
        worst = max(worst, float(rel / ul))
        assert rel <= bound * ul, f"{op} L={L}: rel err {float(rel):.3e} > {float(bound * ul):.3e}"
        # output must be a normalised expansion: |limb_{i+1}| <= ulp(limb_i)
        for i in range(L - 1):
            if r[i] != 0:
                assert abs(r[i + 1]) <= np.spacing(abs(r[i])), f"{op} not normalised: {r}"


@pytest.mark.parametrize("L", [2, 4])
def test_sqrt(lib, L):
    rng = np.random.Generator(np.random.PCG64(30 + L))
    f = lib.t_dd_sqrt if L == 2 else lib.t_qd_sqrt
    ul = U ** L
    for _ in range(500):
        a = np.abs(rand_mp(rng, L))
        a = split(abs(F(a)), L)
        r = np.zeros(L)
        f(np.ascontiguousarray(a).ctypes.data, r.ctypes.data)
        x = F(r)
        # |x^2 - a| / a <= c u^L  (relative error of sqrt is half of that)
        assert abs(x * x - F(a)) / F(a) <= 16 * ul


def test_renorm_many_terms(lib):
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(1000):
        t = rng.standard_normal(16) * 2.0 ** rng.integers(-200, 10, 16).astype(float)
        t = np.ascontiguousarray(t)
        r = np.zeros(4)
        lib.t_qd_renorm16(t.ctypes.data, r.ctypes.data)
        exact = F(t)
        if exact == 0:
            continue
        assert abs(F(r) - exact) / abs(exact) <= 8 * U ** 4
