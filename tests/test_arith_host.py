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
# one library per process: parallel test workers must not load a file another is still writing
LIB = os.path.join(HERE, "host", f"libarith_shim.{os.getpid()}.so")

U = Fraction(1, 2 ** 53)


@pytest.fixture(scope="module")
def lib():
    subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", SRC, "-o", LIB])
    l = ctypes.CDLL(LIB)
    os.unlink(LIB)
    P, D = ctypes.c_void_p, ctypes.c_double
    for name in ("t_dd_add", "t_dd_mul", "t_dd_div", "t_qd_add", "t_qd_mul", "t_qd_div"):
        getattr(l, name).argtypes = [P, P, P]
    for name in ("t_dd_sqrt", "t_qd_sqrt", "t_qd_renorm16"):
        getattr(l, name).argtypes = [P, P]
    l.t_casc3.argtypes = [ctypes.c_int, P, P, P, P]
    l.t_casc4.argtypes = [ctypes.c_int, P, P, P, P]
    l.t_casc_n8.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P]
    l.t_casc_n16.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P]
    l.t_renorm_n8_24.argtypes = [P, P]
    l.t_add_n16_d.argtypes = [P, D, P]
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


def test_cascaded_accumulator_cancelling_sum(lib):
    """Casc3: a long sum of binary64 x double-double products that cancels to
    ~1e-31 of its terms (the residual of an eigenvector of the largest
    eigenvalue) is accurate to ~u^3 n max|term|, far below the ~1e-30 that
    double-double accumulation reaches at n = 1024."""
    rng = np.random.Generator(np.random.PCG64(11))
    n = 1024
    x = rng.standard_normal(n) / 32
    y = [split(Fraction(float(a)) + Fraction(float(b)) * U, 2) for a, b in
         zip(rng.standard_normal(n) / 32, rng.standard_normal(n) / 32)]
    yh = np.array([t[0] for t in y])
    yl = np.array([t[1] for t in y])
    exact = sum((Fraction(float(a)) * (Fraction(float(b)) + Fraction(float(c))) for a, b, c in zip(x, yh, yl)),
                Fraction(0))
    # the last term cancels the sum down to about 1e-31 of the terms
    target = exact - Fraction(1, 10 ** 34)
    last = split(-target, 2)
    xs = np.r_[x, 1.0]
    yhs = np.r_[yh, last[0]]
    yls = np.r_[yl, last[1]]
    total = exact + Fraction(float(last[0])) + Fraction(float(last[1]))
    r = np.zeros(2)
    lib.t_casc3(n + 1, xs.ctypes.data, yhs.ctypes.data, yls.ctypes.data, r.ctypes.data)
    err = abs(F(r) - total)
    mean_term = Fraction(float(np.mean(np.abs(x * yh))))
    # per-term roundings of size u^2 |term| add up like a random walk: allow
    # 16 sqrt(n) u^2 mean|term| (~4e-33 here).  A double-double accumulation
    # of the same terms rounds at u^2 times the running partial sums
    # (~3e-32 here), and dropping the product error or the low product
    # leaves errors of u |term|.
    assert abs(total) < Fraction(1, 10 ** 33)
    assert err <= 16 * 32 * U * U * mean_term, float(err)


@pytest.mark.parametrize("cancel", [False, True])
def test_cascaded_qd_accumulator(lib, cancel):
    """Casc4: sums of +-x*y over quad-double operands (wide exponent spread,
    optionally cancelling to 1e-50 of the terms) within a few u^4 per term."""
    rng = np.random.Generator(np.random.PCG64(12 + cancel))
    n = 64
    xs = [rand_mp(rng, 4, spread=8) for _ in range(n)]
    ys = [rand_mp(rng, 4, spread=8) for _ in range(n)]
    sg = rng.choice([-1.0, 1.0], n)
    exact = sum((Fraction(int(s)) * F(x) * F(y) for s, x, y in zip(sg, xs, ys)), Fraction(0))
    if cancel:
        # one more term cancels the sum down to ~1e-50 of the terms
        last = split(-(exact - exact * Fraction(1, 10 ** 50)), 4)
        xs.append(last)
        ys.append(np.array([1.0, 0.0, 0.0, 0.0]))
        sg = np.r_[sg, 1.0]
        exact = exact * Fraction(1, 10 ** 50) + (F(last) + (exact - exact * Fraction(1, 10 ** 50)))
    m = len(xs)
    X = np.ascontiguousarray(np.concatenate(xs))
    Y = np.ascontiguousarray(np.concatenate(ys))
    S = np.ascontiguousarray(sg)
    r = np.zeros(4)
    lib.t_casc4(m, X.ctypes.data, Y.ctypes.data, S.ctypes.data, r.ctypes.data)
    mag = sum((abs(F(x) * F(y)) for x, y in zip(xs, ys)), Fraction(0))
    err = abs(F(r) - exact)
    # levels 0..3 are exact; the plain last level (order-4 products, order-3
    # product errors, level-3 TwoSum errors) and the dropped order >= 5
    # products leave about u^5 per term: allow u^4 of the terms' total size.
    # A dropped order-3 or order-4 partial product leaves errors of u^3 or u^4
    # per term (the first version of this accumulator stopped at order 3 and
    # measured 10-100 u^4 here).
    assert err <= U ** 4 * mag / 4, float(err / mag)


# ---------------------------------------------- beyond quad-double (L limbs) --
def rand_long(rng, L, e):
    """A value with about 53 L significant bits at exponent e, split into L limbs."""
    x = Fraction(0)
    for q in range(L + 1):
        x += Fraction(int(rng.integers(-2 ** 62, 2 ** 62))) * Fraction(2) ** (e - 62 - 60 * q)
    return split(x, L)


def _nonoverlap(r):
    """each limb at most half an ulp of the one before (or zero after a zero)"""
    for a, b in zip(r[:-1], r[1:]):
        if a == 0.0:
            assert b == 0.0
        else:
            assert abs(b) <= np.spacing(abs(a)) / 2 * (1 + 1e-15)


@pytest.mark.parametrize("L", [8, 16])
@pytest.mark.parametrize("mm", [0, 1])
def test_cascade_n_limbs(lib, L, mm):
    """Sums of exact products at L-limb precision (the precision polishing's
    accumulator): error <= 8 n u^L sum |x_i y_i|, limbs non-overlapping, with
    cancelling terms and a spread of exponents."""
    rng = np.random.default_rng(40 + L + mm)
    f = lib.t_casc_n8 if L == 8 else lib.t_casc_n16
    for trial in range(6):
        n = int(rng.integers(1, 40))
        xs = [rand_long(rng, L, int(rng.integers(-30, 30))) for _ in range(n)]
        ys = [rand_long(rng, L, int(rng.integers(-30, 30))) for _ in range(n)]
        if trial % 2:
            # heavy cancellation: the second half repeats the first with the sign
            # flipped and a tiny relative perturbation (2^-300) of y, renormalised
            h = n // 2
            for i in range(h):
                xs[h + i] = -xs[i]
                ys[h + i] = split(F(ys[i]) * (1 + Fraction(1, 2 ** 300)), L)
        if mm:
            x = np.concatenate(xs)
            exact = sum((F(a) * F(b) for a, b in zip(xs, ys)), Fraction(0))
            mag = sum((abs(F(a) * F(b)) for a, b in zip(xs, ys)), Fraction(0))
        else:
            x = np.array([a[0] for a in xs])
            exact = sum((Fraction(float(a)) * F(b) for a, b in zip(x, ys)), Fraction(0))
            mag = sum((abs(Fraction(float(a)) * F(b)) for a, b in zip(x, ys)), Fraction(0))
        y = np.concatenate(ys)
        r = np.zeros(L)
        f(n, mm, x.ctypes.data, y.ctypes.data, r.ctypes.data)
        err = abs(F(r) - exact)
        assert err <= 8 * n * U ** L * mag, (L, mm, trial, float(err / mag))
        _nonoverlap(r)


def test_renorm_n_exact_sum(lib):
    """24 overlapping terms into 8 limbs: the sum kept to u^8 relative, limbs
    non-overlapping."""
    rng = np.random.default_rng(77)
    for _ in range(20):
        t = np.array([float(rng.standard_normal()) * 2.0 ** int(rng.integers(-200, 10)) for _ in range(24)])
        r = np.zeros(8)
        lib.t_renorm_n8_24(t.ctypes.data, r.ctypes.data)
        exact = F(t)
        mag = sum((abs(Fraction(float(v))) for v in t), Fraction(0))
        assert abs(F(r) - exact) <= 4 * U ** 8 * mag
        _nonoverlap(r)


def test_add_n_d_16(lib):
    """a + b with a 16-limb value exact to u^16 of |a| + |b|."""
    rng = np.random.default_rng(78)
    for _ in range(20):
        a = rand_long(rng, 16, int(rng.integers(-20, 20)))
        b = float(rng.standard_normal()) * 2.0 ** int(rng.integers(-40, 40))
        r = np.zeros(16)
        lib.t_add_n16_d(a.ctypes.data, b, r.ctypes.data)
        exact = F(a) + Fraction(b)
        assert abs(F(r) - exact) <= 4 * U ** 16 * (abs(F(a)) + abs(Fraction(b)))
        _nonoverlap(r)

