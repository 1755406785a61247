"""Seeded synthetic inputs for the Hermitian eigen-solver.

This module only *builds inputs*: it contains none of the solver's arithmetic,
and both the HIP path's tests/bench and the oracle's self-checks draw their
matrices from here.

Matrix families
---------------
* ``householder_hermitian`` -- H = U diag(lam) U^H, U a product of seeded
  random Householder reflectors, built in binary64 by ``gen.c``.  This is the
  "matrix with a designed spectrum" family used for every workload; the stored
  binary64 matrix (not the design) is the ground truth.
* ``hadamard_exact`` -- H = (1/N) Phi P W diag(lam) W P^T Phi^H with W the
  Sylvester Hadamard matrix, P a seeded permutation and Phi seeded phases in
  {1, i, -1, -i}.  Every entry is an exact dyadic rational that is stored
  exactly in L binary64 limbs, so the eigenvalues are *exactly* lam and the
  eigenvectors exactly Phi P W e_k / sqrt(N).
* ``schmidt_pair`` -- the 2x2 density matrix with eigenvalues exactly 1-eps and
  eps, the squared Schmidt coefficients of the controlled-rotation example in
  the paper's introduction (footnote 1, eps = 2^(-n+1)).
* ``random_elements`` -- Hermitian matrix with i.i.d. U(-1,1) real/imag parts,
  the "random elements" matrices of the paper's diagonalisation timing (Sec. 2.1).
* ``circuit_bond_matrices`` -- the reduced density matrices at every cut of the
  n-qubit state of the paper's introductory circuit (footnote 1): n - 1
  control qubits in |+>, the target in |->, and a multi-controlled Z on one
  seeded control pattern.  Entries are exact dyadic rationals, every matrix
  has rank <= 2 (exact zero eigenvalues), and the target's cut carries the
  Schmidt pair 1 - eps, eps with eps = 2^(-n+1).

Layout convention everywhere: a matrix is a numpy complex128 array ``A`` of
shape (n, n); limb inputs are a list of such arrays whose *exact* sum is the
matrix.  ``colmajor(A)`` gives the column-major buffer handed to C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libzkgen.so")
_lib = None

SEED_BASE = 240211868


def build(force: bool = True) -> str:
    """Compile gen.c into libzkgen.so (plain gcc, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", os.path.join(_HERE, "gen.c"), "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.gen_householder_hermitian.restype = ctypes.c_int
        lib.gen_householder_hermitian.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                                  ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def colmajor(A: np.ndarray) -> np.ndarray:
    """Column-major complex128 buffer (entry (i, j) at offset j*n + i)."""
    return np.ascontiguousarray(np.asarray(A, dtype=np.complex128).T)


def seed_for(config: int, index: int = 0) -> int:
    return SEED_BASE + 1000 * config + index


# ---------------------------------------------------------------- families --

def householder_hermitian(lam, seed: int, m: int | None = None) -> np.ndarray:
    """Hermitian matrix with designed spectrum ``lam`` (binary64, exactly Hermitian)."""
    lam = np.ascontiguousarray(np.asarray(lam, dtype=np.float64))
    n = lam.size
    m = n if m is None else int(m)
    rng = np.random.Generator(np.random.PCG64(seed))
    u = np.ascontiguousarray(rng.standard_normal((m, n, 2)))
    # seeded eigenvalue placement: the design order is shuffled so that the
    # Householder product does not align the spectrum with the coordinate axes
    perm = rng.permutation(n)
    lam = np.ascontiguousarray(lam[perm])
    out = np.zeros(2 * n * n, dtype=np.float64)
    rc = _load().gen_householder_hermitian(n, m, lam.ctypes.data, u.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"gen_householder_hermitian failed: {rc}")
    # out is column-major: entry (i, j) at j*n + i
    return out.view(np.complex128).reshape(n, n).T.copy()


def random_elements(n: int, seed: int) -> np.ndarray:
    """Hermitian matrix with i.i.d. U(-1,1) real and imaginary parts (lower triangle drawn)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.uniform(-1.0, 1.0, (n, n))
    im = rng.uniform(-1.0, 1.0, (n, n))
    A = np.tril(re + 1j * im, -1)
    A = A + A.conj().T + np.diag(rng.uniform(-1.0, 1.0, n))
    return A


def _split_limbs(x: Fraction, L: int):
    """Greedy round-to-nearest split of an exact rational into L binary64 limbs.

    Returns (limbs, remainder).  limb_i = RN(x - sum of previous limbs).
    """
    limbs = []
    r = Fraction(x)
    for _ in range(L):
        f = float(r)  # int/int true division: correctly rounded
        limbs.append(f)
        r -= Fraction(f)
    return limbs, r


def _popcount_parity(a: np.ndarray) -> np.ndarray:
    a = a.astype(np.uint64)
    p = np.zeros_like(a)
    while np.any(a):
        p ^= a & np.uint64(1)
        a >>= np.uint64(1)
    return p


class HadamardExact:
    """Exact-spectrum Hermitian matrix on n = 2^m (see module docstring).

    Attributes: n, lam (sorted ascending, Fractions), planes (list of L
    complex128 arrays whose exact sum is H), vectors(k) exact eigenvectors.
    """

    def __init__(self, lam, seed: int, limbs: int = 1, allow_inexact: bool = False):
        lam = [Fraction(x) for x in lam]
        n = len(lam)
        if n < 1 or n & (n - 1):
            raise ValueError("Hadamard family needs n = 2^m")
        self.n = n
        rng = np.random.Generator(np.random.PCG64(seed))
        self.perm = rng.permutation(n)
        self.q = rng.integers(0, 4, n)          # phase of row i is 1j**q[i]
        self.lam_by_column = lam                # lam[k] belongs to Hadamard column k
        # g(c) = sum_k lam_k (-1)^{popcount(c & k)}, by a fast Walsh-Hadamard
        # transform on exact integers (all lam scaled to a common denominator)
        den = 1
        for x in lam:
            den = max(den, x.denominator)
        for x in lam:
            assert den % x.denominator == 0, "lam must be dyadic"
        g = [int(x * den) for x in lam]
        h = 1
        while h < n:
            for i in range(0, n, 2 * h):
                for j in range(i, i + h):
                    a, b = g[j], g[j + h]
                    g[j], g[j + h] = a + b, a - b
            h *= 2
        vals = [Fraction(gc, den * n) for gc in g]      # entry magnitudes x_c = g(c)/N
        limb_tab = np.zeros((limbs, n), dtype=np.float64)
        self.exact = True
        for c, x in enumerate(vals):
            ls, r = _split_limbs(x, limbs)
            if r != 0:
                self.exact = False
            limb_tab[:, c] = ls
        if not self.exact and not allow_inexact:
            raise ValueError("entries are not exactly representable in %d limbs" % limbs)
        idx = self.perm[:, None] ^ self.perm[None, :]
        rot = (self.q[:, None] - self.q[None, :]) % 4
        unit = np.array([1, 1j, -1, -1j], dtype=np.complex128)[rot]
        self.planes = [limb_tab[l][idx] * unit for l in range(limbs)]
        self.lam = sorted(lam)
        self._order = sorted(range(n), key=lambda k: lam[k])

    def vectors_unnormalised(self) -> np.ndarray:
        """Columns (in ascending eigenvalue order) Phi P W e_k, entries in {±1, ±i}; norm sqrt(n)."""
        n = self.n
        W = 1 - 2 * _popcount_parity(self.perm[:, None].astype(np.uint64) &
                                     np.arange(n, dtype=np.uint64)[None, :]).astype(np.int64)
        phase = np.array([1, 1j, -1, -1j], dtype=np.complex128)[self.q]
        V = phase[:, None] * W
        return V[:, self._order]


def hadamard_exact(lam, seed: int, limbs: int = 1) -> HadamardExact:
    return HadamardExact(lam, seed, limbs)


def schmidt_pair(k: int, omega: complex = 1.0, limbs: int = 2):
    """2x2 matrix [[1/2, (1/2-eps) w], [(1/2-eps) conj(w), 1/2]] with eps = 2^-k.

    Its eigenvalues are exactly 1-eps and eps (the squares of the Schmidt
    coefficients sqrt(1-eps), sqrt(eps)).  omega must be in {±1, ±i}.
    Returns (planes, (eps, 1-eps) as Fractions).
    """
    assert omega in (1, -1, 1j, -1j)
    eps = Fraction(1, 2 ** k)
    off = Fraction(1, 2) - eps
    offl, r = _split_limbs(off, limbs)
    if r != 0:
        raise ValueError("1/2 - 2^-%d needs more than %d limbs" % (k, limbs))
    planes = []
    for l in range(limbs):
        d = 0.5 if l == 0 else 0.0
        A = np.array([[d, offl[l] * omega], [offl[l] * np.conj(omega), d]], dtype=np.complex128)
        planes.append(A)
    return planes, (eps, 1 - eps)


# ----------------------------------------------------------------- spectra --
# The readings below fix details that the named workload specifications leave
# open (the paper itself describes its test matrices only as Hermitian with
# random elements, Sec. 2.1).

def spectrum_c1() -> np.ndarray:
    """n=64: one eigenvalue exactly 2^-20; 63 values prop. to 2^(-k/2), k=0..62, summing to 1-2^-20."""
    k = np.arange(63)
    base = 2.0 ** (-k / 2.0)
    lam = base * ((1.0 - 2.0 ** -20) / base.sum())
    return np.concatenate([lam, [2.0 ** -20]])


def spectrum_c2(seed: int) -> tuple[np.ndarray, np.ndarray]:
    """n=128: 10^(-k/8), k=0..123, four seeded distinct k doubled (exact 2-fold degeneracies), trace 1."""
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    dup = np.sort(rng.choice(124, size=4, replace=False))
    k = np.concatenate([np.arange(124), dup])
    lam = 10.0 ** (-k / 8.0)
    return lam / lam.sum(), dup


def spectrum_c3() -> np.ndarray:
    """n=1024: clusters of 8, lam_{j,m} = 2^(-50 j/127) (1 + m 1e-12), j=0..127, m=0..7 (span 1 .. 2^-50)."""
    j = np.arange(128)[:, None]
    m = np.arange(8)[None, :]
    return (2.0 ** (-50.0 * j / 127.0) * (1.0 + m * 1e-12)).ravel()


def spectrum_c4(s: int) -> np.ndarray:
    """Serving sizes: lam_k prop. to 2^(-39 k/(s-1)), k=0..s-1, trace 1 (tail 2^-39, the 40-qubit pair)."""
    k = np.arange(s)
    lam = 2.0 ** (-39.0 * k / (s - 1))
    return lam / lam.sum()


def spectrum_c5(n: int = 2048, exact: bool = False):
    """{1-2^-59, 2^-59} U {2^(-120 k/(n-2)) : k=1..n-2}.  exact=True returns Fractions (1-2^-59 kept)."""
    k = np.arange(1, n - 1)
    geo = 2.0 ** (-120.0 * k / (n - 2))
    if exact:
        return [Fraction(1) - Fraction(1, 2 ** 59), Fraction(1, 2 ** 59)] + [Fraction(float(x)) for x in geo]
    return np.concatenate([[1.0 - 2.0 ** -59, 2.0 ** -59], geo])


def spectrum_c5_dyadic(n: int, bits: int = 40) -> list:
    """Exact form of the quad-double spectrum for the Hadamard family: {1-2^-59, 2^-59}
    and 2^(-120 k/(n-2)), k=1..n-2, each rounded to `bits` significant bits (Fractions)."""
    lam = [Fraction(1) - Fraction(1, 2 ** 59), Fraction(1, 2 ** 59)]
    for k in range(1, n - 1):
        m, e = np.frexp(2.0 ** (-120.0 * k / (n - 2)))
        lam.append(Fraction(int(round(m * 2 ** bits)), 2 ** bits) * Fraction(2) ** int(e))
    return lam


def serving_sizes() -> list[int]:
    return list(range(16, 513, 16))


def poisson_stream(rate_hz: float, count: int, seed: int, sizes=None):
    """Open-loop Poisson arrivals: (arrival_times_s, sizes) with exponential gaps of mean 1/rate."""
    sizes = serving_sizes() if sizes is None else list(sizes)
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, count)
    t = np.cumsum(gaps)
    sz = np.asarray(sizes)[rng.integers(0, len(sizes), count)]
    return t, sz


# ------------------------------------------------------------- workloads --

def workload(config: int, index: int = 0, n: int | None = None) -> dict:
    """The matrices of the named workloads (Householder family, binary64 = 1 limb).

    config 1: 64x64 one matrix; config 2: 256 x 128x128 batch (index selects the
    member); config 3: 1024x1024 clustered; config 4: serving size n (index
    selects the pool member); config 5: 2048x2048 or the 256 companions (n=256).
    """
    seed = seed_for(config, index)
    if config == 1:
        lam = spectrum_c1()
    elif config == 2:
        lam, _ = spectrum_c2(seed)
    elif config == 3:
        lam = spectrum_c3()
    elif config == 4:
        lam = spectrum_c4(n or 512)
    elif config == 5:
        lam = spectrum_c5(n or 2048)
    else:
        raise ValueError(config)
    A = householder_hermitian(lam, seed)
    return {"A": A, "design": np.sort(lam), "seed": seed}


def circuit_bond_matrices(n: int, seed: int = 0):
    """Bond matrices of the state C^(n-1)-Z (|+>^(n-1) |->) (paper, Sec. 1,
    footnote 1, with the rotation U = Z, which maps |-> to the orthogonal |+>).

    The qubits form a chain: n - 1 controls, then the target.  For each cut
    after the first k qubits (k = 1 .. n-1) the reduced density matrix of the
    smaller side is returned (order min(2^k, 2^(n-k))) as a dict with keys
    ``k``, ``rho`` (complex128, exact), ``R`` (integer matrix, rho = R / 2^n)
    and ``scale`` = n.  Amplitudes are s(x) / 2^(n/2) with s(x) = +-1: the
    target bit t gives (-1)^t, except on the control pattern, where the
    target is |+> and s = +1.  The state is a product state plus a product
    correction, so every cut has Schmidt rank <= 2; across the last cut the
    Schmidt coefficients squared are exactly 1 - 2^(-n+1) and 2^(-n+1).
    """
    if n < 2 or n > 24:
        raise ValueError("2 <= n <= 24")
    rng = np.random.Generator(np.random.PCG64(seed + 7919 * n))
    pattern = int(rng.integers(0, 2 ** (n - 1)))
    x = np.arange(2 ** n, dtype=np.int64)
    s = np.where((x & 1) == 1, -1, 1).astype(np.int64)
    s[(x >> 1) == pattern] = 1
    out = []
    for k in range(1, n):
        S = s.reshape(2 ** k, 2 ** (n - k))   # rows: the first k qubits of the chain
        R = S @ S.T if k <= n - k else S.T @ S
        rho = (R.astype(np.float64) / float(2 ** n)).astype(np.complex128)
        out.append({"k": k, "rho": rho, "R": R, "scale": n})
    return out


def cnz_staircase(n: int, dps: int = 80):
    """A nearest-neighbour circuit that prepares the state of the paper's
    introductory circuit, C^(n-1)-Z on |+>^(n-1) |-> (Sec. 1, footnote 1), from
    |0...0>:  psi = |+>^(n-1) |-> + 2^(-(n-2)/2) |1...1>, a sum of two product
    states (bond dimension 2 at every cut).

    Sequential generation of a matrix product state: psi is written in
    right-canonical form B_0 .. B_{n-1} (LQ steps from the right, in mpmath at
    `dps` digits); gate k acts on qubits (k, k+1) and maps |a>_k |0>_{k+1} to
    sum_{s, b} B_k[a, s, b] |s>_k |b>_{k+1} (the last gate folds B_{n-1} in),
    completed to a unitary by Gram-Schmidt.  Returns a list of (k, G_hi, G_lo):
    4 x 4 complex gates (row and column index 2 s_k + s_{k+1}) as two binary64
    limbs.  Applied in order to |0...0>, they give psi to the gates' rounding.
    """
    import mpmath as mp
    if n < 3:
        raise ValueError("n >= 3")
    mp.mp.dps = dps
    r2 = 1 / mp.sqrt(2)
    plus, one, minus = [r2, r2], [mp.mpf(0), mp.mpf(1)], [r2, -r2]
    c = mp.mpf(2) ** (-(n - 2) / mp.mpf(2))
    # raw MPS: M[k][a][s][b]
    M = []
    M.append([[[plus[s], c * one[s]] for s in range(2)]])                      # 1 x 2 x 2
    for _ in range(1, n - 1):
        M.append([[[plus[s] if a == b == 0 else (one[s] if a == b == 1 else mp.mpf(0)) for b in range(2)]
                   for s in range(2)] for a in range(2)])                       # 2 x 2 x 2
    M.append([[[minus[s]] for s in range(2)], [[one[s]] for s in range(2)]])   # 2 x 2 x 1

    def lq(mat):
        """mat (r x c, r <= c) = L Q, Q with orthonormal rows (Gram-Schmidt on rows)."""
        r, cc = len(mat), len(mat[0])
        Q, L = [], [[mp.mpf(0)] * r for _ in range(r)]
        for i in range(r):
            v = list(mat[i])
            for j in range(i):
                d = mp.fsum(v[k] * mp.conj(Q[j][k]) for k in range(cc))
                L[i][j] = d
                v = [v[k] - d * Q[j][k] for k in range(cc)]
            nv = mp.sqrt(mp.fsum(abs(x) ** 2 for x in v))
            L[i][i] = nv
            Q.append([x / nv for x in v])
        return L, Q

    B = [None] * n
    for k in range(n - 1, 0, -1):
        cl, cr = len(M[k]), len(M[k][0][0])
        mat = [[M[k][a][s][b] for s in range(2) for b in range(cr)] for a in range(cl)]
        L, Q = lq(mat)
        B[k] = [[[Q[a][s * cr + b] for b in range(cr)] for s in range(2)] for a in range(cl)]
        # absorb L into site k-1
        pl = len(M[k - 1])
        M[k - 1] = [[[mp.fsum(M[k - 1][a][s][m] * L[m][b] for m in range(cl)) for b in range(cl)]
                     for s in range(2)] for a in range(pl)]
    nrm = mp.sqrt(mp.fsum(abs(M[0][0][s][b]) ** 2 for s in range(2) for b in range(2)))
    B[0] = [[[M[0][0][s][b] / nrm for b in range(2)] for s in range(2)]]

    def complete(cols):
        """4 x 4 unitary whose columns 0 and 2 are the given orthonormal columns."""
        basis = [list(cols[0]), None, list(cols[1]), None] if len(cols) == 2 else [list(cols[0]), None, None, None]
        have = [v for v in basis if v is not None]
        extra = []
        for e in range(4):
            v = [mp.mpf(1) if i == e else mp.mpf(0) for i in range(4)]
            for u in have + extra:
                d = mp.fsum(mp.conj(u[i]) * v[i] for i in range(4))
                v = [v[i] - d * u[i] for i in range(4)]
            nv = mp.sqrt(mp.fsum(abs(x) ** 2 for x in v))
            if nv > mp.mpf(10) ** (-dps // 2):
                extra.append([x / nv for x in v])
        slots = [i for i in range(4) if basis[i] is None]
        for i, v in zip(slots, extra):
            basis[i] = v
        return basis   # list of columns

    gates = []
    for k in range(n - 1):
        if k == 0:
            cols = [[B[0][0][s][b] for s in range(2) for b in range(2)]]
        elif k < n - 2:
            cols = [[B[k][a][s][b] for s in range(2) for b in range(2)] for a in range(2)]
        else:
            cols = [[mp.fsum(B[k][a][s][m] * B[k + 1][m][t][0] for m in range(2)) for s in range(2) for t in range(2)]
                    for a in range(2)]
        U = complete(cols)
        hi = np.zeros((4, 4), dtype=np.complex128)
        lo = np.zeros((4, 4), dtype=np.complex128)
        for col in range(4):
            for row in range(4):
                z = mp.mpc(U[col][row])
                h = complex(float(z.real), float(z.imag))
                l = complex(float(z.real - h.real), float(z.imag - h.imag))
                hi[row, col], lo[row, col] = h, l
        gates.append((k, hi, lo))
    return gates

