"""ORACLE -- test infrastructure, not part of the product.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path
(``paper_2402_11868_amd``) and never imports it.

Contents
--------
* ``heev`` -- MPFR cyclic-Jacobi eigen-solver (``jacobi.c``; 256 bits by
  default, 1024 and more for precisions beyond quad-double) on the exact limb
  sum of the input: the plain definition H = V diag(lam) V^H that
  the paper's FP64-eig + Rayleigh-quotient-iteration method converges to
  (Sec. 2, ZKCM_CUS paragraph).
* ``residuals`` / ``gram`` -- MPFR evaluations of ||H v - lam v|| / ||v|| and
  V^H V on returned limbs exactly as returned.
* ``exact`` -- closed forms and exact rational pins used to check the Jacobi
  solver itself (characteristic polynomial roots at n <= 4, invariants).
* ``svd`` / ``svd_residuals`` -- singular values of a general matrix as the
  nonnegative eigenvalues of its Hermitian dilation [[0, A], [A^H, 0]]
  (eigenvalues +-s_j and |m - n| zeros; Golub & Van Loan, Matrix
  Computations, Sec. 8.6), by the same MPFR Jacobi solver, and the MPFR
  residuals ||A v - s u||, ||A^H u - s v|| of returned triplets.  The paper
  lists the SVD beside the eigendecomposition (Sec. 2).
* ``two_site_theta`` / ``apply_gate`` / ``limb_planes`` -- exact rational
  references for the MPS two-site update (Sec. 1): the contraction
  theta = G (A B) of two site tensors and a two-qubit gate, and the state
  vector of a chain evolved by two-qubit gates, both in Python Fractions,
  plus the greedy split of an exact complex matrix into binary64 limbs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_MPFR_INC = "/opt/conda/include"
_MPFR_LIB = "/opt/conda/lib"
_lib = None

DEFAULT_PREC = 256


def build(force: bool = True) -> str:
    """Compile jacobi.c (gcc + MPFR/GMP from /opt/conda, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", os.path.join(_HERE, "jacobi.c"),
               "-I" + _MPFR_INC, "-L" + _MPFR_LIB, "-Wl,-rpath," + _MPFR_LIB,
               "-lmpfr", "-lgmp", "-lm", "-o", _LIB_PATH + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int
        lib.or_heev.restype = I
        lib.or_heev.argtypes = [I, I, P, I, I, I, I, P, P, P]
        lib.or_heev_limbs.restype = I
        lib.or_heev_limbs.argtypes = [I, I, P, I, I, I, I, I, P, P, P]
        lib.or_residuals.restype = I
        lib.or_residuals.argtypes = [I, I, P, I, I, I, P, I, I, P, I, I, P, P]
        lib.or_gram.restype = I
        lib.or_gram.argtypes = [I, I, I, P, I, I, I, P, P, P]
        lib.or_set_mutation.restype = None
        lib.or_set_mutation.argtypes = [I]
        _lib = lib
    return _lib


def set_mutation(m: int) -> None:
    """Plant deliberate mistake number m in the oracle (0 = none). Pin tests only."""
    _load().or_set_mutation(int(m))


def _planes_colmajor(planes) -> tuple[np.ndarray, int]:
    """Stack limb planes (list of (n,n) complex arrays) into one column-major buffer."""
    if isinstance(planes, np.ndarray) and planes.ndim == 2:
        planes = [planes]
    n = planes[0].shape[0]
    buf = np.empty((len(planes), n, n), dtype=np.complex128)
    for l, P in enumerate(planes):
        buf[l] = np.asarray(P, dtype=np.complex128).T  # row j of buf[l] = column j of P
    return np.ascontiguousarray(buf), n


def _threads(nthreads):
    if nthreads is None:
        nthreads = int(os.environ.get("ORACLE_THREADS", "0")) or (os.cpu_count() or 1)
    return int(nthreads)


class HeevResult:
    def __init__(self, w_limbs, v_limbs, info):
        self.w_limbs = w_limbs          # (limbs, n) limbs of the ascending eigenvalues
        self.v_limbs = v_limbs          # (limbs, n, n) limbs, column k = eigenvector k, or None
        self.sweeps = int(info[0])
        self.rotations = int(info[1])
        self.off_rel = float(info[2])

    @property
    def w(self) -> np.ndarray:
        return self.w_limbs[0]

    @property
    def V(self) -> np.ndarray | None:
        return None if self.v_limbs is None else self.v_limbs[0]


def heev(planes, want_vectors: bool = True, prec: int = DEFAULT_PREC, nthreads=None, limbs: int = 4) -> HeevResult:
    """Eigen-decomposition of sum(planes) (lower triangles read) at `prec` bits;
    results rounded to `limbs` binary64 limbs per value (4 by default, up to 16
    for precisions beyond quad-double; prec must cover 53 * limbs bits)."""
    buf, n = _planes_colmajor(planes)
    L = buf.shape[0]
    w = np.zeros((limbs, n), dtype=np.float64)
    v = np.zeros((limbs, n, n), dtype=np.complex128) if want_vectors else None
    info = np.zeros(3, dtype=np.float64)
    rc = _load().or_heev_limbs(n, L, buf.ctypes.data, n, int(prec), int(bool(want_vectors)), _threads(nthreads),
                               int(limbs), w.ctypes.data, v.ctypes.data if v is not None else None,
                               info.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle or_heev failed: {rc}")
    if v is not None:
        # v[l] is column-major: row k of the buffer holds eigenvector k
        v = np.ascontiguousarray(np.transpose(v, (0, 2, 1)))
    return HeevResult(w, v, info)


def residuals(planes, w_limbs, v_limbs, prec: int = DEFAULT_PREC, nthreads=None):
    """||H v_j - lam_j v_j|| / ||v_j|| and ||v_j|| for every returned pair (MPFR).

    w_limbs: (Lw, k) limbs; v_limbs: (Lv, n, k) complex limbs (column j = pair j).
    """
    buf, n = _planes_colmajor(planes)
    w_limbs = np.ascontiguousarray(np.atleast_2d(np.asarray(w_limbs, dtype=np.float64)))
    v_limbs = np.asarray(v_limbs, dtype=np.complex128)
    if v_limbs.ndim == 2:
        v_limbs = v_limbs[None]
    Lv, nv, k = v_limbs.shape
    assert nv == n and w_limbs.shape[1] == k
    vbuf = np.ascontiguousarray(np.transpose(v_limbs, (0, 2, 1)))  # column-major per plane
    res = np.zeros(k)
    vn = np.zeros(k)
    rc = _load().or_residuals(n, buf.shape[0], buf.ctypes.data, n, k, Lv, vbuf.ctypes.data, n,
                              w_limbs.shape[0], w_limbs.ctypes.data, int(prec), _threads(nthreads),
                              res.ctypes.data, vn.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle or_residuals failed: {rc}")
    return res, vn


def gram(v_limbs, prec: int = DEFAULT_PREC, nthreads=None, full: bool = False):
    """(max_{i!=j} |v_i^H v_j|, max_i |v_i^H v_i - 1| [, |G|]) in MPFR."""
    v_limbs = np.asarray(v_limbs, dtype=np.complex128)
    if v_limbs.ndim == 2:
        v_limbs = v_limbs[None]
    Lv, n, k = v_limbs.shape
    vbuf = np.ascontiguousarray(np.transpose(v_limbs, (0, 2, 1)))
    mo = ctypes.c_double()
    md = ctypes.c_double()
    g = np.zeros((k, k)) if full else None
    rc = _load().or_gram(n, k, Lv, vbuf.ctypes.data, n, int(prec), _threads(nthreads),
                         ctypes.addressof(mo), ctypes.addressof(md),
                         g.ctypes.data if g is not None else None)
    if rc != 0:
        raise RuntimeError(f"oracle or_gram failed: {rc}")
    return (mo.value, md.value, g) if full else (mo.value, md.value)


def _dilation(planes):
    """Limb planes of K = [[0, A], [A^H, 0]] for A given as limb planes (m x n)."""
    out = []
    for A in planes:
        A = np.asarray(A, dtype=np.complex128)
        m, n = A.shape
        K = np.zeros((m + n, m + n), dtype=np.complex128)
        K[:m, m:] = A
        K[m:, :m] = A.conj().T
        out.append(K)
    return out


def svd(planes, prec: int = DEFAULT_PREC, nthreads=None) -> np.ndarray:
    """(4, k) limbs of the k = min(m, n) singular values of sum(planes), descending."""
    planes = [np.asarray(p, dtype=np.complex128) for p in planes]
    m, n = planes[0].shape
    k = min(m, n)
    r = heev(_dilation(planes), want_vectors=False, prec=prec, nthreads=nthreads)
    # the k largest eigenvalues of the dilation, descending
    return np.ascontiguousarray(r.w_limbs[:, ::-1][:, :k])


def svd_residuals(planes, s_limbs, u_limbs, v_limbs, prec: int = DEFAULT_PREC, nthreads=None):
    """For each returned triplet: sqrt(||A v - s u||^2 + ||A^H u - s v||^2) / ||[u; v]||
    (the residual of [u; v] as an eigenvector of the dilation for +s), in MPFR,
    and ||[u; v]||.  u_limbs: (L, m, k), v_limbs: (L, n, k), s_limbs: (Ls, k)."""
    u_limbs = np.asarray(u_limbs, dtype=np.complex128)
    v_limbs = np.asarray(v_limbs, dtype=np.complex128)
    if u_limbs.ndim == 2:
        u_limbs, v_limbs = u_limbs[None], v_limbs[None]
    x = np.concatenate([u_limbs, v_limbs], axis=1)
    return residuals(_dilation(planes), s_limbs, x, prec=prec, nthreads=nthreads)



# ------------------------------------------------ MPS two-site references --
# Exact complex rationals are (re, im) pairs of Fractions.

def _cfr(z):
    from fractions import Fraction
    return (Fraction(float(z.real)), Fraction(float(z.imag)))


def _cmul(a, b):
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def _cadd(a, b):
    return (a[0] + b[0], a[1] + b[1])


def limb_sum_matrix(planes):
    """Exact complex rationals of the limb sum of binary64 complex planes."""
    planes = [np.asarray(p, dtype=np.complex128) for p in planes]
    m, n = planes[0].shape
    out = [[None] * n for _ in range(m)]
    for i in range(m):
        for j in range(n):
            re, im = _cfr(planes[0][i, j])
            for p in planes[1:]:
                r2, i2 = _cfr(p[i, j])
                re, im = re + r2, im + i2
            out[i][j] = (re, im)
    return out


def two_site_theta(A_planes, B_planes, G):
    """theta'[(s1, l), (s2, r)] = sum G[2 s1 + s2, 2 t1 + t2] sum_m A[t1 chi_l + l, m] B[m, t2 chi_r + r]
    exactly: A (2 chi_l x chi) and B (chi x 2 chi_r) as binary64 limb planes, G a 4 x 4
    nested list of exact (re, im) Fractions.  Returns a nested list of (re, im)."""
    from fractions import Fraction
    A = limb_sum_matrix(A_planes)
    B = limb_sum_matrix(B_planes)
    M, K, N = len(A), len(B), len(B[0])
    zero = (Fraction(0), Fraction(0))
    T = [[zero] * N for _ in range(M)]
    for i in range(M):
        for j in range(N):
            acc = zero
            for m in range(K):
                acc = _cadd(acc, _cmul(A[i][m], B[m][j]))
            T[i][j] = acc
    cl, cr = M // 2, N // 2
    out = [[zero] * N for _ in range(M)]
    for l in range(cl):
        for r in range(cr):
            x = [T[t1 * cl + l][t2 * cr + r] for t1 in range(2) for t2 in range(2)]
            for s1 in range(2):
                for s2 in range(2):
                    acc = zero
                    for c in range(4):
                        acc = _cadd(acc, _cmul(G[2 * s1 + s2][c], x[c]))
                    out[s1 * cl + l][s2 * cr + r] = acc
    return out


def limb_planes(T, L=4):
    """Greedy round-to-nearest split of an exact complex matrix into L binary64 limb planes."""
    from fractions import Fraction
    m, n = len(T), len(T[0])
    planes = [np.zeros((m, n), dtype=np.complex128) for _ in range(L)]
    for i in range(m):
        for j in range(n):
            re, im = T[i][j]
            for l in range(L):
                fr, fi = float(re), float(im)
                planes[l][i, j] = complex(fr, fi)
                re -= Fraction(fr)
                im -= Fraction(fi)
    return planes


def apply_gate(psi, n, q, G):
    """Exact state vector of an n-site chain (amplitude index sum s_k 2^(n-1-k), site 0
    most significant) after the gate G (4 x 4, index 2 s_q + s_(q+1)) on sites q, q+1."""
    out = list(psi)
    hi, lo = n - 1 - q, n - 2 - q
    for x in range(2 ** n):
        if (x >> hi) & 1 or (x >> lo) & 1:
            continue
        idx = [x | (a << hi) | (b << lo) for a in range(2) for b in range(2)]
        vals = [psi[i] for i in idx]
        for r in range(4):
            acc = (vals[0][0] * 0, vals[0][1] * 0)
            for c in range(4):
                acc = _cadd(acc, _cmul(G[r][c], vals[c]))
            out[idx[r]] = acc
    return out
