// Multi-limb floating-point arithmetic (double-double and quad-double) built
// from error-free transforms, for host and device code.
//
// The precision-recovery stage of the method (Rayleigh quotient iteration after
// an FP64 eigendecomposition, Sec. 2 "ZKCM_CUS") runs in more than binary64
// precision because eigenvalues as small as 2^-(n-1) (the Schmidt pair of
// Sec. 1, footnote 1) must be resolved.  A value is an unevaluated sum of L
// binary64 limbs: L = 2 is double-double (~106 bits), L = 4 quad-double
// (~212 bits).
//
// Building blocks (all exact, round-to-nearest binary64, no FMA contraction):
//   two_sum       Knuth: s + e == a + b exactly.
//   fast_two_sum  Dekker: same, requires |a| >= |b| (or a == 0).
//   two_prod      p + e == a * b exactly, e = fma(a, b, -p).
// Double-double operations follow the accurate algorithms analysed by Joldes,
// Muller and Popescu (ACM TOMS 44(2), 2017): add with relative error <= 3u^2,
// multiplication with error <= 4u^2 (u = 2^-53).  Quad-double operations build
// an expansion of the exact partial terms and renormalise it with two
// error-free VecSum passes followed by a branch-on-error extraction of the four
// leading non-overlapping limbs (Joldes, Marty, Muller, Popescu, "Arithmetic
// algorithms for extended precision using floating-point expansions", IEEE TC
// 2016), in the spirit of Hida, Li and Bailey's quad-double library (2001).
//
// Every file including this header must be compiled with -ffp-contract=off and
// without fast-math so that the transforms stay error-free.
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define MP_HD __host__ __device__ __forceinline__
#else
#define MP_HD inline
#endif

namespace zk {

// --------------------------------------------------------------- EFTs ----
MP_HD void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

MP_HD void fast_two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    e = b - (s - a);
}

MP_HD void two_prod(double a, double b, double &p, double &e)
{
    p = a * b;
    e = fma(a, b, -p);
}

// Three-level cascaded accumulator of products (binary64) x (double-double).
// The leading product is split exactly (two_prod); its TwoSum error against
// the running sum S goes to a second level C with TwoSum, and so do the
// product error and the low product (rounded once, u^2 relative to the
// term); the second level's TwoSum errors go to a third level D.  The error
// of S + C + D is then a sum of per-term roundings of size u^2 |term| (about
// sqrt(n) u^2 t for n terms of size t) instead of u^2 times the running
// partial sums, which is what limits a plain double-double accumulation.
struct Casc3 {
    double S = 0.0, C = 0.0, D = 0.0;
    MP_HD void add(double x, double yh, double yl)
    {
        const double p1 = x * yh;
        const double e1 = fma(x, yh, -p1);
        const double p2 = x * yl;
        double s, c1, c, c2;
        two_sum(S, p1, s, c1);
        S = s;
        two_sum(C, c1, c, c2);
        C = c;
        D += c2;
        two_sum(C, e1 + p2, c, c2);
        C = c;
        D += c2;
    }
    // the sum as a normalised double-double
    MP_HD void get(double &hi, double &lo) const
    {
        double h, l;
        two_sum(S, C, h, l);
        l += D;
        fast_two_sum(h, l, hi, lo);
    }
};

// ------------------------------------------------------------ types ------
template <int L>
struct mp {
    double x[L];
};

template <int L>
struct cmp {
    mp<L> re, im;
};

using dd = mp<2>;
using qd = mp<4>;

template <int L>
MP_HD mp<L> mp_from(double a)
{
    mp<L> r;
    r.x[0] = a;
    for (int i = 1; i < L; i++) r.x[i] = 0.0;
    return r;
}

template <int L>
MP_HD mp<L> mp_zero() { return mp_from<L>(0.0); }

template <int L>
MP_HD mp<L> mp_neg(const mp<L> &a)
{
    mp<L> r;
    for (int i = 0; i < L; i++) r.x[i] = -a.x[i];
    return r;
}

// ====================================================== double-double ====
MP_HD dd dd_add(const dd &a, const dd &b)
{
    double sh, sl, th, tl;
    two_sum(a.x[0], b.x[0], sh, sl);
    two_sum(a.x[1], b.x[1], th, tl);
    const double c = sl + th;
    double vh, vl;
    fast_two_sum(sh, c, vh, vl);
    const double w = tl + vl;
    dd r;
    fast_two_sum(vh, w, r.x[0], r.x[1]);
    return r;
}

MP_HD dd dd_add_d(const dd &a, double b)
{
    double sh, sl;
    two_sum(a.x[0], b, sh, sl);
    const double v = a.x[1] + sl;
    dd r;
    fast_two_sum(sh, v, r.x[0], r.x[1]);
    return r;
}

MP_HD dd dd_mul(const dd &a, const dd &b)
{
    double ch, cl1;
    two_prod(a.x[0], b.x[0], ch, cl1);
    const double tl0 = a.x[1] * b.x[1];
    const double tl1 = fma(a.x[0], b.x[1], tl0);
    const double cl2 = fma(a.x[1], b.x[0], tl1);
    const double cl3 = cl1 + cl2;
    dd r;
    fast_two_sum(ch, cl3, r.x[0], r.x[1]);
    return r;
}

MP_HD dd dd_mul_d(const dd &a, double b)
{
    double ch, cl1;
    two_prod(a.x[0], b, ch, cl1);
    const double cl3 = fma(a.x[1], b, cl1);
    dd r;
    fast_two_sum(ch, cl3, r.x[0], r.x[1]);
    return r;
}

// Long division with three quotient digits.
MP_HD dd dd_div(const dd &a, const dd &b)
{
    const double q1 = a.x[0] / b.x[0];
    dd r = dd_add(a, mp_neg<2>(dd_mul_d(b, q1)));
    const double q2 = r.x[0] / b.x[0];
    r = dd_add(r, mp_neg<2>(dd_mul_d(b, q2)));
    const double q3 = r.x[0] / b.x[0];
    dd q;
    fast_two_sum(q1, q2, q.x[0], q.x[1]);
    return dd_add_d(q, q3);
}

// sqrt by one Newton correction of the binary64 root (a >= 0).
MP_HD dd dd_sqrt(const dd &a)
{
    if (a.x[0] <= 0.0) return mp_zero<2>();
    const double s = sqrt(a.x[0]);
    double p, e;
    two_prod(s, s, p, e);
    dd sq;
    sq.x[0] = p;
    sq.x[1] = e;
    const dd r = dd_add(a, mp_neg<2>(sq));
    const double c = r.x[0] / (2.0 * s);
    dd out;
    fast_two_sum(s, c, out.x[0], out.x[1]);
    return out;
}

// ======================================================== quad-double ====
// Renormalise M >= 4 terms into four limbs: sort by decreasing magnitude
// (odd-even transposition network, static indices so the terms stay in
// registers), two error-free VecSum passes from the bottom, then extraction
// of the leading non-overlapping limbs (branch on a zero error term).
template <int M>
MP_HD void sort_desc_mag(double t[M])
{
    for (int pass = 0; pass < M; pass++) {
        for (int i = pass & 1; i + 1 < M; i += 2) {
            const double a = t[i], b = t[i + 1];
            const bool sw = fabs(b) > fabs(a);
            t[i] = sw ? b : a;
            t[i + 1] = sw ? a : b;
        }
    }
}

template <int M>
MP_HD qd qd_renorm(double t[M])
{
    sort_desc_mag<M>(t);
    for (int pass = 0; pass < 2; pass++) {
        double s = t[M - 1];
        for (int i = M - 2; i >= 0; i--) {
            double e;
            two_sum(t[i], s, s, e);
            t[i + 1] = e;
        }
        t[0] = s;
    }
    qd r;
    r.x[0] = r.x[1] = r.x[2] = r.x[3] = 0.0;
    int j = 0;
    double eps = t[0];
    for (int i = 1; i < M; i++) {
        double s, e;
        fast_two_sum(eps, t[i], s, e);
        if (e != 0.0) {
            if (j < 4) r.x[j] = s;
            j++;
            eps = e;
        } else {
            eps = s;
        }
    }
    if (j < 4) r.x[j] = eps;
    // final pass: make the four limbs non-overlapping
    double s0, e0, s1, e1, s2, e2;
    fast_two_sum(r.x[2], r.x[3], s2, e2);
    fast_two_sum(r.x[1], s2, s1, e1);
    fast_two_sum(r.x[0], s1, s0, e0);
    r.x[0] = s0;
    fast_two_sum(e0, e1, s1, e1);
    r.x[1] = s1;
    fast_two_sum(e1, e2, s2, e2);
    r.x[2] = s2;
    r.x[3] = e2;
    return r;
}

// Cascaded accumulator of quad-double products.  The partial products of
// x*y are grouped by order (x_i y_j has size ~u^(i+j) |x y|): orders 0..3
// are split exactly (two_prod), order 4 is summed plainly and orders >= 5
// are dropped (below the quad-double rounding).  Level k collects the
// order-k terms, the product errors of order k-1 and the TwoSum errors of
// level k-1; levels 0..3 are accumulated with TwoSum, level 4 plainly.  About
// 230 binary64 operations per product, against a full quad-double multiply
// and add (each renormalising an expansion of 16 or 8 terms by sorting) that
// cost several times more; the error is below u^4 of the terms.
struct Casc4 {
    double S0 = 0.0, S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0;
    MP_HD void init(const qd &x)
    {
        S0 = x.x[0];
        S1 = x.x[1];
        S2 = x.x[2];
        S3 = x.x[3];
        S4 = 0.0;
    }
    MP_HD void put3(double v)
    {
        double s, e;
        two_sum(S3, v, s, e);
        S3 = s;
        S4 += e;
    }
    MP_HD void put2(double v)
    {
        double s, e;
        two_sum(S2, v, s, e);
        S2 = s;
        put3(e);
    }
    MP_HD void put1(double v)
    {
        double s, e;
        two_sum(S1, v, s, e);
        S1 = s;
        put2(e);
    }
    // += sg * x * y  (sg = +1 or -1, applied exactly)
    MP_HD void add(const qd &x, const qd &y, double sg)
    {
        const double x0 = sg * x.x[0], x1 = sg * x.x[1], x2 = sg * x.x[2], x3 = sg * x.x[3];
        const double y0 = y.x[0], y1 = y.x[1], y2 = y.x[2], y3 = y.x[3];
        double p00, e00, p01, e01, p10, e10, p02, e02, p11, e11, p20, e20;
        double p03, e03, p12, e12, p21, e21, p30, e30;
        two_prod(x0, y0, p00, e00);
        two_prod(x0, y1, p01, e01);
        two_prod(x1, y0, p10, e10);
        two_prod(x0, y2, p02, e02);
        two_prod(x1, y1, p11, e11);
        two_prod(x2, y0, p20, e20);
        two_prod(x0, y3, p03, e03);
        two_prod(x1, y2, p12, e12);
        two_prod(x2, y1, p21, e21);
        two_prod(x3, y0, p30, e30);
        double s, e;
        two_sum(S0, p00, s, e);
        S0 = s;
        put1(e);
        put1(e00);
        put1(p01);
        put1(p10);
        put2(e01);
        put2(e10);
        put2(p02);
        put2(p11);
        put2(p20);
        put3(e02);
        put3(e11);
        put3(e20);
        put3(p03);
        put3(p12);
        put3(p21);
        put3(p30);
        S4 += ((e03 + e12) + (e21 + e30)) + ((x1 * y3 + x3 * y1) + x2 * y2);
    }
    MP_HD qd get() const
    {
        double t[5] = {S0, S1, S2, S3, S4};
        return qd_renorm<5>(t);
    }
};

MP_HD qd qd_add(const qd &a, const qd &b)
{
    double t[8] = {a.x[0], b.x[0], a.x[1], b.x[1], a.x[2], b.x[2], a.x[3], b.x[3]};
    return qd_renorm<8>(t);
}

MP_HD qd qd_add_d(const qd &a, double b)
{
    double t[5] = {a.x[0], b, a.x[1], a.x[2], a.x[3]};
    return qd_renorm<5>(t);
}

MP_HD qd qd_mul(const qd &a, const qd &b)
{
    double t[16];
    // order 0
    two_prod(a.x[0], b.x[0], t[0], t[1]);
    // order 1
    two_prod(a.x[0], b.x[1], t[2], t[4]);
    two_prod(a.x[1], b.x[0], t[3], t[5]);
    // order 2
    two_prod(a.x[0], b.x[2], t[6], t[9]);
    two_prod(a.x[1], b.x[1], t[7], t[10]);
    two_prod(a.x[2], b.x[0], t[8], t[11]);
    // order 3 (plain products; their errors are below the last limb)
    t[12] = a.x[0] * b.x[3];
    t[13] = a.x[1] * b.x[2];
    t[14] = a.x[2] * b.x[1];
    t[15] = a.x[3] * b.x[0];
    return qd_renorm<16>(t);
}

MP_HD qd qd_mul_d(const qd &a, double b)
{
    double t[8];
    two_prod(a.x[0], b, t[0], t[1]);
    two_prod(a.x[1], b, t[2], t[3]);
    two_prod(a.x[2], b, t[4], t[5]);
    t[6] = a.x[3] * b;
    t[7] = 0.0;
    return qd_renorm<8>(t);
}

// Long division with five quotient digits.
MP_HD qd qd_div(const qd &a, const qd &b)
{
    double q[5];
    qd r = a;
    for (int i = 0; i < 5; i++) {
        q[i] = r.x[0] / b.x[0];
        r = qd_add(r, mp_neg<4>(qd_mul_d(b, q[i])));
    }
    return qd_renorm<5>(q);
}

// sqrt by Newton corrections x <- x + (a - x^2) / (2x) (a >= 0).
MP_HD qd qd_sqrt(const qd &a)
{
    if (a.x[0] <= 0.0) return mp_zero<4>();
    qd x = mp_from<4>(sqrt(a.x[0]));
    for (int it = 0; it < 3; it++) {
        const qd r = qd_add(a, mp_neg<4>(qd_mul(x, x)));
        const qd c = qd_div(r, qd_add(x, x));
        x = qd_add(x, c);
    }
    return x;
}

// ====================================================== L limbs, generic ====
// Precision beyond quad-double: values of L binary64 limbs (L = 8: about 424
// bits, L = 16: about 848 bits), built from the same error-free transforms.
// Only what the precision polishing needs is provided: exact products of a
// binary64 by an L-limb value, their cascaded accumulation, and the
// renormalisation of a set of terms into L limbs.

// Renormalise M terms into L limbs: the quad-double procedure above (sort by
// magnitude, two VecSum passes, extraction of the leading non-overlapping
// terms) for any L, then a bottom-up and a top-down Fast2Sum pass over the
// limbs.
template <int L, int M>
MP_HD mp<L> renorm_n(double t[M])
{
    sort_desc_mag<M>(t);
#pragma unroll
    for (int pass = 0; pass < 2; pass++) {
        double s = t[M - 1];
#pragma unroll
        for (int i = M - 2; i >= 0; i--) {
            double e;
            two_sum(t[i], s, s, e);
            t[i + 1] = e;
        }
        t[0] = s;
    }
    mp<L> r;
#pragma unroll
    for (int k = 0; k < L; k++) r.x[k] = 0.0;
    int j = 0;
    double eps = t[0];
#pragma unroll
    for (int i = 1; i < M; i++) {
        double s, e;
        fast_two_sum(eps, t[i], s, e);
        if (e != 0.0) {
#pragma unroll
            for (int k = 0; k < L; k++)
                if (k == j) r.x[k] = s;
            j++;
            eps = e;
        } else {
            eps = s;
        }
    }
#pragma unroll
    for (int k = 0; k < L; k++)
        if (k == j) r.x[k] = eps;
    double s = r.x[L - 1];
#pragma unroll
    for (int k = L - 2; k >= 0; k--) {
        double e;
        fast_two_sum(r.x[k], s, s, e);
        r.x[k + 1] = e;
    }
    r.x[0] = s;
#pragma unroll
    for (int k = 0; k + 1 < L; k++) fast_two_sum(r.x[k], r.x[k + 1], r.x[k], r.x[k + 1]);
    return r;
}

// Cascaded accumulator at L-limb precision.  Level k (0 <= k < L) collects
// terms of order k (about u^k times the largest term) with TwoSum; the error
// of a TwoSum at level k goes on to level k + 1, and level L is a plain sum
// (below the L-limb rounding).  An exact product x y_b of a binary64 x of
// order o and limb b of y is p + e with p of order o + b and e of order
// o + b + 1; orders above L are dropped.  The accumulated value is exact to
// about u^L times the sum of the magnitudes of the terms.
template <int L>
struct CascN {
    double S[L + 1];
    MP_HD void zero()
    {
#pragma unroll
        for (int k = 0; k <= L; k++) S[k] = 0.0;
    }
    MP_HD void put(int k, double v)
    {
#pragma unroll
        for (int q = 0; q < L; q++)
            if (q >= k) {
                double s, e;
                two_sum(S[q], v, s, e);
                S[q] = s;
                v = e;
            }
        S[L] += v;
    }
    // += x * y, x binary64 of order `off`, y an L-limb value
    MP_HD void add(double x, const double *y, int off)
    {
#pragma unroll
        for (int b = 0; b < L; b++) {
            const int k = off + b;
            if (k < L) {
                double p, e;
                two_prod(x, y[b], p, e);
                put(k, p);
                if (k + 1 < L) put(k + 1, e);
                else S[L] += e;
            } else if (k == L) {
                S[L] += x * y[b];
            }
        }
    }
    // += x * y, both L-limb values (limb a of x has order a)
    MP_HD void add_mm(const double *x, const double *y)
    {
#pragma unroll
        for (int a = 0; a < L; a++) add(x[a], y, a);
    }
    MP_HD mp<L> get() const
    {
        double t[L + 1];
#pragma unroll
        for (int k = 0; k <= L; k++) t[k] = S[k];
        return renorm_n<L, L + 1>(t);
    }
};

// a + b for L-limb a and binary64 b
template <int L>
MP_HD mp<L> add_n_d(const mp<L> &a, double b)
{
    double t[L + 1];
#pragma unroll
    for (int k = 0; k < L; k++) t[k] = a.x[k];
    t[L] = b;
    return renorm_n<L, L + 1>(t);
}

// ================================================= generic dispatch =====
template <int L> struct ops;

template <>
struct ops<2> {
    static MP_HD dd add(const dd &a, const dd &b) { return dd_add(a, b); }
    static MP_HD dd mul(const dd &a, const dd &b) { return dd_mul(a, b); }
    static MP_HD dd mul_d(const dd &a, double b) { return dd_mul_d(a, b); }
    static MP_HD dd add_d(const dd &a, double b) { return dd_add_d(a, b); }
    static MP_HD dd div(const dd &a, const dd &b) { return dd_div(a, b); }
    static MP_HD dd sqrt_(const dd &a) { return dd_sqrt(a); }
};

template <>
struct ops<4> {
    static MP_HD qd add(const qd &a, const qd &b) { return qd_add(a, b); }
    static MP_HD qd mul(const qd &a, const qd &b) { return qd_mul(a, b); }
    static MP_HD qd mul_d(const qd &a, double b) { return qd_mul_d(a, b); }
    static MP_HD qd add_d(const qd &a, double b) { return qd_add_d(a, b); }
    static MP_HD qd div(const qd &a, const qd &b) { return qd_div(a, b); }
    static MP_HD qd sqrt_(const qd &a) { return qd_sqrt(a); }
};

template <int L> MP_HD mp<L> add(const mp<L> &a, const mp<L> &b) { return ops<L>::add(a, b); }
template <int L> MP_HD mp<L> sub(const mp<L> &a, const mp<L> &b) { return ops<L>::add(a, mp_neg<L>(b)); }
template <int L> MP_HD mp<L> mul(const mp<L> &a, const mp<L> &b) { return ops<L>::mul(a, b); }
template <int L> MP_HD mp<L> mul_d(const mp<L> &a, double b) { return ops<L>::mul_d(a, b); }
template <int L> MP_HD mp<L> add_d(const mp<L> &a, double b) { return ops<L>::add_d(a, b); }
template <int L> MP_HD mp<L> div(const mp<L> &a, const mp<L> &b) { return ops<L>::div(a, b); }
template <int L> MP_HD mp<L> sqrt_mp(const mp<L> &a) { return ops<L>::sqrt_(a); }

// exact scaling by a power of two
template <int L>
MP_HD mp<L> ldexp_mp(const mp<L> &a, int e)
{
    mp<L> r;
    for (int i = 0; i < L; i++) r.x[i] = ldexp(a.x[i], e);
    return r;
}

// ---------------------------------------------------------- complex -----
template <int L>
MP_HD cmp<L> c_zero()
{
    cmp<L> r;
    r.re = mp_zero<L>();
    r.im = mp_zero<L>();
    return r;
}

template <int L> MP_HD cmp<L> c_add(const cmp<L> &a, const cmp<L> &b) { return {add(a.re, b.re), add(a.im, b.im)}; }
template <int L> MP_HD cmp<L> c_sub(const cmp<L> &a, const cmp<L> &b) { return {sub(a.re, b.re), sub(a.im, b.im)}; }
template <int L> MP_HD cmp<L> c_conj(const cmp<L> &a) { return {a.re, mp_neg<L>(a.im)}; }

template <int L>
MP_HD cmp<L> c_mul(const cmp<L> &a, const cmp<L> &b)
{
    return {sub(mul(a.re, b.re), mul(a.im, b.im)), add(mul(a.re, b.im), mul(a.im, b.re))};
}

// conj(a) * b
template <int L>
MP_HD cmp<L> c_mulc(const cmp<L> &a, const cmp<L> &b)
{
    return {add(mul(a.re, b.re), mul(a.im, b.im)), sub(mul(a.re, b.im), mul(a.im, b.re))};
}

template <int L>
MP_HD cmp<L> c_scale(const cmp<L> &a, const mp<L> &s)
{
    return {mul(a.re, s), mul(a.im, s)};
}

template <int L>
MP_HD mp<L> c_abs2(const cmp<L> &a)
{
    return add(mul(a.re, a.re), mul(a.im, a.im));
}

// 1 / b, computed with a power-of-two prescaling so |b|^2 cannot overflow
template <int L>
MP_HD cmp<L> c_recip(const cmp<L> &b)
{
    const double m = fmax(fabs(b.re.x[0]), fabs(b.im.x[0]));
    int e = 0;
    if (m > 0.0) frexp(m, &e);
    const cmp<L> bs = {ldexp_mp(b.re, -e), ldexp_mp(b.im, -e)};
    const mp<L> d = c_abs2(bs);
    const mp<L> one = mp_from<L>(1.0);
    const mp<L> inv = div(one, d);
    cmp<L> r = {mul(bs.re, inv), mp_neg<L>(mul(bs.im, inv))};
    r.re = ldexp_mp(r.re, -e);
    r.im = ldexp_mp(r.im, -e);
    return r;
}

// binary64 magnitude estimate |re_0| + |im_0| (pivot choice)
template <int L>
MP_HD double c_mag1(const cmp<L> &a)
{
    return fabs(a.re.x[0]) + fabs(a.im.x[0]);
}

}  // namespace zk
