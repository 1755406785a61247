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
