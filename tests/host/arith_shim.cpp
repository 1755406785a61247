// Host build of the product's multi-limb arithmetic header, exported with C
// linkage so the tests can compare every operation with exact rationals.
#include "../../paper_2402_11868_amd/csrc/mp.h"

using namespace zk;

extern "C" {
void t_two_sum(double a, double b, double *s, double *e) { two_sum(a, b, *s, *e); }
void t_two_prod(double a, double b, double *p, double *e) { two_prod(a, b, *p, *e); }

#define BIN(name, L, fn)                                                       \
    void name(const double *a, const double *b, double *r)                    \
    {                                                                          \
        mp<L> x, y;                                                            \
        for (int i = 0; i < L; i++) { x.x[i] = a[i]; y.x[i] = b[i]; }          \
        mp<L> z = fn(x, y);                                                    \
        for (int i = 0; i < L; i++) r[i] = z.x[i];                             \
    }
BIN(t_dd_add, 2, dd_add)
BIN(t_dd_mul, 2, dd_mul)
BIN(t_dd_div, 2, dd_div)
BIN(t_qd_add, 4, qd_add)
BIN(t_qd_mul, 4, qd_mul)
BIN(t_qd_div, 4, qd_div)

void t_dd_sqrt(const double *a, double *r) { dd x = {{a[0], a[1]}}; dd z = dd_sqrt(x); r[0] = z.x[0]; r[1] = z.x[1]; }
void t_qd_sqrt(const double *a, double *r)
{
    qd x;
    for (int i = 0; i < 4; i++) x.x[i] = a[i];
    qd z = qd_sqrt(x);
    for (int i = 0; i < 4; i++) r[i] = z.x[i];
}
void t_casc3(int n, const double *x, const double *yh, const double *yl, double *r)
{
    Casc3 a;
    for (int i = 0; i < n; i++) a.add(x[i], yh[i], yl[i]);
    a.get(r[0], r[1]);
}
void t_casc4(int n, const double *x, const double *y, const double *sg, double *r)
{
    Casc4 a;
    for (int i = 0; i < n; i++) {
        qd xx, yy;
        for (int l = 0; l < 4; l++) { xx.x[l] = x[4 * i + l]; yy.x[l] = y[4 * i + l]; }
        a.add(xx, yy, sg[i]);
    }
    qd z = a.get();
    for (int l = 0; l < 4; l++) r[l] = z.x[l];
}
void t_qd_renorm16(const double *t, double *r)
{
    double w[16];
    for (int i = 0; i < 16; i++) w[i] = t[i];
    qd z = qd_renorm<16>(w);
    for (int i = 0; i < 4; i++) r[i] = z.x[i];
}

// L-limb cascades: sum_i x_i y_i with both factors L-limb (mm = 1) or x_i binary64 (mm = 0)
#define CASCN(name, L)                                                         \
    void name(int n, int mm, const double *x, const double *y, double *r)     \
    {                                                                          \
        CascN<L> a;                                                            \
        a.zero();                                                              \
        for (int i = 0; i < n; i++) {                                          \
            if (mm) a.add_mm(x + L * i, y + L * i);                           \
            else a.add(x[i], y + L * i, 0);                                    \
        }                                                                      \
        mp<L> z = a.get();                                                     \
        for (int l = 0; l < L; l++) r[l] = z.x[l];                             \
    }
CASCN(t_casc_n8, 8)
CASCN(t_casc_n16, 16)
void t_renorm_n8_24(const double *t, double *r)
{
    double w[24];
    for (int i = 0; i < 24; i++) w[i] = t[i];
    mp<8> z = renorm_n<8, 24>(w);
    for (int i = 0; i < 8; i++) r[i] = z.x[i];
}
void t_add_n16_d(const double *a, double b, double *r)
{
    mp<16> x;
    for (int i = 0; i < 16; i++) x.x[i] = a[i];
    mp<16> z = add_n_d<16>(x, b);
    for (int i = 0; i < 16; i++) r[i] = z.x[i];
}
}
