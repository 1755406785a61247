/*
 * ORACLE -- test infrastructure only.  Nothing on the product path may link,
 * load or call this file; only the tests, the smoke check and the bench's CPU
 * baseline leg do.
 *
 * What it computes: the exact eigendecomposition H = V diag(lam) V^H of a
 * complex Hermitian matrix given as an exact sum of binary64 limb planes, to
 * `prec` bits (256 by default).  The paper's method (an FP64 eigendecomposition
 * followed by Rayleigh quotient iteration, Sec. 2 "ZKCM_CUS") converges to this
 * decomposition to working precision, so the oracle evaluates the plain
 * definition with a different, textbook algorithm: cyclic two-sided Jacobi.
 *
 * Algorithm (complex Hermitian Jacobi, round-robin ordering):
 *   1. A <- sum of the limb planes at `prec` bits (exact: limbs span < prec
 *      bits).  Only the lower triangle is read; the upper triangle is its
 *      conjugate and the imaginary part of the diagonal is ignored.  V <- I.
 *   2. One sweep visits every pair p < q once, in n-1 rounds of n/2 disjoint
 *      pairs (circle method); the rotations of a round commute and are applied
 *      together.  For b = A(p,q) = |b| e^{i phi}:
 *        D = diag(1, e^{-i phi}) makes the 2x2 block real symmetric
 *        [[a, |b|], [|b|, d]]; the symmetric Schur rotation J = [[c, s], [-s, c]]
 *        with zeta = (d - a)/(2|b|), t = sign(zeta)/(|zeta| + sqrt(1 + zeta^2))
 *        (t = 1 for zeta = 0), c = 1/sqrt(1+t^2), s = t c diagonalises it
 *        (Golub & Van Loan, Matrix Computations, Sec. 8.5, "sym.schur2").
 *        A <- G^H A G and V <- V G with G = D J embedded at (p, q); then
 *        A(p,q) = A(q,p) = 0, A(p,p) = a - t|b|, A(q,q) = d + t|b| exactly.
 *   3. Stop when off(A) = sqrt(sum_{i != j} |A_ij|^2) <= 2^(16-prec) ||A||_F
 *      after a sweep (at most 40 sweeps, else error -3).
 *   4. lam = diag(A) sorted ascending, columns of V permuted to match.
 *
 * Checkers (same precision): residual norms ||H v - lam v|| / ||v|| and the
 * Gram matrix of returned vectors, each evaluated on the exact limb sums.
 *
 * Limb conventions: a "plane set" with L limbs is L consecutive arrays; the
 * represented value is the exact sum of the limbs.  Matrices are column-major
 * complex128 (re, im interleaved) with leading dimension lda.
 */
#include <math.h>
#include <mpfr.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define RN MPFR_RNDN

/* Mutation switch for the pin tests: a nonzero value plants one deliberate
 * mistake so the tests can show that the pins catch it.  Always 0 otherwise. */
static int g_mutation = 0;
void or_set_mutation(int m) { g_mutation = m; }

typedef struct { mpfr_t re, im; } cmp_t;

static void c_init(cmp_t *z, int prec) { mpfr_init2(z->re, prec); mpfr_init2(z->im, prec); mpfr_set_zero(z->re, 1); mpfr_set_zero(z->im, 1); }
static void c_clear(cmp_t *z) { mpfr_clear(z->re); mpfr_clear(z->im); }

static cmp_t *c_alloc(size_t count, int prec)
{
    cmp_t *a = (cmp_t *)malloc(sizeof(cmp_t) * count);
    if (!a) return NULL;
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < (long)count; i++) c_init(&a[i], prec);
    return a;
}

static void c_free(cmp_t *a, size_t count)
{
    if (!a) return;
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < (long)count; i++) c_clear(&a[i]);
    free(a);
}

/* x = exact sum of limbs of a complex128 plane set at element offset `off`. */
static void c_from_limbs(cmp_t *x, int L, const double *planes, size_t plane_stride, size_t off)
{
    mpfr_set_zero(x->re, 1);
    mpfr_set_zero(x->im, 1);
    int Luse = (g_mutation == 6 && L > 1) ? 1 : L;   /* mutation 6: ignore all but the first limb */
    for (int l = 0; l < Luse; l++) {
        const double *p = planes + 2 * (l * plane_stride + off);
        mpfr_add_d(x->re, x->re, p[0], RN);
        mpfr_add_d(x->im, x->im, p[1], RN);
    }
}

static void r_from_limbs(mpfr_t x, int L, const double *v, size_t plane_stride, size_t off)
{
    mpfr_set_zero(x, 1);
    for (int l = 0; l < L; l++) mpfr_add_d(x, x, v[l * plane_stride + off], RN);
}

/* Split an MPFR value into `L` binary64 limbs, each the round-to-nearest of the remainder. */
static void split_limbs(mpfr_t x, int L, double *out, size_t stride, mpfr_t tmp)
{
    mpfr_set(tmp, x, RN);
    for (int l = 0; l < L; l++) {
        double d = mpfr_get_d(tmp, RN);
        out[l * stride] = d;
        mpfr_sub_d(tmp, tmp, d, RN);
    }
}

/* Full Hermitian matrix from the lower triangle of the limb planes (row-major A[i*n+j]). */
static void load_hermitian(cmp_t *A, int n, int L, const double *planes, int lda)
{
    const size_t ps = (size_t)lda * n;
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
        for (int j = 0; j <= i; j++) {
            size_t off = (g_mutation == 3) ? (size_t)i * lda + j   /* mutation 3: read the upper triangle */
                                           : (size_t)j * lda + i;
            c_from_limbs(&A[(size_t)i * n + j], L, planes, ps, off);
        }
        mpfr_set_zero(A[(size_t)i * n + i].im, 1);
    }
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++) {
            mpfr_set(A[(size_t)i * n + j].re, A[(size_t)j * n + i].re, RN);
            if (g_mutation == 1) mpfr_set(A[(size_t)i * n + j].im, A[(size_t)j * n + i].im, RN); /* mutation 1: no conjugate */
            else mpfr_neg(A[(size_t)i * n + j].im, A[(size_t)j * n + i].im, RN);
        }
}

typedef struct {
    int p, q, active;
    mpfr_t c, s;        /* real rotation */
    mpfr_t er, ei;      /* e^{-i phi} */
    mpfr_t tb;          /* t |b| */
    mpfr_t a, d;        /* A(p,p), A(q,q) before the round */
} rot_t;

/* Compute the rotation for pair (p,q) from the current A; marks inactive if b is negligible. */
static void make_rot(rot_t *r, cmp_t *A, int n, int prec, mpfr_t *tmp /* 6 temps */)
{
    const int p = r->p, q = r->q;
    cmp_t *b = &A[(size_t)p * n + q];
    mpfr_ptr a = A[(size_t)p * n + p].re, d = A[(size_t)q * n + q].re;
    mpfr_ptr absb = tmp[0], zeta = tmp[1], t = tmp[2], u = tmp[3], w = tmp[4];
    mpfr_hypot(absb, b->re, b->im, RN);
    r->active = 0;
    if (mpfr_zero_p(absb)) return;
    /* negligible: |b| <= 2^-(prec+20) (|a| + |d|) */
    mpfr_abs(u, a, RN);
    mpfr_abs(w, d, RN);
    mpfr_add(u, u, w, RN);
    mpfr_mul_2si(u, u, -(prec + 20), RN);
    if (mpfr_cmp(absb, u) <= 0) return;
    r->active = 1;
    mpfr_set(r->a, a, RN);
    mpfr_set(r->d, d, RN);
    /* e^{-i phi} = conj(b)/|b| */
    mpfr_div(r->er, b->re, absb, RN);
    mpfr_div(r->ei, b->im, absb, RN);
    mpfr_neg(r->ei, r->ei, RN);
    if (g_mutation == 4) { mpfr_set_ui(r->er, 1, RN); mpfr_set_zero(r->ei, 1); }   /* mutation 4: drop the phase */
    /* zeta = (d - a) / (2|b|) */
    mpfr_sub(zeta, d, a, RN);
    mpfr_div(zeta, zeta, absb, RN);
    mpfr_div_2ui(zeta, zeta, 1, RN);
    if (mpfr_zero_p(zeta)) {
        mpfr_set_ui(t, 1, RN);
    } else {
        mpfr_sqr(u, zeta, RN);
        mpfr_add_ui(u, u, 1, RN);
        mpfr_sqrt(u, u, RN);
        mpfr_abs(w, zeta, RN);
        mpfr_add(u, u, w, RN);
        mpfr_ui_div(t, 1, u, RN);
        if (mpfr_sgn(zeta) < 0) mpfr_neg(t, t, RN);
    }
    if (g_mutation == 2) mpfr_neg(t, t, RN);   /* mutation 2: wrong sign of the rotation */
    mpfr_sqr(u, t, RN);
    mpfr_add_ui(u, u, 1, RN);
    mpfr_rec_sqrt(r->c, u, RN);
    mpfr_mul(r->s, t, r->c, RN);
    mpfr_mul(r->tb, t, absb, RN);
}

/* Column op on one row: [x, y] <- [c x - s e y, s x + c e y] with e = e^{-i phi}. */
static void col_op(cmp_t *x, cmp_t *y, const rot_t *r, mpfr_t *tmp)
{
    mpfr_ptr yr = tmp[0], yi = tmp[1], nr = tmp[2], ni = tmp[3];
    /* y' = e * y */
    mpfr_fmms(yr, r->er, y->re, r->ei, y->im, RN);
    mpfr_fmma(yi, r->er, y->im, r->ei, y->re, RN);
    /* x'' = c x - s y' ; y'' = s x + c y' */
    mpfr_fmms(nr, r->c, x->re, r->s, yr, RN);
    mpfr_fmms(ni, r->c, x->im, r->s, yi, RN);
    mpfr_fmma(y->re, r->s, x->re, r->c, yr, RN);
    mpfr_fmma(y->im, r->s, x->im, r->c, yi, RN);
    mpfr_set(x->re, nr, RN);
    mpfr_set(x->im, ni, RN);
}

/* Row op on one column: [x; y] <- [c x - s conj(e) y ; s x + c conj(e) y]. */
static void row_op(cmp_t *x, cmp_t *y, const rot_t *r, mpfr_t *tmp)
{
    mpfr_ptr yr = tmp[0], yi = tmp[1], nr = tmp[2], ni = tmp[3];
    /* y' = conj(e) * y,  conj(e) = er - i ei */
    mpfr_fmma(yr, r->er, y->re, r->ei, y->im, RN);
    mpfr_fmms(yi, r->er, y->im, r->ei, y->re, RN);
    mpfr_fmms(nr, r->c, x->re, r->s, yr, RN);
    mpfr_fmms(ni, r->c, x->im, r->s, yi, RN);
    mpfr_fmma(y->re, r->s, x->re, r->c, yr, RN);
    mpfr_fmma(y->im, r->s, x->im, r->c, yi, RN);
    mpfr_set(x->re, nr, RN);
    mpfr_set(x->im, ni, RN);
}

/* off(A)^2 and ||A||_F^2 */
static void frob_parts(cmp_t *A, int n, int prec, mpfr_t off2, mpfr_t all2)
{
    mpfr_set_zero(off2, 1);
    mpfr_set_zero(all2, 1);
    #pragma omp parallel
    {
        mpfr_t lo, la, t;
        mpfr_inits2(prec + 32, lo, la, t, (mpfr_ptr)0);
        mpfr_set_zero(lo, 1);
        mpfr_set_zero(la, 1);
        #pragma omp for schedule(static)
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) {
                cmp_t *z = &A[(size_t)i * n + j];
                mpfr_fmma(t, z->re, z->re, z->im, z->im, RN);
                mpfr_add(la, la, t, RN);
                if (i != j) mpfr_add(lo, lo, t, RN);
            }
        #pragma omp critical
        {
            mpfr_add(off2, off2, lo, RN);
            mpfr_add(all2, all2, la, RN);
        }
        mpfr_clears(lo, la, t, (mpfr_ptr)0);
    }
}

typedef struct { int idx; cmp_t *A; int n; } sortkey_t;
static int cmp_diag(const void *x, const void *y)
{
    const sortkey_t *a = (const sortkey_t *)x, *b = (const sortkey_t *)y;
    int c = mpfr_cmp(a->A[(size_t)a->idx * a->n + a->idx].re, b->A[(size_t)b->idx * b->n + b->idx].re);
    if (c) return c;
    return a->idx - b->idx;
}

/*
 * or_heev: eigenvalues (ascending) and optionally eigenvectors of the Hermitian
 * matrix sum_l planes[l] (lower triangle read).
 *   w_out: 4 limbs per eigenvalue, limb l of eigenvalue k at w_out[l*n + k].
 *   v_out: NULL or 4 limb planes, each n*n complex128 column-major (ld n).
 *   info[0] = sweeps, info[1] = rotations applied (double), info[2] = off(A)/||A||_F.
 * Returns 0, -1 (bad args), -2 (alloc), -3 (no convergence in 40 sweeps).
 */
static int heev_impl(int n, int L, const double *planes, int lda, int prec, int want_vectors, int nthreads,
                     int nlimbs, double *w_out, double *v_out, double *info)
{
    if (n < 1 || L < 1 || L > 16 || lda < n || prec < 64 || nlimbs < 1 || nlimbs > 16) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int m = n + (n & 1);   /* pad to even with a dummy index n (never rotated) */
    cmp_t *A = c_alloc((size_t)n * n, prec);
    cmp_t *V = want_vectors ? c_alloc((size_t)n * n, prec) : NULL;
    int *order = (int *)malloc(sizeof(int) * m);
    rot_t *rots = (rot_t *)malloc(sizeof(rot_t) * (m / 2));
    if (!A || (want_vectors && !V) || !order || !rots) return -2;
    load_hermitian(A, n, L, planes, lda);
    if (V)
        for (int i = 0; i < n; i++) mpfr_set_ui(V[(size_t)i * n + i].re, 1, RN);
    for (int k = 0; k < m / 2; k++) {
        mpfr_inits2(prec, rots[k].c, rots[k].s, rots[k].er, rots[k].ei, rots[k].tb, rots[k].a, rots[k].d, (mpfr_ptr)0);
    }
    for (int i = 0; i < m; i++) order[i] = i;

    mpfr_t off2, all2, thr;
    mpfr_inits2(prec + 32, off2, all2, thr, (mpfr_ptr)0);
    int sweeps = 0, converged = 0;
    double nrot = 0;
    frob_parts(A, n, prec, off2, all2);
    for (sweeps = 0; sweeps < 40; ) {
        /* stop test: off^2 <= 2^(32-2prec) ||A||_F^2 */
        mpfr_mul_2si(thr, all2, 32 - 2 * prec, RN);
        if (mpfr_cmp(off2, thr) <= 0) { converged = 1; break; }
        int any = 0;
        for (int round = 0; round < m - 1; round++) {
            int np = 0;
            for (int k = 0; k < m / 2; k++) {
                int p = order[k], q = order[m - 1 - k];
                if (p > q) { int t = p; p = q; q = t; }
                if (q >= n) continue;   /* dummy partner */
                rots[np].p = p; rots[np].q = q; np++;
            }
            #pragma omp parallel
            {
                mpfr_t tmp[6];
                for (int z = 0; z < 6; z++) mpfr_init2(tmp[z], prec);
                #pragma omp for schedule(static)
                for (int k = 0; k < np; k++) make_rot(&rots[k], A, n, prec, tmp);
                /* column ops (A G), one row per iteration */
                #pragma omp for schedule(static)
                for (int i = 0; i < n; i++)
                    for (int k = 0; k < np; k++) {
                        if (!rots[k].active) continue;
                        col_op(&A[(size_t)i * n + rots[k].p], &A[(size_t)i * n + rots[k].q], &rots[k], tmp);
                    }
                /* row ops (G^H B), one column per iteration */
                #pragma omp for schedule(static)
                for (int j = 0; j < n; j++)
                    for (int k = 0; k < np; k++) {
                        if (!rots[k].active) continue;
                        row_op(&A[(size_t)rots[k].p * n + j], &A[(size_t)rots[k].q * n + j], &rots[k], tmp);
                    }
                if (V) {
                    #pragma omp for schedule(static)
                    for (int i = 0; i < n; i++)
                        for (int k = 0; k < np; k++) {
                            if (!rots[k].active) continue;
                            if (g_mutation == 5) continue;   /* mutation 5: vectors never rotated */
                            col_op(&V[(size_t)i * n + rots[k].p], &V[(size_t)i * n + rots[k].q], &rots[k], tmp);
                        }
                }
                for (int z = 0; z < 6; z++) mpfr_clear(tmp[z]);
            }
            /* exact 2x2 block values */
            for (int k = 0; k < np; k++) {
                if (!rots[k].active) continue;
                any = 1;
                nrot += 1;
                const int p = rots[k].p, q = rots[k].q;
                /* 2x2 block from the closed form: a - t|b|, d + t|b|, zero off-diagonal */
                mpfr_sub(A[(size_t)p * n + p].re, rots[k].a, rots[k].tb, RN);
                mpfr_add(A[(size_t)q * n + q].re, rots[k].d, rots[k].tb, RN);
                mpfr_set_zero(A[(size_t)p * n + q].re, 1);
                mpfr_set_zero(A[(size_t)p * n + q].im, 1);
                mpfr_set_zero(A[(size_t)q * n + p].re, 1);
                mpfr_set_zero(A[(size_t)q * n + p].im, 1);
                mpfr_set_zero(A[(size_t)p * n + p].im, 1);
                mpfr_set_zero(A[(size_t)q * n + q].im, 1);
            }
            /* rotate the circle: keep order[0], shift order[1..m-1] by one */
            int last = order[m - 1];
            for (int k = m - 1; k > 1; k--) order[k] = order[k - 1];
            order[1] = last;
        }
        sweeps++;
        frob_parts(A, n, prec, off2, all2);
        if (!any) { converged = 1; break; }
    }
    if (!converged) {
        mpfr_mul_2si(thr, all2, 32 - 2 * prec, RN);
        converged = mpfr_cmp(off2, thr) <= 0;
    }

    /* outputs */
    sortkey_t *keys = (sortkey_t *)malloc(sizeof(sortkey_t) * n);
    for (int i = 0; i < n; i++) { keys[i].idx = i; keys[i].A = A; keys[i].n = n; }
    qsort(keys, n, sizeof(sortkey_t), cmp_diag);
    mpfr_t tmp;
    mpfr_init2(tmp, prec);
    for (int k = 0; k < n; k++) split_limbs(A[(size_t)keys[k].idx * n + keys[k].idx].re, nlimbs, w_out + k, n, tmp);
    if (V && v_out) {
        const size_t ps = (size_t)n * n;
        #pragma omp parallel
        {
            mpfr_t t2;
            mpfr_init2(t2, prec);
            #pragma omp for schedule(static)
            for (int k = 0; k < n; k++)
                for (int i = 0; i < n; i++) {
                    cmp_t *z = &V[(size_t)i * n + keys[k].idx];
                    size_t off = 2 * ((size_t)k * n + i);
                    split_limbs(z->re, nlimbs, v_out + off, 2 * ps, t2);
                    split_limbs(z->im, nlimbs, v_out + off + 1, 2 * ps, t2);
                }
            mpfr_clear(t2);
        }
    }
    if (info) {
        info[0] = sweeps;
        info[1] = nrot;
        mpfr_sqrt(off2, off2, RN);
        mpfr_sqrt(all2, all2, RN);
        info[2] = mpfr_zero_p(all2) ? 0.0 : mpfr_get_d(off2, RN) / mpfr_get_d(all2, RN);
    }
    mpfr_clear(tmp);
    free(keys);
    mpfr_clears(off2, all2, thr, (mpfr_ptr)0);
    for (int k = 0; k < m / 2; k++) mpfr_clears(rots[k].c, rots[k].s, rots[k].er, rots[k].ei, rots[k].tb, rots[k].a, rots[k].d, (mpfr_ptr)0);
    free(rots);
    free(order);
    c_free(A, (size_t)n * n);
    c_free(V, (size_t)n * n);
    return converged ? 0 : -3;
}

int or_heev(int n, int L, const double *planes, int lda, int prec, int want_vectors, int nthreads,
            double *w_out, double *v_out, double *info)
{
    return heev_impl(n, L, planes, lda, prec, want_vectors, nthreads, 4, w_out, v_out, info);
}

/* or_heev with `nlimbs` (1..16) output limbs per value (w_out: nlimbs x n,
 * v_out: nlimbs planes), for precisions beyond quad-double. */
int or_heev_limbs(int n, int L, const double *planes, int lda, int prec, int want_vectors, int nthreads,
                  int nlimbs, double *w_out, double *v_out, double *info)
{
    return heev_impl(n, L, planes, lda, prec, want_vectors, nthreads, nlimbs, w_out, v_out, info);
}

/*
 * or_residuals: for each of k pairs, res[j] = ||H v_j - lam_j v_j||_2 / ||v_j||_2
 * and vnorm[j] = ||v_j||_2 (as doubles), all in `prec`-bit arithmetic on the exact
 * limb sums.
 *   H: LH planes of n x n (lda), lower triangle read.
 *   V: LV planes, each n x k complex128 column-major with leading dimension ldv
 *      (plane stride ldv*k complex).
 *   w: LW limb arrays of length k (plane stride k).
 */
int or_residuals(int n, int LH, const double *H, int lda, int k, int LV, const double *V, int ldv,
                 int LW, const double *w, int prec, int nthreads, double *res, double *vnorm)
{
    if (n < 1 || k < 0 || lda < n || ldv < n) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    cmp_t *A = c_alloc((size_t)n * n, prec);
    if (!A) return -2;
    load_hermitian(A, n, LH, H, lda);
    const size_t vps = (size_t)ldv * k;
    #pragma omp parallel
    {
        cmp_t *v = (cmp_t *)malloc(sizeof(cmp_t) * n);
        for (int i = 0; i < n; i++) c_init(&v[i], prec);
        cmp_t acc;
        c_init(&acc, prec + 32);
        mpfr_t lam, t, rn, vn;
        mpfr_inits2(prec + 32, lam, t, rn, vn, (mpfr_ptr)0);
        #pragma omp for schedule(dynamic, 1)
        for (int j = 0; j < k; j++) {
            for (int i = 0; i < n; i++) c_from_limbs(&v[i], LV, V, vps, (size_t)j * ldv + i);
            r_from_limbs(lam, LW, w, (size_t)k, (size_t)j);
            mpfr_set_zero(rn, 1);
            mpfr_set_zero(vn, 1);
            for (int i = 0; i < n; i++) {
                /* acc = sum_c A(i,c) v_c - lam v_i */
                mpfr_mul(acc.re, lam, v[i].re, RN);
                mpfr_mul(acc.im, lam, v[i].im, RN);
                mpfr_neg(acc.re, acc.re, RN);
                mpfr_neg(acc.im, acc.im, RN);
                for (int c = 0; c < n; c++) {
                    cmp_t *a = &A[(size_t)i * n + c];
                    mpfr_fmms(t, a->re, v[c].re, a->im, v[c].im, RN);
                    mpfr_add(acc.re, acc.re, t, RN);
                    mpfr_fmma(t, a->re, v[c].im, a->im, v[c].re, RN);
                    mpfr_add(acc.im, acc.im, t, RN);
                }
                mpfr_fmma(t, acc.re, acc.re, acc.im, acc.im, RN);
                mpfr_add(rn, rn, t, RN);
                mpfr_fmma(t, v[i].re, v[i].re, v[i].im, v[i].im, RN);
                mpfr_add(vn, vn, t, RN);
            }
            mpfr_sqrt(rn, rn, RN);
            mpfr_sqrt(vn, vn, RN);
            vnorm[j] = mpfr_get_d(vn, RN);
            if (mpfr_zero_p(vn)) res[j] = INFINITY;
            else { mpfr_div(rn, rn, vn, RN); res[j] = mpfr_get_d(rn, RN); }
        }
        for (int i = 0; i < n; i++) c_clear(&v[i]);
        free(v);
        c_clear(&acc);
        mpfr_clears(lam, t, rn, vn, (mpfr_ptr)0);
    }
    c_free(A, (size_t)n * n);
    return 0;
}

/*
 * or_gram: G = V^H V for the k columns of V (LV planes, n x k, ldv).
 *   max_off = max_{i != j} |G_ij|; max_diag = max_i |G_ii - 1|.
 *   If gabs != NULL it receives |G_ij| as a k x k row-major double array.
 */
int or_gram(int n, int k, int LV, const double *V, int ldv, int prec, int nthreads,
            double *max_off, double *max_diag, double *gabs)
{
    if (n < 1 || k < 0 || ldv < n) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const size_t vps = (size_t)ldv * k;
    cmp_t *X = c_alloc((size_t)n * k, prec);
    if (!X) return -2;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < k; j++)
        for (int i = 0; i < n; i++) c_from_limbs(&X[(size_t)j * n + i], LV, V, vps, (size_t)j * ldv + i);
    double moff = 0.0, mdiag = 0.0;
    #pragma omp parallel
    {
        cmp_t acc;
        c_init(&acc, prec + 32);
        mpfr_t t;
        mpfr_init2(t, prec + 32);
        double lo = 0.0, ld = 0.0;
        #pragma omp for schedule(dynamic, 1)
        for (int a = 0; a < k; a++)
            for (int b = a; b < k; b++) {
                mpfr_set_zero(acc.re, 1);
                mpfr_set_zero(acc.im, 1);
                for (int i = 0; i < n; i++) {
                    cmp_t *x = &X[(size_t)a * n + i], *y = &X[(size_t)b * n + i];
                    /* conj(x) * y */
                    mpfr_fmma(t, x->re, y->re, x->im, y->im, RN);
                    mpfr_add(acc.re, acc.re, t, RN);
                    mpfr_fmms(t, x->re, y->im, x->im, y->re, RN);
                    mpfr_add(acc.im, acc.im, t, RN);
                }
                if (a == b) {
                    mpfr_sub_ui(acc.re, acc.re, 1, RN);
                    double d = fabs(mpfr_get_d(acc.re, RN));
                    if (d > ld) ld = d;
                    if (gabs) gabs[(size_t)a * k + a] = d;
                } else {
                    mpfr_hypot(t, acc.re, acc.im, RN);
                    double d = mpfr_get_d(t, RN);
                    if (d > lo) lo = d;
                    if (gabs) { gabs[(size_t)a * k + b] = d; gabs[(size_t)b * k + a] = d; }
                }
            }
        #pragma omp critical
        {
            if (lo > moff) moff = lo;
            if (ld > mdiag) mdiag = ld;
        }
        c_clear(&acc);
        mpfr_clear(t);
    }
    *max_off = moff;
    *max_diag = mdiag;
    c_free(X, (size_t)n * k);
    return 0;
}
