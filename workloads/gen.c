/*
 * Seeded synthetic input generators (shared by the tests, the bench and the
 * oracle's self-checks).  This file holds NO part of the eigen-solver: it only
 * builds test matrices of a prescribed spectrum.
 *
 * householder_hermitian():
 *   H = U diag(lam) U^H with U = P_1 P_2 ... P_m, P_j = I - 2 u_j u_j^H/(u_j^H u_j).
 *   The matrix is built in plain binary64 by m two-sided rank-2 updates applied
 *   for j = m..1 to diag(lam).  Every entry is computed by a fixed sequence of
 *   operations (no BLAS, no reassociation, -ffp-contract=off at build time), so
 *   the stored matrix is bit-for-bit reproducible on any x86-64 host and with any
 *   thread count.  The stored matrix, not the design, is the ground truth the
 *   solvers are checked against.
 *
 * Storage: column-major complex128 (re, im interleaved), leading dimension n.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* y = H u for the full (Hermitian) matrix H stored column-major. */
static void hermv(int n, const double *H, const double *u, double *y)
{
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
        double re = 0.0, im = 0.0;
        for (int j = 0; j < n; j++) {
            const double hr = H[2 * ((size_t)j * n + i)], hi = H[2 * ((size_t)j * n + i) + 1];
            const double ur = u[2 * j], ui = u[2 * j + 1];
            re += hr * ur - hi * ui;
            im += hr * ui + hi * ur;
        }
        y[2 * i] = re;
        y[2 * i + 1] = im;
    }
}

/*
 * lam: n real eigenvalues.  uvec: m x n x 2 doubles (reflector j, component i,
 * re/im).  out: n*n complex128, column-major.  Returns 0 on success.
 */
int gen_householder_hermitian(int n, int m, const double *lam, const double *uvec, double *out)
{
    if (n < 1 || m < 0) return -1;
    double *y = (double *)malloc(sizeof(double) * 2 * n);
    double *w = (double *)malloc(sizeof(double) * 2 * n);
    if (!y || !w) { free(y); free(w); return -2; }
    memset(out, 0, sizeof(double) * 2 * (size_t)n * n);
    for (int i = 0; i < n; i++) out[2 * ((size_t)i * n + i)] = lam[i];

    for (int j = m - 1; j >= 0; j--) {
        const double *u = uvec + (size_t)j * 2 * n;
        double uu = 0.0;
        for (int i = 0; i < n; i++) uu += u[2 * i] * u[2 * i] + u[2 * i + 1] * u[2 * i + 1];
        if (uu == 0.0) continue;
        const double beta = 2.0 / uu;
        hermv(n, out, u, y);
        double gam = 0.0; /* Re(u^H y); the imaginary part is zero in exact arithmetic */
        for (int i = 0; i < n; i++) gam += u[2 * i] * y[2 * i] + u[2 * i + 1] * y[2 * i + 1];
        const double c = 0.5 * beta * beta * gam;
        for (int i = 0; i < n; i++) {
            w[2 * i] = beta * y[2 * i] - c * u[2 * i];
            w[2 * i + 1] = beta * y[2 * i + 1] - c * u[2 * i + 1];
        }
        /* H <- H - u w^H - w u^H */
        #pragma omp parallel for schedule(static)
        for (int col = 0; col < n; col++) {
            const double wr = w[2 * col], wi = -w[2 * col + 1];   /* conj(w_col) */
            const double ur = u[2 * col], ui = -u[2 * col + 1];   /* conj(u_col) */
            double *hc = out + 2 * (size_t)col * n;
            for (int i = 0; i < n; i++) {
                const double a_r = u[2 * i] * wr - u[2 * i + 1] * wi;
                const double a_i = u[2 * i] * wi + u[2 * i + 1] * wr;
                const double b_r = w[2 * i] * ur - w[2 * i + 1] * ui;
                const double b_i = w[2 * i] * ui + w[2 * i + 1] * ur;
                hc[2 * i] -= a_r + b_r;
                hc[2 * i + 1] -= a_i + b_i;
            }
        }
    }
    /* Make the stored matrix exactly Hermitian: mirror the lower triangle, real diagonal. */
    for (int col = 0; col < n; col++) {
        out[2 * ((size_t)col * n + col) + 1] = 0.0;
        for (int i = col + 1; i < n; i++) {
            out[2 * ((size_t)i * n + col)] = out[2 * ((size_t)col * n + i)];
            out[2 * ((size_t)i * n + col) + 1] = -out[2 * ((size_t)col * n + i) + 1];
        }
    }
    free(y);
    free(w);
    return 0;
}
