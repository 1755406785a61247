// Singular value decomposition through the Hermitian dilation: for A (m x n)
// the matrix K = [[0, A], [A^H, 0]] of order m + n has the eigenvalues
// +-sigma_j (j < min(m, n)) and |m - n| zeros, and the eigenvector of
// +sigma_j is [u_j; v_j] / sqrt(2) (A v_j = sigma_j u_j, A^H u_j = sigma_j v_j).
// The paper names the SVD beside the eigendecomposition for its GPU extension,
// with the same precision recovery (Sec. 2); the dilation gives it from the
// Hermitian solver without squaring the condition number (as A^H A would).
#include <hip/hip_runtime.h>

#include "common.h"
#include "stage.h"

namespace zk {

namespace {

// K's limb planes (complex128, column-major, leading dimension N = m + n)
// from A's limb planes: limb l of K(i, m + j) = limb l of A(i, j), of
// K(m + j, i) = its conjugate; the diagonal blocks are zero.
__global__ void __launch_bounds__(256) k_svd_build(SvdDesc D)
{
    const int m = D.m, n = D.n, N = m + n;
    const size_t NN = (size_t)N * N;
    const int c = blockIdx.y;   // column of K
    for (int r = blockIdx.x * 256 + threadIdx.x; r < N; r += gridDim.x * 256) {
        for (int l = 0; l < D.limbs; l++) {
            double2 z = make_double2(0.0, 0.0);
            if (r < m && c >= m) z = ld2(D.A[l] + 2 * ((size_t)(c - m) * D.lda + r));
            else if (r >= m && c < m) {
                const double2 a = ld2(D.A[l] + 2 * ((size_t)(r - m) * D.lda + c));
                z = make_double2(a.x, -a.y);
            }
            st2(D.K + 2 * ((size_t)l * NN + (size_t)c * N + r), z);
        }
    }
}

// singular triplet j from eigenpair N - 1 - j (eigenvalues ascending):
// sigma_j = lambda, u_j = x[0:m] / ||x[0:m]||, v_j = x[m:N] / ||x[m:N]||, in
// double-double.  Normalising each half (instead of multiplying both by
// sqrt 2) removes, to first order, the component of x along the eigenvector
// of -sigma_j, which an eigen-solver leaves at about (residual / 2 sigma_j)
// and which would otherwise scale u_j by (1 + e) and v_j by (1 - e).  One
// block per triplet.
__global__ void __launch_bounds__(256) k_svd_extract(SvdDesc D)
{
    const int m = D.m, n = D.n, N = m + n, j = blockIdx.x;
    const int e = N - 1 - j;
    __shared__ dd red[16];
    if (threadIdx.x == 0) {
        D.s[0][j] = D.w[0][e];
        D.s[1][j] = D.w[1][e];
    }
    if (!D.u[0]) return;
    // squared norms of the two halves, in double-double (exact squares)
    dd nu = mp_zero<2>(), nv = mp_zero<2>();
    for (int r = threadIdx.x; r < N; r += blockDim.x) {
        const size_t o = (size_t)e * N + r;
        const double2 h = ld2(D.V[0] + 2 * o), lo = ld2(D.V[1] + 2 * o);
        const dd re = dd{{h.x, lo.x}}, im = dd{{h.y, lo.y}};
        const dd q = dd_add(dd_mul(re, re), dd_mul(im, im));
        if (r < m) nu = dd_add(nu, q);
        else nv = dd_add(nv, q);
    }
    nu = block_sum_mp<2>(nu, red);
    nv = block_sum_mp<2>(nv, red);
    // 1 / ||half|| (a zero half, possible only for a zero singular value, is left as is)
    const dd one = dd{{1.0, 0.0}};
    const dd su = nu.x[0] > 0.0 ? dd_div(one, dd_sqrt(nu)) : one;
    const dd sv = nv.x[0] > 0.0 ? dd_div(one, dd_sqrt(nv)) : one;
    for (int r = threadIdx.x; r < N; r += blockDim.x) {
        const size_t o = (size_t)e * N + r;
        const double2 h = ld2(D.V[0] + 2 * o), lo = ld2(D.V[1] + 2 * o);
        const dd sc = r < m ? su : sv;
        const dd re = dd_mul(dd{{h.x, lo.x}}, sc), im = dd_mul(dd{{h.y, lo.y}}, sc);
        if (r < m) {
            const size_t q = (size_t)j * D.ldu + r;
            st2(D.u[0] + 2 * q, make_double2(re.x[0], im.x[0]));
            st2(D.u[1] + 2 * q, make_double2(re.x[1], im.x[1]));
        } else {
            const size_t q = (size_t)j * D.ldv + (r - m);
            st2(D.v[0] + 2 * q, make_double2(re.x[0], im.x[0]));
            st2(D.v[1] + 2 * q, make_double2(re.x[1], im.x[1]));
        }
    }
}

// Separate orthonormalisation of the U and V columns.  The eigenvectors of
// +sigma_i and +sigma_j are orthogonal to the eigen-solver's tolerance, but a
// half of one against the same half of the other is only orthogonal to about
// residual / (sigma_i + sigma_j), which for tiny singular values is far above
// it.  First-order Loewdin step on each side: X <- X - X (X^H X - I) / 2,
// which moves each column by about that angle and so changes the residuals
// only by about the residual level (sigma times the angle).
// Gram entries in double-double (they come from cancelling O(1) terms),
// rounded to binary64 (their size is the angle): grid (k, k), block 256.
__global__ void __launch_bounds__(256) k_svd_gram(SvdDesc D, int side, double *G)
{
    const int k = D.m < D.n ? D.m : D.n;
    const int i = blockIdx.x, j = blockIdx.y;
    if (i > j) return;
    if (i == j) {
        if (threadIdx.x == 0) st2(G + 2 * ((size_t)j * k + i), make_double2(0.0, 0.0));
        return;
    }
    const int rows = side ? D.n : D.m;
    const size_t ld = side ? D.ldv : D.ldu;
    const double *X0 = side ? D.v[0] : D.u[0], *X1 = side ? D.v[1] : D.u[1];
    __shared__ dd red[16];
    dd sr = mp_zero<2>(), si = mp_zero<2>();
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        const size_t oi = (size_t)i * ld + r, oj = (size_t)j * ld + r;
        const double2 ah = ld2(X0 + 2 * oi), al = ld2(X1 + 2 * oi);
        const double2 bh = ld2(X0 + 2 * oj), bl = ld2(X1 + 2 * oj);
        const dd ar = dd{{ah.x, al.x}}, ai = dd{{ah.y, al.y}};
        const dd br = dd{{bh.x, bl.x}}, bi = dd{{bh.y, bl.y}};
        // conj(a) b
        sr = dd_add(sr, dd_add(dd_mul(ar, br), dd_mul(ai, bi)));
        si = dd_add(si, dd_add(dd_mul(ar, bi), mp_neg<2>(dd_mul(ai, br))));
    }
    sr = block_sum_mp<2>(sr, red);
    si = block_sum_mp<2>(si, red);
    if (threadIdx.x == 0) {
        st2(G + 2 * ((size_t)j * k + i), make_double2(sr.x[0], si.x[0]));
        st2(G + 2 * ((size_t)i * k + j), make_double2(sr.x[0], -si.x[0]));
    }
}

// C(r, j) = sum_i X(r, i) G(i, j) from the leading limbs (the correction is
// of the size of the angle, so binary64 carries it to far below the
// double-double rounding of X); grid (ceil(rows / 256), k)
__global__ void __launch_bounds__(256) k_svd_corr(SvdDesc D, int side, const double *G, double *C)
{
    const int k = D.m < D.n ? D.m : D.n;
    const int rows = side ? D.n : D.m;
    const int r = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    if (r >= rows) return;
    const size_t ld = side ? D.ldv : D.ldu;
    const double *X0 = side ? D.v[0] : D.u[0];
    double cr = 0.0, ci = 0.0;
    for (int i = 0; i < k; i++) {
        const double2 x = ld2(X0 + 2 * ((size_t)i * ld + r));
        const double2 g = ld2(G + 2 * ((size_t)j * k + i));
        cr = fma(x.x, g.x, fma(-x.y, g.y, cr));
        ci = fma(x.x, g.y, fma(x.y, g.x, ci));
    }
    st2(C + 2 * ((size_t)j * rows + r), make_double2(cr, ci));
}

// X(r, j) -= C(r, j) / 2 in double-double; grid (ceil(rows / 256), k)
__global__ void __launch_bounds__(256) k_svd_apply(SvdDesc D, int side, const double *C)
{
    const int rows = side ? D.n : D.m;
    const int r = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    if (r >= rows) return;
    const size_t ld = side ? D.ldv : D.ldu;
    double *X0 = side ? D.v[0] : D.u[0], *X1 = side ? D.v[1] : D.u[1];
    const size_t o = (size_t)j * ld + r;
    const double2 h = ld2(X0 + 2 * o), lo = ld2(X1 + 2 * o);
    const double2 c = ld2(C + 2 * ((size_t)j * rows + r));
    const dd re = dd_add_d(dd{{h.x, lo.x}}, -0.5 * c.x), im = dd_add_d(dd{{h.y, lo.y}}, -0.5 * c.y);
    st2(X0 + 2 * o, make_double2(re.x[0], im.x[0]));
    st2(X1 + 2 * o, make_double2(re.x[1], im.x[1]));
}

}  // namespace

int svd_build(const SvdDesc &D, hipStream_t st)
{
    const int N = D.m + D.n;
    hipLaunchKernelGGL(k_svd_build, dim3((N + 255) / 256, N), dim3(256), 0, st, D);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int svd_extract(const SvdDesc &D, hipStream_t st)
{
    const int k = D.m < D.n ? D.m : D.n;
    if (k <= 0) return 0;
    hipLaunchKernelGGL(k_svd_extract, dim3(k), dim3(256), 0, st, D);
    if (D.u[0] && k > 1) {
        // the dilation's eigenvectors are consumed: their planes (N x N
        // complex each, N = m + n) hold the k x k Gram matrix and the
        // rows x k correction
        double *G = D.V[0], *C = D.V[1];
        for (int side = 0; side < 2; side++) {
            const int rows = side ? D.n : D.m;
            hipLaunchKernelGGL(k_svd_gram, dim3(k, k), dim3(256), 0, st, D, side, G);
            hipLaunchKernelGGL(k_svd_corr, dim3((rows + 255) / 256, k), dim3(256), 0, st, D, side, G, C);
            hipLaunchKernelGGL(k_svd_apply, dim3((rows + 255) / 256, k), dim3(256), 0, st, D, side, C);
        }
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace zk
