// Two-site update of a matrix product state in double-double: the step of the
// MPS simulation whose cost the paper attributes to the Hermitian
// eigendecomposition (Sec. 1 and Sec. 2.1).  For neighbouring site tensors A
// (chi_l x 2 x chi) and B (chi x 2 x chi_r) and a two-qubit gate G:
//   theta[(s1, l), (s2, r)] = sum_m A[(s1, l), m] B[m, (s2, r)]
//   theta'[(s1, l), (s2, r)] = sum_{s1', s2'} G[(s1, s2), (s1', s2')] theta[(s1', l), (s2', r)]
// then theta' = U diag(s) V^H (the double-double SVD) is cut to chi' columns:
// A' = U[:, :chi'], B' = diag(s[:chi']) V[:, :chi']^H.
// Layout: complex128 limb planes (hi, lo), column-major; the row index of A
// and of theta is s1 chi_l + l, the column index of B and of theta s2 chi_r + r.
#include <hip/hip_runtime.h>

#include "common.h"
#include "stage.h"

namespace zk {

namespace {

__device__ __forceinline__ cmp<2> ld_c2(const double *const *P, size_t idx)
{
    const double2 h = ld2(P[0] + 2 * idx), l = ld2(P[1] + 2 * idx);
    cmp<2> z;
    z.re = dd{{h.x, l.x}};
    z.im = dd{{h.y, l.y}};
    return z;
}

__device__ __forceinline__ void st_c2(double *const *P, size_t idx, const cmp<2> &z)
{
    st2(P[0] + 2 * idx, make_double2(z.re.x[0], z.im.x[0]));
    st2(P[1] + 2 * idx, make_double2(z.re.x[1], z.im.x[1]));
}

// theta = A B: one thread per entry, the sum over m in double-double;
// grid ceil(M N / 256)
__global__ void __launch_bounds__(256) k_mps_theta(MpsDesc D)
{
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)D.M * D.N) return;
    const int i = (int)(t % D.M), j = (int)(t / D.M);
    cmp<2> acc = c_zero<2>();
    for (int m = 0; m < D.K; m++)
        acc = c_add(acc, c_mul(ld_c2(D.A, (size_t)m * D.lda + i), ld_c2(D.B, (size_t)j * D.ldb + m)));
    st_c2(D.T, (size_t)j * D.M + i, acc);
}

// theta' = G theta on the physical indices, in place: one thread per (l, r)
// owns the four entries (s1, s2); grid ceil(chi_l chi_r / 256)
__global__ void __launch_bounds__(256) k_mps_gate(MpsDesc D)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= D.chil * D.chir) return;
    const int l = t % D.chil, r = t / D.chil;
    cmp<2> x[4];
    for (int s1 = 0; s1 < 2; s1++)
        for (int s2 = 0; s2 < 2; s2++)
            x[2 * s1 + s2] = ld_c2(D.T, (size_t)(s2 * D.chir + r) * D.M + s1 * D.chil + l);
    for (int s1 = 0; s1 < 2; s1++)
        for (int s2 = 0; s2 < 2; s2++) {
            const int row = 2 * s1 + s2;
            cmp<2> acc = c_zero<2>();
            for (int c = 0; c < 4; c++) acc = c_add(acc, c_mul(ld_c2(D.G, (size_t)c * 4 + row), x[c]));
            st_c2(D.T, (size_t)(s2 * D.chir + r) * D.M + s1 * D.chil + l, acc);
        }
}

// B'[j, q] = s_j conj(V[q, j]) for j < chi', q < N (ld chi'); grid ceil(chi' N / 256)
__global__ void __launch_bounds__(256) k_mps_bout(MpsDesc D)
{
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)D.chi * D.N) return;
    const int j = (int)(t % D.chi), q = (int)(t / D.chi);
    const cmp<2> v = ld_c2(D.V, (size_t)j * D.ldv + q);
    const dd s = dd{{D.s[0][j], D.s[1][j]}};
    cmp<2> b;
    b.re = mul(s, v.re);
    b.im = mp_neg<2>(mul(s, v.im));
    st_c2(D.Bo, (size_t)q * D.chi + j, b);
}

}  // namespace

int mps_theta(const MpsDesc &D, hipStream_t st)
{
    const size_t total = (size_t)D.M * D.N;
    hipLaunchKernelGGL(k_mps_theta, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, D);
    hipLaunchKernelGGL(k_mps_gate, dim3((unsigned)((D.chil * D.chir + 255) / 256)), dim3(256), 0, st, D);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int mps_bout(const MpsDesc &D, hipStream_t st)
{
    const size_t total = (size_t)D.chi * D.N;
    if (total == 0) return 0;
    hipLaunchKernelGGL(k_mps_bout, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, D);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace zk
