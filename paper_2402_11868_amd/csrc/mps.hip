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

#include <algorithm>

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

// ------------------------------------------------- MPS simulation ----
// Sites in right-canonical form with bond weights (Hastings' form of the
// Vidal decomposition): site q is B_q[l, s, r], stored cl x (2 cr) with
// column index s cr + r; bond q carries lambda_q (Schmidt values).

// theta[(s1 l), (s2 r)] = sum_m Bq[l, s1, m] Bq1[m, s2, r]: one thread per entry
__global__ void __launch_bounds__(256) k_sim_theta(MpsSimDesc D)
{
    const int M = 2 * D.cl, N = 2 * D.cr;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)M * N) return;
    const int i = (int)(t % M), j = (int)(t / M);
    const int s1 = i / D.cl, l = i % D.cl, s2 = j / D.cr, r = j % D.cr;
    cmp<2> acc = c_zero<2>();
    for (int m = 0; m < D.cm; m++)
        acc = c_add(acc, c_mul(ld_c2(D.Bq, (size_t)(s1 * D.cm + m) * D.cl + l),
                               ld_c2(D.Bq1, (size_t)(s2 * D.cr + r) * D.cm + m)));
    st_c2(D.T, (size_t)j * M + i, acc);
}

// theta' = G theta on the physical indices (in place), one thread per (l, r)
__global__ void __launch_bounds__(256) k_sim_gate2(MpsSimDesc D)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= D.cl * D.cr) return;
    const int M = 2 * D.cl;
    const int l = t % D.cl, r = t / D.cl;
    cmp<2> x[4];
    for (int s1 = 0; s1 < 2; s1++)
        for (int s2 = 0; s2 < 2; s2++) x[2 * s1 + s2] = ld_c2(D.T, (size_t)(s2 * D.cr + r) * M + s1 * D.cl + l);
    for (int s1 = 0; s1 < 2; s1++)
        for (int s2 = 0; s2 < 2; s2++) {
            const int row = 2 * s1 + s2;
            cmp<2> acc = c_zero<2>();
            for (int c = 0; c < 4; c++) acc = c_add(acc, c_mul(ld_c2(D.G, (size_t)c * 4 + row), x[c]));
            st_c2(D.T, (size_t)(s2 * D.cr + r) * M + s1 * D.cl + l, acc);
        }
}

// bond matrix rho = theta^H diag(lambda_{q-1}^2 per row block) theta (order
// 2 cr, both triangles), one thread per entry
__global__ void __launch_bounds__(256) k_sim_rho(MpsSimDesc D)
{
    const int M = 2 * D.cl, N = 2 * D.cr;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)N * N) return;
    const int a = (int)(t % N), b = (int)(t / N);
    cmp<2> acc = c_zero<2>();
    for (int i = 0; i < M; i++) {
        const int l = i % D.cl;
        cmp<2> p = c_mulc(ld_c2(D.T, (size_t)a * M + i), ld_c2(D.T, (size_t)b * M + i));
        if (D.lam[0]) {
            const dd w = dd{{D.lam[0][l], D.lam[1][l]}};
            const dd w2 = mul(w, w);
            p.re = mul(p.re, w2);
            p.im = mul(p.im, w2);
        }
        acc = c_add(acc, p);
    }
    st_c2(D.rho, (size_t)b * N + a, acc);
}

// after the bond matrix's eigendecomposition (ascending eigenvalues w, vectors
// V, order N = 2 cr): keep the chi largest, j = 0 .. chi-1 <-> k = N-1-j:
//   B'_{q+1}[j, (s2 r)] = conj(V[(s2 r), k]),  B'_q[l, s1, j] = sum_b theta[(s1 l), b] V[b, k],
//   lambda'_j = sqrt(max(w_k, 0)), eig'_j = w_k
__global__ void __launch_bounds__(256) k_sim_split(MpsSimDesc D)
{
    const int M = 2 * D.cl, N = 2 * D.cr, chi = D.chi;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t n1 = (size_t)chi * N, n2 = (size_t)M * chi;
    if (t < n1) {
        const int j = (int)(t % chi), q = (int)(t / chi);
        const cmp<2> v = ld_c2(D.V, (size_t)(N - 1 - j) * N + q);
        st_c2(D.Bq1_out, (size_t)q * chi + j, c_conj<2>(v));
    }
    if (t < n2) {
        const int i = (int)(t % M), j = (int)(t / M);
        const int s1 = i / D.cl, l = i % D.cl;
        cmp<2> acc = c_zero<2>();
        for (int b = 0; b < N; b++)
            acc = c_add(acc, c_mul(ld_c2(D.T, (size_t)b * M + i), ld_c2(D.V, (size_t)(N - 1 - j) * N + b)));
        st_c2(D.Bq_out, (size_t)(s1 * chi + j) * D.cl + l, acc);
    }
    if (t < (size_t)chi) {
        const int j = (int)t;
        const dd w = dd{{D.w[0][N - 1 - j], D.w[1][N - 1 - j]}};
        const dd s = w.x[0] > 0.0 ? sqrt_mp<2>(w) : mp_zero<2>();
        D.lam_out[0][j] = s.x[0];
        D.lam_out[1][j] = s.x[1];
        D.eig_out[0][j] = w.x[0];
        D.eig_out[1][j] = w.x[1];
    }
}

// one-qubit gate on site q in place: B[l, s, r] <- sum_s' G[s, s'] B[l, s', r]
__global__ void __launch_bounds__(256) k_sim_gate1(MpsSimDesc D)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= D.cl * D.cm) return;
    const int l = t % D.cl, r = t / D.cl;
    double *const *B = D.T;   // the site, in place
    const cmp<2> x0 = ld_c2(B, (size_t)(0 * D.cm + r) * D.cl + l), x1 = ld_c2(B, (size_t)(1 * D.cm + r) * D.cl + l);
    for (int s = 0; s < 2; s++) {
        const cmp<2> y = c_add(c_mul(ld_c2(D.G, (size_t)0 * 2 + s), x0), c_mul(ld_c2(D.G, (size_t)1 * 2 + s), x1));
        st_c2(B, (size_t)(s * D.cm + r) * D.cl + l, y);
    }
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

int mps_sim_bond(const MpsSimDesc &D, hipStream_t st)
{
    const size_t MN = (size_t)4 * D.cl * D.cr, NN = (size_t)4 * D.cr * D.cr;
    hipLaunchKernelGGL(k_sim_theta, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st, D);
    hipLaunchKernelGGL(k_sim_gate2, dim3((unsigned)((D.cl * D.cr + 255) / 256)), dim3(256), 0, st, D);
    hipLaunchKernelGGL(k_sim_rho, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, st, D);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int mps_sim_split(const MpsSimDesc &D, hipStream_t st)
{
    const size_t n = std::max((size_t)D.chi * 2 * D.cr, (size_t)2 * D.cl * D.chi);
    hipLaunchKernelGGL(k_sim_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, D);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int mps_sim_gate1(const MpsSimDesc &D, hipStream_t st)
{
    hipLaunchKernelGGL(k_sim_gate1, dim3((unsigned)((D.cl * D.cm + 255) / 256)), dim3(256), 0, st, D);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace zk

