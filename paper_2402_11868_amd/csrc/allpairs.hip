// All-pairs refinement of a binary64 eigendecomposition to double-double
// accuracy in O(n^3) work per matrix: every eigenpair of the matrix is
// corrected at once from the residual matrix, instead of one shifted LU
// factorisation per pair and iteration.
//
// One iteration on the basis X (double-double, columns x_j) with shifts
// lam_j (double-double):
//   R = H X - X diag(lam)        exact products, cascaded sums; binary64 result
//   F = X_hi^H R                 binary64 (FP64-MFMA GEMM): f_ij = x_i^H r_j
//   theta_j = lam_j + Re f_jj / |x_j|^2        Rayleigh quotients
//   pairs i, j are coupled when |f_ij| + |f_ji| > eta |theta_j - theta_i|;
//   the connected runs of the sorted thetas are the blocks.
//   Separated pairs get the first-order correction
//       e_ij = (f'_ij + conj(f'_ji)) / (2 (theta_j - theta_i)) - g_ij / 2,
//       e_jj = (1 - g_jj) / 2,     f'_ij = f_ij - (theta_j - lam_j) g_ij,
//   G = X^H X in double-double: in exact arithmetic this is
//   f'_ij / (theta_j - theta_i), and its Hermitian part -G/2 restores
//   orthonormality to first order whatever the rounding noise of F divided
//   by a small gap does to the anti-Hermitian part.  A block whose members still miss the
//   tolerance is rotated by the eigenvectors Q_J of its projected matrix
//   F_JJ + G_JJ (Lam_J - mu), computed by the binary64 stage at the block's own
//   scale, and the corrections of the other pairs are taken in the rotated
//   basis; inside a block the columns are orthonormalised (Lowdin, first
//   order).  X <- X + X M with M = Q (I + E) - I, one double-double GEMM.
// The projected blocks give the multi-level behaviour: eigenvalues that
// binary64 cannot separate relative to ||H|| are separated relative to their
// block's scale, and the next iteration treats them as separated pairs.
// This is the O(n^3) alternative to the paper's per-pair Rayleigh quotient
// iteration (Sec. 2, ZKCM_CUS); the correction formula is the Hermitian form
// of Ogita and Aishima's refinement (Japan J. Indust. Appl. Math. 2018), the
// block treatment our own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/zk.h"
#include "ap_host.h"
#include "api_internal.h"
#include "common.h"
#include "stage.h"

int run_stage1(zk_ctx *ctx, int count, const zk_herm *A, const std::vector<double *> &hf, const std::vector<double *> &w0,
               const std::vector<double *> &V0, const std::vector<int *> &flag, const std::vector<int> &fp32);

namespace zk {

int zgemm_batched(const GemmDesc *d_descs, int count, int M, int N, int K, int opA, int opB, hipStream_t st);

namespace {

constexpr double kApEta = 1e-8;   // coupling threshold |f_ij| + |f_ji| vs |theta_j - theta_i|

// One matrix of an all-pairs batch (device pointers).  Matrices are n x n,
// column-major, leading dimension n.  Double-double matrices are four planes
// (re_hi, re_lo, im_hi, im_lo); binary64 complex matrices are interleaved.
// Double-double vectors are two planes (hi[0..n), lo[n..2n)).
struct ApProb {
    int n, limbs_in, nbc, pad;
    const double *hf;        // 2 limbs_in planes: re and im of each input limb
    double *X, *Xn;          // basis and the next basis
    double2 *Xh;             // leading limbs of X, interleaved
    double2 *R, *F, *E, *M;  // residual matrix, X_hi^H R, correction, update
    double2 *Gf;             // X^H X (binary64 rounding of the double-double product)
    double2 *Fc;             // n x nbc: rotated F columns of the block columns
    double *lam, *theta, *g, *rnorm, *orth;
    const double *w0;
    const double2 *V0;
    int *pos, *reach;
    int *blk, *loc, *bcol, *boff, *brot, *qoff;
    double2 *Q, *Gh, *W, *T; // packed m x m per rotated block (column-major, offset qoff)
    double *th;              // eigenvalues of the rotated blocks' projected matrices, by slot
};

struct RotBlk {
    int prob, b;
};

// ------------------------------------------------------------ helpers -----
__device__ __forceinline__ double dd_diff(double ah, double al, double bh, double bl)
{
    double s, e;
    two_sum(ah, -bh, s, e);
    return s + (e + (al - bl));
}

// (S, C) += x * y, x double-double, y double-double
__device__ __forceinline__ void ap_acc(double &S, double &C, double xh, double xl, double yh, double yl)
{
    const double p = xh * yh;
    const double e = fma(xh, yh, -p);
    const double s = S + p;
    const double bb = s - S;
    const double t = (S - (s - bb)) + (p - bb);
    S = s;
    C += fma(xh, yl, fma(xl, yh, t + e));
}

// (S, C) += x * y, x double-double, y binary64
__device__ __forceinline__ void ap_acc_d(double &S, double &C, double xh, double xl, double y)
{
    const double p = xh * y;
    const double e = fma(xh, y, -p);
    const double s = S + p;
    const double bb = s - S;
    const double t = (S - (s - bb)) + (p - bb);
    S = s;
    C += fma(xl, y, t + e);
}

__device__ __forceinline__ double2 cmulz(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ double2 cmulcz(double2 a, double2 b)   // conj(a) b
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ void dd_norm(double &s, double &c)
{
    double h, l;
    two_sum(s, c, h, l);
    s = h;
    c = l;
}

// ------------------------------------------------------------ kernels -----
__global__ void __launch_bounds__(256) k_ap_init(const ApProb *pp)
{
    const ApProb &P = pp[blockIdx.y];
    const int n = P.n;
    const size_t nn = (size_t)n * n;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (size_t)gridDim.x * 256) {
        const double2 v = P.V0[e];
        P.X[e] = v.x;
        P.X[nn + e] = 0.0;
        P.X[2 * nn + e] = v.y;
        P.X[3 * nn + e] = 0.0;
        P.Xh[e] = v;
        if (e < (size_t)n) {
            P.lam[e] = P.w0[e];
            P.lam[n + e] = 0.0;
        }
    }
}

// R = H X - X diag(lam): 64 x 16 tiles, 4 outputs per thread (rows tx + 16a,
// column ty), cascaded accumulation of exact products (Casc3), so that the
// entries of R, which are small next to ||H||, are exact to about u^3 ||H||
// before their rounding to binary64.
constexpr int kRK = 16;

template <int LIN>
__global__ void __launch_bounds__(256) k_ap_resid(const ApProb *pp)
{
    const ApProb &P = pp[blockIdx.y];
    const int n = P.n;
    const int tilesI = (n + 63) / 64;
    const int ti = blockIdx.x % tilesI, tj = blockIdx.x / tilesI;
    if (tj * 16 >= n) return;
    const int i0 = ti * 64, j0 = tj * 16;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const size_t nn = (size_t)n * n;
    __shared__ double sH[2 * LIN][kRK][64];
    __shared__ double sX[4][kRK][17];
    Casc3 re[4], im[4];
    for (int k0 = 0; k0 < n; k0 += kRK) {
        __syncthreads();
        for (int e = tid; e < 64 * kRK; e += 256) {
            const int ii = e & 63, kk = e >> 6;
            const int gi = i0 + ii, gk = k0 + kk;
            const bool ok = gi < n && gk < n;
#pragma unroll
            for (int pl = 0; pl < 2 * LIN; pl++) sH[pl][kk][ii] = ok ? P.hf[pl * nn + (size_t)gk * n + gi] : 0.0;
        }
        {
            const int kk = tid & 15, jj = tid >> 4;
            const int gk = k0 + kk, gj = j0 + jj;
            const bool ok = gk < n && gj < n;
#pragma unroll
            for (int pl = 0; pl < 4; pl++) sX[pl][kk][jj] = ok ? P.X[pl * nn + (size_t)gj * n + gk] : 0.0;
        }
        __syncthreads();
        for (int kk = 0; kk < kRK; kk++) {
            const double xrh = sX[0][kk][ty], xrl = sX[1][kk][ty], xih = sX[2][kk][ty], xil = sX[3][kk][ty];
#pragma unroll
            for (int a = 0; a < 4; a++) {
#pragma unroll
                for (int l = 0; l < LIN; l++) {
                    const double hr = sH[2 * l][kk][tx + 16 * a], hi = sH[2 * l + 1][kk][tx + 16 * a];
                    re[a].add(hr, xrh, xrl);
                    re[a].add(-hi, xih, xil);
                    im[a].add(hr, xih, xil);
                    im[a].add(hi, xrh, xrl);
                }
            }
        }
    }
    const int j = j0 + ty;
    if (j >= n) return;
    const double lh = P.lam[j], ll = P.lam[n + j];
    for (int a = 0; a < 4; a++) {
        const int i = i0 + tx + 16 * a;
        if (i >= n) continue;
        const size_t o = (size_t)j * n + i;
        const double xrh = P.X[o], xrl = P.X[nn + o], xih = P.X[2 * nn + o], xil = P.X[3 * nn + o];
        re[a].add(-lh, xrh, xrl);
        re[a].add(-ll, xrh, xrl);
        im[a].add(-lh, xih, xil);
        im[a].add(-ll, xih, xil);
        double rh, rl, ih, il;
        re[a].get(rh, rl);
        im[a].get(ih, il);
        P.R[o] = make_double2(rh, ih);
    }
}

// per column: ||r_j|| (binary64) and |x_j|^2 (double-double)
__global__ void __launch_bounds__(256) k_ap_colstats(const ApProb *pp)
{
    const ApProb &P = pp[blockIdx.y];
    const int n = P.n, j = blockIdx.x;
    if (j >= n) return;
    const size_t nn = (size_t)n * n;
    __shared__ double red[3][4];
    double r2 = 0.0, S = 0.0, C = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const size_t o = (size_t)j * n + i;
        const double2 r = P.R[o];
        r2 += r.x * r.x + r.y * r.y;
        const double a = P.X[o], al = P.X[nn + o], b = P.X[2 * nn + o], bl = P.X[3 * nn + o];
        ap_acc(S, C, a, al, a, al);
        ap_acc(S, C, b, bl, b, bl);
    }
    dd_norm(S, C);
    for (int off = 32; off > 0; off >>= 1) {
        r2 += __shfl_xor(r2, off, 64);
        const double os = __shfl_xor(S, off, 64), oc = __shfl_xor(C, off, 64);
        double s, e;
        two_sum(S, os, s, e);
        C = C + oc + e;
        S = s;
        dd_norm(S, C);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wid] = r2;
        red[1][wid] = S;
        red[2][wid] = C;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t2 = 0.0, s = 0.0, c = 0.0;
        for (int w = 0; w < 4; w++) {
            t2 += red[0][w];
            double h, e;
            two_sum(s, red[1][w], h, e);
            c = c + red[2][w] + e;
            s = h;
            dd_norm(s, c);
        }
        P.rnorm[j] = sqrt(t2);
        P.g[j] = s;
        P.g[n + j] = c;
    }
}

// orth_j = max(max_{i != j} |g_ij|, | |x_j|^2 - 1 |): departure from orthonormality
__global__ void __launch_bounds__(256) k_ap_orth(const ApProb *pp)
{
    const ApProb &P = pp[blockIdx.y];
    const int n = P.n, j = blockIdx.x;
    if (j >= n) return;
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        if (i == j) continue;
        const double2 g = P.Gf[(size_t)j * n + i];
        m = fmax(m, fabs(g.x) + fabs(g.y));
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double d = fabs((P.g[j] - 1.0) + P.g[n + j]);
        P.orth[j] = fmax(fmax(fmax(red[0], red[1]), fmax(red[2], red[3])), d);
    }
}

// theta_j = lam_j + Re(f_jj) / |x_j|^2
__global__ void __launch_bounds__(256) k_ap_theta(const ApProb *pp)
{
    const ApProb &P = pp[blockIdx.y];
    const int n = P.n, j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const double q = P.F[(size_t)j * n + j].x / P.g[j];
    double s, e;
    two_sum(P.lam[j], q, s, e);
    e += P.lam[n + j];
    fast_two_sum(s, e, s, e);
    P.theta[j] = s;
    P.theta[n + j] = e;
}

// reach[pos_j] = smallest sorted position of a pair coupled to j and placed
// before it (pos_j itself when there is none)
__global__ void __launch_bounds__(256) k_ap_couple(const ApProb *pp, double eta)
{
    const ApProb &P = pp[blockIdx.y];
    const int n = P.n, j = blockIdx.x;
    if (j >= n) return;
    const int pj = P.pos[j];
    const double tjh = P.theta[j], tjl = P.theta[n + j];
    int best = pj;
    for (int i = threadIdx.x; i < n; i += 256) {
        const int pi = P.pos[i];
        if (pi >= pj) continue;
        const double2 a = P.F[(size_t)j * n + i], b = P.F[(size_t)i * n + j];
        const double c = fabs(a.x) + fabs(a.y) + fabs(b.x) + fabs(b.y);
        const double d = fabs(dd_diff(tjh, tjl, P.theta[i], P.theta[n + i]));
        if (d == 0.0 || c > eta * d) best = min(best, pi);
    }
    for (int off = 32; off > 0; off >>= 1) best = min(best, __shfl_xor(best, off, 64));
    __shared__ int red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) P.reach[pj] = min(min(red[0], red[1]), min(red[2], red[3]));
}

// projected matrix of a rotated block, Hermitian part, for the binary64 stage:
// T(a, c) = F(J_a, J_c) + G(J_a, J_c) (lam_{J_c} - mu), mu = lam of the first member
__global__ void __launch_bounds__(256) k_ap_tbuild(const ApProb *pp, const RotBlk *rb)
{
    const RotBlk B = rb[blockIdx.y];
    const ApProb &P = pp[B.prob];
    const int n = P.n, o = P.boff[B.b], m = P.boff[B.b + 1] - o;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= m * m) return;
    const int a = e % m, c = e / m;
    const int ja = P.bcol[o + a], jc = P.bcol[o + c];
    const int j0 = P.bcol[o];
    const double muh = P.lam[j0], mul = P.lam[n + j0];
    const double dc = dd_diff(P.lam[jc], P.lam[n + jc], muh, mul);
    const double da = dd_diff(P.lam[ja], P.lam[n + ja], muh, mul);
    const double2 f1 = P.F[(size_t)jc * n + ja], g1 = P.Gf[(size_t)jc * n + ja];
    const double2 f2 = P.F[(size_t)ja * n + jc], g2 = P.Gf[(size_t)ja * n + jc];
    const double2 t1 = make_double2(f1.x + g1.x * dc, f1.y + g1.y * dc);   // T(a, c)
    const double2 t2 = make_double2(f2.x + g2.x * da, f2.y + g2.y * da);   // T(c, a)
    double2 t = make_double2(0.5 * (t1.x + t2.x), 0.5 * (t1.y - t2.y));
    if (a == c) t.y = 0.0;
    P.T[P.qoff[B.b] + (size_t)c * m + a] = t;
}

// rotated F columns of the rotated blocks:
// Fc(:, c) = sum_k F(:, J_k) Q(k, c) + sum_k G(:, J_k) (lam_{J_k} - theta_c) Q(k, c)
__global__ void __launch_bounds__(256) k_ap_fcols(const ApProb *pp, const RotBlk *rb, int cmax)
{
    const RotBlk B = rb[blockIdx.z];
    const ApProb &P = pp[B.prob];
    const int n = P.n, o = P.boff[B.b], m = P.boff[B.b + 1] - o;
    const int c = blockIdx.y;
    if (c >= m) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    (void)cmax;
    const int j0 = P.bcol[o];
    const double muh = P.lam[j0], mul = P.lam[n + j0];
    const double thc = P.th[o + c];
    const double2 *Q = P.Q + P.qoff[B.b];
    double2 acc = make_double2(0.0, 0.0);
    for (int k = 0; k < m; k++) {
        const int jk = P.bcol[o + k];
        const double2 q = Q[(size_t)c * m + k];
        const double d = dd_diff(P.lam[jk], P.lam[n + jk], muh, mul) - thc;
        const double2 f = P.F[(size_t)jk * n + i], gg = P.Gf[(size_t)jk * n + i];
        const double2 v = make_double2(f.x + gg.x * d, f.y + gg.y * d);
        const double2 p = cmulz(v, q);
        acc.x += p.x;
        acc.y += p.y;
    }
    P.Fc[(size_t)(o + c) * n + i] = acc;
}

// W = G_JJ Q, then Gh = Q^H W, per rotated block
__global__ void __launch_bounds__(256) k_ap_gq(const ApProb *pp, const RotBlk *rb)
{
    const RotBlk B = rb[blockIdx.y];
    const ApProb &P = pp[B.prob];
    const int n = P.n, o = P.boff[B.b], m = P.boff[B.b + 1] - o;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= m * m) return;
    const int a = e % m, c = e / m;
    const double2 *Q = P.Q + P.qoff[B.b];
    const int ja = P.bcol[o + a];
    double2 acc = make_double2(0.0, 0.0);
    for (int b = 0; b < m; b++) {
        const double2 p = cmulz(P.Gf[(size_t)P.bcol[o + b] * n + ja], Q[(size_t)c * m + b]);
        acc.x += p.x;
        acc.y += p.y;
    }
    P.W[P.qoff[B.b] + (size_t)c * m + a] = acc;
}

__global__ void __launch_bounds__(256) k_ap_qhw(const ApProb *pp, const RotBlk *rb)
{
    const RotBlk B = rb[blockIdx.y];
    const ApProb &P = pp[B.prob];
    const int o = P.boff[B.b], m = P.boff[B.b + 1] - o;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= m * m) return;
    const int a = e % m, c = e / m;
    const double2 *Q = P.Q + P.qoff[B.b], *Wm = P.W + P.qoff[B.b];
    double2 acc = make_double2(0.0, 0.0);
    for (int b = 0; b < m; b++) {
        const double2 p = cmulcz(Q[(size_t)a * m + b], Wm[(size_t)c * m + b]);
        acc.x += p.x;
        acc.y += p.y;
    }
    P.Gh[P.qoff[B.b] + (size_t)c * m + a] = acc;
}

// new Rayleigh-quotient estimate of column j: mu + theta of its rotated block, else theta_j
__device__ __forceinline__ void ap_newlam(const ApProb &P, int j, double &h, double &l)
{
    const int n = P.n, b = P.blk[j];
    if (b >= 0 && P.brot[b]) {
        const int j0 = P.bcol[P.boff[b]];
        double s, e;
        two_sum(P.lam[j0], P.th[P.boff[b] + P.loc[j]], s, e);
        e += P.lam[n + j0];
        fast_two_sum(s, e, h, l);
    } else {
        h = P.theta[j];
        l = P.theta[n + j];
    }
}

// E (in the rotated basis of the rotated blocks)
__global__ void __launch_bounds__(256) k_ap_ehat(const ApProb *pp)
{
    const ApProb &P = pp[blockIdx.z];
    const int n = P.n, j = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (j >= n || i >= n) return;
    const int bj = P.blk[j], bi = P.blk[i];
    const bool rj = bj >= 0 && P.brot[bj], ri = bi >= 0 && P.brot[bi];
    double2 e;
    if (i == j) {
        if (rj) {
            const int m = P.boff[bj + 1] - P.boff[bj], c = P.loc[j];
            e = make_double2(0.5 * (1.0 - P.Gh[P.qoff[bj] + (size_t)c * m + c].x), 0.0);
        } else {
            e = make_double2(0.5 * ((1.0 - P.g[j]) - P.g[n + j]), 0.0);
        }
    } else if (bi >= 0 && bi == bj) {
        double2 gv;
        if (rj) {
            const int m = P.boff[bj + 1] - P.boff[bj];
            gv = P.Gh[P.qoff[bj] + (size_t)P.loc[j] * m + P.loc[i]];
        } else {
            gv = P.Gf[(size_t)j * n + i];
        }
        e = make_double2(-0.5 * gv.x, -0.5 * gv.y);
    } else {
        // column j of X^H (H - theta_j) X: the rotated column of a rotated
        // block (taken at its new Ritz value), else F(:, j) - (theta_j - lam_j) G(:, j)
        const double2 *fcol = rj ? P.Fc + (size_t)(P.boff[bj] + P.loc[j]) * n : P.F + (size_t)j * n;
        const double2 *gcol = P.Gf + (size_t)j * n;
        const double dj = rj ? 0.0 : dd_diff(P.theta[j], P.theta[n + j], P.lam[j], P.lam[n + j]);
        double2 f;
        if (ri) {
            const int o = P.boff[bi], m = P.boff[bi + 1] - o, a = P.loc[i];
            const double2 *Q = P.Q + P.qoff[bi];
            f = make_double2(0.0, 0.0);
            for (int b = 0; b < m; b++) {
                const int r = P.bcol[o + b];
                const double2 v = make_double2(fcol[r].x - dj * gcol[r].x, fcol[r].y - dj * gcol[r].y);
                const double2 p = cmulcz(Q[(size_t)a * m + b], v);
                f.x += p.x;
                f.y += p.y;
            }
        } else {
            f = make_double2(fcol[i].x - dj * gcol[i].x, fcol[i].y - dj * gcol[i].y);
        }
        double thj, tlj, thi, tli;
        ap_newlam(P, j, thj, tlj);
        ap_newlam(P, i, thi, tli);
        const double d = dd_diff(thj, tlj, thi, tli);
        if (!ri && !rj) {
            // Hermitian part -g_ij / 2 taken from G (orthonormality to first
            // order, exactly as accurate as G), anti-Hermitian part from the
            // symmetrised F, so that rounding noise in F, divided by a small
            // gap, rotates the pair instead of breaking its orthogonality
            const double di = dd_diff(P.theta[i], P.theta[n + i], P.lam[i], P.lam[n + i]);
            const double2 fji = P.F[(size_t)i * n + j];
            const double2 g = gcol[i];
            const double2 s2 = make_double2(fcol[i].x + fji.x - (di + dj) * g.x, fcol[i].y - fji.y - (di + dj) * g.y);
            e = d != 0.0 ? make_double2(0.5 * (s2.x / d - g.x), 0.5 * (s2.y / d - g.y)) : make_double2(-0.5 * g.x, -0.5 * g.y);
        } else {
            e = d != 0.0 ? make_double2(f.x / d, f.y / d) : make_double2(0.0, 0.0);
        }
    }
    P.E[(size_t)j * n + i] = e;
}

// M = Q (I + E) - I: rows of the rotated blocks mixed by Q
__global__ void __launch_bounds__(256) k_ap_mbuild(const ApProb *pp)
{
    const ApProb &P = pp[blockIdx.z];
    const int n = P.n, j = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (j >= n || i >= n) return;
    const int bi = P.blk[i];
    double2 v;
    if (bi >= 0 && P.brot[bi]) {
        const int o = P.boff[bi], m = P.boff[bi + 1] - o, a = P.loc[i];
        const double2 *Q = P.Q + P.qoff[bi];
        v = make_double2(0.0, 0.0);
        for (int b = 0; b < m; b++) {
            const double2 p = cmulz(Q[(size_t)b * m + a], P.E[(size_t)j * n + P.bcol[o + b]]);
            v.x += p.x;
            v.y += p.y;
        }
        if (P.blk[j] == bi) {
            const double2 q = Q[(size_t)P.loc[j] * m + a];
            v.x += q.x - (P.loc[j] == a ? 1.0 : 0.0);
            v.y += q.y;
        }
    } else {
        v = P.E[(size_t)j * n + i];
    }
    P.M[(size_t)j * n + i] = v;
}

__global__ void __launch_bounds__(256) k_ap_lamset(const ApProb *pp)
{
    const ApProb &P = pp[blockIdx.y];
    const int n = P.n, j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    double h, l;
    ap_newlam(P, j, h, l);
    P.lam[j] = h;
    P.lam[n + j] = l;
}

// ------------------------------------------------------- dd GEMM -----------
// C = C0 + op(A) B, 64 x 64 tiles, 4 x 4 outputs per thread (rows tx + 16a,
// columns ty + 16b), operands staged through LDS in double-buffered chunks of
// 4 k-steps.  A: double-double planes, op = N or C (conjugate transpose).
// B: double-double planes with an optional column map, or binary64 complex.
// Output: double-double planes (plus an interleaved copy of the leading
// limbs), or binary64 complex.
struct DdGemm {
    const double *A;
    const double *B;
    const int *bmap;
    const double *C0;
    double *C;
    double2 *Cz;
    size_t pa, pb, pc;
    int lda, ldb, ldc, M, N, K, pad;
    size_t pc0;   // plane stride of C0 (0: that of C)
};

constexpr int kGK = 4;

template <bool CONJA, bool BDD, bool OUTDD>
__global__ void __launch_bounds__(256, 2) k_ap_ddgemm(const DdGemm *gd)
{
    const DdGemm &G = gd[blockIdx.y];
    const int tilesI = (G.M + 63) / 64;
    const int ti = blockIdx.x % tilesI, tj = blockIdx.x / tilesI;
    if (tj * 64 >= G.N) return;
    const int i0 = ti * 64, j0 = tj * 64;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    __shared__ double sA[2][4][kGK][64];
    __shared__ double sB[2][4][kGK][64];
    double pA[4], pB[4];
    auto fetch = [&](int kc) {
        if (!CONJA) {
            const int kk = tid >> 6, ii = tid & 63;
            const int k = kc + kk, i = i0 + ii;
            const bool ok = k < G.K && i < G.M;
            const size_t o = (size_t)k * G.lda + i;
#pragma unroll
            for (int pl = 0; pl < 4; pl++) pA[pl] = ok ? G.A[pl * G.pa + o] : 0.0;
        } else {
            const int kk = tid & (kGK - 1), ii = tid / kGK;
            const int k = kc + kk, i = i0 + ii;
            const bool ok = k < G.K && i < G.M;
            const size_t o = (size_t)i * G.lda + k;
#pragma unroll
            for (int pl = 0; pl < 4; pl++) pA[pl] = ok ? G.A[pl * G.pa + o] : 0.0;
            pA[2] = -pA[2];
            pA[3] = -pA[3];
        }
        {
            const int kk = tid & (kGK - 1), jj = tid / kGK;
            const int k = kc + kk, j = j0 + jj;
            const bool ok = k < G.K && j < G.N;
            if (BDD) {
                const int cj = ok ? (G.bmap ? G.bmap[j] : j) : 0;
                const size_t o = (size_t)cj * G.ldb + k;
#pragma unroll
                for (int pl = 0; pl < 4; pl++) pB[pl] = ok ? G.B[pl * G.pb + o] : 0.0;
            } else {
                const double2 b = ok ? reinterpret_cast<const double2 *>(G.B)[(size_t)j * G.ldb + k] : make_double2(0.0, 0.0);
                pB[0] = b.x;
                pB[1] = 0.0;
                pB[2] = b.y;
                pB[3] = 0.0;
            }
        }
    };
    auto stash = [&](int buf) {
        if (!CONJA) {
#pragma unroll
            for (int pl = 0; pl < 4; pl++) sA[buf][pl][tid >> 6][tid & 63] = pA[pl];
        } else {
#pragma unroll
            for (int pl = 0; pl < 4; pl++) sA[buf][pl][tid & (kGK - 1)][tid / kGK] = pA[pl];
        }
#pragma unroll
        for (int pl = 0; pl < 4; pl++) sB[buf][pl][tid & (kGK - 1)][tid / kGK] = pB[pl];
    };
    fetch(0);
    // the product is accumulated from zero and C0 added once at the end, so
    // that the compensation stays at the size of the product (C0 + small
    // corrections is the common use)
    double S[4][4][2], C[4][4][2];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) S[a][b][0] = C[a][b][0] = S[a][b][1] = C[a][b][1] = 0.0;
    stash(0);
    __syncthreads();
    int buf = 0;
    for (int kc = 0; kc < G.K; kc += kGK) {
        const bool more = kc + kGK < G.K;
        if (more) fetch(kc + kGK);
        const int kmax = min(kGK, G.K - kc);
        for (int kk = 0; kk < kmax; kk++) {
            double brh[4], brl[4], bih[4], bil[4];
#pragma unroll
            for (int b = 0; b < 4; b++) {
                brh[b] = sB[buf][0][kk][ty + 16 * b];
                bih[b] = sB[buf][2][kk][ty + 16 * b];
                if (BDD) {
                    brl[b] = sB[buf][1][kk][ty + 16 * b];
                    bil[b] = sB[buf][3][kk][ty + 16 * b];
                }
            }
#pragma unroll
            for (int a = 0; a < 4; a++) {
                const double arh = sA[buf][0][kk][tx + 16 * a], arl = sA[buf][1][kk][tx + 16 * a];
                const double aih = sA[buf][2][kk][tx + 16 * a], ail = sA[buf][3][kk][tx + 16 * a];
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    if (BDD) {
                        ap_acc(S[a][b][0], C[a][b][0], arh, arl, brh[b], brl[b]);
                        ap_acc(S[a][b][0], C[a][b][0], -aih, -ail, bih[b], bil[b]);
                        ap_acc(S[a][b][1], C[a][b][1], arh, arl, bih[b], bil[b]);
                        ap_acc(S[a][b][1], C[a][b][1], aih, ail, brh[b], brl[b]);
                    } else {
                        ap_acc_d(S[a][b][0], C[a][b][0], arh, arl, brh[b]);
                        ap_acc_d(S[a][b][0], C[a][b][0], -aih, -ail, bih[b]);
                        ap_acc_d(S[a][b][1], C[a][b][1], arh, arl, bih[b]);
                        ap_acc_d(S[a][b][1], C[a][b][1], aih, ail, brh[b]);
                    }
                }
            }
        }
        // renormalise: the compensation stays at the rounding size of the
        // running sum instead of growing with the number of products (a long
        // sum with heavy cancellation, such as an off-diagonal entry of X^H X,
        // would otherwise carry about K u^2 times its largest partial sum)
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++) {
                dd_norm(S[a][b][0], C[a][b][0]);
                dd_norm(S[a][b][1], C[a][b][1]);
            }
        if (more) stash(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const int i = i0 + tx + 16 * a, j = j0 + ty + 16 * b;
            if (i >= G.M || j >= G.N) continue;
            double rh, rl, ih, il;
            two_sum(S[a][b][0], C[a][b][0], rh, rl);
            two_sum(S[a][b][1], C[a][b][1], ih, il);
            const size_t o = (size_t)j * G.ldc + i;
            if (G.C0) {
                const size_t p0 = G.pc0 ? G.pc0 : G.pc;
                const dd r = dd_add(dd{{G.C0[o], G.C0[p0 + o]}}, dd{{rh, rl}});
                const dd m = dd_add(dd{{G.C0[2 * p0 + o], G.C0[3 * p0 + o]}}, dd{{ih, il}});
                rh = r.x[0];
                rl = r.x[1];
                ih = m.x[0];
                il = m.x[1];
            }
            if (OUTDD) {
                G.C[o] = rh;
                G.C[G.pc + o] = rl;
                G.C[2 * G.pc + o] = ih;
                G.C[3 * G.pc + o] = il;
                if (G.Cz) G.Cz[o] = make_double2(rh, ih);
            } else {
                G.Cz[o] = make_double2(rh, ih);
            }
        }
}

// ------------------------------------------- Lowdin orthonormalisation ----
// One step X <- X (3 I - X^H X) / 2 = X - X (G - I) / 2 on column windows of
// double-double limb-planar matrices: G by one dd GEMM, the coefficients in
// place, X + X C into a packed copy by a second dd GEMM, and the copy back.
// A window orthonormal to d leaves the step orthonormal to about d^2 (the
// symmetric, smallest correction of the basis).
struct LowdinDesc {
    double *X;     // first column of the window, plane 0
    double *G;     // 4 planes of m x m
    double *T;     // 4 planes of n x m
    size_t px;     // plane stride of X
    int n, m;
};

__global__ void __launch_bounds__(256) k_lowdin_coef(const LowdinDesc *d)
{
    const LowdinDesc D = d[blockIdx.y];
    const size_t mm = (size_t)D.m * D.m;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < mm; e += (size_t)gridDim.x * 256) {
        // C = (I - G) / 2: halving is exact on both limbs
        double rh = -0.5 * D.G[e], rl = -0.5 * D.G[mm + e];
        double ih = -0.5 * D.G[2 * mm + e], il = -0.5 * D.G[3 * mm + e];
        if (e % D.m == e / D.m) {
            const dd r = dd_add(dd{{rh, rl}}, dd{{0.5, 0.0}});
            rh = r.x[0];
            rl = r.x[1];
            ih = il = 0.0;
        }
        D.G[e] = rh;
        D.G[mm + e] = rl;
        D.G[2 * mm + e] = ih;
        D.G[3 * mm + e] = il;
    }
}

__global__ void __launch_bounds__(256) k_lowdin_copy(const LowdinDesc *d)
{
    const LowdinDesc D = d[blockIdx.y];
    const size_t nm = (size_t)D.n * D.m;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nm; e += (size_t)gridDim.x * 256)
#pragma unroll
        for (int pl = 0; pl < 4; pl++) D.X[pl * D.px + e] = D.T[pl * nm + e];
}

// sorted output: w[l][k] = limb l of the eigenvalue of column perm[k], v[l](:, k) likewise
struct ApOut {
    double *w[2];
    double2 *v[2];
    int ldv, pad;
    const int *perm;
};

__global__ void __launch_bounds__(256) k_ap_output(const ApProb *pp, const ApOut *po)
{
    const ApProb &P = pp[blockIdx.z];
    const ApOut &O = po[blockIdx.z];
    const int n = P.n, k = blockIdx.y;
    if (k >= n) return;
    const int j = O.perm[k];
    const size_t nn = (size_t)n * n;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        O.w[0][k] = P.theta[j];
        O.w[1][k] = P.theta[n + j];
    }
    if (!O.v[0]) return;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const size_t o = (size_t)j * n + i;
        O.v[0][(size_t)k * O.ldv + i] = make_double2(P.X[o], P.X[2 * nn + o]);
        O.v[1][(size_t)k * O.ldv + i] = make_double2(P.X[nn + o], P.X[3 * nn + o]);
    }
}

inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }
inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

#define APCHK(expr)                                                                                   \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) {                                                                       \
            ctx->poisoned = true;                                                                     \
            return ctx->fail(ZK_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));              \
        }                                                                                             \
    } while (0)
#define APLAUNCH()                                                                                    \
    do {                                                                                              \
        hipError_t e_ = hipGetLastError();                                                            \
        if (e_ != hipSuccess) {                                                                       \
            ctx->poisoned = true;                                                                     \
            return ctx->fail(ZK_EDEVICE, "all-pairs launch failed: %s", hipGetErrorString(e_));        \
        }                                                                                             \
    } while (0)

// bytes of the per-matrix arrays of order n
size_t ap_matrix_bytes(int n)
{
    const size_t nn = (size_t)n * n;
    return 2 * al256(32 * nn)      // X, Xn
           + 7 * al256(16 * nn)    // Xh, R, F, E, M, Gf, Fc
           + 4 * al256(16 * nn)    // Q, Gh, W, T
           + 3 * al256(16 * (size_t)n) + 3 * al256(8 * (size_t)n)   // lam, theta, g, rnorm, orth, th
           + 8 * al256(4 * (size_t)n + 4);                          // pos, reach, blk, loc, bcol, boff, brot, qoff
}

struct HostProb {
    ApProb d;             // device pointers
    int n = 0, limbs_in = 1;
    double hnorm = 1.0;
    bool rotated_last = true, converged = false, inited = false, fin = false;
    int iters = 0;
    double tol = 1e-30;
    int max_iter = 12, want_vectors = 1;
    zk_eig_out out;
    void *cookie = nullptr;
    int chunk = -1;
    std::vector<double> theta, rnorm, orth;   // theta: 2n
    std::vector<int> pos, srt, reach;         // sorted positions, sorted order, coupling reach
    std::vector<int> cluster;                 // sorted index of the first member of each pair's block
    // block tables of this iteration
    std::vector<int> blk, loc, bcol, boff, brot, qoff;
    int nrot_cols = 0;
    double *hf_s1 = nullptr;   // binary64-stage scratch for the rotated blocks
    double *w_s1 = nullptr;
    int *flag_s1 = nullptr;
};

}  // namespace

size_t dd_lowdin_bytes(const std::vector<DdWindow> &w)
{
    size_t b = 0;
    for (const DdWindow &x : w) b += al256(32 * (size_t)x.m * x.m) + al256(32 * (size_t)x.n * x.m);
    return b + al256(sizeof(LowdinDesc) * w.size()) + 2 * al256(sizeof(DdGemm) * w.size());
}

int dd_lowdin(const std::vector<DdWindow> &w, int steps, void *scratch, hipStream_t st)
{
    const int cnt = (int)w.size();
    if (cnt == 0) return 0;
    char *b = (char *)scratch;
    std::vector<LowdinDesc> ld(cnt);
    std::vector<DdGemm> g1(cnt), g2(cnt);
    int max_m = 0, max_n = 0;
    for (int q = 0; q < cnt; q++) {
        LowdinDesc &D = ld[q];
        D.X = w[q].X;
        D.px = w[q].px;
        D.n = w[q].n;
        D.m = w[q].m;
        D.G = (double *)b;
        b += al256(32 * (size_t)D.m * D.m);
        D.T = (double *)b;
        b += al256(32 * (size_t)D.n * D.m);
        max_m = std::max(max_m, D.m);
        max_n = std::max(max_n, D.n);
        DdGemm &G = g1[q];   // G = X^H X
        std::memset(&G, 0, sizeof G);
        G.A = G.B = D.X;
        G.C = D.G;
        G.pa = G.pb = D.px;
        G.pc = (size_t)D.m * D.m;
        G.lda = G.ldb = D.n;
        G.ldc = D.m;
        G.M = G.N = D.m;
        G.K = D.n;
        DdGemm &H = g2[q];   // T = X + X C
        std::memset(&H, 0, sizeof H);
        H.A = D.X;
        H.B = D.G;
        H.C0 = D.X;
        H.C = D.T;
        H.pa = D.px;
        H.pb = (size_t)D.m * D.m;
        H.pc = (size_t)D.n * D.m;
        H.pc0 = D.px;
        H.lda = H.ldc = D.n;
        H.ldb = D.m;
        H.M = D.n;
        H.N = D.m;
        H.K = D.m;
    }
    LowdinDesc *d_ld = (LowdinDesc *)b;
    b += al256(sizeof(LowdinDesc) * cnt);
    DdGemm *d_g1 = (DdGemm *)b;
    b += al256(sizeof(DdGemm) * cnt);
    DdGemm *d_g2 = (DdGemm *)b;
    if (hipMemcpyAsync(d_ld, ld.data(), sizeof(LowdinDesc) * cnt, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d_g1, g1.data(), sizeof(DdGemm) * cnt, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d_g2, g2.data(), sizeof(DdGemm) * cnt, hipMemcpyHostToDevice, st) != hipSuccess)
        return -1;
    const unsigned t1 = cdiv(max_m, 64) * cdiv(max_m, 64), t2 = cdiv(max_n, 64) * cdiv(max_m, 64);
    const unsigned e1 = std::min<unsigned>(cdiv((size_t)max_m * max_m, 256), 4096u);
    const unsigned e2 = std::min<unsigned>(cdiv((size_t)max_n * max_m, 256), 4096u);
    for (int s = 0; s < steps; s++) {
        hipLaunchKernelGGL((k_ap_ddgemm<true, true, true>), dim3(t1, cnt), dim3(256), 0, st, d_g1);
        hipLaunchKernelGGL(k_lowdin_coef, dim3(e1, cnt), dim3(256), 0, st, d_ld);
        hipLaunchKernelGGL((k_ap_ddgemm<false, true, true>), dim3(t2, cnt), dim3(256), 0, st, d_g2);
        hipLaunchKernelGGL(k_lowdin_copy, dim3(e2, cnt), dim3(256), 0, st, d_ld);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}


// All-pairs refinement engine: matrices join with add() (their binary64 stage
// done), every round() runs one whole-basis iteration for each live matrix
// (matrices of equal order and input limbs share launches); a matrix that
// meets the stopping rule, or reaches its iteration limit, is written to its
// output in that round and listed in `finished`.  Device memory: one block per
// add() call, released when its last matrix finishes.
struct ApEngine::Impl {
    zk_ctx *ctx;
    std::vector<HostProb *> live;
    struct Chunk {
        void *p = nullptr;
        size_t bytes = 0;
        int left = 0;
    };
    std::vector<Chunk> chunks;
    void *meta = nullptr;
    size_t meta_bytes = 0;
    bool trace = false;
    explicit Impl(zk_ctx *c) : ctx(c) { trace = std::getenv("ZK_TRACE") != nullptr; }
    ~Impl()
    {
        hipStreamSynchronize(ctx->stream);
        for (HostProb *h : live) delete h;
        for (Chunk &c : chunks)
            if (c.p) {
                ctx->dev_free(c.p);
                ctx->extra -= c.bytes;
            }
        if (meta) {
            ctx->dev_free(meta);
            ctx->extra -= meta_bytes;
        }
    }
    // room for b more bytes under the context budget; the shifted-LU slots of
    // the Rayleigh-quotient engine are scratch between its rounds (it sizes
    // them again, from what is left, at its next round), so they are given
    // back when the budget is short
    bool room(size_t b) { return ctx->make_room(b); }
    int ensure_meta(size_t b)
    {
        if (b <= meta_bytes) return ZK_OK;
        if (meta) {
            hipStreamSynchronize(ctx->stream);
            ctx->dev_free(meta);
            ctx->extra -= meta_bytes;
            meta = nullptr;
            meta_bytes = 0;
        }
        if (!room(b)) return ctx->fail(ZK_ENOMEM, "all-pairs descriptors need %zu more bytes", b);
        if (ctx->dev_alloc(&meta, b) != ZK_OK) return ZK_ENOMEM;
        meta_bytes = b;
        ctx->extra += b;
        ctx->note_held();
        return ZK_OK;
    }
    void release(HostProb *h)
    {
        Chunk &c = chunks[h->chunk];
        if (--c.left == 0 && c.p) {
            hipStreamSynchronize(ctx->stream);
            ctx->dev_free(c.p);
            ctx->extra -= c.bytes;
            c.p = nullptr;
            c.bytes = 0;
        }
        delete h;
    }
    int add(const std::vector<ApReq> &reqs);
    int round(std::vector<ApDone> &finished);
    int iterate(std::vector<HostProb *> &grp, std::vector<ApDone> &finished);
    int output(std::vector<HostProb *> &done, std::vector<ApDone> &finished);
};

ApEngine::ApEngine(zk_ctx *ctx) : impl(new Impl(ctx)) {}
ApEngine::~ApEngine() { delete impl; }
bool ApEngine::any_live() const { return !impl->live.empty(); }
int ApEngine::add(const std::vector<ApReq> &reqs) { return impl->add(reqs); }
int ApEngine::round() { return impl->round(finished); }

int ApEngine::Impl::add(const std::vector<ApReq> &reqs)
{
    if (reqs.empty()) return ZK_OK;
    hipStream_t st = ctx->stream;
    size_t total = 0;
    for (const ApReq &r : reqs) {
        const size_t n = r.A.n, nn = n * n;
        total += ap_matrix_bytes((int)n) + al256(16 * nn) + al256(8 * n) + al256(4 * n);
    }
    if (!room(total)) return ctx->fail(ZK_ENOMEM, "all-pairs refinement needs %zu more bytes", total);
    Chunk ch;
    if (ctx->dev_alloc(&ch.p, total) != ZK_OK) return ZK_ENOMEM;
    ch.bytes = total;
    ch.left = (int)reqs.size();
    ctx->extra += total;
    ctx->note_held();
    chunks.push_back(ch);
    const int cid = (int)chunks.size() - 1;
    char *c = (char *)ch.p;
    std::vector<HostProb *> fresh;
    for (const ApReq &r : reqs) {
        HostProb *H = new HostProb;
        const int n = r.A.n;
        const size_t nn = (size_t)n * n;
        H->n = n;
        H->limbs_in = r.A.limbs;
        H->tol = r.tol;
        H->max_iter = r.max_iter;
        H->want_vectors = r.want_vectors;
        H->out = r.out;
        H->cookie = r.cookie;
        H->chunk = cid;
        ApProb &D = H->d;
        std::memset(&D, 0, sizeof D);
        D.n = n;
        D.limbs_in = r.A.limbs;
        D.hf = r.hf;
        D.w0 = r.w0;
        D.V0 = (const double2 *)r.V0;
        auto take = [&](size_t b) {
            char *q = c;
            c += al256(b);
            return q;
        };
        D.X = (double *)take(32 * nn);
        D.Xn = (double *)take(32 * nn);
        D.Xh = (double2 *)take(16 * nn);
        D.R = (double2 *)take(16 * nn);
        D.F = (double2 *)take(16 * nn);
        D.E = (double2 *)take(16 * nn);
        D.M = (double2 *)take(16 * nn);
        D.Gf = (double2 *)take(16 * nn);
        D.Fc = (double2 *)take(16 * nn);
        D.Q = (double2 *)take(16 * nn);
        D.Gh = (double2 *)take(16 * nn);
        D.W = (double2 *)take(16 * nn);
        D.T = (double2 *)take(16 * nn);
        D.lam = (double *)take(16 * (size_t)n);
        D.theta = (double *)take(16 * (size_t)n);
        D.g = (double *)take(16 * (size_t)n);
        D.rnorm = (double *)take(8 * (size_t)n);
        D.orth = (double *)take(8 * (size_t)n);
        D.th = (double *)take(8 * (size_t)n);
        D.pos = (int *)take(4 * (size_t)n + 4);
        D.reach = (int *)take(4 * (size_t)n + 4);
        D.blk = (int *)take(4 * (size_t)n + 4);
        D.loc = (int *)take(4 * (size_t)n + 4);
        D.bcol = (int *)take(4 * (size_t)n + 4);
        D.boff = (int *)take(4 * (size_t)n + 4);
        D.brot = (int *)take(4 * (size_t)n + 4);
        D.qoff = (int *)take(4 * (size_t)n + 4);
        H->hf_s1 = (double *)take(16 * nn);
        H->w_s1 = (double *)take(8 * (size_t)n);
        H->flag_s1 = (int *)take(4 * (size_t)n);
        H->cluster.assign(n, -1);
        fresh.push_back(H);
    }
    // ||H||_2 from the binary64 eigenvalues
    size_t tot_n = 0;
    for (HostProb *H : fresh) tot_n += H->n;
    std::vector<double> wv(tot_n);
    size_t o = 0;
    for (HostProb *H : fresh) {
        APCHK(hipMemcpyAsync(wv.data() + o, H->d.w0, 8 * (size_t)H->n, hipMemcpyDeviceToHost, st));
        o += H->n;
    }
    APCHK(hipStreamSynchronize(st));
    o = 0;
    for (HostProb *H : fresh) {
        double h = 0.0;
        for (int k = 0; k < H->n; k++) h = std::max(h, std::fabs(wv[o + k]));
        H->hnorm = h > 0.0 ? h : 1.0;
        o += H->n;
        live.push_back(H);
    }
    return ZK_OK;
}

int ApEngine::Impl::round(std::vector<ApDone> &finished)
{
    // one group per number of input limbs (the residual kernel is specialised
    // on it); matrices of different orders share every launch
    std::vector<std::vector<HostProb *>> groups;
    for (HostProb *H : live) {
        bool placed = false;
        for (auto &g : groups)
            if (g[0]->limbs_in == H->limbs_in) {
                g.push_back(H);
                placed = true;
                break;
            }
        if (!placed) groups.push_back(std::vector<HostProb *>(1, H));
    }
    for (auto &g : groups) {
        int rc = iterate(g, finished);
        if (rc != ZK_OK) return rc;
    }
    std::vector<HostProb *> keep;
    for (HostProb *H : live) {
        if (H->fin) release(H);
        else keep.push_back(H);
    }
    live = keep;
    return ZK_OK;
}

// one whole-basis iteration for matrices of equal input limbs (any orders):
// grids are sized for the largest order, each block reads its matrix's order
int ApEngine::Impl::iterate(std::vector<HostProb *> &grp, std::vector<ApDone> &finished)
{
    hipStream_t st = ctx->stream;
    int n = 0;   // the largest order of the group
    for (HostProb *H : grp) n = std::max(n, H->n);
    const size_t nn = (size_t)n * n;
    const int count = (int)grp.size();
    int rc;
    const size_t meta_need = al256(sizeof(ApProb) * count) + al256(sizeof(DdGemm) * count) + al256(sizeof(GemmDesc) * count) +
                             al256(sizeof(RotBlk) * (size_t)count * n) + al256(sizeof(ApOut) * count) +
                             al256(4 * (size_t)count * n);
    if ((rc = ensure_meta(meta_need)) != ZK_OK) return rc;
    char *mb = (char *)meta;
    ApProb *d_probs = (ApProb *)mb;
    mb += al256(sizeof(ApProb) * count);
    DdGemm *d_gemm = (DdGemm *)mb;
    mb += al256(sizeof(DdGemm) * count);
    GemmDesc *d_zg = (GemmDesc *)mb;
    mb += al256(sizeof(GemmDesc) * count);
    RotBlk *d_rot = (RotBlk *)mb;
    mb += al256(sizeof(RotBlk) * (size_t)count * n);
    ApOut *d_out = (ApOut *)mb;
    mb += al256(sizeof(ApOut) * count);
    int *d_perm = (int *)mb;

    KernelTimer *T = ctx->tp();
    auto tb = [&](int cls, double w) { return T ? T->begin(cls, w, st) : -1; };
    auto te = [&](int id) {
        if (T) T->end(id, st);
    };
    // start the matrices that joined since the last round
    {
        std::vector<ApProb> fresh;
        for (HostProb *H : grp)
            if (!H->inited) fresh.push_back(H->d);
        if (!fresh.empty()) {
            APCHK(hipMemcpyAsync(d_probs, fresh.data(), sizeof(ApProb) * fresh.size(), hipMemcpyHostToDevice, st));
            const int id = tb(KC_AP_OTHER, 0.0);
            hipLaunchKernelGGL(k_ap_init, dim3(std::min<unsigned>(cdiv(nn, 256), 4096), (unsigned)fresh.size()), dim3(256),
                               0, st, d_probs);
            te(id);
            APLAUNCH();
            APCHK(hipStreamSynchronize(st));
            for (HostProb *H : grp) H->inited = true;
        }
    }
    std::vector<ApProb> act;
    for (HostProb *H : grp) act.push_back(H->d);
    APCHK(hipMemcpyAsync(d_probs, act.data(), sizeof(ApProb) * count, hipMemcpyHostToDevice, st));
    const int tilesR = (int)(cdiv(n, 64) * cdiv(n, 16));
    const int tilesG = (int)(cdiv(n, 64) * cdiv(n, 64));
    const int na = count;
    // residual matrix, column statistics, F, G, Rayleigh quotients, orthonormality
    {
        double wk = 0.0;
        for (int q = 0; q < na; q++) wk += (double)act[q].n * act[q].n * act[q].n;
        const int id = tb(KC_AP_RESID, wk);
        const int lin = grp[0]->limbs_in;
        if (lin == 1)
            hipLaunchKernelGGL(k_ap_resid<1>, dim3(tilesR, na), dim3(256), 0, st, d_probs);
        else if (lin == 2)
            hipLaunchKernelGGL(k_ap_resid<2>, dim3(tilesR, na), dim3(256), 0, st, d_probs);
        else
            hipLaunchKernelGGL(k_ap_resid<4>, dim3(tilesR, na), dim3(256), 0, st, d_probs);
        te(id);
        APLAUNCH();
    }
    {
        const int id = tb(KC_AP_OTHER, 0.0);
        hipLaunchKernelGGL(k_ap_colstats, dim3(n, na), dim3(256), 0, st, d_probs);
        te(id);
        APLAUNCH();
    }
    {
        // F = X_hi^H R: one launch per order (the GEMM takes one shape per launch)
        std::vector<GemmDesc> zg(na);
        std::vector<int> ords;
        for (int q = 0; q < na; q++)
            if (std::find(ords.begin(), ords.end(), act[q].n) == ords.end()) ords.push_back(act[q].n);
        int zo = 0;
        double fl = 0.0;
        std::vector<std::pair<int, int>> zr;   // (offset, count) per order
        for (int m : ords) {
            const int z0 = zo;
            for (int q = 0; q < na; q++)
                if (act[q].n == m) {
                    GemmDesc &Z = zg[zo++];
                    Z.A = (const double *)act[q].Xh;
                    Z.B = (const double *)act[q].R;
                    Z.C = (double *)act[q].F;
                    Z.lda = Z.ldb = Z.ldc = m;
                    Z.pad = 0;
                    fl += 8.0 * m * (double)m * m;
                }
            zr.push_back(std::make_pair(z0, zo - z0));
        }
        APCHK(hipMemcpyAsync(d_zg, zg.data(), sizeof(GemmDesc) * na, hipMemcpyHostToDevice, st));
        const int id = tb(KC_AP_FGEMM, fl);
        for (size_t k = 0; k < ords.size(); k++)
            if (zgemm_batched(d_zg + zr[k].first, zr[k].second, ords[k], ords[k], ords[k], 1, 0, st))
                return ctx->fail(ZK_EDEVICE, "binary64 GEMM launch failed");
        te(id);
        // G = X^H X in double-double, rounded to binary64 (its off-diagonal
        // entries are small, so the rounding is relative to their own size)
        std::vector<DdGemm> gd(na);
        double wk = 0.0;
        for (int q = 0; q < na; q++) {
            DdGemm &G = gd[q];
            std::memset(&G, 0, sizeof G);
            const int m = act[q].n;
            G.A = act[q].X;
            G.B = act[q].X;
            G.Cz = act[q].Gf;
            G.pa = G.pb = (size_t)m * m;
            G.lda = G.ldb = G.ldc = m;
            G.M = G.N = G.K = m;
            wk += (double)m * m * m;
        }
        APCHK(hipMemcpyAsync(d_gemm, gd.data(), sizeof(DdGemm) * na, hipMemcpyHostToDevice, st));
        const int id2 = tb(KC_AP_DDGEMM, wk);
        hipLaunchKernelGGL((k_ap_ddgemm<true, true, false>), dim3(tilesG, na), dim3(256), 0, st, d_gemm);
        te(id2);
        APLAUNCH();
        const int id3 = tb(KC_AP_OTHER, 0.0);
        hipLaunchKernelGGL(k_ap_theta, dim3(cdiv(n, 256), na), dim3(256), 0, st, d_probs);
        hipLaunchKernelGGL(k_ap_orth, dim3(n, na), dim3(256), 0, st, d_probs);
        te(id3);
        APLAUNCH();
        for (HostProb *H : grp) {
            const int m = H->n;
            H->theta.resize(2 * (size_t)m);
            H->rnorm.resize(m);
            H->orth.resize(m);
            APCHK(hipMemcpyAsync(H->theta.data(), H->d.theta, 16 * (size_t)m, hipMemcpyDeviceToHost, st));
            APCHK(hipMemcpyAsync(H->rnorm.data(), H->d.rnorm, 8 * (size_t)m, hipMemcpyDeviceToHost, st));
            APCHK(hipMemcpyAsync(H->orth.data(), H->d.orth, 8 * (size_t)m, hipMemcpyDeviceToHost, st));
        }
        APCHK(hipStreamSynchronize(st));   // zg, gd go out of scope; the statistics are on the host
    }
    // stopping rule
    std::vector<HostProb *> done, lv;
    for (HostProb *H : grp) {
        double rmax = 0.0, omax = 0.0;
        bool finite = true;
        for (int j = 0; j < H->n; j++) {
            rmax = std::max(rmax, H->rnorm[j]);
            omax = std::max(omax, H->orth[j]);
            if (!(H->rnorm[j] == H->rnorm[j]) || !(H->orth[j] == H->orth[j])) finite = false;
        }
        if (trace)
            std::fprintf(stderr, "[zk] all-pairs n=%d iteration %d: max resid %.3e, max orth %.3e%s\n", H->n, H->iters,
                         rmax / H->hnorm, omax, H->rotated_last ? " (after rotation)" : "");
        if (finite && rmax <= 0.5 * H->tol * H->hnorm && omax <= H->tol && !H->rotated_last) {
            H->converged = true;
            done.push_back(H);
        } else if (!finite || H->iters >= H->max_iter) {
            done.push_back(H);
        } else {
            lv.push_back(H);
        }
    }
    if (!done.empty() && (rc = output(done, finished)) != ZK_OK) return rc;
    if (lv.empty()) return ZK_OK;
    // the matrices that iterate: sorted positions, coupling, blocks
    act.clear();
    for (HostProb *H : lv) act.push_back(H->d);
    const int nl = (int)lv.size();
    for (HostProb *H : lv) {
        const int m = H->n;
        std::vector<int> order;
        ap_sorted_order(H->theta.data(), m, order);
        H->pos.resize(m);
        for (int k = 0; k < m; k++) H->pos[order[k]] = k;
        APCHK(hipMemcpyAsync(H->d.pos, H->pos.data(), 4 * (size_t)m, hipMemcpyHostToDevice, st));
        H->srt = order;
    }
    APCHK(hipMemcpyAsync(d_probs, act.data(), sizeof(ApProb) * nl, hipMemcpyHostToDevice, st));
    {
        const int id = tb(KC_AP_OTHER, 0.0);
        hipLaunchKernelGGL(k_ap_couple, dim3(n, nl), dim3(256), 0, st, d_probs, kApEta);
        te(id);
        APLAUNCH();
    }
    for (HostProb *H : lv) {
        H->reach.resize(H->n);
        APCHK(hipMemcpyAsync(H->reach.data(), H->d.reach, 4 * (size_t)H->n, hipMemcpyDeviceToHost, st));
    }
    APCHK(hipStreamSynchronize(st));
    std::vector<RotBlk> rots;
    std::vector<zk_herm> s1h;
    std::vector<double *> s1hf, s1w, s1V;
    std::vector<int *> s1f;
    int maxm = 1;
    for (int q = 0; q < nl; q++) {
        HostProb &H = *lv[q];
        const int n = H.n;   // this matrix's order (shadows the group's largest)
        const std::vector<int> &reach = H.reach;
        const std::vector<int> &srt = H.srt;
        std::vector<std::pair<int, int>> runs;   // [start, end) in sorted positions
        ap_runs(reach.data(), n, runs);
        H.blk.assign(n, -1);
        H.loc.assign(n, 0);
        H.bcol.clear();
        H.boff.clear();
        H.brot.clear();
        H.qoff.clear();
        int qo = 0, nb = 0, nblk_rot = 0;
        H.nrot_cols = 0;
        for (const auto &r : runs) {
            for (int p = r.first; p < r.second; p++) H.cluster[srt[p]] = r.first;
            const int m = r.second - r.first;
            if (m < 2) continue;
            double rm = 0.0;
            for (int p = r.first; p < r.second; p++) rm = std::max(rm, H.rnorm[srt[p]]);
            const bool rot = rm > 0.25 * H.tol * H.hnorm;
            H.boff.push_back((int)H.bcol.size());
            for (int p = r.first; p < r.second; p++) {
                H.blk[srt[p]] = nb;
                H.loc[srt[p]] = p - r.first;
                H.bcol.push_back(srt[p]);
            }
            H.brot.push_back(rot ? 1 : 0);
            H.qoff.push_back(rot ? qo : -1);
            if (rot) {
                RotBlk rb;
                rb.prob = q;
                rb.b = nb;
                rots.push_back(rb);
                zk_herm h;
                std::memset(&h, 0, sizeof h);
                h.n = m;
                h.lda = m;
                h.limbs = 1;
                h.plane[0] = H.d.T + qo;
                s1h.push_back(h);
                // binary64-stage outputs: eigenvectors into Q, eigenvalues into th (by slot)
                s1V.push_back((double *)(H.d.Q + qo));
                s1w.push_back(H.d.th + H.bcol.size() - m);
                s1hf.push_back(H.hf_s1 + 2 * (size_t)qo);
                s1f.push_back(H.flag_s1 + (nblk_rot++ % n));
                qo += m * m;
                H.nrot_cols += m;
                maxm = std::max(maxm, m);
            }
            nb++;
        }
        H.boff.push_back((int)H.bcol.size());
        H.d.nbc = (int)H.bcol.size();
        act[q].nbc = H.d.nbc;
        if (trace) {
            int mx = 0;
            for (size_t b = 0; b + 1 < H.boff.size(); b++) mx = std::max(mx, H.boff[b + 1] - H.boff[b]);
            std::fprintf(stderr, "[zk]   blocks %zu (largest %d, %d columns), rotated columns %d\n", H.brot.size(), mx,
                         H.d.nbc, H.nrot_cols);
        }
        APCHK(hipMemcpyAsync(H.d.blk, H.blk.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st));
        APCHK(hipMemcpyAsync(H.d.loc, H.loc.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st));
        if (!H.bcol.empty()) {
            APCHK(hipMemcpyAsync(H.d.bcol, H.bcol.data(), 4 * H.bcol.size(), hipMemcpyHostToDevice, st));
            APCHK(hipMemcpyAsync(H.d.brot, H.brot.data(), 4 * H.brot.size(), hipMemcpyHostToDevice, st));
            APCHK(hipMemcpyAsync(H.d.qoff, H.qoff.data(), 4 * H.qoff.size(), hipMemcpyHostToDevice, st));
        }
        APCHK(hipMemcpyAsync(H.d.boff, H.boff.data(), 4 * H.boff.size(), hipMemcpyHostToDevice, st));
    }
    APCHK(hipMemcpyAsync(d_probs, act.data(), sizeof(ApProb) * nl, hipMemcpyHostToDevice, st));
    APCHK(hipStreamSynchronize(st));   // the host tables stay untouched until the copies are done
    const int nrot = (int)rots.size();
    if (nrot > 0) {
        APCHK(hipMemcpyAsync(d_rot, rots.data(), sizeof(RotBlk) * nrot, hipMemcpyHostToDevice, st));
        const int id = tb(KC_AP_OTHER, 0.0);
        hipLaunchKernelGGL(k_ap_tbuild, dim3(cdiv((size_t)maxm * maxm, 256), nrot), dim3(256), 0, st, d_probs, d_rot);
        te(id);
        APLAUNCH();
        // binary64 eigendecomposition of every projected block
        if ((rc = run_stage1(ctx, nrot, s1h.data(), s1hf, s1w, s1V, s1f, std::vector<int>())) != ZK_OK) return rc;
        const int id2 = tb(KC_AP_OTHER, 0.0);
        hipLaunchKernelGGL(k_ap_fcols, dim3(cdiv(n, 256), maxm, nrot), dim3(256), 0, st, d_probs, d_rot, maxm);
        hipLaunchKernelGGL(k_ap_gq, dim3(cdiv((size_t)maxm * maxm, 256), nrot), dim3(256), 0, st, d_probs, d_rot);
        hipLaunchKernelGGL(k_ap_qhw, dim3(cdiv((size_t)maxm * maxm, 256), nrot), dim3(256), 0, st, d_probs, d_rot);
        te(id2);
        APLAUNCH();
    }
    {
        const int id = tb(KC_AP_OTHER, 0.0);
        hipLaunchKernelGGL(k_ap_ehat, dim3(cdiv(n, 256), n, nl), dim3(256), 0, st, d_probs);
        hipLaunchKernelGGL(k_ap_mbuild, dim3(cdiv(n, 256), n, nl), dim3(256), 0, st, d_probs);
        te(id);
        APLAUNCH();
    }
    // X <- X + X M
    {
        std::vector<DdGemm> gd(nl);
        double wk = 0.0;
        for (int q = 0; q < nl; q++) {
            DdGemm &G = gd[q];
            std::memset(&G, 0, sizeof G);
            const int m = act[q].n;
            G.A = act[q].X;
            G.B = (const double *)act[q].M;
            G.C0 = act[q].X;
            G.C = act[q].Xn;
            G.Cz = act[q].Xh;
            G.pa = G.pc = (size_t)m * m;
            G.lda = G.ldb = G.ldc = m;
            G.M = G.N = G.K = m;
            wk += (double)m * m * m;
        }
        APCHK(hipMemcpyAsync(d_gemm, gd.data(), sizeof(DdGemm) * nl, hipMemcpyHostToDevice, st));
        const int id = tb(KC_AP_DDGEMM, wk);
        hipLaunchKernelGGL((k_ap_ddgemm<false, false, true>), dim3(tilesG, nl), dim3(256), 0, st, d_gemm);
        te(id);
        APLAUNCH();
        const int id2 = tb(KC_AP_OTHER, 0.0);
        hipLaunchKernelGGL(k_ap_lamset, dim3(cdiv(n, 256), nl), dim3(256), 0, st, d_probs);
        te(id2);
        APLAUNCH();
        APCHK(hipStreamSynchronize(st));   // gd goes out of scope
    }
    for (HostProb *H : lv) {
        std::swap(H->d.X, H->d.Xn);
        H->rotated_last = H->nrot_cols > 0;
        H->iters++;
    }
    return ZK_OK;
}

// sorted outputs and per-pair information of the matrices that stop
int ApEngine::Impl::output(std::vector<HostProb *> &done, std::vector<ApDone> &finished)
{
    hipStream_t st = ctx->stream;
    const int count = (int)done.size();
    int n = 0;   // the largest order (permutation rows are n apart)
    for (HostProb *H : done) n = std::max(n, H->n);
    char *mb = (char *)meta;
    ApProb *d_probs = (ApProb *)mb;   // rewritten below (the round's launches that used it are enqueued before)
    mb += al256(sizeof(ApProb) * count);
    (void)mb;
    // the output descriptors go after the round's other tables (sized for the group)
    const size_t off_out = meta_bytes - al256(sizeof(ApOut) * count) - al256(4 * (size_t)count * n);
    ApOut *d_out = (ApOut *)((char *)meta + off_out);
    int *d_perm = (int *)((char *)meta + off_out + al256(sizeof(ApOut) * count));
    std::vector<ApProb> all(count);
    std::vector<ApOut> ao(count);
    std::vector<int> perm_all((size_t)count * n);
    for (int p = 0; p < count; p++) {
        HostProb &H = *done[p];
        const int m = H.n;
        all[p] = H.d;
        std::vector<int> ord;
        ap_sorted_order(H.theta.data(), m, ord);
        std::memcpy(&perm_all[(size_t)p * n], ord.data(), 4 * (size_t)m);
        ApOut &O = ao[p];
        std::memset(&O, 0, sizeof O);
        O.w[0] = H.out.w[0];
        O.w[1] = H.out.w[1];
        O.v[0] = H.want_vectors ? (double2 *)H.out.v[0] : nullptr;
        O.v[1] = H.want_vectors ? (double2 *)H.out.v[1] : nullptr;
        O.ldv = H.out.ldv;
        O.perm = d_perm + (size_t)p * n;
        bool all_ok = true;
        for (int k = 0; k < m; k++) {
            const int j = ord[k];
            const double r = H.rnorm[j] / H.hnorm;
            const bool ok = (r == r) && H.rnorm[j] <= H.tol * H.hnorm;
            all_ok = all_ok && ok;
            if (H.out.info) {
                zk_pair_info &I = H.out.info[k];
                I.iters = H.iters;
                I.flags = ok ? ZK_PAIR_CONVERGED : 0;
                I.cluster = H.cluster[j] >= 0 ? H.cluster[j] : k;
                I.reserved = 0;
                I.resid = r;
            }
        }
        ApDone d;
        d.cookie = H.cookie;
        d.status = (all_ok && H.converged) ? ZK_OK : ZK_ENOCONV;
        H.fin = true;
        d.iters = H.iters;
        finished.push_back(d);
    }
    APCHK(hipStreamSynchronize(st));   // earlier launches of the round read the descriptor area
    APCHK(hipMemcpyAsync(d_perm, perm_all.data(), 4 * perm_all.size(), hipMemcpyHostToDevice, st));
    APCHK(hipMemcpyAsync(d_probs, all.data(), sizeof(ApProb) * count, hipMemcpyHostToDevice, st));
    APCHK(hipMemcpyAsync(d_out, ao.data(), sizeof(ApOut) * count, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_ap_output, dim3(cdiv(n, 256), n, count), dim3(256), 0, st, d_probs, d_out);
    APLAUNCH();
    APCHK(hipStreamSynchronize(st));
    return ZK_OK;
}

// device bytes the engine holds for one matrix of order n
size_t ap_bytes(int n)
{
    const size_t nn = (size_t)n * n;
    return ap_matrix_bytes(n) + al256(16 * nn) + al256(8 * (size_t)n) + al256(4 * (size_t)n);
}

// Synchronous use: `count` matrices whose binary64 stage is done (hf, w0, V0
// as produced by run_stage1), refined until every one has stopped.  Returns
// ZK_OK, ZK_ENOCONV or an error status.
int allpairs_run(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out *out, double tol, int max_iter, int want_vectors,
                 const std::vector<double *> &hf, const std::vector<double *> &w0, const std::vector<double *> &V0,
                 int *iters_used)
{
    ApEngine eng(ctx);
    std::vector<ApReq> reqs(count);
    for (int p = 0; p < count; p++) {
        ApReq &r = reqs[p];
        r.A = A[p];
        r.out = out[p];
        r.hf = hf[p];
        r.w0 = w0[p];
        r.V0 = V0[p];
        r.tol = tol;
        r.max_iter = max_iter;
        r.want_vectors = want_vectors;
        r.cookie = (void *)(size_t)(p + 1);
    }
    int rc = eng.add(reqs);
    if (rc != ZK_OK) return rc;
    while (eng.any_live())
        if ((rc = eng.round()) != ZK_OK) return rc;
    int status = ZK_OK;
    for (const ApDone &d : eng.finished) {
        if (d.status != ZK_OK) status = ZK_ENOCONV;
        if (iters_used) iters_used[(size_t)d.cookie - 1] = d.iters;
    }
    return status;
}

}  // namespace zk
