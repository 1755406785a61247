// Precision beyond double-double: whole-basis polishing of a double-double
// eigendecomposition to L binary64 limbs (L = 4: quad-double, about 212 bits;
// L = 8: about 424 bits; L = 16: about 848 bits).
//
// The paper resolves eigenvalues far below binary64 (Schmidt coefficients of
// order 2^((1-n)/2), Sec. 1 and its footnote 1) and runs its multiple-
// precision diagonalisations at up to 768 bits (Sec. 2.1, Fig. 1).  Here the
// eigenpairs of the double-double all-pairs refinement are the start, and
// each iteration on the basis X (L limbs) with shifts lam (L limbs) is
//   R = H X - X diag(lam)      exact products, L-level cascaded sums; binary64
//   F = X_hi^H R               binary64 (FP64-MFMA GEMM)
//   G = X^H X - I              L-level cascaded sums; binary64
//   theta_j = lam_j + Re f_jj / (1 + g_jj)       (L limbs)
//   E_ij = N_ij / (theta_j - theta_i) - g_ij / 2,  N = (F' + F'^H) / 2,
//          F'_ij = f_ij - (theta_j - lam_j) g_ij   (separated pairs)
//   E_ij = -g_ij / 2                               (coupled pairs: |N_ij| > eta gap, or gap 0)
//   E_jj = -g_jj / 2
//   X <- X + X E   (L-level cascaded sums),  lam <- theta
// i.e. the first-order correction of Ogita and Aishima's refinement of
// symmetric eigendecompositions (Japan J. Indust. Appl. Math. 35, 2018) in its
// Hermitian form.  E + E^H = -G to first order whatever the rounding of F, so
// orthonormality is restored at every step; the residual falls by about the
// binary64 unit per iteration, since F is formed from R rounded to binary64.
// Pairs coupled beyond first order form blocks (connected runs of the sorted
// Rayleigh quotients); a block holding a coupling between different
// eigenvalues is rotated by the binary64 eigenvectors Q_J of its projected
// matrix X_J^H H X_J - mu I (mu its first shift), computed by the binary64
// stage itself at the block's own scale: X <- X ((I + E_c) Q_bd), where E_c
// holds the first-order corrections between blocks and -G/2 inside them.
// Eigenvalues that binary64 cannot separate relative to ||H|| are so
// separated relative to their block's scale, and the next iteration treats
// them as separated pairs.
// Pairs whose residuals are both within half the tolerance take -G/2 only:
// what coupling is left between them is the rounding of their residuals, and a
// first-order rotation by it would cost orthonormality at second order,
// (residual / gap)^2, which for the tiny gaps of a geometric spectrum tail
// sits above the tolerance.
// The iteration runs on 2^s H with ||2^s H|| in [1, 2) (exact scaling), so
// residuals at the tolerance stay inside the binary64 range, and column norms
// are formed from scaled squares for the same reason.
// The iteration stops when every residual is within half the tolerance and
// the departure from orthonormality within the tolerance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/zk.h"
#include "api_internal.h"
#include "common.h"
#include "stage.h"

int run_stage1(zk_ctx *ctx, int count, const zk_herm *A, const std::vector<double *> &hf, const std::vector<double *> &w0,
               const std::vector<double *> &V0, const std::vector<int *> &flag, const std::vector<int> &fp32);

namespace zk {

int zgemm_batched(const GemmDesc *d_descs, int count, int M, int N, int K, int opA, int opB, hipStream_t st);

namespace {

constexpr double kMpEta = 1e-4;   // largest first-order correction taken for a pair
constexpr int kMpKR = 8;          // k-chunk of the tiled products
constexpr double kMpRotMargin = 1e8;   // block spread needed over the noise of its projected matrix

// One matrix (device pointers; n x n column-major, leading dimension n).
// L-limb matrices: 2L planes, plane c * L + l holds limb l of the real (c = 0)
// or imaginary (c = 1) part.  L-limb vectors: limb l of entry j at l * n + j.
struct MpProb {
    int n, limbs_in, pad0, pad1;
    const double *hf;           // 2 limbs_in planes: re and im of each input limb (full Hermitian)
    const double *w_dd;         // double-double start: eigenvalue limbs (2 x n)
    const double2 *v_dd[2];     // double-double start: eigenvector limb planes (complex128)
    double *X, *Xn;             // basis and the next basis
    double2 *Xh;                // leading limbs of X, interleaved
    double2 *R, *F, *Gm, *E;    // residual matrix, X_hi^H R, X^H X - I, correction
    double *lam, *theta;        // L x n
    double *q;                  // theta - lam (binary64)
    double *rnorm, *orth;       // per column
    double *stat;               // [0] max residual, [1] max departure from orthonormality
    const int *perm;            // output order (ascending theta)
    int *reach;                 // per column j: the smallest i coupled to j (j itself if none)
    int *rot;                   // per column j: 1 if j is coupled to a pair of a different eigenvalue
    int *blk, *boff;            // block of each column; first column of each block (nblk + 1 entries)
    int *brot;                  // per block: 1 if rotated this iteration
    double2 *Q;                 // per rotated block b: its m x m eigenvectors at Q + qoff[b]
    int *qoff;
    double *tw;                 // per rotated block: its m eigenvalues at tw + boff[b]
    double2 *E2;                // correction with the block rotations
    double *w_out;              // caller: limbs x n
    double2 *v_out;             // caller: limbs planes of ldv x n complex128, or null
    int ldv, pad2;
    double thr;                 // residual a converged pair is at (half the tolerance, absolute)
    double sc;                  // power of two the iteration scales H by (||H|| sc in [1, 2))
};

template <int L>
__global__ void __launch_bounds__(256) k_mp_init(const MpProb *pp)
{
    const MpProb &P = pp[blockIdx.y];
    const int n = P.n;
    const size_t nn = (size_t)n * n;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (size_t)gridDim.x * 256) {
        const double2 a = P.v_dd[0][e], b = P.v_dd[1][e];
        P.X[0 * nn + e] = a.x;
        P.X[1 * nn + e] = b.x;
        P.X[(size_t)L * nn + e] = a.y;
        P.X[(size_t)(L + 1) * nn + e] = b.y;
#pragma unroll
        for (int l = 2; l < L; l++) {
            P.X[(size_t)l * nn + e] = 0.0;
            P.X[(size_t)(L + l) * nn + e] = 0.0;
        }
        P.Xh[e] = a;
        if (e < (size_t)n) {
            P.lam[e] = P.w_dd[e] * P.sc;
            P.lam[n + e] = P.w_dd[n + e] * P.sc;
#pragma unroll
            for (int l = 2; l < L; l++) P.lam[(size_t)l * n + e] = 0.0;
        }
    }
}

// rows per thread of the tiled kernels: enough registers for the L-level accumulators
template <int L>
struct MpTile {
    static constexpr int OUT = L <= 4 ? 4 : (L <= 8 ? 2 : 1);
    static constexpr int ROWS = 16 * OUT;
};

// R = H X - X diag(lam) (tiles of ROWS x 16, OUT rows per thread)
template <int L, int LIN>
__global__ void __launch_bounds__(256) k_mp_resid(const MpProb *pp)
{
    constexpr int OUT = MpTile<L>::OUT, ROWS = MpTile<L>::ROWS;
    const MpProb &P = pp[blockIdx.y];
    const int n = P.n;
    const int tilesI = (n + ROWS - 1) / ROWS;
    const int ti = blockIdx.x % tilesI, tj = blockIdx.x / tilesI;
    if (tj * 16 >= n) return;
    const int i0 = ti * ROWS, j0 = tj * 16;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const size_t nn = (size_t)n * n;
    __shared__ double sH[2 * LIN][kMpKR][ROWS];
    __shared__ double sX[2 * L][kMpKR][17];
    CascN<L> re[OUT], im[OUT];
#pragma unroll
    for (int a = 0; a < OUT; a++) {
        re[a].zero();
        im[a].zero();
    }
    for (int k0 = 0; k0 < n; k0 += kMpKR) {
        __syncthreads();
        for (int e = tid; e < ROWS * kMpKR; e += 256) {
            const int ii = e % ROWS, kk = e / ROWS;
            const int gi = i0 + ii, gk = k0 + kk;
            const bool ok = gi < n && gk < n;
#pragma unroll
            for (int pl = 0; pl < 2 * LIN; pl++) sH[pl][kk][ii] = ok ? P.hf[pl * nn + (size_t)gk * n + gi] * P.sc : 0.0;
        }
        for (int e = tid; e < 16 * kMpKR; e += 256) {
            const int kk = e & (kMpKR - 1), jj = e / kMpKR;
            const int gk = k0 + kk, gj = j0 + jj;
            const bool ok = gk < n && gj < n;
#pragma unroll
            for (int pl = 0; pl < 2 * L; pl++) sX[pl][kk][jj] = ok ? P.X[pl * nn + (size_t)gj * n + gk] : 0.0;
        }
        __syncthreads();
        for (int kk = 0; kk < kMpKR; kk++) {
            double xr[L], xi[L];
#pragma unroll
            for (int l = 0; l < L; l++) {
                xr[l] = sX[l][kk][ty];
                xi[l] = sX[L + l][kk][ty];
            }
#pragma unroll
            for (int a = 0; a < OUT; a++) {
#pragma unroll
                for (int l = 0; l < LIN; l++) {
                    const double hr = sH[2 * l][kk][tx + 16 * a], hi = sH[2 * l + 1][kk][tx + 16 * a];
                    re[a].add(hr, xr, l);
                    re[a].add(-hi, xi, l);
                    im[a].add(hr, xi, l);
                    im[a].add(hi, xr, l);
                }
            }
        }
    }
    const int j = j0 + ty;
    if (j >= n) return;
    double nl[L];
#pragma unroll
    for (int l = 0; l < L; l++) nl[l] = -P.lam[(size_t)l * n + j];
#pragma unroll
    for (int a = 0; a < OUT; a++) {
        const int i = i0 + tx + 16 * a;
        if (i >= n) continue;
        const size_t o = (size_t)j * n + i;
        double xr[L], xi[L];
#pragma unroll
        for (int l = 0; l < L; l++) {
            xr[l] = P.X[(size_t)l * nn + o];
            xi[l] = P.X[(size_t)(L + l) * nn + o];
        }
        re[a].add_mm(nl, xr);
        im[a].add_mm(nl, xi);
        P.R[o] = make_double2(re[a].get().x[0], im[a].get().x[0]);
    }
}

// G = X^H X - I
template <int L>
__global__ void __launch_bounds__(256) k_mp_gram(const MpProb *pp)
{
    constexpr int OUT = MpTile<L>::OUT, ROWS = MpTile<L>::ROWS;
    const MpProb &P = pp[blockIdx.y];
    const int n = P.n;
    const int tilesI = (n + ROWS - 1) / ROWS;
    const int ti = blockIdx.x % tilesI, tj = blockIdx.x / tilesI;
    if (tj * 16 >= n) return;
    const int i0 = ti * ROWS, j0 = tj * 16;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const size_t nn = (size_t)n * n;
    __shared__ double sA[2 * L][kMpKR][ROWS];
    __shared__ double sB[2 * L][kMpKR][17];
    CascN<L> re[OUT], im[OUT];
#pragma unroll
    for (int a = 0; a < OUT; a++) {
        re[a].zero();
        im[a].zero();
    }
    for (int k0 = 0; k0 < n; k0 += kMpKR) {
        __syncthreads();
        for (int e = tid; e < ROWS * kMpKR; e += 256) {
            const int kk = e % kMpKR, ii = e / kMpKR;
            const int gi = i0 + ii, gk = k0 + kk;
            const bool ok = gi < n && gk < n;
#pragma unroll
            for (int pl = 0; pl < 2 * L; pl++) sA[pl][kk][ii] = ok ? P.X[pl * nn + (size_t)gi * n + gk] : 0.0;
        }
        for (int e = tid; e < 16 * kMpKR; e += 256) {
            const int kk = e % kMpKR, jj = e / kMpKR;
            const int gk = k0 + kk, gj = j0 + jj;
            const bool ok = gk < n && gj < n;
#pragma unroll
            for (int pl = 0; pl < 2 * L; pl++) sB[pl][kk][jj] = ok ? P.X[pl * nn + (size_t)gj * n + gk] : 0.0;
        }
        __syncthreads();
        for (int kk = 0; kk < kMpKR; kk++) {
            double br[L], bi[L];
#pragma unroll
            for (int l = 0; l < L; l++) {
                br[l] = sB[l][kk][ty];
                bi[l] = sB[L + l][kk][ty];
            }
#pragma unroll
            for (int a = 0; a < OUT; a++) {
                double ar[L], ai[L], nai[L];
#pragma unroll
                for (int l = 0; l < L; l++) {
                    ar[l] = sA[l][kk][tx + 16 * a];
                    ai[l] = sA[L + l][kk][tx + 16 * a];
                    nai[l] = -ai[l];
                }
                // conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
                re[a].add_mm(ar, br);
                re[a].add_mm(ai, bi);
                im[a].add_mm(ar, bi);
                im[a].add_mm(nai, br);
            }
        }
    }
    const int j = j0 + ty;
    if (j >= n) return;
#pragma unroll
    for (int a = 0; a < OUT; a++) {
        const int i = i0 + tx + 16 * a;
        if (i >= n) continue;
        if (i == j) re[a].put(0, -1.0);
        P.Gm[(size_t)j * n + i] = make_double2(re[a].get().x[0], im[a].get().x[0]);
    }
}

// per column j: ||r_j||, max_i |g_ij| (diagonal included), theta_j and q_j
template <int L>
__global__ void __launch_bounds__(256) k_mp_colstat(const MpProb *pp)
{
    const MpProb &P = pp[blockIdx.y];
    const int n = P.n, j = blockIdx.x;
    if (j >= n) return;
    // ||r_j|| as 2^e sqrt(sum (2^-e r_ij)^2) with 2^e near max |r_ij|: residuals
    // far below the square root of the smallest binary64 (about 1e-154) are
    // the normal case beyond quad-double, and their squares would vanish
    double rm = 0.0, go = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double2 r = P.R[(size_t)j * n + i];
        const double2 g = P.Gm[(size_t)j * n + i];
        rm = fmax(rm, fmax(fabs(r.x), fabs(r.y)));
        go = fmax(go, fabs(g.x) + fabs(g.y));
    }
    __shared__ double red[2][4];
    __shared__ int s_e;
    for (int off = 32; off > 0; off >>= 1) {
        rm = fmax(rm, __shfl_xor(rm, off, 64));
        go = fmax(go, __shfl_xor(go, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = rm;
        red[1][threadIdx.x >> 6] = go;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double m = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
        s_e = m > 0.0 ? ilogb(m) : 0;
    }
    __syncthreads();
    const int ex = s_e;
    double r2 = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double2 r = P.R[(size_t)j * n + i];
        const double a = ldexp(r.x, -ex), b = ldexp(r.y, -ex);
        r2 += a * a + b * b;
    }
    for (int off = 32; off > 0; off >>= 1) r2 += __shfl_xor(r2, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[0][threadIdx.x >> 6] = r2;
    __syncthreads();
    if (threadIdx.x == 0) {
        P.rnorm[j] = ldexp(sqrt((red[0][0] + red[0][1]) + (red[0][2] + red[0][3])), ex);
        P.orth[j] = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
        const double q = P.F[(size_t)j * n + j].x / (1.0 + P.Gm[(size_t)j * n + j].x);
        mp<L> lam;
#pragma unroll
        for (int l = 0; l < L; l++) lam.x[l] = P.lam[(size_t)l * n + j];
        const mp<L> th = add_n_d<L>(lam, q);
#pragma unroll
        for (int l = 0; l < L; l++) P.theta[(size_t)l * n + j] = th.x[l];
        P.q[j] = q;
    }
}

// per matrix: the largest residual and departure from orthonormality
__global__ void __launch_bounds__(256) k_mp_maxstat(const MpProb *pp)
{
    const MpProb &P = pp[blockIdx.x];
    double r = 0.0, o = 0.0;
    for (int j = threadIdx.x; j < P.n; j += 256) {
        r = fmax(r, P.rnorm[j]);
        o = fmax(o, P.orth[j]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        r = fmax(r, __shfl_xor(r, off, 64));
        o = fmax(o, __shfl_xor(o, off, 64));
    }
    __shared__ double red[2][4];
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = r;
        red[1][threadIdx.x >> 6] = o;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        P.stat[0] = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
        P.stat[1] = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
    }
}

// theta_j - theta_i to binary64 (the limbs of two normalised expansions)
template <int L>
__device__ __forceinline__ double mp_gap(const double *th, int n, int j, int i)
{
    double s = 0.0, c = 0.0;
#pragma unroll
    for (int l = 0; l < L; l++) {
        double d, e;
        two_sum(th[(size_t)l * n + j], -th[(size_t)l * n + i], d, e);
        double t, f;
        two_sum(s, d, t, f);
        s = t;
        c += f + e;
    }
    return s + c;
}

// N_ij = (F'_ij + conj(F'_ji)) / 2 with F'_ij = f_ij - q_j g_ij
__device__ __forceinline__ double2 mp_nsym(const MpProb &P, int n, int i, int j)
{
    const double2 gij = P.Gm[(size_t)j * n + i], gji = P.Gm[(size_t)i * n + j];
    const double2 fij = P.F[(size_t)j * n + i], fji = P.F[(size_t)i * n + j];
    const double qj = P.q[j], qi = P.q[i];
    const double2 a = make_double2(fij.x - qj * gij.x, fij.y - qj * gij.y);
    const double2 b = make_double2(fji.x - qi * gji.x, -(fji.y - qi * gji.y));
    return make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
}

// reach[j] = smallest i coupled to j (|N_ij| > eta |gap| or gap 0), rot[j] = 1
// if j is coupled to a pair of a different eigenvalue; one block per column
template <int L>
__global__ void __launch_bounds__(256) k_mp_couple(const MpProb *pp, double eta)
{
    const MpProb &P = pp[blockIdx.y];
    const int n = P.n, j = blockIdx.x;
    if (j >= n) return;
    int best = j, rt = 0;
    for (int i = threadIdx.x; i < n; i += 256) {
        if (i == j) continue;
        const double2 N = mp_nsym(P, n, i, j);
        const double gap = mp_gap<L>(P.theta, n, j, i);
        const double mag = fabs(N.x) + fabs(N.y);
        if (gap == 0.0 || mag > eta * fabs(gap)) {
            best = min(best, i);
            if (gap != 0.0) rt = 1;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        best = min(best, __shfl_xor(best, off, 64));
        rt = max(rt, __shfl_xor(rt, off, 64));
    }
    __shared__ int red[2][4];
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = best;
        red[1][threadIdx.x >> 6] = rt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        P.reach[j] = min(min(red[0][0], red[0][1]), min(red[0][2], red[0][3]));
        P.rot[j] = max(max(red[1][0], red[1][1]), max(red[1][2], red[1][3]));
    }
}

// projected matrix of a rotated block, Hermitian part, at the block's scale:
// T(a, c) = F_ac + lam_c Gm_ac + (lam_c - mu) delta_ac, mu = lam of the first member
struct MpBlk {
    int prob, b;
};

template <int L>
__global__ void __launch_bounds__(256) k_mp_tbuild(const MpProb *pp, const MpBlk *rb, double2 *const *tout)
{
    const MpBlk B = rb[blockIdx.y];
    const MpProb &P = pp[B.prob];
    const int n = P.n, o = P.boff[B.b], m = P.boff[B.b + 1] - o;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= m * m) return;
    const int a = e % m, c = e / m;
    const int ja = o + a, jc = o + c;
    auto entry = [&](int x, int y) {   // T(x, y), x, y block-local
        const int jx = o + x, jy = o + y;
        const double2 f = P.F[(size_t)jy * n + jx], g = P.Gm[(size_t)jy * n + jx];
        const double ly = P.lam[jy];
        double2 t = make_double2(f.x + ly * g.x, f.y + ly * g.y);
        if (x == y) t.x += mp_gap<L>(P.lam, n, jy, o);
        return t;
    };
    (void)ja;
    (void)jc;
    const double2 t1 = entry(a, c), t2 = entry(c, a);
    // Hermitian part, column-major complex128 (the input of the binary64 stage)
    tout[blockIdx.y][(size_t)c * m + a] = make_double2(0.5 * (t1.x + t2.x), a == c ? 0.0 : 0.5 * (t1.y - t2.y));
}

template <int L>
__global__ void __launch_bounds__(256) k_mp_corr(const MpProb *pp, double eta)
{
    const MpProb &P = pp[blockIdx.y];
    const int n = P.n;
    const size_t nn = (size_t)n * n;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (size_t)gridDim.x * 256) {
        const int i = (int)(e % n), j = (int)(e / n);
        const double2 gij = P.Gm[e];
        double2 out;
        if (i == j) {
            out = make_double2(-0.5 * gij.x, 0.0);
        } else {
            const double2 N = mp_nsym(P, n, i, j);
            const double gap = mp_gap<L>(P.theta, n, j, i);
            const double mag = fabs(N.x) + fabs(N.y);
            // inside a block (and for any pair too close for first order): -G/2
            // only; between two converged pairs too, since the coupling left
            // there is the rounding of the residuals, and rotating by it would
            // cost orthonormality at second order ((residual / gap)^2)
            const bool settled = P.rnorm[i] <= P.thr && P.rnorm[j] <= P.thr;
            if (settled || P.blk[i] == P.blk[j] || gap == 0.0 || mag > eta * fabs(gap))
                out = make_double2(-0.5 * gij.x, -0.5 * gij.y);
            else
                out = make_double2(N.x / gap - 0.5 * gij.x, N.y / gap - 0.5 * gij.y);
        }
        P.E[e] = out;
    }
}

// E2 = (I + E) Q_bd - I, Q_bd the block-diagonal rotation (identity outside
// the rotated blocks)
__global__ void __launch_bounds__(256) k_mp_rot(const MpProb *pp)
{
    const MpProb &P = pp[blockIdx.y];
    const int n = P.n;
    const size_t nn = (size_t)n * n;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (size_t)gridDim.x * 256) {
        const int k = (int)(e % n), j = (int)(e / n);
        const int b = P.blk[j];
        if (!P.brot[b]) {
            P.E2[e] = P.E[e];
            continue;
        }
        const int o = P.boff[b], m = P.boff[b + 1] - o, c = j - o;
        const double2 *Q = P.Q + P.qoff[b];
        double re = 0.0, im = 0.0;
        for (int a = 0; a < m; a++) {
            double2 ea = P.E[(size_t)(o + a) * n + k];
            if (k == o + a) ea.x += 1.0;
            const double2 q = Q[(size_t)c * m + a];
            re += ea.x * q.x - ea.y * q.y;
            im += ea.x * q.y + ea.y * q.x;
        }
        if (k == j) re -= 1.0;
        P.E2[e] = make_double2(re, im);
    }
}

// shifts of the rotated blocks' members: mu + their projected eigenvalues
// (one thread per block)
template <int L>
__global__ void __launch_bounds__(64) k_mp_lamrot(const MpProb *pp, const MpBlk *rb, int nrb)
{
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t >= nrb) return;
    const MpBlk B = rb[t];
    const MpProb &P = pp[B.prob];
    const int n = P.n, o = P.boff[B.b], m = P.boff[B.b + 1] - o;
    mp<L> mu;
#pragma unroll
    for (int l = 0; l < L; l++) mu.x[l] = P.lam[(size_t)l * n + o];
    for (int a = 0; a < m; a++) {
        const mp<L> v = add_n_d<L>(mu, P.tw[o + a]);
#pragma unroll
        for (int l = 0; l < L; l++) P.theta[(size_t)l * n + o + a] = v.x[l];
    }
}

// Xn = X + X E, and the leading limbs of Xn
template <int L>
__global__ void __launch_bounds__(256) k_mp_update(const MpProb *pp)
{
    constexpr int OUT = MpTile<L>::OUT, ROWS = MpTile<L>::ROWS;
    const MpProb &P = pp[blockIdx.y];
    const int n = P.n;
    const int tilesI = (n + ROWS - 1) / ROWS;
    const int ti = blockIdx.x % tilesI, tj = blockIdx.x / tilesI;
    if (tj * 16 >= n) return;
    const int i0 = ti * ROWS, j0 = tj * 16;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const size_t nn = (size_t)n * n;
    __shared__ double sX[2 * L][kMpKR][ROWS];
    __shared__ double2 sE[kMpKR][17];
    const int j = j0 + ty;
    CascN<L> re[OUT], im[OUT];
#pragma unroll
    for (int a = 0; a < OUT; a++) {
        re[a].zero();
        im[a].zero();
        const int i = i0 + tx + 16 * a;
        if (i < n && j < n) {
            const size_t o = (size_t)j * n + i;
#pragma unroll
            for (int l = 0; l < L; l++) {
                re[a].put(l, P.X[(size_t)l * nn + o]);
                im[a].put(l, P.X[(size_t)(L + l) * nn + o]);
            }
        }
    }
    for (int k0 = 0; k0 < n; k0 += kMpKR) {
        __syncthreads();
        for (int e = tid; e < ROWS * kMpKR; e += 256) {
            const int ii = e % ROWS, kk = e / ROWS;
            const int gi = i0 + ii, gk = k0 + kk;
            const bool ok = gi < n && gk < n;
#pragma unroll
            for (int pl = 0; pl < 2 * L; pl++) sX[pl][kk][ii] = ok ? P.X[pl * nn + (size_t)gk * n + gi] : 0.0;
        }
        for (int e = tid; e < 16 * kMpKR; e += 256) {
            const int kk = e % kMpKR, jj = e / kMpKR;
            const int gk = k0 + kk, gj = j0 + jj;
            sE[kk][jj] = (gk < n && gj < n) ? P.E2[(size_t)gj * n + gk] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int kk = 0; kk < kMpKR; kk++) {
            const double2 ek = sE[kk][ty];
#pragma unroll
            for (int a = 0; a < OUT; a++) {
                double xr[L], xi[L];
#pragma unroll
                for (int l = 0; l < L; l++) {
                    xr[l] = sX[l][kk][tx + 16 * a];
                    xi[l] = sX[L + l][kk][tx + 16 * a];
                }
                re[a].add(ek.x, xr, 0);
                re[a].add(-ek.y, xi, 0);
                im[a].add(ek.y, xr, 0);
                im[a].add(ek.x, xi, 0);
            }
        }
    }
    if (j >= n) return;
#pragma unroll
    for (int a = 0; a < OUT; a++) {
        const int i = i0 + tx + 16 * a;
        if (i >= n) continue;
        const size_t o = (size_t)j * n + i;
        const mp<L> r = re[a].get(), m = im[a].get();
#pragma unroll
        for (int l = 0; l < L; l++) {
            P.Xn[(size_t)l * nn + o] = r.x[l];
            P.Xn[(size_t)(L + l) * nn + o] = m.x[l];
        }
        P.Xh[o] = make_double2(r.x[0], m.x[0]);
    }
}

// lam <- theta
template <int L>
__global__ void __launch_bounds__(256) k_mp_lamset(const MpProb *pp)
{
    const MpProb &P = pp[blockIdx.y];
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= P.n) return;
#pragma unroll
    for (int l = 0; l < L; l++) P.lam[(size_t)l * P.n + j] = P.theta[(size_t)l * P.n + j];
}

// outputs in ascending order of theta: eigenvalue limbs and eigenvector limb planes
template <int L>
__global__ void __launch_bounds__(256) k_mp_output(const MpProb *pp)
{
    const MpProb &P = pp[blockIdx.y];
    const int n = P.n;
    const size_t nn = (size_t)n * n;
    const double isc = 1.0 / P.sc;   // exact: a power of two within the normal range
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (size_t)gridDim.x * 256) {
        const int i = (int)(e % n), k = (int)(e / n);
        const int src = P.perm[k];
        if (i == 0) {
#pragma unroll
            for (int l = 0; l < L; l++) P.w_out[(size_t)l * n + k] = P.theta[(size_t)l * n + src] * isc;
        }
        if (P.v_out) {
            const size_t o = (size_t)src * n + i;
#pragma unroll
            for (int l = 0; l < L; l++)
                P.v_out[(size_t)l * P.ldv * n + (size_t)k * P.ldv + i] =
                    make_double2(P.X[(size_t)l * nn + o], P.X[(size_t)(L + l) * nn + o]);
        }
    }
}

inline unsigned cdivu(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

template <int L>
int launch_resid(const MpProb *d, int np, int n, int limbs_in, hipStream_t st)
{
    constexpr int ROWS = MpTile<L>::ROWS;
    const dim3 grid(cdivu(n, ROWS) * cdivu(n, 16), np);
    if (limbs_in == 1) hipLaunchKernelGGL((k_mp_resid<L, 1>), grid, dim3(256), 0, st, d);
    else if (limbs_in == 2) hipLaunchKernelGGL((k_mp_resid<L, 2>), grid, dim3(256), 0, st, d);
    else hipLaunchKernelGGL((k_mp_resid<L, 4>), grid, dim3(256), 0, st, d);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t mp_polish_bytes(int n, int L)
{
    const size_t nn = (size_t)n * n;
    return 2 * al256(8 * 2 * (size_t)L * nn) + 5 * al256(16 * nn) + 2 * al256(8 * (size_t)L * n) + 3 * al256(8 * (size_t)n) +
           al256(4 * (size_t)n) + al256(64) + al256(sizeof(GemmDesc)) + al256(sizeof(MpProb)) +
           // blocks: reach, rot, blk, boff, brot, qoff, flags; Q, T, the binary64 stage's copy, E2; tw
           7 * al256(4 * ((size_t)n + 1)) + 3 * al256(16 * nn) + al256(16 * nn) + al256(8 * (size_t)n) +
           al256(sizeof(MpBlk) * (size_t)n) + 2 * al256(sizeof(void *) * (size_t)n);
}

// Polish `np` matrices of equal order n from their double-double eigenpairs
// (w_dd: 2 x n limbs, v_dd: two complex128 limb planes, ld n; inputs hf as
// laid out by the stage-2 ingest) to L limbs.  Outputs w_out[p] (L x n) and
// v_out[p] (L planes, leading dimension ldv[p]; null: no vectors).  info[p]
// (host, may be null): iterations and final residual per pair.
template <int L>
int mp_polish_run(zk_ctx *ctx, int np, int n, const int *limbs_in, const double *const *hf,
                  const double *const *w_dd, const double2 *const *v_dd, double *const *w_out, double2 *const *v_out,
                  const int *ldv, zk_pair_info *const *info, double tol, int max_iter, int *iters_used)
{
    hipStream_t st = ctx->stream;
    const size_t nn = (size_t)n * n, per = mp_polish_bytes(n, L);
    const size_t total = per * np;
    if (!ctx->make_room(total)) return ctx->fail(ZK_ENOMEM, "precision polishing needs %zu bytes", total);
    void *buf = nullptr;
    if (ctx->dev_alloc(&buf, total) != ZK_OK) return ZK_ENOMEM;
    ctx->extra += total;
    ctx->note_held();
    std::vector<MpProb> hp(np);
    std::vector<GemmDesc> hg(np);
    std::vector<int *> bflag(np);
    std::vector<double2 *> btin(np);
    std::vector<double *> bhf(np);
    std::vector<int> perm((size_t)n * np);
    char *b = (char *)buf;
    MpProb *d_probs = nullptr;
    GemmDesc *d_gemm = nullptr;
    int *d_perm = nullptr;
    double *d_stat = nullptr;
    for (int p = 0; p < np; p++) {
        MpProb &P = hp[p];
        std::memset(&P, 0, sizeof P);
        P.n = n;
        P.limbs_in = limbs_in[p];
        P.hf = hf[p];
        P.w_dd = w_dd[p];
        P.v_dd[0] = v_dd[2 * p];
        P.v_dd[1] = v_dd[2 * p + 1];
        P.X = (double *)b; b += al256(8 * 2 * (size_t)L * nn);
        P.Xn = (double *)b; b += al256(8 * 2 * (size_t)L * nn);
        P.Xh = (double2 *)b; b += al256(16 * nn);
        P.R = (double2 *)b; b += al256(16 * nn);
        P.F = (double2 *)b; b += al256(16 * nn);
        P.Gm = (double2 *)b; b += al256(16 * nn);
        P.E = (double2 *)b; b += al256(16 * nn);
        P.lam = (double *)b; b += al256(8 * (size_t)L * n);
        P.theta = (double *)b; b += al256(8 * (size_t)L * n);
        P.q = (double *)b; b += al256(8 * (size_t)n);
        P.rnorm = (double *)b; b += al256(8 * (size_t)n);
        P.orth = (double *)b; b += al256(8 * (size_t)n);
        P.stat = (double *)b; b += al256(64);
        P.reach = (int *)b; b += al256(4 * ((size_t)n + 1));
        P.rot = (int *)b; b += al256(4 * ((size_t)n + 1));
        P.blk = (int *)b; b += al256(4 * ((size_t)n + 1));
        P.boff = (int *)b; b += al256(4 * ((size_t)n + 1));
        P.brot = (int *)b; b += al256(4 * ((size_t)n + 1));
        P.qoff = (int *)b; b += al256(4 * ((size_t)n + 1));
        bflag[p] = (int *)b; b += al256(4 * ((size_t)n + 1));
        P.Q = (double2 *)b; b += al256(16 * nn);
        btin[p] = (double2 *)b; b += al256(16 * nn);
        bhf[p] = (double *)b; b += al256(16 * nn);
        P.E2 = (double2 *)b; b += al256(16 * nn);
        P.tw = (double *)b; b += al256(8 * (size_t)n);
        P.w_out = w_out[p];
        P.v_out = v_out[p];
        P.ldv = ldv[p];
        GemmDesc &g = hg[p];
        g.A = (const double *)P.Xh;
        g.B = (const double *)P.R;
        g.C = (double *)P.F;
        g.lda = g.ldb = g.ldc = n;
        g.pad = 0;
    }
    // descriptor tables after the per-matrix blocks
    d_gemm = (GemmDesc *)b; b += al256(sizeof(GemmDesc) * np);
    d_probs = (MpProb *)b; b += al256(sizeof(MpProb) * np);
    d_perm = (int *)b; b += al256(4 * (size_t)n * np);
    MpBlk *d_rb = (MpBlk *)b; b += al256(sizeof(MpBlk) * (size_t)n * np);
    double2 **d_tptr = (double2 **)b; b += al256(sizeof(void *) * (size_t)n * np);
    (void)d_stat;
    int rc = ZK_OK;
    auto done = [&](int r) {
        hipStreamSynchronize(st);
        ctx->dev_free(buf);
        ctx->extra -= total;
        return r;
    };
    // the limbs in-flight use per matrix: limbs_in may differ inside the batch
    std::vector<int> lin(limbs_in, limbs_in + np);
    std::vector<double> stat(2 * (size_t)np), hn(np, 1.0);
    // ||H||_2 from the double-double eigenvalues (ascending)
    for (int p = 0; p < np; p++) {
        double lo = 0.0, hi = 0.0;
        if (hipMemcpyAsync(&lo, w_dd[p], 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&hi, w_dd[p] + (n - 1), 8, hipMemcpyDeviceToHost, st) != hipSuccess)
            return done(ctx->fail(ZK_EDEVICE, "read-back failed"));
        hipStreamSynchronize(st);
        hn[p] = std::max(std::fabs(lo), std::fabs(hi));
        if (!(hn[p] > 0.0)) hn[p] = 1.0;
        // the iteration runs on sc H with ||sc H|| in [1, 2): residuals at the
        // tolerance stay inside the binary64 range whatever ||H|| is
        const int e = std::min(1000, std::max(-1000, std::ilogb(hn[p])));
        hp[p].sc = std::ldexp(1.0, -e);
        hn[p] *= hp[p].sc;
    }
    // (the descriptor tables were counted inside `per`: np copies of each)
    for (int p = 0; p < np; p++) hp[p].perm = d_perm + (size_t)p * n;
    if (hipMemcpyAsync(d_probs, hp.data(), sizeof(MpProb) * np, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d_gemm, hg.data(), sizeof(GemmDesc) * np, hipMemcpyHostToDevice, st) != hipSuccess)
        return done(ctx->fail(ZK_EDEVICE, "descriptor upload failed"));
    constexpr int ROWS = MpTile<L>::ROWS;
    const dim3 tiles(cdivu(n, ROWS) * cdivu(n, 16), np);
    const dim3 elems(std::min<unsigned>(cdivu(nn, 256), 4096u), np);
    hipLaunchKernelGGL(k_mp_init<L>, elems, dim3(256), 0, st, d_probs);
    // Blocks of coupled pairs: runs [b0, b1) of the sorted shifts that no
    // coupling crosses; a block with a coupling between different eigenvalues
    // and a member above the tolerance is rotated by its projected matrix's
    // binary64 eigenvectors (the binary64 stage on all such blocks at once).
    std::vector<int> reach(n), rotf(n), blk(n), boff, brot, qoff;
    std::vector<double> rn(n), th2(2 * (size_t)n);
    std::vector<MpBlk> rb;
    std::vector<double2 *> tptr;
    auto plan_blocks = [&]() -> int {
        hipLaunchKernelGGL(k_mp_couple<L>, dim3(n, np), dim3(256), 0, st, d_probs, kMpEta);
        rb.clear();
        tptr.clear();
        std::vector<zk_herm> ha;
        std::vector<double *> s1hf, s1w, s1v;
        std::vector<int *> s1f;
        for (int p = 0; p < np; p++) {
            if (hipMemcpyAsync(th2.data(), hp[p].theta, 16 * (size_t)n, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(reach.data(), hp[p].reach, 4 * (size_t)n, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(rotf.data(), hp[p].rot, 4 * (size_t)n, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(rn.data(), hp[p].rnorm, 8 * (size_t)n, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return ctx->fail(ZK_EDEVICE, "coupling read-back failed");
            // boundary b: no pair j >= b reaches below b
            std::vector<int> minr(n + 1, n);
            for (int j = n - 1; j >= 0; j--) minr[j] = std::min(minr[j + 1], reach[j]);
            boff.clear();
            brot.clear();
            qoff.clear();
            int nb = 0, qo = 0, ho = 0, nf = 0;
            for (int j = 0; j < n; j++) {
                if (minr[j] >= j) {
                    boff.push_back(j);
                    nb++;
                }
                blk[j] = nb - 1;
            }
            boff.push_back(n);
            for (int b2 = 0; b2 < nb; b2++) {
                const int o = boff[b2], m = boff[b2 + 1] - o;
                // rotate only what the projected matrix can resolve: the spread of
                // the block's shifts well above the rounding of its binary64 F
                // entries (about u ||r||); a spread at that noise is a
                // degenerate eigenspace, where any basis is right
                bool need = false, flagged = false;
                double rmax = 0.0, tmin = 0.0, tmax = 0.0;
                for (int j = o; j < o + m; j++) {
                    flagged = flagged || rotf[j];
                    need = need || rn[j] > 0.5 * tol * hn[p];
                    rmax = std::max(rmax, rn[j]);
                    const double t = th2[j] + th2[n + j];
                    tmin = j == o ? t : std::min(tmin, t);
                    tmax = j == o ? t : std::max(tmax, t);
                }
                const double spread = (th2[o + m - 1] - th2[o]) + (th2[n + o + m - 1] - th2[n + o]);
                const bool resolvable = std::max(spread, tmax - tmin) > kMpRotMargin * 0x1p-53 * rmax;
                const bool r = m >= 2 && flagged && need && resolvable;
                brot.push_back(r ? 1 : 0);
                qoff.push_back(r ? qo : 0);
                if (r) {
                    MpBlk x;
                    x.prob = p;
                    x.b = b2;
                    rb.push_back(x);
                    tptr.push_back(btin[p] + qo);
                    zk_herm h;
                    std::memset(&h, 0, sizeof h);
                    h.n = m;
                    h.lda = m;
                    h.limbs = 1;
                    h.plane[0] = btin[p] + qo;
                    ha.push_back(h);
                    s1hf.push_back(bhf[p] + 2 * (size_t)ho);
                    s1w.push_back(hp[p].tw + o);
                    s1v.push_back((double *)(hp[p].Q + qo));
                    s1f.push_back(bflag[p] + nf++);
                    qo += m * m;
                    ho += m * m;
                }
            }
            if (hipMemcpyAsync(hp[p].blk, blk.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st) != hipSuccess ||
                hipMemcpyAsync(hp[p].boff, boff.data(), 4 * boff.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
                hipMemcpyAsync(hp[p].brot, brot.data(), 4 * brot.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
                hipMemcpyAsync(hp[p].qoff, qoff.data(), 4 * qoff.size(), hipMemcpyHostToDevice, st) != hipSuccess)
                return ctx->fail(ZK_EDEVICE, "block upload failed");
        }
        if (rb.empty()) return ZK_OK;
        const int nrb = (int)rb.size();
        int mmax = 0;
        for (const zk_herm &h : ha) mmax = std::max(mmax, h.n);
        if (hipMemcpyAsync(d_rb, rb.data(), sizeof(MpBlk) * nrb, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(d_tptr, tptr.data(), sizeof(void *) * nrb, hipMemcpyHostToDevice, st) != hipSuccess)
            return ctx->fail(ZK_EDEVICE, "block upload failed");
        hipLaunchKernelGGL(k_mp_tbuild<L>, dim3(cdivu((size_t)mmax * mmax, 256), nrb), dim3(256), 0, st, d_probs, d_rb,
                           d_tptr);
        if (hipGetLastError() != hipSuccess) return ctx->fail(ZK_EDEVICE, "projected matrix launch failed");
        return run_stage1(ctx, nrb, ha.data(), s1hf, s1w, s1v, s1f, std::vector<int>());
    };
    for (int p = 0; p < np; p++) hp[p].thr = 0.5 * tol * hn[p];
    if (hipMemcpyAsync(d_probs, hp.data(), sizeof(MpProb) * np, hipMemcpyHostToDevice, st) != hipSuccess)
        return done(ctx->fail(ZK_EDEVICE, "descriptor upload failed"));
    const bool trace = std::getenv("ZK_TRACE") != nullptr;
    int it = 0;
    std::vector<char> conv(np, 0);
    for (;; it++) {
        // residuals with the batch's input limb counts (launched per distinct count)
        for (int lc : {1, 2, 4}) {
            std::vector<int> ids;
            for (int p = 0; p < np; p++)
                if (lin[p] == lc) ids.push_back(p);
            if (ids.empty()) continue;
            if ((int)ids.size() == np) {
                if (launch_resid<L>(d_probs, np, n, lc, st)) return done(ctx->fail(ZK_EDEVICE, "residual launch failed"));
            } else {
                for (int p : ids)
                    if (launch_resid<L>(d_probs + p, 1, n, lc, st)) return done(ctx->fail(ZK_EDEVICE, "residual launch failed"));
            }
        }
        hipLaunchKernelGGL(k_mp_gram<L>, tiles, dim3(256), 0, st, d_probs);
        if (zgemm_batched(d_gemm, np, n, n, n, 1, 0, st)) return done(ctx->fail(ZK_EDEVICE, "F GEMM launch failed"));
        hipLaunchKernelGGL(k_mp_colstat<L>, dim3(n, np), dim3(256), 0, st, d_probs);
        hipLaunchKernelGGL(k_mp_maxstat, dim3(np), dim3(256), 0, st, d_probs);
        for (int p = 0; p < np; p++)
            if (hipMemcpyAsync(&stat[2 * p], hp[p].stat, 16, hipMemcpyDeviceToHost, st) != hipSuccess)
                return done(ctx->fail(ZK_EDEVICE, "read-back failed"));
        if (hipStreamSynchronize(st) != hipSuccess) return done(ctx->fail(ZK_EDEVICE, "polishing failed"));
        bool all = true;
        for (int p = 0; p < np; p++) {
            conv[p] = std::isfinite(stat[2 * p]) && stat[2 * p] <= 0.5 * tol * hn[p] && stat[2 * p + 1] <= tol;
            all = all && conv[p];
            if (trace)
                std::fprintf(stderr, "[zk mp L=%d] n=%d matrix %d iteration %d: max residual %.3e, orthonormality %.3e, "
                             "rotated blocks %d\n", L, n, p, it, stat[2 * p] / hn[p], stat[2 * p + 1], (int)rb.size());
        }
        if (all || it >= max_iter) break;
        if ((rc = plan_blocks()) != ZK_OK) return done(rc);
        hipLaunchKernelGGL(k_mp_corr<L>, elems, dim3(256), 0, st, d_probs, kMpEta);
        hipLaunchKernelGGL(k_mp_rot, elems, dim3(256), 0, st, d_probs);
        // the rotated blocks' members take their projected eigenvalues as shifts
        if (!rb.empty())
            hipLaunchKernelGGL(k_mp_lamrot<L>, dim3(cdivu(rb.size(), 64)), dim3(64), 0, st, d_probs, d_rb, (int)rb.size());
        hipLaunchKernelGGL(k_mp_update<L>, tiles, dim3(256), 0, st, d_probs);
        hipLaunchKernelGGL(k_mp_lamset<L>, dim3(cdivu(n, 256), np), dim3(256), 0, st, d_probs);
        // the next basis becomes the basis
        for (int p = 0; p < np; p++) std::swap(hp[p].X, hp[p].Xn);
        if (hipMemcpyAsync(d_probs, hp.data(), sizeof(MpProb) * np, hipMemcpyHostToDevice, st) != hipSuccess)
            return done(ctx->fail(ZK_EDEVICE, "descriptor upload failed"));
        if (hipGetLastError() != hipSuccess) return done(ctx->fail(ZK_EDEVICE, "polishing launch failed"));
    }
    if (iters_used) *iters_used = it;
    // ascending order of theta (lexicographic on the normalised limbs)
    std::vector<double> th((size_t)L * n);
    for (int p = 0; p < np; p++) {
        if (hipMemcpyAsync(th.data(), hp[p].theta, 8 * (size_t)L * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(rn.data(), hp[p].rnorm, 8 * (size_t)n, hipMemcpyDeviceToHost, st) != hipSuccess)
            return done(ctx->fail(ZK_EDEVICE, "read-back failed"));
        hipStreamSynchronize(st);
        int *pm = perm.data() + (size_t)p * n;
        std::iota(pm, pm + n, 0);
        std::stable_sort(pm, pm + n, [&](int a, int c) {
            for (int l = 0; l < L; l++) {
                const double x = th[(size_t)l * n + a], y = th[(size_t)l * n + c];
                if (x != y) return x < y;
            }
            return false;
        });
        if (info && info[p])
            for (int k = 0; k < n; k++) {
                zk_pair_info &f = info[p][k];
                f.iters = it;
                f.resid = rn[pm[k]] / hn[p];
                f.cluster = k;
                f.reserved = 0;
                f.flags = (f.resid <= tol && conv[p]) ? ZK_PAIR_CONVERGED : 0;
            }
    }
    if (hipMemcpyAsync(d_perm, perm.data(), 4 * (size_t)n * np, hipMemcpyHostToDevice, st) != hipSuccess)
        return done(ctx->fail(ZK_EDEVICE, "permutation upload failed"));
    hipLaunchKernelGGL(k_mp_output<L>, elems, dim3(256), 0, st, d_probs);
    if (hipGetLastError() != hipSuccess) return done(ctx->fail(ZK_EDEVICE, "output launch failed"));
    for (int p = 0; p < np; p++)
        if (!conv[p]) rc = ZK_ENOCONV;
    return done(rc);
}

template int mp_polish_run<4>(zk_ctx *, int, int, const int *, const double *const *, const double *const *,
                              const double2 *const *, double *const *, double2 *const *, const int *,
                              zk_pair_info *const *, double, int, int *);
template int mp_polish_run<8>(zk_ctx *, int, int, const int *, const double *const *, const double *const *,
                              const double2 *const *, double *const *, double2 *const *, const int *,
                              zk_pair_info *const *, double, int, int *);
template int mp_polish_run<16>(zk_ctx *, int, int, const int *, const double *const *, const double *const *,
                               const double2 *const *, double *const *, double2 *const *, const int *,
                               zk_pair_info *const *, double, int, int *);

}  // namespace zk
