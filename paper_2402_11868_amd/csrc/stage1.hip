// Stage 1 of the method: binary64 eigendecomposition of a batch of complex
// Hermitian matrices of equal order (the double-precision part of the paper's
// GPU routine, Sec. 2 "ZKCM_CUS"; the routine names no algorithm, the one
// here is the classical two-phase reduction).
//
//   ingest     limb sum -> binary64 working copy, limb-planar full copy for
//              stage 2, NaN/Inf scan
//   hetrd      blocked Householder tridiagonalisation, lower triangle:
//              per column a panel update + reflector (norm accumulated in
//              double-double), a tiled Hermitian matrix-vector product that
//              reads every lower-triangle element once and uses it for both
//              A and A^H, and the W-vector finish; per panel a rank-2*NB
//              trailing update C -= [V W][W V]^H on FP64 MFMA
//   stebz      Sturm-count bisection, one thread per eigenvalue
//   stein      inverse iteration, one thread per eigenvalue, then modified
//              Gram-Schmidt inside clusters (one wave per cluster)
//   unmtr      back-transformation V = Q Z with compact-WY block reflectors,
//              three FP64-MFMA GEMMs per panel
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "stage.h"

namespace zk {

// ------------------------------------------------------------- helpers ----
__device__ __forceinline__ double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) { return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }  // conj(a) b
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

__device__ __forceinline__ double2 wave_sum2(double2 v)
{
    v.x = wave_sum(v.x);
    v.y = wave_sum(v.y);
    return v;
}

// ---------------------------------------------------------------- ingest --
// grid (n columns, nprob), block 256: lower triangle of column j.
// fp32 != 0: the working copy is rounded to complex64 (the FP32-MFMA variant
// of the binary64 stage); the binary64 planes for the refinement stay exact.
__global__ void k_ingest(ProbDesc *probs, int fp32)
{
    const ProbDesc &P = probs[blockIdx.y];
    const int n = P.n, j = blockIdx.x;
    if (j >= n) return;
    const size_t nn = (size_t)n * n;
    if (threadIdx.x < 2) P.cnt[2 * j + threadIdx.x] = 0;   // finishing counters of column j
    int bad = 0;
    for (int i = j + threadIdx.x; i < n; i += blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int l = 0; l < P.limbs_in; l++) {
            const double2 z = ld2(P.in[l] + 2 * ((size_t)j * P.lda_in + i));
            if (!isfinite(z.x) || !isfinite(z.y)) bad = 1;
            const double zi = (i == j) ? 0.0 : z.y;
            re += z.x;
            im += zi;
            P.hf[(2 * l) * nn + (size_t)j * n + i] = z.x;
            P.hf[(2 * l + 1) * nn + (size_t)j * n + i] = zi;
            if (i != j) {
                P.hf[(2 * l) * nn + (size_t)i * n + j] = z.x;
                P.hf[(2 * l + 1) * nn + (size_t)i * n + j] = -zi;
            }
        }
        if (fp32) {
            re = (double)(float)re;
            im = (double)(float)im;
        }
        st2(P.A + 2 * ((size_t)j * n + i), make_double2(re, im));
    }
    if (bad) atomicOr(P.flag, 1);
}

// zero P and Q (n x 2NB complex each) of every problem; grid (ceil(2*NB*n/256), nprob)
__global__ void k_zero_panel(ProbDesc *probs)
{
    const ProbDesc &P = probs[blockIdx.y];
    const size_t cnt = (size_t)2 * kNB * P.n * 2;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += (size_t)gridDim.x * blockDim.x) {
        P.P[t] = 0.0;
        P.Q[t] = 0.0;
    }
}

// ------------------------------------------------- column update + larfg --
// Column c = k0 + i of the panel, in chunks of kColRows rows (grid
// (chunks, problems)): each chunk applies the panel's earlier reflectors to
// its rows and writes a partial norm; the last chunk to finish forms the
// reflector and writes it for every row.
constexpr int kColRows = 64;
constexpr int kLdU = 4;   // loads issued together in the per-column kernels' panel loops

__global__ void __launch_bounds__(256) k_trd_col(ProbDesc *probs, int c, int k0, int crows)
{
    const ProbDesc &P = probs[blockIdx.y];
    const int n = P.n, i = c - k0;
    const int G = (n - c + crows - 1) / crows;   // row chunks of column c (rows c .. n-1)
    const int g = blockIdx.x;
    if (g >= G) return;
    const int ntile = (n + 63) / 64;
    __shared__ double2 sVc[kNB], sWc[kNB];   // row c of V and W (conjugated later)
    __shared__ double2 sacc[4][64];
    __shared__ double2 sx[64];
    __shared__ double2 sdot[2 * kNB];
    __shared__ dd red_dd[16];
    __shared__ double2 s_scale;
    __shared__ int s_last;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid < i) {
        sVc[tid] = ld2(P.P + 2 * ((size_t)tid * n + c));
        sWc[tid] = ld2(P.P + 2 * ((size_t)(kNB + tid) * n + c));
    }
    if (tid < 2 * kNB) sdot[tid] = make_double2(0.0, 0.0);
    __syncthreads();
    // 1. a[r,c] -= sum_j V[r,j] conj(W[c,j]) + W[r,j] conj(V[c,j]) for the chunk's rows (the four
    //    waves split the j terms), then the chunk's share of ||x||^2 and of the panel dot
    //    products W_j^H x, V_j^H x over rows >= c+2 (x: the updated column; the reflector
    //    is x times a scale, applied by k_trd_wfin)
    dd nrm = mp_zero<2>();
    const int rend = min(n, c + (g + 1) * crows);
    for (int r0 = c + g * crows; r0 < rend; r0 += 64) {
        const int r = r0 + lane;
        double2 s = make_double2(0.0, 0.0);
        if (r < rend) {
            for (int j0 = wid; j0 < i; j0 += 4 * kLdU) {
                double2 v[kLdU], w[kLdU];
#pragma unroll
                for (int u = 0; u < kLdU; u++) {
                    const int j = min(j0 + 4 * u, i - 1);
                    v[u] = ld2(P.P + 2 * ((size_t)j * n + r));
                    w[u] = ld2(P.P + 2 * ((size_t)(kNB + j) * n + r));
                }
#pragma unroll
                for (int u = 0; u < kLdU; u++) {
                    const int j = j0 + 4 * u;
                    if (j < i)
                        s = cadd(s, cadd(cmul(v[u], make_double2(sWc[j].x, -sWc[j].y)), cmul(w[u], make_double2(sVc[j].x, -sVc[j].y))));
                }
            }
        }
        sacc[wid][lane] = s;
        __syncthreads();
        if (wid == 0) {
            double2 a = make_double2(0.0, 0.0);
            if (r < rend) {
                a = ld2(P.A + 2 * ((size_t)c * n + r));
                a = csub(a, cadd(cadd(sacc[0][lane], sacc[1][lane]), cadd(sacc[2][lane], sacc[3][lane])));
                if (r == c) a.y = 0.0;
                st2(P.A + 2 * ((size_t)c * n + r), a);
                if (r >= c + 2) {
                    // |x_r|^2 in double-double (exact squares)
                    double p, e;
                    two_prod(a.x, a.x, p, e);
                    nrm = dd_add(nrm, dd{{p, e}});
                    two_prod(a.y, a.y, p, e);
                    nrm = dd_add(nrm, dd{{p, e}});
                }
            }
            sx[lane] = (r < rend && r >= c + 2) ? a : make_double2(0.0, 0.0);
        }
        __syncthreads();
        {
            // every lane takes part in the wave sums (zero outside the chunk)
            const double2 x = sx[lane];
            const int rr = r < rend ? r : c;   // a valid row for lanes outside the chunk (their terms are zero)
            for (int j0 = wid; j0 < i; j0 += 4 * kLdU) {
                double2 wv[kLdU], vv[kLdU];
#pragma unroll
                for (int u = 0; u < kLdU; u++) {
                    const int j = min(j0 + 4 * u, i - 1);
                    wv[u] = ld2(P.P + 2 * ((size_t)(kNB + j) * n + rr));
                    vv[u] = ld2(P.P + 2 * ((size_t)j * n + rr));
                }
#pragma unroll
                for (int u = 0; u < kLdU; u++) {
                    const int j = j0 + 4 * u;
                    if (j >= i) break;
                    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
                    if (r < rend) {
                        a = cmulc(wv[u], x);
                        b = cmulc(vv[u], x);
                    }
                    a = wave_sum2(a);
                    b = wave_sum2(b);
                    if (lane == 0) {
                        sdot[j] = cadd(sdot[j], a);
                        sdot[kNB + j] = cadd(sdot[kNB + j], b);
                    }
                }
            }
        }
        __syncthreads();
    }
    const dd part = block_sum_mp<2>(nrm, red_dd);
    double *snorm = P.scr;
    double2 *sd = reinterpret_cast<double2 *>(P.scr + 2 * ntile) + (size_t)g * 2 * kNB;
    if (tid == 0) {
        snorm[2 * g] = part.x[0];
        snorm[2 * g + 1] = part.x[1];
    }
    if (tid < 2 * i) sd[tid < i ? tid : kNB + tid - i] = sdot[tid < i ? tid : kNB + tid - i];
    // the last chunk to finish forms the reflector (device-scope fences around
    // the counter make every chunk's column entries and partial sums visible)
    bool last = true;
    if (G > 1) {
        __threadfence();
        __syncthreads();
        if (tid == 0) s_last = atomicAdd(P.cnt + 2 * c, 1) == G - 1;
        __syncthreads();
        last = s_last;
        if (last) __threadfence();
    } else {
        __syncthreads();
    }
    if (!last) return;
    if (tid == 0) {
        const double2 diag = ld2(P.A + 2 * ((size_t)c * n + c));
        const double2 alpha = ld2(P.A + 2 * ((size_t)c * n + c + 1));
        // the chunks' norms in chunk order, their loads issued 8 at a time
        dd xn2 = mp_zero<2>();
        for (int q0 = 0; q0 < G; q0 += 8) {
            dd pn[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int q = min(q0 + u, G - 1);
                pn[u] = dd{{snorm[2 * q], snorm[2 * q + 1]}};
            }
#pragma unroll
            for (int u = 0; u < 8; u++)
                if (q0 + u < G) xn2 = dd_add(xn2, pn[u]);
        }
        P.d[c] = diag.x;
        double2 tau = make_double2(0.0, 0.0);
        double beta = alpha.x;
        double2 scale = make_double2(0.0, 0.0);
        if (!(xn2.x[0] == 0.0 && alpha.y == 0.0)) {
            // beta = -sign(Re alpha) * sqrt(|alpha|^2 + ||x||^2), the norm in double-double
            double p, e;
            dd sq = xn2;
            two_prod(alpha.x, alpha.x, p, e);
            sq = dd_add(sq, dd{{p, e}});
            two_prod(alpha.y, alpha.y, p, e);
            sq = dd_add(sq, dd{{p, e}});
            const dd rt = dd_sqrt(sq);
            beta = (alpha.x >= 0.0) ? -rt.x[0] : rt.x[0];
            tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
            // scale = 1 / (alpha - beta)
            const double2 den = make_double2(alpha.x - beta, alpha.y);
            const double m2 = den.x * den.x + den.y * den.y;
            scale = make_double2(den.x / m2, -den.y / m2);
        }
        P.e[c] = beta;
        st2(P.tau + 2 * c, tau);
        st2(P.scr + 2 * ntile + 4 * kNB * ntile + 2 * ntile, scale);   // for k_trd_wfin
        s_scale = scale;
    }
    __syncthreads();
    const double2 sc = s_scale;
    // 2. reflector v (v[c+1] = 1) into Y[:, c], V column i of P, V column NB+i of Q
    for (int r0 = c + 1; r0 < n; r0 += 4 * 256) {
        double2 av[4];
#pragma unroll
        for (int u = 0; u < 4; u++) av[u] = ld2(P.A + 2 * ((size_t)c * n + min(r0 + 256 * u + tid, n - 1)));
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int r2 = r0 + 256 * u + tid;
            if (r2 >= n) continue;
            const double2 v = (r2 == c + 1) ? make_double2(1.0, 0.0) : cmul(av[u], sc);
            st2(P.Y + 2 * ((size_t)c * n + r2), v);
            st2(P.P + 2 * ((size_t)i * n + r2), v);
            st2(P.Q + 2 * ((size_t)(kNB + i) * n + r2), v);
        }
    }
}

__global__ void __launch_bounds__(256) k_trd_hemv(ProbDesc *probs, int c)
{
    const ProbDesc &P = probs[blockIdx.y];
    const int n = P.n, base = c + 1, m = n - base;
    if (m <= 0) return;
    const int T = (m + 63) / 64;
    const int t = blockIdx.x;
    if (t >= T * (T + 1) / 2) return;
    int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) I--;
    while ((I + 1) * (I + 2) / 2 <= t) I++;
    const int J = t - I * (I + 1) / 2;
    __shared__ double2 tile[64][65];
    __shared__ double2 vI[64], vJ[64];
    __shared__ double2 red[4][64];
    const int tid = threadIdx.x;
    const double2 *A = reinterpret_cast<const double2 *>(P.A);
    const double2 *Yc = reinterpret_cast<const double2 *>(P.Y) + (size_t)c * n + base;
    // load tile: column jj (0..63) of the tile, rows ii
    // the tile's 16 loads per thread issued together (a clamped address for
    // entries outside the lower triangle of A22, whose values are discarded)
#pragma unroll
    for (int q0 = 0; q0 < 64 * 64; q0 += 256 * 8) {
        double2 av[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int q = q0 + 256 * u + tid, ii = q & 63, jj = q >> 6;
            const int gi = I * 64 + ii, gj = J * 64 + jj;
            const bool ok = gi < m && gj < m && gi >= gj;
            av[u] = A[ok ? (size_t)(base + gj) * n + base + gi : (size_t)base * n + base];
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int q = q0 + 256 * u + tid, ii = q & 63, jj = q >> 6;
            const int gi = I * 64 + ii, gj = J * 64 + jj;
            double2 a = make_double2(0.0, 0.0);
            if (gi < m && gj < m && gi >= gj) {
                a = av[u];
                if (gi == gj) a.y = 0.0;
            }
            tile[ii][jj] = a;
        }
    }
    if (tid < 64) {
        const int gi = I * 64 + tid, gj = J * 64 + tid;
        vI[tid] = gi < m ? Yc[gi] : make_double2(0.0, 0.0);
        vJ[tid] = gj < m ? Yc[gj] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int lane = tid & 63, grp = tid >> 6;
    // direct: row ii = lane, columns grp*16 .. +16
    {
        double2 s = make_double2(0.0, 0.0);
        for (int jj = grp * 16; jj < grp * 16 + 16; jj++) {
            const bool use = (I != J) || (jj <= lane);
            if (use) s = cadd(s, cmul(tile[lane][jj], vJ[jj]));
        }
        red[grp][lane] = s;
    }
    __syncthreads();
    if (tid < 64) {
        const int gi = I * 64 + tid;
        double2 s = cadd(cadd(red[0][tid], red[1][tid]), cadd(red[2][tid], red[3][tid]));
        if (gi < m) st2(P.part + 2 * ((size_t)J * n + base + gi), s);
    }
    __syncthreads();
    // mirror: column jj = lane, rows grp*16 .. +16, strictly below the diagonal
    {
        double2 s = make_double2(0.0, 0.0);
        for (int ii = grp * 16; ii < grp * 16 + 16; ii++) {
            const bool use = (I != J) || (ii > lane);
            if (use) s = cadd(s, cmulc(tile[ii][lane], vI[ii]));
        }
        red[grp][lane] = s;
    }
    __syncthreads();
    if (tid < 64) {
        const int gj = J * 64 + tid;
        double2 s = cadd(cadd(red[0][tid], red[1][tid]), cadd(red[2][tid], red[3][tid]));
        if (gj < m) st2(P.part + 2 * ((size_t)(T + I) * n + base + gj), s);
    }
}

// ------------------------------------------------------------- w finish ---
// Row chunks of wrows rows (grid (chunks, problems)): y = sum of the hemv
// partials - V (W^H v) - W (V^H v) for the chunk's rows, w = tau y, and the
// chunk's share of w^H v; the dot products W_j^H v, V_j^H v come from the
// column kernel's chunk sums (taken on the unscaled column, times the
// reflector's scale, plus the v[c+1] = 1 term).  The last chunk to finish adds
// (-tau/2 w^H v) v to every row and stores W column i into P[:, NB+i] and Q[:, i].
__global__ void __launch_bounds__(256) k_trd_wfin(ProbDesc *probs, int c, int k0, int crows, int wrows)
{
    const ProbDesc &P = probs[blockIdx.y];
    const int n = P.n, base = c + 1, m = n - base, i = c - k0;
    if (m <= 0) return;
    const int T = (m + 63) / 64;             // hemv row blocks
    const int G = (m + wrows - 1) / wrows;   // chunks of this kernel
    const int Gc = (n - c + crows - 1) / crows;   // chunks of the column kernel
    const int g = blockIdx.x;
    if (g >= G) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int ntile = (n + 63) / 64;
    __shared__ double2 t1[kNB], t2[kNB];
    __shared__ double2 sacc[4][64];
    __shared__ double2 s_alpha;
    __shared__ int s_last;
    const double2 *Pv = reinterpret_cast<const double2 *>(P.P);
    double2 *Pw = reinterpret_cast<double2 *>(P.P);
    const double2 *Yc = reinterpret_cast<const double2 *>(P.Y) + (size_t)c * n;
    const double2 *sd = reinterpret_cast<const double2 *>(P.scr + 2 * ntile);
    double2 *swv = reinterpret_cast<double2 *>(P.scr + 2 * ntile + 4 * kNB * ntile);
    const double2 scale = ld2(P.scr + 2 * ntile + 4 * kNB * ntile + 2 * ntile);
    // t1_j = W_j^H v, t2_j = V_j^H v (j < i)
    if (tid < 2 * i) {
        const int j = tid < i ? tid : tid - i, o = tid < i ? j : kNB + j;
        double2 a = make_double2(0.0, 0.0);
        for (int q0 = 0; q0 < Gc; q0 += 8) {
            double2 pv[8];
#pragma unroll
            for (int u = 0; u < 8; u++) pv[u] = sd[(size_t)min(q0 + u, Gc - 1) * 2 * kNB + o];
#pragma unroll
            for (int u = 0; u < 8; u++)
                if (q0 + u < Gc) a = cadd(a, pv[u]);
        }
        const double2 top = Pv[(size_t)(tid < i ? kNB + j : j) * n + base];   // row c+1, where v = 1
        a = cadd(make_double2(top.x, -top.y), cmul(scale, a));
        if (tid < i) t1[j] = a;
        else t2[j] = a;
    }
    __syncthreads();
    const double2 tau = ld2(P.tau + 2 * c);
    double2 wv = make_double2(0.0, 0.0);
    const int rend = min(n, base + (g + 1) * wrows);
    for (int r0 = base + g * wrows; r0 < rend; r0 += 64) {
        const int r = r0 + lane;
        double2 s = make_double2(0.0, 0.0);
        if (r < rend)
            for (int j0 = wid; j0 < i; j0 += 4 * kLdU) {
                double2 v[kLdU], w[kLdU];
#pragma unroll
                for (int u = 0; u < kLdU; u++) {
                    const int j = min(j0 + 4 * u, i - 1);
                    v[u] = Pv[(size_t)j * n + r];
                    w[u] = Pv[(size_t)(kNB + j) * n + r];
                }
#pragma unroll
                for (int u = 0; u < kLdU; u++) {
                    const int j = j0 + 4 * u;
                    if (j < i) {
                        s = cadd(s, cmul(v[u], t1[j]));
                        s = cadd(s, cmul(w[u], t2[j]));
                    }
                }
            }
        sacc[wid][lane] = s;
        __syncthreads();
        if (wid == 0 && r < rend) {
            const int b = (r - base) / 64;
            double2 y = make_double2(0.0, 0.0);
            // the partials in the same order, their loads issued kLdU at a time
            for (int J0 = 0; J0 <= b; J0 += kLdU) {
                double2 pv[kLdU];
#pragma unroll
                for (int u = 0; u < kLdU; u++) pv[u] = ld2(P.part + 2 * ((size_t)min(J0 + u, b) * n + r));
#pragma unroll
                for (int u = 0; u < kLdU; u++)
                    if (J0 + u <= b) y = cadd(y, pv[u]);
            }
            for (int I0 = b; I0 < T; I0 += kLdU) {
                double2 pv[kLdU];
#pragma unroll
                for (int u = 0; u < kLdU; u++) pv[u] = ld2(P.part + 2 * ((size_t)(T + min(I0 + u, T - 1)) * n + r));
#pragma unroll
                for (int u = 0; u < kLdU; u++)
                    if (I0 + u < T) y = cadd(y, pv[u]);
            }
            y = csub(y, cadd(cadd(sacc[0][lane], sacc[1][lane]), cadd(sacc[2][lane], sacc[3][lane])));
            y = cmul(tau, y);
            Pw[(size_t)(kNB + i) * n + r] = y;
            wv = cadd(wv, cmulc(y, Yc[r]));
        }
        __syncthreads();
    }
    if (wid == 0) {
        wv = wave_sum2(wv);
        if (lane == 0) swv[g] = wv;
    }
    bool last = true;
    if (G > 1) {
        __threadfence();
        __syncthreads();
        if (tid == 0) s_last = atomicAdd(P.cnt + 2 * c + 1, 1) == G - 1;
        __syncthreads();
        last = s_last;
        if (last) __threadfence();
    } else {
        __syncthreads();
    }
    if (!last) return;
    if (tid == 0) {
        double2 t = make_double2(0.0, 0.0);
        for (int q0 = 0; q0 < G; q0 += 8) {
            double2 pv[8];
#pragma unroll
            for (int u = 0; u < 8; u++) pv[u] = swv[min(q0 + u, G - 1)];
#pragma unroll
            for (int u = 0; u < 8; u++)
                if (q0 + u < G) t = cadd(t, pv[u]);
        }
        s_alpha = cmul(make_double2(-0.5 * tau.x, -0.5 * tau.y), t);
    }
    __syncthreads();
    const double2 alpha = s_alpha;
    for (int r0 = base; r0 < n; r0 += 4 * 256) {
        double2 wv[4], yv[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int r2 = min(r0 + 256 * u + tid, n - 1);
            wv[u] = Pw[(size_t)(kNB + i) * n + r2];
            yv[u] = Yc[r2];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int r2 = r0 + 256 * u + tid;
            if (r2 >= n) continue;
            const double2 w = cadd(wv[u], cmul(alpha, yv[u]));
            Pw[(size_t)(kNB + i) * n + r2] = w;
            reinterpret_cast<double2 *>(P.Q)[(size_t)i * n + r2] = w;
        }
    }
}

// --------------------------------------------------------- MFMA ZGEMM -----
// C(MxN) = alpha * op(A) op(B) + beta * C, complex128, column-major.
// op 0 = N, 1 = C (conjugate transpose).  lower != 0: only tiles that
// intersect the lower triangle (row >= col) are computed (her2k).
// Block 256 = 4 waves, tile 32 x 32, each wave one 16 x 16 block computed as
// its transpose D = (op(A) op(B))^T with v_mfma_f64_16x16x4f64 (a complex
// product is four real MFMAs), so that each accumulator register of a wave
// maps to 16 consecutive rows of one column of C (coalesced epilogue).
// Operand layout of the 16x16x4 f64 MFMA (wave64): lane l holds X[l%16][l/16]
// and Y[l/16][l%16]; the 4 accumulator values of lane l are D[4r + l/16][l%16].
// The operands of 8 consecutive k-steps are loaded before their MFMAs so
// that the loads are in flight together.
// Operand loads without branches: an index outside the operand is clamped to
// element (0, 0) (always present when a load runs, M, N, K >= 1), the load is
// issued unconditionally and its bits are cleared afterwards with an integer
// mask; op (uniform per launch) selects the address.  A load under a branch
// ends in a wait for that load, so the loads of a k-chunk would be issued one
// after another instead of together.
struct OpLd {
    size_t off;
    unsigned long long mask;   // all ones inside the operand, zero outside
};

__device__ __forceinline__ OpLd opA_at(int lda, int op, int i, int k, int M, int K)
{
    const bool ok = i < M && k < K;
    const int ii = ok ? i : 0, kk = ok ? k : 0;
    return OpLd{op == 0 ? (size_t)kk * lda + ii : (size_t)ii * lda + kk, ok ? ~0ull : 0ull};
}

__device__ __forceinline__ OpLd opB_at(int ldb, int op, int k, int j, int K, int N)
{
    const bool ok = k < K && j < N;
    const int kk = ok ? k : 0, jj = ok ? j : 0;
    return OpLd{op == 0 ? (size_t)jj * ldb + kk : (size_t)kk * ldb + jj, ok ? ~0ull : 0ull};
}

// the loaded value with the mask applied and the conjugate taken for op != 0
__device__ __forceinline__ double2 op_val(double2 v, unsigned long long mask, int op)
{
    const unsigned long long sgn = op == 0 ? 0ull : 0x8000000000000000ull;
    return make_double2(__longlong_as_double(__double_as_longlong(v.x) & mask),
                        __longlong_as_double((__double_as_longlong(v.y) ^ sgn) & mask));
}

__device__ __forceinline__ double2 opA_ld(const double2 *A, int lda, int op, int i, int k, int M, int K)
{
    const OpLd a = opA_at(lda, op, i, k, M, K);
    return op_val(A[a.off], a.mask, op);
}

__device__ __forceinline__ double2 opB_ld(const double2 *B, int ldb, int op, int k, int j, int K, int N)
{
    const OpLd b = opB_at(ldb, op, k, j, K, N);
    return op_val(B[b.off], b.mask, op);
}

constexpr int kGemmKc = 8;   // k-steps of 4 whose operands are loaded together

// One 32 x 32 tile (tm, tn) of C by the four waves of a work-group.
__device__ __forceinline__ void zgemm_tile(const GemmDesc &G, int M, int N, int K, int opA, int opB, double2 alpha,
                                           double2 beta, int lower, int tm, int tn)
{
    const int row0 = tm * 32, col0 = tn * 32;
    if (lower && row0 + 31 < col0) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = row0 + (wid & 1) * 16, wc = col0 + (wid >> 1) * 16;
    if (lower && wr + 15 < wc) return;
    const double2 *A = reinterpret_cast<const double2 *>(G.A);
    const double2 *B = reinterpret_cast<const double2 *>(G.B);
    // four independent accumulator chains (the real and imaginary parts of
    // the two real products each), so that consecutive MFMAs do not wait on
    // each other's results
    f64x4 crr = f64x4{0.0, 0.0, 0.0, 0.0}, cii = crr, cri = crr, cir = crr;
    const int li = lane & 15, lk = lane >> 4;
    const int lda = G.lda, ldb = G.ldb;
    for (int k0 = 0; k0 < K; k0 += 4 * kGemmKc) {
        double2 xv[kGemmKc], yv[kGemmKc];
        unsigned long long xm[kGemmKc], ym[kGemmKc];
        // X[j][k] = op(B)[k][j], Y[k][i] = op(A)[i][k]: every load of the
        // chunk issued before any is used
#pragma unroll
        for (int s = 0; s < kGemmKc; s++) {
            const OpLd b = opB_at(ldb, opB, k0 + 4 * s + lk, wc + li, K, N);
            const OpLd a = opA_at(lda, opA, wr + li, k0 + 4 * s + lk, M, K);
            xv[s] = B[b.off];
            yv[s] = A[a.off];
            xm[s] = b.mask;
            ym[s] = a.mask;
        }
#pragma unroll
        for (int s = 0; s < kGemmKc; s++) {
            xv[s] = op_val(xv[s], xm[s], opB);
            yv[s] = op_val(yv[s], ym[s], opA);
        }
#pragma unroll
        for (int s = 0; s < kGemmKc; s++) {
            crr = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[s].x, yv[s].x, crr, 0, 0, 0);
            cii = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[s].y, yv[s].y, cii, 0, 0, 0);
            cri = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[s].x, yv[s].y, cri, 0, 0, 0);
            cir = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[s].y, yv[s].x, cir, 0, 0, 0);
        }
    }
    double2 *C = reinterpret_cast<double2 *>(G.C);
    const int i = wr + li;
    if (i >= M) return;
    for (int r = 0; r < 4; r++) {
        const int j = wc + 4 * r + lk;
        if (j >= N || (lower && i < j)) continue;
        double2 out = cmul(alpha, make_double2(crr[r] - cii[r], cri[r] + cir[r]));
        if (beta.x != 0.0 || beta.y != 0.0) out = cadd(out, cmul(beta, C[(size_t)j * G.ldc + i]));
        C[(size_t)j * G.ldc + i] = out;
    }
}

__global__ void __launch_bounds__(256) k_zgemm(const GemmDesc *descs, int M, int N, int K, int opA, int opB,
                                               double2 alpha, double2 beta, int lower)
{
    const int tilesM = (M + 31) / 32;
    zgemm_tile(descs[blockIdx.y], M, N, K, opA, opB, alpha, beta, lower, blockIdx.x % tilesM, blockIdx.x / tilesM);
}

// C = op(A) op(B) for `count` descriptors of equal shape (M x N, inner K).
int zgemm_batched(const GemmDesc *d_descs, int count, int M, int N, int K, int opA, int opB, hipStream_t st)
{
    if (count <= 0 || M <= 0 || N <= 0) return 0;
    const unsigned tiles = (unsigned)(((M + 31) / 32) * ((N + 31) / 32));
    hipLaunchKernelGGL(k_zgemm, dim3(tiles, count), dim3(256), 0, st, d_descs, M, N, K, opA, opB, make_double2(1.0, 0.0),
                       make_double2(0.0, 0.0), 0);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// The same product with FP32 MFMA (v_mfma_f32_16x16x4f32) on operands rounded
// to complex64 and FP32 accumulation; alpha, beta and C stay binary64.  Output
// layout of that MFMA: the 4 accumulator values of lane l are
// D[4 (l/16) + r][l%16].
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_cgemm32(const GemmDesc *descs, int M, int N, int K, int opA, int opB,
                                                 double2 alpha, double2 beta, int lower)
{
    const GemmDesc &G = descs[blockIdx.y];
    const int tilesM = (M + 31) / 32;
    const int tm = blockIdx.x % tilesM, tn = blockIdx.x / tilesM;
    const int row0 = tm * 32, col0 = tn * 32;
    if (lower && row0 + 31 < col0) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = row0 + (wid & 1) * 16, wc = col0 + (wid >> 1) * 16;
    if (lower && wr + 15 < wc) return;
    const double2 *A = reinterpret_cast<const double2 *>(G.A);
    const double2 *B = reinterpret_cast<const double2 *>(G.B);
    f32x4 cre = f32x4{0.f, 0.f, 0.f, 0.f}, cim = f32x4{0.f, 0.f, 0.f, 0.f};
    const int li = lane & 15, lk = lane >> 4;
    for (int k0 = 0; k0 < K; k0 += 4 * kGemmKc) {
        float2 xv[kGemmKc], yv[kGemmKc];
#pragma unroll
        for (int s = 0; s < kGemmKc; s++) {
            const double2 x = opB_ld(B, G.ldb, opB, k0 + 4 * s + lk, wc + li, K, N);
            const double2 y = opA_ld(A, G.lda, opA, wr + li, k0 + 4 * s + lk, M, K);
            xv[s] = make_float2((float)x.x, (float)x.y);
            yv[s] = make_float2((float)y.x, (float)y.y);
        }
#pragma unroll
        for (int s = 0; s < kGemmKc; s++) {
            cre = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[s].x, yv[s].x, cre, 0, 0, 0);
            cre = __builtin_amdgcn_mfma_f32_16x16x4f32(-xv[s].y, yv[s].y, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[s].x, yv[s].y, cim, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[s].y, yv[s].x, cim, 0, 0, 0);
        }
    }
    double2 *C = reinterpret_cast<double2 *>(G.C);
    const int i = wr + li;
    if (i >= M) return;
    for (int r = 0; r < 4; r++) {
        const int j = wc + 4 * lk + r;
        if (j >= N || (lower && i < j)) continue;
        double2 out = cmul(alpha, make_double2((double)cre[r], (double)cim[r]));
        if (beta.x != 0.0 || beta.y != 0.0) out = cadd(out, cmul(beta, C[(size_t)j * G.ldc + i]));
        C[(size_t)j * G.ldc + i] = out;
    }
}

// ------------------------------------------------------------- bisection --
// One thread per eigenvalue index k: Sturm count bisection on (d, e).
__device__ int sturm_count(const double *d, const double *e, int n, double x, double pivmin)
{
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) cnt++;
    for (int i = 1; i < n; i++) {
        q = d[i] - x - (e[i - 1] * e[i - 1]) / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) cnt++;
    }
    return cnt;
}

// Multisection: one wave per eigenvalue k.  Each round the 64 lanes count the
// eigenvalues below 64 points spread evenly over the current interval and the
// interval shrinks to the gap that holds eigenvalue k: about 6 bits per round
// with the round's counts in parallel, where bisection gains one bit per
// count.  Same bracket, stopping rule and final midpoint as bisection.
__global__ void __launch_bounds__(256) k_bisect(ProbDesc *probs)
{
    const ProbDesc &P = probs[blockIdx.y];
    const int n = P.n;
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= n) return;   // uniform per wave; no barriers below
    double gl = INFINITY, gu = -INFINITY, emax = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double r = (i > 0 ? fabs(P.e[i - 1]) : 0.0) + (i < n - 1 ? fabs(P.e[i]) : 0.0);
        gl = fmin(gl, P.d[i] - r);
        gu = fmax(gu, P.d[i] + r);
        if (i < n - 1) emax = fmax(emax, fabs(P.e[i]));
    }
    for (int off = 32; off > 0; off >>= 1) {
        gl = fmin(gl, __shfl_xor(gl, off, 64));
        gu = fmax(gu, __shfl_xor(gu, off, 64));
        emax = fmax(emax, __shfl_xor(emax, off, 64));
    }
    const double tnorm = fmax(fabs(gl), fabs(gu));
    const double pivmin = fmax(2.2250738585072014e-308, 2.2250738585072014e-308 * emax * emax);
    const double eps = 1.1102230246251565e-16;
    double lo = gl - 2.0 * eps * tnorm - 2.0 * pivmin, hi = gu + 2.0 * eps * tnorm + 2.0 * pivmin;
    for (int it = 0; it < 64; it++) {
        if (hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin) break;
        const double x = lo + (hi - lo) * ((double)(lane + 1) / 65.0);
        const unsigned long long above = __ballot(sturm_count(P.d, P.e, n, x, pivmin) > k);
        const int f = above ? __ffsll((long long)above) - 1 : 64;   // first point above eigenvalue k
        const double xl = __shfl(x, f > 0 ? f - 1 : 0, 64), xh = __shfl(x, f < 64 ? f : 63, 64);
        const double nlo = f > 0 ? xl : lo, nhi = f < 64 ? xh : hi;
        if (nlo == lo && nhi == hi) break;
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) P.w0[k] = 0.5 * (lo + hi);
}

// ------------------------------------------------------ inverse iteration --
// One thread per eigenvalue k: three inverse iterations with the tridiagonal
// LU (partial pivoting) of T - lam I from a hashed pseudo-random start.  Work
// arrays are interleaved across eigenvalues (entry i of eigenvalue k at
// [i*n + k]) so neighbouring threads touch neighbouring addresses.  Output
// Zt[i*n + k], scaled to max-norm 1 (the cluster Gram-Schmidt normalises).
__device__ __forceinline__ double hash_uniform(uint64_t x)
{
    // SplitMix64 finaliser (Steele, Lea, Flood 2014) -> uniform in (-1, 1)
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return ((double)(x >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
}

__global__ void k_invit(ProbDesc *probs)
{
    const ProbDesc &P = probs[blockIdx.y];
    const int n = P.n;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const size_t nn = (size_t)n * n;
    double *U0 = P.tri, *U1 = P.tri + nn, *U2 = P.tri + 2 * nn, *LM = P.tri + 3 * nn, *FL = P.tri + 4 * nn;
    double *X = P.Zt;
    const double lam = P.w0[k];
    double tnorm = 0.0;
    for (int i = 0; i < n; i++)
        tnorm = fmax(tnorm, fabs(P.d[i]) + (i > 0 ? fabs(P.e[i - 1]) : 0.0) + (i < n - 1 ? fabs(P.e[i]) : 0.0));
    const double guard = fmax(tnorm, 1e-300) * 1.1102230246251565e-16;
    // A coupling negligible against the entries of T - lam I it connects
    // (|e_i| <= eps (|d_i - lam| + |d_(i+1) - lam|)) is taken as an exact zero,
    // so T - lam I splits into blocks.  An eigenvalue shared by two blocks
    // (the +-s pairs of a dilation with equal singular values, a direct sum)
    // then has a guarded pivot in each block and every start vector keeps both
    // null directions; through a coupling of, say, 1e-17 between entries of
    // size 1 the row exchange would drop one of them and all the inverse
    // iterates of that eigenvalue would be the same vector.  The threshold
    // follows the shifted diagonal, so the couplings of tiny eigenvalues
    // (tiny diagonal entries) are kept.
    auto cpl = [&](int i) {
        const double x = P.e[i];
        const double scale = fabs(P.d[i] - lam) + fabs(P.d[i + 1] - lam);
        return fabs(x) <= 1.1102230246251565e-16 * scale ? 0.0 : x;
    };
    // P L U factorisation of T - lam I by Gaussian elimination with partial
    // pivoting.  The row being eliminated always has two entries (a at
    // column i, b at column i+1); U row i has up to three (u0, u1, u2).
    double a = P.d[0] - lam, b = (n > 1) ? cpl(0) : 0.0;
    for (int i = 0; i < n - 1; i++) {
        const double sub = cpl(i);                                  // T[i+1][i]
        const double na = P.d[i + 1] - lam;                         // T[i+1][i+1]
        const double nb = (i + 1 < n - 1) ? cpl(i + 1) : 0.0;       // T[i+1][i+2]
        const size_t o = (size_t)i * n + k;
        if (fabs(a) >= fabs(sub)) {
            double piv = a;
            if (fabs(piv) < guard) piv = (piv < 0.0) ? -guard : guard;
            const double l = sub / piv;
            U0[o] = piv; U1[o] = b; U2[o] = 0.0; LM[o] = l; FL[o] = 0.0;
            a = na - l * b;
            b = nb;
        } else {
            // rows exchanged: the pivot is the subdiagonal entry, which can be
            // far below the guard (a split or nearly split T); unclamped, its
            // direction would be amplified by 1 / |sub| instead of 1 / guard
            // and every member of a cluster would collapse onto it
            double piv = sub;
            if (fabs(piv) < guard) piv = (piv < 0.0) ? -guard : guard;
            const double l = a / piv;
            U0[o] = piv; U1[o] = na; U2[o] = nb; LM[o] = l; FL[o] = 1.0;
            a = b - l * na;
            b = -l * nb;
        }
    }
    double last = a;
    if (fabs(last) < guard) last = (last < 0.0) ? -guard : guard;
    for (int i = 0; i < n; i++) X[(size_t)i * n + k] = hash_uniform(((uint64_t)k << 32) ^ (uint64_t)i ^ 0x5bd1e995ull);
    for (int it = 0; it < 3; it++) {
        for (int i = 0; i < n - 1; i++) {
            const size_t o = (size_t)i * n + k;
            double xi = X[o], xj = X[o + n];
            if (FL[o] != 0.0) {
                const double t = xi;
                xi = xj;
                xj = t;
                X[o] = xi;
            }
            X[o + n] = xj - LM[o] * xi;
        }
        double x1 = 0.0, x2 = 0.0, smax = 0.0;
        for (int i = n - 1; i >= 0; i--) {
            const size_t o = (size_t)i * n + k;
            const double u0 = (i == n - 1) ? last : U0[o];
            const double u1 = (i < n - 1) ? U1[o] : 0.0;
            const double u2 = (i < n - 2) ? U2[o] : 0.0;
            const double xi = (X[o] - u1 * x1 - u2 * x2) / u0;
            X[o] = xi;
            x2 = x1;
            x1 = xi;
            smax = fmax(smax, fabs(xi));
        }
        const double inv = (smax > 0.0) ? 1.0 / smax : 1.0;
        for (int i = 0; i < n; i++) X[(size_t)i * n + k] *= inv;
    }
}

// Zt (row-interleaved) -> Z (column-major) ; grid (ceil(n/16), ceil(n/16), nprob), block 16x16
__global__ void k_transpose(ProbDesc *probs)
{
    const ProbDesc &P = probs[blockIdx.z];
    const int n = P.n;
    __shared__ double t[16][17];
    const double *src = P.Zt;
    const int i0 = blockIdx.x * 16, k0 = blockIdx.y * 16;
    const int tx = threadIdx.x, ty = threadIdx.y;
    if (i0 + ty < n && k0 + tx < n) t[ty][tx] = src[(size_t)(i0 + ty) * n + k0 + tx];
    __syncthreads();
    if (k0 + ty < n && i0 + tx < n) P.Z[(size_t)(k0 + ty) * n + i0 + tx] = t[tx][ty];
}

// Gram-Schmidt inside clusters of the binary64 spectrum.  Cluster:
// consecutive eigenvalues closer than gap_rel * ||T||.  Members are handled
// in blocks of kTriRB (block b = positions [kTriRB b, kTriRB (b+1)) inside the
// cluster): each member of block b is projected against all members of the
// earlier blocks by classical Gram-Schmidt, twice (one work-group per member,
// every member of every cluster in parallel), then the block is
// orthogonalised inside (classical Gram-Schmidt twice, member by member) and
// normalised.  The same vectors as in-order Gram-Schmidt over the whole
// cluster, with the long chains of the spectrum's tail spread over the chip.
constexpr int kTriRB = 32;

// plan: first index of the cluster of every eigenvalue index (kept in the
// inverse-iteration scratch, free by now); grid (ceil(n/256), nprob)
__global__ void k_tri_plan(ProbDesc *probs, double gap_rel)
{
    const ProbDesc &P = probs[blockIdx.y];
    const int n = P.n;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double tn = fmax(fabs(P.w0[0]), fabs(P.w0[n - 1]));
    const double thr = gap_rel * fmax(tn, 1e-300);
    int cs = k;
    while (cs > 0 && P.w0[cs] - P.w0[cs - 1] <= thr) cs--;
    reinterpret_cast<int *>(P.tri)[k] = cs;
}

// block b > 0: member k (position in [kTriRB b, kTriRB (b+1))) against the
// members of the earlier blocks; grid (n, nprob), block 256
__global__ void __launch_bounds__(256) k_tri_proj(ProbDesc *probs, int b)
{
    const ProbDesc &P = probs[blockIdx.y];
    const int n = P.n;
    const int k = blockIdx.x;
    if (k >= n) return;
    const int cs = reinterpret_cast<const int *>(P.tri)[k];
    const int pos = k - cs;
    if (pos < kTriRB * b || pos >= kTriRB * (b + 1)) return;
    const int m = kTriRB * b;   // earlier members: cs .. cs + m - 1
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    __shared__ double coef[4096];
    double *zk = P.Z + (size_t)k * n;
    for (int pass = 0; pass < 2; pass++) {
        for (int q = wid; q < m; q += 4) {
            const double *zq = P.Z + (size_t)(cs + q) * n;
            double s = 0.0;
            for (int i = lane; i < n; i += 64) s += zq[i] * zk[i];
            s = wave_sum(s);
            if (lane == 0) coef[q] = s;
        }
        __syncthreads();
        for (int i = tid; i < n; i += 256) {
            double x = zk[i];
            for (int q = 0; q < m; q++) x -= coef[q] * P.Z[(size_t)(cs + q) * n + i];
            zk[i] = x;
        }
        __syncthreads();
    }
}

// block b inside: the work-group of the block's first member orthogonalises
// the block's members one after another and normalises them; grid (n, nprob)
__global__ void __launch_bounds__(256) k_tri_intra(ProbDesc *probs, int b)
{
    const ProbDesc &P = probs[blockIdx.y];
    const int n = P.n;
    const int k = blockIdx.x;
    if (k >= n) return;
    const int *plan = reinterpret_cast<const int *>(P.tri);
    const int cs = plan[k];
    if (k - cs != kTriRB * b) return;
    int end = k + 1;
    while (end < n && end < k + kTriRB && plan[end] == cs) end++;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    __shared__ double coef[kTriRB];
    __shared__ double red[4];
    for (int j = k; j < end; j++) {
        double *zj = P.Z + (size_t)j * n;
        for (int pass = 0; pass < 2 && j > k; pass++) {
            for (int q = k + wid; q < j; q += 4) {
                const double *zq = P.Z + (size_t)q * n;
                double s = 0.0;
                for (int i = lane; i < n; i += 64) s += zq[i] * zj[i];
                s = wave_sum(s);
                if (lane == 0) coef[q - k] = s;
            }
            __syncthreads();
            for (int i = tid; i < n; i += 256) {
                double x = zj[i];
                for (int q = k; q < j; q++) x -= coef[q - k] * P.Z[(size_t)q * n + i];
                zj[i] = x;
            }
            __syncthreads();
        }
        double s = 0.0;
        for (int i = tid; i < n; i += 256) s += zj[i] * zj[i];
        s = wave_sum(s);
        if (lane == 0) red[wid] = s;
        __syncthreads();
        s = red[0] + red[1] + red[2] + red[3];
        const double inv = (s > 0.0) ? 1.0 / sqrt(s) : 0.0;
        for (int i = tid; i < n; i += 256) zj[i] *= inv;
        if (s == 0.0 && tid == 0) zj[j] = 1.0;
        __syncthreads();
    }
}

// ----------------------------------------------------------- back-transform
// V0 = complex(Z); grid (ceil(n*n/256), nprob)
__global__ void k_init_v0(ProbDesc *probs)
{
    const ProbDesc &P = probs[blockIdx.y];
    const size_t nn = (size_t)P.n * P.n;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < nn; t += (size_t)gridDim.x * blockDim.x)
        st2(P.V0 + 2 * t, make_double2(P.Z[t], 0.0));
}

// Block-reflector factor T of every panel (forward, columnwise):
// T[i][i] = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] (Y_p[:, 0:i]^H y_i).
// grid (npanels, nprob), block 64 (one wave).
__global__ void k_larft(ProbDesc *probs)
{
    const ProbDesc &P = probs[blockIdx.y];
    const int n = P.n, p = blockIdx.x;
    const int k0 = p * kNB;
    if (k0 >= n - 1) return;
    const int nbw = min(kNB, n - 1 - k0);
    const int lane = threadIdx.x;
    double2 *T = reinterpret_cast<double2 *>(P.T) + (size_t)p * kNB * kNB;   // column-major nbw x nbw, ld NB
    const double2 *Y = reinterpret_cast<const double2 *>(P.Y);
    __shared__ double2 g[kNB];
    for (int q = lane; q < kNB * kNB; q += 64) T[q] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int i = 0; i < nbw; i++) {
        const int ci = k0 + i;
        const double2 tau = ld2(P.tau + 2 * ci);
        // g_j = y_j^H y_i for j < i (rows ci+1.. where y_i is nonzero)
        for (int j = 0; j < i; j++) {
            double2 s = make_double2(0.0, 0.0);
            for (int r = ci + 1 + lane; r < n; r += 64) s = cadd(s, cmulc(Y[(size_t)(k0 + j) * n + r], Y[(size_t)ci * n + r]));
            s = wave_sum2(s);
            if (lane == 0) g[j] = s;
        }
        __syncthreads();
        if (lane < i) {
            // T[lane, i] = -tau * sum_{j} T[lane, j] g_j   (T upper triangular, j >= lane)
            double2 s = make_double2(0.0, 0.0);
            for (int j = lane; j < i; j++) s = cadd(s, cmul(T[(size_t)j * kNB + lane], g[j]));
            T[(size_t)i * kNB + lane] = cmul(make_double2(-tau.x, -tau.y), s);
        }
        if (lane == 0) T[(size_t)i * kNB + i] = tau;
        __syncthreads();
    }
}

// 1 x 1 matrices: eigenvalue = diagonal, eigenvector = 1
__global__ void k_n1(ProbDesc *probs, int np)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const ProbDesc &P = probs[p];
    const double a = P.A[0];
    P.d[0] = a;
    P.w0[0] = a;
    P.Z[0] = 1.0;
    P.V0[0] = 1.0;
    P.V0[1] = 0.0;
}

__global__ void k_last_diag(ProbDesc *probs, int np)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const ProbDesc &P = probs[p];
    const int n = P.n;
    P.d[n - 1] = P.A[2 * ((size_t)(n - 1) * n + n - 1)];
}

// ===================================================================== host
static inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

size_t stage1_gemm_desc_count(int n, int np)
{
    const int npan = (n - 1 + kNB - 1) / kNB;
    return (size_t)np * (size_t)(4 * npan + 1);
}

// Fill the host array of GEMM descriptors: for panel p, slot 4p = her2k,
// 4p+1..4p+3 = the three back-transformation products.
void stage1_fill_gemm_descs(const ProbDesc *hp, int np, GemmDesc *out)
{
    const int n = hp[0].n;
    const int npan = (n - 1 + kNB - 1) / kNB;
    for (int p = 0; p < npan; p++) {
        const int k0 = p * kNB;
        const int nbw = std::min(kNB, n - 1 - k0);
        const int r0 = k0 + nbw;
        for (int q = 0; q < np; q++) {
            const ProbDesc &P = hp[q];
            GemmDesc *g = out + (size_t)(4 * p) * np + q;
            g->A = P.P + 2 * (size_t)r0;
            g->B = P.Q + 2 * (size_t)r0;
            g->C = P.A + 2 * ((size_t)r0 * n + r0);
            g->lda = n; g->ldb = n; g->ldc = n;
            g = out + (size_t)(4 * p + 1) * np + q;   // X = Yp^H V0[k0+1:, :]
            g->A = P.Y + 2 * ((size_t)k0 * n + k0 + 1);
            g->B = P.V0 + 2 * (size_t)(k0 + 1);
            g->C = P.X;
            g->lda = n; g->ldb = n; g->ldc = kNB;
            g = out + (size_t)(4 * p + 2) * np + q;   // X2 = T_p X
            g->A = P.T + 2 * (size_t)p * kNB * kNB;
            g->B = P.X;
            g->C = P.X2;
            g->lda = kNB; g->ldb = kNB; g->ldc = kNB;
            g = out + (size_t)(4 * p + 3) * np + q;   // V0[k0+1:, :] -= Yp X2
            g->A = P.Y + 2 * ((size_t)k0 * n + k0 + 1);
            g->B = P.X2;
            g->C = P.V0 + 2 * (size_t)(k0 + 1);
            g->lda = n; g->ldb = kNB; g->ldc = n;
        }
    }
}

int stage1_ingest(const Stage1Batch &B, hipStream_t st)
{
    const int n = B.n, np = B.nprob;
    ProbDesc *pd = B.dev_probs;
    if (n < 1 || np < 1) return 0;
    hipLaunchKernelGGL(k_ingest, dim3(n, np), dim3(256), 0, st, pd, B.fp32);
    if (n == 1) {
        hipLaunchKernelGGL(k_n1, dim3(cdiv(np, 64)), dim3(64), 0, st, pd, np);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// the per-column launches of the tridiagonalisation (n >= 2)
int stage1_trd(const Stage1Batch &B, hipStream_t st)
{
    auto gemm = B.fp32 ? k_cgemm32 : k_zgemm;
    const int n = B.n, np = B.nprob;
    ProbDesc *pd = B.dev_probs;
    const GemmDesc *gd = B.dev_gemm;
    if (n < 2 || np < 1) return 0;
    // ---- tridiagonalisation
    // large matrices: the per-column kernels spread each column over chunks of
    // 64 rows; smaller ones: one chunk per matrix (batches of them fill the
    // chip).  The choice depends on n only, so that a matrix's result does not
    // depend on the batch it runs in.
    const int crows = n >= 512 ? kColRows : ((n + 63) / 64) * 64;
    const int wrows = crows;
    const int npan = (n - 1 + kNB - 1) / kNB;
    for (int p = 0; p < npan; p++) {
        const int k0 = p * kNB;
        const int nbw = std::min(kNB, n - 1 - k0);
        hipLaunchKernelGGL(k_zero_panel, dim3(cdiv((size_t)2 * kNB * n * 2, 256), np), dim3(256), 0, st, pd);
        for (int i = 0; i < nbw; i++) {
            const int c = k0 + i;
            int idv = B.timer ? B.timer->begin(KC_TRD_VEC, 0.0, st) : -1;
            hipLaunchKernelGGL(k_trd_col, dim3(cdiv(n - c, crows), np), dim3(256), 0, st, pd, c, k0, crows);
            if (B.timer) B.timer->end(idv, st);
            const int m = n - c - 1;
            const int T = (m + 63) / 64;
            // algorithmic bytes: the lower triangle of A22 once (16 bytes per complex entry)
            const int id = B.timer ? B.timer->begin(KC_HEMV, 8.0 * (double)m * (m + 1) * np, st) : -1;
            hipLaunchKernelGGL(k_trd_hemv, dim3(T * (T + 1) / 2, np), dim3(256), 0, st, pd, c);
            if (B.timer) B.timer->end(id, st);
            idv = B.timer ? B.timer->begin(KC_TRD_VEC, 0.0, st) : -1;
            hipLaunchKernelGGL(k_trd_wfin, dim3(cdiv(m, wrows), np), dim3(256), 0, st, pd, c, k0, crows, wrows);
            if (B.timer) B.timer->end(idv, st);
        }
        const int r0 = k0 + nbw;
        const int m = n - r0;
        if (m > 0) {
            const unsigned tiles = cdiv(m, 32) * cdiv(m, 32);
            // algorithmic flops of the lower-triangle rank-2*nbw update: 8 nbw m (m+1)
            const int id = B.timer ? B.timer->begin(KC_HER2K, 8.0 * nbw * (double)m * (m + 1) * np, st) : -1;
            hipLaunchKernelGGL(gemm, dim3(tiles, np), dim3(256), 0, st, gd + (size_t)(4 * p) * np, m, m, 2 * kNB, 0, 1,
                               make_double2(-1.0, 0.0), make_double2(1.0, 0.0), 1);
            if (B.timer) B.timer->end(id, st);
        }
    }
    hipLaunchKernelGGL(k_last_diag, dim3(cdiv(np, 64)), dim3(64), 0, st, pd, np);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// tridiagonal eigen-solver and back-transformation (n >= 2, after the tridiagonalisation)
int stage1_solve(const Stage1Batch &B, hipStream_t st)
{
    auto gemm = B.fp32 ? k_cgemm32 : k_zgemm;
    const int n = B.n, np = B.nprob;
    ProbDesc *pd = B.dev_probs;
    const GemmDesc *gd = B.dev_gemm;
    if (n < 2 || np < 1) return 0;
    const int npan = (n - 1 + kNB - 1) / kNB;
    // ---- tridiagonal eigen-solver
    const int idt = B.timer ? B.timer->begin(KC_TRIDIAG, 0.0, st) : -1;
    hipLaunchKernelGGL(k_bisect, dim3(cdiv(n, 4), np), dim3(256), 0, st, pd);
    hipLaunchKernelGGL(k_invit, dim3(cdiv(n, 64), np), dim3(64), 0, st, pd);
    hipLaunchKernelGGL(k_transpose, dim3(cdiv(n, 16), cdiv(n, 16), np), dim3(16, 16), 0, st, pd);
    hipLaunchKernelGGL(k_tri_plan, dim3(cdiv(n, 256), np), dim3(256), 0, st, pd, B.tri_gap_rel);
    for (int b = 0; b < cdiv(n, kTriRB); b++) {
        if (b > 0) hipLaunchKernelGGL(k_tri_proj, dim3(n, np), dim3(256), 0, st, pd, b);
        hipLaunchKernelGGL(k_tri_intra, dim3(n, np), dim3(256), 0, st, pd, b);
    }
    if (B.timer) B.timer->end(idt, st);
    // ---- back-transformation
    const int idb = B.timer ? B.timer->begin(KC_BACKT, 8.0 * (double)n * n * n * np, st) : -1;
    hipLaunchKernelGGL(k_init_v0, dim3(cdiv((size_t)n * n, 256), np), dim3(256), 0, st, pd);
    hipLaunchKernelGGL(k_larft, dim3(npan, np), dim3(64), 0, st, pd);
    for (int p = npan - 1; p >= 0; p--) {
        const int k0 = p * kNB;
        const int nbw = std::min(kNB, n - 1 - k0);
        const int m = n - k0 - 1;
        hipLaunchKernelGGL(gemm, dim3(cdiv(nbw, 32) * cdiv(n, 32), np), dim3(256), 0, st, gd + (size_t)(4 * p + 1) * np,
                           nbw, n, m, 1, 0, make_double2(1.0, 0.0), make_double2(0.0, 0.0), 0);
        hipLaunchKernelGGL(gemm, dim3(cdiv(nbw, 32) * cdiv(n, 32), np), dim3(256), 0, st, gd + (size_t)(4 * p + 2) * np,
                           nbw, n, nbw, 0, 0, make_double2(1.0, 0.0), make_double2(0.0, 0.0), 0);
        hipLaunchKernelGGL(gemm, dim3(cdiv(m, 32) * cdiv(n, 32), np), dim3(256), 0, st, gd + (size_t)(4 * p + 3) * np,
                           m, n, nbw, 0, 0, make_double2(-1.0, 0.0), make_double2(1.0, 0.0), 0);
    }
    if (B.timer) B.timer->end(idb, st);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int stage1_run(const Stage1Batch &B, hipStream_t st)
{
    if (stage1_ingest(B, st)) return -1;
    if (B.n < 2) return 0;
    if (stage1_trd(B, st)) return -1;
    return stage1_solve(B, st);
}

}  // namespace zk
