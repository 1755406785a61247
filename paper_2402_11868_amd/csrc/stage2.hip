// Stage 2 of the method: Rayleigh quotient iteration in double-double (L=2)
// or quad-double (L=4) arithmetic that brings the binary64 eigenpairs to the
// working precision (Sec. 2, ZKCM_CUS paragraph: the iteration runs after the
// double-precision solver to regain the precision it lacks).  For each pair k:
//
//   v <- binary64 eigenvector, sigma <- v^H H v
//   repeat:  solve (H - sigma I) w = v     L limbs: Hermitian LDL^H with
//                                          Bunch-Kaufman pivoting (default) or
//                                          LU with partial pivoting
//            Gram-Schmidt w against the converged members of its eigenvalue
//            cluster and the lower-index members of the same iteration (twice)
//            v <- w / ||w||,  y = H v,  sigma <- v^H y,  r = y - sigma v
//   until ||r|| <= tol ||H||_2  (or the iteration limit / stagnation)
//
// Kernels (each launch covers the active pairs of a batch; the LDL^H
// factorisation may split them into two groups on two streams whose trailing
// updates alternate, stage2_solve_pair):
//   build      M = [H - sigma I | v], limb-planar
//   ldl_panel  one work-group per pair factorises its next panel (at most NB
//              columns, left-looking, symmetric interchanges), writes W = L D
//              column-major and forward-substitutes the right-hand side; a
//              memory-window form and a register-window form (the same steps
//              and results), chosen by order and pairs per launch
//   lu_panel   (LU) one work-group per pair factorises an n x NB panel
//   lu_trsm    (LU) applies the panel's row interchanges to the trailing
//              columns and computes U12 = L11^{-1} A12
//   lu_update  the O(n^3) part: A22 -= L21 W21^H on the lower triangle of
//              tiles (LDL^H) or A22 -= L21 U12 (LU); a 64x64 (dd) or 32x32
//              (qd) output tile per work-group, operands staged in LDS, every
//              product accumulated error-free into a (sum, compensation) pair
//   backsolve  w = P^T L^{-H} D^{-1} y (LDL^H) or w = U^{-1} y (LU), y the
//              transformed right-hand side (column n)
//   gs, rq     as above; rq also decides convergence on the device
#include <hip/hip_runtime.h>

#include "common.h"
#include "stage.h"

namespace zk {

// limb-planar accessors: plane (c*L + l), c = 0 real / 1 imaginary
template <int L>
__device__ __forceinline__ cmp<L> ld_cmp(const double *base, size_t plane, size_t idx)
{
    cmp<L> z;
    for (int l = 0; l < L; l++) {
        z.re.x[l] = base[(size_t)l * plane + idx];
        z.im.x[l] = base[(size_t)(L + l) * plane + idx];
    }
    return z;
}

template <int L>
__device__ __forceinline__ void st_cmp(double *base, size_t plane, size_t idx, const cmp<L> &z)
{
    for (int l = 0; l < L; l++) {
        base[(size_t)l * plane + idx] = z.re.x[l];
        base[(size_t)(L + l) * plane + idx] = z.im.x[l];
    }
}

// H(i, j) of a problem as an L-limb complex value (limb sum of the input planes)
template <int L>
__device__ __forceinline__ cmp<L> ld_h(const RqiProb &P, int i, int j)
{
    const size_t nn = (size_t)P.n * P.n, o = (size_t)j * P.n + i;
    cmp<L> z;
    z.re = mp_from<L>(P.hf[o]);
    z.im = mp_from<L>(P.hf[nn + o]);
    for (int l = 1; l < P.limbs_in; l++) {
        z.re = add_d(z.re, P.hf[(2 * l) * nn + o]);
        z.im = add_d(z.im, P.hf[(2 * l + 1) * nn + o]);
    }
    return z;
}

template <int L>
__device__ __forceinline__ mp<L> ld_sigma(const RqiProb &P, int k)
{
    mp<L> s;
    for (int l = 0; l < L; l++) s.x[l] = P.sigma[(size_t)l * P.n + k];
    return s;
}

// ----------------------------------------------------- error-free accumulator
// (S, C): S accumulates the leading products through TwoSum, C the exact
// product errors, the TwoSum errors and the cross terms.  The small terms of
// one product are summed first (the cross terms through two fused
// multiply-adds) and reach C in one addition, so C is rounded once per
// product.  One real product x*y of two double-doubles costs 12 binary64
// operations.
__device__ __forceinline__ void acc_dd(double &S, double &C, double xh, double xl, double yh, double yl)
{
    const double p = xh * yh;
    const double e = fma(xh, yh, -p);
    const double s = S + p;
    const double bb = s - S;
    const double t = (S - (s - bb)) + (p - bb);
    S = s;
    C += fma(xh, yl, fma(xl, yh, t + e));
}

__device__ __forceinline__ dd acc_dd_final(double S, double C)
{
    dd r;
    two_sum(S, C, r.x[0], r.x[1]);
    return r;
}

// complex multi-limb accumulator; the double-double form keeps (sum,
// compensation) pairs and costs 12 binary64 operations per real product
template <int L>
struct CAcc {
    cmp<L> v;
    __device__ void init(const cmp<L> &x) { v = x; }
    __device__ void add_mulc(const cmp<L> &a, const cmp<L> &b) { v = c_add(v, c_mulc(a, b)); }   // += conj(a) b
    __device__ void sub_mul(const cmp<L> &a, const cmp<L> &b) { v = c_sub(v, c_mul(a, b)); }     // -= a b
    __device__ cmp<L> get() const { return v; }
    __device__ void renorm() {}
};

template <>
struct CAcc<2> {
    double Sr, Cr, Si, Ci;
    __device__ void init(const cmp<2> &x) { Sr = x.re.x[0]; Cr = x.re.x[1]; Si = x.im.x[0]; Ci = x.im.x[1]; }
    __device__ void add_mulc(const cmp<2> &a, const cmp<2> &b)
    {
        // re += ar br + ai bi ; im += ar bi - ai br
        acc_dd(Sr, Cr, a.re.x[0], a.re.x[1], b.re.x[0], b.re.x[1]);
        acc_dd(Sr, Cr, a.im.x[0], a.im.x[1], b.im.x[0], b.im.x[1]);
        acc_dd(Si, Ci, a.re.x[0], a.re.x[1], b.im.x[0], b.im.x[1]);
        acc_dd(Si, Ci, -a.im.x[0], -a.im.x[1], b.re.x[0], b.re.x[1]);
    }
    __device__ void sub_mul(const cmp<2> &a, const cmp<2> &b)
    {
        // re -= ar br - ai bi ; im -= ar bi + ai br
        acc_dd(Sr, Cr, -a.re.x[0], -a.re.x[1], b.re.x[0], b.re.x[1]);
        acc_dd(Sr, Cr, a.im.x[0], a.im.x[1], b.im.x[0], b.im.x[1]);
        acc_dd(Si, Ci, -a.re.x[0], -a.re.x[1], b.im.x[0], b.im.x[1]);
        acc_dd(Si, Ci, -a.im.x[0], -a.im.x[1], b.re.x[0], b.re.x[1]);
    }
    __device__ cmp<2> get() const { return {acc_dd_final(Sr, Cr), acc_dd_final(Si, Ci)}; }
    // fold the compensation back into (sum, rounding error of the sum): in a
    // long sum with cancellation the compensation would otherwise grow with
    // the number of products, and so would its own rounding errors (about
    // K u^2 times the largest partial sum after K products)
    __device__ void renorm()
    {
        double h, l;
        two_sum(Sr, Cr, h, l);
        Sr = h;
        Cr = l;
        two_sum(Si, Ci, h, l);
        Si = h;
        Ci = l;
    }
};

// quad-double form: four-level cascaded sums (Casc4 in mp.h), renormalised
// once when the value is read
template <>
struct CAcc<4> {
    Casc4 re, im;
    __device__ void init(const cmp<4> &x)
    {
        re.init(x.re);
        im.init(x.im);
    }
    __device__ void add_mulc(const cmp<4> &a, const cmp<4> &b)
    {
        // re += ar br + ai bi ; im += ar bi - ai br
        re.add(a.re, b.re, 1.0);
        re.add(a.im, b.im, 1.0);
        im.add(a.re, b.im, 1.0);
        im.add(a.im, b.re, -1.0);
    }
    __device__ void sub_mul(const cmp<4> &a, const cmp<4> &b)
    {
        // re -= ar br - ai bi ; im -= ar bi + ai br
        re.add(a.re, b.re, -1.0);
        re.add(a.im, b.im, 1.0);
        im.add(a.re, b.im, -1.0);
        im.add(a.im, b.re, -1.0);
    }
    __device__ cmp<4> get() const { return cmp<4>{re.get(), im.get()}; }
    __device__ void renorm() {}
};

// ================================================================ init ====
// v_k <- binary64 eigenvector (exact), sigma_k <- binary64 eigenvalue.
// grid (npairs), block 256.
template <int L>
__global__ void k_s2_init(PairDesc *pairs, RqiProb *probs)
{
    PairDesc &Q = pairs[blockIdx.x];
    const RqiProb &P = probs[Q.prob];
    const int n = P.n, k = Q.k;
    const size_t nn = (size_t)n * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 z = ld2(P.V0 + 2 * ((size_t)k * P.ldv0 + i));
        cmp<L> c;
        c.re = mp_from<L>(z.x);
        c.im = mp_from<L>(z.y);
        st_cmp<L>(P.vec, nn, (size_t)k * n + i, c);
    }
    if (threadIdx.x == 0) {
        const mp<L> s = mp_from<L>(P.w0[k]);
        for (int l = 0; l < L; l++) P.sigma[(size_t)l * n + k] = s.x[l];
        Q.status = 0;
        Q.iters = 0;
        Q.flags = 0;
        Q.tiny = 0;
        Q.resid = INFINITY;
        Q.prev_resid = INFINITY;
    }
}

// ============================================================== normalise ==
template <int L>
__device__ void normalise_vec(double *vec, size_t nn, int n, int k, mp<L> *red)
{
    mp<L> s = mp_zero<L>();
    for (int i = threadIdx.x; i < n; i += blockDim.x) s = add(s, c_abs2(ld_cmp<L>(vec, nn, (size_t)k * n + i)));
    s = block_sum_mp<L>(s, red);
    if (!(s.x[0] > 0.0)) return;
    const mp<L> inv = div(mp_from<L>(1.0), sqrt_mp(s));
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const size_t o = (size_t)k * n + i;
        st_cmp<L>(vec, nn, o, c_scale(ld_cmp<L>(vec, nn, o), inv));
    }
    __syncthreads();
}

// ================================================================== RQ ====
// The double-double residual is accumulated with Casc3 (mp.h): the
// residual of an eigenvector of the largest eigenvalues (terms of size
// ||H|| / sqrt(n) cancelling down to 1e-32 ||H||) is then not limited by the
// ~sqrt(n) * 3 u^2 ||H|| rounding of plain double-double sums (~1e-30 at
// n = 1024).
// re/im of sum_j H(i, j) v_j (all input limbs) into two cascaded accumulators
__device__ __forceinline__ void hv_row_casc(const RqiProb &P, const double *vec, size_t nn, int n, int k, int i, Casc3 &re,
                                            Casc3 &im)
{
    for (int j = 0; j < n; j++) {
        const cmp<2> v = ld_cmp<2>(vec, nn, (size_t)k * n + j);
        const size_t o = (size_t)j * n + i;
        for (int l = 0; l < P.limbs_in; l++) {
            const double hr = P.hf[(2 * l) * nn + o], hi = P.hf[(2 * l + 1) * nn + o];
            re.add(hr, v.re.x[0], v.re.x[1]);
            re.add(-hi, v.im.x[0], v.im.x[1]);
            im.add(hr, v.im.x[0], v.im.x[1]);
            im.add(hi, v.re.x[0], v.re.x[1]);
        }
    }
}

constexpr int kRqRows = 4;   // rows per thread whose cascaded sums k_s2_rq keeps between its passes

// hv_row_casc for the rows i0 + 256 q (q < kRqRows, rows below n) in one pass
// over j: the same operations per row, the rows' sums independent of each
// other (so they overlap in the pipeline) and v_j loaded once for all of them
__device__ __forceinline__ void hv_rows_casc(const RqiProb &P, const double *vec, size_t nn, int n, int k, int i0,
                                             Casc3 *re, Casc3 *im)
{
    for (int j = 0; j < n; j++) {
        const cmp<2> v = ld_cmp<2>(vec, nn, (size_t)k * n + j);
        for (int l = 0; l < P.limbs_in; l++) {
#pragma unroll
            for (int q = 0; q < kRqRows; q++) {
                const int i = i0 + 256 * q;
                if (i < n) {
                    const size_t o = (size_t)j * n + i;
                    const double hr = P.hf[(2 * l) * nn + o], hi = P.hf[(2 * l + 1) * nn + o];
                    re[q].add(hr, v.re.x[0], v.re.x[1]);
                    re[q].add(-hi, v.im.x[0], v.im.x[1]);
                    im[q].add(hr, v.im.x[0], v.im.x[1]);
                    im[q].add(hi, v.re.x[0], v.re.x[1]);
                }
            }
        }
    }
}

// One work-group per active pair: y = H v, sigma = Re(v^H y), r = y - sigma v;
// convergence, stagnation and iteration-limit decisions.
template <int L>
__global__ void __launch_bounds__(256) k_s2_rq(PairDesc *pairs, RqiProb *probs, const int *active, int final_pass, int ldl)
{
    PairDesc &Q = pairs[active[blockIdx.x]];
    const RqiProb &P = probs[Q.prob];
    const int n = P.n, k = Q.k;
    const size_t nn = (size_t)n * n;
    __shared__ mp<L> red[16];
    __shared__ double redd[16];
    const double *vec = P.vec;
    mp<L> sigma;
    double r2 = 0.0;
    if constexpr (L == 2) {
        if (n <= 256 * kRqRows) {
            // the cascaded sums of pass 1 stay in registers (at most kRqRows rows
            // per thread) and pass 2 continues them: the same operations as the
            // recomputing form below, with one product H v instead of two
            Casc3 yr[kRqRows], yi[kRqRows];
            mp<2> sacc = mp_zero<2>();
            hv_rows_casc(P, vec, nn, n, k, threadIdx.x, yr, yi);
#pragma unroll
            for (int q = 0; q < kRqRows; q++) {
                const int i = threadIdx.x + 256 * q;
                if (i < n) {
                    const cmp<2> vi = ld_cmp<2>(vec, nn, (size_t)k * n + i);
                    dd a, b;
                    yr[q].get(a.x[0], a.x[1]);
                    yi[q].get(b.x[0], b.x[1]);
                    sacc = add(sacc, add(mul(vi.re, a), mul(vi.im, b)));
                }
            }
            sigma = block_sum_mp<2>(sacc, red);
#pragma unroll
            for (int q = 0; q < kRqRows; q++) {
                const int i = threadIdx.x + 256 * q;
                if (i < n) {
                    const cmp<2> vi = ld_cmp<2>(vec, nn, (size_t)k * n + i);
                    yr[q].add(-sigma.x[0], vi.re.x[0], vi.re.x[1]);
                    yr[q].add(-sigma.x[1], vi.re.x[0], vi.re.x[1]);
                    yi[q].add(-sigma.x[0], vi.im.x[0], vi.im.x[1]);
                    yi[q].add(-sigma.x[1], vi.im.x[0], vi.im.x[1]);
                    double a, b, lo;
                    yr[q].get(a, lo);
                    yi[q].get(b, lo);
                    r2 += a * a + b * b;
                }
            }
        } else {
            // pass 1: sigma = sum_i Re(conj(v_i) y_i), y_i from the cascaded sums
            mp<2> sacc = mp_zero<2>();
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                Casc3 yr, yi;
                hv_row_casc(P, vec, nn, n, k, i, yr, yi);
                const cmp<2> vi = ld_cmp<2>(vec, nn, (size_t)k * n + i);
                dd a, b;
                yr.get(a.x[0], a.x[1]);
                yi.get(b.x[0], b.x[1]);
                sacc = add(sacc, add(mul(vi.re, a), mul(vi.im, b)));
            }
            sigma = block_sum_mp<2>(sacc, red);
            // pass 2: r_i = sum_j H(i, j) v_j - sigma v_i in one cascaded sum per component
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                Casc3 rr, ri;
                hv_row_casc(P, vec, nn, n, k, i, rr, ri);
                const cmp<2> vi = ld_cmp<2>(vec, nn, (size_t)k * n + i);
                rr.add(-sigma.x[0], vi.re.x[0], vi.re.x[1]);
                rr.add(-sigma.x[1], vi.re.x[0], vi.re.x[1]);
                ri.add(-sigma.x[0], vi.im.x[0], vi.im.x[1]);
                ri.add(-sigma.x[1], vi.im.x[0], vi.im.x[1]);
                double a, b, lo;
                rr.get(a, lo);
                ri.get(b, lo);
                r2 += a * a + b * b;
            }
        }
    } else {
        // pass 1: sigma = sum_i Re(conj(v_i) y_i)
        mp<L> sacc = mp_zero<L>();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            CAcc<L> ya;
            ya.init(c_zero<L>());
            for (int j = 0; j < n; j++) {
                const cmp<L> h = ld_h<L>(P, i, j);
                ya.sub_mul(cmp<L>{mp_neg<L>(h.re), mp_neg<L>(h.im)}, ld_cmp<L>(vec, nn, (size_t)k * n + j));
            }
            const cmp<L> y = ya.get();
            const cmp<L> vi = ld_cmp<L>(vec, nn, (size_t)k * n + i);
            sacc = add(sacc, add(mul(vi.re, y.re), mul(vi.im, y.im)));
        }
        sigma = block_sum_mp<L>(sacc, red);
        // pass 2: ||y - sigma v||^2 (recomputes y to keep registers bounded)
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            // r_i = sum_j H(i, j) v_j - sigma v_i in one accumulation
            CAcc<L> ra;
            ra.init(c_zero<L>());
            for (int j = 0; j < n; j++) {
                const cmp<L> h = ld_h<L>(P, i, j);
                ra.sub_mul(cmp<L>{mp_neg<L>(h.re), mp_neg<L>(h.im)}, ld_cmp<L>(vec, nn, (size_t)k * n + j));
            }
            ra.sub_mul(cmp<L>{sigma, mp_zero<L>()}, ld_cmp<L>(vec, nn, (size_t)k * n + i));
            const cmp<L> r = ra.get();
            r2 += r.re.x[0] * r.re.x[0] + r.im.x[0] * r.im.x[0];
        }
    }
    r2 = block_sum(r2, redd);
    if (threadIdx.x == 0) {
        for (int l = 0; l < L; l++) P.sigma[(size_t)l * n + k] = sigma.x[l];
        const double res = sqrt(r2) / P.hnorm;
        Q.prev_resid = Q.resid;
        Q.resid = res;
        if (final_pass) {
            // after the global re-orthogonalisation: re-judge every pair
            const bool ok = (res == res) && res * P.hnorm <= P.tol_abs;
            Q.status = ok ? 1 : 2;
            Q.flags = ok ? (Q.flags | 1) : (Q.flags & ~1);
        } else if (!(res == res)) {
            Q.status = 2;
            Q.flags |= 8;
        } else if (res * P.hnorm <= 0.5 * P.tol_abs && Q.tiny < 2) {
            // internal target half the tolerance: the final
            // re-orthogonalisation may add a little to the residuals of the
            // pairs it touches (a pair pushed above gets polished).  A solve
            // with two or more tiny pivots (a degenerate eigenvalue) is never
            // the last: its vector can be good on its own yet nearly parallel
            // to its cluster partners, so the offset shift of k_s2_build
            // takes one more solve
            Q.status = 1;
            Q.flags |= 1;
        } else if (Q.iters >= P.max_iter) {
            Q.status = 2;
        } else if (Q.iters >= 2 && res > 0.5 * Q.prev_resid && res * P.hnorm <= 64.0 * P.tol_abs && Q.tiny < 2) {
            // the last solve did not halve the residual, which is near the
            // tolerance: the vector is at its rounding floor and more solves
            // would not move it (the final judgement decides, and a pair
            // that the re-orthogonalisation left above the tolerance is
            // polished).  Far above it a pair keeps iterating (up to
            // max_iter): inside a long chain its Gram-Schmidt partners still
            // move.  A pair whose LDL^H solves stalled above the tolerance
            // gets LU solves first (ZK_PAIR_LU_SOLVES): Bunch-Kaufman's
            // backward error, a few times LU's, can hold a residual just above
            if (ldl && !(Q.flags & 16) && res * P.hnorm > P.tol_abs) Q.flags |= 16;
            else Q.status = 2;
        }
    }
}

// =============================================================== build ====
// M = [H - sigma I | v] (LDL^H: the lower triangle and v); grid
// (ceil((n+1)/8), count), block 256.
template <int L>
__global__ void __launch_bounds__(256) k_s2_build(Stage2Batch B)
{
    const int t = blockIdx.y;
    PairDesc &Q = B.dev_pairs[B.dev_active[t]];
    const RqiProb &P = B.dev_probs[Q.prob];
    const int n = P.n, k = Q.k, ldm = lu_ldm_of(n);
    double *M = B.lu_base + (size_t)t * B.lu_stride;
    const size_t plane = lu_plane_of(n);
    const size_t nn = (size_t)n * n;
    mp<L> sigma = ld_sigma<L>(P, k);
    if (blockIdx.x == 0 && threadIdx.x == 0) {   // LDL^H: no panel factorised yet
        Q.lk0 = 0;
        Q.lkb = 0;
    }
    // Two or more tiny pivots in the pair's last factorisation: sigma sits on
    // an eigenvalue that is degenerate at working precision, and the pivots
    // of its eigenspace were rounding noise.  The solve then inverted a
    // random block (the LU's rounding, not the iterate, fixed the map on the
    // eigenspace), so the cluster's members collapse onto a few directions
    // and Gram-Schmidt has to separate nearly parallel vectors.  A shift
    // 2^20 guard thresholds away (far above that noise) makes the inverse on
    // the eigenspace the scalar -1/delta: each member keeps its own
    // orthogonal projection, and the rest of the spectrum is still damped by
    // delta / gap per solve.
    if (Q.tiny >= 2) sigma = add_d<L>(sigma, 1048576.0 * P.piv_tol);
    for (int jj = 0; jj < 8; jj++) {
        const int j = blockIdx.x * 8 + jj;
        if (j > n) break;
        // LDL^H reads the lower triangle only
        const int i0 = (B.ldl && j < n) ? j : 0;
        for (int i = i0 + threadIdx.x; i < n; i += blockDim.x) {
            cmp<L> z;
            if (j < n) {
                z = ld_h<L>(P, i, j);
                if (i == j) z.re = sub(z.re, sigma);
            } else {
                z = ld_cmp<L>(P.vec, nn, (size_t)k * n + i);
            }
            st_cmp<L>(M, plane, (size_t)j * ldm + i, z);
        }
    }
}

// ============================================================ LU panel ====
// One work-group (256) per pair: columns [k0, k0+nbw), rows [k0, n).
// Row interchanges are applied inside the panel only; lu_trsm applies them
// to the trailing columns.  The panel is factorised in sub-panels of
// kLuSub columns: a sub-panel first receives the deferred update from the
// columns left of it (its rows in the panel's top block by forward
// substitution with the unit lower factor, the rows below by one rank-s0
// update per row), then its columns are factorised right-looking inside
// the sub-panel only.  Each panel element is then read and written a few
// times instead of once per column step.  Interchanges swap the rows across
// all panel columns, so deferred columns are always in the current order.
constexpr int kLuSub = 8;

template <int L>
__global__ void __launch_bounds__(256) k_s2_lu_panel(Stage2Batch B, int k0, int nbw)
{
    const int t = blockIdx.x;
    PairDesc &Q = B.dev_pairs[B.dev_active[t]];
    const RqiProb &P = B.dev_probs[Q.prob];
    const int n = P.n, ldm = lu_ldm_of(n);
    if (k0 >= n) return;        // a launch of mixed orders: this pair's factorisation has ended
    nbw = min(nbw, n - k0);     // the pair's own panel width at this step
    double *M = B.lu_base + (size_t)t * B.lu_stride;
    int *ipiv = B.piv_base + (size_t)t * B.piv_stride;
    const size_t plane = lu_plane_of(n);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    __shared__ double smax[4];
    __shared__ int sidx[4];
    __shared__ int s_piv;
    __shared__ cmp<L> s_inv;
    __shared__ cmp<L> s_row[kLuSub];
    __shared__ cmp<L> sU[kLuNB][kLuSub];
    __shared__ int s_guard;
    __shared__ int s_tiny;
    if (tid == 0) s_guard = s_tiny = 0;
    for (int s0 = 0; s0 < nbw; s0 += kLuSub) {
        const int w = min(kLuSub, nbw - s0);
        if (s0 > 0) {
            // (a) rows [k0, k0+s0) of the sub-panel: U = L11^-1 A (unit lower L11)
            if (tid >= w && tid < kLuSub)
                for (int i = 0; i < s0; i++) sU[i][tid] = c_zero<L>();
            if (tid < w) {
                const size_t col = (size_t)(k0 + s0 + tid) * ldm;
                for (int i = 0; i < s0; i++) {
                    CAcc<L> x;
                    x.init(ld_cmp<L>(M, plane, col + k0 + i));
                    for (int q = 0; q < i; q++) x.sub_mul(ld_cmp<L>(M, plane, (size_t)(k0 + q) * ldm + k0 + i), sU[q][tid]);
                    const cmp<L> u = x.get();
                    sU[i][tid] = u;
                    st_cmp<L>(M, plane, col + k0 + i, u);
                }
            }
            __syncthreads();
            // (b) rows [k0+s0, n): A(r, c) -= sum_q L(r, q) U(q, c)
            for (int r = k0 + s0 + tid; r < n; r += 256) {
                CAcc<L> acc[kLuSub];
#pragma unroll
                for (int c = 0; c < kLuSub; c++)
                    acc[c].init(c < w ? ld_cmp<L>(M, plane, (size_t)(k0 + s0 + c) * ldm + r) : c_zero<L>());
                for (int q = 0; q < s0; q++) {
                    const cmp<L> l = ld_cmp<L>(M, plane, (size_t)(k0 + q) * ldm + r);
#pragma unroll
                    for (int c = 0; c < kLuSub; c++) acc[c].sub_mul(l, sU[q][c]);
                }
#pragma unroll
                for (int c = 0; c < kLuSub; c++)
                    if (c < w) st_cmp<L>(M, plane, (size_t)(k0 + s0 + c) * ldm + r, acc[c].get());
            }
            __syncthreads();
        }
        for (int jj = 0; jj < w; jj++) {
            const int c = k0 + s0 + jj;
            // pivot search
            double best = -1.0;
            int bidx = n;
            for (int r = c + tid; r < n; r += 256) {
                const double m = c_mag1(ld_cmp<L>(M, plane, (size_t)c * ldm + r));
                if (m > best) { best = m; bidx = r; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_xor(best, off, 64);
                const int oi = __shfl_xor(bidx, off, 64);
                if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
            }
            if (lane == 0) { smax[wid] = best; sidx[wid] = bidx; }
            __syncthreads();
            if (tid == 0) {
                double bb = smax[0];
                int bi = sidx[0];
                for (int q = 1; q < 4; q++)
                    if (smax[q] > bb || (smax[q] == bb && sidx[q] < bi)) { bb = smax[q]; bi = sidx[q]; }
                if (bi >= n) bi = c;
                s_piv = bi;
                ipiv[c] = bi;
            }
            __syncthreads();
            const int p = s_piv;
            // swap rows c and p across the whole panel
            if (p != c && tid < nbw) {
                const size_t oc = (size_t)(k0 + tid) * ldm + c, op = (size_t)(k0 + tid) * ldm + p;
                const cmp<L> x = ld_cmp<L>(M, plane, oc), y = ld_cmp<L>(M, plane, op);
                st_cmp<L>(M, plane, oc, y);
                st_cmp<L>(M, plane, op, x);
            }
            __syncthreads();
            if (tid == 0) {
                cmp<L> u = ld_cmp<L>(M, plane, (size_t)c * ldm + c);
                if (c_mag1(u) < 2048.0 * P.piv_tol) s_tiny++;
                if (c_mag1(u) < P.piv_tol) {
                    // zero-pivot guard: replace by the threshold, keeping the phase
                    const double sr = (u.re.x[0] < 0.0) ? -1.0 : 1.0;
                    u.re = mp_from<L>(sr * P.piv_tol);
                    u.im = mp_zero<L>();
                    st_cmp<L>(M, plane, (size_t)c * ldm + c, u);
                    s_guard = 1;
                }
                s_inv = c_recip<L>(u);
            }
            if (tid > 0 && tid < w - jj) s_row[tid] = ld_cmp<L>(M, plane, (size_t)(c + tid) * ldm + c);
            __syncthreads();
            const cmp<L> inv = s_inv;
            // scale the column and update the rest of the sub-panel (one row per thread)
            for (int r = c + 1 + tid; r < n; r += 256) {
                const cmp<L> l = c_mul(ld_cmp<L>(M, plane, (size_t)c * ldm + r), inv);
                st_cmp<L>(M, plane, (size_t)c * ldm + r, l);
                for (int q = 1; q < w - jj; q++) {
                    const size_t o = (size_t)(c + q) * ldm + r;
                    CAcc<L> x;
                    x.init(ld_cmp<L>(M, plane, o));
                    x.sub_mul(l, s_row[q]);
                    st_cmp<L>(M, plane, o, x.get());
                }
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        if (s_guard) Q.flags |= 4;
        // count of the whole factorisation (its first panel starts at zero)
        Q.tiny = (k0 == 0 ? 0 : Q.tiny) + s_tiny;
    }
}

// ============================================================= LU trsm ====
// Trailing columns j in [k0+nbw, n]: apply the panel's interchanges, then
// U12(:, j) = L11^{-1} A12(:, j).  Eight columns per work-group of 256, 32
// threads per column (one per row of the block): x_q is final at step q and
// broadcast by a wave shuffle, every other row subtracts l_rq x_q into its
// compensated accumulator.  grid (ceil(ncols/8), count).
template <int L>
__device__ __forceinline__ cmp<L> shfl_cmp(const cmp<L> &v, int src)
{
    cmp<L> r;
    for (int l = 0; l < L; l++) {
        r.re.x[l] = __shfl(v.re.x[l], src, 64);
        r.im.x[l] = __shfl(v.im.x[l], src, 64);
    }
    return r;
}

constexpr int kTrsmGroups = 4;   // groups of 8 columns per work-group (L11 loaded once)

template <int L>
__global__ void __launch_bounds__(256) k_s2_lu_trsm(Stage2Batch B, int k0, int nbw)
{
    const int t = blockIdx.y;
    const PairDesc &Q = B.dev_pairs[B.dev_active[t]];
    const RqiProb &P = B.dev_probs[Q.prob];
    const int n = P.n, ldm = lu_ldm_of(n);
    if (k0 >= n) return;
    nbw = min(nbw, n - k0);
    double *M = B.lu_base + (size_t)t * B.lu_stride;
    const int *ipiv = B.piv_base + (size_t)t * B.piv_stride;
    const size_t plane = lu_plane_of(n);
    __shared__ cmp<L> l11t[kLuNB][kLuNB];   // l11t[q][r] = L11(r, q)
    // the panel's interchanges as one permutation of at most 2 nbw rows:
    // row dst[i] receives the value of row src[i]
    __shared__ int s_dst[2 * kLuNB], s_src[2 * kLuNB];
    __shared__ int s_m;
    for (int e = threadIdx.x; e < nbw * nbw; e += 256) {
        const int r = e % nbw, q = e / nbw;
        if (r > q) l11t[q][r] = ld_cmp<L>(M, plane, (size_t)(k0 + q) * ldm + k0 + r);
    }
    if (threadIdx.x == 0) {
        int m = 0;
        // rows touched, with their current content (a row index of the original order)
        for (int r = 0; r < nbw; r++) {
            const int a = k0 + r, b = ipiv[k0 + r];
            if (a == b) continue;
            int ia = -1, ib = -1;
            for (int i = 0; i < m; i++) {
                if (s_dst[i] == a) ia = i;
                if (s_dst[i] == b) ib = i;
            }
            if (ia < 0) { s_dst[m] = a; s_src[m] = a; ia = m++; }
            if (ib < 0) { s_dst[m] = b; s_src[m] = b; ib = m++; }
            const int tmp = s_src[ia];
            s_src[ia] = s_src[ib];
            s_src[ib] = tmp;
        }
        s_m = m;
    }
    __syncthreads();
    const int m = s_m;
    const int cl = threadIdx.x >> 5, rr = threadIdx.x & 31, lane = threadIdx.x & 63;
    const int src0 = lane & 32;
    for (int grp = 0; grp < kTrsmGroups; grp++) {
        const int j = k0 + nbw + (blockIdx.x * kTrsmGroups + grp) * 8 + cl;
        const bool valid = j <= n;
        const size_t col = (size_t)j * ldm;
        // interchanges: gather every touched row's source, then scatter
        cmp<L> g0 = c_zero<L>(), g1 = c_zero<L>();
        if (valid) {
            if (rr < m) g0 = ld_cmp<L>(M, plane, col + s_src[rr]);
            if (rr + 32 < m) g1 = ld_cmp<L>(M, plane, col + s_src[rr + 32]);
        }
        __syncthreads();
        if (valid) {
            if (rr < m) st_cmp<L>(M, plane, col + s_dst[rr], g0);
            if (rr + 32 < m) st_cmp<L>(M, plane, col + s_dst[rr + 32], g1);
        }
        __syncthreads();
        CAcc<L> acc;
        acc.init((valid && rr < nbw) ? ld_cmp<L>(M, plane, col + k0 + rr) : c_zero<L>());
        cmp<L> x = c_zero<L>();
        for (int q = 0; q < nbw; q++) {
            const cmp<L> mine = acc.get();
            const cmp<L> xq = shfl_cmp<L>(mine, src0 + q);
            if (rr == q) x = mine;
            if (rr > q) acc.sub_mul(l11t[q][rr], xq);
        }
        if (valid && rr < nbw) st_cmp<L>(M, plane, col + k0 + rr, x);
    }
}

// =========================================================== LU update ====
// Output tile of a work-group: the LU covers the trailing block row-tile
// fastest (ti = x mod tilesI); the LDL^H only its lower triangle of tiles,
// enumerated row by row (tile q: ti (ti + 1) / 2 <= q < (ti + 1) (ti + 2) / 2).
template <bool LDL>
__device__ __forceinline__ bool tile_of(int mrows, int tsz, int &ti, int &tj)
{
    const int T = (mrows + tsz - 1) / tsz;
    const int q = blockIdx.x;
    if (!LDL) {
        ti = q % T;
        tj = q / T;
        return true;
    }
    if (q >= T * (T + 1) / 2) return false;
    int a = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
    while ((a + 1) * (a + 2) / 2 <= q) a++;
    while (a * (a + 1) / 2 > q) a--;
    ti = a;
    tj = q - a * (a + 1) / 2;
    return true;
}

// A22 -= L21 U12 for rows [r0, n), columns [r0, n] (r0 = k0 + nbw).
// dd: 64x64 tile per work-group of 256, 4x4 outputs per thread (rows
// tx + 16a, columns ty + 16b, so that the 16 lanes of a row group read and
// write 16 consecutive rows of a column), operands staged in LDS in chunks
// of KC (U12 staged with consecutive lanes along k, its unit-stride index).
constexpr int KC = 8;
constexpr int KCD = 4;   // k-chunk of the double-double update (256 threads stage 4 x 64 of L and U)

template <bool LDL>
__global__ void __launch_bounds__(256, 2) k_s2_lu_update_dd(Stage2Batch B, int k0, int nbw)
{
    const int t = blockIdx.y;
    const PairDesc &Q = B.dev_pairs[B.dev_active[t]];
    const int n = B.dev_probs[Q.prob].n, ldm = lu_ldm_of(n);
    if (LDL) {
        k0 = Q.lk0;
        nbw = Q.lkb;
        if (nbw <= 0) return;
    } else {
        if (k0 >= n) return;
        nbw = min(nbw, n - k0);
    }
    double *M = B.lu_base + (size_t)t * B.lu_stride;
    const size_t plane = lu_plane_of(n);
    const int r0 = k0 + nbw;
    const int jend = LDL ? n : n + 1;   // LU: the right-hand side column too
    const int mrows = n - r0, mcols = jend - r0;
    if (mrows <= 0) return;
    int ti, tj;
    if (!tile_of<LDL>(mrows, 64, ti, tj)) return;
    const int i0 = r0 + ti * 64, j0 = r0 + tj * 64;
    if (ti * 64 >= mrows || tj * 64 >= mcols) return;
    // LDL^H diagonal tile: its 16x16 sub-blocks above the diagonal (b > a) are not needed
    const bool diag = LDL && ti == tj;
    // 16-row groups of the tile that hold rows of the block (a tile of the
    // last tile row may hold fewer than 64; the groups past the end are skipped)
    const int amax = min(4, (n - i0 + 15) / 16);
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    // planes: 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo; two buffers: the next chunk
    // is loaded from global memory while the current one is multiplied
    __shared__ double sL[2][4][KCD][64];
    __shared__ double sU[2][4][KCD][64];
    double pL[4], pU[4];   // staging registers: one entry x 4 planes each
    auto fetch = [&](int kc) {
        {
            const int q = tid;
            {
                const int kk = q >> 6, ii = q & 63;
                const int kcol = k0 + kc + kk, gi = i0 + ii;
                const bool ok = kc + kk < nbw && gi < n;
                for (int pl = 0; pl < 4; pl++) pL[pl] = ok ? M[pl * plane + (size_t)kcol * ldm + gi] : 0.0;
            }
            if (LDL) {
                // U(c, j) = conj W(j, c), W column-major after the slot's working columns
                const int kk = q >> 6, jj = q & 63;
                const int gj = j0 + jj;
                const bool ok = kc + kk < nbw && gj < jend;
                const size_t o = (size_t)(ldl_wcol(n) + kc + kk) * ldm + gj;
                for (int pl = 0; pl < 4; pl++) pU[pl] = ok ? M[pl * plane + o] : 0.0;
                pU[2] = -pU[2];
                pU[3] = -pU[3];
            } else {
                const int kk = q & (KCD - 1), jj = q / KCD;
                const int kcol = k0 + kc + kk, gj = j0 + jj;
                const bool ok = kc + kk < nbw && gj < jend;
                for (int pl = 0; pl < 4; pl++) pU[pl] = ok ? M[pl * plane + (size_t)gj * ldm + kcol] : 0.0;
            }
        }
    };
    auto stash = [&](int buf) {
        const int q = tid;
        for (int pl = 0; pl < 4; pl++) {
            sL[buf][pl][q >> 6][q & 63] = pL[pl];
            if (LDL) sU[buf][pl][q >> 6][q & 63] = pU[pl];
            else sU[buf][pl][q & (KCD - 1)][q / KCD] = pU[pl];
        }
    };
    fetch(0);
    double S[4][4][2], C[4][4][2];   // [a][b][re/im]
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) {
            const int i = i0 + tx + 16 * a, j = j0 + ty + 16 * b;
            double rh = 0.0, rl = 0.0, ih = 0.0, il = 0.0;
            if (i < n && j < jend && !(diag && b > a)) {
                const size_t o = (size_t)j * ldm + i;
                rh = M[o]; rl = M[plane + o]; ih = M[2 * plane + o]; il = M[3 * plane + o];
            }
            S[a][b][0] = rh; C[a][b][0] = rl;
            S[a][b][1] = ih; C[a][b][1] = il;
        }
    stash(0);
    __syncthreads();
    int buf = 0;
    for (int kc = 0; kc < nbw; kc += KCD) {
        const bool more = kc + KCD < nbw;
        if (more) fetch(kc + KCD);
        const int kmax = min(KCD, nbw - kc);
        for (int kk = 0; kk < kmax; kk++) {
            double urh[4], url[4], uih[4], uil[4];
            for (int b = 0; b < 4; b++) {
                urh[b] = sU[buf][0][kk][ty + 16 * b]; url[b] = sU[buf][1][kk][ty + 16 * b];
                uih[b] = sU[buf][2][kk][ty + 16 * b]; uil[b] = sU[buf][3][kk][ty + 16 * b];
            }
            for (int a = 0; a < 4; a++) {
                if (a >= amax) continue;
                // negated L: the update subtracts
                const double lrh = -sL[buf][0][kk][tx + 16 * a], lrl = -sL[buf][1][kk][tx + 16 * a];
                const double lih = sL[buf][2][kk][tx + 16 * a], lil = sL[buf][3][kk][tx + 16 * a];
                for (int b = 0; b < 4; b++) {
                    if (diag && b > a) continue;
                    // re -= lr ur - li ui  ->  re += (-lr) ur + li ui
                    acc_dd(S[a][b][0], C[a][b][0], lrh, lrl, urh[b], url[b]);
                    acc_dd(S[a][b][0], C[a][b][0], lih, lil, uih[b], uil[b]);
                    // im -= lr ui + li ur  ->  im += (-lr) ui + (-li) ur
                    acc_dd(S[a][b][1], C[a][b][1], lrh, lrl, uih[b], uil[b]);
                    acc_dd(S[a][b][1], C[a][b][1], -lih, -lil, urh[b], url[b]);
                }
            }
        }
        if (more) stash(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) {
            const int i = i0 + tx + 16 * a, j = j0 + ty + 16 * b;
            if (i < n && j < jend && !(diag && b > a)) {
                const size_t o = (size_t)j * ldm + i;
                const dd re = acc_dd_final(S[a][b][0], C[a][b][0]);
                const dd im = acc_dd_final(S[a][b][1], C[a][b][1]);
                M[o] = re.x[0]; M[plane + o] = re.x[1];
                M[2 * plane + o] = im.x[0]; M[3 * plane + o] = im.x[1];
            }
        }
}

// Generic (quad-double) update: 32x32 tile, 2x2 outputs per thread.
template <int L, bool LDL>
__global__ void __launch_bounds__(256) k_s2_lu_update_gen(Stage2Batch B, int k0, int nbw)
{
    const int t = blockIdx.y;
    const PairDesc &Q = B.dev_pairs[B.dev_active[t]];
    const int n = B.dev_probs[Q.prob].n, ldm = lu_ldm_of(n);
    if (LDL) {
        k0 = Q.lk0;
        nbw = Q.lkb;
        if (nbw <= 0) return;
    } else {
        if (k0 >= n) return;
        nbw = min(nbw, n - k0);
    }
    double *M = B.lu_base + (size_t)t * B.lu_stride;
    const size_t plane = lu_plane_of(n);
    const int r0 = k0 + nbw;
    const int jend = LDL ? n : n + 1;
    const int mrows = n - r0, mcols = jend - r0;
    if (mrows <= 0) return;
    int ti, tj;
    if (!tile_of<LDL>(mrows, 32, ti, tj)) return;
    const int i0 = r0 + ti * 32, j0 = r0 + tj * 32;
    if (ti * 32 >= mrows || tj * 32 >= mcols) return;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    // LDL^H diagonal tile: the 16x16 sub-block above the diagonal (b > a) is
    // not needed; 16-row groups past the last row are skipped
    const bool diag = LDL && ti == tj;
    const int amax = min(2, (n - i0 + 15) / 16);
    __shared__ cmp<L> sL[KC][32];
    __shared__ cmp<L> sU[KC][32];
    // outputs (rows tx + 16a, columns ty + 16b): 16 lanes touch 16 consecutive rows
    CAcc<L> acc[2][2];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            const int i = i0 + tx + 16 * a, j = j0 + ty + 16 * b;
            acc[a][b].init((i < n && j < jend) ? ld_cmp<L>(M, plane, (size_t)j * ldm + i) : c_zero<L>());
        }
    for (int kc = 0; kc < nbw; kc += KC) {
        __syncthreads();
        for (int q = tid; q < KC * 32; q += 256) {
            {
                const int kk = q >> 5, ii = q & 31;
                const int kcol = k0 + kc + kk;
                sL[kk][ii] = (kc + kk < nbw && i0 + ii < n) ? ld_cmp<L>(M, plane, (size_t)kcol * ldm + i0 + ii) : c_zero<L>();
            }
            if (LDL) {
                const int kk = q >> 5, jj = q & 31;
                sU[kk][jj] = (kc + kk < nbw && j0 + jj < jend)
                                 ? c_conj<L>(ld_cmp<L>(M, plane, (size_t)(ldl_wcol(n) + kc + kk) * ldm + j0 + jj))
                                 : c_zero<L>();
            } else {
                const int kk = q & (KC - 1), jj = q / KC;
                const int kcol = k0 + kc + kk;
                sU[kk][jj] = (kc + kk < nbw && j0 + jj < jend) ? ld_cmp<L>(M, plane, (size_t)(j0 + jj) * ldm + kcol) : c_zero<L>();
            }
        }
        __syncthreads();
        const int kmax = min(KC, nbw - kc);
        for (int kk = 0; kk < kmax; kk++)
            for (int a = 0; a < 2; a++) {
                if (a >= amax) continue;
                for (int b = 0; b < 2; b++) {
                    if (diag && b > a) continue;
                    acc[a][b].sub_mul(sL[kk][tx + 16 * a], sU[kk][ty + 16 * b]);
                }
            }
    }
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            const int i = i0 + tx + 16 * a, j = j0 + ty + 16 * b;
            if (i < n && j < jend && !(diag && b > a)) st_cmp<L>(M, plane, (size_t)j * ldm + i, acc[a][b].get());
        }
}

// ========================================================= back-solve ====
// w = U^{-1} y, y = column n of the factorised augmented matrix; w is scaled
// by a power of two to max-norm ~1 and written as the new iterate of the pair.
// One work-group (256) per pair; y is updated in place.
template <int L>
__global__ void __launch_bounds__(256) k_s2_backsolve(Stage2Batch B)
{
    const int t = blockIdx.x;
    PairDesc &Q = B.dev_pairs[B.dev_active[t]];
    const RqiProb &P = B.dev_probs[Q.prob];
    const int n = P.n, ldm = lu_ldm_of(n), k = Q.k;
    double *M = B.lu_base + (size_t)t * B.lu_stride;
    const size_t plane = lu_plane_of(n);
    const size_t nn = (size_t)n * n;
    const size_t ycol = (size_t)n * ldm;
    __shared__ cmp<L> s_w;
    __shared__ double redd[16];
    for (int i = n - 1; i >= 0; i--) {
        if (threadIdx.x == 0) {
            const cmp<L> y = ld_cmp<L>(M, plane, ycol + i);
            const cmp<L> w = c_mul(y, c_recip<L>(ld_cmp<L>(M, plane, (size_t)i * ldm + i)));
            st_cmp<L>(M, plane, ycol + i, w);
            s_w = w;
        }
        __syncthreads();
        const cmp<L> w = s_w;
        for (int r = threadIdx.x; r < i; r += 256) {
            CAcc<L> x;
            x.init(ld_cmp<L>(M, plane, ycol + r));
            x.sub_mul(ld_cmp<L>(M, plane, (size_t)i * ldm + r), w);
            st_cmp<L>(M, plane, ycol + r, x.get());
        }
        __syncthreads();
    }
    double mx = 0.0;
    for (int r = threadIdx.x; r < n; r += 256) mx = fmax(mx, c_mag1(ld_cmp<L>(M, plane, ycol + r)));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) redd[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = fmax(fmax(redd[0], redd[1]), fmax(redd[2], redd[3]));
    int e = 0;
    if (mx > 0.0 && isfinite(mx)) frexp(mx, &e);
    for (int r = threadIdx.x; r < n; r += 256) {
        cmp<L> w = ld_cmp<L>(M, plane, ycol + r);
        w.re = ldexp_mp(w.re, -e);
        w.im = ldexp_mp(w.im, -e);
        st_cmp<L>(P.vec, nn, (size_t)k * n + r, w);
    }
    if (threadIdx.x == 0) Q.iters++;
}

// =========================================================== LDL^H ====
// Hermitian indefinite factorisation P (H - sigma I) P^T = L D L^H with
// Bunch-Kaufman pivoting (diagonal blocks of order 1 and 2; Bunch and
// Kaufman, Math. Comp. 31 (1977), with the |re| + |im| magnitude), blocked:
// one work-group factorises a panel of at most kLuNB columns left-looking,
// then the trailing update A22 -= L21 W21^H (W = L D) covers the lower
// triangle only, half the multiply-adds of the LU's A22 -= L21 U12.
// Storage of a pair's slot (n rows; columns 0 .. n+5+kLuNB):
//   lower triangle  A, then L below the diagonal blocks;
//   diagonal        D (2x2 blocks keep d21 at (k+1, k), where their unit L
//                   has a structural zero);
//   column n        right-hand side, forward-substituted as the columns are
//                   factorised (every row below a new column at once);
//   column n+1      the candidate pivot column when it is outside the window;
//   n+2 .. n+5      the panel's look-ahead window (Schur-complement columns);
//   n+6 ..          W = L D of the panel last factorised, column-major (its
//                   rows r > c for column c), read by the trailing update;
//   upper triangle  unused (the update's diagonal tiles write there).
// ipiv[k] >= 0: 1x1 block at k with rows k and ipiv[k] interchanged;
// ipiv[k] = -(p+1), ipiv[k+1] = kIpiv2nd: 2x2 block at (k, k+1) with rows
// k+1 and p interchanged.  An interchange reaches the current panel's
// columns, the right-hand side and the not yet factorised part only (rows of
// earlier panels' L keep their order), so the back-substitution undoes each
// panel's interchanges after that panel's columns; ipiv[n + k] = 1 marks the
// first column of a panel.  A panel never ends inside a 2x2 block: it stops
// one column short instead, so panel widths are per pair (PairDesc lk0, lkb).
constexpr int kIpiv2nd = -2147483647 - 1;
constexpr double kBkAlpha = 0.64038820320220756872767623199676;   // (1 + sqrt 17) / 8

// work-group arg-max over NT threads (largest value, smallest index on
// ties); every thread returns the result
template <int NT>
__device__ __forceinline__ void wg_argmax(double &v, int &i, double *sv, int *si)
{
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oi = __shfl_xor(i, off, 64);
        if (ov > v || (ov == v && oi < i)) {
            v = ov;
            i = oi;
        }
    }
    if (NT == 64) return;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        sv[threadIdx.x >> 6] = v;
        si[threadIdx.x >> 6] = i;
    }
    __syncthreads();
    v = sv[0];
    i = si[0];
    for (int q = 1; q < NT / 64; q++)
        if (sv[q] > v || (sv[q] == v && si[q] < i)) {
            v = sv[q];
            i = si[q];
        }
}

template <int L>
__device__ __forceinline__ void swap_cmp(double *M, size_t plane, size_t a, size_t b)
{
    const cmp<L> x = ld_cmp<L>(M, plane, a), y = ld_cmp<L>(M, plane, b);
    st_cmp<L>(M, plane, a, y);
    st_cmp<L>(M, plane, b, x);
}

// Row r of the panel's L columns c0 .. c0 + U - 1 (U = ldl_ldu<L>; columns
// past nk - 1 repeat column nk - 1 and are not used): the loads are issued
// together, so that one memory latency covers U columns of a Schur-complement
// sum (issued one by one, each column's load latency adds up along the sum).
template <int L>
constexpr int ldl_ldu() { return L == 2 ? 8 : 4; }

template <int L>
__device__ __forceinline__ void ldl_load_l(cmp<L> *lb, const double *M, size_t plane, int ldm, int k0, int c0, int nk, int r)
{
#pragma unroll
    for (int u = 0; u < ldl_ldu<L>(); u++) lb[u] = ld_cmp<L>(M, plane, (size_t)(k0 + min(c0 + u, nk - 1)) * ldm + r);
}

// one work-group (NT threads: 256, or one wave for small orders) per pair:
// the pair's next panel, from column lk0 + lkb.
// Left-looking with a look-ahead window: one pass over the panel's L columns
// forms the Schur-complement columns of the next kLdlLA columns at once
// (window vectors, rows [k, n)); each factorised column then updates the
// window's remaining vectors right-looking, so the panel's L is read about
// kLdlLA times less often than column by column.  A candidate pivot column
// inside the window is its window vector; one outside is formed from the
// stored matrix and the panel's L and W.
template <int L, int NT>
__global__ void __launch_bounds__(NT) k_s2_ldl_panel(Stage2Batch B)
{
    const int t = blockIdx.x;
    PairDesc &Q = B.dev_pairs[B.dev_active[t]];
    const RqiProb &P = B.dev_probs[Q.prob];
    const int n = P.n, ldm = lu_ldm_of(n);
    const int k0 = Q.lk0 + Q.lkb;
    __syncthreads();   // every thread has read the panel state before it changes
    if (k0 >= n) {
        if (threadIdx.x == 0) {
            Q.lk0 = n;
            Q.lkb = 0;
        }
        return;
    }
    double *M = B.lu_base + (size_t)t * B.lu_stride;
    int *ipiv = B.piv_base + (size_t)t * B.piv_stride;
    const size_t plane = lu_plane_of(n);
    const size_t bc = (size_t)n * ldm, xc = (size_t)(n + 1) * ldm, vc0 = (size_t)(n + 2) * ldm;
    const size_t wb = (size_t)ldl_wcol(n) * ldm;   // W column c - k0 at wb + (c - k0) ldm
    const int kend = min(k0 + kLuNB, n);
    const int tid = threadIdx.x;
    const double ptol = P.piv_tol;
    __shared__ cmp<L> s_wt[kLdlLA][kLuNB];
    __shared__ cmp<L> s_pj[2][kLdlLA];   // conj W(j, k) (and W(j, k+1)) of the window's later columns
    __shared__ double s_v[NT / 64 > 4 ? NT / 64 : 4];
    __shared__ int s_i[NT / 64 > 4 ? NT / 64 : 4];
    __shared__ int s_kstep, s_kp, s_stop;
    __shared__ mp<L> s_inv;
    __shared__ cmp<L> s_d21;
    __shared__ mp<L> s_d11, s_d22, s_idet;
    __shared__ cmp<L> s_y[2];
    int guard = 0, tiny = 0;   // thread 0's counts
    int wbase = k0, wend = k0;   // the window [wbase, wend); vector of column j at vc0 + (j - wbase) ldm
    int k = k0;
    while (k < kend) {
        const int nk = k - k0;
        if (k >= wend) {
            // refill: window vectors of columns [k, min(k + kLdlLA, kend)), rows [k, n)
            wbase = k;
            wend = min(k + kLdlLA, kend);
            const int nw = wend - wbase;
            for (int e = tid; e < nw * nk; e += NT) {
                const int j = e / nk, c = e - j * nk;
                s_wt[j][c] = c_conj<L>(ld_cmp<L>(M, plane, wb + (size_t)c * ldm + wbase + j));
            }
            __syncthreads();
            for (int r = k + tid; r < n; r += NT) {
                CAcc<L> a[kLdlLA];
#pragma unroll
                for (int j = 0; j < kLdlLA; j++) {
                    const int col = wbase + j;
                    cmp<L> z = c_zero<L>();
                    if (j < nw)
                        z = r >= col ? ld_cmp<L>(M, plane, (size_t)col * ldm + r)
                                     : c_conj<L>(ld_cmp<L>(M, plane, (size_t)r * ldm + col));
                    a[j].init(z);
                }
                for (int c = 0; c < nk; c++) {
                    const cmp<L> l = ld_cmp<L>(M, plane, (size_t)(k0 + c) * ldm + r);
#pragma unroll
                    for (int j = 0; j < kLdlLA; j++)
                        if (j < nw) a[j].sub_mul(l, s_wt[j][c]);
                }
#pragma unroll
                for (int j = 0; j < kLdlLA; j++)
                    if (j < nw) st_cmp<L>(M, plane, vc0 + (size_t)j * ldm + r, a[j].get());
            }
            __syncthreads();
        }
        const size_t vk = vc0 + (size_t)(k - wbase) * ldm;
        // pivot search in column k
        double best = -1.0;
        int bi = n;
        for (int r = k + 1 + tid; r < n; r += NT) {
            const double m = c_mag1(ld_cmp<L>(M, plane, vk + r));
            if (m > best) {
                best = m;
                bi = r;
            }
        }
        wg_argmax<NT>(best, bi, s_v, s_i);
        const double colmax = fmax(best, 0.0);
        const int imax = bi;
        const double absakk = fabs(ld_cmp<L>(M, plane, vk + k).re.x[0]);
        const bool cand = !(colmax < fmax(ptol, 1e-300) || absakk >= kBkAlpha * colmax);
        double rowmax = 0.0, absimax = 0.0;
        // the candidate's column: its window vector, or formed into column n+1
        const size_t xv = (cand && imax < wend) ? vc0 + (size_t)(imax - wbase) * ldm : xc;
        if (cand) {
            if (imax >= wend) {
                __syncthreads();
                if (tid < nk) s_wt[0][tid] = c_conj<L>(ld_cmp<L>(M, plane, wb + (size_t)tid * ldm + imax));
                __syncthreads();
                for (int r = k + tid; r < n; r += NT) {
                    CAcc<L> a;
                    a.init(r >= imax ? ld_cmp<L>(M, plane, (size_t)imax * ldm + r)
                                     : c_conj<L>(ld_cmp<L>(M, plane, (size_t)r * ldm + imax)));
                    for (int c = 0; c < nk; c++) a.sub_mul(ld_cmp<L>(M, plane, (size_t)(k0 + c) * ldm + r), s_wt[0][c]);
                    st_cmp<L>(M, plane, xc + r, a.get());
                }
                __syncthreads();
            }
            double rb = 0.0;
            int ri = 0;
            for (int r = k + tid; r < n; r += NT)
                if (r != imax) rb = fmax(rb, c_mag1(ld_cmp<L>(M, plane, xv + r)));
            wg_argmax<NT>(rb, ri, s_v, s_i);
            rowmax = rb;
            absimax = fabs(ld_cmp<L>(M, plane, xv + imax).re.x[0]);
        }
        if (tid == 0) {
            int kstep = 1, kp = k;
            if (cand) {
                if (absakk >= kBkAlpha * colmax * (colmax / rowmax)) kp = k;
                else if (absimax >= kBkAlpha * rowmax) kp = imax;
                else {
                    kstep = 2;
                    kp = imax;
                }
            }
            s_kstep = kstep;
            s_kp = kp;
            s_stop = (kstep == 2 && k + 1 >= kend) ? 1 : 0;
        }
        __syncthreads();
        const int kstep = s_kstep, kp = s_kp;
        if (s_stop) break;   // the 2x2 block opens the next panel
        const int kk = k + kstep - 1;
        // the block's pivot columns: v0 = column k, v1 = column k+1 (2x2)
        const size_t v0 = vk;
        const size_t v1 = (kstep == 2) ? (k + 1 < wend ? vk + ldm : xc) : vk;
        if (kp != kk) {
            const bool kp_in = kp < wend;
            // the panel's L rows and W rows, the right-hand side
            for (int c = tid; c < nk; c += NT) {
                swap_cmp<L>(M, plane, (size_t)(k0 + c) * ldm + kk, (size_t)(k0 + c) * ldm + kp);
                swap_cmp<L>(M, plane, wb + (size_t)c * ldm + kk, wb + (size_t)c * ldm + kp);
            }
            // stored part: column kk moves to row / column kp.  Needed for a
            // kp inside the window too: a candidate column formed later from
            // the stored matrix reads the window columns' stored rows
            for (int r = kk + 1 + tid; r < n; r += NT) {
                if (r < kp) st_cmp<L>(M, plane, (size_t)r * ldm + kp, c_conj<L>(ld_cmp<L>(M, plane, (size_t)kk * ldm + r)));
                else if (r > kp) st_cmp<L>(M, plane, (size_t)kp * ldm + r, ld_cmp<L>(M, plane, (size_t)kk * ldm + r));
            }
            // window vectors: column kk takes the candidate's vector, and a
            // candidate inside the window takes column kk's
            const size_t vkk = vc0 + (size_t)(kk - wbase) * ldm;
            if (kk < wend) {
                if (kp_in) {
                    const size_t vkp = vc0 + (size_t)(kp - wbase) * ldm;
                    for (int r = k + tid; r < n; r += NT) swap_cmp<L>(M, plane, vkk + r, vkp + r);
                } else {
                    for (int r = k + tid; r < n; r += NT) st_cmp<L>(M, plane, vkk + r, ld_cmp<L>(M, plane, xc + r));
                }
            }
            if (tid == 0) {
                swap_cmp<L>(M, plane, bc + kk, bc + kp);
                st_cmp<L>(M, plane, (size_t)kp * ldm + kp, ld_cmp<L>(M, plane, (size_t)kk * ldm + kk));
            }
            __syncthreads();
            // rows kk and kp of every live window vector (and of column n+1
            // when it is the 2x2 block's second column)
            const int nlive = wend - k;
            if (tid < nlive) swap_cmp<L>(M, plane, vk + (size_t)tid * ldm + kk, vk + (size_t)tid * ldm + kp);
            if (tid == nlive && v1 == xc && kstep == 2) swap_cmp<L>(M, plane, xc + kk, xc + kp);
            __syncthreads();
        }
        const int j1 = k + kstep;   // first window column after the block
        if (tid == 0) {
            if (kstep == 1) {
                mp<L> d = ld_cmp<L>(M, plane, v0 + k).re;
                if (fabs(d.x[0]) < 2048.0 * ptol) tiny++;
                if (fabs(d.x[0]) < ptol) {
                    d = mp_from<L>(d.x[0] < 0.0 ? -ptol : ptol);
                    guard = 1;
                }
                s_inv = div(mp_from<L>(1.0), d);
                cmp<L> dz;
                dz.re = d;
                dz.im = mp_zero<L>();
                st_cmp<L>(M, plane, (size_t)k * ldm + k, dz);
                ipiv[k] = kp;
                s_y[0] = ld_cmp<L>(M, plane, bc + k);
            } else {
                const mp<L> d11 = ld_cmp<L>(M, plane, v0 + k).re;
                const mp<L> d22 = ld_cmp<L>(M, plane, v1 + k + 1).re;
                const cmp<L> d21 = ld_cmp<L>(M, plane, v0 + k + 1);
                const mp<L> det = sub(mul(d11, d22), c_abs2(d21));
                s_d11 = d11;
                s_d22 = d22;
                s_d21 = d21;
                s_idet = div(mp_from<L>(1.0), det);
                // tiny-eigenvalue count of the block (binary64 estimate)
                const double a = d11.x[0], b = d22.x[0];
                const double big = fabs(0.5 * (a + b)) + sqrt(0.25 * (a - b) * (a - b) + c_mag1(d21) * c_mag1(d21));
                if (big > 0.0 && fabs(det.x[0]) / big < 2048.0 * ptol) tiny++;
                cmp<L> z;
                z.re = d11;
                z.im = mp_zero<L>();
                st_cmp<L>(M, plane, (size_t)k * ldm + k, z);
                z.re = d22;
                st_cmp<L>(M, plane, (size_t)(k + 1) * ldm + k + 1, z);
                st_cmp<L>(M, plane, (size_t)k * ldm + k + 1, d21);
                ipiv[k] = -(kp + 1);
                ipiv[k + 1] = kIpiv2nd;
                s_y[0] = ld_cmp<L>(M, plane, bc + k);
                s_y[1] = ld_cmp<L>(M, plane, bc + k + 1);
            }
            for (int q = 0; q < kstep; q++) ipiv[n + k + q] = (k + q == k0) ? 1 : 0;
        }
        // W(j, k) (and W(j, k+1)) of the window's later columns j
        if (tid < wend - j1) {
            s_pj[0][tid] = c_conj<L>(ld_cmp<L>(M, plane, v0 + j1 + tid));
            if (kstep == 2) s_pj[1][tid] = c_conj<L>(ld_cmp<L>(M, plane, v1 + j1 + tid));
        }
        __syncthreads();
        const int nl = max(0, wend - j1);
        const size_t vj1 = vc0 + (size_t)(j1 - wbase) * ldm;
        if (kstep == 1) {
            const mp<L> inv = s_inv;
            const cmp<L> y = s_y[0];
            for (int r = j1 + tid; r < n; r += NT) {
                const cmp<L> w = ld_cmp<L>(M, plane, v0 + r);
                const cmp<L> l = c_scale(w, inv);
                st_cmp<L>(M, plane, (size_t)k * ldm + r, l);
                st_cmp<L>(M, plane, wb + (size_t)nk * ldm + r, w);
                CAcc<L> b;
                b.init(ld_cmp<L>(M, plane, bc + r));
                b.sub_mul(l, y);
                st_cmp<L>(M, plane, bc + r, b.get());
                for (int j = 0; j < nl; j++) {
                    const size_t o = vj1 + (size_t)j * ldm + r;
                    CAcc<L> v;
                    v.init(ld_cmp<L>(M, plane, o));
                    v.sub_mul(l, s_pj[0][j]);
                    st_cmp<L>(M, plane, o, v.get());
                }
            }
        } else {
            const mp<L> d11 = s_d11, d22 = s_d22, idet = s_idet;
            const cmp<L> d21 = s_d21, y0 = s_y[0], y1 = s_y[1];
            for (int r = j1 + tid; r < n; r += NT) {
                const cmp<L> a = ld_cmp<L>(M, plane, v0 + r), b2 = ld_cmp<L>(M, plane, v1 + r);
                // [L(r,k) L(r,k+1)] = [a b2] D^{-1},  D^{-1} = [[d22, -conj d21], [-d21, d11]] / det
                const cmp<L> l0 = c_scale(c_sub(c_scale(a, d22), c_mul(b2, d21)), idet);
                const cmp<L> l1 = c_scale(c_sub(c_scale(b2, d11), c_mul(a, c_conj<L>(d21))), idet);
                st_cmp<L>(M, plane, (size_t)k * ldm + r, l0);
                st_cmp<L>(M, plane, (size_t)(k + 1) * ldm + r, l1);
                st_cmp<L>(M, plane, wb + (size_t)nk * ldm + r, a);
                st_cmp<L>(M, plane, wb + (size_t)(nk + 1) * ldm + r, b2);
                CAcc<L> b;
                b.init(ld_cmp<L>(M, plane, bc + r));
                b.sub_mul(l0, y0);
                b.sub_mul(l1, y1);
                st_cmp<L>(M, plane, bc + r, b.get());
                for (int j = 0; j < nl; j++) {
                    const size_t o = vj1 + (size_t)j * ldm + r;
                    CAcc<L> v;
                    v.init(ld_cmp<L>(M, plane, o));
                    v.sub_mul(l0, s_pj[0][j]);
                    v.sub_mul(l1, s_pj[1][j]);
                    st_cmp<L>(M, plane, o, v.get());
                }
            }
        }
        k += kstep;
        __syncthreads();
    }
    if (tid == 0) {
        Q.lk0 = k0;
        Q.lkb = k - k0;
        if (guard) Q.flags |= 4;
        Q.tiny = (k0 == 0 ? 0 : Q.tiny) + tiny;
    }
}

// Register-resident form of k_s2_ldl_panel (double-double, n - k0 <= NT R):
// the look-ahead window lives in registers.  Row r of the window is held by
// thread (r - wbase) % NT in slot (r - wbase) / NT, and after every block the
// window is shifted so that the current column is always vector 0: its
// right-looking updates, whole-column swaps and the pivot-column reads then
// touch no memory, and single elements (the pivot, interchanged rows, the
// window's W entries) pass through LDS.  Same steps and results as the
// memory form.
template <int NT, int R>
__global__ void __launch_bounds__(NT) k_s2_ldl_panel_reg(Stage2Batch B)
{
    constexpr int L = 2;
    const int t = blockIdx.x;
    PairDesc &Q = B.dev_pairs[B.dev_active[t]];
    const RqiProb &P = B.dev_probs[Q.prob];
    const int n = P.n, ldm = lu_ldm_of(n);
    const int k0 = Q.lk0 + Q.lkb;
    __syncthreads();   // every thread has read the panel state before it changes
    if (k0 >= n) {
        if (threadIdx.x == 0) {
            Q.lk0 = n;
            Q.lkb = 0;
        }
        return;
    }
    double *M = B.lu_base + (size_t)t * B.lu_stride;
    int *ipiv = B.piv_base + (size_t)t * B.piv_stride;
    const size_t plane = lu_plane_of(n);
    const size_t bc = (size_t)n * ldm, xc = (size_t)(n + 1) * ldm;
    const size_t wb = (size_t)ldl_wcol(n) * ldm;   // W column c - k0 at wb + (c - k0) ldm
    const int kend = min(k0 + kLuNB, n);
    const int tid = threadIdx.x;
    const double ptol = P.piv_tol;
    __shared__ cmp<L> s_wt[kLdlLA][kLuNB];
    __shared__ cmp<L> s_pj[2][kLdlLA];
    __shared__ cmp<L> s_ex[2][kLdlLA];   // rows kk and kp of the live window vectors
    __shared__ cmp<L> s_el[4];           // V0(k), V0(k+1), V1(k+1), candidate(imax)
    __shared__ double s_v[NT / 64 > 4 ? NT / 64 : 4];
    __shared__ int s_i[NT / 64 > 4 ? NT / 64 : 4];
    __shared__ int s_kstep, s_kp, s_stop;
    __shared__ mp<L> s_inv;
    __shared__ cmp<L> s_d21;
    __shared__ mp<L> s_d11, s_d22, s_idet;
    __shared__ cmp<L> s_y[2];
    int guard = 0, tiny = 0;   // thread 0's counts
    cmp<L> V[kLdlLA][R];
#pragma unroll
    for (int j = 0; j < kLdlLA; j++)
#pragma unroll
        for (int q = 0; q < R; q++) V[j][q] = c_zero<L>();
    int wbase = k0, wend = k0;
    // element (window vector j, slot q) with run-time j and q, for the owner thread
    auto vget = [&](int j, int q) {
        cmp<L> x = c_zero<L>();
#pragma unroll
        for (int jj = 0; jj < kLdlLA; jj++)
#pragma unroll
            for (int qq = 0; qq < R; qq++)
                if (jj == j && qq == q) x = V[jj][qq];
        return x;
    };
    auto vput = [&](int j, int q, const cmp<L> &x) {
#pragma unroll
        for (int jj = 0; jj < kLdlLA; jj++)
#pragma unroll
            for (int qq = 0; qq < R; qq++)
                if (jj == j && qq == q) V[jj][qq] = x;
    };
    int k = k0;
    while (k < kend) {
        const int nk = k - k0;
        if (k >= wend) {
            // refill: window vectors of columns [k, min(k + kLdlLA, kend)), rows [k, n)
            wbase = k;
            wend = min(k + kLdlLA, kend);
            const int nw = wend - wbase;
            for (int e = tid; e < nw * nk; e += NT) {
                const int j = e / nk, c = e - j * nk;
                s_wt[j][c] = c_conj<L>(ld_cmp<L>(M, plane, wb + (size_t)c * ldm + wbase + j));
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < R; q++) {
                const int r = wbase + tid + NT * q;
                CAcc<L> a[kLdlLA];
#pragma unroll
                for (int j = 0; j < kLdlLA; j++) {
                    const int col = wbase + j;
                    cmp<L> z = c_zero<L>();
                    if (r < n && j < nw)
                        z = r >= col ? ld_cmp<L>(M, plane, (size_t)col * ldm + r)
                                     : c_conj<L>(ld_cmp<L>(M, plane, (size_t)r * ldm + col));
                    a[j].init(z);
                }
                if (r < n)
                    for (int c0 = 0; c0 < nk; c0 += ldl_ldu<L>()) {
                        cmp<L> lb[ldl_ldu<L>()];
                        ldl_load_l<L>(lb, M, plane, ldm, k0, c0, nk, r);
#pragma unroll
                        for (int u = 0; u < ldl_ldu<L>(); u++)
                            if (c0 + u < nk)
#pragma unroll
                                for (int j = 0; j < kLdlLA; j++)
                                    if (j < nw) a[j].sub_mul(lb[u], s_wt[j][c0 + u]);
                    }
#pragma unroll
                for (int j = 0; j < kLdlLA; j++) V[j][q] = a[j].get();
            }
            __syncthreads();
        }
        const int live = wend - k;
        // pivot search in column k (vector 0)
        double best = -1.0;
        int bi = n;
#pragma unroll
        for (int q = 0; q < R; q++) {
            const int r = wbase + tid + NT * q;
            if (r > k && r < n) {
                const double m = c_mag1(V[0][q]);
                if (m > best) {
                    best = m;
                    bi = r;
                }
            }
        }
        if ((k - wbase) % NT == tid) s_el[0] = vget(0, (k - wbase) / NT);
        wg_argmax<NT>(best, bi, s_v, s_i);
        __syncthreads();
        const double colmax = fmax(best, 0.0);
        const int imax = bi;
        const double absakk = fabs(s_el[0].re.x[0]);
        const bool cand = !(colmax < fmax(ptol, 1e-300) || absakk >= kBkAlpha * colmax);
        const int jx = (cand && imax < wend) ? imax - k : -1;   // candidate in the window: vector jx
        double rowmax = 0.0, absimax = 0.0;
        if (cand) {
            if (jx < 0) {
                // the candidate column, formed into column n+1 from the stored matrix
                if (tid < nk) s_wt[0][tid] = c_conj<L>(ld_cmp<L>(M, plane, wb + (size_t)tid * ldm + imax));
                __syncthreads();
                for (int r = k + tid; r < n; r += NT) {
                    CAcc<L> a;
                    a.init(r >= imax ? ld_cmp<L>(M, plane, (size_t)imax * ldm + r)
                                     : c_conj<L>(ld_cmp<L>(M, plane, (size_t)r * ldm + imax)));
                    for (int c0 = 0; c0 < nk; c0 += ldl_ldu<L>()) {
                        cmp<L> lb[ldl_ldu<L>()];
                        ldl_load_l<L>(lb, M, plane, ldm, k0, c0, nk, r);
#pragma unroll
                        for (int u = 0; u < ldl_ldu<L>(); u++)
                            if (c0 + u < nk) a.sub_mul(lb[u], s_wt[0][c0 + u]);
                    }
                    st_cmp<L>(M, plane, xc + r, a.get());
                }
                __syncthreads();
            }
            double rb = 0.0;
            int ri = 0;
#pragma unroll
            for (int q = 0; q < R; q++) {
                const int r = wbase + tid + NT * q;
                if (r >= k && r < n && r != imax) {
                    cmp<L> x;
                    if (jx >= 0) {
                        x = c_zero<L>();
#pragma unroll
                        for (int jj = 1; jj < kLdlLA; jj++)
                            if (jj == jx) x = V[jj][q];
                    } else {
                        x = ld_cmp<L>(M, plane, xc + r);
                    }
                    rb = fmax(rb, c_mag1(x));
                }
            }
            if (jx >= 0 && (imax - wbase) % NT == tid) s_el[3] = vget(jx, (imax - wbase) / NT);
            if (jx < 0 && tid == 0) s_el[3] = ld_cmp<L>(M, plane, xc + imax);
            wg_argmax<NT>(rb, ri, s_v, s_i);
            __syncthreads();
            rowmax = rb;
            absimax = fabs(s_el[3].re.x[0]);
        }
        if (tid == 0) {
            int kstep = 1, kp = k;
            if (cand) {
                if (absakk >= kBkAlpha * colmax * (colmax / rowmax)) kp = k;
                else if (absimax >= kBkAlpha * rowmax) kp = imax;
                else {
                    kstep = 2;
                    kp = imax;
                }
            }
            s_kstep = kstep;
            s_kp = kp;
            s_stop = (kstep == 2 && k + 1 >= kend) ? 1 : 0;
        }
        __syncthreads();
        const int kstep = s_kstep, kp = s_kp;
        if (s_stop) break;   // the 2x2 block opens the next panel
        const int kk = k + kstep - 1;
        const bool v1_in = k + 1 < wend;   // the 2x2 block's second column is window vector 1 (else column n+1)
        if (kp != kk) {
            const bool kp_in = kp < wend;
            // the panel's L rows and W rows; the stored part: column kk moves to
            // row / column kp (also for kp inside the window: a candidate formed
            // later from the stored matrix reads the window columns' stored rows)
            for (int c = tid; c < nk; c += NT) {
                swap_cmp<L>(M, plane, (size_t)(k0 + c) * ldm + kk, (size_t)(k0 + c) * ldm + kp);
                swap_cmp<L>(M, plane, wb + (size_t)c * ldm + kk, wb + (size_t)c * ldm + kp);
            }
            for (int r = kk + 1 + tid; r < n; r += NT) {
                if (r < kp) st_cmp<L>(M, plane, (size_t)r * ldm + kp, c_conj<L>(ld_cmp<L>(M, plane, (size_t)kk * ldm + r)));
                else if (r > kp) st_cmp<L>(M, plane, (size_t)kp * ldm + r, ld_cmp<L>(M, plane, (size_t)kk * ldm + r));
            }
            if (tid == 0) {
                swap_cmp<L>(M, plane, bc + kk, bc + kp);
                st_cmp<L>(M, plane, (size_t)kp * ldm + kp, ld_cmp<L>(M, plane, (size_t)kk * ldm + kk));
            }
            // window vectors: column kk takes the candidate's vector, and a
            // candidate inside the window takes column kk's
            const int jkk = kk - k;
            if (kk < wend) {
                if (kp_in) {
                    const int jp = kp - k;
#pragma unroll
                    for (int a = 0; a < 2; a++)
#pragma unroll
                        for (int b = 1; b < kLdlLA; b++)
                            if (a == jkk && b == jp && a < b)
#pragma unroll
                                for (int q = 0; q < R; q++) {
                                    const cmp<L> x = V[a][q];
                                    V[a][q] = V[b][q];
                                    V[b][q] = x;
                                }
                } else {
#pragma unroll
                    for (int q = 0; q < R; q++) {
                        const int r = wbase + tid + NT * q;
                        if (r >= k && r < n) {
                            const cmp<L> x = ld_cmp<L>(M, plane, xc + r);
                            if (jkk == 0) V[0][q] = x;
                            else V[1][q] = x;
                        }
                    }
                }
            }
            // rows kk and kp of every live window vector, through LDS
            const int okk = (kk - wbase) % NT, skk = (kk - wbase) / NT;
            const int okp = (kp - wbase) % NT, skp = (kp - wbase) / NT;
            if (tid == okk)
                for (int j = 0; j < live; j++) s_ex[0][j] = vget(j, skk);
            if (tid == okp)
                for (int j = 0; j < live; j++) s_ex[1][j] = vget(j, skp);
            __syncthreads();
            if (tid == okk)
                for (int j = 0; j < live; j++) vput(j, skk, s_ex[1][j]);
            if (tid == okp)
                for (int j = 0; j < live; j++) vput(j, skp, s_ex[0][j]);
            if (tid == 0 && kstep == 2 && !v1_in) swap_cmp<L>(M, plane, xc + kk, xc + kp);
            __syncthreads();
        }
        const int j1 = k + kstep;   // first window column after the block
        // the pivot block's entries and W(j, k) (, W(j, k+1)) of the window's later columns
        if ((k - wbase) % NT == tid) s_el[0] = vget(0, (k - wbase) / NT);
        if (kstep == 2) {
            if ((k + 1 - wbase) % NT == tid) {
                s_el[1] = vget(0, (k + 1 - wbase) / NT);
                if (v1_in) s_el[2] = vget(1, (k + 1 - wbase) / NT);
            }
            if (!v1_in && tid == 0) s_el[2] = ld_cmp<L>(M, plane, xc + k + 1);
        }
        for (int j = kstep; j < live; j++) {
            const int r = k + j;
            if ((r - wbase) % NT == tid) {
                s_pj[0][j - kstep] = c_conj<L>(vget(0, (r - wbase) / NT));
                if (kstep == 2) s_pj[1][j - kstep] = c_conj<L>(vget(1, (r - wbase) / NT));
            }
        }
        __syncthreads();
        if (tid == 0) {
            if (kstep == 1) {
                mp<L> d = s_el[0].re;
                if (fabs(d.x[0]) < 2048.0 * ptol) tiny++;
                if (fabs(d.x[0]) < ptol) {
                    d = mp_from<L>(d.x[0] < 0.0 ? -ptol : ptol);
                    guard = 1;
                }
                s_inv = div(mp_from<L>(1.0), d);
                cmp<L> dz;
                dz.re = d;
                dz.im = mp_zero<L>();
                st_cmp<L>(M, plane, (size_t)k * ldm + k, dz);
                ipiv[k] = kp;
                s_y[0] = ld_cmp<L>(M, plane, bc + k);
            } else {
                const mp<L> d11 = s_el[0].re, d22 = s_el[2].re;
                const cmp<L> d21 = s_el[1];
                const mp<L> det = sub(mul(d11, d22), c_abs2(d21));
                s_d11 = d11;
                s_d22 = d22;
                s_d21 = d21;
                s_idet = div(mp_from<L>(1.0), det);
                const double a = d11.x[0], b = d22.x[0];
                const double big = fabs(0.5 * (a + b)) + sqrt(0.25 * (a - b) * (a - b) + c_mag1(d21) * c_mag1(d21));
                if (big > 0.0 && fabs(det.x[0]) / big < 2048.0 * ptol) tiny++;
                cmp<L> z;
                z.re = d11;
                z.im = mp_zero<L>();
                st_cmp<L>(M, plane, (size_t)k * ldm + k, z);
                z.re = d22;
                st_cmp<L>(M, plane, (size_t)(k + 1) * ldm + k + 1, z);
                st_cmp<L>(M, plane, (size_t)k * ldm + k + 1, d21);
                ipiv[k] = -(kp + 1);
                ipiv[k + 1] = kIpiv2nd;
                s_y[0] = ld_cmp<L>(M, plane, bc + k);
                s_y[1] = ld_cmp<L>(M, plane, bc + k + 1);
            }
            for (int q = 0; q < kstep; q++) ipiv[n + k + q] = (k + q == k0) ? 1 : 0;
        }
        __syncthreads();
        if (kstep == 1) {
            const mp<L> inv = s_inv;
            const cmp<L> y = s_y[0];
#pragma unroll
            for (int q = 0; q < R; q++) {
                const int r = wbase + tid + NT * q;
                if (r >= j1 && r < n) {
                    const cmp<L> w = V[0][q];
                    const cmp<L> l = c_scale(w, inv);
                    st_cmp<L>(M, plane, (size_t)k * ldm + r, l);
                    st_cmp<L>(M, plane, wb + (size_t)nk * ldm + r, w);
                    CAcc<L> b;
                    b.init(ld_cmp<L>(M, plane, bc + r));
                    b.sub_mul(l, y);
                    st_cmp<L>(M, plane, bc + r, b.get());
#pragma unroll
                    for (int j = 1; j < kLdlLA; j++)
                        if (j < live) {
                            CAcc<L> v;
                            v.init(V[j][q]);
                            v.sub_mul(l, s_pj[0][j - 1]);
                            V[j][q] = v.get();
                        }
                }
            }
#pragma unroll
            for (int q = 0; q < R; q++) {
                V[0][q] = V[1][q];
                V[1][q] = V[2][q];
                V[2][q] = V[3][q];
            }
        } else {
            const mp<L> d11 = s_d11, d22 = s_d22, idet = s_idet;
            const cmp<L> d21 = s_d21, y0 = s_y[0], y1 = s_y[1];
#pragma unroll
            for (int q = 0; q < R; q++) {
                const int r = wbase + tid + NT * q;
                if (r >= j1 && r < n) {
                    const cmp<L> a = V[0][q];
                    const cmp<L> b2 = v1_in ? V[1][q] : ld_cmp<L>(M, plane, xc + r);
                    const cmp<L> l0 = c_scale(c_sub(c_scale(a, d22), c_mul(b2, d21)), idet);
                    const cmp<L> l1 = c_scale(c_sub(c_scale(b2, d11), c_mul(a, c_conj<L>(d21))), idet);
                    st_cmp<L>(M, plane, (size_t)k * ldm + r, l0);
                    st_cmp<L>(M, plane, (size_t)(k + 1) * ldm + r, l1);
                    st_cmp<L>(M, plane, wb + (size_t)nk * ldm + r, a);
                    st_cmp<L>(M, plane, wb + (size_t)(nk + 1) * ldm + r, b2);
                    CAcc<L> b;
                    b.init(ld_cmp<L>(M, plane, bc + r));
                    b.sub_mul(l0, y0);
                    b.sub_mul(l1, y1);
                    st_cmp<L>(M, plane, bc + r, b.get());
#pragma unroll
                    for (int j = 2; j < kLdlLA; j++)
                        if (j < live) {
                            CAcc<L> v;
                            v.init(V[j][q]);
                            v.sub_mul(l0, s_pj[0][j - 2]);
                            v.sub_mul(l1, s_pj[1][j - 2]);
                            V[j][q] = v.get();
                        }
                }
            }
#pragma unroll
            for (int q = 0; q < R; q++) {
                V[0][q] = V[2][q];
                V[1][q] = V[3][q];
            }
        }
        k += kstep;
        __syncthreads();
    }
    if (tid == 0) {
        Q.lk0 = k0;
        Q.lkb = k - k0;
        if (guard) Q.flags |= 4;
        Q.tiny = (k0 == 0 ? 0 : Q.tiny) + tiny;
    }
}

// work-group sum of a complex multi-limb value over NT threads (thread 0
// returns it)
template <int L, int NT>
__device__ __forceinline__ cmp<L> wg_sum(cmp<L> v, cmp<L> *red)
{
    for (int off = 32; off > 0; off >>= 1) {
        cmp<L> o;
        for (int l = 0; l < L; l++) {
            o.re.x[l] = __shfl_xor(v.re.x[l], off, 64);
            o.im.x[l] = __shfl_xor(v.im.x[l], off, 64);
        }
        v = c_add(v, o);
    }
    if (NT == 64) return v;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    cmp<L> t = red[0];
    for (int q = 1; q < NT / 64; q++) t = c_add(t, red[q]);
    return t;
}

// x = P^T L^{-H} D^{-1} y (y = column n after the factorisation), scaled by a
// power of two to max-norm ~1 and written as the pair's new iterate.  One
// work-group (256) per pair; column n is overwritten.
template <int L, int NT>
__global__ void __launch_bounds__(NT) k_s2_ldl_backsolve(Stage2Batch B)
{
    const int t = blockIdx.x;
    PairDesc &Q = B.dev_pairs[B.dev_active[t]];
    const RqiProb &P = B.dev_probs[Q.prob];
    const int n = P.n, ldm = lu_ldm_of(n), k = Q.k;
    double *M = B.lu_base + (size_t)t * B.lu_stride;
    const int *ipiv = B.piv_base + (size_t)t * B.piv_stride;
    const size_t plane = lu_plane_of(n);
    const size_t nn = (size_t)n * n;
    const size_t yc = (size_t)n * ldm;
    __shared__ cmp<L> red[4];
    __shared__ double redd[4];
    // z = D^{-1} y
    for (int i = threadIdx.x; i < n; i += NT) {
        const int p = ipiv[i];
        if (p >= 0) {
            const mp<L> d = ld_cmp<L>(M, plane, (size_t)i * ldm + i).re;
            st_cmp<L>(M, plane, yc + i, c_scale(ld_cmp<L>(M, plane, yc + i), div(mp_from<L>(1.0), d)));
        } else if (p != kIpiv2nd) {
            const mp<L> d11 = ld_cmp<L>(M, plane, (size_t)i * ldm + i).re;
            const mp<L> d22 = ld_cmp<L>(M, plane, (size_t)(i + 1) * ldm + i + 1).re;
            const cmp<L> d21 = ld_cmp<L>(M, plane, (size_t)i * ldm + i + 1);
            const mp<L> idet = div(mp_from<L>(1.0), sub(mul(d11, d22), c_abs2(d21)));
            const cmp<L> y0 = ld_cmp<L>(M, plane, yc + i), y1 = ld_cmp<L>(M, plane, yc + i + 1);
            st_cmp<L>(M, plane, yc + i, c_scale(c_sub(c_scale(y0, d22), c_mul(c_conj<L>(d21), y1)), idet));
            st_cmp<L>(M, plane, yc + i + 1, c_scale(c_sub(c_scale(y1, d11), c_mul(d21, y0)), idet));
        }
    }
    __syncthreads();
    // L^H x = z, last column first; a panel's interchanges are undone once
    // its first column is done
    int pend = n;
    for (int i = n - 1; i >= 0;) {
        const bool two = ipiv[i] == kIpiv2nd;   // (i-1, i) is a 2x2 block: L(i, i-1) = 0
        const int c0 = two ? i - 1 : i;
        CAcc<L> a0, a1;
        a0.init(c_zero<L>());
        a1.init(c_zero<L>());
        for (int r = i + 1 + threadIdx.x; r < n; r += NT) {
            const cmp<L> x = ld_cmp<L>(M, plane, yc + r);
            a0.add_mulc(ld_cmp<L>(M, plane, (size_t)i * ldm + r), x);
            if (two) a1.add_mulc(ld_cmp<L>(M, plane, (size_t)c0 * ldm + r), x);
        }
        const cmp<L> s0 = wg_sum<L, NT>(a0.get(), red);
        cmp<L> s1 = c_zero<L>();
        if (two) {
            __syncthreads();
            s1 = wg_sum<L, NT>(a1.get(), red);
        }
        if (threadIdx.x == 0) {
            st_cmp<L>(M, plane, yc + i, c_sub(ld_cmp<L>(M, plane, yc + i), s0));
            if (two) st_cmp<L>(M, plane, yc + c0, c_sub(ld_cmp<L>(M, plane, yc + c0), s1));
            if (ipiv[n + c0] == 1) {
                for (int j = pend - 1; j >= c0; j--) {
                    const int p = ipiv[j];
                    if (p == kIpiv2nd) {
                        swap_cmp<L>(M, plane, yc + j, yc + (-ipiv[j - 1] - 1));
                        j--;
                    } else if (p >= 0 && p != j) {
                        swap_cmp<L>(M, plane, yc + j, yc + p);
                    }
                }
            }
        }
        if (ipiv[n + c0] == 1) pend = c0;
        __syncthreads();
        i = c0 - 1;
    }
    double mx = 0.0;
    for (int r = threadIdx.x; r < n; r += NT) mx = fmax(mx, c_mag1(ld_cmp<L>(M, plane, yc + r)));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) redd[threadIdx.x >> 6] = mx;
    __syncthreads();
    for (int q = 0; q < NT / 64; q++) mx = fmax(mx, redd[q]);
    int e = 0;
    if (mx > 0.0 && isfinite(mx)) frexp(mx, &e);
    for (int r = threadIdx.x; r < n; r += NT) {
        cmp<L> w = ld_cmp<L>(M, plane, yc + r);
        w.re = ldexp_mp(w.re, -e);
        w.im = ldexp_mp(w.im, -e);
        st_cmp<L>(P.vec, nn, (size_t)k * n + r, w);
    }
    if (threadIdx.x == 0) Q.iters++;
}

// ============================================================= output ====
// Pair k of a matrix goes to output position dst[pair]; limbs copied as is.
// grid (npairs), block 256.
template <int L>
__global__ void k_s2_output(PairDesc *pairs, RqiProb *probs, const int *dst)
{
    const int g = blockIdx.x;
    const PairDesc &Q = pairs[g];
    const RqiProb &P = probs[Q.prob];
    const int n = P.n, k = Q.k, pos = dst[g];
    const size_t nn = (size_t)n * n;
    if (threadIdx.x < L && P.w_out[threadIdx.x]) P.w_out[threadIdx.x][pos] = P.sigma[(size_t)threadIdx.x * n + k];
    if (!P.v_out[0]) return;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const cmp<L> z = ld_cmp<L>(P.vec, nn, (size_t)k * n + i);
        for (int l = 0; l < L; l++)
            st2(P.v_out[l] + 2 * ((size_t)pos * P.ldv_out + i), make_double2(z.re.x[l], z.im.x[l]));
    }
}

// ====================================================== Gram-Schmidt ====
// Block classical Gram-Schmidt in index order over a list of vector columns.
// For a cluster the list is [converged members..., active members in index
// order]; the converged prefix is left untouched and every active member is
// made orthogonal (twice) to everything before it in the list: the converged
// members and the active members of lower index.  The same kernels, with a
// list of all columns of a matrix and an empty prefix, re-orthogonalise a
// whole eigenbasis.  Blocks of RB active members: the block is projected
// against all earlier entries (coefficients by 16x16 tiles, then the update),
// then orthonormalised inside the block by Cholesky QR applied twice: the
// block's Gram matrix (row slices summed in a fixed order), its Cholesky factor
// R and R^-1 in L limbs, V <- V R^-1.  In exact arithmetic this is the same
// basis as Gram-Schmidt in index order (R has a positive diagonal).  When a
// pivot shows a member within 1e-8 (angle) of the span of the earlier ones --
// two members that converged to the same vector -- the block falls back to
// modified Gram-Schmidt (twice), which separates such members.
constexpr int RB = 32;
constexpr int RBP = RB * (RB + 1) / 2;   // packed upper triangle, column by column
__device__ __forceinline__ int pk(int a, int c) { return c * (c + 1) / 2 + a; }

// Row slices of the coefficient dot products: a cluster of order n splits its
// n rows into gs_slices(n) slices; each slice writes its partial sums into its
// own plane set of the cluster's scratch and k_gs_dsum adds them in slice
// order.
template <int L>
__global__ void __launch_bounds__(256) k_gs_dot(const GsCluster *cls, const int *list, const RqiProb *probs, int b,
                                                double *scratch)
{
    const GsCluster C = cls[blockIdx.z];
    const int j0 = C.nconv + b * RB, bw = min(RB, C.nact - b * RB);
    if (bw <= 0 || j0 == 0) return;
    const int tile = blockIdx.x / kGsSlices, slice = blockIdx.x % kGsSlices;
    if (tile * 16 >= j0 || blockIdx.y * 16 >= bw) return;
    const RqiProb &P = probs[C.prob];
    const int n = P.n;
    const int kd = gs_slices(n);
    if (slice >= kd) return;
    const int rc = ((n + kd - 1) / kd + 15) / 16 * 16;
    const int rbeg = slice * rc, rend = min(n, rbeg + rc);
    const size_t nn = (size_t)n * n;
    const int *lst = list + C.off;
    const size_t cplane = (size_t)C.size * RB;
    double *Cm = scratch + C.sofs + (size_t)slice * 2 * L * cplane;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i = tile * 16 + ty, jb = blockIdx.y * 16 + tx;
    __shared__ cmp<L> si[16][16], sj[16][16];   // [row][vector]
    const int vi = tile * 16 + ty, vj = blockIdx.y * 16 + ty;
    const int ci = vi < j0 ? lst[vi] : -1, cj = vj < bw ? lst[j0 + vj] : -1;
    CAcc<L> acc;
    acc.init(c_zero<L>());
    for (int r0 = rbeg; r0 < rend; r0 += 16) {
        __syncthreads();
        const int r = r0 + tx;
        si[tx][ty] = (r < rend && ci >= 0) ? ld_cmp<L>(P.vec, nn, (size_t)ci * n + r) : c_zero<L>();
        sj[tx][ty] = (r < rend && cj >= 0) ? ld_cmp<L>(P.vec, nn, (size_t)cj * n + r) : c_zero<L>();
        __syncthreads();
        for (int q = 0; q < 16; q++) acc.add_mulc(si[q][ty], sj[q][tx]);
        acc.renorm();
    }
    if (i < j0 && jb < bw) st_cmp<L>(Cm, cplane, (size_t)jb * C.size + i, acc.get());
}

// coefficients = sum of the slices' partial sums, in slice order, into slice 0
template <int L>
__global__ void __launch_bounds__(256) k_gs_dsum(const GsCluster *cls, const RqiProb *probs, int b, double *scratch)
{
    const GsCluster C = cls[blockIdx.z];
    const int j0 = C.nconv + b * RB, bw = min(RB, C.nact - b * RB);
    if (bw <= 0 || j0 == 0) return;
    const int kd = gs_slices(probs[C.prob].n);
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (kd == 1 || e >= j0 * bw) return;
    const int jb = e / j0, i = e - jb * j0;
    const size_t cplane = (size_t)C.size * RB, o = (size_t)jb * C.size + i;
    double *Cm = scratch + C.sofs;
    cmp<L> x = ld_cmp<L>(Cm, cplane, o);
    for (int sl = 1; sl < kd; sl++) x = c_add(x, ld_cmp<L>(Cm + (size_t)sl * 2 * L * cplane, cplane, o));
    st_cmp<L>(Cm, cplane, o, x);
}

template <int L>
__global__ void __launch_bounds__(256) k_gs_update(const GsCluster *cls, const int *list, RqiProb *probs, int b,
                                                   const double *scratch)
{
    const GsCluster C = cls[blockIdx.z];
    const int j0 = C.nconv + b * RB, bw = min(RB, C.nact - b * RB);
    if (bw <= 0 || j0 == 0) return;
    const RqiProb &P = probs[C.prob];
    const int n = P.n;
    const size_t nn = (size_t)n * n;
    const int r = blockIdx.x * 64 + (threadIdx.x & 63);
    const int jb = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (r >= n || jb >= bw) return;
    const int *lst = list + C.off;
    const double *Cm = scratch + C.sofs;
    const size_t cplane = (size_t)C.size * RB;
    const int cj = lst[j0 + jb];
    CAcc<L> acc;
    acc.init(ld_cmp<L>(P.vec, nn, (size_t)cj * n + r));
    for (int i = 0; i < j0; i++) {
        acc.sub_mul(ld_cmp<L>(Cm, cplane, (size_t)jb * C.size + i), ld_cmp<L>(P.vec, nn, (size_t)lst[i] * n + r));
        if ((i & 15) == 15) acc.renorm();
    }
    st_cmp<L>(P.vec, nn, (size_t)cj * n + r, acc.get());
}

// inside the block: modified Gram-Schmidt (twice) and normalisation; the
// coefficients of a member are computed by the four waves in parallel
// Gram matrix of the block, one row slice per blockIdx.x; tiles of 16 x 16
// (blockIdx.y: 0 = (0,0), 1 = (0,1), 2 = (1,1)); entry (a, c) = v_a^H v_c.
template <int L>
__global__ void __launch_bounds__(256) k_gs_gram(const GsCluster *cls, const int *list, const RqiProb *probs, int b,
                                                 double *gram, int ks)
{
    const GsCluster C = cls[blockIdx.z];
    const int j0 = C.nconv + b * RB, bw = min(RB, C.nact - b * RB);
    const int ta = blockIdx.y == 2 ? 1 : 0, tc = blockIdx.y == 0 ? 0 : 1;
    if (bw <= 0 || tc * 16 >= bw) return;
    const RqiProb &P = probs[C.prob];
    const int n = P.n;
    const size_t nn = (size_t)n * n;
    const int *lst = list + C.off;
    const int rc = ((n + ks - 1) / ks + 15) / 16 * 16;
    const int rbeg = blockIdx.x * rc, rend = min(n, rbeg + rc);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    __shared__ cmp<L> sa[16][16], sc[16][16];   // [row][vector]
    const int va = ta * 16 + ty, vc = tc * 16 + ty;
    const int ca = va < bw ? lst[j0 + va] : -1, cc = vc < bw ? lst[j0 + vc] : -1;
    CAcc<L> acc;
    acc.init(c_zero<L>());
    for (int r0 = rbeg; r0 < rend; r0 += 16) {
        __syncthreads();
        const int r = r0 + tx;
        sa[tx][ty] = (r < rend && ca >= 0) ? ld_cmp<L>(P.vec, nn, (size_t)ca * n + r) : c_zero<L>();
        sc[tx][ty] = (r < rend && cc >= 0) ? ld_cmp<L>(P.vec, nn, (size_t)cc * n + r) : c_zero<L>();
        __syncthreads();
        for (int q = 0; q < 16; q++) acc.add_mulc(sa[q][ty], sc[q][tx]);
        acc.renorm();
    }
    const int a = ta * 16 + ty, c = tc * 16 + tx;
    double *g = gram + ((size_t)blockIdx.z * ks + blockIdx.x) * (2 * L * RB * RB);
    if (a < bw && c < bw) st_cmp<L>(g, (size_t)RB * RB, (size_t)a * RB + c, acc.get());
}

// Cholesky factor of the block's Gram matrix and its inverse, one wave per
// cluster.  pass 0 sets the fallback flag; pass 1 is skipped for a flagged
// cluster.  The packed inverse overwrites the cluster's first Gram slice.
__device__ __forceinline__ void unpack_tri(int e, int &a, int &c)
{
    c = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (c * (c + 1) / 2 > e) c--;
    while ((c + 1) * (c + 2) / 2 <= e) c++;
    a = e - c * (c + 1) / 2;
}

template <int L>
__global__ void __launch_bounds__(256) k_gs_chol(const GsCluster *cls, int b, double *gram, int ks, int *flag, int pass)
{
    const GsCluster C = cls[blockIdx.x];
    const int bw = min(RB, C.nact - b * RB);
    if (bw <= 0) return;
    if (pass == 1 && flag[blockIdx.x]) return;
    const int tid = threadIdx.x;
    __shared__ cmp<L> R[RBP];
    __shared__ cmp<L> part[8][RB];
    __shared__ double dg[RB];
    double *g0 = gram + (size_t)blockIdx.x * ks * (2 * L * RB * RB);
    const int np = bw * (bw + 1) / 2;
    for (int e = tid; e < np; e += 256) {
        int a, c;
        unpack_tri(e, a, c);
        cmp<L> x = c_zero<L>();
        for (int s = 0; s < ks; s++) x = c_add(x, ld_cmp<L>(g0 + (size_t)s * (2 * L * RB * RB), (size_t)RB * RB, (size_t)a * RB + c));
        if (a == c) {
            x.im = mp_zero<L>();
            dg[c] = x.re.x[0];
        }
        R[e] = x;
    }
    __syncthreads();
    // right-looking factorisation G = R^H R (entries of the trailing triangle spread over the block)
    bool bad = false;
    for (int j = 0; j < bw; j++) {
        const mp<L> d = R[pk(j, j)].re;
        if (!(d.x[0] > 1e-16 * dg[j])) {
            bad = true;   // the same decision in every thread
            break;
        }
        const mp<L> rj = sqrt_mp(d), inv = div(mp_from<L>(1.0), rj);
        __syncthreads();
        if (tid > j && tid < bw) R[pk(j, tid)] = c_scale(R[pk(j, tid)], inv);
        if (tid == j) R[pk(j, j)] = cmp<L>{rj, mp_zero<L>()};
        __syncthreads();
        const int m = bw - j - 1;
        for (int e = tid; e < m * (m + 1) / 2; e += 256) {
            int a, c;
            unpack_tri(e, a, c);
            a += j + 1;
            c += j + 1;
            // R(a,c) -= conj(R(j,a)) R(j,c)
            R[pk(a, c)] = c_sub(R[pk(a, c)], c_mulc(R[pk(j, a)], R[pk(j, c)]));
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) flag[blockIdx.x] = 1;
        return;
    }
    // in-place inverse of the upper triangle, column by column; the sum of
    // every entry is split over 8 thread groups and reduced through LDS
    const int i = tid & (RB - 1), g = tid / RB;
    for (int j = 0; j < bw; j++) {
        const mp<L> dinv = div(mp_from<L>(1.0), R[pk(j, j)].re);
        cmp<L> t = c_zero<L>();
        if (i < j)
            for (int k = i + g; k < j; k += 8) t = c_add(t, c_mul(R[pk(i, k)], R[pk(k, j)]));
        part[g][i] = t;
        __syncthreads();
        if (g == 0 && i <= j) {
            cmp<L> val = cmp<L>{dinv, mp_zero<L>()};
            if (i < j) {
                cmp<L> s = part[0][i];
                for (int q = 1; q < 8; q++) s = c_add(s, part[q][i]);
                val = c_scale(s, mp_neg<L>(dinv));
            }
            R[pk(i, j)] = val;
        }
        __syncthreads();
    }
    for (int e = tid; e < np; e += 256) st_cmp<L>(g0, (size_t)RBP, (size_t)e, R[e]);
    if (tid == 0 && pass == 0) flag[blockIdx.x] = 0;
}

// V_block <- V_block R^-1, rows in slices of 8 per work-group (8 x 32 threads)
template <int L>
__global__ void __launch_bounds__(256) k_gs_apply(const GsCluster *cls, const int *list, RqiProb *probs, PairDesc *pairs, int b,
                                                  const double *gram, int ks, const int *flag)
{
    const GsCluster C = cls[blockIdx.y];
    const int j0 = C.nconv + b * RB, bw = min(RB, C.nact - b * RB);
    if (bw <= 0 || flag[blockIdx.y]) return;
    const RqiProb &P = probs[C.prob];
    const int n = P.n;
    const size_t nn = (size_t)n * n;
    const int *lst = list + C.off;
    const int tid = threadIdx.x, k = tid & 31, ty = tid >> 5;
    const int r = blockIdx.x * 8 + ty;
    __shared__ cmp<L> Ri[RBP];
    __shared__ cmp<L> X[8][RB];
    const double *g0 = gram + (size_t)blockIdx.y * ks * (2 * L * RB * RB);
    for (int e = tid; e < bw * (bw + 1) / 2; e += 256) Ri[e] = ld_cmp<L>(g0, (size_t)RBP, (size_t)e);
    const bool live = r < n && k < bw;
    X[ty][k] = live ? ld_cmp<L>(P.vec, nn, (size_t)lst[j0 + k] * n + r) : c_zero<L>();
    __syncthreads();
    if (!live) return;
    CAcc<L> acc;
    acc.init(c_zero<L>());
    for (int i = 0; i <= k; i++) {
        const cmp<L> ri = Ri[pk(i, k)];
        acc.sub_mul(cmp<L>{mp_neg<L>(ri.re), mp_neg<L>(ri.im)}, X[ty][i]);   // += R^-1(i,k) x_i
    }
    st_cmp<L>(P.vec, nn, (size_t)lst[j0 + k] * n + r, acc.get());
    if (pairs && C.size > 1 && r == 0) pairs[C.pair_base + lst[j0 + k]].flags |= 2;
}

// fallback for flagged clusters: modified Gram-Schmidt (twice) inside the
// block and normalisation; the coefficients of a member are computed by the
// four waves in parallel
template <int L>
__global__ void __launch_bounds__(256) k_gs_intra(const GsCluster *cls, const int *list, RqiProb *probs, PairDesc *pairs, int b,
                                                  const int *flag)
{
    const GsCluster C = cls[blockIdx.x];
    const int j0 = C.nconv + b * RB, bw = min(RB, C.nact - b * RB);
    if (bw <= 0 || !flag[blockIdx.x]) return;
    const RqiProb &P = probs[C.prob];
    const int n = P.n;
    const size_t nn = (size_t)n * n;
    const int *lst = list + C.off;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    __shared__ mp<L> red[16];
    __shared__ cmp<L> coef[RB];
    for (int a = 0; a < bw; a++) {
        const int ka = lst[j0 + a];
        for (int pass = 0; pass < 2 && a > 0; pass++) {
            for (int q = wid; q < a; q += 4) {
                const int kq = lst[j0 + q];
                CAcc<L> s;
                s.init(c_zero<L>());
                for (int i = lane; i < n; i += 64)
                    s.add_mulc(ld_cmp<L>(P.vec, nn, (size_t)kq * n + i), ld_cmp<L>(P.vec, nn, (size_t)ka * n + i));
                cmp<L> c = s.get();
                c.re = wave_sum_mp<L>(c.re);
                c.im = wave_sum_mp<L>(c.im);
                if (lane == 0) coef[q] = c;
            }
            __syncthreads();
            for (int i = tid; i < n; i += 256) {
                const size_t o = (size_t)ka * n + i;
                CAcc<L> x;
                x.init(ld_cmp<L>(P.vec, nn, o));
                for (int q = 0; q < a; q++) x.sub_mul(coef[q], ld_cmp<L>(P.vec, nn, (size_t)lst[j0 + q] * n + i));
                st_cmp<L>(P.vec, nn, o, x.get());
            }
            __syncthreads();
        }
        normalise_vec<L>(P.vec, nn, n, ka, red);
        if (tid == 0 && C.size > 1 && pairs) pairs[C.pair_base + ka].flags |= 2;
    }
}

template <int L>
int stage2_gs(const GsPlan &G, RqiProb *probs, PairDesc *pairs, hipStream_t st)
{
    if (G.ncl <= 0) return 0;
    for (int b = 0; b < G.max_blocks; b++) {
        const int j0max = G.max_nconv + b * RB;
        if (j0max > 0) {
            for (int pass = 0; pass < 2; pass++) {
                hipLaunchKernelGGL(k_gs_dot<L>, dim3((j0max + 15) / 16 * kGsSlices, RB / 16, G.ncl), dim3(256), 0, st,
                                   G.dev_cls, G.dev_list, (const RqiProb *)probs, b, G.scratch);
                hipLaunchKernelGGL(k_gs_dsum<L>, dim3((j0max * RB + 255) / 256, 1, G.ncl), dim3(256), 0, st, G.dev_cls,
                                   (const RqiProb *)probs, b, G.scratch);
                hipLaunchKernelGGL(k_gs_update<L>, dim3((G.max_n + 63) / 64, RB / 4, G.ncl), dim3(256), 0, st, G.dev_cls,
                                   G.dev_list, probs, b, (const double *)G.scratch);
            }
        }
        for (int pass = 0; pass < 2; pass++) {
            hipLaunchKernelGGL(k_gs_gram<L>, dim3(G.ks, 3, G.ncl), dim3(256), 0, st, G.dev_cls, G.dev_list,
                               (const RqiProb *)probs, b, G.gram, G.ks);
            hipLaunchKernelGGL(k_gs_chol<L>, dim3(G.ncl), dim3(256), 0, st, G.dev_cls, b, G.gram, G.ks, G.flag, pass);
            hipLaunchKernelGGL(k_gs_apply<L>, dim3((G.max_n + 7) / 8, G.ncl), dim3(256), 0, st, G.dev_cls, G.dev_list, probs,
                               pairs, b, (const double *)G.gram, G.ks, (const int *)G.flag);
        }
        hipLaunchKernelGGL(k_gs_intra<L>, dim3(G.ncl), dim3(256), 0, st, G.dev_cls, G.dev_list, probs, pairs, b,
                           (const int *)G.flag);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int stage2_gs<2>(const GsPlan &, RqiProb *, PairDesc *, hipStream_t);
template int stage2_gs<4>(const GsPlan &, RqiProb *, PairDesc *, hipStream_t);

// ============================================ projected Rayleigh-Ritz ====
// A cluster longer than the in-LDS Rayleigh-Ritz holds (chains of eigenvalues
// closer than the cluster tolerance, typically the tail of tiny eigenvalues
// that binary64 cannot separate relative to ||H||): C = V^H H V is formed in
// L limbs, so its entries carry the cluster's own scale, rounded to binary64
// and eigendecomposed by the binary64 stage on the host side of the engine;
// V <- V Q then gives Ritz vectors that separate the members relative to the
// cluster's scale instead of ||H||.
template <int L>
__global__ void __launch_bounds__(256) k_prr_hv(const PrrDesc *descs, const RqiProb *probs)
{
    const PrrDesc D = descs[blockIdx.y];
    const int a = blockIdx.x;
    if (a >= D.size) return;
    const RqiProb &P = probs[D.prob];
    const int n = P.n;
    const size_t nn = (size_t)n * n, yplane = (size_t)n * D.size;
    const int ka = D.k0 + a;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        CAcc<L> y;
        y.init(c_zero<L>());
        for (int j = 0; j < n; j++) {
            const cmp<L> h = ld_h<L>(P, i, j);
            y.sub_mul(cmp<L>{mp_neg<L>(h.re), mp_neg<L>(h.im)}, ld_cmp<L>(P.vec, nn, (size_t)ka * n + j));
            if ((j & 15) == 15) y.renorm();
        }
        st_cmp<L>(D.Y, yplane, (size_t)a * n + i, y.get());
    }
}

// C(a, c) = v_a^H y_c by 16 x 16 tiles; written as binary64 (the leading limb)
template <int L>
__global__ void __launch_bounds__(256) k_prr_c(const PrrDesc *descs, const RqiProb *probs)
{
    const PrrDesc D = descs[blockIdx.z];
    if (blockIdx.x * 16 >= D.size || blockIdx.y * 16 >= D.size) return;
    const RqiProb &P = probs[D.prob];
    const int n = P.n, m = D.size;
    const size_t nn = (size_t)n * n, yplane = (size_t)n * m;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    __shared__ cmp<L> sv[16][16], sy[16][16];   // [row][vector]
    const int va = blockIdx.x * 16 + ty, vc = blockIdx.y * 16 + ty;
    CAcc<L> acc;
    acc.init(c_zero<L>());
    for (int r0 = 0; r0 < n; r0 += 16) {
        __syncthreads();
        const int r = r0 + tx;
        sv[tx][ty] = (r < n && va < m) ? ld_cmp<L>(P.vec, nn, (size_t)(D.k0 + va) * n + r) : c_zero<L>();
        sy[tx][ty] = (r < n && vc < m) ? ld_cmp<L>(D.Y, yplane, (size_t)vc * n + r) : c_zero<L>();
        __syncthreads();
        for (int q = 0; q < 16; q++) acc.add_mulc(sv[q][ty], sy[q][tx]);
        acc.renorm();
    }
    const int a = blockIdx.x * 16 + ty, c = blockIdx.y * 16 + tx;
    if (a < m && c < m) {
        const cmp<L> v = acc.get();
        st2(D.C + 2 * ((size_t)c * m + a), make_double2(v.re.x[0], a == c ? 0.0 : v.im.x[0]));
    }
}

// Y(:, j) = sum_i v_i Q(i, j); grid (ceil(n/64), ceil(size/4), nd)
template <int L>
__global__ void __launch_bounds__(256) k_prr_rot(const PrrDesc *descs, const RqiProb *probs)
{
    const PrrDesc D = descs[blockIdx.z];
    const RqiProb &P = probs[D.prob];
    const int n = P.n, m = D.size;
    const int r = blockIdx.x * 64 + (threadIdx.x & 63), j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (r >= n || j >= m) return;
    const size_t nn = (size_t)n * n, yplane = (size_t)n * m;
    CAcc<L> acc;
    acc.init(c_zero<L>());
    for (int i = 0; i < m; i++) {
        const double2 q = ld2(D.Q + 2 * ((size_t)j * m + i));
        acc.sub_mul(cmp<L>{mp_from<L>(-q.x), mp_from<L>(-q.y)}, ld_cmp<L>(P.vec, nn, (size_t)(D.k0 + i) * n + r));
        if ((i & 15) == 15) acc.renorm();
    }
    st_cmp<L>(D.Y, yplane, (size_t)j * n + r, acc.get());
}

template <int L>
__global__ void __launch_bounds__(256) k_prr_back(const PrrDesc *descs, RqiProb *probs)
{
    const PrrDesc D = descs[blockIdx.z];
    const int j = blockIdx.y;
    if (j >= D.size) return;
    const RqiProb &P = probs[D.prob];
    const int n = P.n;
    const size_t nn = (size_t)n * n, yplane = (size_t)n * D.size;
    for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256)
        st_cmp<L>(P.vec, nn, (size_t)(D.k0 + j) * n + r, ld_cmp<L>(D.Y, yplane, (size_t)j * n + r));
}

template <int L>
int stage2_prr_project(const PrrDesc *d, int nd, int max_size, int max_n, RqiProb *probs, hipStream_t st)
{
    if (nd <= 0) return 0;
    (void)max_n;
    hipLaunchKernelGGL(k_prr_hv<L>, dim3(max_size, nd), dim3(256), 0, st, d, (const RqiProb *)probs);
    hipLaunchKernelGGL(k_prr_c<L>, dim3((max_size + 15) / 16, (max_size + 15) / 16, nd), dim3(256), 0, st, d,
                       (const RqiProb *)probs);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int L>
int stage2_prr_rotate(const PrrDesc *d, int nd, int max_size, int max_n, RqiProb *probs, hipStream_t st)
{
    if (nd <= 0) return 0;
    hipLaunchKernelGGL(k_prr_rot<L>, dim3((max_n + 63) / 64, (max_size + 3) / 4, nd), dim3(256), 0, st, d,
                       (const RqiProb *)probs);
    hipLaunchKernelGGL(k_prr_back<L>, dim3((max_n + 255) / 256, max_size, nd), dim3(256), 0, st, d, probs);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int stage2_prr_project<2>(const PrrDesc *, int, int, int, RqiProb *, hipStream_t);
template int stage2_prr_project<4>(const PrrDesc *, int, int, int, RqiProb *, hipStream_t);
template int stage2_prr_rotate<2>(const PrrDesc *, int, int, int, RqiProb *, hipStream_t);
template int stage2_prr_rotate<4>(const PrrDesc *, int, int, int, RqiProb *, hipStream_t);

// ====================================================== Rayleigh-Ritz ====
// For a small cluster (2..RRMAX members, binary64 vectors already made
// orthonormal in L limbs): C = V^H H V (k x k), its eigendecomposition
// C = Q diag(theta) Q^H by cyclic two-sided Jacobi in L limbs (round-robin
// ordering, k/2 rotations per round), then V <- V Q and sigma_j <- theta_j.
// The Ritz vectors separate the members of the cluster, which the binary64
// vectors mix when the gaps inside the cluster are near binary64 resolution.
constexpr int RRMAX = 32;
constexpr int kRrV = 4;   // cluster members per work-group of k_rr_hv
constexpr int kRrS = 4;   // row slices of k_rr_hv

// Y = H V for every member of the Rayleigh-Ritz clusters; one work-group per
// member; Y in scratch at cluster offset + member * n (limb-planar, 2L planes
// of n*RRMAX per cluster).
template <int L>
__global__ void __launch_bounds__(256) k_rr_hv(const GsCluster *cls, const int *list, const RqiProb *probs, double *scratch)
{
    // kRrV members per work-group (each H entry loaded serves all of them),
    // rows interleaved over kRrS work-groups in slices of 256
    const GsCluster C = cls[blockIdx.y];
    const int a0 = (blockIdx.x / kRrS) * kRrV, slice = blockIdx.x % kRrS;
    if (a0 >= C.size) return;
    const RqiProb &P = probs[C.prob];
    const int n = P.n;
    const size_t nn = (size_t)n * n;
    int ka[kRrV];
#pragma unroll
    for (int v = 0; v < kRrV; v++) ka[v] = list[C.off + min(a0 + v, C.size - 1)];
    double *Y = scratch + C.sofs;
    const size_t yplane = (size_t)n * RRMAX;
    for (int i = threadIdx.x + 256 * slice; i < n; i += 256 * kRrS) {
        CAcc<L> y[kRrV];
#pragma unroll
        for (int v = 0; v < kRrV; v++) y[v].init(c_zero<L>());
        for (int j = 0; j < n; j++) {
            const cmp<L> h = ld_h<L>(P, i, j);
            const cmp<L> nh = cmp<L>{mp_neg<L>(h.re), mp_neg<L>(h.im)};
#pragma unroll
            for (int v = 0; v < kRrV; v++) {
                // y += h v  ==  y -= (-h) v
                y[v].sub_mul(nh, ld_cmp<L>(P.vec, nn, (size_t)ka[v] * n + j));
                if ((j & 15) == 15) y[v].renorm();
            }
        }
#pragma unroll
        for (int v = 0; v < kRrV; v++)
            if (a0 + v < C.size) st_cmp<L>(Y, yplane, (size_t)(a0 + v) * n + i, y[v].get());
    }
}

template <int L>
__device__ void rr_rotate_params(const cmp<L> &b, const mp<L> &a, const mp<L> &d, mp<L> &c, mp<L> &s, cmp<L> &e, mp<L> &tb,
                                 bool &active)
{
    const mp<L> ab2 = c_abs2(b);
    active = ab2.x[0] > 0.0;
    if (!active) return;
    const mp<L> ab = sqrt_mp(ab2);
    // negligible coupling
    const double scale = fabs(a.x[0]) + fabs(d.x[0]);
    if (ab.x[0] <= ldexp(scale, -53 * L - 8)) {
        active = false;
        return;
    }
    const mp<L> inv = div(mp_from<L>(1.0), ab);
    e.re = mul(b.re, inv);                 // e = conj(b)/|b|
    e.im = mp_neg<L>(mul(b.im, inv));
    mp<L> zeta = mul_d(div(sub(d, a), ab), 0.5);
    mp<L> t;
    if (zeta.x[0] == 0.0) {
        t = mp_from<L>(1.0);
    } else {
        const mp<L> az = zeta.x[0] < 0.0 ? mp_neg<L>(zeta) : zeta;
        const mp<L> den = add(az, sqrt_mp(add_d(mul(zeta, zeta), 1.0)));
        t = div(mp_from<L>(zeta.x[0] < 0.0 ? -1.0 : 1.0), den);
    }
    c = div(mp_from<L>(1.0), sqrt_mp(add_d(mul(t, t), 1.0)));
    s = mul(t, c);
    tb = mul(t, ab);
}

template <int L>
__global__ void __launch_bounds__(256) k_rr_solve(const GsCluster *cls, const int *list, RqiProb *probs, const double *scratch,
                                                  int sweeps)
{
    const GsCluster C = cls[blockIdx.x];
    const int k = C.size;
    const RqiProb &P = probs[C.prob];
    const int n = P.n;
    const size_t nn = (size_t)n * n;
    const int *lst = list + C.off;
    const double *Y = scratch + C.sofs;
    const size_t yplane = (size_t)n * RRMAX;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    __shared__ cmp<L> Cm[RRMAX][RRMAX + 1];
    __shared__ cmp<L> Qm[RRMAX][RRMAX + 1];
    __shared__ int pp[RRMAX / 2], qq[RRMAX / 2], ord[RRMAX];
    __shared__ mp<L> rc[RRMAX / 2], rs[RRMAX / 2], rtb[RRMAX / 2], ra[RRMAX / 2], rd[RRMAX / 2];
    __shared__ cmp<L> re_[RRMAX / 2];
    __shared__ int ract[RRMAX / 2];
    // C(i, j) = v_i^H y_j, i <= j, one wave per entry
    for (int e = wid; e < k * k; e += 4) {
        const int i = e % k, j = e / k;
        if (i > j) continue;
        CAcc<L> acc;
        acc.init(c_zero<L>());
        for (int r = lane; r < n; r += 64)
            acc.add_mulc(ld_cmp<L>(P.vec, nn, (size_t)lst[i] * n + r), ld_cmp<L>(Y, yplane, (size_t)j * n + r));
        cmp<L> v = acc.get();
        v.re = wave_sum_mp<L>(v.re);
        v.im = wave_sum_mp<L>(v.im);
        if (lane == 0) {
            if (i == j) v.im = mp_zero<L>();
            Cm[i][j] = v;
            Cm[j][i] = c_conj(v);
        }
    }
    for (int e = tid; e < k * k; e += 256) {
        const int i = e % k, j = e / k;
        Qm[i][j] = c_zero<L>();
        if (i == j) Qm[i][j].re = mp_from<L>(1.0);
    }
    const int m = k + (k & 1);   // pad odd k with a dummy index k
    if (tid < m) ord[tid] = tid;
    __syncthreads();
    for (int sw = 0; sw < sweeps; sw++) {
        for (int round = 0; round < m - 1; round++) {
            const int npair = m / 2;
            if (tid < npair) {
                int p = ord[tid], q = ord[m - 1 - tid];
                if (p > q) { const int tt = p; p = q; q = tt; }
                pp[tid] = p;
                qq[tid] = q;
                bool act = false;
                if (q < k) {
                    mp<L> c, s_, tb;
                    cmp<L> e;
                    rr_rotate_params<L>(Cm[p][q], Cm[p][p].re, Cm[q][q].re, c, s_, e, tb, act);
                    if (act) {
                        rc[tid] = c; rs[tid] = s_; re_[tid] = e; rtb[tid] = tb;
                        ra[tid] = Cm[p][p].re; rd[tid] = Cm[q][q].re;
                    }
                }
                ract[tid] = act ? 1 : 0;
            }
            __syncthreads();
            // column ops on C and Q: [x, y] <- [c x - s e y, s x + c e y]
            for (int w = tid; w < npair * k * 2; w += 256) {
                const int mat = w / (npair * k), rem = w % (npair * k);
                const int r = rem % npair, i = rem / npair;
                if (!ract[r]) continue;
                cmp<L>(*A)[RRMAX + 1] = mat ? Qm : Cm;
                const int p = pp[r], q = qq[r];
                const cmp<L> x = A[i][p], y = c_mul(re_[r], A[i][q]);
                A[i][p] = c_sub(c_scale(x, rc[r]), c_scale(y, rs[r]));
                A[i][q] = c_add(c_scale(x, rs[r]), c_scale(y, rc[r]));
            }
            __syncthreads();
            // row ops on C: [x; y] <- [c x - s conj(e) y ; s x + c conj(e) y]
            for (int w = tid; w < npair * k; w += 256) {
                const int r = w % npair, j = w / npair;
                if (!ract[r]) continue;
                const int p = pp[r], q = qq[r];
                const cmp<L> x = Cm[p][j], y = c_mul(c_conj(re_[r]), Cm[q][j]);
                Cm[p][j] = c_sub(c_scale(x, rc[r]), c_scale(y, rs[r]));
                Cm[q][j] = c_add(c_scale(x, rs[r]), c_scale(y, rc[r]));
            }
            __syncthreads();
            if (tid < npair && ract[tid]) {
                const int p = pp[tid], q = qq[tid];
                Cm[p][q] = c_zero<L>();
                Cm[q][p] = c_zero<L>();
                Cm[p][p].re = sub(ra[tid], rtb[tid]);
                Cm[p][p].im = mp_zero<L>();
                Cm[q][q].re = add(rd[tid], rtb[tid]);
                Cm[q][q].im = mp_zero<L>();
            }
            __syncthreads();
            if (tid == 0) {
                const int last = ord[m - 1];
                for (int q = m - 1; q > 1; q--) ord[q] = ord[q - 1];
                ord[1] = last;
            }
            __syncthreads();
        }
    }
    // ascending Ritz values (selection by rank; ties by index)
    if (tid < k) {
        int rank = 0;
        const double ti = Cm[tid][tid].re.x[0], tl = (L > 1) ? Cm[tid][tid].re.x[1] : 0.0;
        for (int j = 0; j < k; j++) {
            const double tj = Cm[j][j].re.x[0], tjl = (L > 1) ? Cm[j][j].re.x[1] : 0.0;
            if (tj < ti || (tj == ti && (tjl < tl || (tjl == tl && j < tid)))) rank++;
        }
        ord[rank] = tid;
    }
    __syncthreads();
    // sigma of member j <- Ritz value ord[j]
    if (tid < k) {
        const mp<L> th = Cm[ord[tid]][ord[tid]].re;
        for (int l = 0; l < L; l++) P.sigma[(size_t)l * n + lst[tid]] = th.x[l];
    }
    // V <- V Q (columns permuted to ascending order); one row per thread
    for (int r = tid; r < n; r += 256) {
        cmp<L> old[RRMAX];
        for (int i = 0; i < RRMAX; i++)
            if (i < k) old[i] = ld_cmp<L>(P.vec, nn, (size_t)lst[i] * n + r);
        for (int j = 0; j < k; j++) {
            CAcc<L> acc;
            acc.init(c_zero<L>());
            for (int i = 0; i < RRMAX; i++)
                if (i < k) acc.sub_mul(cmp<L>{mp_neg<L>(old[i].re), mp_neg<L>(old[i].im)}, Qm[i][ord[j]]);
            st_cmp<L>(P.vec, nn, (size_t)lst[j] * n + r, acc.get());
        }
    }
}

template <int L>
int stage2_rr(const GsPlan &G, RqiProb *probs, int sweeps, hipStream_t st)
{
    if (G.ncl <= 0) return 0;
    hipLaunchKernelGGL(k_rr_hv<L>, dim3(RRMAX / kRrV * kRrS, G.ncl), dim3(256), 0, st, G.dev_cls, G.dev_list,
                       (const RqiProb *)probs, G.scratch);
    hipLaunchKernelGGL(k_rr_solve<L>, dim3(G.ncl), dim3(256), 0, st, G.dev_cls, G.dev_list, probs, (const double *)G.scratch,
                       sweeps);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int stage2_rr<2>(const GsPlan &, RqiProb *, int, hipStream_t);
template int stage2_rr<4>(const GsPlan &, RqiProb *, int, hipStream_t);

// ================================================================ host ====
static inline unsigned cdiv2(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

template <int L>
int stage2_init(PairDesc *pairs, RqiProb *probs, int npairs, hipStream_t st)
{
    hipLaunchKernelGGL(k_s2_init<L>, dim3(npairs), dim3(256), 0, st, pairs, probs);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int L>
int stage2_rq(const Stage2Batch &B, hipStream_t st)
{
    if (B.count <= 0) return 0;
    hipLaunchKernelGGL(k_s2_rq<L>, dim3(B.count), dim3(256), 0, st, B.dev_pairs, B.dev_probs, B.dev_active, B.final_pass,
                       B.ldl);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// The LDL^H launch sequence in parts, so that two groups of pairs on two
// streams can interleave theirs.  Panels of kLuNB - 1 or kLuNB columns (per
// pair): after s steps every pair has factorised at least
// min(order, s (kLuNB - 1)) columns.
constexpr int kLdlStepW = kLuNB - 1;
constexpr int kRegPanelPairs = 256;

static inline int ldl_steps(int n) { return (n + kLdlStepW - 1) / kLdlStepW; }

// pairs (leading entries of the non-increasing order list) that take part in step s
static inline int ldl_live(const int *orders, int cnt, int s)
{
    int c = cnt;
    while (c > 0 && orders[c - 1] <= s * kLdlStepW) c--;
    return c;
}

template <int L>
static void ldl_build(const Stage2Batch &B, KernelTimer &T, hipStream_t st)
{
    const int id = T.begin(KC_BUILD, 0.0, st);
    hipLaunchKernelGGL(k_s2_build<L>, dim3(cdiv2(B.n + 1, 8), B.count), dim3(256), 0, st, B);
    T.end(id, st);
}

template <int L>
static void ldl_panel(const Stage2Batch &B, const int *orders, int s, int c, KernelTimer &T, hipStream_t st)
{
    const int n = B.n;
    double wp = 0.0;
    for (int q = 0; q < c; q++) {
        const int m = orders[q], k0 = std::min(m, s * kLuNB);
        wp += 0.5 * (double)(m - k0) * kLuNB * kLuNB;
    }
    const int id = T.begin(KC_LU_PANEL, wp, st);
    // dd orders up to 128: one wave per pair with the window in registers.
    // Larger dd orders: the 512-thread register form while the launch has at
    // most kRegPanelPairs pairs (its time is then the latency of one
    // work-group, which the register window and the rows spread over 512
    // threads shorten), else the memory form (a register form at order 1024
    // allows one work-group per CU; with hundreds of pairs it was measured
    // slower)
    if (L == 2 && n <= 128) hipLaunchKernelGGL((k_s2_ldl_panel_reg<64, 2>), dim3(c), dim3(64), 0, st, B);
    else if (n <= 128) hipLaunchKernelGGL((k_s2_ldl_panel<L, 64>), dim3(c), dim3(64), 0, st, B);
    else if (L == 2 && c <= kRegPanelPairs && n <= 512) hipLaunchKernelGGL((k_s2_ldl_panel_reg<512, 1>), dim3(c), dim3(512), 0, st, B);
    else if (L == 2 && c <= kRegPanelPairs && n <= 1024) hipLaunchKernelGGL((k_s2_ldl_panel_reg<512, 2>), dim3(c), dim3(512), 0, st, B);
    else hipLaunchKernelGGL((k_s2_ldl_panel<L, 256>), dim3(c), dim3(256), 0, st, B);
    T.end(id, st);
}

// the trailing update of step s; false when no pair has a trailing block left
template <int L>
static bool ldl_update(const Stage2Batch &B, const int *orders, int s, int c, KernelTimer &T, hipStream_t st)
{
    const int n = B.n;
    // the largest trailing block any pair can have after this step
    const int mrows = n - std::min(n, (s + 1) * kLdlStepW);
    if (mrows <= 0) return false;
    double wu = 0.0;
    for (int q = 0; q < c; q++) {
        const int m = orders[q], k0 = std::min(m, s * kLuNB), r0 = std::min(m, k0 + kLuNB);
        wu += 0.5 * (double)(m - r0) * (m - r0 + 1) * (r0 - k0);   // complex multi-limb multiply-adds of the lower triangle
    }
    const int id = T.begin(KC_LU_UPDATE, wu, st);
    if (L == 2) {
        const unsigned tt = cdiv2(mrows, 64);
        hipLaunchKernelGGL(k_s2_lu_update_dd<true>, dim3(tt * (tt + 1) / 2, c), dim3(256), 0, st, B, 0, 0);
    } else {
        const unsigned tt = cdiv2(mrows, 32);
        hipLaunchKernelGGL((k_s2_lu_update_gen<L, true>), dim3(tt * (tt + 1) / 2, c), dim3(256), 0, st, B, 0, 0);
    }
    T.end(id, st);
    return true;
}

template <int L>
static void ldl_backsolve(const Stage2Batch &B, const int *orders, KernelTimer &T, hipStream_t st)
{
    double wb = 0.0;
    for (int q = 0; q < B.count; q++) wb += 0.5 * (double)orders[q] * orders[q];
    const int id = T.begin(KC_BACKSOLVE, wb, st);
    if (B.n <= 128) hipLaunchKernelGGL((k_s2_ldl_backsolve<L, 64>), dim3(B.count), dim3(64), 0, st, B);
    else hipLaunchKernelGGL((k_s2_ldl_backsolve<L, 256>), dim3(B.count), dim3(256), 0, st, B);
    T.end(id, st);
}

template <int L>
int stage2_solve(const Stage2Batch &B, const int *orders, hipStream_t st)
{
    // orders[0..count-1]: the pairs' matrix orders, non-increasing (host).
    // Pairs of different orders share every launch: at panel step k0 only the
    // leading pairs with order > k0 take part (grid.y), each kernel works with
    // its pair's own order and panel width, and the grid.x extents follow the
    // largest order (smaller pairs' extra work-groups exit at once), so a
    // pair's arithmetic is the same in any mix.
    const int n = B.n, cnt = B.count;
    if (cnt <= 0) return 0;
    KernelTimer dummy;
    KernelTimer &T = B.timer ? *B.timer : dummy;
    if (B.ldl) {
        ldl_build<L>(B, T, st);
        const int steps = ldl_steps(n);
        for (int s = 0; s < steps; s++) {
            const int c = ldl_live(orders, cnt, s);
            if (c == 0) break;
            ldl_panel<L>(B, orders, s, c, T, st);
            ldl_update<L>(B, orders, s, c, T, st);
        }
        ldl_backsolve<L>(B, orders, T, st);
        if (!B.timer) dummy.collect();
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    int id = T.begin(KC_BUILD, 0.0, st);
    hipLaunchKernelGGL(k_s2_build<L>, dim3(cdiv2(n + 1, 8), cnt), dim3(256), 0, st, B);
    T.end(id, st);
    for (int k0 = 0; k0 < n; k0 += kLuNB) {
        int c = cnt;
        while (c > 0 && orders[c - 1] <= k0) c--;
        const int nbw = std::min(kLuNB, n - k0);
        double wp = 0.0, wt = 0.0, wu = 0.0;
        for (int q = 0; q < c; q++) {
            const int m = orders[q], b = std::min(kLuNB, m - k0), r0 = k0 + b;
            wp += 0.5 * (double)(m - k0) * b * b;
            wt += 0.5 * (double)(m + 1 - r0) * b * b;
            wu += (double)(m - r0) * (m + 1 - r0) * b;   // complex multi-limb multiply-adds of A22 -= L21 U12
        }
        id = T.begin(KC_LU_PANEL, wp, st);
        hipLaunchKernelGGL(k_s2_lu_panel<L>, dim3(c), dim3(256), 0, st, B, k0, nbw);
        T.end(id, st);
        const int r0 = k0 + nbw;
        const int ncols = n + 1 - r0;
        id = T.begin(KC_LU_TRSM, wt, st);
        hipLaunchKernelGGL(k_s2_lu_trsm<L>, dim3(cdiv2(ncols, 8 * kTrsmGroups), c), dim3(256), 0, st, B, k0, nbw);
        T.end(id, st);
        const int mrows = n - r0;
        if (mrows > 0) {
            id = T.begin(KC_LU_UPDATE, wu, st);
            if (L == 2) {
                const unsigned tiles = cdiv2(mrows, 64) * cdiv2(ncols, 64);
                hipLaunchKernelGGL(k_s2_lu_update_dd<false>, dim3(tiles, c), dim3(256), 0, st, B, k0, nbw);
            } else {
                const unsigned tiles = cdiv2(mrows, 32) * cdiv2(ncols, 32);
                hipLaunchKernelGGL((k_s2_lu_update_gen<L, false>), dim3(tiles, c), dim3(256), 0, st, B, k0, nbw);
            }
            T.end(id, st);
        }
    }
    double wb = 0.0;
    for (int q = 0; q < cnt; q++) wb += 0.5 * (double)orders[q] * orders[q];
    id = T.begin(KC_BACKSOLVE, wb, st);
    hipLaunchKernelGGL(k_s2_backsolve<L>, dim3(cnt), dim3(256), 0, st, B);
    T.end(id, st);
    if (!B.timer) dummy.collect();
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Two groups of pairs (LDL^H), group g on stream st[g], in disjoint slots:
// the trailing updates of the two groups alternate (group 0's update of step
// s, then group 1's, then group 0's of step s + 1, ...; ev[g] marks group g's
// last update), so that while one group's update has the chip, the other
// group factorises its next panel beside it, and no two updates overlap.
template <int L>
int stage2_solve_pair(const Stage2Batch *B, const int *const *orders, const hipStream_t *st, const hipEvent_t *ev)
{
    KernelTimer dummy[2];
    KernelTimer *T[2];
    int steps = 0;
    for (int g = 0; g < 2; g++) {
        T[g] = B[g].timer ? B[g].timer : &dummy[g];
        if (B[g].count > 0) {
            ldl_build<L>(B[g], *T[g], st[g]);
            steps = std::max(steps, ldl_steps(B[g].n));
        }
    }
    bool upd[2] = {false, false};   // group g has an update enqueued (ev[g] recorded)
    for (int s = 0; s < steps; s++)
        for (int g = 0; g < 2; g++) {
            if (B[g].count <= 0 || s >= ldl_steps(B[g].n)) continue;
            const int c = ldl_live(orders[g], B[g].count, s);
            if (c == 0) continue;
            ldl_panel<L>(B[g], orders[g], s, c, *T[g], st[g]);
            if (upd[1 - g] && hipStreamWaitEvent(st[g], ev[1 - g], 0) != hipSuccess) return -1;
            if (ldl_update<L>(B[g], orders[g], s, c, *T[g], st[g])) {
                if (hipEventRecord(ev[g], st[g]) != hipSuccess) return -1;
                upd[g] = true;
            }
        }
    for (int g = 0; g < 2; g++)
        if (B[g].count > 0) ldl_backsolve<L>(B[g], orders[g], *T[g], st[g]);
    for (int g = 0; g < 2; g++)
        if (!B[g].timer) dummy[g].collect();
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int L>
int stage2_output(PairDesc *pairs, RqiProb *probs, const int *dst, int npairs, hipStream_t st)
{
    hipLaunchKernelGGL(k_s2_output<L>, dim3(npairs), dim3(256), 0, st, pairs, probs, dst);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int stage2_init<2>(PairDesc *, RqiProb *, int, hipStream_t);
template int stage2_init<4>(PairDesc *, RqiProb *, int, hipStream_t);
template int stage2_rq<2>(const Stage2Batch &, hipStream_t);
template int stage2_rq<4>(const Stage2Batch &, hipStream_t);
template int stage2_solve<2>(const Stage2Batch &, const int *, hipStream_t);
template int stage2_solve<4>(const Stage2Batch &, const int *, hipStream_t);
template int stage2_solve_pair<2>(const Stage2Batch *, const int *const *, const hipStream_t *, const hipEvent_t *);
template int stage2_solve_pair<4>(const Stage2Batch *, const int *const *, const hipStream_t *, const hipEvent_t *);
template int stage2_output<2>(PairDesc *, RqiProb *, const int *, int, hipStream_t);
template int stage2_output<4>(PairDesc *, RqiProb *, const int *, int, hipStream_t);

// ------------------------------------------------------------- ingest -----
struct IngestArgs {
    int n, lda, limbs;
    const double *pl[4];
    double *hf;
    int *flag;
};

__global__ void k_s2_ingest(IngestArgs a)
{
    const int n = a.n, j = blockIdx.x;
    if (j >= n) return;
    const size_t nn = (size_t)n * n;
    int bad = 0;
    for (int i = j + threadIdx.x; i < n; i += blockDim.x) {
        for (int l = 0; l < a.limbs; l++) {
            const double2 z = ld2(a.pl[l] + 2 * ((size_t)j * a.lda + i));
            if (!isfinite(z.x) || !isfinite(z.y)) bad = 1;
            const double zi = (i == j) ? 0.0 : z.y;
            a.hf[(2 * l) * nn + (size_t)j * n + i] = z.x;
            a.hf[(2 * l + 1) * nn + (size_t)j * n + i] = zi;
            if (i != j) {
                a.hf[(2 * l) * nn + (size_t)i * n + j] = z.x;
                a.hf[(2 * l + 1) * nn + (size_t)i * n + j] = -zi;
            }
        }
    }
    if (bad) atomicOr(a.flag, 1);
}

int stage2_ingest(int n, int lda, int limbs, const double *const *planes, double *hf, int *flag, hipStream_t st)
{
    IngestArgs a;
    a.n = n;
    a.lda = lda;
    a.limbs = limbs;
    for (int l = 0; l < 4; l++) a.pl[l] = l < limbs ? planes[l] : nullptr;
    a.hf = hf;
    a.flag = flag;
    hipLaunchKernelGGL(k_s2_ingest, dim3(n), dim3(256), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace zk
