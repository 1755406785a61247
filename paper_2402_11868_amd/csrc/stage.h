// Internal interfaces between the host driver (api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <vector>

#include "common.h"

namespace zk {

constexpr int kMaxN = 4096;   // largest matrix order accepted

// Per-kernel-class timing with HIP events recorded on the launch stream
// around each launch (instrumentation; off unless enabled on the context).
enum KernelClass { KC_LU_UPDATE = 0, KC_LU_PANEL, KC_LU_TRSM, KC_BACKSOLVE, KC_RQ, KC_GS, KC_REORTH, KC_STAGE1,
                   KC_HER2K, KC_HEMV, KC_BUILD, KC_TRD_VEC, KC_TRIDIAG, KC_BACKT, KC_AP_RESID, KC_AP_FGEMM,
                   KC_AP_DDGEMM, KC_AP_OTHER, KC_COUNT };

struct KernelTimer {
    bool on = false;
    unsigned mask = ~0u;   // kernel classes that are timed (bit c = class c)
    struct Rec {
        int cls;
        hipEvent_t a, b;
        double work;
    };
    std::vector<Rec> open;
    std::vector<hipEvent_t> pool;
    double ms[KC_COUNT] = {0};
    double work[KC_COUNT] = {0};
    long long launches[KC_COUNT] = {0};
    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        hipEventCreate(&e);
        return e;
    }
    // returns the index of the record to close with end()
    int begin(int cls, double w, hipStream_t st)
    {
        if (!on || !((mask >> cls) & 1u)) return -1;
        Rec r{cls, get(), get(), w};
        hipEventRecord(r.a, st);
        open.push_back(r);
        return (int)open.size() - 1;
    }
    void end(int id, hipStream_t st)
    {
        if (id >= 0) hipEventRecord(open[id].b, st);
    }
    // fold finished records into the totals (synchronises on the events)
    void collect()
    {
        for (Rec &r : open) {
            hipEventSynchronize(r.b);
            float t = 0.0f;
            hipEventElapsedTime(&t, r.a, r.b);
            ms[r.cls] += t;
            work[r.cls] += r.work;
            launches[r.cls]++;
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        open.clear();
    }
    void reset()
    {
        collect();
        for (int c = 0; c < KC_COUNT; c++) ms[c] = work[c] = 0, launches[c] = 0;
    }
    ~KernelTimer()
    {
        for (Rec &r : open) { hipEventDestroy(r.a); hipEventDestroy(r.b); }
        for (hipEvent_t e : pool) hipEventDestroy(e);
    }
};

struct GemmDesc {
    const double *A;
    const double *B;
    double *C;
    int lda, ldb, ldc, pad;
};

// A batch of stage-1 problems of equal order n.
struct Stage1Batch {
    KernelTimer *timer;        // may be null
    int n;
    int nprob;
    ProbDesc *dev_probs;       // nprob descriptors (device)
    const GemmDesc *dev_gemm;  // stage1_gemm_desc_count(n, nprob) descriptors (device)
    double tri_gap_rel;        // cluster gap (relative) for the binary64 Gram-Schmidt
    int fp32;                  // FP32-MFMA variant: complex64-rounded input, FP32 MFMA GEMMs
};

size_t stage1_gemm_desc_count(int n, int np);
void stage1_fill_gemm_descs(const ProbDesc *host_probs, int np, GemmDesc *out);
int stage1_run(const Stage1Batch &B, hipStream_t st);
// the three parts of stage1_run: ingest (and the order-1 case), the
// per-column tridiagonalisation launches, the tridiagonal solver and
// back-transformation
int stage1_ingest(const Stage1Batch &B, hipStream_t st);
int stage1_trd(const Stage1Batch &B, hipStream_t st);
int stage1_solve(const Stage1Batch &B, hipStream_t st);


// ------------------------------------------------------------------- SVD
// One singular value decomposition through the Hermitian dilation (svd.hip).
struct SvdDesc {
    int m, n, lda, limbs, ldu, ldv;
    const double *A[4];   // input limb planes, complex128 m x n (leading dimension lda)
    double *K;            // limbs planes of (m+n) x (m+n) complex128, leading dimension m+n
    const double *w[2];   // eigenvalue limbs of K (ascending)
    double *V[2];         // eigenvector limb planes of K (complex128, leading dimension m+n); scratch after extraction
    double *s[2];         // singular value limbs (min(m, n), descending)
    double *u[2];         // left singular vector limb planes (m x min(m,n), leading dimension ldu), or null
    double *v[2];         // right singular vector limb planes (n x min(m,n), leading dimension ldv)
};
int svd_build(const SvdDesc &D, hipStream_t st);
int svd_extract(const SvdDesc &D, hipStream_t st);

// ------------------------------------------------------------------- MPS
// One two-site update (mps.hip).  All pointers are device pointers to
// complex128 limb planes (hi, lo), column-major.
struct MpsDesc {
    int M, K, N;          // theta is M x N (M = 2 chi_l, N = 2 chi_r), inner dimension K = chi
    int chil, chir;
    int lda, ldb;         // A: M x K (lda >= M), B: K x N (ldb >= K)
    int chi, ldv, pad;    // kept bond dimension chi'; V leading dimension
    const double *A[2];
    const double *B[2];
    double *T[2];         // theta (M x N, leading dimension M), the gate applied in place
    const double *G[2];   // 4 x 4 gate, row and column index 2 s1 + s2
    const double *V[2];   // right singular vectors of theta (N x min(M, N), leading dimension ldv)
    const double *s[2];   // singular value limbs
    double *Bo[2];        // B' (chi' x N, leading dimension chi')
};
// theta = A B, then the gate on the physical indices
int mps_theta(const MpsDesc &D, hipStream_t st);
// B' = diag(s[:chi']) V[:, :chi']^H
int mps_bout(const MpsDesc &D, hipStream_t st);

// One bond of the MPS simulation (mps.hip): sites q (cl x (2 cm)) and q+1
// (cm x (2 cr)) in right-canonical form, column index s chi + r; all matrices
// are two complex128 limb planes (hi, lo), column-major.
struct MpsSimDesc {
    int cl, cm, cr;       // chi_{q-1}, chi_q, chi_{q+1}
    int chi;              // kept bond dimension (split)
    const double *Bq[2];  // site q
    const double *Bq1[2]; // site q+1
    const double *lam[2]; // lambda_{q-1} (cl values, limb planes), or null (all ones)
    double *T[2];         // theta (2 cl) x (2 cr), row s1 cl + l, column s2 cr + r; the site for gate1
    const double *G[2];   // gate: 4 x 4 (index 2 s1 + s2) or 2 x 2, column-major
    double *rho[2];       // bond matrix (2 cr) x (2 cr)
    const double *V[2];   // its eigenvectors (ld 2 cr), ascending eigenvalues
    const double *w[2];   // its eigenvalues
    double *Bq_out[2];    // cl x (2 chi)
    double *Bq1_out[2];   // chi x (2 cr)
    double *lam_out[2];   // chi Schmidt values
    double *eig_out[2];   // chi Schmidt values squared (the kept eigenvalues)
};
// theta = G (B_q B_{q+1}), rho = theta^H diag(lambda_{q-1}^2) theta
int mps_sim_bond(const MpsSimDesc &D, hipStream_t st);
// the new sites and bond from rho's eigendecomposition
int mps_sim_split(const MpsSimDesc &D, hipStream_t st);
// one-qubit gate on a site (D.T = the site, D.cl x (2 D.cm))
int mps_sim_gate1(const MpsSimDesc &D, hipStream_t st);

// ---------------------------------------------------------------- stage 2
// Workspace of one concurrently factorised pair (shifted factorisation of
// order n, augmented with the right-hand side as column n; columns n+1 ..
// n+5 are the LDL^H panel's working columns (candidate pivot column, the
// look-ahead window), columns n+6 .. n+5+kLuNB its W = L D of the panel last
// factorised).
constexpr int kLdlLA = 4;   // look-ahead window of the LDL^H panel
__host__ __device__ inline int ldl_wcol(int n) { return n + 2 + kLdlLA; }
struct LuSlot {
    double *M;      // 2L planes of ldm x (n+6+kLuNB) doubles
    int *ipiv;      // 2n: interchanges, then the LDL^H panel-start marks
};

// Stage-2 launch table: `count` active pairs (indices into the pair table).
// leading dimension of a pair's factorisation planes, and the plane size
// (ldm x (n+6+kLuNB) doubles: the matrix, the right-hand side, the working
// columns, the panel's W)
__host__ __device__ inline int lu_ldm_of(int n) { return (n + 7) & ~7; }
__host__ __device__ inline size_t lu_plane_of(int n) { return (size_t)lu_ldm_of(n) * (size_t)(ldl_wcol(n) + kLuNB); }

struct Stage2Batch {
    int L;                  // 2 (dd) or 4 (qd)
    int n;                  // largest order of the pairs of this launch (grid extents)
    int count;
    const int *dev_active;  // pair indices (device)
    PairDesc *dev_pairs;
    RqiProb *dev_probs;
    double *lu_base;        // slot s at lu_base + s * lu_stride
    size_t lu_stride;       // doubles
    int *piv_base;          // slot s at piv_base + s * piv_stride
    size_t piv_stride;
    int ldm;                // unused by the solve (each pair's planes use lu_ldm_of(its order))
    int ldl;                // 1: Hermitian LDL^H with Bunch-Kaufman pivoting, 0: LU with partial pivoting
    int max_iter;
    int final_pass;         // rq: re-judge converged pairs after re-orthogonalisation
    KernelTimer *timer;     // host object, may be null
};

// ingest of a matrix for stage 2 alone (refinement of caller pairs):
// limb-planar full copy + NaN/Inf flag
int stage2_ingest(int n, int lda, int limbs, const double *const *planes, double *hf, int *flag, hipStream_t st);

template <int L> int stage2_init(PairDesc *pairs, RqiProb *probs, int npairs, hipStream_t st);
// Gram-Schmidt plan: clusters with their column lists (see stage2.hip)
struct GsCluster {
    int prob;        // problem index
    int pair_base;   // pair-table index of the problem's pair 0
    int off;         // offset of the column list
    int nconv;       // leading entries left untouched
    int nact;        // entries orthogonalised, in order
    int size;        // nconv + nact
    long long sofs;  // scratch offset (doubles): Gram-Schmidt, kGsSlices sets of 2L planes of
                     // size * 32 values; Rayleigh-Ritz, 2L planes of n * 32 values
};
constexpr int kGsSlices = 8;   // row slices of the Gram-Schmidt coefficient sums, at most
// row slices for a cluster of order n: a function of n alone, so that a
// matrix's coefficients do not depend on the other matrices of a call
__host__ __device__ inline int gs_slices(int n) { return n / 128 < 1 ? 1 : (n / 128 > kGsSlices ? kGsSlices : n / 128); }
struct GsPlan {
    int ncl;
    int max_blocks;   // max over clusters of ceil(nact / 32)
    int max_nconv;
    int max_n;
    const GsCluster *dev_cls;
    const int *dev_list;
    double *scratch;
    // inside-block Cholesky QR: Gram partial sums (ks row slices per cluster,
    // 2L planes of 32 x 32 each), reused for the packed inverse factor, and one
    // fallback flag per cluster
    double *gram;
    int ks;
    int *flag;
};
template <int L> int stage2_gs(const GsPlan &G, RqiProb *probs, PairDesc *pairs, hipStream_t st);
// Rayleigh-Ritz inside clusters of 2..32 members (plan entries: nconv = 0,
// scratch per cluster 2L * n * 32 doubles)
template <int L> int stage2_rr(const GsPlan &G, RqiProb *probs, int sweeps, hipStream_t st);
// Projected Rayleigh-Ritz for clusters longer than 32: one descriptor per
// block of consecutive pairs of one problem.
struct PrrDesc {
    int prob;          // problem index in the uploaded table
    int k0;            // first pair (local index) of the block
    int size;          // members
    int pad;
    double *Y;         // 2L planes of n * size: H V, later V Q
    double *C;         // size x size complex128, column-major: binary64 rounding of V^H H V
    const double *Q;   // size x size complex128 eigenvectors of C (column j = vector j)
};
// C = V^H H V (rounded to binary64) for every descriptor
template <int L> int stage2_prr_project(const PrrDesc *d, int nd, int max_size, int max_n, RqiProb *probs, hipStream_t st);
// V <- V Q for every descriptor
template <int L> int stage2_prr_rotate(const PrrDesc *d, int nd, int max_size, int max_n, RqiProb *probs, hipStream_t st);
// Lowdin orthonormalisation of column windows of double-double limb-planar
// matrices (planes re_hi, re_lo, im_hi, im_lo, px apart; columns of n rows
// consecutive): `steps` steps X <- X - X (X^H X - I) / 2 by dd GEMMs;
// scratch of dd_lowdin_bytes(windows) bytes
struct DdWindow {
    double *X;    // first column of the window, plane 0
    size_t px;    // plane stride
    int n, m;     // rows, columns
};
size_t dd_lowdin_bytes(const std::vector<DdWindow> &w);
int dd_lowdin(const std::vector<DdWindow> &w, int steps, void *scratch, hipStream_t st);
template <int L> int stage2_rq(const Stage2Batch &B, hipStream_t st);
// orders: the pairs' matrix orders (host, count entries, non-increasing);
// B.n = orders[0] sets the grid extents, the LU slots are B.lu_stride apart
template <int L> int stage2_solve(const Stage2Batch &B, const int *orders, hipStream_t st);
// LDL^H solves of two groups of pairs in disjoint slots, group g on stream
// st[g]; their trailing updates alternate (ev[g]: group g's last update)
template <int L>
int stage2_solve_pair(const Stage2Batch *B, const int *const *orders, const hipStream_t *st, const hipEvent_t *ev);
template <int L> int stage2_output(PairDesc *pairs, RqiProb *probs, const int *dst, int npairs, hipStream_t st);

}  // namespace zk
