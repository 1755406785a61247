// Internal interfaces between the host driver (api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>

#include "common.h"

namespace zk {

constexpr int kMaxN = 4096;   // largest matrix order accepted

struct GemmDesc {
    const double *A;
    const double *B;
    double *C;
    int lda, ldb, ldc, pad;
};

// A batch of stage-1 problems of equal order n.
struct Stage1Batch {
    int n;
    int nprob;
    ProbDesc *dev_probs;       // nprob descriptors (device)
    const GemmDesc *dev_gemm;  // stage1_gemm_desc_count(n, nprob) descriptors (device)
    double tri_gap_rel;        // cluster gap (relative) for the binary64 Gram-Schmidt
};

size_t stage1_gemm_desc_count(int n, int np);
void stage1_fill_gemm_descs(const ProbDesc *host_probs, int np, GemmDesc *out);
int stage1_run(const Stage1Batch &B, hipStream_t st);

// ---------------------------------------------------------------- stage 2
// Workspace of one concurrently factorised pair (shifted LU of order n,
// augmented with the right-hand side as column n).
struct LuSlot {
    double *M;      // 2L planes of ldm x (n+1) doubles
    int *ipiv;      // n
};

// Stage-2 launch table: `count` active pairs (indices into the pair table).
struct Stage2Batch {
    int L;                  // 2 (dd) or 4 (qd)
    int n;                  // order shared by the pairs of this launch group
    int count;
    const int *dev_active;  // pair indices (device)
    PairDesc *dev_pairs;
    RqiProb *dev_probs;
    double *lu_base;        // slot s at lu_base + s * lu_stride
    size_t lu_stride;       // doubles
    int *piv_base;          // slot s at piv_base + s * piv_stride
    size_t piv_stride;
    int ldm;                // leading dimension of the LU planes
    int max_iter;
    int final_pass;         // rq: re-judge converged pairs after re-orthogonalisation
};

// ingest of a matrix for stage 2 alone (refinement of caller pairs):
// limb-planar full copy + NaN/Inf flag
int stage2_ingest(int n, int lda, int limbs, const double *const *planes, double *hf, int *flag, hipStream_t st);

template <int L> int stage2_init(PairDesc *pairs, RqiProb *probs, int npairs, hipStream_t st);
template <int L> int stage2_gs(PairDesc *pairs, RqiProb *probs, const int *cluster_heads, int nclusters, hipStream_t st);
template <int L> int stage2_rq(const Stage2Batch &B, hipStream_t st);
template <int L> int stage2_solve(const Stage2Batch &B, hipStream_t st);
// scratch: nprob * sstride doubles, sstride >= 2L * n * 32
template <int L> int stage2_reorth(RqiProb *probs, const int *plist, int nprob, int n, double *scratch, size_t sstride,
                                   hipStream_t st);
template <int L> int stage2_output(PairDesc *pairs, RqiProb *probs, const int *dst, int npairs, hipStream_t st);

}  // namespace zk
