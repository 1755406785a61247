// Shared device helpers and descriptors of libzk (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mp.h"

namespace zk {

constexpr int kNB = 32;          // panel width of the binary64 tridiagonalisation
constexpr int kLuNB = 32;        // panel width of the shifted LU factorisations

typedef double __attribute__((ext_vector_type(4))) f64x4;

// One matrix of a binary64-stage batch.  All pointers are device pointers
// into the library's workspace, except `in[]` (caller's input planes).
struct ProbDesc {
    int n;
    int lda_in;
    int limbs_in;
    int pad0;
    const double *in[4];   // caller planes (complex128 interleaved), column-major
    double *hf;            // full Hermitian copy, limb-planar: plane (l*2+c) of n*n doubles
    double *A;             // n x n complex128 working copy (lower triangle used)
    double *Y;             // n x n complex128 reflectors (column c: rows c+1.., Y[c+1,c] = 1)
    double *tau;           // n complex128
    double *P;             // n x 2NB complex128: [V | W] of the current panel
    double *Q;             // n x 2NB complex128: [W | V]
    double *part;          // hemv partial sums: (2*ntile) x n complex128
    double *tri;           // 5 n^2 doubles: inverse-iteration LU factors, interleaved
    double *Zt;            // n x n: inverse-iteration vectors, entry i of vector k at [i*n + k]
    double *d;             // n   (tridiagonal diagonal)
    double *e;             // n   (off-diagonal, e[n-1] unused)
    double *w0;            // n   ascending binary64 eigenvalues
    double *Z;             // n x n real tridiagonal eigenvectors
    double *V0;            // n x n complex128 back-transformed eigenvectors
    double *T;             // (n/NB+1) x NB x NB complex128 block-reflector factors
    double *X;             // NB x n complex128 scratch
    double *X2;            // NB x n complex128 scratch
    int *flag;             // [0]: NaN/Inf seen in the input
    int *cnt;              // 2n finishing counters (column update, W finish), zeroed at ingest
    double *scr;           // per row chunk: partial norm (dd), panel dot products, w^H v; reflector scale
};

// Pair (eigenvector) state of the Rayleigh quotient stage.
struct PairDesc {
    int prob;      // index of its matrix in the stage-2 problem table
    int k;         // pair index inside the matrix (ascending binary64 order)
    int cl_start;  // first pair (index k) of its cluster
    int cl_size;
    int status;    // 0 active, 1 converged, 2 stopped (not converged)
    int iters;
    int flags;
    int slot;      // LU workspace slot while active
    int tiny;      // pivots below 2^11 guard thresholds in the pair's last shifted factorisation
    int lk0, lkb;  // LDL^H: first column and width of the pair's current panel
    int pad0;
    double resid;  // ||H v - sigma v|| / hnorm
    double prev_resid;
};

// A matrix of the Rayleigh quotient stage.
struct RqiProb {
    int n;
    int limbs_in;
    int ldv_out;
    int ldv0;
    int max_iter;          // iteration limit of this matrix's pairs
    int pad1;
    const double *hf;      // limb-planar full Hermitian copy (ld n)
    const double *w0;      // binary64 starting eigenvalues (n)
    const double *V0;      // binary64 starting eigenvectors, complex128 n x n (ld ldv0)
    double hnorm;          // ||H||_2 estimate (max |binary64 eigenvalue|)
    double tol_abs;        // tol * hnorm
    double piv_tol;        // zero-pivot guard threshold
    double *vec;           // 2L planes of n x n doubles: iterate of pair k in column k
    double *sigma;         // L x n doubles: Rayleigh quotient of pair k (limb l at l*n + k)
    double *w_out[4];      // caller eigenvalue limbs (length n)
    double *v_out[4];      // caller eigenvector limb planes (complex128, ld ldv_out)
};

__device__ __forceinline__ double2 ld2(const double *p) { return *reinterpret_cast<const double2 *>(p); }
__device__ __forceinline__ void st2(double *p, double2 v) { *reinterpret_cast<double2 *>(p) = v; }

// wave-level sum of a double (64 lanes)
__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int L>
__device__ __forceinline__ mp<L> wave_sum_mp(mp<L> v)
{
    for (int off = 32; off > 0; off >>= 1) {
        mp<L> o;
        for (int l = 0; l < L; l++) o.x[l] = __shfl_xor(v.x[l], off, 64);
        v = add(v, o);
    }
    return v;
}

// block-level sum for blockDim.x <= 1024 (all threads get the result); red needs 16 slots
template <int L>
__device__ mp<L> block_sum_mp(mp<L> v, mp<L> *red)
{
    v = wave_sum_mp<L>(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    mp<L> s = red[0];
    for (int w = 1; w < nw; w++) s = add(s, red[w]);
    __syncthreads();
    return s;
}

__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; w++) s += red[w];
    __syncthreads();
    return s;
}

}  // namespace zk
