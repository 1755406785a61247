/*
 * zk.h -- C-ABI of libzk: accurate complex Hermitian eigendecomposition on one
 * AMD Instinct MI355X (gfx950) GPU.
 *
 * The method is the one the paper describes for its GPU extension (Sec. 2,
 * ZKCM_CUS paragraph): a binary64 eigendecomposition of the Hermitian matrix
 * followed by Rayleigh quotient iteration that recovers the precision.  The
 * diagonalisation of Hermitian (bond reduced density) matrices dominates the
 * cost of the MPS simulation (Sec. 2.1), and the precision must resolve
 * Schmidt coefficients as small as 2^((1-n)/2) (Sec. 1 and its footnote 1).
 *
 * Stage 1 (binary64): blocked Householder tridiagonalisation, tridiagonal
 * eigen-solver (bisection + inverse iteration), back-transformation.
 * Stage 2 (double-double or quad-double): per-eigenpair Rayleigh quotient
 * iteration with shifted LU solves, Gram-Schmidt inside eigenvalue clusters,
 * residual-based convergence test.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are complex128 (re, im interleaved), COLUMN-MAJOR, in DEVICE
 *   memory.  Only the LOWER triangle (i >= j) is read; the upper triangle is
 *   taken as its conjugate and the imaginary part of the diagonal is ignored.
 * - "Limbs": an input or output value may be an unevaluated sum of 1, 2 or 4
 *   binary64 numbers.  A limb plane set is an array of pointers, one per limb;
 *   the value is the exact sum of the limbs.  1 limb = plain complex128.
 * - Eigenvalues are returned in ASCENDING order; eigenvectors have unit norm;
 *   the phase of a vector and the basis inside an exactly degenerate
 *   eigenspace are unspecified.
 * - The caller owns every buffer in zk_herm / zk_eig_out and keeps it alive
 *   until the call returns (zk_heev_*, zk_rqi_refine are synchronous with
 *   respect to the host) or until zk_session_poll reports completion.  The
 *   library allocates and frees only its own workspace, bounded by the
 *   context's HBM budget; it never frees caller memory.
 * - Status codes are returned, never thrown.  On ZK_EINVAL nothing is
 *   written.  On ZK_ENOCONV every output is written and the per-pair flags say
 *   which pairs missed the tolerance.
 * - A zk_ctx is used by one host thread at a time.  Work is enqueued on the
 *   context's HIP stream.
 */
#ifndef ZK_H
#define ZK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct zk_ctx zk_ctx;
typedef struct zk_session zk_session;
typedef uint64_t zk_ticket;

enum {
    ZK_OK = 0,
    ZK_ENOCONV = 1,      /* outputs written; some pairs missed tol (see info flags) */
    ZK_EINVAL = -1,      /* bad argument or NaN/Inf in the input; nothing written */
    ZK_ENOMEM = -2,      /* request cannot fit the HBM budget / device allocation failed */
    ZK_EDEVICE = -3,     /* HIP runtime error; the context is poisoned */
    ZK_EAGAIN = -4,      /* session: queue full (submit) or request pending (poll) */
    ZK_ECANCELED = -5,   /* session destroyed before the request ran */
    ZK_EINTERNAL = -6
};

/* per-pair flags in zk_pair_info.flags */
enum {
    ZK_PAIR_CONVERGED = 1,   /* residual <= tol * ||H||_2 */
    ZK_PAIR_REORTH = 2,      /* Gram-Schmidt against cluster members was applied */
    ZK_PAIR_PIVOT_GUARD = 4, /* a zero pivot was replaced in some shifted LU */
    ZK_PAIR_NAN = 8,
    ZK_PAIR_LU_SOLVES = 16   /* the residual stalled with LDL^H solves; the later solves used LU */
};

/* A Hermitian input.  plane[0..limbs-1] are device pointers to n x n
 * complex128 column-major arrays with leading dimension lda (elements). */
typedef struct {
    int n;
    int lda;
    int limbs;            /* 1, 2 or 4 */
    const void *plane[4];
} zk_herm;

typedef struct {
    int32_t iters;        /* Rayleigh quotient iterations (shifted solves) used */
    int32_t flags;        /* ZK_PAIR_* */
    int32_t cluster;      /* index of the first eigenvalue of this pair's cluster */
    int32_t reserved;
    double resid;         /* final ||H v - lam v|| / ||H||_2, rounded to binary64 */
} zk_pair_info;

/* Output of one decomposition.  w[l] (device) holds limb l of the n ascending
 * eigenvalues; v[l] (device) limb l of the eigenvectors, an n x n complex128
 * column-major array with leading dimension ldv (column k = eigenvector k);
 * v[*] may be NULL when opts->want_vectors == 0.  info: HOST array of n
 * entries, or NULL. */
typedef struct {
    int n;
    int ldv;
    int limbs;            /* 2 for dd output, 4 for qd output */
    double *w[4];
    void *v[4];
    zk_pair_info *info;
} zk_eig_out;

typedef struct {
    int init_fp32;        /* 1: binary64 stage on the complex64-rounded input with FP32-MFMA trailing
                             updates and back-transform (the refinement always uses the exact input) */
    double tol;           /* residual/eigenvalue tolerance relative to ||H||_2; 0 = default (1e-30 dd, 1e-60 qd) */
    int max_iter;         /* RQI iterations per pair; 0 = default (8 dd, 10 qd) */
    double cluster_tol;   /* eigenvalues closer than cluster_tol*||H||_2 are one cluster; 0 = default 1e-10 */
    int want_vectors;     /* 1 (default): write eigenvectors */
    int reorth;           /* 1 (default): after the iteration, re-orthogonalise all eigenvectors of a
                             matrix (classical Gram-Schmidt twice, in the output precision) and
                             recompute every Rayleigh quotient and residual; 0: only inside clusters */
    int refine;           /* 0 (default): per-pair Rayleigh quotient iteration (the paper's method);
                             1: the all-pairs refinement of zk_heev_dd_allpairs (double-double output
                             only; ZK_EINVAL with 4 output limbs).  Honoured by zk_heev_dd and by
                             session requests; zk_rqi_refine always iterates per pair. */
    int shifted_solve;    /* factorisation of the shifted systems (H - sigma I) w = v of the Rayleigh
                             quotient iteration: 0 = default (LDL^H), 1 = LU with partial pivoting,
                             2 = Hermitian LDL^H with Bunch-Kaufman pivoting (half the multiply-adds
                             of LU in the trailing updates).  Sessions use the default.  With LDL^H
                             the pairs of a launch run in two groups on the context stream and a
                             side stream of default priority (one group inside
                             zk_heev_dd_noalloc); the results are the same bits either way
                             (environment variable ZK_S2_SPLIT=0: one group). */
} zk_opts;

/* Fill *o with the defaults (init_fp32 0, tol 0, max_iter 0, cluster_tol 0, want_vectors 1, reorth 1, refine 0,
 * shifted_solve 0). */
void zk_opts_default(zk_opts *o);

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t of the
 * caller (e.g. torch.cuda.current_stream().cuda_stream) or NULL for a private
 * stream.  hbm_budget: maximum workspace bytes the library may hold (0 = 64 GiB).
 * Returns ZK_OK and *out, or ZK_EINVAL / ZK_EDEVICE. */
int zk_ctx_create(int device, void *hip_stream, size_t hbm_budget, zk_ctx **out);

/* Release the context and all its workspace.  NULL is accepted. */
int zk_ctx_destroy(zk_ctx *ctx);

/* Static string for a status code. */
const char *zk_status_str(int status);

/* Message of the last failure on ctx ("" if none).  Valid until the next call on ctx. */
const char *zk_ctx_last_error(const zk_ctx *ctx);

/* Bytes of workspace one decomposition of order n with `limbs` output limbs
 * needs when `concurrent_pairs` shifted LU factorisations run at once. */
size_t zk_workspace_bytes(int n, int limbs, int concurrent_pairs);

/* Device workspace of the context: *held = bytes it holds now, *budget = its
 * HBM budget, *high_water = the most it has held at once since creation,
 * *transient = the part of *held that belongs to matrices in flight
 * (iterate storage and plans of the refinement engines; 0 between
 * synchronous calls, whether they succeeded or failed; the rest are
 * grow-only workspaces kept for the next call).  Any pointer may be NULL.
 * ZK_EINVAL for a NULL ctx. */
int zk_ctx_memory(const zk_ctx *ctx, size_t *held, size_t *budget, size_t *high_water, size_t *transient);

/* Counters of the per-pair Rayleigh quotient iteration of the last
 * zk_heev_dd / zk_heev_qd call on ctx (all matrices of the call):
 * iters_hist16[i] = number of pairs that took i shifted solves (i >= 15
 * counted in the last bin), *rounds = iteration rounds, *solves = shifted
 * solves in total.  Zeros after a call with opts->refine = 1.  Any pointer
 * may be NULL.  ZK_EINVAL for a NULL ctx. */
int zk_ctx_last_stats(const zk_ctx *ctx, int *iters_hist16, int *rounds, long long *solves);

/*
 * zk_heev_dd / zk_heev_qd: eigendecompose `count` independent Hermitian
 * matrices A[0..count-1] (sizes may differ) to double-double (out[i].limbs ==
 * 2) or quad-double (out[i].limbs == 4) accuracy.  Stage 1 runs in binary64,
 * stage 2 is the Rayleigh quotient iteration (Sec. 2, ZKCM_CUS).  Synchronous:
 * returns when the outputs are in place.
 * Errors: ZK_EINVAL for count < 1, n < 1, lda < n, limbs not in {1,2,4}, NULL
 * planes, ldv < n, a limbs mismatch, or NaN/Inf in an input; ZK_ENOMEM if one
 * matrix alone exceeds the budget; ZK_ENOCONV if some pair missed tol.
 */
int zk_heev_dd(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out *out, const zk_opts *opts);
int zk_heev_qd(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out *out, const zk_opts *opts);

/*
 * zk_heev_dd_allpairs: the same double-double decomposition as zk_heev_dd,
 * with stage 2 replaced by an all-pairs refinement of O(n^3) work per matrix
 * instead of one O(n^3) shifted LU factorisation per pair and iteration.  It
 * is not the paper's method (Sec. 2 names only Rayleigh quotient iteration):
 * every iteration forms the residual matrix R = H X - X diag(lam) with exact
 * products and cascaded sums, F = X^H R in binary64, and corrects all pairs
 * at once by the first-order formula of Ogita and Aishima's refinement of
 * symmetric eigendecompositions (Japan J. Indust. Appl. Math. 35, 2018), in
 * its Hermitian form; pairs too close for that formula form blocks that are
 * rotated by the binary64 eigenvectors of their projected matrix, at the
 * block's own scale, before the correction.  Arguments, layouts, ownership,
 * outputs and errors are those of zk_heev_dd (out[i].limbs == 2).  opts:
 * tol, want_vectors and init_fp32 as for zk_heev_dd; max_iter bounds the
 * whole-basis iterations (0 = default 12); cluster_tol and reorth are not
 * used.  info[k].iters is the number of whole-basis iterations of the matrix,
 * info[k].cluster the first index of the block of the pair in the last
 * iteration.  Synchronous.
 */
int zk_heev_dd_allpairs(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out *out, const zk_opts *opts);

/* Output of zk_heev_mp: `limbs` binary64 limbs per value (4, 8 or 16).
 * w (device): limbs x n doubles, limb l of eigenvalue k at w[l * n + k].
 * v (device): `limbs` planes of complex128, plane l starting at element
 * l * ldv * n; each plane n x n column-major with leading dimension ldv
 * (column k = eigenvector k); NULL when opts->want_vectors == 0.
 * info: HOST array of n entries, or NULL. */
typedef struct {
    int n;
    int ldv;
    int limbs;
    double *w;
    void *v;
    zk_pair_info *info;
} zk_eig_out_mp;

/*
 * zk_heev_mp: eigendecomposition beyond double-double: quad-double (limbs 4,
 * about 212 bits), 8 limbs (about 424 bits) or 16 limbs (about 848 bits;
 * the paper's multiple-precision diagonalisations run at up to 768 bits,
 * Sec. 2.1, Fig. 1).  Stage 1 in binary64, the all-pairs refinement of
 * zk_heev_dd_allpairs to double-double, then whole-basis polishing in L
 * limbs: residual matrix and Gram matrix with exact products and L-level
 * cascaded sums, the first-order correction of every pair from them in
 * binary64 (pairs whose correction would exceed 1e-4 of their gap, or whose
 * gap is zero, are only re-orthogonalised; runs of such pairs with distinct
 * eigenvalues are rotated by the eigenvectors of their projected matrix),
 * about sixteen more binary digits per iteration.  The iteration scales H by
 * a power of two internally; the outputs are binary64 limb expansions, so an
 * eigenvalue near 2^e resolves 2^(e - 1074) at best (at ||H||_2 = 2^e the
 * 16-limb default tolerance needs e above about -270).
 * All out[i].limbs must be equal.  opts: tol (default 1e-60,
 * 1e-120, 1e-240 for 4, 8, 16 limbs; relative to ||H||_2, for every residual;
 * the departure from orthonormality is brought within tol too), max_iter
 * (polishing iterations, default 8 + 3 limbs), want_vectors.  info[k].iters =
 * polishing iterations of the matrix, info[k].resid = residual before the
 * last Rayleigh-quotient update (an upper bound).  Eigenvalues ascending.
 * Synchronous.  ZK_ENOCONV if max_iter iterations leave a residual or the
 * departure from orthonormality above tol (the outputs are still written).
 * Errors: as zk_heev_dd; ZK_EINVAL for limbs not in {4, 8, 16} or unequal
 * across the call, ldv < n, or NULL w / v.
 */
int zk_heev_mp(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out_mp *out, const zk_opts *opts);

/* A general complex matrix: plane[0..limbs-1] are device pointers to m x n
 * complex128 column-major arrays with leading dimension lda (elements). */
typedef struct {
    int m;
    int n;
    int lda;
    int limbs;            /* 1, 2 or 4 */
    const void *plane[4];
} zk_mat;

/* Output of one singular value decomposition, k = min(m, n): s[l] (device)
 * limb l of the k singular values in DESCENDING order; u[l] (device) limb l of
 * the left singular vectors, m x k complex128 column-major, leading dimension
 * ldu; v[l] likewise for the right singular vectors (n x k, ldv); u, v may be
 * NULL when opts->want_vectors == 0.  info: HOST array of k entries (the
 * information of the eigenpair each triplet comes from), or NULL. */
typedef struct {
    int m;
    int n;
    int limbs;            /* 2 (double-double) */
    double *s[4];
    void *u[4];
    int ldu;
    void *v[4];
    int ldv;
    zk_pair_info *info;
} zk_svd_out;

/*
 * zk_svd_dd: singular value decomposition A = U diag(s) V^H of `count`
 * general complex matrices to double-double accuracy.  The paper lists the
 * SVD beside the eigendecomposition for its GPU extension, with the same
 * precision recovery (Sec. 2).  Method: the Hermitian dilation
 * K = [[0, A], [A^H, 0]] of order m + n is eigendecomposed exactly as by
 * zk_heev_dd (binary64 stage, then the Rayleigh quotient iteration, or the
 * all-pairs refinement with opts->refine = 1); its eigenvalues are +-s_j and
 * |m - n| zeros, the eigenvector of +s_j is [u_j; v_j] / sqrt(2).  No
 * squaring: the bound is |s_j - s~_j| <= tol * s_1 and
 * ||A v_j - s_j u_j||, ||A^H u_j - s_j v_j|| <= tol * s_1 (tol as in
 * zk_heev_dd); U and V each get one first-order orthonormalisation step, so
 * their columns are orthonormal to about tol.  Singular vectors of singular
 * values below tol * s_1 are not unique (they span the null spaces) and are
 * not specified.  The status counts the k returned triplets only
 * (ZK_ENOCONV when one of them misses the tolerance; the dilation's other
 * pairs are not outputs).  Synchronous.
 * Errors: as zk_heev_dd, and ZK_EINVAL for m < 1, n < 1, lda < m, out->limbs
 * != 2, ldu < m or ldv < n.
 */
int zk_svd_dd(zk_ctx *ctx, int count, const zk_mat *A, zk_svd_out *out, const zk_opts *opts);

/*
 * zk_mps_two_site_dd: one two-site update of a matrix product state in
 * double-double, the step of the paper's MPS simulation (Sec. 1) whose cost is
 * the decomposition of the bond (Sec. 2.1).  Site tensors A (chi_l x 2 x chi)
 * and B (chi x 2 x chi_r) and a two-qubit gate G give
 *   theta = G . (A B)      (contraction over the shared bond, G on (s1, s2))
 *   theta = U diag(s) V^H  (zk_svd_dd, either refinement by opts->refine)
 *   A' = U[:, :chi'],  B' = diag(s[:chi']) V[:, :chi']^H,
 * chi' = the number of singular values s_j > cutoff * s_1, at most chi_max
 * (and at least 1).
 * Layout: every operand is two device planes (hi, lo) of complex128,
 * column-major.  A: (2 chi_l) x chi, leading dimension 2 chi_l, row index
 * s1 chi_l + l.  B: chi x (2 chi_r), leading dimension chi, column index
 * s2 chi_r + r.  gate: 4 x 4, row and column index 2 s1 + s2.
 * A_out: room for (2 chi_l) x chi_max, written with leading dimension
 * 2 chi_l; B_out: room for chi_max x (2 chi_r), written chi' x (2 chi_r) with
 * leading dimension chi'; s_out: room for chi_max doubles per plane (singular
 * value limbs, descending); *chi_out (host) receives chi'.  The library
 * allocates its scratch (theta and the SVD's buffers) within the context
 * budget.  Synchronous.
 * Errors: ZK_EINVAL for chi_l, chi, chi_r < 1, 2 chi_l + 2 chi_r above the
 * largest order, chi_max outside 1 .. min(2 chi_l, 2 chi_r), a negative or
 * NaN cutoff, or a NULL pointer; ZK_ENOMEM; then as zk_svd_dd (ZK_ENOCONV
 * when a kept triplet misses the tolerance).
 */
int zk_mps_two_site_dd(zk_ctx *ctx, int chi_l, int chi, int chi_r, const void *const *A, const void *const *B,
                       const void *const *gate, int chi_max, double cutoff, void *const *A_out, void *const *B_out,
                       double *const *s_out, int *chi_out, const zk_opts *opts);

/*
 * zk_heev_dd_noalloc: for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same decomposition as zk_heev_dd (same arguments, layouts,
 * options, outputs, ownership and errors; bitwise the same results), but no
 * device memory is allocated or freed during the call: all of its workspace
 * comes from one static device array of ZK_NOALLOC_SCRATCH_BYTES per GPU,
 * which the library holds from its first use on a device until the process
 * ends, and the context's own workspace is neither used nor grown.  The
 * caller still passes the inputs and outputs.  The binary64 stage runs on the
 * context stream only, and kernel-class timing (zk_prof_*) records nothing
 * during the call.
 * Limit: ZK_ENOMEM, before any work, when the call needs more than the array
 * holds (the binary64 stage, inputs and iterates of all `count` matrices at
 * once plus one shifted-LU slot of the largest order, as zk_workspace_bytes
 * counts them: one matrix of order up to 647, or e.g. 6 matrices of order
 * 256, 26 of order 128), and ZK_ENOMEM if the array runs out during the call.
 * Concurrency: the array is shared by every call on that GPU and keeps the
 * last call's contents (nothing reads them).  Calls from threads of one
 * process are serialised per device; calls that overlap on one GPU through
 * another copy of the library would race.  Synchronous.
 */
#define ZK_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
int zk_heev_dd_noalloc(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out *out, const zk_opts *opts);

/*
 * MPS simulation.  A chain of nq qubits as a matrix product state in
 * double-double (sites in right-canonical form with the Schmidt values of
 * every bond, Hastings' form of the Vidal decomposition), the paper's MPS
 * method (Sec. 1) whose cost is the diagonalisation of the bond matrices
 * (Sec. 2.1).  A two-qubit gate G on qubits (q, q+1) forms
 * theta = G (B_q B_{q+1}) and the Hermitian PSD bond matrix
 * rho = theta^H diag(lambda_{q-1}^2) theta of order 2 chi_{q+1}; rho is
 * eigendecomposed in double-double through a serving session (the gates of
 * one call share its launches); the chi' largest eigenvalues w above
 * cutoff^2 w_max (at most chi_max) are kept: B_{q+1} = V^H, B_q = theta V,
 * lambda_q = sqrt(w).  No Schmidt value is ever inverted.
 * Gates are HOST arrays of two limb planes (hi, lo) of complex128,
 * column-major: 2 x 2 (8 doubles per plane) for zk_mps_apply1, 4 x 4 with
 * row and column index 2 s_q + s_{q+1} (32 doubles per plane) for
 * zk_mps_apply2.  The MPS holds its own session on a second context of the
 * same device; the caller's context runs the other kernels and holds the
 * sites (budget-counted).  All calls are synchronous.
 */
typedef struct zk_mps zk_mps;

/* |0...0> on nq qubits (2 <= nq <= 4096); chi_max <= 256, cutoff >= 0.
 * ZK_EINVAL, ZK_ENOMEM, ZK_EDEVICE. */
int zk_mps_create(zk_ctx *ctx, int nq, int chi_max, double cutoff, zk_mps **out);
int zk_mps_destroy(zk_mps *m);
/* One-qubit gate on qubit q. */
int zk_mps_apply1(zk_mps *m, int q, const double *gate);
/* `count` two-qubit gates, gate k on (q[k], q[k] + 1); the pairs must be
 * disjoint (ZK_EINVAL otherwise).  ZK_ENOCONV if a bond matrix missed the
 * double-double tolerance (the state is updated all the same). */
int zk_mps_apply2(zk_mps *m, int count, const int *q, const double *const *gates);
/* Bond b (between qubits b-1 and b; 0 and nq are the ends): *chi = its
 * dimension; eig (host, 2 * max doubles, may be NULL) receives the limbs of
 * the first min(max, chi) squared Schmidt values, descending: limb 0 at
 * eig[j], limb 1 at eig[max + j]. */
int zk_mps_bond(zk_mps *m, int b, int max, double *eig, int *chi);
/* Site q as two limb planes (host, capacity doubles in total) of the
 * chi_l x (2 chi_r) complex128 matrix B_q[l, s, r] at column s chi_r + r. */
int zk_mps_site(zk_mps *m, int q, int *chi_l, int *chi_r, double *out, size_t capacity);
/* Every bond matrix diagonalised so far: submit-to-done seconds and order. */
int zk_mps_latencies(zk_mps *m, int max, double *seconds, int *orders, int *count);

/*
 * zk_heev_fp64: stage 1 alone (the binary64 eigendecomposition that seeds the
 * Rayleigh quotient iteration).  For each matrix i: w[i] (device, n doubles,
 * ascending) and V[i] (device, n x n complex128 column-major, leading
 * dimension ldv[i] >= n).  Synchronous.  Errors as zk_heev_*.
 */
int zk_heev_fp64(zk_ctx *ctx, int count, const zk_herm *A, double *const *w, void *const *V, const int *ldv);

/*
 * zk_rqi_refine: stage 2 alone.  Refines k caller-supplied binary64
 * eigenpairs of one Hermitian matrix A: w0 (device, k doubles, ascending) and
 * V0 (device, n x k complex128 column-major, leading dimension ldv0, unit
 * columns) to `limbs_out` (2 or 4) limbs.  out->n must equal k (the number of
 * pairs), out->ldv >= A->n.  Same errors as zk_heev_*.
 */
int zk_rqi_refine(zk_ctx *ctx, int limbs_out, const zk_herm *A, int k, const double *w0,
                  const void *V0, int ldv0, zk_eig_out *out, const zk_opts *opts);

/*
 * Instrumentation.  When enabled, the context records a pair of HIP events on
 * its stream around every launch of a kernel class and accumulates elapsed
 * milliseconds, launch counts and the algorithmic work of each launch.
 * Classes: 0 shifted-LU trailing update (work: complex multi-limb
 * multiply-adds), 1 LU panel, 2 LU triangular solve + interchanges,
 * 3 back-substitution, 4 Rayleigh quotient/residual, 5 cluster Gram-Schmidt,
 * 6 global re-orthogonalisation, 7 whole binary64 stage, 8 FP64-MFMA trailing
 * update of the tridiagonalisation (work: flops), 9 Hermitian mat-vec of the
 * tridiagonalisation (work: bytes), 10 shifted-matrix build, 11 column update,
 * reflector and W-vector of the tridiagonalisation, 12 tridiagonal
 * eigen-solver (bisection, inverse iteration, Gram-Schmidt), 13
 * back-transformation (work: flops), 14 residual matrix of the all-pairs
 * refinement (work: complex products of H and X), 15 its binary64 GEMM
 * X^H R (work: flops), 16 its double-double GEMMs (work: complex
 * double-double multiply-adds), 17 its other kernels.
 * zk_prof_read waits for the recorded events.
 */
int zk_prof_enable(zk_ctx *ctx, int on);
/* Restrict the timing to the classes whose bit (1u << class) is set in mask
 * (default: all); the others record no events. */
int zk_prof_classes(zk_ctx *ctx, unsigned mask);
int zk_prof_reset(zk_ctx *ctx);
int zk_prof_read(zk_ctx *ctx, int kernel_class, double *ms, long long *launches, double *work);

/*
 * Serving form.  A session runs a scheduler thread that admits submitted
 * requests while their workspace fits the session budget, batches the binary64
 * stage of requests of equal order, and runs the Rayleigh quotient iterations
 * of every admitted request together in shared launches (continuous
 * batching).  Results are bitwise identical to a request run alone.
 * budget: bytes of admitted footprints at once (0 = 16 GiB); a request's
 * footprint is its stage-2 inputs plus its iterates and one shifted-LU slot
 * (or the all-pairs state).  max_queue: requests waiting for admission at
 * once (0 = unbounded); all work runs on the context's stream.  The session
 * uses the context from its own thread: do not call other entry points on
 * the same context while it lives.
 */
int zk_session_create(zk_ctx *ctx, size_t budget, int max_queue, zk_session **out);

/* Queue one request; returns at once.  *ticket identifies it.  ZK_EAGAIN if
 * the queue holds max_queue requests, ZK_ENOMEM if the request alone exceeds
 * the session budget, ZK_EINVAL for bad arguments. */
int zk_session_submit(zk_session *s, const zk_herm *A, zk_eig_out *out, int limbs_out,
                      const zk_opts *opts, zk_ticket *ticket);

/* Wait up to timeout_us microseconds (0: do not wait, <0: forever) for the
 * request.  Returns ZK_OK when done (*req_status = its status), ZK_EAGAIN if
 * still pending, ZK_ECANCELED if the session is being destroyed (a poll
 * blocked at that moment wakes with it), ZK_EINVAL for an unknown ticket. */
int zk_session_poll(zk_session *s, zk_ticket ticket, int timeout_us, int *req_status);

/* Host-clock stamps of a finished request: submit, admission, completion (seconds). */
int zk_session_times(zk_session *s, zk_ticket ticket, double *t_submit, double *t_admit, double *t_done);

/* Stop the scheduler; pending requests (queued or running) are cancelled:
 * threads blocked in zk_session_poll return ZK_ECANCELED, and destroy
 * returns only after they have left.  The session handle is invalid after
 * the call. */
int zk_session_destroy(zk_session *s);

#ifdef __cplusplus
}
#endif

#endif /* ZK_H */
