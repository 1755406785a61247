// C-ABI of libzk: argument checking, workspace, and the host side of the
// two-stage method (binary64 eigendecomposition, then Rayleigh quotient
// iteration in double-double or quad-double; Sec. 2, ZKCM_CUS paragraph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/zk.h"
#include "api_internal.h"
#include "engine.h"
#include "stage.h"

using namespace zk;

// ------------------------------------------------------------ status ----
extern "C" const char *zk_status_str(int s)
{
    switch (s) {
    case ZK_OK: return "ZK_OK";
    case ZK_ENOCONV: return "ZK_ENOCONV: some pairs did not reach the tolerance";
    case ZK_EINVAL: return "ZK_EINVAL: invalid argument or non-finite input";
    case ZK_ENOMEM: return "ZK_ENOMEM: workspace exceeds the HBM budget or allocation failed";
    case ZK_EDEVICE: return "ZK_EDEVICE: HIP runtime error";
    case ZK_EAGAIN: return "ZK_EAGAIN: try again";
    case ZK_ECANCELED: return "ZK_ECANCELED: request cancelled";
    case ZK_EINTERNAL: return "ZK_EINTERNAL: internal error";
    default: return "unknown status";
    }
}

extern "C" void zk_opts_default(zk_opts *o)
{
    if (!o) return;
    o->init_fp32 = 0;
    o->tol = 0.0;
    o->max_iter = 0;
    o->cluster_tol = 0.0;
    o->want_vectors = 1;
    o->reorth = 1;
    o->refine = 0;
    o->shifted_solve = 0;
}

extern "C" const char *zk_ctx_last_error(const zk_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

// ---------------------------------------------------------- context -----
extern "C" int zk_ctx_create(int device, void *hip_stream, size_t hbm_budget, zk_ctx **out)
{
    if (!out) return ZK_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return ZK_EDEVICE;
    if (device < 0 || device >= ndev) return ZK_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return ZK_EDEVICE;
    zk_ctx *c = new zk_ctx();
    c->device = device;
    c->budget = hbm_budget ? hbm_budget : ((size_t)64 << 30);
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return ZK_EDEVICE;
        }
        c->own_stream = true;
    }
    *out = c;
    return ZK_OK;
}

extern "C" int zk_ctx_destroy(zk_ctx *ctx)
{
    if (!ctx) return ZK_OK;
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    for (DevBuf *b : {&ctx->s1, &ctx->s2in, &ctx->s2vec, &ctx->s2lu, &ctx->meta}) b->release();
    for (hipStream_t &x : ctx->side)
        if (x) {
            hipStreamSynchronize(x);
            hipStreamDestroy(x);
        }
    for (hipEvent_t &e : ctx->ev)
        if (e) hipEventDestroy(e);
    if (ctx->own_stream) hipStreamDestroy(ctx->stream);
    delete ctx;
    return ZK_OK;
}

size_t zk_ctx::held() const { return s1.bytes + s2in.bytes + s2vec.bytes + s2lu.bytes + meta.bytes + extra; }

// Grow a workspace buffer (contents are not preserved).  ZK_ENOMEM if the
// budget would be exceeded.
bool zk_ctx::make_room(size_t bytes)
{
    if (held() + bytes <= budget) return true;
    if (s2lu.p) {
        hipStreamSynchronize(stream);
        drop(s2lu);
    }
    return held() + bytes <= budget;
}

int zk_ctx::ensure(DevBuf &b, size_t bytes)
{
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes <= b.bytes) return ZK_OK;
    if (&b != &s2lu && held() - b.bytes + bytes > budget) make_room(bytes - b.bytes);
    if (held() - b.bytes + bytes > budget) return fail(ZK_ENOMEM, "workspace of %zu bytes exceeds the budget", bytes);
    drop(b);
    int rc = dev_alloc(&b.p, bytes);
    if (rc != ZK_OK) return rc;
    b.bytes = bytes;
    note_held();
    return ZK_OK;
}

int zk_ctx::dev_alloc(void **p, size_t bytes)
{
    *p = nullptr;
    if (arena) {
        *p = arena->take(bytes);
        if (!*p)
            return fail(ZK_ENOMEM, "scratch array exhausted: %zu bytes wanted, %zu of %zu in use", bytes, arena->in_use,
                        arena->size);
        return ZK_OK;
    }
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        hipGetLastError();
        return fail(ZK_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    return ZK_OK;
}

void zk_ctx::dev_free(void *p)
{
    if (!p) return;
    if (arena && arena->owns(p))
        arena->give(p);
    else
        hipFree(p);
}

void zk_ctx::drop(DevBuf &b)
{
    dev_free(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

int zk_ctx::fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    if (status == ZK_EDEVICE) poisoned = true;
    return status;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) return ctx->fail(ZK_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------ sizes / layout --
static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// stage-1 scratch per problem (bytes), excluding hf/w0/V0 which live in s2in
static size_t s1_bytes(int n)
{
    const size_t nn = (size_t)n * n, ntile = (size_t)(n + 63) / 64, npan = (size_t)(n + kNB - 1) / kNB + 1;
    size_t b = 0;
    b += align_up(16 * nn);                 // A
    b += align_up(16 * nn);                 // Y
    b += align_up(16 * (size_t)n);          // tau
    b += 2 * align_up(16 * (size_t)n * 2 * kNB);   // P, Q
    b += align_up(16 * 2 * ntile * n);      // part
    b += align_up(8 * 5 * nn);              // tri
    b += align_up(8 * nn);                  // Zt
    b += 3 * align_up(8 * (size_t)n);       // d, e, cnt
    b += align_up(8 * (ntile * (4 + 4 * (size_t)kNB) + 2));   // scr
    b += align_up(8 * nn);                  // Z
    b += align_up(16 * npan * kNB * kNB);   // T
    b += 2 * align_up(16 * (size_t)kNB * n);   // X, X2
    b += align_up(64);                      // flag
    return b;
}

// stage-2 inputs per problem: hf, w0, V0
static size_t s2in_bytes(int n, int limbs_in)
{
    const size_t nn = (size_t)n * n;
    return align_up(8 * 2 * (size_t)limbs_in * nn) + align_up(8 * (size_t)n) + align_up(16 * nn) + align_up(64);
}

// stage-2 iterate storage per problem: vec, sigma
static size_t s2vec_bytes(int n, int L)
{
    const size_t nn = (size_t)n * n;
    return align_up(8 * 2 * (size_t)L * nn) + align_up(8 * (size_t)L * n);
}


static size_t lu_slot_doubles(int n, int L) { return (size_t)2 * L * zk::lu_plane_of(n); }

extern "C" size_t zk_workspace_bytes(int n, int limbs, int concurrent_pairs)
{
    if (n < 1 || (limbs != 2 && limbs != 4) || concurrent_pairs < 0) return 0;
    const size_t lu = align_up(8 * lu_slot_doubles(n, limbs)) + align_up(8 * (size_t)n);
    return s1_bytes(n) + s2in_bytes(n, 4) + s2vec_bytes(n, limbs) + (size_t)concurrent_pairs * lu + align_up(64 * (size_t)n + 4096);
}

// ------------------------------------------------------ argument checks --
static int check_herm(const zk_herm &A)
{
    if (A.n < 1 || A.n > kMaxN || A.lda < A.n) return ZK_EINVAL;
    if (A.limbs != 1 && A.limbs != 2 && A.limbs != 4) return ZK_EINVAL;
    for (int l = 0; l < A.limbs; l++)
        if (!A.plane[l]) return ZK_EINVAL;
    return ZK_OK;
}

static int check_out(const zk_eig_out &o, int n_pairs, int n_rows, int L, bool want_vectors)
{
    if (o.n != n_pairs || o.limbs != L) return ZK_EINVAL;
    for (int l = 0; l < L; l++) {
        if (!o.w[l]) return ZK_EINVAL;
        if (want_vectors && !o.v[l]) return ZK_EINVAL;
    }
    if (want_vectors && o.ldv < n_rows) return ZK_EINVAL;
    return ZK_OK;
}



ResolvedOpts zk_resolve_opts(const zk_opts *o, int L)
{
    ResolvedOpts r;
    r.tol = (o && o->tol > 0.0) ? o->tol : (L == 2 ? 1e-30 : 1e-60);
    r.max_iter = (o && o->max_iter > 0) ? o->max_iter : (L == 2 ? 8 : 10);
    if (o && o->max_iter < 0) r.max_iter = 0;
    r.cluster_tol = (o && o->cluster_tol > 0.0) ? o->cluster_tol : 1e-10;
    r.want_vectors = o ? (o->want_vectors != 0) : 1;
    r.init_fp32 = o ? o->init_fp32 : 0;
    r.reorth = o ? (o->reorth != 0) : 1;
    r.refine = o ? o->refine : 0;
    r.ldl = (o && o->shifted_solve == 1) ? 0 : 1;
    r.max_iter_set = (o && o->max_iter > 0) ? o->max_iter : 0;
    return r;
}

int zk_check_request(const zk_herm &A, const zk_eig_out &o, int L, bool want_vectors)
{
    if (check_herm(A) != ZK_OK) return ZK_EINVAL;
    return check_out(o, A.n, A.n, L, want_vectors);
}

// ============================================================ stage 2 ====
// One-shot use of the stage-2 engine: every matrix joins at once, rounds run
// until all pairs have stopped.
template <int L>
static int run_stage2(zk_ctx *ctx, std::vector<RqiProb> &probs, const std::vector<int> &npair_of,
                      std::vector<zk_pair_info *> infos, const ResolvedOpts &O, Stage2Stats *stats)
{
    std::vector<S2Prob> store(probs.size());
    std::vector<S2Prob *> batch;
    for (size_t i = 0; i < probs.size(); i++) {
        store[i].rp = probs[i];
        store[i].opts = O;
        store[i].npairs = npair_of[i];
        store[i].info = infos[i];
        batch.push_back(&store[i]);
    }
    Stage2Engine<L> eng(ctx, O, stats);
    int rc = eng.add(batch);
    while (rc == ZK_OK && eng.any_live()) rc = eng.round();
    if (stats) stats->rounds = eng.rounds;
    if (rc != ZK_OK) return rc;
    for (auto &p : store)
        if (p.status != ZK_OK) return p.status;
    return ZK_OK;
}

// ============================================================ heev ========
// stage-2 inputs (hf, w0, V0, flag) of every matrix, carved from ctx->s2in
static int carve_s2in(zk_ctx *ctx, int count, const zk_herm *A, std::vector<double *> &hf, std::vector<double *> &w0,
                      std::vector<double *> &V0, std::vector<int *> &flag)
{
    size_t in_total = 0;
    for (int i = 0; i < count; i++) in_total += s2in_bytes(A[i].n, A[i].limbs);
    int rc = ctx->ensure(ctx->s2in, in_total);
    if (rc != ZK_OK) return rc;
    char *b = (char *)ctx->s2in.p;
    for (int i = 0; i < count; i++) {
        const size_t nn = (size_t)A[i].n * A[i].n;
        hf[i] = (double *)b;
        b += align_up(8 * 2 * (size_t)A[i].limbs * nn);
        w0[i] = (double *)b;
        b += align_up(8 * (size_t)A[i].n);
        V0[i] = (double *)b;
        b += align_up(16 * nn);
        flag[i] = (int *)b;
        b += align_up(64);
    }
    return ZK_OK;
}

// Descriptors of one stage-1 batch: np matrices of order n carved from `b`
// (per-matrix scratch, then the descriptor tables), host copies in hp / hg.
static char *carve_stage1(char *b, int n, const std::vector<int> &ids, size_t c0, int np, const zk_herm *A,
                          const std::vector<double *> &hf, const std::vector<double *> &w0, const std::vector<double *> &V0,
                          const std::vector<int *> &flag, std::vector<ProbDesc> &hp, std::vector<GemmDesc> &hg,
                          ProbDesc *&d_probs, GemmDesc *&d_gemm)
{
    hp.assign(np, ProbDesc());
    const size_t nn = (size_t)n * n, ntile = (size_t)(n + 63) / 64, npan = (size_t)(n + kNB - 1) / kNB + 1;
    for (int q = 0; q < np; q++) {
        const int i = ids[c0 + q];
        ProbDesc &P = hp[q];
        std::memset(&P, 0, sizeof P);
        P.n = n;
        P.lda_in = A[i].lda;
        P.limbs_in = A[i].limbs;
        for (int l = 0; l < A[i].limbs; l++) P.in[l] = (const double *)A[i].plane[l];
        P.hf = hf[i];
        P.w0 = w0[i];
        P.V0 = V0[i];
        P.flag = flag[i];
        P.A = (double *)b; b += align_up(16 * nn);
        P.Y = (double *)b; b += align_up(16 * nn);
        P.tau = (double *)b; b += align_up(16 * (size_t)n);
        P.P = (double *)b; b += align_up(16 * (size_t)n * 2 * kNB);
        P.Q = (double *)b; b += align_up(16 * (size_t)n * 2 * kNB);
        P.part = (double *)b; b += align_up(16 * 2 * ntile * n);
        P.tri = (double *)b; b += align_up(8 * 5 * nn);
        P.Zt = (double *)b; b += align_up(8 * nn);
        P.d = (double *)b; b += align_up(8 * (size_t)n);
        P.e = (double *)b; b += align_up(8 * (size_t)n);
        P.cnt = (int *)b; b += align_up(8 * (size_t)n);
        P.scr = (double *)b; b += align_up(8 * (ntile * (4 + 4 * (size_t)kNB) + 2));
        P.Z = (double *)b; b += align_up(8 * nn);
        P.T = (double *)b; b += align_up(16 * npan * kNB * kNB);
        P.X = (double *)b; b += align_up(16 * (size_t)kNB * n);
        P.X2 = (double *)b; b += align_up(16 * (size_t)kNB * n);
        b += align_up(64);
    }
    d_probs = (ProbDesc *)b;
    b += align_up(sizeof(ProbDesc) * np);
    d_gemm = (GemmDesc *)b;
    hg.assign(stage1_gemm_desc_count(n, np), GemmDesc());
    if (n > 1) stage1_fill_gemm_descs(hp.data(), np, hg.data());
    b += align_up(sizeof(GemmDesc) * hg.size());
    return b;
}

static size_t stage1_batch_bytes(int n, int np)
{
    return (size_t)np * s1_bytes(n) + align_up(sizeof(ProbDesc) * np) + align_up(sizeof(GemmDesc) * stage1_gemm_desc_count(n, np));
}

// Stage 1 for `count` matrices into caller-chosen buffers: hf (limb-planar
// copy, 2*limbs*n*n doubles), w0 (n), V0 (n*n complex), flag (int, zeroed
// here); ZK_EINVAL on non-finite input.  Matrices are batched by order; when
// every batch fits the budget at once, batches of different orders run
// concurrently on the context stream and up to three side streams (each
// batch is a chain of small per-column launches, so they overlap well).
int run_stage1(zk_ctx *ctx, int count, const zk_herm *A, const std::vector<double *> &hf, const std::vector<double *> &w0,
               const std::vector<double *> &V0, const std::vector<int *> &flag, const std::vector<int> &fp32)
{
    hipStream_t st = ctx->stream;
    int rc;
    for (int i = 0; i < count; i++) HIPCHK(hipMemsetAsync(flag[i], 0, 4, st));
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int i = 0; i < count; i++) groups[std::make_pair(A[i].n, fp32.empty() ? 0 : (fp32[i] ? 1 : 0))].push_back(i);
    size_t total = 0;
    for (auto &kv : groups) total += stage1_batch_bytes(kv.first.first, (int)kv.second.size());
    if (total > ctx->s1.bytes) ctx->make_room(total - ctx->s1.bytes);
    const size_t avail = ctx->budget > ctx->held() - ctx->s1.bytes ? ctx->budget - (ctx->held() - ctx->s1.bytes) : 0;
    // (inside the no-allocation entry point the side streams and events are
    // not created: every batch runs on the context stream)
    if (groups.size() > 1 && total <= avail && !ctx->arena) {
        if ((rc = ctx->ensure(ctx->s1, total)) != ZK_OK) return rc;
        for (int k = 0; k < 3; k++)
            if (!ctx->side[k]) HIPCHK(hipStreamCreateWithFlags(&ctx->side[k], hipStreamNonBlocking));
        for (int k = 0; k < 4; k++)
            if (!ctx->ev[k]) HIPCHK(hipEventCreateWithFlags(&ctx->ev[k], hipEventDisableTiming));
        // the side streams start after everything already enqueued on the context stream
        HIPCHK(hipEventRecord(ctx->ev[0], st));
        for (int k = 0; k < 3; k++) HIPCHK(hipStreamWaitEvent(ctx->side[k], ctx->ev[0], 0));
        std::vector<std::vector<ProbDesc>> hps(groups.size());
        std::vector<std::vector<GemmDesc>> hgs(groups.size());
        char *b = (char *)ctx->s1.p;
        int gi = 0;
        bool used[3] = {false, false, false};
        for (auto &kv : groups) {
            const int n = kv.first.first;
            const std::vector<int> &ids = kv.second;
            const int np = (int)ids.size();
            const int lane = gi % 4;
            hipStream_t sg = lane == 0 ? st : ctx->side[lane - 1];
            if (lane > 0) used[lane - 1] = true;
            ProbDesc *d_probs;
            GemmDesc *d_gemm;
            std::vector<ProbDesc> &hp = hps[gi];
            std::vector<GemmDesc> &hg = hgs[gi];
            b = carve_stage1(b, n, ids, 0, np, A, hf, w0, V0, flag, hp, hg, d_probs, d_gemm);
            // the reflector array must start zero (entries above row c+1 are read as zeros)
            for (int q = 0; q < np; q++) HIPCHK(hipMemsetAsync(hp[q].Y, 0, 16 * (size_t)n * n, sg));
            HIPCHK(hipMemcpyAsync(d_probs, hp.data(), sizeof(ProbDesc) * np, hipMemcpyHostToDevice, sg));
            if (!hg.empty()) HIPCHK(hipMemcpyAsync(d_gemm, hg.data(), sizeof(GemmDesc) * hg.size(), hipMemcpyHostToDevice, sg));
            Stage1Batch S1;
            S1.n = n;
            S1.nprob = np;
            S1.dev_probs = d_probs;
            S1.dev_gemm = d_gemm;
            S1.tri_gap_rel = 1e-12;
            S1.fp32 = kv.first.second;
            S1.timer = ctx->tp();
            const int t1 = S1.timer ? S1.timer->begin(KC_STAGE1, (double)np, sg) : -1;
            if (stage1_run(S1, sg)) return ctx->fail(ZK_EDEVICE, "stage1 launch failed: %s", hipGetErrorString(hipGetLastError()));
            if (S1.timer) S1.timer->end(t1, sg);
            gi++;
        }
        // join: the context stream waits for every side stream that ran a batch
        for (int k = 0; k < 3; k++)
            if (used[k]) {
                HIPCHK(hipEventRecord(ctx->ev[k + 1], ctx->side[k]));
                HIPCHK(hipStreamWaitEvent(st, ctx->ev[k + 1], 0));
            }
        HIPCHK(hipStreamSynchronize(st));   // host descriptor arrays go out of scope
    } else {
        // one batch at a time, as many matrices of a batch as the budget allows
        for (auto &kv : groups) {
            const int n = kv.first.first;
            const std::vector<int> &ids = kv.second;
            const size_t per = s1_bytes(n);
            const size_t av = ctx->budget > ctx->held() - ctx->s1.bytes ? ctx->budget - (ctx->held() - ctx->s1.bytes) : 0;
            int chunk = (int)std::min<size_t>(ids.size(), av / std::max<size_t>(per, 1));
            if (chunk < 1) return ctx->fail(ZK_ENOMEM, "binary64 stage of order %d needs %zu bytes", n, per);
            if ((rc = ctx->ensure(ctx->s1, stage1_batch_bytes(n, chunk))) != ZK_OK) return rc;
            for (size_t c0 = 0; c0 < ids.size(); c0 += (size_t)chunk) {
                const int np = (int)std::min<size_t>((size_t)chunk, ids.size() - c0);
                std::vector<ProbDesc> hp;
                std::vector<GemmDesc> hg;
                ProbDesc *d_probs;
                GemmDesc *d_gemm;
                carve_stage1((char *)ctx->s1.p, n, ids, c0, np, A, hf, w0, V0, flag, hp, hg, d_probs, d_gemm);
                for (int q = 0; q < np; q++) HIPCHK(hipMemsetAsync(hp[q].Y, 0, 16 * (size_t)n * n, st));
                HIPCHK(hipMemcpyAsync(d_probs, hp.data(), sizeof(ProbDesc) * np, hipMemcpyHostToDevice, st));
                if (!hg.empty()) HIPCHK(hipMemcpyAsync(d_gemm, hg.data(), sizeof(GemmDesc) * hg.size(), hipMemcpyHostToDevice, st));
                Stage1Batch S1;
                S1.n = n;
                S1.nprob = np;
                S1.dev_probs = d_probs;
                S1.dev_gemm = d_gemm;
                S1.tri_gap_rel = 1e-12;
                S1.fp32 = kv.first.second;
                S1.timer = ctx->tp();
                const int t1 = S1.timer ? S1.timer->begin(KC_STAGE1, (double)np, st) : -1;
                if (stage1_run(S1, st)) return ctx->fail(ZK_EDEVICE, "stage1 launch failed: %s", hipGetErrorString(hipGetLastError()));
                if (S1.timer) S1.timer->end(t1, st);
                HIPCHK(hipStreamSynchronize(st));   // host descriptor arrays go out of scope
            }
        }
    }
    // non-finite input?
    std::vector<int> fl(count, 0);
    for (int i = 0; i < count; i++) HIPCHK(hipMemcpyAsync(&fl[i], flag[i], 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < count; i++)
        if (fl[i]) return ctx->fail(ZK_EINVAL, "matrix %d has NaN/Inf entries", i);
    return ZK_OK;
}

template <int L>
static int run_heev(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out *out, const zk_opts *opts, Stage2Stats *stats)
{
    if (!ctx) return ZK_EINVAL;
    if (ctx->poisoned) return ctx->fail(ZK_EDEVICE, "context poisoned by an earlier device error");
    if (count < 1 || !A || !out) return ctx->fail(ZK_EINVAL, "count < 1 or NULL arrays");
    const ResolvedOpts O = zk_resolve_opts(opts, L);
    for (int i = 0; i < count; i++) {
        if (check_herm(A[i]) != ZK_OK) return ctx->fail(ZK_EINVAL, "matrix %d: bad n/lda/limbs/planes", i);
        if (check_out(out[i], A[i].n, A[i].n, L, O.want_vectors) != ZK_OK)
            return ctx->fail(ZK_EINVAL, "output %d: bad n/limbs/ldv or NULL pointers", i);
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(ZK_EDEVICE, "hipSetDevice failed");
    std::vector<double *> hf(count), w0(count), V0(count);
    std::vector<int *> flag(count);
    int rc = carve_s2in(ctx, count, A, hf, w0, V0, flag);
    if (rc != ZK_OK) return rc;
    if ((rc = run_stage1(ctx, count, A, hf, w0, V0, flag, std::vector<int>(count, O.init_fp32))) != ZK_OK) return rc;
    std::vector<RqiProb> rp(count);
    std::vector<int> npair_of(count);
    std::vector<zk_pair_info *> infos(count);
    for (int i = 0; i < count; i++) {
        RqiProb &P = rp[i];
        std::memset(&P, 0, sizeof P);
        P.n = A[i].n;
        P.limbs_in = A[i].limbs;
        P.hf = hf[i];
        P.w0 = w0[i];
        P.V0 = V0[i];
        P.ldv0 = A[i].n;
        P.hnorm = 0.0;
        P.ldv_out = out[i].ldv;
        for (int l = 0; l < L; l++) {
            P.w_out[l] = out[i].w[l];
            P.v_out[l] = O.want_vectors ? (double *)out[i].v[l] : nullptr;
        }
        npair_of[i] = A[i].n;
        infos[i] = out[i].info;
    }
    return run_stage2<L>(ctx, rp, npair_of, infos, O, stats);
}

namespace zk {
int allpairs_run(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out *out, double tol, int max_iter, int want_vectors,
                 const std::vector<double *> &hf, const std::vector<double *> &w0, const std::vector<double *> &V0,
                 int *iters_used);
}

static int run_heev_allpairs(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out *out, const zk_opts *opts)
{
    if (!ctx) return ZK_EINVAL;
    if (ctx->poisoned) return ctx->fail(ZK_EDEVICE, "context poisoned by an earlier device error");
    if (count < 1 || !A || !out) return ctx->fail(ZK_EINVAL, "count < 1 or NULL arrays");
    const ResolvedOpts O = zk_resolve_opts(opts, 2);
    for (int i = 0; i < count; i++) {
        if (check_herm(A[i]) != ZK_OK) return ctx->fail(ZK_EINVAL, "matrix %d: bad n/lda/limbs/planes", i);
        if (check_out(out[i], A[i].n, A[i].n, 2, O.want_vectors) != ZK_OK)
            return ctx->fail(ZK_EINVAL, "output %d: bad n/limbs/ldv or NULL pointers", i);
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(ZK_EDEVICE, "hipSetDevice failed");
    std::vector<double *> hf(count), w0(count), V0(count);
    std::vector<int *> flag(count);
    int rc = carve_s2in(ctx, count, A, hf, w0, V0, flag);
    if (rc != ZK_OK) return rc;
    if ((rc = run_stage1(ctx, count, A, hf, w0, V0, flag, std::vector<int>(count, O.init_fp32))) != ZK_OK) return rc;
    const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 12;
    // matrices of equal order are refined together
    std::map<int, std::vector<int>> groups;
    for (int i = 0; i < count; i++) groups[A[i].n].push_back(i);
    int status = ZK_OK;
    for (auto &kv : groups) {
        const std::vector<int> &ids = kv.second;
        std::vector<zk_herm> a;
        std::vector<zk_eig_out> o;
        std::vector<double *> h, w, v;
        for (int i : ids) {
            a.push_back(A[i]);
            o.push_back(out[i]);
            h.push_back(hf[i]);
            w.push_back(w0[i]);
            v.push_back(V0[i]);
        }
        rc = zk::allpairs_run(ctx, (int)ids.size(), a.data(), o.data(), O.tol, max_iter, O.want_vectors, h, w, v, nullptr);
        if (rc < 0) return rc;
        if (rc == ZK_ENOCONV) status = ZK_ENOCONV;
    }
    return status;
}

extern "C" int zk_heev_dd_allpairs(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out *out, const zk_opts *opts)
{
    return run_heev_allpairs(ctx, count, A, out, opts);
}

namespace zk {
template <int L>
int mp_polish_run(zk_ctx *ctx, int np, int n, const int *limbs_in, const double *const *hf,
                  const double *const *w_dd, const double2 *const *v_dd, double *const *w_out, double2 *const *v_out,
                  const int *ldv, zk_pair_info *const *info, double tol, int max_iter, int *iters_used);
}

// Eigendecomposition beyond double-double: the double-double all-pairs
// refinement, then the L-limb polishing (mp_polish.hip).
extern "C" int zk_heev_mp(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out_mp *out, const zk_opts *opts)
{
    if (!ctx) return ZK_EINVAL;
    if (ctx->poisoned) return ctx->fail(ZK_EDEVICE, "context poisoned by an earlier device error");
    if (count < 1 || !A || !out) return ctx->fail(ZK_EINVAL, "count < 1 or NULL arrays");
    const int L = out[0].limbs;
    if (L != 4 && L != 8 && L != 16) return ctx->fail(ZK_EINVAL, "limbs must be 4, 8 or 16");
    const bool want = opts ? (opts->want_vectors != 0) : true;
    for (int i = 0; i < count; i++) {
        if (check_herm(A[i]) != ZK_OK) return ctx->fail(ZK_EINVAL, "matrix %d: bad n/lda/limbs/planes", i);
        const zk_eig_out_mp &o = out[i];
        if (o.limbs != L || o.n != A[i].n || !o.w || (want && (!o.v || o.ldv < A[i].n)))
            return ctx->fail(ZK_EINVAL, "output %d: bad n/limbs/ldv or NULL pointers", i);
    }
    const double tol = (opts && opts->tol > 0.0) ? opts->tol : (L == 4 ? 1e-60 : (L == 8 ? 1e-120 : 1e-240));
    const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 8 + 3 * L;
    if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(ZK_EDEVICE, "hipSetDevice failed");
    std::vector<double *> hf(count), w0(count), V0(count);
    std::vector<int *> flag(count);
    int rc = carve_s2in(ctx, count, A, hf, w0, V0, flag);
    if (rc != ZK_OK) return rc;
    if ((rc = run_stage1(ctx, count, A, hf, w0, V0, flag, std::vector<int>(count, 0))) != ZK_OK) return rc;
    // double-double start of every matrix: eigenvalue limbs and eigenvector limb planes
    std::vector<size_t> off(count + 1, 0);
    for (int i = 0; i < count; i++) {
        const size_t n = A[i].n;
        off[i + 1] = off[i] + align_up(16 * n) + 2 * align_up(16 * n * n);
    }
    if (!ctx->make_room(off[count])) return ctx->fail(ZK_ENOMEM, "the double-double start needs %zu bytes", off[count]);
    void *buf = nullptr;
    if (ctx->dev_alloc(&buf, off[count]) != ZK_OK) return ZK_ENOMEM;
    ctx->extra += off[count];
    ctx->note_held();
    auto release = [&](int r) {
        hipStreamSynchronize(ctx->stream);
        ctx->dev_free(buf);
        ctx->extra -= off[count];
        return r;
    };
    std::vector<zk_eig_out> dd(count);
    for (int i = 0; i < count; i++) {
        const size_t n = A[i].n;
        char *b = (char *)buf + off[i];
        zk_eig_out &o = dd[i];
        std::memset(&o, 0, sizeof o);
        o.n = A[i].n;
        o.ldv = A[i].n;
        o.limbs = 2;
        o.w[0] = (double *)b;
        o.w[1] = (double *)b + n;
        o.v[0] = b + align_up(16 * n);
        o.v[1] = b + align_up(16 * n) + align_up(16 * n * n);
        o.info = nullptr;
    }
    std::map<int, std::vector<int>> groups;
    for (int i = 0; i < count; i++) groups[A[i].n].push_back(i);
    int status = ZK_OK;
    for (auto &kv : groups) {
        const int n = kv.first;
        const std::vector<int> &ids = kv.second;
        std::vector<zk_herm> a;
        std::vector<zk_eig_out> o;
        std::vector<double *> h, w, v;
        for (int i : ids) {
            a.push_back(A[i]);
            o.push_back(dd[i]);
            h.push_back(hf[i]);
            w.push_back(w0[i]);
            v.push_back(V0[i]);
        }
        rc = zk::allpairs_run(ctx, (int)ids.size(), a.data(), o.data(), 1e-31, 12, 1, h, w, v, nullptr);
        if (rc < 0) return release(rc);
        std::vector<int> lin;
        std::vector<const double *> hfp, wdd;
        std::vector<const double2 *> vdd;
        std::vector<double *> wo;
        std::vector<double2 *> vo;
        std::vector<int> ldv;
        std::vector<zk_pair_info *> inf;
        for (int i : ids) {
            lin.push_back(A[i].limbs);
            hfp.push_back(hf[i]);
            wdd.push_back(dd[i].w[0]);
            vdd.push_back((const double2 *)dd[i].v[0]);
            vdd.push_back((const double2 *)dd[i].v[1]);
            wo.push_back(out[i].w);
            vo.push_back(want ? (double2 *)out[i].v : nullptr);
            ldv.push_back(want ? out[i].ldv : n);
            inf.push_back(out[i].info);
        }
        const int np = (int)ids.size();
        if (L == 4)
            rc = zk::mp_polish_run<4>(ctx, np, n, lin.data(), hfp.data(), wdd.data(), vdd.data(), wo.data(), vo.data(),
                                      ldv.data(), inf.data(), tol, max_iter, nullptr);
        else if (L == 8)
            rc = zk::mp_polish_run<8>(ctx, np, n, lin.data(), hfp.data(), wdd.data(), vdd.data(), wo.data(), vo.data(),
                                      ldv.data(), inf.data(), tol, max_iter, nullptr);
        else
            rc = zk::mp_polish_run<16>(ctx, np, n, lin.data(), hfp.data(), wdd.data(), vdd.data(), wo.data(), vo.data(),
                                       ldv.data(), inf.data(), tol, max_iter, nullptr);
        if (rc < 0) return release(rc);
        if (rc == ZK_ENOCONV) status = ZK_ENOCONV;
    }
    return release(status);
}

extern "C" int zk_svd_dd(zk_ctx *ctx, int count, const zk_mat *A, zk_svd_out *out, const zk_opts *opts)
{
    if (!ctx) return ZK_EINVAL;
    if (ctx->poisoned) return ctx->fail(ZK_EDEVICE, "context poisoned by an earlier device error");
    if (count < 1 || !A || !out) return ctx->fail(ZK_EINVAL, "count < 1 or NULL arrays");
    const ResolvedOpts O = zk_resolve_opts(opts, 2);
    for (int i = 0; i < count; i++) {
        const zk_mat &a = A[i];
        const zk_svd_out &o = out[i];
        bool bad = a.m < 1 || a.n < 1 || a.lda < a.m || (a.limbs != 1 && a.limbs != 2 && a.limbs != 4);
        for (int l = 0; !bad && l < a.limbs; l++) bad = !a.plane[l];
        bad = bad || o.m != a.m || o.n != a.n || o.limbs != 2 || !o.s[0] || !o.s[1];
        if (!bad && O.want_vectors) bad = !o.u[0] || !o.u[1] || !o.v[0] || !o.v[1] || o.ldu < a.m || o.ldv < a.n;
        if (bad) return ctx->fail(ZK_EINVAL, "matrix %d: bad m/n/lda/limbs/planes or output descriptor", i);
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(ZK_EDEVICE, "hipSetDevice failed");
    hipStream_t st = ctx->stream;
    // per matrix: K (limbs planes), eigenvalues (2 limbs), eigenvectors (2 limb planes)
    std::vector<size_t> off(count + 1, 0);
    for (int i = 0; i < count; i++) {
        const size_t N = (size_t)A[i].m + A[i].n;
        off[i + 1] = off[i] + align_up(16 * N * N * A[i].limbs) + 2 * align_up(8 * N) + 2 * align_up(16 * N * N);
    }
    if (!ctx->make_room(off[count])) return ctx->fail(ZK_ENOMEM, "the dilations need %zu bytes", off[count]);
    void *buf = nullptr;
    if (ctx->dev_alloc(&buf, off[count]) != ZK_OK) return ZK_ENOMEM;
    ctx->extra += off[count];
    ctx->note_held();
    std::vector<SvdDesc> D(count);
    std::vector<zk_herm> K(count);
    std::vector<zk_eig_out> E(count);
    std::vector<std::vector<zk_pair_info>> inf(count);
    int rc = ZK_OK;
    for (int i = 0; i < count && rc == ZK_OK; i++) {
        const int m = A[i].m, n = A[i].n, N = m + n;
        const size_t NN = (size_t)N * N;
        char *b = (char *)buf + off[i];
        SvdDesc &d = D[i];
        std::memset(&d, 0, sizeof d);
        d.m = m;
        d.n = n;
        d.lda = A[i].lda;
        d.limbs = A[i].limbs;
        for (int l = 0; l < A[i].limbs; l++) d.A[l] = (const double *)A[i].plane[l];
        d.K = (double *)b;
        b += align_up(16 * NN * A[i].limbs);
        double *w0 = (double *)b;
        b += align_up(8 * (size_t)N);
        double *w1 = (double *)b;
        b += align_up(8 * (size_t)N);
        double *v0 = (double *)b;
        b += align_up(16 * NN);
        double *v1 = (double *)b;
        d.w[0] = w0;
        d.w[1] = w1;
        d.V[0] = v0;
        d.V[1] = v1;
        d.s[0] = out[i].s[0];
        d.s[1] = out[i].s[1];
        if (O.want_vectors) {
            d.u[0] = (double *)out[i].u[0];
            d.u[1] = (double *)out[i].u[1];
            d.v[0] = (double *)out[i].v[0];
            d.v[1] = (double *)out[i].v[1];
            d.ldu = out[i].ldu;
            d.ldv = out[i].ldv;
        }
        if (svd_build(d, st)) rc = ctx->fail(ZK_EDEVICE, "dilation build failed");
        zk_herm &h = K[i];
        std::memset(&h, 0, sizeof h);
        h.n = N;
        h.lda = N;
        h.limbs = A[i].limbs;
        for (int l = 0; l < A[i].limbs; l++) h.plane[l] = d.K + 2 * NN * l;
        zk_eig_out &e = E[i];
        std::memset(&e, 0, sizeof e);
        e.n = N;
        e.ldv = N;
        e.limbs = 2;
        e.w[0] = w0;
        e.w[1] = w1;
        e.v[0] = v0;
        e.v[1] = v1;
        inf[i].resize(N);
        e.info = inf[i].data();
    }
    if (rc == ZK_OK) {
        // the eigenvectors are needed for the singular vectors; the dilation's
        // pairs iterate like any other matrix's
        zk_opts oo;
        zk_opts_default(&oo);
        if (opts) oo = *opts;
        oo.want_vectors = 1;
        rc = oo.refine == 1 ? run_heev_allpairs(ctx, count, K.data(), E.data(), &oo)
                            : run_heev<2>(ctx, count, K.data(), E.data(), &oo, nullptr);
    }
    if (rc >= 0) {
        // only the k returned triplets decide the status: the dilation's
        // -s_j and |m - n| zero pairs are not outputs
        bool all_ok = true;
        for (int i = 0; i < count; i++) {
            if (svd_extract(D[i], st)) {
                rc = ctx->fail(ZK_EDEVICE, "singular triplet extraction failed");
                break;
            }
            const int N = A[i].m + A[i].n, k = std::min(A[i].m, A[i].n);
            for (int j = 0; j < k; j++) {
                const zk_pair_info &p = inf[i][N - 1 - j];
                all_ok = all_ok && (p.flags & ZK_PAIR_CONVERGED);
                if (out[i].info) out[i].info[j] = p;
            }
        }
        if (rc >= 0) rc = all_ok ? ZK_OK : ZK_ENOCONV;
    }
    hipStreamSynchronize(st);
    ctx->dev_free(buf);
    ctx->extra -= off[count];
    return rc;
}

extern "C" int zk_mps_two_site_dd(zk_ctx *ctx, int chi_l, int chi, int chi_r, const void *const *A,
                                  const void *const *B, const void *const *gate, int chi_max, double cutoff,
                                  void *const *A_out, void *const *B_out, double *const *s_out, int *chi_out,
                                  const zk_opts *opts)
{
    if (!ctx) return ZK_EINVAL;
    if (ctx->poisoned) return ctx->fail(ZK_EDEVICE, "context poisoned by an earlier device error");
    if (chi_l < 1 || chi < 1 || chi_r < 1) return ctx->fail(ZK_EINVAL, "bond dimensions must be >= 1");
    const int M = 2 * chi_l, N = 2 * chi_r, k = std::min(M, N);
    if (M + N > kMaxN) return ctx->fail(ZK_EINVAL, "2 chi_l + 2 chi_r = %d above the largest order %d", M + N, kMaxN);
    if (chi_max < 1 || chi_max > k) return ctx->fail(ZK_EINVAL, "chi_max %d outside 1 .. %d", chi_max, k);
    if (!(cutoff >= 0.0)) return ctx->fail(ZK_EINVAL, "cutoff must be >= 0");
    if (!A || !B || !gate || !A_out || !B_out || !s_out || !chi_out) return ctx->fail(ZK_EINVAL, "NULL argument");
    for (int l = 0; l < 2; l++)
        if (!A[l] || !B[l] || !gate[l] || !A_out[l] || !B_out[l] || !s_out[l])
            return ctx->fail(ZK_EINVAL, "NULL plane");
    if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(ZK_EDEVICE, "hipSetDevice failed");
    hipStream_t st = ctx->stream;
    // scratch: theta, U, V (two planes each) and the singular value limbs
    const size_t bT = align_up(16 * (size_t)M * N), bU = align_up(16 * (size_t)M * k), bV = align_up(16 * (size_t)N * k),
                 bS = align_up(8 * (size_t)k);
    const size_t bytes = 2 * (bT + bU + bV + bS);
    if (!ctx->make_room(bytes)) return ctx->fail(ZK_ENOMEM, "the two-site update needs %zu bytes", bytes);
    void *buf = nullptr;
    if (ctx->dev_alloc(&buf, bytes) != ZK_OK) return ZK_ENOMEM;
    ctx->extra += bytes;
    ctx->note_held();
    char *b = (char *)buf;
    double *T[2], *U[2], *V[2], *S[2];
    for (int l = 0; l < 2; l++) { T[l] = (double *)b; b += bT; }
    for (int l = 0; l < 2; l++) { U[l] = (double *)b; b += bU; }
    for (int l = 0; l < 2; l++) { V[l] = (double *)b; b += bV; }
    for (int l = 0; l < 2; l++) { S[l] = (double *)b; b += bS; }
    MpsDesc D;
    std::memset(&D, 0, sizeof D);
    D.M = M;
    D.K = chi;
    D.N = N;
    D.chil = chi_l;
    D.chir = chi_r;
    D.lda = M;
    D.ldb = chi;
    for (int l = 0; l < 2; l++) {
        D.A[l] = (const double *)A[l];
        D.B[l] = (const double *)B[l];
        D.T[l] = T[l];
        D.G[l] = (const double *)gate[l];
        D.V[l] = V[l];
        D.s[l] = S[l];
        D.Bo[l] = (double *)B_out[l];
    }
    int rc = ZK_OK;
    if (mps_theta(D, st)) rc = ctx->fail(ZK_EDEVICE, "two-site contraction launch failed");
    if (rc == ZK_OK) {
        zk_mat mat;
        std::memset(&mat, 0, sizeof mat);
        mat.m = M;
        mat.n = N;
        mat.lda = M;
        mat.limbs = 2;
        mat.plane[0] = T[0];
        mat.plane[1] = T[1];
        zk_svd_out so;
        std::memset(&so, 0, sizeof so);
        so.m = M;
        so.n = N;
        so.limbs = 2;
        for (int l = 0; l < 2; l++) {
            so.s[l] = S[l];
            so.u[l] = U[l];
            so.v[l] = V[l];
        }
        so.ldu = M;
        so.ldv = N;
        rc = zk_svd_dd(ctx, 1, &mat, &so, opts);
    }
    if (rc >= 0) {
        std::vector<double> sh(k);
        if (hipMemcpyAsync(sh.data(), S[0], 8 * (size_t)k, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            rc = ctx->fail(ZK_EDEVICE, "singular value download failed");
        int kept = 0;
        if (rc >= 0) {
            while (kept < chi_max && sh[kept] > 0.0 && sh[kept] > cutoff * sh[0]) kept++;
            kept = std::max(kept, 1);
            D.chi = kept;
            D.ldv = N;
            for (int l = 0; l < 2 && rc >= 0; l++) {
                if (hipMemcpyAsync(A_out[l], U[l], 16 * (size_t)M * kept, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                    hipMemcpyAsync(s_out[l], S[l], 8 * (size_t)kept, hipMemcpyDeviceToDevice, st) != hipSuccess)
                    rc = ctx->fail(ZK_EDEVICE, "output copy failed");
            }
            if (rc >= 0 && mps_bout(D, st)) rc = ctx->fail(ZK_EDEVICE, "B' launch failed");
            *chi_out = kept;
        }
    }
    hipStreamSynchronize(st);
    ctx->dev_free(buf);
    ctx->extra -= bytes;
    return rc;
}

extern "C" int zk_heev_fp64(zk_ctx *ctx, int count, const zk_herm *A, double *const *w, void *const *V, const int *ldv)
{
    if (!ctx) return ZK_EINVAL;
    if (ctx->poisoned) return ctx->fail(ZK_EDEVICE, "context poisoned by an earlier device error");
    if (count < 1 || !A || !w || !V || !ldv) return ctx->fail(ZK_EINVAL, "count < 1 or NULL arrays");
    for (int i = 0; i < count; i++) {
        if (check_herm(A[i]) != ZK_OK) return ctx->fail(ZK_EINVAL, "matrix %d: bad n/lda/limbs/planes", i);
        if (!w[i] || !V[i] || ldv[i] < A[i].n) return ctx->fail(ZK_EINVAL, "output %d: NULL or ldv < n", i);
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(ZK_EDEVICE, "hipSetDevice failed");
    std::vector<double *> hf(count), w0(count), V0(count);
    std::vector<int *> flag(count);
    int rc = carve_s2in(ctx, count, A, hf, w0, V0, flag);
    if (rc != ZK_OK) return rc;
    if ((rc = run_stage1(ctx, count, A, hf, w0, V0, flag, std::vector<int>())) != ZK_OK) return rc;
    hipStream_t st = ctx->stream;
    for (int i = 0; i < count; i++) {
        const int n = A[i].n;
        HIPCHK(hipMemcpyAsync(w[i], w0[i], 8 * (size_t)n, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpy2DAsync(V[i], 16 * (size_t)ldv[i], V0[i], 16 * (size_t)n, 16 * (size_t)n, n, hipMemcpyDeviceToDevice, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    return ZK_OK;
}

// The per-pair iteration's counters of the call are kept in the context
// (zk_ctx_last_stats); collecting them is host bookkeeping only.
extern "C" int zk_heev_dd(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out *out, const zk_opts *opts)
{
    if (ctx) ctx->last = Stage2Stats();
    if (opts && opts->refine == 1) return run_heev_allpairs(ctx, count, A, out, opts);
    return run_heev<2>(ctx, count, A, out, opts, ctx ? &ctx->last : nullptr);
}

extern "C" int zk_heev_qd(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out *out, const zk_opts *opts)
{
    if (ctx) ctx->last = Stage2Stats();
    if (opts && opts->refine != 0) return ctx ? ctx->fail(ZK_EINVAL, "the all-pairs refinement gives double-double output only") : ZK_EINVAL;
    return run_heev<4>(ctx, count, A, out, opts, ctx ? &ctx->last : nullptr);
}

extern "C" int zk_ctx_last_stats(const zk_ctx *ctx, int *iters_hist16, int *rounds, long long *solves)
{
    if (!ctx) return ZK_EINVAL;
    if (iters_hist16)
        for (int i = 0; i < 16; i++) iters_hist16[i] = ctx->last.iters_hist[i];
    if (rounds) *rounds = ctx->last.rounds;
    if (solves) *solves = ctx->last.solves;
    return ZK_OK;
}

extern "C" int zk_ctx_memory(const zk_ctx *ctx, size_t *held, size_t *budget, size_t *high_water, size_t *transient)
{
    if (!ctx) return ZK_EINVAL;
    if (held) *held = ctx->held();
    if (budget) *budget = ctx->budget;
    if (high_water) *high_water = std::max(ctx->high_water, ctx->held());
    if (transient) *transient = ctx->extra;
    return ZK_OK;
}

// ====================================================== rqi_refine ========
template <int L>
static int run_refine(zk_ctx *ctx, const zk_herm *A, int k, const double *w0, const void *V0, int ldv0,
                      zk_eig_out *out, const zk_opts *opts)
{
    if (!ctx) return ZK_EINVAL;
    if (ctx->poisoned) return ctx->fail(ZK_EDEVICE, "context poisoned by an earlier device error");
    if (!A || !out || !w0 || !V0) return ctx->fail(ZK_EINVAL, "NULL argument");
    if (check_herm(*A) != ZK_OK) return ctx->fail(ZK_EINVAL, "bad n/lda/limbs/planes");
    const ResolvedOpts O = zk_resolve_opts(opts, L);
    if (k < 1 || k > A->n || ldv0 < A->n) return ctx->fail(ZK_EINVAL, "bad k or ldv0");
    if (check_out(*out, k, A->n, L, O.want_vectors) != ZK_OK) return ctx->fail(ZK_EINVAL, "bad output descriptor");
    if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(ZK_EDEVICE, "hipSetDevice failed");
    hipStream_t st = ctx->stream;
    const int n = A->n;
    int rc;
    if ((rc = ctx->ensure(ctx->s2in, s2in_bytes(n, A->limbs))) != ZK_OK) return rc;
    char *b = (char *)ctx->s2in.p;
    double *hf = (double *)b;
    b += align_up(8 * 2 * (size_t)A->limbs * (size_t)n * n);
    b += align_up(8 * (size_t)n) + align_up(16 * (size_t)n * n);
    int *flag = (int *)b;
    HIPCHK(hipMemsetAsync(flag, 0, 4, st));
    const double *pl[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int l = 0; l < A->limbs; l++) pl[l] = (const double *)A->plane[l];
    if (stage2_ingest(n, A->lda, A->limbs, pl, hf, flag, st)) return ctx->fail(ZK_EDEVICE, "ingest launch failed");
    int f = 0;
    HIPCHK(hipMemcpyAsync(&f, flag, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (f) return ctx->fail(ZK_EINVAL, "input has NaN/Inf entries");
    std::vector<RqiProb> rp(1);
    RqiProb &P = rp[0];
    std::memset(&P, 0, sizeof P);
    P.n = n;
    P.limbs_in = A->limbs;
    P.hf = hf;
    P.w0 = w0;
    P.V0 = (const double *)V0;
    P.ldv0 = ldv0;
    P.ldv_out = out->ldv;
    for (int l = 0; l < L; l++) {
        P.w_out[l] = out->w[l];
        P.v_out[l] = O.want_vectors ? (double *)out->v[l] : nullptr;
    }
    std::vector<int> npair_of(1, k);
    std::vector<zk_pair_info *> infos(1, out->info);
    return run_stage2<L>(ctx, rp, npair_of, infos, O, nullptr);
}

extern "C" int zk_rqi_refine(zk_ctx *ctx, int limbs_out, const zk_herm *A, int k, const double *w0, const void *V0,
                             int ldv0, zk_eig_out *out, const zk_opts *opts)
{
    if (limbs_out == 2) return run_refine<2>(ctx, A, k, w0, V0, ldv0, out, opts);
    if (limbs_out == 4) return run_refine<4>(ctx, A, k, w0, V0, ldv0, out, opts);
    if (ctx) ctx->fail(ZK_EINVAL, "limbs_out must be 2 or 4");
    return ZK_EINVAL;
}

// ------------------------------------------------------ instrumentation --
extern "C" int zk_prof_enable(zk_ctx *ctx, int on)
{
    if (!ctx) return ZK_EINVAL;
    ctx->timer.collect();
    ctx->timer.on = on != 0;
    return ZK_OK;
}

extern "C" int zk_prof_classes(zk_ctx *ctx, unsigned mask)
{
    if (!ctx) return ZK_EINVAL;
    ctx->timer.collect();
    ctx->timer.mask = mask;
    return ZK_OK;
}

extern "C" int zk_prof_reset(zk_ctx *ctx)
{
    if (!ctx) return ZK_EINVAL;
    ctx->timer.reset();
    return ZK_OK;
}

extern "C" int zk_prof_read(zk_ctx *ctx, int cls, double *ms, long long *launches, double *work)
{
    if (!ctx || cls < 0 || cls >= KC_COUNT) return ZK_EINVAL;
    ctx->timer.collect();
    if (ms) *ms = ctx->timer.ms[cls];
    if (launches) *launches = ctx->timer.launches[cls];
    if (work) *work = ctx->timer.work[cls];
    return ZK_OK;
}

