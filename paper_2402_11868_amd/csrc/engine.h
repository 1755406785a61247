// Stage-2 engine: the Rayleigh quotient iteration of any number of matrices,
// driven round by round.  Matrices can join (add) and leave (when all their
// pairs have finished) between rounds, which is what the serving session
// uses for continuous batching; the one-shot zk_heev_* calls add everything
// at once and run rounds until nothing is active.  Every kernel works per
// pair, per cluster or per matrix, so a matrix's result does not depend on
// what else is in the batch.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "../../include/zk.h"
#include "api_internal.h"
#include "stage.h"

int run_stage1(zk_ctx *ctx, int count, const zk_herm *A, const std::vector<double *> &hf, const std::vector<double *> &w0,
               const std::vector<double *> &V0, const std::vector<int *> &flag, const std::vector<int> &fp32);

#define HIPCHK_(expr)                                          \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return HIPFAIL(e_, #expr);       \
    } while (0)

namespace zk {

struct ResolvedOpts {
    double tol;
    int max_iter;
    double cluster_tol;
    int want_vectors;
    int init_fp32;
    int reorth;
    int refine;
    int ldl;            // shifted solves by LDL^H (Bunch-Kaufman) instead of LU
    int max_iter_set;   // the caller's max_iter (0: default)
};

inline size_t s2_align(size_t x) { return (x + 255) & ~(size_t)255; }
inline int s2_lu_ldm(int n) { return (n + 7) & ~7; }
inline size_t s2_lu_slot_doubles(int n, int L) { return (size_t)2 * L * lu_plane_of(n); }

// One matrix in the engine.  The caller sets rp (n, limbs_in, hf, w0, V0,
// ldv0, ldv_out, w_out, v_out, hnorm lower bound), npairs and info.
struct S2Prob {
    RqiProb rp;
    ResolvedOpts opts;
    int npairs = 0;
    zk_pair_info *info = nullptr;
    std::vector<PairDesc> pairs;   // authoritative host copy of the pair states
    std::vector<int> heads;        // local index of every cluster's first pair
    std::vector<std::pair<int, int>> rrb;   // Rayleigh-Ritz blocks (first pair, members), 2..32 members
    std::vector<double> w0h;       // binary64 eigenvalues (ascending) the clusters were planned on
    std::vector<double> ritz0;     // shift for the first solve from the deepest projected level (NaN: none)
    std::vector<int> redo;         // pairs sent back for more iterations after the re-orthogonalisation
    int polish = 0;                // number of such passes so far
    void *vecbuf = nullptr;
    size_t vecbytes = 0;
    int status = ZK_OK;
    bool done = false;
    void *cookie = nullptr;        // owner's handle (session request)
};

template <int L>
class Stage2Engine {
  public:
    Stage2Engine(zk_ctx *c, const ResolvedOpts &o, Stage2Stats *s) : ctx(c), O(o), stats(s)
    {
        st = c->stream;
        // ZK_S2_SPLIT=0: every chunk of pairs in one group (for measurements)
        const char *e = std::getenv("ZK_S2_SPLIT");
        s2_split_ = !(e && e[0] == '0');
    }
    ~Stage2Engine()
    {
        for (S2Prob *p : live) release(p);
        if (gsbuf) {
            ctx->dev_free(gsbuf);
            ctx->extra -= gsbytes;
        }
    }

    std::vector<S2Prob *> live;      // matrices still iterating
    std::vector<S2Prob *> finished;  // filled by round(); the owner takes them

    bool any_live() const { return !live.empty(); }

    // Prepare new matrices (clusters, start vectors, Gram-Schmidt, Rayleigh-Ritz,
    // first Rayleigh quotients) and let them join the iteration.  On failure,
    // the iterate storage of every batch member that did not join is given
    // back, so a failed add leaves the context's budget as it found it.
    int add(const std::vector<S2Prob *> &batch)
    {
        const int rc = add_batch(batch);
        if (rc != ZK_OK)
            for (S2Prob *p : batch)
                if (std::find(live.begin(), live.end(), p) == live.end()) release(p);
        return rc;
    }

  private:
    int add_batch(const std::vector<S2Prob *> &batch)
    {
        int rc;
        std::vector<double> w0h;
        for (S2Prob *p : batch) {
            RqiProb &P = p->rp;
            const int n = P.n, kp = p->npairs;
            p->vecbytes = s2_align(8 * 2 * (size_t)L * n * n) + s2_align(8 * (size_t)L * n);
            if (!ctx->make_room(p->vecbytes)) return ctx->fail(ZK_ENOMEM, "iterate storage exceeds the budget");
            if (ctx->dev_alloc(&p->vecbuf, p->vecbytes) != ZK_OK) return ZK_ENOMEM;
            ctx->extra += p->vecbytes;
            ctx->note_held();
            P.vec = (double *)p->vecbuf;
            P.sigma = (double *)((char *)p->vecbuf + s2_align(8 * 2 * (size_t)L * n * n));
            w0h.resize(kp);
            HIPCHK_(hipMemcpyAsync(w0h.data(), P.w0, 8 * (size_t)kp, hipMemcpyDeviceToHost, st));
            HIPCHK_(hipStreamSynchronize(st));
            p->w0h = w0h;
            double hn = 0.0;
            for (int k = 0; k < kp; k++) hn = std::max(hn, std::fabs(w0h[k]));
            hn = std::max(hn, P.hnorm);
            if (!(hn > 0.0)) hn = 1.0;   // zero matrix: absolute tolerances
            P.hnorm = hn;
            P.tol_abs = p->opts.tol * hn;
            P.piv_tol = std::ldexp(hn, -53 * L);
            P.max_iter = p->opts.max_iter;
            plan_clusters(p, w0h, p->opts.init_fp32 ? 2 : 0);
        }
        if ((rc = upload(batch)) != ZK_OK) return rc;
        if (stage2_init<L>(d_pairs, d_probs, total_pairs, st)) return ctx->fail(ZK_EDEVICE, "init launch failed");
        for (S2Prob *p : batch)
            for (auto &q : p->pairs) q.status = 0;
        // An FP32 start resolves the spectrum only to about 2^-24 ||H||: one
        // Rayleigh-Ritz step on the whole basis (made orthonormal in L limbs
        // first) gives binary64-quality pairs, and the clusters are planned
        // again on its Ritz values.
        bool any32 = false;
        for (S2Prob *p : batch) any32 = any32 || p->opts.init_fp32;
        if (any32) {
            // only the FP32-start matrices take part (the others' pairs are
            // frozen for this step), so every result stays independent of
            // the rest of the batch
            for (S2Prob *p : batch)
                if (!p->opts.init_fp32)
                    for (auto &q : p->pairs) q.status = 1;
            rc = run_gs(batch, false);
            for (S2Prob *p : batch)
                if (!p->opts.init_fp32)
                    for (auto &q : p->pairs) q.status = 0;
            if (rc != ZK_OK) return rc;
            std::vector<PrrBlock> whole;
            for (size_t pi = 0; pi < batch.size(); pi++)
                if (batch[pi]->opts.init_fp32 && batch[pi]->npairs >= 2) whole.push_back({(int)pi, 0, batch[pi]->npairs});
            std::vector<std::vector<double>> rz;
            if ((rc = prr_project(batch, whole, rz)) != ZK_OK) return rc;
            for (size_t b = 0; b < whole.size(); b++) {
                S2Prob *p = batch[whole[b].pi];
                p->w0h = rz[b];   // the Ritz values replace the binary64 eigenvalues
                plan_clusters(p, p->w0h, 0);
                for (auto &q : p->pairs) q.status = 0;
            }
            if ((rc = upload(batch)) != ZK_OK) return rc;
        }
        if ((rc = run_gs(batch, false)) != ZK_OK) return rc;
        bool projected = false;
        if ((rc = run_prr(batch, projected)) != ZK_OK) return rc;
        if (projected && (rc = run_gs(batch, false)) != ZK_OK) return rc;
        if ((rc = run_rr(batch, true)) != ZK_OK) return rc;
        std::vector<int> all(total_pairs);
        for (int g = 0; g < total_pairs; g++) all[g] = g;
        if ((rc = run_rq(all, 0)) != ZK_OK) return rc;
        if (projected && (rc = first_shifts(batch)) != ZK_OK) return rc;
        if ((rc = download(batch)) != ZK_OK) return rc;
        if (std::getenv("ZK_TRACE") && std::atoi(std::getenv("ZK_TRACE")) >= 2) dump(batch, "add");
        for (S2Prob *p : batch) live.push_back(p);
        return settle();
    }

  public:
    // One round over every live matrix: shifted solves of all active pairs,
    // Gram-Schmidt in their clusters, Rayleigh quotients and convergence.
    // Matrices whose pairs have all stopped are finalised and moved to `finished`.
    int round()
    {
        int rc;
        if (live.empty()) return ZK_OK;
        if ((rc = upload(live)) != ZK_OK) return rc;
        // Solves use the LDL^H factorisation (when selected) until a pair's
        // residual stalls near the tolerance (flag 16, set by the Rayleigh
        // quotient step), then LU, whose smaller backward error decides there
        // (the SVD dilations of random matrices: some of their smallest
        // singular values stall at 2e-30 with LDL^H alone)
        std::map<int, std::vector<int>> by_n, first, later;
        int nact = 0, nfirst = 0;
        for (size_t pi = 0; pi < live.size(); pi++)
            for (int k = 0; k < live[pi]->npairs; k++)
                if (live[pi]->pairs[k].status == 0) {
                    const int g = base[pi] + k, n = live[pi]->rp.n;
                    by_n[n].push_back(g);
                    const bool f = O.ldl && !(live[pi]->pairs[k].flags & 16);
                    (f ? first : later)[n].push_back(g);
                    nfirst += f ? 1 : 0;
                    nact++;
                }
        if (stats) stats->active_per_iter.push_back(nact);
        if (nact > 0) {
            if (!first.empty() && (rc = solve_pairs(first, nfirst, true)) != ZK_OK) return rc;
            if (!later.empty() && (rc = solve_pairs(later, nact - nfirst, false)) != ZK_OK) return rc;
            if ((rc = run_gs(live, false)) != ZK_OK) return rc;
            if ((rc = run_rr(live, false)) != ZK_OK) return rc;
            std::vector<int> all;
            for (auto &kv : by_n) all.insert(all.end(), kv.second.begin(), kv.second.end());
            if ((rc = run_rq(all, 0)) != ZK_OK) return rc;
            if ((rc = download(live)) != ZK_OK) return rc;
            rounds++;
            if (std::getenv("ZK_TRACE")) trace();
            if (std::getenv("ZK_TRACE") && std::atoi(std::getenv("ZK_TRACE")) >= 2) dump(live, "round");
        }
        return settle();
    }

    int rounds = 0;
    static constexpr int kPolishPasses = 2;
    static constexpr int kPrrLevels = 40;
    static constexpr double kPrrDeep = 1e-3;
    static constexpr double kPurify = 1e-18;
    static constexpr double kReorthWindow = 0.1;
    static constexpr int kSplitMin = 8;   // pairs per group below which a chunk is not split

  private:
    bool s2_split_ = false;
    zk_ctx *ctx;
    ResolvedOpts O;
    Stage2Stats *stats;
    hipStream_t st;
    // device tables of the current upload
    std::vector<int> base;   // pair-table offset of every uploaded matrix
    int total_pairs = 0;
    PairDesc *d_pairs = nullptr;
    RqiProb *d_probs = nullptr;
    int *d_active = nullptr, *d_dst = nullptr, *d_glist = nullptr;
    GsCluster *d_gcls = nullptr;
    double *d_gscratch = nullptr;
    size_t gs_scratch_bytes = 0;
    int S = 0, slot_n = 0;
    void *slots_p = nullptr;   // the slot buffer (and its size) S and slot_n were laid out in
    size_t slots_bytes = 0;

    int HIPFAIL(hipError_t e, const char *what) { return ctx->fail(ZK_EDEVICE, "%s: %s", what, hipGetErrorString(e)); }

    void *gsbuf = nullptr;
    size_t gsbytes = 0;

    // ensure_gs without recording a failure (the caller has a fallback)
    bool try_ensure_gs(size_t bytes)
    {
        if (bytes <= gsbytes) return true;
        if (gsbuf) {
            ctx->dev_free(gsbuf);
            ctx->extra -= gsbytes;
            gsbuf = nullptr;
            gsbytes = 0;
        }
        bytes = std::max(bytes, (size_t)1 << 20);
        if (!ctx->make_room(bytes)) return false;
        const std::string err = ctx->err;   // a refused allocation is not the call's error
        if (ctx->dev_alloc(&gsbuf, bytes) != ZK_OK) {
            gsbuf = nullptr;
            ctx->err = err;
            return false;
        }
        gsbytes = bytes;
        ctx->extra += bytes;
        ctx->note_held();
        return true;
    }

    int ensure_gs(size_t bytes)
    {
        if (bytes <= gsbytes) return ZK_OK;
        if (gsbuf) {
            ctx->dev_free(gsbuf);
            ctx->extra -= gsbytes;
            gsbuf = nullptr;
            gsbytes = 0;
        }
        bytes = std::max(bytes, (size_t)1 << 20);
        if (!ctx->make_room(bytes)) return ctx->fail(ZK_ENOMEM, "Gram-Schmidt plan exceeds the budget");
        if (ctx->dev_alloc(&gsbuf, bytes) != ZK_OK) return ZK_ENOMEM;
        gsbytes = bytes;
        ctx->extra += bytes;
        ctx->note_held();
        return ZK_OK;
    }

    void release(S2Prob *p)
    {
        if (p->vecbuf) {
            ctx->dev_free(p->vecbuf);
            ctx->extra -= p->vecbytes;
            p->vecbuf = nullptr;
        }
    }

    Stage2Batch batch_base()
    {
        Stage2Batch B;
        std::memset(&B, 0, sizeof B);
        B.L = L;
        B.dev_pairs = d_pairs;
        B.dev_probs = d_probs;
        B.dev_active = d_active;
        B.max_iter = O.max_iter;
        B.ldl = O.ldl;
        B.lu_base = (double *)ctx->s2lu.p;
        B.piv_base = (int *)((char *)ctx->s2lu.p + (size_t)S * s2_align(8 * s2_lu_slot_doubles(std::max(slot_n, 1), L)));
        B.timer = ctx->tp();
        return B;
    }

    // LU slots for orders up to n: as many as the budget allows (<= wanted).
    // The slot buffer belongs to the context and is shared with the other
    // engines of the context (the double-double and quad-double engines size
    // it for their own limbs, the all-pairs engine may give it back when the
    // budget is short), so the layout S x slot_n is trusted only while the
    // buffer is the very one this engine laid out.
    int ensure_slots(int n, int wanted)
    {
        if (ctx->s2lu.p != slots_p || ctx->s2lu.bytes != slots_bytes) {
            S = 0;
            slot_n = 0;
        }
        if (n <= slot_n && S >= std::min(wanted, 64) && ctx->s2lu.p) return ZK_OK;
        const int nn = std::max(n, slot_n);
        const size_t per = s2_align(8 * s2_lu_slot_doubles(nn, L)) + s2_align(8 * (size_t)nn);
        const size_t others = ctx->held() - ctx->s2lu.bytes;
        const size_t avail = ctx->budget > others ? ctx->budget - others : 0;
        int want = std::max(wanted, S);
        int s = (int)std::min<size_t>((size_t)want, avail / per);
        if (s < 1) return ctx->fail(ZK_ENOMEM, "one shifted LU of order %d needs %zu bytes", nn, per);
        int rc = ctx->ensure(ctx->s2lu, (size_t)s * per);
        // a fixed scratch region may be too fragmented for the count the
        // budget allows: fewer slots then
        while (rc != ZK_OK && ctx->arena && s > 1) {
            s /= 2;
            rc = ctx->ensure(ctx->s2lu, (size_t)s * per);
        }
        if (rc != ZK_OK) return rc;
        S = s;
        slot_n = nn;
        slots_p = ctx->s2lu.p;
        slots_bytes = ctx->s2lu.bytes;
        return ZK_OK;
    }

    // upload the tables of `set` (matrix i gets table index i)
    int upload(const std::vector<S2Prob *> &set)
    {
        base.assign(set.size(), 0);
        total_pairs = 0;
        for (size_t i = 0; i < set.size(); i++) {
            base[i] = total_pairs;
            total_pairs += set[i]->npairs;
        }
        const size_t np = set.size();
        gs_scratch_bytes = s2_align((size_t)total_pairs * 32 * 2 * L * 8);
        const size_t need = s2_align(sizeof(PairDesc) * total_pairs) + s2_align(sizeof(RqiProb) * np) +
                            3 * s2_align(4 * (size_t)total_pairs) + s2_align(sizeof(GsCluster) * total_pairs) + gs_scratch_bytes;
        int rc = ctx->ensure(ctx->meta, need);
        if (rc != ZK_OK) return rc;
        char *mb = (char *)ctx->meta.p;
        d_pairs = (PairDesc *)mb;
        mb += s2_align(sizeof(PairDesc) * total_pairs);
        d_probs = (RqiProb *)mb;
        mb += s2_align(sizeof(RqiProb) * np);
        d_active = (int *)mb;
        mb += s2_align(4 * (size_t)total_pairs);
        d_dst = (int *)mb;
        mb += s2_align(4 * (size_t)total_pairs);
        d_glist = (int *)mb;
        mb += s2_align(4 * (size_t)total_pairs);
        d_gcls = (GsCluster *)mb;
        mb += s2_align(sizeof(GsCluster) * total_pairs);
        d_gscratch = (double *)mb;
        hp.resize(total_pairs);
        hprobs.resize(np);
        for (size_t i = 0; i < np; i++) {
            hprobs[i] = set[i]->rp;
            for (int k = 0; k < set[i]->npairs; k++) {
                hp[base[i] + k] = set[i]->pairs[k];
                hp[base[i] + k].prob = (int)i;
            }
        }
        HIPCHK_(hipMemcpyAsync(d_pairs, hp.data(), sizeof(PairDesc) * total_pairs, hipMemcpyHostToDevice, st));
        HIPCHK_(hipMemcpyAsync(d_probs, hprobs.data(), sizeof(RqiProb) * np, hipMemcpyHostToDevice, st));
        HIPCHK_(hipStreamSynchronize(st));
        up = set;
        return ZK_OK;
    }

    int download(const std::vector<S2Prob *> &set)
    {
        HIPCHK_(hipMemcpyAsync(hp.data(), d_pairs, sizeof(PairDesc) * total_pairs, hipMemcpyDeviceToHost, st));
        HIPCHK_(hipStreamSynchronize(st));
        for (size_t i = 0; i < set.size(); i++)
            for (int k = 0; k < set[i]->npairs; k++) set[i]->pairs[k] = hp[base[i] + k];
        return ZK_OK;
    }

    int run_rq(const std::vector<int> &idx, int final_pass)
    {
        if (idx.empty()) return ZK_OK;
        HIPCHK_(hipMemcpyAsync(d_active, idx.data(), 4 * idx.size(), hipMemcpyHostToDevice, st));
        Stage2Batch B = batch_base();
        B.count = (int)idx.size();
        B.final_pass = final_pass;
        KernelTimer *tm = ctx->tp();
        const int id = tm ? tm->begin(KC_RQ, (double)idx.size(), st) : -1;
        if (stage2_rq<L>(B, st)) return ctx->fail(ZK_EDEVICE, "rq launch failed");
        if (tm) tm->end(id, st);
        HIPCHK_(hipStreamSynchronize(st));
        return ZK_OK;
    }

    // Gram-Schmidt over the uploaded set: clusters with active members
    // (global = every vector of the matrices in `only`, nobody frozen)
    int run_gs(const std::vector<S2Prob *> &set, bool global, const std::vector<int> *only = nullptr)
    {
        std::vector<GsCluster> cls;
        std::vector<int> list;
        GsPlan G;
        std::memset(&G, 0, sizeof G);
        long long sofs = 0;
        auto add = [&](int pi, const std::vector<int> &fro, const std::vector<int> &act) {
            GsCluster c;
            c.prob = pi;
            c.pair_base = base[pi];
            c.off = (int)list.size();
            c.nconv = (int)fro.size();
            c.nact = (int)act.size();
            c.size = c.nconv + c.nact;
            c.sofs = sofs;
            sofs += (long long)c.size * 32 * 2 * L * gs_slices(set[pi]->rp.n);
            list.insert(list.end(), fro.begin(), fro.end());
            list.insert(list.end(), act.begin(), act.end());
            cls.push_back(c);
            G.max_blocks = std::max(G.max_blocks, (c.nact + 31) / 32);
            G.max_nconv = std::max(G.max_nconv, c.nconv);
            G.max_n = std::max(G.max_n, set[pi]->rp.n);
        };
        // double-double windows re-orthogonalised whole (nobody frozen): two
        // Lowdin steps by dd GEMMs instead of block Gram-Schmidt
        std::vector<DdWindow> lw;
        std::vector<std::pair<int, std::vector<int>>> lw_act;   // the same windows for block Gram-Schmidt
        double lw_cols = 0.0;
        if (global) {
            // The eigenbasis in windows: consecutive pairs whose binary64
            // eigenvalues are closer than kReorthWindow * ||H|| share a window.
            // Pairs further apart are orthogonal to residual / gap <= tol /
            // kReorthWindow already; re-orthogonalising them against each
            // other would only add to their residuals (each projection adds
            // its coefficient times the eigenvalue difference).  Inside a
            // window: every pair in index order, or (after a polishing pass)
            // only the re-iterated pairs against the rest of their window.
            for (int pi : *only) {
                S2Prob *p = set[pi];
                const int n = p->npairs;
                if (n < 2 || (int)p->w0h.size() != n) continue;
                std::vector<char> r(n, 0);
                for (int k : p->redo) r[k] = 1;
                const double win = kReorthWindow * p->rp.hnorm;
                int g0 = 0;
                for (int e = 1; e <= n; e++) {
                    if (e < n && p->w0h[e] - p->w0h[e - 1] <= win) continue;
                    if (e - g0 >= 2) {
                        std::vector<int> act, fro;
                        for (int k = g0; k < e; k++) {
                            if (p->redo.empty() || r[k])
                                act.push_back(k);
                            else
                                fro.push_back(k);
                        }
                        if (L == 2 && fro.empty()) {
                            DdWindow x;
                            x.X = p->rp.vec + (size_t)g0 * p->rp.n;
                            x.px = (size_t)p->rp.n * p->rp.n;
                            x.n = p->rp.n;
                            x.m = e - g0;
                            lw.push_back(x);
                            lw_act.emplace_back(pi, act);
                            lw_cols += x.m;
                        } else if (!act.empty()) {
                            add(pi, fro, act);
                        }
                    }
                    g0 = e;
                }
            }
        } else {
            for (size_t pi = 0; pi < set.size(); pi++) {
                S2Prob *p = set[pi];
                for (size_t hi = 0; hi < p->heads.size(); hi++) {
                    const int h = p->heads[hi];
                    const int sz = p->pairs[h].cl_size;
                    std::vector<int> fro, act;
                    for (int q = 0; q < sz; q++) (p->pairs[h + q].status == 0 ? act : fro).push_back(p->pairs[h + q].k);
                    if (act.empty()) continue;
                    add((int)pi, fro, act);
                }
            }
        }
        if (!lw.empty() && !try_ensure_gs(dd_lowdin_bytes(lw))) {
            // the GEMMs' workspace does not fit: block Gram-Schmidt instead
            for (const auto &wa : lw_act) add(wa.first, std::vector<int>(), wa.second);
            lw.clear();
        }
        if (!lw.empty()) {
            KernelTimer *tm = ctx->tp();
            const int id = tm ? tm->begin(KC_REORTH, lw_cols, st) : -1;
            if (dd_lowdin(lw, 2, gsbuf, st)) return ctx->fail(ZK_EDEVICE, "re-orthogonalisation launch failed");
            if (tm) tm->end(id, st);
            HIPCHK_(hipStreamSynchronize(st));
        }
        if (cls.empty()) return ZK_OK;
        // plan storage sized from the plan itself: clusters, column lists,
        // coefficient scratch, Gram slices (row slices of 256) and flags
        G.ks = std::min(16, std::max(1, (G.max_n + 255) / 256));
        const size_t b_cls = s2_align(sizeof(GsCluster) * cls.size()), b_list = s2_align(4 * list.size());
        const size_t b_scr = s2_align((size_t)sofs * 8);
        const size_t b_gram = s2_align(cls.size() * (size_t)G.ks * 2 * L * 32 * 32 * 8);
        const size_t b_flag = s2_align(4 * cls.size());
        int rc = ensure_gs(b_cls + b_list + b_scr + b_gram + b_flag);
        if (rc != ZK_OK) return rc;
        GsCluster *g_cls = (GsCluster *)gsbuf;
        int *g_list = (int *)((char *)gsbuf + b_cls);
        double *g_scr = (double *)((char *)gsbuf + b_cls + b_list);
        HIPCHK_(hipMemcpyAsync(g_cls, cls.data(), sizeof(GsCluster) * cls.size(), hipMemcpyHostToDevice, st));
        HIPCHK_(hipMemcpyAsync(g_list, list.data(), 4 * list.size(), hipMemcpyHostToDevice, st));
        G.ncl = (int)cls.size();
        G.dev_cls = g_cls;
        G.dev_list = g_list;
        G.scratch = g_scr;
        G.gram = (double *)((char *)gsbuf + b_cls + b_list + b_scr);
        G.flag = (int *)((char *)gsbuf + b_cls + b_list + b_scr + b_gram);
        KernelTimer *tm = ctx->tp();
        const int id = tm ? tm->begin(global ? KC_REORTH : KC_GS, (double)list.size(), st) : -1;
        if (stage2_gs<L>(G, d_probs, global ? nullptr : d_pairs, st)) return ctx->fail(ZK_EDEVICE, "Gram-Schmidt launch failed");
        if (tm) tm->end(id, st);
        HIPCHK_(hipStreamSynchronize(st));
        return ZK_OK;
    }

    struct PrrBlock {
        int pi, k0, size;
    };

    // shifted solves of the given pairs (pair-table indices grouped by order):
    // every order in the same launches, largest orders first, in chunks of
    // as many pairs as there are LU slots; one host synchronisation at the end
    int solve_pairs(const std::map<int, std::vector<int>> &by_n, int nact, bool ldl)
    {
        int max_n = 0;
        for (auto &kv : by_n) max_n = std::max(max_n, kv.first);
        int rc = ensure_slots(max_n, nact);
        if (rc != ZK_OK) return rc;
        std::vector<int> lst, ord;
        for (auto it = by_n.rbegin(); it != by_n.rend(); ++it)
            for (int g : it->second) {
                lst.push_back(g);
                ord.push_back(it->first);
            }
        // Two groups of pairs on two streams (LDL^H, enough pairs): the pairs
        // at even and at odd positions of each chunk (both lists stay ordered
        // by non-increasing order).  Their trailing updates alternate, so one
        // group's panels (bound by latency and memory) run beside the other
        // group's update (bound by the FP64 VALU).  A pair's arithmetic is the
        // same in either group and in either slot.
        const bool split = ldl && s2_split_ && !ctx->arena;
        if (split) {
            for (size_t c0 = 0; c0 < lst.size(); c0 += (size_t)S) {
                const size_t cnt = std::min<size_t>((size_t)S, lst.size() - c0);
                if (cnt < 2 * (size_t)kSplitMin) continue;
                std::vector<int> l2, o2;
                for (int par = 0; par < 2; par++)
                    for (size_t q = par; q < cnt; q += 2) {
                        l2.push_back(lst[c0 + q]);
                        o2.push_back(ord[c0 + q]);
                    }
                std::copy(l2.begin(), l2.end(), lst.begin() + c0);
                std::copy(o2.begin(), o2.end(), ord.begin() + c0);
            }
            for (int k = 0; k < 1; k++)
                if (!ctx->side[k]) HIPCHK_(hipStreamCreateWithFlags(&ctx->side[k], hipStreamNonBlocking));
            for (int k = 0; k < 3; k++)
                if (!ctx->ev[k]) HIPCHK_(hipEventCreateWithFlags(&ctx->ev[k], hipEventDisableTiming));
        }
        HIPCHK_(hipMemcpyAsync(d_active, lst.data(), 4 * lst.size(), hipMemcpyHostToDevice, st));
        Stage2Batch B = batch_base();
        B.ldl = ldl ? 1 : 0;
        for (size_t c0 = 0; c0 < lst.size(); c0 += (size_t)S) {
            const int cnt = (int)std::min<size_t>((size_t)S, lst.size() - c0);
            const int n = ord[c0];
            B.dev_active = d_active + c0;
            B.n = n;
            B.count = cnt;
            B.ldm = s2_lu_ldm(n);
            B.lu_stride = s2_lu_slot_doubles(n, L);
            B.piv_stride = 2 * (size_t)n;
            if (split && cnt >= 2 * kSplitMin) {
                const int h = (cnt + 1) / 2;
                Stage2Batch G[2] = {B, B};
                G[0].count = h;
                G[1].dev_active = d_active + c0 + h;
                G[1].n = ord[c0 + h];
                G[1].count = cnt - h;
                G[1].lu_base = B.lu_base + (size_t)h * B.lu_stride;
                G[1].piv_base = B.piv_base + (size_t)h * B.piv_stride;
                const int *og[2] = {ord.data() + c0, ord.data() + c0 + h};
                const hipStream_t sg[2] = {st, ctx->side[0]};
                const hipEvent_t eg[2] = {ctx->ev[1], ctx->ev[2]};
                // the side stream starts after everything enqueued on the context stream
                HIPCHK_(hipEventRecord(ctx->ev[0], st));
                HIPCHK_(hipStreamWaitEvent(sg[1], ctx->ev[0], 0));
                if (stage2_solve_pair<L>(G, og, sg, eg)) return ctx->fail(ZK_EDEVICE, "solve launch failed");
                HIPCHK_(hipEventRecord(ctx->ev[0], sg[1]));
                HIPCHK_(hipStreamWaitEvent(st, ctx->ev[0], 0));
                continue;
            }
            if (stage2_solve<L>(B, ord.data() + c0, st)) return ctx->fail(ZK_EDEVICE, "solve launch failed");
        }
        HIPCHK_(hipStreamSynchronize(st));
        return ZK_OK;
    }

    // One inverse-iteration step with shift zero on the given blocks (every
    // member solves H w = v), then Gram-Schmidt inside their clusters in
    // index order (the other matrices' pairs frozen).  Components along
    // eigenvalues outside a chain shrink against the chain's tail by the
    // ratio of the eigenvalues, which removes the binary64 stage's pollution
    // of the tail subspace.
    int purify(const std::vector<S2Prob *> &set, const std::vector<PrrBlock> &blocks)
    {
        std::map<int, std::vector<int>> by_n;
        std::vector<std::vector<char>> mark(set.size());
        int cnt = 0;
        for (const auto &b : blocks) {
            S2Prob *p = set[b.pi];
            if (mark[b.pi].empty()) mark[b.pi].assign(p->npairs, 0);
            for (int q = 0; q < b.size; q++) {
                mark[b.pi][b.k0 + q] = 1;
                by_n[p->rp.n].push_back(base[b.pi] + b.k0 + q);
                cnt++;
            }
        }
        for (size_t pi = 0; pi < set.size(); pi++) {
            if (mark[pi].empty()) continue;
            S2Prob *p = set[pi];
            const int n = p->rp.n;
            std::vector<double> sig((size_t)L * n);
            HIPCHK_(hipMemcpyAsync(sig.data(), p->rp.sigma, 8 * sig.size(), hipMemcpyDeviceToHost, st));
            HIPCHK_(hipStreamSynchronize(st));
            for (int k = 0; k < p->npairs; k++)
                if (mark[pi][k])
                    for (int l = 0; l < L; l++) sig[(size_t)l * n + k] = 0.0;
            HIPCHK_(hipMemcpyAsync(p->rp.sigma, sig.data(), 8 * sig.size(), hipMemcpyHostToDevice, st));
            HIPCHK_(hipStreamSynchronize(st));
        }
        int rc = solve_pairs(by_n, cnt, false);
        if (rc != ZK_OK) return rc;
        for (size_t pi = 0; pi < set.size(); pi++)
            for (int k = 0; k < set[pi]->npairs; k++)
                set[pi]->pairs[k].status = (!mark[pi].empty() && mark[pi][k]) ? 0 : 1;
        rc = run_gs(set, false);
        for (S2Prob *p : set)
            for (auto &q : p->pairs) q.status = 0;
        return rc;
    }

    // Clusters from ascending binary64 eigenvalues: gaps <= cluster_tol ||H||
    // (mode 2: the whole spectrum is one cluster, for a start that is about
    // to be projected as a whole); Rayleigh-Ritz blocks for 2..32 members.
    void plan_clusters(S2Prob *p, const std::vector<double> &w, int mode)
    {
        const int kp = p->npairs;
        const double thr = p->opts.cluster_tol * p->rp.hnorm;
        p->pairs.assign(kp, PairDesc());
        int start = 0;
        for (int k = 0; k < kp; k++) {
            if (mode != 2 && k > 0 && !(w[k] - w[k - 1] <= thr)) start = k;
            PairDesc &q = p->pairs[k];
            std::memset(&q, 0, sizeof q);
            q.k = k;
            q.cl_start = start;
        }
        p->heads.clear();
        int k = 0;
        while (k < kp) {
            int e = k + 1;
            while (e < kp && p->pairs[e].cl_start == k) e++;
            for (int q = k; q < e; q++) p->pairs[q].cl_size = (q == k) ? e - k : 0;
            p->heads.push_back(k);
            k = e;
        }
        p->rrb.clear();
        if (mode != 2)
            for (int h : p->heads)
                if (p->pairs[h].cl_size >= 2 && p->pairs[h].cl_size <= 32) p->rrb.push_back(std::make_pair(h, p->pairs[h].cl_size));
    }

    // A projected level resolves its Ritz values to about u times its own
    // scale, but its Ritz vectors keep the pollution of the level above (the
    // enclosing block's resolution over the gap at the block's boundary), and
    // the Rayleigh quotient of such a vector is off by that pollution squared
    // times the outside eigenvalues -- far more than the tail eigenvalues
    // themselves.  So an unconverged pair resolved by a projected level and
    // not in a Rayleigh-Ritz block starts from its Ritz value: the first
    // shifted solve then removes the pollution.
    int first_shifts(const std::vector<S2Prob *> &set)
    {
        for (S2Prob *p : set) {
            if ((int)p->ritz0.size() != p->npairs) continue;
            std::vector<char> inblk(p->npairs, 0);
            for (const auto &bk : p->rrb)
                for (int q = 0; q < bk.second; q++) inblk[bk.first + q] = 1;
            const int n = p->rp.n;
            std::vector<double> sig((size_t)L * n);
            bool any = false;
            for (int k = 0; k < p->npairs; k++) any = any || (!inblk[k] && p->ritz0[k] == p->ritz0[k]);
            if (!any) continue;
            HIPCHK_(hipMemcpyAsync(sig.data(), p->rp.sigma, 8 * sig.size(), hipMemcpyDeviceToHost, st));
            HIPCHK_(hipStreamSynchronize(st));
            for (int k = 0; k < p->npairs; k++) {
                if (inblk[k] || !(p->ritz0[k] == p->ritz0[k])) continue;
                sig[k] = p->ritz0[k];
                for (int l = 1; l < L; l++) sig[(size_t)l * n + k] = 0.0;
            }
            HIPCHK_(hipMemcpyAsync(p->rp.sigma, sig.data(), 8 * sig.size(), hipMemcpyHostToDevice, st));
            HIPCHK_(hipStreamSynchronize(st));
        }
        return ZK_OK;
    }

    // Projected Rayleigh-Ritz on the clusters longer than 32 members: C =
    // V^H H V in L limbs, the binary64 stage on C (rounded), V <- V Q.  The
    // Ritz values split the cluster into sub-chains relative to its own scale
    // (gaps <= cluster_tol * max |Ritz value|); sub-chains of 2..32 become
    // Rayleigh-Ritz blocks, longer ones are projected again at the next level.
    int run_prr(const std::vector<S2Prob *> &set, bool &projected)
    {
        for (S2Prob *p : set) p->ritz0.assign(p->npairs, std::nan(""));
        std::vector<PrrBlock> todo;
        for (size_t pi = 0; pi < set.size(); pi++)
            for (int h : set[pi]->heads)
                if (set[pi]->pairs[h].cl_size > 32) todo.push_back({(int)pi, h, set[pi]->pairs[h].cl_size});
        if (todo.empty()) return ZK_OK;
        projected = true;
        std::vector<std::vector<double>> ritz;
        int rc = prr_project(set, todo, ritz);
        if (rc != ZK_OK) return rc;
        // Ritz values below the binary64 stage's pollution floor: purify the
        // chain (one shift-zero inverse-iteration step) and project again
        std::vector<PrrBlock> pur;
        std::vector<int> pidx;
        for (size_t b = 0; b < todo.size(); b++) {
            double mn = INFINITY;
            for (double x : ritz[b]) mn = std::min(mn, std::fabs(x));
            if (mn < kPurify * set[todo[b].pi]->rp.hnorm) {
                pur.push_back(todo[b]);
                pidx.push_back((int)b);
            }
        }
        if (!pur.empty()) {
            if ((rc = purify(set, pur)) != ZK_OK) return rc;
            std::vector<std::vector<double>> rp;
            if ((rc = prr_project(set, pur, rp)) != ZK_OK) return rc;
            for (size_t i = 0; i < pur.size(); i++) ritz[pidx[i]] = rp[i];
        }
        for (int level = 0; level < kPrrLevels; level++) {
            std::vector<PrrBlock> next;
            prr_split(set, todo, ritz, next);
            if (next.empty()) break;
            todo = next;
            if ((rc = prr_project(set, todo, ritz)) != ZK_OK) return rc;
        }
        return ZK_OK;
    }

    // Ritz values of a projected level -> first shifts, Rayleigh-Ritz blocks
    // and the blocks of the next level.  The next level takes the members
    // whose Ritz values lie below kPrrDeep times the level's scale (if there
    // are more than 32 of them): the level resolves its Ritz vectors to about
    // u times its scale, so the pollution of that sub-block by the members
    // above stays below u / kPrrDeep, and the next level's Ritz values are
    // accurate far below the scale of the members above.  Members above it
    // form chains by gaps <= cluster_tol * scale: 2..32 members become
    // Rayleigh-Ritz blocks, longer chains are projected at the next level.
    void prr_split(const std::vector<S2Prob *> &set, const std::vector<PrrBlock> &todo,
                   const std::vector<std::vector<double>> &ritz, std::vector<PrrBlock> &next)
    {
        for (size_t b = 0; b < todo.size(); b++) {
            const std::vector<double> &w = ritz[b];
            const int m = todo[b].size, k0 = todo[b].k0;
            S2Prob *p = set[todo[b].pi];
            if (std::getenv("ZK_TRACE"))
                std::fprintf(stderr, "[zk] projected level: block %d+%d, Ritz values %.3e .. %.3e\n", k0, m, w[0], w[m - 1]);
            // the deepest level's Ritz values are the first shifts of its pairs
            if ((int)p->ritz0.size() >= k0 + m) std::copy(w.begin(), w.end(), p->ritz0.begin() + k0);
            double sc = 0.0;
            for (double x : w) sc = std::max(sc, std::fabs(x));
            const double thr = p->opts.cluster_tol * sc, deep = kPrrDeep * sc;
            int j0 = 0;
            while (j0 < m && !(std::fabs(w[j0]) < deep)) j0++;
            int j1 = j0;
            while (j1 < m && std::fabs(w[j1]) < deep) j1++;
            const bool sub = (j1 - j0 > 32) && (j1 - j0 < m);
            if (sub) next.push_back({todo[b].pi, k0 + j0, j1 - j0});
            int s0 = 0;
            for (int e = 1; e <= m; e++) {
                const bool brk = (e == m) || !(w[e] - w[e - 1] <= thr) || (sub && (e == j0 || e == j1));
                if (!brk) continue;
                const int len = e - s0;
                if (!(sub && s0 >= j0 && s0 < j1)) {
                    if (len >= 2 && len <= 32) p->rrb.push_back(std::make_pair(k0 + s0, len));
                    if (len > 32 && len < m) next.push_back({todo[b].pi, k0 + s0, len});
                }
                s0 = e;
            }
        }
    }

    // One projected Rayleigh-Ritz step on the given blocks: C = V^H H V in L
    // limbs, the binary64 stage on C (rounded), V <- V Q; the Ritz values
    // (ascending) are returned per block.
    int prr_project(const std::vector<S2Prob *> &set, const std::vector<PrrBlock> &todo,
                    std::vector<std::vector<double>> &ritz)
    {
        const int nd = (int)todo.size();
        ritz.assign(nd, std::vector<double>());
        if (nd == 0) return ZK_OK;
        int max_size = 0, max_n = 0;
        size_t bytes = s2_align(sizeof(PrrDesc) * nd);
        std::vector<size_t> off(nd);
        for (int b = 0; b < nd; b++) {
            const size_t m = (size_t)todo[b].size, n = (size_t)set[todo[b].pi]->rp.n;
            max_size = std::max(max_size, todo[b].size);
            max_n = std::max(max_n, (int)n);
            off[b] = bytes;
            // Y, C, hf, V0, w0, flag
            bytes += s2_align(8 * 2 * (size_t)L * n * m) + 3 * s2_align(16 * m * m) + s2_align(8 * m) + s2_align(4);
        }
        if (!ctx->make_room(bytes)) return ctx->fail(ZK_ENOMEM, "projected Rayleigh-Ritz exceeds the budget");
        void *buf = nullptr;
        if (ctx->dev_alloc(&buf, bytes) != ZK_OK) return ZK_ENOMEM;
        ctx->extra += bytes;
        ctx->note_held();
        std::vector<PrrDesc> hd(nd);
        std::vector<zk_herm> hm(nd);
        std::vector<double *> hf(nd), w0(nd), V0(nd);
        std::vector<int *> flag(nd);
        for (int b = 0; b < nd; b++) {
            const size_t m = (size_t)todo[b].size, n = (size_t)set[todo[b].pi]->rp.n;
            char *c = (char *)buf + off[b];
            PrrDesc &D = hd[b];
            std::memset(&D, 0, sizeof D);
            D.prob = todo[b].pi;
            D.k0 = todo[b].k0;
            D.size = (int)m;
            D.Y = (double *)c;
            c += s2_align(8 * 2 * (size_t)L * n * m);
            D.C = (double *)c;
            c += s2_align(16 * m * m);
            hf[b] = (double *)c;
            c += s2_align(16 * m * m);
            V0[b] = (double *)c;
            D.Q = V0[b];
            c += s2_align(16 * m * m);
            w0[b] = (double *)c;
            c += s2_align(8 * m);
            flag[b] = (int *)c;
            std::memset(&hm[b], 0, sizeof(zk_herm));
            hm[b].n = (int)m;
            hm[b].lda = (int)m;
            hm[b].limbs = 1;
            hm[b].plane[0] = D.C;
        }
        PrrDesc *d_desc = (PrrDesc *)buf;
        int rc = ZK_OK;
        auto cleanup = [&]() {
            hipStreamSynchronize(st);
            ctx->dev_free(buf);
            ctx->extra -= bytes;
        };
        if (hipMemcpyAsync(d_desc, hd.data(), sizeof(PrrDesc) * nd, hipMemcpyHostToDevice, st) != hipSuccess ||
            stage2_prr_project<L>(d_desc, nd, max_size, max_n, d_probs, st)) {
            cleanup();
            return ctx->fail(ZK_EDEVICE, "projected Rayleigh-Ritz launch failed");
        }
        if ((rc = run_stage1(ctx, nd, hm.data(), hf, w0, V0, flag, std::vector<int>())) != ZK_OK) {
            cleanup();
            return rc;
        }
        if (stage2_prr_rotate<L>(d_desc, nd, max_size, max_n, d_probs, st)) {
            cleanup();
            return ctx->fail(ZK_EDEVICE, "projected Rayleigh-Ritz launch failed");
        }
        for (int b = 0; b < nd; b++) {
            ritz[b].resize(todo[b].size);
            if (hipMemcpyAsync(ritz[b].data(), w0[b], 8 * (size_t)todo[b].size, hipMemcpyDeviceToHost, st) != hipSuccess) {
                cleanup();
                return ctx->fail(ZK_EDEVICE, "projected Rayleigh-Ritz read-back failed");
            }
        }
        cleanup();
        return ZK_OK;
    }

    // Rayleigh-Ritz on the blocks of 2..32 members (the clusters of that size
    // and the sub-chains that the projected step found inside longer ones).
    // first = true: every member; otherwise the active members of a block,
    // when at least two are active.  Scratch comes from the engine's own
    // buffer, sized from the plan, so the step never depends on what other
    // buffers hold.
    int run_rr(const std::vector<S2Prob *> &set, bool first)
    {
        std::vector<GsCluster> cls;
        std::vector<int> list;
        long long sofs = 0;
        for (size_t pi = 0; pi < set.size(); pi++) {
            S2Prob *p = set[pi];
            for (const auto &bk : p->rrb) {
                std::vector<int> mem;
                for (int q = 0; q < bk.second; q++)
                    if (first || p->pairs[bk.first + q].status == 0) mem.push_back(p->pairs[bk.first + q].k);
                if (mem.size() < 2) continue;
                GsCluster c;
                c.prob = (int)pi;
                c.pair_base = base[pi];
                c.off = (int)list.size();
                c.nconv = 0;
                c.nact = (int)mem.size();
                c.size = (int)mem.size();
                c.sofs = sofs;
                sofs += (long long)2 * L * p->rp.n * 32;
                list.insert(list.end(), mem.begin(), mem.end());
                cls.push_back(c);
            }
        }
        if (cls.empty()) return ZK_OK;
        const size_t b_cls = s2_align(sizeof(GsCluster) * cls.size()), b_list = s2_align(4 * list.size());
        int rc = ensure_gs(b_cls + b_list + s2_align((size_t)sofs * 8));
        if (rc != ZK_OK) return rc;
        GsCluster *g_cls = (GsCluster *)gsbuf;
        int *g_list = (int *)((char *)gsbuf + b_cls);
        HIPCHK_(hipMemcpyAsync(g_cls, cls.data(), sizeof(GsCluster) * cls.size(), hipMemcpyHostToDevice, st));
        HIPCHK_(hipMemcpyAsync(g_list, list.data(), 4 * list.size(), hipMemcpyHostToDevice, st));
        GsPlan G;
        std::memset(&G, 0, sizeof G);
        G.ncl = (int)cls.size();
        G.dev_cls = g_cls;
        G.dev_list = g_list;
        G.scratch = (double *)((char *)gsbuf + b_cls + b_list);
        KernelTimer *tm = ctx->tp();
        const int id = tm ? tm->begin(KC_GS, (double)list.size(), st) : -1;
        if (stage2_rr<L>(G, d_probs, L == 2 ? 10 : 14, st)) return ctx->fail(ZK_EDEVICE, "Rayleigh-Ritz launch failed");
        if (tm) tm->end(id, st);
        HIPCHK_(hipStreamSynchronize(st));
        return ZK_OK;
    }

    // finalise the live matrices that have no active pair
    int settle()
    {
        std::vector<int> fin;
        for (size_t pi = 0; pi < live.size(); pi++) {
            bool act = false;
            for (auto &q : live[pi]->pairs) act = act || q.status == 0;
            if (!act) fin.push_back((int)pi);
        }
        if (fin.empty()) return ZK_OK;
        int rc;
        if ((rc = upload(live)) != ZK_OK) return rc;
        std::vector<int> ro;
        for (int pi : fin)
            if (live[pi]->opts.reorth) ro.push_back(pi);
        if (!ro.empty())
            if ((rc = run_gs(live, true, &ro)) != ZK_OK) return rc;
        {
            // every finished pair is judged once more against the tolerance
            std::vector<int> idx;
            for (int pi : fin)
                for (int k = 0; k < live[pi]->npairs; k++) idx.push_back(base[pi] + k);
            if ((rc = run_rq(idx, 1)) != ZK_OK) return rc;
            if ((rc = download(live)) != ZK_OK) return rc;
        }
        {
            // polishing: a pair that the re-orthogonalisation pushed above the
            // tolerance, with iterations left, goes back for more iterations;
            // the next settle re-orthogonalises only those pairs against the rest
            std::vector<int> keep_fin;
            for (int pi : fin) {
                S2Prob *p = live[pi];
                p->redo.clear();
                if (p->opts.reorth && p->polish < kPolishPasses)
                    for (int k = 0; k < p->npairs; k++) {
                        const PairDesc &q = p->pairs[k];
                        if (q.status == 2 && !(q.flags & 8) && q.iters < p->rp.max_iter) p->redo.push_back(k);
                    }
                if (p->redo.empty()) {
                    keep_fin.push_back(pi);
                    continue;
                }
                p->polish++;
                for (int k : p->redo) p->pairs[k].status = 0;
            }
            fin = keep_fin;
            if (fin.empty()) return ZK_OK;
        }
        // ascending order of the refined eigenvalues inside each matrix
        std::vector<int> dst(total_pairs, 0);
        std::vector<int> outidx;
        std::vector<double> sig;
        for (int pi : fin) {
            S2Prob *p = live[pi];
            const int n = p->rp.n, kp = p->npairs;
            sig.resize((size_t)L * n);
            HIPCHK_(hipMemcpyAsync(sig.data(), p->rp.sigma, 8 * (size_t)L * n, hipMemcpyDeviceToHost, st));
            HIPCHK_(hipStreamSynchronize(st));
            std::vector<int> ord(kp);
            for (int k = 0; k < kp; k++) ord[k] = k;
            std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
                for (int l = 0; l < L; l++) {
                    const double x = sig[(size_t)l * n + a], y = sig[(size_t)l * n + b];
                    if (x != y) return x < y;
                }
                return false;
            });
            for (int pos = 0; pos < kp; pos++) dst[base[pi] + ord[pos]] = pos;
            for (int k = 0; k < kp; k++) outidx.push_back(base[pi] + k);
        }
        // output kernel over the finished pairs only: pass their indices as the pair list
        std::vector<PairDesc> sub(outidx.size());
        std::vector<int> subdst(outidx.size());
        for (size_t i = 0; i < outidx.size(); i++) {
            sub[i] = hp[outidx[i]];
            subdst[i] = dst[outidx[i]];
        }
        HIPCHK_(hipMemcpyAsync(d_pairs, sub.data(), sizeof(PairDesc) * sub.size(), hipMemcpyHostToDevice, st));
        HIPCHK_(hipMemcpyAsync(d_dst, subdst.data(), 4 * subdst.size(), hipMemcpyHostToDevice, st));
        if (stage2_output<L>(d_pairs, d_probs, d_dst, (int)sub.size(), st)) return ctx->fail(ZK_EDEVICE, "output launch failed");
        HIPCHK_(hipStreamSynchronize(st));
        std::vector<S2Prob *> keep;
        std::vector<char> isfin(live.size(), 0);
        for (int pi : fin) isfin[pi] = 1;
        for (size_t pi = 0; pi < live.size(); pi++) {
            S2Prob *p = live[pi];
            if (!isfin[pi]) {
                keep.push_back(p);
                continue;
            }
            bool all_conv = true;
            for (int k = 0; k < p->npairs; k++) {
                const PairDesc &q = p->pairs[k];
                if (q.status != 1) all_conv = false;
                if (stats) {
                    stats->iters_hist[std::min(q.iters, 15)]++;
                    stats->solves += q.iters;
                }
                if (p->info) {
                    zk_pair_info &o = p->info[dst[base[pi] + k]];
                    o.iters = q.iters;
                    o.flags = q.flags;
                    o.cluster = q.cl_start;
                    o.reserved = 0;
                    o.resid = q.resid;
                }
            }
            p->status = all_conv ? ZK_OK : ZK_ENOCONV;
            p->done = true;
            release(p);
            finished.push_back(p);
        }
        live = keep;
        return ZK_OK;
    }

    void dump(const std::vector<S2Prob *> &set, const char *what)
    {
        for (S2Prob *p : set) {
            std::vector<double> sig((size_t)L * p->rp.n);
            hipMemcpy(sig.data(), p->rp.sigma, 8 * sig.size(), hipMemcpyDeviceToHost);
            for (int k = 0; k < std::min(p->npairs, 8); k++)
                std::fprintf(stderr, "[zk2] %s n=%d k=%d st=%d it=%d res=%.17e sig=%.17e %.17e\n", what, p->rp.n, k, p->pairs[k].status,
                             p->pairs[k].iters, p->pairs[k].resid, sig[k], sig[(size_t)p->rp.n + k]);
        }
    }

    void trace()
    {
        std::vector<double> rs;
        int nact = 0;
        for (S2Prob *p : live)
            for (auto &q : p->pairs) {
                if (q.iters == rounds) rs.push_back(q.resid);
                nact += q.status == 0;
            }
        std::sort(rs.begin(), rs.end());
        auto qt = [&](double f) { return rs.empty() ? 0.0 : rs[std::min(rs.size() - 1, (size_t)(f * rs.size()))]; };
        std::fprintf(stderr, "[zk] round %d: still active %d, judged %zu, resid q10 %.2e q50 %.2e q90 %.2e max %.2e\n", rounds, nact,
                     rs.size(), qt(0.1), qt(0.5), qt(0.9), rs.empty() ? 0.0 : rs.back());
    }

    std::vector<PairDesc> hp;
    std::vector<RqiProb> hprobs;
    std::vector<S2Prob *> up;
};

}  // namespace zk

#undef HIPCHK_
