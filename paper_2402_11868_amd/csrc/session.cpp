// Serving form of libzk: a scheduler thread that turns a stream of
// eigendecomposition requests (the bond matrices an MPS sweep emits) into
// continuously batched GPU work.
//
//   submit   validates, stamps the arrival time, queues (bounded queue)
//   admit    at every round boundary the scheduler admits queued requests in
//            arrival order while the sum of admitted footprints fits the
//            session budget (a request larger than the whole budget is
//            refused at submit)
//   stage 1  newly admitted requests of equal order share the binary64
//            launches
//   stage 2  every admitted request's pairs join the same Rayleigh-quotient
//            rounds: one round's shifted LU launches mix pairs of different
//            requests; a request leaves as soon as all its pairs stopped
//   poll     waits for completion; completion time is stamped after the
//            request's outputs are in place
//
// Every kernel works per pair, per cluster or per matrix, so a request's
// result is bitwise the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/zk.h"
#include "api_internal.h"
#include "engine.h"
#include "stage.h"

using namespace zk;

int run_stage1(zk_ctx *ctx, int count, const zk_herm *A, const std::vector<double *> &hf, const std::vector<double *> &w0,
               const std::vector<double *> &V0, const std::vector<int *> &flag, const std::vector<int> &fp32);
ResolvedOpts zk_resolve_opts(const zk_opts *o, int L);
int zk_check_request(const zk_herm &A, const zk_eig_out &o, int L, bool want_vectors);

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

enum { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2, RQ_CANCELLED = 3 };

struct Request {
    zk_ticket id = 0;
    zk_herm A;
    zk_eig_out out;
    int L = 2;
    ResolvedOpts O;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int state = RQ_QUEUED;
    int status = ZK_OK;
    size_t foot = 0;
    void *inbuf = nullptr;   // hf, w0, V0, flag
    S2Prob prob;
};

// Bytes of the stage-2 inputs of one request (limb-planar copy, binary64 pairs, flag).
size_t in_bytes(int n, int limbs_in)
{
    const size_t nn = (size_t)n * n;
    return al(8 * 2 * (size_t)limbs_in * nn) + al(8 * (size_t)n) + al(16 * nn) + al(64);
}

// Admission footprint: the inputs, then either the all-pairs state or the
// iterates plus one shifted-LU slot with its pivots (the least a request
// needs to make progress; the engine adds slots as the context budget allows).
size_t footprint(int n, int limbs_in, int L, int refine)
{
    const size_t nn = (size_t)n * n;
    const size_t in = in_bytes(n, limbs_in);
    if (refine == 1) return in + zk::ap_bytes(n);
    const size_t slot = al(8 * zk::s2_lu_slot_doubles(n, L)) + al(4 * (size_t)n);
    return in + al(8 * 2 * (size_t)L * nn) + al(8 * (size_t)L * n) + slot;
}

// Device memory for request inputs, recycled across requests: blocks are
// kept in free lists by size class (powers of two from 64 KiB) and given back
// to HIP only when the session ends, so the scheduler does not call hipMalloc
// once the stream's sizes have been seen.
class InPool {
  public:
    ~InPool() { clear(); }
    void *get(size_t bytes)
    {
        const size_t c = cls(bytes);
        auto it = free_.find(c);
        if (it != free_.end() && !it->second.empty()) {
            void *p = it->second.back();
            it->second.pop_back();
            return p;
        }
        void *p = nullptr;
        if (hipMalloc(&p, c) != hipSuccess) {
            hipGetLastError();
            return nullptr;
        }
        size_[p] = c;
        total_ += c;
        return p;
    }
    void put(void *p)
    {
        if (p) free_[size_.at(p)].push_back(p);
    }
    void clear()
    {
        for (auto &kv : size_) hipFree(kv.first);
        size_.clear();
        free_.clear();
        total_ = 0;
    }
    size_t total() const { return total_; }

  private:
    static size_t cls(size_t b)
    {
        size_t c = (size_t)64 << 10;
        while (c < b) c <<= 1;
        return c;
    }
    std::map<size_t, std::vector<void *>> free_;
    std::map<void *, size_t> size_;
    size_t total_ = 0;
};

}  // namespace

struct zk_session {
    zk_ctx *ctx = nullptr;
    size_t budget = 0;
    int max_queue = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::map<zk_ticket, Request *> all;
    std::thread th;
    bool stop = false;
    zk_ticket next = 1;
    size_t inflight = 0;
    int fatal = ZK_OK;
    Stage2Engine<2> *e2 = nullptr;
    Stage2Engine<4> *e4 = nullptr;
    zk::ApEngine *ap = nullptr;   // requests with the all-pairs refinement
    std::vector<Request *> running;
    InPool pool;          // request input buffers (scheduler thread only)
    int waiters = 0;      // threads inside zk_session_poll (guarded by mu)
    bool closing = false; // zk_session_destroy has begun
    std::condition_variable cv_left;

    void loop();
    int admit_and_start(std::vector<Request *> &fresh);
    template <int L> void finish(Stage2Engine<L> *e);
    void finish_ap();
};

int zk_session::admit_and_start(std::vector<Request *> &fresh)
{
    // binary64 stage for the fresh requests (grouped by order inside run_stage1)
    const int cnt = (int)fresh.size();
    std::vector<zk_herm> A(cnt);
    std::vector<double *> hf(cnt), w0(cnt), V0(cnt);
    std::vector<int *> flag(cnt);
    std::vector<int> fp32(cnt);
    for (int i = 0; i < cnt; i++) {
        Request *r = fresh[i];
        A[i] = r->A;
        fp32[i] = r->O.init_fp32;
        const int n = r->A.n;
        const size_t nn = (size_t)n * n;
        r->inbuf = pool.get(in_bytes(n, r->A.limbs));
        if (!r->inbuf) return ZK_ENOMEM;
        char *b = (char *)r->inbuf;
        hf[i] = (double *)b;
        b += al(8 * 2 * (size_t)r->A.limbs * nn);
        w0[i] = (double *)b;
        b += al(8 * (size_t)n);
        V0[i] = (double *)b;
        b += al(16 * nn);
        flag[i] = (int *)b;
    }
    int rc = run_stage1(ctx, cnt, A.data(), hf, w0, V0, flag, fp32);
    if (rc != ZK_OK) return rc;
    std::vector<S2Prob *> b2, b4;
    std::vector<zk::ApReq> ba;
    for (int i = 0; i < cnt; i++) {
        Request *r = fresh[i];
        if (r->O.refine == 1) {
            zk::ApReq q;
            q.A = r->A;
            q.out = r->out;
            q.hf = hf[i];
            q.w0 = w0[i];
            q.V0 = V0[i];
            q.tol = r->O.tol;
            q.max_iter = r->O.max_iter_set > 0 ? r->O.max_iter_set : 12;
            q.want_vectors = r->O.want_vectors;
            q.cookie = r;
            ba.push_back(q);
            continue;
        }
        S2Prob &p = r->prob;
        std::memset(&p.rp, 0, sizeof p.rp);
        p.rp.n = r->A.n;
        p.rp.limbs_in = r->A.limbs;
        p.rp.hf = hf[i];
        p.rp.w0 = w0[i];
        p.rp.V0 = V0[i];
        p.rp.ldv0 = r->A.n;
        p.rp.ldv_out = r->out.ldv;
        for (int l = 0; l < r->L; l++) {
            p.rp.w_out[l] = r->out.w[l];
            p.rp.v_out[l] = r->O.want_vectors ? (double *)r->out.v[l] : nullptr;
        }
        p.opts = r->O;
        p.npairs = r->A.n;
        p.info = r->out.info;
        p.cookie = r;
        (r->L == 2 ? b2 : b4).push_back(&p);
    }
    if (!b2.empty() && (rc = e2->add(b2)) != ZK_OK) return rc;
    if (!b4.empty() && (rc = e4->add(b4)) != ZK_OK) return rc;
    if (!ba.empty() && (rc = ap->add(ba)) != ZK_OK) return rc;
    return ZK_OK;
}

void zk_session::finish_ap()
{
    if (ap->finished.empty()) return;
    const double t = now_s();
    std::lock_guard<std::mutex> g(mu);
    for (const zk::ApDone &d : ap->finished) {
        Request *r = (Request *)d.cookie;
        pool.put(r->inbuf);
        r->inbuf = nullptr;
        r->status = d.status;
        r->state = RQ_DONE;
        r->t_done = t;
        inflight -= r->foot;
    }
    ap->finished.clear();
    cv_done.notify_all();
}

template <int L>
void zk_session::finish(Stage2Engine<L> *e)
{
    if (e->finished.empty()) return;
    const double t = now_s();
    std::lock_guard<std::mutex> g(mu);
    for (S2Prob *p : e->finished) {
        Request *r = (Request *)p->cookie;
        pool.put(r->inbuf);
        r->inbuf = nullptr;
        r->status = p->status;
        r->state = RQ_DONE;
        r->t_done = t;
        inflight -= r->foot;
    }
    e->finished.clear();
    cv_done.notify_all();
}

void zk_session::loop()
{
    hipSetDevice(ctx->device);
    for (;;) {
        std::vector<Request *> fresh;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (!stop && queue.empty() && !e2->any_live() && !e4->any_live() && !ap->any_live())
                cv_work.wait(lk, [&] { return stop || !queue.empty(); });
            if (stop) break;
            // admission by footprint, in arrival order
            while (!queue.empty() && (inflight == 0 || inflight + queue.front()->foot <= budget)) {
                Request *r = queue.front();
                queue.pop_front();
                r->state = RQ_RUNNING;
                r->t_admit = now_s();
                inflight += r->foot;
                fresh.push_back(r);
            }
        }
        int rc = ZK_OK;
        if (!fresh.empty()) rc = admit_and_start(fresh);
        if (rc == ZK_OK && e2->any_live()) rc = e2->round();
        if (rc == ZK_OK && e4->any_live()) rc = e4->round();
        if (rc == ZK_OK && ap->any_live()) rc = ap->round();
        finish<2>(e2);
        finish<4>(e4);
        finish_ap();
        if (rc != ZK_OK) {
            // a device or resource failure ends every admitted request
            std::lock_guard<std::mutex> g(mu);
            fatal = rc;
            for (auto &kv : all) {
                Request *r = kv.second;
                if (r->state == RQ_RUNNING) {
                    r->state = RQ_DONE;
                    r->status = rc;
                    r->t_done = now_s();
                    pool.put(r->inbuf);
                    r->inbuf = nullptr;
                }
            }
            inflight = 0;
            cv_done.notify_all();
            delete e2;
            delete e4;
            delete ap;
            e2 = new Stage2Engine<2>(ctx, zk_resolve_opts(nullptr, 2), nullptr);
            e4 = new Stage2Engine<4>(ctx, zk_resolve_opts(nullptr, 4), nullptr);
            ap = new zk::ApEngine(ctx);
        }
    }
}

extern "C" int zk_session_create(zk_ctx *ctx, size_t budget, int max_queue, zk_session **out)
{
    if (!ctx || !out) return ZK_EINVAL;
    *out = nullptr;
    if (ctx->poisoned) return ZK_EDEVICE;
    zk_session *s = new zk_session();
    s->ctx = ctx;
    s->budget = budget ? budget : ((size_t)16 << 30);
    s->max_queue = max_queue > 0 ? max_queue : 1 << 20;
    s->e2 = new Stage2Engine<2>(ctx, zk_resolve_opts(nullptr, 2), nullptr);
    s->e4 = new Stage2Engine<4>(ctx, zk_resolve_opts(nullptr, 4), nullptr);
    s->ap = new zk::ApEngine(ctx);
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return ZK_OK;
}

extern "C" int zk_session_submit(zk_session *s, const zk_herm *A, zk_eig_out *out, int limbs_out, const zk_opts *opts,
                                 zk_ticket *ticket)
{
    if (!s || !A || !out || !ticket || (limbs_out != 2 && limbs_out != 4)) return ZK_EINVAL;
    const ResolvedOpts O = zk_resolve_opts(opts, limbs_out);
    if (zk_check_request(*A, *out, limbs_out, O.want_vectors) != ZK_OK) return ZK_EINVAL;
    if (O.refine != 0 && (O.refine != 1 || limbs_out != 2)) return ZK_EINVAL;
    const size_t foot = footprint(A->n, A->limbs, limbs_out, O.refine);
    if (foot > s->budget) return ZK_ENOMEM;
    Request *r = new Request();
    r->A = *A;
    r->out = *out;
    r->L = limbs_out;
    r->O = O;
    r->foot = foot;
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> g(s->mu);
        if ((int)s->queue.size() >= s->max_queue) {
            delete r;
            return ZK_EAGAIN;
        }
        r->id = s->next++;
        s->all[r->id] = r;
        s->queue.push_back(r);
    }
    s->cv_work.notify_one();
    *ticket = r->id;
    return ZK_OK;
}

extern "C" int zk_session_poll(zk_session *s, zk_ticket ticket, int timeout_us, int *req_status)
{
    if (!s) return ZK_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->closing) return ZK_ECANCELED;
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return ZK_EINVAL;
    Request *r = it->second;
    auto ready = [&] { return r->state == RQ_DONE || r->state == RQ_CANCELLED; };
    if (!ready()) {
        // zk_session_destroy waits for every waiter to leave before it frees
        // the request and the session, so r and the condition variables
        // stay valid for the whole wait
        s->waiters++;
        if (timeout_us < 0) s->cv_done.wait(lk, ready);
        else if (timeout_us > 0) s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
        if (--s->waiters == 0 && s->closing) s->cv_left.notify_all();
    }
    if (r->state == RQ_CANCELLED) return ZK_ECANCELED;
    if (r->state != RQ_DONE) return ZK_EAGAIN;
    if (req_status) *req_status = r->status;
    return ZK_OK;
}

extern "C" int zk_session_times(zk_session *s, zk_ticket ticket, double *t_submit, double *t_admit, double *t_done)
{
    if (!s) return ZK_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return ZK_EINVAL;
    if (t_submit) *t_submit = it->second->t_submit;
    if (t_admit) *t_admit = it->second->t_admit;
    if (t_done) *t_done = it->second->t_done;
    return ZK_OK;
}

extern "C" int zk_session_destroy(zk_session *s)
{
    if (!s) return ZK_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->th.joinable()) s->th.join();
    hipStreamSynchronize(s->ctx->stream);
    delete s->e2;   // releases the iterate storage of unfinished requests
    delete s->e4;
    delete s->ap;
    {
        // pending requests are cancelled: a thread blocked in zk_session_poll
        // wakes with ZK_ECANCELED, and the session is freed only after every
        // such thread has left
        std::unique_lock<std::mutex> lk(s->mu);
        s->closing = true;
        for (auto &kv : s->all) {
            Request *r = kv.second;
            if (r->state == RQ_QUEUED || r->state == RQ_RUNNING) r->state = RQ_CANCELLED;
        }
        s->cv_done.notify_all();
        s->cv_left.wait(lk, [&] { return s->waiters == 0; });
        for (auto &kv : s->all) delete kv.second;
        s->all.clear();
    }
    s->pool.clear();
    delete s;
    return ZK_OK;
}
