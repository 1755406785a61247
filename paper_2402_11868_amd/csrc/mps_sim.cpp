// MPS simulation driver: a chain of qubits in matrix product form whose
// two-qubit gates turn into the stream of Hermitian bond matrices that the
// paper names as the dominant cost of its MPS method (Sec. 1, Sec. 2.1), and
// that a serving session diagonalises with continuous batching.
//
// Form: sites in right-canonical form with the Schmidt values of every bond
// (Hastings' form of the Vidal decomposition).  A two-qubit gate G on qubits
// (q, q+1):
//   theta = G (B_q B_{q+1})                       (double-double)
//   rho   = theta^H diag(lambda_{q-1}^2) theta    (order 2 chi_{q+1}, PSD)
//   rho   = V diag(w) V^H                         (the session, double-double)
//   keep the chi' largest w above cutoff^2 w_max (at most chi_max):
//   B_{q+1} <- V^H,  B_q <- theta V,  lambda_q <- sqrt(w)
// No Schmidt value is ever inverted, so tiny ones stay harmless.  The gates
// of one layer act on disjoint pairs, so their bond matrices are submitted
// together and share the session's launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/zk.h"
#include "api_internal.h"
#include "stage.h"

using namespace zk;

namespace {
size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct Slot {             // device scratch of one gate of a layer
    double *T[2], *rho[2], *V[2], *w[2], *G[2];
};
}  // namespace

struct zk_mps {
    zk_ctx *ctx = nullptr;       // kernels and storage (the caller's context)
    zk_ctx *sctx = nullptr;      // the session's own context
    zk_session *sess = nullptr;
    int nq = 0, chi_max = 0;
    double cutoff = 0.0;
    std::vector<int> chi;        // chi[b], b = 0 .. nq (chi[0] = chi[nq] = 1)
    void *buf = nullptr;         // every device array below
    size_t bytes = 0;
    std::vector<double *> site;  // per site: two planes of chi_max x (2 chi_max) complex (stride sp doubles)
    std::vector<double *> lam;   // per bond: Schmidt values, two planes of chi_max
    std::vector<double *> eig;   // per bond: their squares
    size_t sp = 0;               // doubles per site plane
    std::vector<double *> tmp;   // per slot: next-site buffers for q and q+1 (two each)
    std::vector<Slot> slot;
    std::vector<double> lat;     // submit-to-done seconds of every bond matrix
    std::vector<int> order;      // their orders
};

static int mps_fail(zk_mps *m, int st, const char *msg) { return m->ctx->fail(st, "%s", msg); }

extern "C" int zk_mps_create(zk_ctx *ctx, int nq, int chi_max, double cutoff, zk_mps **out)
{
    if (!ctx || !out || nq < 2 || nq > 4096 || chi_max < 1 || chi_max > 256 || !(cutoff >= 0.0)) return ZK_EINVAL;
    *out = nullptr;
    if (ctx->poisoned) return ctx->fail(ZK_EDEVICE, "context poisoned by an earlier device error");
    if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(ZK_EDEVICE, "hipSetDevice failed");
    zk_mps *m = new zk_mps();
    m->ctx = ctx;
    m->nq = nq;
    m->chi_max = chi_max;
    m->cutoff = cutoff;
    m->chi.assign(nq + 1, 1);
    const int X = chi_max, N = 2 * chi_max;
    m->sp = 2 * (size_t)X * 2 * X;   // complex entries x 2 doubles
    const int nslot = nq / 2;
    const size_t site_b = al(8 * m->sp), vec_b = al(8 * (size_t)X), mat_b = al(8 * 2 * (size_t)N * N), w_b = al(8 * (size_t)N);
    m->bytes = (size_t)nq * 2 * site_b + (size_t)(nq + 1) * 4 * vec_b + (size_t)nslot * (4 * site_b + 6 * mat_b + 2 * w_b + 2 * al(8 * 32));
    if (!ctx->make_room(m->bytes)) {
        delete m;
        return ctx->fail(ZK_ENOMEM, "the MPS needs %zu bytes", m->bytes);
    }
    if (ctx->dev_alloc(&m->buf, m->bytes) != ZK_OK) {
        delete m;
        return ZK_ENOMEM;
    }
    ctx->extra += m->bytes;
    ctx->note_held();
    char *b = (char *)m->buf;
    for (int q = 0; q < nq; q++)
        for (int p = 0; p < 2; p++) {
            m->site.push_back((double *)b);
            b += site_b;
        }
    for (int q = 0; q <= nq; q++)
        for (int p = 0; p < 4; p++) {
            (p < 2 ? m->lam : m->eig).push_back((double *)b);
            b += vec_b;
        }
    for (int k = 0; k < nslot; k++) {
        for (int p = 0; p < 4; p++) {
            m->tmp.push_back((double *)b);
            b += site_b;
        }
        Slot s;
        for (int p = 0; p < 2; p++) {
            s.T[p] = (double *)b; b += mat_b;
            s.rho[p] = (double *)b; b += mat_b;
            s.V[p] = (double *)b; b += mat_b;
            s.w[p] = (double *)b; b += w_b;
            s.G[p] = (double *)b; b += al(8 * 32);
        }
        m->slot.push_back(s);
    }
    // |0...0>: every site [[1], [0]] (chi 1), every bond weight 1
    hipStream_t st = ctx->stream;
    int rc = ZK_OK;
    if (hipMemsetAsync(m->buf, 0, m->bytes, st) != hipSuccess) rc = ZK_EDEVICE;
    const double one = 1.0;
    for (int q = 0; q < nq && rc == ZK_OK; q++)
        if (hipMemcpyAsync(m->site[2 * q], &one, 8, hipMemcpyHostToDevice, st) != hipSuccess) rc = ZK_EDEVICE;
    for (int q = 0; q <= nq && rc == ZK_OK; q++)
        if (hipMemcpyAsync(m->lam[2 * q], &one, 8, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(m->eig[2 * q], &one, 8, hipMemcpyHostToDevice, st) != hipSuccess)
            rc = ZK_EDEVICE;
    if (rc == ZK_OK && hipStreamSynchronize(st) != hipSuccess) rc = ZK_EDEVICE;
    if (rc == ZK_OK) rc = zk_ctx_create(ctx->device, nullptr, 0, &m->sctx);
    if (rc == ZK_OK) rc = zk_session_create(m->sctx, 0, 0, &m->sess);
    if (rc != ZK_OK) {
        zk_mps_destroy(m);
        return ctx->fail(rc == ZK_EDEVICE ? ZK_EDEVICE : rc, "MPS set-up failed");
    }
    *out = m;
    return ZK_OK;
}

extern "C" int zk_mps_destroy(zk_mps *m)
{
    if (!m) return ZK_OK;
    if (m->sess) zk_session_destroy(m->sess);
    if (m->sctx) zk_ctx_destroy(m->sctx);
    if (m->buf) {
        hipStreamSynchronize(m->ctx->stream);
        m->ctx->dev_free(m->buf);
        m->ctx->extra -= m->bytes;
    }
    delete m;
    return ZK_OK;
}

extern "C" int zk_mps_apply1(zk_mps *m, int q, const double *gate)
{
    if (!m || !gate || q < 0 || q >= m->nq) return ZK_EINVAL;
    zk_ctx *ctx = m->ctx;
    hipStream_t st = ctx->stream;
    Slot &s = m->slot[0];
    // gate: two limb planes of 2 x 2 complex (column-major), host
    if (hipMemcpyAsync(s.G[0], gate, 64, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s.G[1], gate + 8, 64, hipMemcpyHostToDevice, st) != hipSuccess)
        return ctx->fail(ZK_EDEVICE, "gate upload failed");
    MpsSimDesc D;
    std::memset(&D, 0, sizeof D);
    D.cl = m->chi[q];
    D.cm = m->chi[q + 1];
    D.T[0] = m->site[2 * q];
    D.T[1] = m->site[2 * q + 1];
    D.G[0] = s.G[0];
    D.G[1] = s.G[1];
    if (mps_sim_gate1(D, st) || hipStreamSynchronize(st) != hipSuccess)
        return ctx->fail(ZK_EDEVICE, "one-qubit gate failed");
    return ZK_OK;
}

extern "C" int zk_mps_apply2(zk_mps *m, int count, const int *q, const double *const *gates)
{
    if (!m || count < 0 || (count > 0 && (!q || !gates))) return ZK_EINVAL;
    if (count > (int)m->slot.size()) return m->ctx->fail(ZK_EINVAL, "more gates than disjoint pairs");
    std::vector<char> used(m->nq, 0);
    for (int k = 0; k < count; k++) {
        if (q[k] < 0 || q[k] + 1 >= m->nq || !gates[k]) return m->ctx->fail(ZK_EINVAL, "gate %d: bad qubit pair", k);
        if (used[q[k]] || used[q[k] + 1]) return m->ctx->fail(ZK_EINVAL, "gates of one layer must act on disjoint pairs");
        used[q[k]] = used[q[k] + 1] = 1;
    }
    zk_ctx *ctx = m->ctx;
    hipStream_t st = ctx->stream;
    std::vector<MpsSimDesc> D(count);
    for (int k = 0; k < count; k++) {
        Slot &s = m->slot[k];
        const int a = q[k];
        if (hipMemcpyAsync(s.G[0], gates[k], 256, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(s.G[1], gates[k] + 32, 256, hipMemcpyHostToDevice, st) != hipSuccess)
            return ctx->fail(ZK_EDEVICE, "gate upload failed");
        MpsSimDesc &d = D[k];
        std::memset(&d, 0, sizeof d);
        d.cl = m->chi[a];
        d.cm = m->chi[a + 1];
        d.cr = m->chi[a + 2];
        for (int p = 0; p < 2; p++) {
            d.Bq[p] = m->site[2 * a + p];
            d.Bq1[p] = m->site[2 * (a + 1) + p];
            d.lam[p] = m->lam[2 * a + p];
            d.T[p] = s.T[p];
            d.G[p] = s.G[p];
            d.rho[p] = s.rho[p];
            d.V[p] = s.V[p];
            d.w[p] = s.w[p];
            d.Bq_out[p] = m->tmp[4 * k + p];
            d.Bq1_out[p] = m->tmp[4 * k + 2 + p];
            d.lam_out[p] = m->lam[2 * (a + 1) + p];
            d.eig_out[p] = m->eig[2 * (a + 1) + p];
        }
        if (mps_sim_bond(d, st)) return ctx->fail(ZK_EDEVICE, "bond matrix launch failed");
    }
    if (hipStreamSynchronize(st) != hipSuccess) return ctx->fail(ZK_EDEVICE, "bond matrices failed");
    // every bond matrix of the layer into the session at once
    std::vector<zk_ticket> tk(count);
    std::vector<zk_herm> H(count);
    std::vector<zk_eig_out> O(count);
    for (int k = 0; k < count; k++) {
        const int N = 2 * D[k].cr;
        std::memset(&H[k], 0, sizeof(zk_herm));
        H[k].n = N;
        H[k].lda = N;
        H[k].limbs = 2;
        H[k].plane[0] = D[k].rho[0];
        H[k].plane[1] = D[k].rho[1];
        std::memset(&O[k], 0, sizeof(zk_eig_out));
        O[k].n = N;
        O[k].ldv = N;
        O[k].limbs = 2;
        O[k].w[0] = m->slot[k].w[0];
        O[k].w[1] = m->slot[k].w[1];
        O[k].v[0] = m->slot[k].V[0];
        O[k].v[1] = m->slot[k].V[1];
        int rc;
        while ((rc = zk_session_submit(m->sess, &H[k], &O[k], 2, nullptr, &tk[k])) == ZK_EAGAIN) {
        }
        if (rc != ZK_OK) return ctx->fail(rc, "bond matrix %d: session submit failed", k);
    }
    int status = ZK_OK;
    std::vector<double> wh;
    for (int k = 0; k < count; k++) {
        int rs = ZK_OK;
        const int rc = zk_session_poll(m->sess, tk[k], -1, &rs);
        if (rc != ZK_OK) return ctx->fail(rc, "bond matrix %d: session poll failed", k);
        if (rs < 0) return ctx->fail(rs, "bond matrix %d: eigendecomposition failed", k);
        if (rs == ZK_ENOCONV) status = ZK_ENOCONV;
        double t0 = 0, t1 = 0, t2 = 0;
        zk_session_times(m->sess, tk[k], &t0, &t1, &t2);
        m->lat.push_back(t2 - t0);
        const int N = 2 * D[k].cr;
        m->order.push_back(N);
        // kept: the largest eigenvalues above cutoff^2 w_max, at most chi_max (and at most 2 chi_{q})
        wh.resize(N);
        if (hipMemcpy(wh.data(), m->slot[k].w[0], 8 * (size_t)N, hipMemcpyDeviceToHost) != hipSuccess)
            return ctx->fail(ZK_EDEVICE, "eigenvalue read-back failed");
        const double wmax = std::max(wh[N - 1], 0.0);
        int keep = 0;
        while (keep < N && keep < m->chi_max && keep < 2 * D[k].cl && wh[N - 1 - keep] > m->cutoff * m->cutoff * wmax)
            keep++;
        D[k].chi = std::max(keep, 1);
        if (mps_sim_split(D[k], st)) return ctx->fail(ZK_EDEVICE, "split launch failed");
    }
    if (hipStreamSynchronize(st) != hipSuccess) return ctx->fail(ZK_EDEVICE, "split failed");
    // the new sites replace the old ones
    for (int k = 0; k < count; k++) {
        const int a = q[k];
        for (int p = 0; p < 2; p++) {
            std::swap(m->site[2 * a + p], m->tmp[4 * k + p]);
            std::swap(m->site[2 * (a + 1) + p], m->tmp[4 * k + 2 + p]);
        }
        m->chi[a + 1] = D[k].chi;
    }
    return status;
}

extern "C" int zk_mps_bond(zk_mps *m, int bond, int max, double *eig, int *chi)
{
    if (!m || bond < 0 || bond > m->nq || !chi) return ZK_EINVAL;
    *chi = m->chi[bond];
    if (!eig || max < 1) return ZK_OK;
    const int c = std::min(max, m->chi[bond]);
    if (hipMemcpy(eig, m->eig[2 * bond], 8 * (size_t)c, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(eig + max, m->eig[2 * bond + 1], 8 * (size_t)c, hipMemcpyDeviceToHost) != hipSuccess)
        return m->ctx->fail(ZK_EDEVICE, "read-back failed");
    return ZK_OK;
}

extern "C" int zk_mps_site(zk_mps *m, int q, int *chi_l, int *chi_r, double *out, size_t capacity)
{
    if (!m || q < 0 || q >= m->nq || !chi_l || !chi_r) return ZK_EINVAL;
    *chi_l = m->chi[q];
    *chi_r = m->chi[q + 1];
    const size_t cnt = 2 * (size_t)m->chi[q] * 2 * m->chi[q + 1];   // doubles per plane
    if (!out) return ZK_OK;
    if (capacity < 2 * cnt) return ZK_EINVAL;
    if (hipMemcpy(out, m->site[2 * q], 8 * cnt, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(out + cnt, m->site[2 * q + 1], 8 * cnt, hipMemcpyDeviceToHost) != hipSuccess)
        return m->ctx->fail(ZK_EDEVICE, "read-back failed");
    return ZK_OK;
}

extern "C" int zk_mps_latencies(zk_mps *m, int max, double *seconds, int *orders, int *count)
{
    if (!m || !count) return ZK_EINVAL;
    *count = (int)m->lat.size();
    const int c = std::min(max, *count);
    for (int i = 0; i < c; i++) {
        if (seconds) seconds[i] = m->lat[i];
        if (orders) orders[i] = m->order[i];
    }
    return ZK_OK;
}
