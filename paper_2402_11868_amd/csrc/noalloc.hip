// zk_heev_dd_noalloc: the double-double eigendecomposition of zk_heev_dd with
// every byte of its device workspace taken from one static device array per
// GPU, for callers that cannot call the HIP allocator.
//
// The array `scratch` below is a device symbol: in host code its name is a
// host-side stand-in, not a device address.  Its address on each device is
// read once, with that device current, by hipGetSymbolAddress and kept per
// device; only that pointer is handed to the workspace sub-allocator, and so
// to the kernels, memsets and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/zk.h"
#include "api_internal.h"

static __device__ __align__(256) char scratch[ZK_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu[kMaxDevices];          // one call at a time per device (the array is shared)
void *g_ptr[kMaxDevices] = {nullptr};  // device address of `scratch`, per device
std::mutex g_ptr_mu;

// The array's address on the current device `dev` (looked up once).
int scratch_address(zk_ctx *ctx, int dev, void **out)
{
    std::lock_guard<std::mutex> g(g_ptr_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            hipGetLastError();
            return ctx->fail(ZK_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                             hipGetErrorString(e));
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return ZK_OK;
}
}  // namespace

extern "C" int zk_heev_dd_noalloc(zk_ctx *ctx, int count, const zk_herm *A, zk_eig_out *out, const zk_opts *opts)
{
    if (!ctx) return ZK_EINVAL;
    if (ctx->poisoned) return ctx->fail(ZK_EDEVICE, "context poisoned by an earlier device error");
    if (count < 1 || !A || !out) return ctx->fail(ZK_EINVAL, "count < 1 or NULL arrays");
    if (ctx->device < 0 || ctx->device >= kMaxDevices) return ctx->fail(ZK_EINVAL, "device index out of range");
    // the least the call needs: every matrix's binary64 stage, inputs and
    // iterates at once, plus one shifted-LU slot of the largest order
    size_t need = 0;
    int nmax = 0;
    for (int i = 0; i < count; i++) {
        if (A[i].n < 1) return ctx->fail(ZK_EINVAL, "matrix %d: n < 1", i);
        need += zk_workspace_bytes(A[i].n, 2, 0);
        if (A[i].n > nmax) nmax = A[i].n;
    }
    need += zk_workspace_bytes(nmax, 2, 1) - zk_workspace_bytes(nmax, 2, 0);
    if (need > ZK_NOALLOC_SCRATCH_BYTES)
        return ctx->fail(ZK_ENOMEM, "the call needs at least %zu bytes of scratch; the static array holds %zu",
                         need, (size_t)ZK_NOALLOC_SCRATCH_BYTES);
    if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(ZK_EDEVICE, "hipSetDevice failed");
    void *ptr = nullptr;
    int rc = scratch_address(ctx, ctx->device, &ptr);
    if (rc != ZK_OK) return rc;

    std::lock_guard<std::mutex> guard(g_mu[ctx->device]);
    // The context's own workspaces step aside for the call: every buffer the
    // call takes comes from the arena over the array, and none is kept.
    DevBuf *bufs[5] = {&ctx->s1, &ctx->s2in, &ctx->s2vec, &ctx->s2lu, &ctx->meta};
    DevBuf saved[5];
    for (int k = 0; k < 5; k++) {
        saved[k] = *bufs[k];
        *bufs[k] = DevBuf();
    }
    const size_t saved_budget = ctx->budget, saved_extra = ctx->extra, saved_hw = ctx->high_water;
    const bool saved_timer = ctx->timer.on;
    ctx->timer.on = false;   // event records would create events
    Arena arena;
    arena.reset((char *)ptr, ZK_NOALLOC_SCRATCH_BYTES);
    ctx->arena = &arena;
    ctx->budget = ZK_NOALLOC_SCRATCH_BYTES;
    ctx->extra = 0;

    rc = zk_heev_dd(ctx, count, A, out, opts);

    // nothing may still run in the array when the next call reuses it
    if (hipStreamSynchronize(ctx->stream) != hipSuccess && rc >= 0)
        rc = ctx->fail(ZK_EDEVICE, "stream synchronisation failed after the call");
    for (int k = 0; k < 5; k++) {
        ctx->drop(*bufs[k]);
        *bufs[k] = saved[k];
    }
    ctx->arena = nullptr;
    ctx->budget = saved_budget;
    ctx->extra = saved_extra;
    ctx->high_water = saved_hw;
    ctx->timer.on = saved_timer;
    return rc;
}
