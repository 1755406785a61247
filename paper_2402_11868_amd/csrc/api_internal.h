// Host-side context of libzk (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <map>
#include <string>
#include <vector>

#include "../../include/zk.h"
#include "stage.h"

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void release()
    {
        if (p) hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

// First-fit sub-allocator over one device region that the library does not
// own (the static scratch array of the no-allocation entry point): blocks are
// 256-byte aligned, freed blocks merge with free neighbours.  Host-side
// bookkeeping only; it never calls the HIP allocator.
struct Arena {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length of free runs
    std::map<size_t, size_t> used_;   // offset -> length of taken blocks
    size_t in_use = 0, peak = 0;
    void reset(char *b, size_t s)
    {
        base = b;
        size = s;
        free_.clear();
        used_.clear();
        if (s) free_[0] = s;
        in_use = peak = 0;
    }
    void *take(size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            used_[off] = bytes;
            in_use += bytes;
            if (in_use > peak) peak = in_use;
            return base + off;
        }
        return nullptr;
    }
    bool owns(const void *p) const { return base && (const char *)p >= base && (const char *)p < base + size; }
    void give(void *p)
    {
        auto u = used_.find((size_t)((char *)p - base));
        if (u == used_.end()) return;
        size_t off = u->first, len = u->second;
        used_.erase(u);
        in_use -= len;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && nx->first == off + len) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += len;
                return;
            }
        }
        free_[off] = len;
    }
};

// Counters of the per-pair iteration of one call (zk_ctx_last_stats).
struct Stage2Stats {
    int iters_hist[16] = {0};
    int rounds = 0;
    long long solves = 0;
    std::vector<int> active_per_iter;
};

struct zk_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t budget = 0;
    bool poisoned = false;
    std::string err;
    // grow-only workspaces, all counted against the budget
    DevBuf s1;      // binary64-stage scratch
    DevBuf s2in;    // stage-2 inputs: limb-planar matrix copies, binary64 pairs
    DevBuf s2vec;   // stage-2 iterates and Rayleigh quotients
    DevBuf s2lu;    // shifted-LU slots
    DevBuf meta;    // descriptor tables
    size_t extra = 0;        // per-matrix iterate buffers held by stage-2 engines
    // side streams (default priority) on which the binary64 stage runs groups
    // of different orders concurrently, and the events that join them
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    Stage2Stats last;        // counters of the last zk_heev_dd / zk_heev_qd call
    zk::KernelTimer timer;   // per-kernel-class HIP-event timing (instrumentation)
    zk::KernelTimer *tp() { return timer.on ? &timer : nullptr; }
    size_t held() const;
    size_t high_water = 0;   // largest held() seen at a growth
    void note_held()
    {
        const size_t h = held();
        if (h > high_water) high_water = h;
    }
    int ensure(DevBuf &b, size_t bytes);
    // Device workspace: from the HIP allocator, or, while `arena` is set
    // (inside the no-allocation entry point), from the arena alone.
    Arena *arena = nullptr;
    int dev_alloc(void **p, size_t bytes);
    void dev_free(void *p);
    void drop(DevBuf &b);
    // Room for `bytes` more under the budget: the shifted-LU slots are
    // scratch between iteration rounds (every engine lays them out again when
    // the buffer changed), so they are given back when the budget is short.
    bool make_room(size_t bytes);
    int fail(int status, const char *fmt, ...);
};

namespace zk {
// One matrix for the all-pairs refinement (its binary64 stage done: hf, w0,
// V0 as produced by run_stage1), and the record of a finished one.
struct ApReq {
    zk_herm A;
    zk_eig_out out;
    const double *hf, *w0, *V0;
    double tol;
    int max_iter, want_vectors;
    void *cookie;
};
struct ApDone {
    void *cookie;
    int status;
    int iters;
};
// device bytes the all-pairs engine holds for one matrix of order n
size_t ap_bytes(int n);
// The all-pairs refinement engine (allpairs.hip): add() matrices, round()
// runs one whole-basis iteration for every live one; stopped matrices are
// written to their outputs and appended to `finished` (cleared by the caller).
class ApEngine {
public:
    explicit ApEngine(zk_ctx *ctx);
    ~ApEngine();
    ApEngine(const ApEngine &) = delete;
    ApEngine &operator=(const ApEngine &) = delete;
    int add(const std::vector<ApReq> &reqs);
    bool any_live() const;
    int round();
    std::vector<ApDone> finished;
    struct Impl;

private:
    Impl *impl;
};
}  // namespace zk
