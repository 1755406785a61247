// Host-side context of libzk (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <string>
#include <vector>

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
    zk::KernelTimer timer;   // per-kernel-class HIP-event timing (instrumentation)
    zk::KernelTimer *tp() { return timer.on ? &timer : nullptr; }
    size_t held() const;
    int ensure(DevBuf &b, size_t bytes);
    int fail(int status, const char *fmt, ...);
};

// Counters the benchmark reads through zk_heev_stats().
struct Stage2Stats {
    int iters_hist[16] = {0};
    int rounds = 0;
    long long solves = 0;
    std::vector<int> active_per_iter;
};
