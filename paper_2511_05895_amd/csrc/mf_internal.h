// Internal declarations shared by the host driver (mf_api.cpp) and the gfx950
// kernels (mf_kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf {

// A vertex whose arc list is at most this long is handled by one lane in the
// push/relabel and invalid-edge sweeps; longer lists get a whole wavefront.
constexpr int kLightMaxDeg = 32;
// Arcs per BFS frontier item: a frontier vertex with a longer list is split
// into several items so that hubs are expanded by many wavefronts at once.
constexpr int kChunk = 256;
// Threads per workgroup of the multi-workgroup persistent kernel and of the
// one-workgroup variant.
constexpr int kBlock = 256;
constexpr int kBlockSingle = 1024;

// Loop status written by the persistent kernel.
enum : int32_t { kRunning = 0, kSolved = 1, kIterLimit = 2, kAborted = 3, kDeadline = 4 };

// Counter slots (all int64).
enum : int {
    kStGlobalRelabels = 0,
    kStLevels,
    kStBfsVertices,
    kStBfsArcs,
    kStPrCycles,
    kStPrArcs,
    kStPushes,
    kStRelabels,
    kStRieArcs,
    kStRieSat,
    kStUpdates,
    kStClamps,
    kStSourcePushes,
    kStIterations,
    kStCount
};

struct alignas(128) PaddedU32 {
    uint32_t v;
    uint32_t pad[31];
};

// Device control block: barrier words on their own cache lines, then loop
// counters.  Reset by k_reset_ctrl before every solving call.
struct Ctrl {
    PaddedU32 bar_count;
    PaddedU32 bar_gen;
    PaddedU32 abort;
    int32_t qcount[4];  // frontier items per BFS level, triple-buffered
    int32_t nlight;     // active vertices with short arc lists
    int32_t nheavy;     // active vertices with long arc lists
    int32_t status;
    int32_t err;        // update validation: 1 id range, 2 capacity range, 4 duplicate
    int32_t stop;       // set by the leader when the time budget ran out
    int32_t pad_;
    int64_t deficit;    // sum of e(v) < 0 over v not in {s, t} at termination
    int64_t e_t;        // e(t) at termination
    int64_t cut;        // cut capacity (k_min_cut)
    int64_t stat[kStCount];
};

// Device-resident graph and state.  arc[a] = {head, residual capacity}; the
// tail of arc a is the head of its twin.
struct DevGraph {
    int32_t n, s, t, A;
    int64_t m;
    int32_t *row_ptr;   // n+1
    int2 *arc;          // A
    int32_t *twin;      // A
    int32_t *cap;       // A
    int32_t *edge2arc;  // m
    int32_t *ecap;      // m
    int32_t *stamp;     // m, duplicate detection inside one batch
    int64_t *e;         // n
    int32_t *h;         // n
    int2 *q[2];         // BFS frontier items {vertex, first arc}, double-buffered
    int64_t qcap;       // items per frontier buffer
    int32_t *wl_light;  // n
    int32_t *wl_heavy;  // n
    int32_t *heavy_all; // vertices with long arc lists (topology-driven sweeps)
    int32_t n_heavy_all;
    Ctrl *ctrl;
};

struct LoopParams {
    int32_t kc;              // KERNELCYCLES
    int32_t mode;            // 0 data-driven, 1 topology-driven
    int64_t max_iter;        // < 0 unlimited
    int64_t deadline_ticks;  // wall-clock ticks allowed for one launch (> 0)
    int64_t barrier_ticks;   // wall-clock ticks one grid-barrier wait may take
};

// ---- launch wrappers (mf_kernels.hip) ----
hipError_t launch_reset_ctrl(const DevGraph &g, hipStream_t st);
hipError_t launch_init_state(const DevGraph &g, hipStream_t st);
hipError_t launch_saturate_source(const DevGraph &g, hipStream_t st);
hipError_t launch_validate_updates(const DevGraph &g, const int64_t *ids, const int32_t *caps,
                                   int64_t k, int32_t epoch, int32_t cap_limit, hipStream_t st);
hipError_t launch_apply_delta(const DevGraph &g, const int64_t *ids, const int32_t *caps, int64_t k,
                              hipStream_t st);
hipError_t launch_clamp(const DevGraph &g, const int64_t *ids, int64_t k, hipStream_t st);
hipError_t launch_loop(const DevGraph &g, const LoopParams &p, int grid, hipStream_t st);
hipError_t launch_min_cut(const DevGraph &g, uint8_t *d_side, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t st);
// Largest co-resident workgroup count of the multi-workgroup loop kernel.
hipError_t loop_max_coresident(int device, int *blocks);

}  // namespace mf
