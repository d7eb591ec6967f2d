// C-ABI of the library (include/mf.h): handle lifecycle, argument checks and
// the per-call launch sequences.  All arithmetic of the method runs in the
// kernels of mf_kernels.hip; this file only validates, builds the arc-pair
// layout once per handle, allocates, launches and reads back results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mf.h"
#include "build_pairs.h"
#include "ctrl_stats.h"
#include "mf_internal.h"

namespace {

enum class State { NoFlow, Partial, Solved, NeedsSolve };

thread_local std::string g_create_error;

// Registered when the library is loaded, i.e. after the HIP runtime it links
// against, so it runs before the runtime's own exit handlers.
std::atomic<bool> g_exiting{false};
void mark_exiting() { g_exiting.store(true); }
struct ExitHook {
    ExitHook() { std::atexit(mark_exiting); }
} g_exit_hook;

}  // namespace

bool mf::process_exiting() { return g_exiting.load(); }

struct mf_handle {
    int device = 0;
    // device memory of the handle: the caller's allocator, or hipMalloc / hipFree
    void *(*alloc_fn)(size_t, void *) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *alloc_ctx = nullptr;
    int32_t debug_checks = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    mf::DevGraph g{};
    std::vector<void *> allocs;
    mf::Ctrl *h_ctrl = nullptr;  // pinned read-back of the control block
    // staging of host update batches: one device buffer and its pinned host
    // copy, ids then capacities back to back, so that one copy uploads both;
    // d_ids / d_caps point into it for the current call
    void *d_stage = nullptr;
    unsigned char *p_stage = nullptr;
    int64_t staging_cap = 0;  // updates the buffers hold
    int64_t *d_ids = nullptr;
    int32_t *d_caps = nullptr;
    uint8_t *d_side = nullptr;
    int32_t cap_limit = 0;
    int32_t kc = 1;
    int32_t mode = MF_MODE_DATA;
    int32_t grid = 1;
    int64_t max_iter = -1;
    int64_t deadline_ticks = 0;
    int64_t barrier_ticks = 0;
    int64_t relabel_budget = 0;
    int32_t max_rounds = 0;
    int32_t rounds_per_level = 1;
    int32_t use_gap = 0;
    int32_t stall_rounds = 3;
    int32_t solo_items = 0;
    int32_t lazy_items = 0;
    int32_t bu_alpha = 0;  // direction rule of the BFS (0: top-down only)
    int32_t walk = 1;      // long arc lists visited by the downhill walk (else scan first)
    int32_t local_stage = 1;  // dynamic updates run the local stage before the global loop
    int32_t *d_pmark = nullptr;  // n: list tags of the local pulls
    int32_t ptag = 0;            // last tag used
    // Vertex numbering of the layout: the caller's vertex v is the handle's
    // new_of_old[v] (both empty: the caller's numbering); caller_of_arc maps
    // an arc of the layout to its index in the layout of the caller's
    // numbering, computed on the first export or import that needs it.
    std::vector<int32_t> new_of_old, old_of_new, caller_of_arc;
    int32_t combine = 0;
    double tick_ms = 1e-5;  // one wall-clock tick in ms
    int32_t seq = 1;  // next round id; round ids stamp mark[] and rmark[]
    // learned phase schedule (mf_set_policy)
    const mf_policy_t *policy = nullptr;
    int32_t policy_mode = MF_POLICY_FIXED;
    float policy_margin = 0.f;
    float policy_explore = 0.f;
    uint64_t policy_seed = 0;
    int32_t policy_action = 0;
    int32_t policy_per_call = 0;
    float *d_ptrace = nullptr;
    float batch_fraction = 1.f;  // of the current call
    int32_t epoch = 0;
    int64_t nhuge = 0;          // vertices visited by whole workgroups (huge-list capacity)
    int32_t push_pull = 0;      // dynamic updates by Dynamic Push-Pull (MF_FLAG_PUSH_PULL)
    // Second view of the state, allocated on the first push-pull update or
    // flow extraction: part tags, the reversed view with its own state and
    // work arrays (rv), the forward copy of the flow extraction (fv: own arcs,
    // excesses, heights and control block, the handle's work arrays), and the
    // per-arc / per-edge flow buffers.
    bool views = false;
    uint8_t *d_part = nullptr;
    int64_t *d_work = nullptr;
    mf::DevGraph rv{};
    mf::DevGraph fv{};
    int32_t *d_rem = nullptr;
    int32_t *d_eflow = nullptr;
    mf::Ctrl *h_vctrl = nullptr;  // pinned read-back of the two views' control blocks
    mf::DevGraph *d_tviews = nullptr;     // the two-team kernel's table of views
    mf::LoopParams *d_tparams = nullptr;  // and of their loop parameters
    unsigned char *h_tdesc = nullptr;     // pinned staging of both tables
    int32_t vseq = 1;             // next round id of rv's marks
    bool teams_fit = false;       // the two-team kernel's grid fits the device at once
    State state = State::NoFlow;
    int64_t value = 0;
    mf_stats_t stats{};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    std::string err;
};

namespace {

// Default frontier size (items) up to which one workgroup runs BFS levels alone.
constexpr int32_t kSoloItems = 128;
constexpr int32_t kLazyItems = 1024;
// Direction rule of the BFS: bottom-up when frontier arcs x alpha exceed the
// arcs not reached yet; back to top-down below n / beta frontier vertices.
constexpr int32_t kBuAlpha = 14;
constexpr int32_t kBuBeta = 24;
// Rounds of local pulls into the deficits a batch leaves (the last one
// without handing deficits on).
constexpr int kPullRounds = 4;

int fail(mf_handle_t *h, int code, const std::string &msg) {
    if (h) h->err = msg;
    else g_create_error = msg;
    return code;
}

int hip_fail(mf_handle_t *h, hipError_t e, const char *what) {
    return fail(h, MF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(h, expr)                                       \
    do {                                                       \
        hipError_t _e = (expr);                                \
        if (_e != hipSuccess) return hip_fail((h), _e, #expr); \
    } while (0)

// Device memory through the caller's allocator when one was given.
hipError_t raw_alloc(mf_handle_t *h, void **q, size_t bytes) {
    if (h->alloc_fn) {
        *q = h->alloc_fn(bytes, h->alloc_ctx);
        return *q ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMalloc(q, bytes);
}

void raw_free(mf_handle_t *h, void *q) {
    if (!q) return;
    if (h->free_fn) h->free_fn(q, h->alloc_ctx);
    else (void)hipFree(q);
}

template <typename T>
hipError_t dev_alloc(mf_handle_t *h, T **p, int64_t count) {
    size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    void *q = nullptr;
    hipError_t e = raw_alloc(h, &q, bytes);
    if (e != hipSuccess) return e;
    h->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return hipSuccess;
}

void release(mf_handle_t *h) {
    if (!h || mf::process_exiting()) return;
    if (h->device >= 0) (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (void *p : h->allocs) raw_free(h, p);
    h->allocs.clear();
    raw_free(h, h->d_stage);
    if (h->p_stage) (void)hipHostFree(h->p_stage);
    raw_free(h, h->d_ptrace);
    if (h->h_ctrl) (void)hipHostFree(h->h_ctrl);
    if (h->h_vctrl) (void)hipHostFree(h->h_vctrl);
    if (h->h_tdesc) (void)hipHostFree(h->h_tdesc);
    for (auto &e : h->ev)
        if (e) (void)hipEventDestroy(e);
    if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
}

// Read back the control block and wait for the call's GPU work.
int finish_call(mf_handle_t *h) {
    HIP_TRY(h, hipMemcpyAsync(h->h_ctrl, h->g.ctrl, sizeof(mf::Ctrl), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipEventRecord(h->ev[3], h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return MF_OK;
}

void fill_stats(mf_handle_t *h, bool ran_loop) {
    mf_stats_t &s = h->stats;
    mf::stats_from_ctrl(*h->h_ctrl, h->tick_ms, &s);
    s.grid_blocks = h->grid;
    if (ran_loop) {
        float ms = 0.f;
        s.loop_launches = 1;
        if (hipEventElapsedTime(&ms, h->ev[1], h->ev[2]) == hipSuccess) s.loop_kernel_ms = ms;
    }
    float cm = 0.f;
    if (hipEventElapsedTime(&cm, h->ev[0], h->ev[3]) == hipSuccess) s.call_ms = cm;
}

// Loop parameters of the handle's solving calls (schedule included).
mf::LoopParams loop_params(const mf_handle_t *h) {
    mf::LoopParams p{};
    p.kc = h->kc;
    p.mode = h->mode;
    p.max_iter = h->max_iter;
    p.deadline_ticks = h->deadline_ticks;
    p.barrier_ticks = h->barrier_ticks;
    p.relabel_budget = h->relabel_budget;
    p.max_rounds = h->max_rounds;
    p.seq_base = h->seq;
    p.rounds_per_level = h->rounds_per_level;
    p.use_gap = h->use_gap;
    p.stall_rounds = h->stall_rounds;
    p.solo_items = h->solo_items;
    p.lazy_items = h->lazy_items;
    p.bu_alpha = h->bu_alpha;
    p.bu_beta = kBuBeta;
    p.walk = h->walk;
    p.combine = h->combine;
    p.policy_mode = h->policy_mode;
    p.policy_w = mf::policy_device_params(h->policy);
    p.policy_margin = h->policy_margin;
    p.policy_explore = h->policy_explore;
    p.policy_seed = h->policy_seed;
    p.policy_action = h->policy_action;
    p.batch_fraction = h->batch_fraction;
    p.policy_per_call = h->policy_per_call;
    return p;
}

// Round ids stamp mark[] and rmark[]; restart them with clean stamps before
// they could wrap.
int fresh_round_ids(mf_handle_t *h, mf::DevGraph &g, int32_t &seq) {
    if (seq > (1 << 30)) {
        HIP_TRY(h, mf::launch_fill_i32(g.mark, g.n, 0, h->stream));
        HIP_TRY(h, mf::launch_fill_i32(g.rmark, g.n, 0, h->stream));
        seq = 1;
    }
    return MF_OK;
}

// Add the counters of an earlier launch of the same call.
void add_stats(mf_stats_t &s, const mf_stats_t &x) {
    s.iterations += x.iterations;
    s.global_relabels += x.global_relabels;
    s.bfs_levels += x.bfs_levels;
    s.bfs_vertices += x.bfs_vertices;
    s.bfs_arcs += x.bfs_arcs;
    s.pr_vertex_cycles += x.pr_vertex_cycles;
    s.pr_arcs += x.pr_arcs;
    s.pushes += x.pushes;
    s.relabels += x.relabels;
    s.rie_arcs += x.rie_arcs;
    s.rie_saturations += x.rie_saturations;
    s.updates += x.updates;
    s.clamps += x.clamps;
    s.source_pushes += x.source_pushes;
    s.rounds += x.rounds;
    s.loop_launches += x.loop_launches;
    s.bfs_ms += x.bfs_ms;
    s.pr_ms += x.pr_ms;
    s.rie_ms += x.rie_ms;
    s.loop_kernel_ms += x.loop_kernel_ms;
}

// Launch the persistent loop on g (the handle's graph, or a part-restricted
// view of it), read back, interpret the status.  prior: counters of earlier
// launches of the same call, added to the call's statistics.
int run_loop_and_finish(mf_handle_t *h, const mf::DevGraph *gsel = nullptr, const mf_stats_t *prior = nullptr) {
    int rc = fresh_round_ids(h, h->g, h->seq);
    if (rc) return rc;
    const mf::DevGraph &g = gsel ? *gsel : h->g;
    mf::LoopParams p = loop_params(h);
    // height counts of the gap heuristic start at zero (the loop clears them
    // again before every later global relabel); only the heuristic reads them
    if (h->use_gap) HIP_TRY(h, mf::launch_fill_i32(h->g.hcount, (int64_t)h->g.n + 1, 0, h->stream));
    HIP_TRY(h, hipEventRecord(h->ev[1], h->stream));
    HIP_TRY(h, mf::launch_loop(g, p, h->grid, h->stream));
    HIP_TRY(h, hipEventRecord(h->ev[2], h->stream));
    rc = finish_call(h);
    if (rc) return rc;
    const mf::Ctrl &c = *h->h_ctrl;
    if (c.err) return MF_EINVAL;  // caller reports the message
    h->seq += c.rounds + 1;
    fill_stats(h, true);
    if (prior) add_stats(h->stats, *prior);
    if (c.status == mf::kSolved) {
        h->state = State::Solved;
        h->value = c.e_t + c.deficit;
        return MF_OK;
    }
    if (c.status == mf::kIterLimit) {
        h->state = State::Partial;
        return fail(h, MF_ETIMEOUT, "iteration limit reached; mf_resume continues from this state");
    }
    h->state = State::Partial;
    if (c.status == mf::kDeadline)
        return fail(h, MF_ETIMEOUT, "time budget of the solve kernel ran out; mf_resume continues");
    return fail(h, MF_EDEVICE, "solve kernel aborted (grid barrier wait ran out)");
}

int update_error_text(mf_handle_t *h, int32_t err) {
    std::string msg = "invalid update batch:";
    if (err & 1) msg += " edge id out of range;";
    if (err & 2) msg += " capacity outside [0, " + std::to_string(h->cap_limit) + "];";
    if (err & 4) msg += " duplicate edge id (a batch is a set);";
    return fail(h, MF_EINVAL, msg);
}

int next_epoch(mf_handle_t *h) {
    if (h->epoch == INT32_MAX) {
        HIP_TRY(h, mf::launch_fill_i32(h->g.stamp, h->g.m, 0, h->stream));
        h->epoch = 0;
    }
    h->epoch++;
    return MF_OK;
}

// Upload a host batch through pinned staging (an upload from pageable memory
// is staged by the runtime, synchronously).  A call that failed part-way may
// have left the previous copies queued, so the stream is drained before the
// pinned buffers are written or freed (a no-op after a completed call).
int stage_host_batch(mf_handle_t *h, const int64_t *ids, const int32_t *caps, int64_t k) {
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    constexpr size_t kPer = sizeof(int64_t) + sizeof(int32_t);
    if (k > h->staging_cap) {
        // geometric growth from a floor of min(m, 2^17) updates (1.5 MB): a
        // stream of growing requests reallocates (device and pinned memory,
        // both slow calls) a few times over the handle's life, not per request
        const int64_t floor_k = std::min<int64_t>(std::max<int64_t>(h->g.m, 1), 1 << 17);
        const int64_t want = std::max({k, 2 * h->staging_cap, floor_k});
        raw_free(h, h->d_stage);
        if (h->p_stage) (void)hipHostFree(h->p_stage);
        h->d_stage = nullptr;
        h->p_stage = nullptr;
        h->staging_cap = 0;
        if (raw_alloc(h, &h->d_stage, kPer * want) != hipSuccess) {
            h->d_stage = nullptr;
            return fail(h, MF_ENOMEM, "cannot allocate the update staging buffers");
        }
        if (hipHostMalloc((void **)&h->p_stage, kPer * want, hipHostMallocDefault) != hipSuccess) {
            h->p_stage = nullptr;
            return fail(h, MF_ENOMEM, "cannot allocate the update staging buffers");
        }
        h->staging_cap = want;
    }
    // ids at [0, 8k), capacities at [8k, 12k) of both buffers
    h->d_ids = static_cast<int64_t *>(h->d_stage);
    h->d_caps = reinterpret_cast<int32_t *>(static_cast<unsigned char *>(h->d_stage) + sizeof(int64_t) * k);
    if (k > 0) {
        std::memcpy(h->p_stage, ids, sizeof(int64_t) * k);
        std::memcpy(h->p_stage + sizeof(int64_t) * k, caps, sizeof(int32_t) * k);
        HIP_TRY(h, hipMemcpyAsync(h->d_stage, h->p_stage, kPer * k, hipMemcpyHostToDevice, h->stream));
    }
    return MF_OK;
}

// Allocate the second view of the state (see mf_handle::views).
int ensure_views(mf_handle_t *h) {
    if (h->views) return MF_OK;
    const mf::DevGraph &d = h->g;
    const int64_t n = d.n, A = d.A, m = d.m;
    mf::DevGraph r = d;
    mf::DevGraph f = d;
    hipError_t e;
#define VALLOC(ptr, count)                                                                 \
    do {                                                                                   \
        if ((e = dev_alloc(h, &(ptr), (count))) != hipSuccess)                             \
            return fail(h, MF_ENOMEM, std::string("hipMalloc " #ptr ": ") + hipGetErrorString(e)); \
    } while (0)
    VALLOC(h->d_part, n);
    VALLOC(h->d_work, 2);
    VALLOC(r.arc, A);
    VALLOC(r.e, n);
    VALLOC(r.h, n);
    VALLOC(r.q[0], d.qcap);
    VALLOC(r.q[1], d.qcap);
    VALLOC(r.list[0], n);
    VALLOC(r.list[1], n);
    VALLOC(r.list[2], n);
    VALLOC(r.huge[0], h->nhuge);
    VALLOC(r.huge[1], h->nhuge);
    VALLOC(r.huge[2], h->nhuge);
    VALLOC(r.mark, n);
    VALLOC(r.rmark, n);
    VALLOC(r.relab, n);
    VALLOC(r.hcount, n + 1);
    VALLOC(r.ctrl, 1);
    VALLOC(f.arc, A);
    VALLOC(f.e, n);
    VALLOC(f.h, n);
    VALLOC(f.ctrl, 1);
    VALLOC(h->d_rem, A);
    VALLOC(h->d_eflow, m);
    VALLOC(h->d_tviews, 2);
    VALLOC(h->d_tparams, 2);
#undef VALLOC
    r.ptrace = nullptr;
    f.ptrace = nullptr;
    if (!h->h_vctrl &&
        hipHostMalloc((void **)&h->h_vctrl, 2 * sizeof(mf::Ctrl), hipHostMallocDefault) != hipSuccess)
        return fail(h, MF_ENOMEM, "pinned control blocks of the views");
    if (!h->h_tdesc && hipHostMalloc((void **)&h->h_tdesc, 2 * (sizeof(mf::DevGraph) + sizeof(mf::LoopParams)),
                                     hipHostMallocDefault) != hipSuccess)
        return fail(h, MF_ENOMEM, "pinned staging of the views' table");
    HIP_TRY(h, mf::launch_fill_i32(r.mark, n, 0, h->stream));
    HIP_TRY(h, mf::launch_fill_i32(r.rmark, n, 0, h->stream));
    int tmax = 0;
    HIP_TRY(h, mf::teams_max_coresident(h->device, &tmax));
    h->teams_fit = h->grid >= 2 && h->grid <= tmax;
    h->rv = r;
    h->fv = f;
    h->vseq = 1;
    h->views = true;
    return MF_OK;
}

// Part tags from the heights of the last global relabel (T: h < |V|), with
// the arcs of each part in d_work[0] (S) and d_work[1] (T).
int tag_parts(mf_handle_t *h) {
    HIP_TRY(h, mf::launch_fill_i32(reinterpret_cast<int32_t *>(h->d_work), 4, 0, h->stream));
    HIP_TRY(h, mf::launch_part_from_heights(h->g, h->d_part, h->d_work, h->stream));
    return MF_OK;
}

// Run two disjoint views side by side: one cooperative launch of two teams,
// or, with a one-workgroup handle, one after the other.  a works on the S
// side (its arcs counted in d_work[0]), b on the T side.  Reads both control
// blocks back into h_vctrl[0] / h_vctrl[1] and advances the round ids.
int run_two_views(mf_handle_t *h, const mf::DevGraph &a, mf::LoopParams pa, int32_t &seq_a, const mf::DevGraph &b,
                  mf::LoopParams pb, int32_t &seq_b) {
    mf::DevGraph ga = a, gb = b;
    int rc = fresh_round_ids(h, ga, seq_a);
    if (rc) return rc;
    rc = fresh_round_ids(h, gb, seq_b);
    if (rc) return rc;
    pa.seq_base = seq_a;
    pb.seq_base = seq_b;
    HIP_TRY(h, mf::launch_reset_ctrl(ga, h->stream));
    HIP_TRY(h, mf::launch_reset_ctrl(gb, h->stream));
    if (pa.use_gap) HIP_TRY(h, mf::launch_fill_i32(ga.hcount, (int64_t)ga.n + 1, 0, h->stream));
    if (pb.use_gap) HIP_TRY(h, mf::launch_fill_i32(gb.hcount, (int64_t)gb.n + 1, 0, h->stream));
    if (h->teams_fit) {
        // the table of both views and their parameters (the last call's
        // copies are done: every call ends with a stream synchronisation)
        mf::DevGraph *tv = reinterpret_cast<mf::DevGraph *>(h->h_tdesc);
        mf::LoopParams *tp = reinterpret_cast<mf::LoopParams *>(h->h_tdesc + 2 * sizeof(mf::DevGraph));
        tv[0] = ga;
        tv[1] = gb;
        tp[0] = pa;
        tp[1] = pb;
        hipError_t le = hipMemcpyAsync(h->d_tviews, tv, 2 * sizeof(mf::DevGraph), hipMemcpyHostToDevice, h->stream);
        if (le == hipSuccess)
            le = hipMemcpyAsync(h->d_tparams, tp, 2 * sizeof(mf::LoopParams), hipMemcpyHostToDevice, h->stream);
        if (le == hipSuccess) le = mf::launch_teams(h->d_tviews, h->d_tparams, pa.walk != 0, h->d_work, h->grid, h->stream);
        if (le != hipSuccess) {
            (void)hipStreamSynchronize(h->stream);  // the staging is free again for the next call
            return hip_fail(h, le, "two-team launch");
        }
    } else {  // one workgroup (or a grid the two-team kernel cannot hold): one side after the other
        HIP_TRY(h, mf::launch_loop(ga, pa, h->grid, h->stream));
        HIP_TRY(h, mf::launch_loop(gb, pb, h->grid, h->stream));
    }
    HIP_TRY(h, hipMemcpyAsync(&h->h_vctrl[0], ga.ctrl, sizeof(mf::Ctrl), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipMemcpyAsync(&h->h_vctrl[1], gb.ctrl, sizeof(mf::Ctrl), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    seq_a += h->h_vctrl[0].rounds + 1;
    seq_b += h->h_vctrl[1].rounds + 1;
    for (int i = 0; i < 2; ++i) {
        const int32_t st = h->h_vctrl[i].status;
        if (st == mf::kSolved) continue;
        if (st == mf::kDeadline || st == mf::kIterLimit)
            return fail(h, MF_ETIMEOUT, "a side of the two-sided loop ran out of its time budget");
        return fail(h, MF_EDEVICE, "a side of the two-sided loop aborted (grid barrier wait ran out)");
    }
    return MF_OK;
}

// Dynamic Push-Pull (Sec. 4.2, Alg. 8) after the capacity changes of the
// batch landed (Alg. 5): S / T from the last heights; every residual arc from
// S to T saturated; then pulls into the deficient vertices of S (from s and
// the overflowing vertices of S, forward BFS of h_-, as pushes in the
// reversed view) side by side with pushes out of the overflowing vertices of
// T (to t and the deficient vertices of T, backward BFS of h_+); then the
// dynamic push-relabel loop on P, the vertices neither BFS reached.
int push_pull(mf_handle_t *h) {
    int rc = ensure_views(h);
    if (rc) return rc;
    rc = tag_parts(h);
    if (rc) return rc;
    HIP_TRY(h, mf::launch_saturate_cut(h->g, h->d_part, h->stream));
    HIP_TRY(h, mf::launch_view_make(h->g, h->rv.arc, h->rv.e, 1, h->stream));
    // S side, reversed: roots s (as the view's sink) and the overflowing
    // vertices of S (negative in the view); t is the view's never-entered end
    mf::DevGraph gs = h->rv;
    gs.s = h->g.t;
    gs.t = h->g.s;
    gs.part = h->d_part;
    gs.part_want = mf::kPartS;
    gs.part_restrict = 0;
    // T side, as it is: roots t and the deficient vertices of T
    mf::DevGraph gt = h->g;
    gt.part = h->d_part;
    gt.part_want = mf::kPartT;
    gt.part_restrict = 0;
    mf::LoopParams p = loop_params(h);
    p.policy_mode = mf::kPolicyFixed;
    p.policy_w = nullptr;
    p.policy_per_call = 0;
    HIP_TRY(h, hipEventRecord(h->ev[1], h->stream));
    rc = run_two_views(h, gs, p, h->vseq, gt, p, h->seq);
    if (rc) return rc;
    HIP_TRY(h, hipEventRecord(h->ev[2], h->stream));
    mf_stats_t first{};
    {
        mf_stats_t x{};
        mf::stats_from_ctrl(h->h_vctrl[0], h->tick_ms, &first);
        mf::stats_from_ctrl(h->h_vctrl[1], h->tick_ms, &x);
        add_stats(first, x);
        first.updates = h->h_ctrl->stat[mf::kStUpdates];  // booked by the repair kernels before the loops
        first.clamps = h->h_ctrl->stat[mf::kStClamps];
        float ms = 0.f;
        first.loop_launches = h->teams_fit ? 1 : 2;
        if (hipEventElapsedTime(&ms, h->ev[1], h->ev[2]) == hipSuccess) first.loop_kernel_ms = ms;
    }
    // the S side's vertices and arc pairs back into the handle's state
    HIP_TRY(h, mf::launch_view_merge(h->g, h->rv.arc, h->rv.e, h->d_part, mf::kPartS, 1, h->stream));
    // P: reached by neither BFS; the loop on P alone (roots: its deficient
    // vertices; the BFS enters only P and leaves every other height alone)
    HIP_TRY(h, mf::launch_part_localized(h->g, h->rv.h, h->d_part, h->stream));
    mf::DevGraph gp = h->g;
    gp.part = h->d_part;
    gp.part_want = mf::kPartP;
    gp.part_restrict = 1;
    HIP_TRY(h, mf::launch_reset_ctrl(h->g, h->stream));
    return run_loop_and_finish(h, &gp, &first);
}

// The debug check after a solving call that returned rc: the state's
// invariants, and once solved the cut's.  Returns rc, or MF_EDEVICE naming the
// first failed check.
int debug_check(mf_handle_t *h, int rc) {
    if (!h->debug_checks || (rc != MF_OK && rc != MF_ETIMEOUT)) return rc;
    const int solved = rc == MF_OK ? 1 : 0;
    HIP_TRY(h, mf::launch_check_state(h->g, solved, h->stream));
    int32_t f = 0;
    HIP_TRY(h, hipMemcpyAsync(&h->h_ctrl->check, &h->g.ctrl->check, sizeof(int32_t), hipMemcpyDeviceToHost,
                              h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    f = h->h_ctrl->check;
    if (!f) return rc;
    static const char *what[] = {"a negative residual", "an arc pair whose residuals do not sum to its capacities",
                                 "an excess that differs from its vertex's residual change",
                                 "an active vertex left after the loop",
                                 "a residual arc from the source side to the sink side"};
    for (int b = 0; b < 5; ++b)
        if (f & (1 << b)) return fail(h, MF_EDEVICE, std::string("debug check failed: ") + what[b]);
    return fail(h, MF_EDEVICE, "debug check failed");
}

// Dynamic repair and re-solve with batch arrays already on the device.
int apply_device(mf_handle_t *h, const int64_t *d_ids, const int32_t *d_caps, int64_t k) {
    if (h->state != State::Solved && h->state != State::Partial)
        return fail(h, MF_ESTATE, "mf_apply_updates needs a flow: call mf_solve first");
    if (k < 0 || k > h->g.m) return fail(h, MF_EINVAL, "batch size k must be in [0, m]");
    if (k > 0 && (!d_ids || !d_caps)) return fail(h, MF_EINVAL, "null batch arrays");
    int rc = next_epoch(h);
    if (rc) return rc;
    HIP_TRY(h, hipEventRecord(h->ev[0], h->stream));
    HIP_TRY(h, mf::launch_reset_ctrl(h->g, h->stream));
    HIP_TRY(h, mf::launch_validate_updates(h->g, d_ids, d_caps, k, h->epoch, h->cap_limit, h->stream));
    HIP_TRY(h, mf::launch_apply_delta(h->g, d_ids, d_caps, k, h->stream));
    HIP_TRY(h, mf::launch_clamp(h->g, d_ids, k, h->stream));
    h->batch_fraction = h->g.m > 0 ? (float)((double)k / (double)h->g.m) : 0.f;
    if (h->push_pull) {
        // the batch is checked before anything runs on the two sides
        HIP_TRY(h, hipMemcpyAsync(h->h_ctrl, h->g.ctrl, sizeof(mf::Ctrl), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        if (h->h_ctrl->err) return update_error_text(h, h->h_ctrl->err);
        h->state = State::Partial;
        rc = push_pull(h);
    } else {
        HIP_TRY(h, mf::launch_saturate_source(h->g, h->stream));
        // the local stage reads the cut of the last global relabel: only from
        // a solved state
        if (h->local_stage && h->state == State::Solved && k > 0) {
            if (h->ptag > INT32_MAX - 2 * (kPullRounds + 1)) {
                HIP_TRY(h, mf::launch_fill_i32(h->d_pmark, h->g.n, 0, h->stream));
                h->ptag = 0;
            }
            HIP_TRY(h, mf::launch_local_stage(h->g, d_ids, k, h->d_pmark, h->ptag + 1, kPullRounds, h->stream));
            h->ptag += kPullRounds + 1;
        }
        rc = run_loop_and_finish(h);
    }
    if (rc == MF_EINVAL) return update_error_text(h, h->h_ctrl->err);
    return debug_check(h, rc);
}

// caller_of_arc of a renumbered handle, computed on the device on first use.
int ensure_caller_order(mf_handle_t *h) {
    if (h->new_of_old.empty() || (int64_t)h->caller_of_arc.size() == (int64_t)h->g.A) return MF_OK;
    mf::BuildAlloc mem;
    mem.alloc = [h](void **q, size_t bytes) { return raw_alloc(h, q, bytes); };
    mem.release = [h](void *q) { raw_free(h, q); };
    mem.alloc_keep = mem.alloc;
    hipError_t e;
    try {
        e = mf::caller_arc_order(h->g.n, h->g.A, h->g.arc, h->g.twin, h->old_of_new, mem, h->stream,
                                 &h->caller_of_arc);
    } catch (const std::bad_alloc &) {
        h->caller_of_arc.clear();
        return fail(h, MF_ENOMEM, "host allocation failed while ordering the arcs");
    }
    if (e != hipSuccess) {
        h->caller_of_arc.clear();
        return fail(h, (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? MF_ENOMEM : MF_EDEVICE,
                    std::string("arc order of the caller's numbering: ") + hipGetErrorString(e));
    }
    return MF_OK;
}

bool opts_valid(const mf_opts_t &o, std::string *why) {
    if (o.kernel_cycles < 0) { *why = "kernel_cycles must be >= 0"; return false; }
    if (o.mode != MF_MODE_DATA && o.mode != MF_MODE_TOPOLOGY) { *why = "unknown mode"; return false; }
    if (o.grid_blocks < 0) { *why = "grid_blocks must be >= 0"; return false; }
    if (o.device < 0) { *why = "device must be >= 0"; return false; }
    if (o.time_budget_ms < 0) { *why = "time_budget_ms must be >= 0"; return false; }
    if (o.max_rounds < 0) { *why = "max_rounds must be >= 0"; return false; }
    if (o.relabel_budget < 0) { *why = "relabel_budget must be >= 0"; return false; }
    if (o.flags & ~(MF_FLAG_GAP | MF_FLAG_PUSH_PULL | MF_FLAG_DEBUG_CHECKS | MF_FLAG_SCAN_FIRST | MF_FLAG_GLOBAL_ONLY)) {
        *why = "unknown flags";
        return false;
    }
    if (!o.dev_alloc != !o.dev_free) { *why = "dev_alloc and dev_free go together"; return false; }
    if (o.vertex_order < MF_ORDER_AUTO || o.vertex_order > MF_ORDER_DEGREE) {
        *why = "unknown vertex_order";
        return false;
    }
    return true;
}

}  // namespace

extern "C" {

MF_API void mf_default_opts(mf_opts_t *opts) {
    if (!opts) return;
    std::memset(opts, 0, sizeof(*opts));
    opts->kernel_cycles = 0;
    opts->mode = MF_MODE_DATA;
    opts->grid_blocks = 0;
    opts->device = 0;
    opts->max_iterations = -1;
}

MF_API const char *mf_last_error(const mf_handle_t *h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

MF_API int mf_create(const mf_csr_t *g, const int32_t *cap, int32_t s, int32_t t, const mf_opts_t *opts,
                     mf_handle_t **out) {
    if (!out) return fail(nullptr, MF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g || !cap || !g->row_ptr || (g->m > 0 && !g->col))
        return fail(nullptr, MF_EINVAL, "null graph or capacity array");
    const int32_t n = g->n;
    const int64_t m = g->m;
    std::string why;
    if (mf::check_graph(n, m, g->row_ptr, g->col, cap, s, t, &why)) return fail(nullptr, MF_EINVAL, why);
    mf_opts_t o;
    mf_default_opts(&o);
    if (opts) o = *opts;
    if (!opts_valid(o, &why)) return fail(nullptr, MF_EINVAL, why);
    // the per-edge capacity limit falls with the edges merged into one pair:
    // a capacity above the limit of an unshared pair is refused at once (the
    // exact limit is checked after the build)
    {
        const int64_t lim1 = mf::edge_cap_limit(1);
        for (int64_t i = 0; i < m; ++i)
            if (cap[i] > lim1)
                return fail(nullptr, MF_EINVAL, "capacity above the per-edge limit " + std::to_string(lim1));
    }

    mf_handle_t *h = new (std::nothrow) mf_handle_t();
    if (!h) return fail(nullptr, MF_ENOMEM, "host allocation failed");
    h->device = o.device;
    h->alloc_fn = o.dev_alloc;
    h->free_fn = o.dev_free;
    h->alloc_ctx = o.alloc_ctx;
    h->debug_checks = (o.flags & MF_FLAG_DEBUG_CHECKS) ? 1 : 0;
    h->mode = o.mode;
    h->max_iter = o.max_iterations;
    const int64_t budget_ms = o.time_budget_ms > 0 ? o.time_budget_ms : 60000;
    h->max_rounds = o.max_rounds > 0 ? o.max_rounds : 65536;
    h->relabel_budget = o.relabel_budget > 0 ? o.relabel_budget : std::max<int64_t>(1024, n / 16);
    h->rounds_per_level = o.rounds_per_level == 0 ? 1 : (o.rounds_per_level < 0 ? 0 : o.rounds_per_level);
    h->use_gap = (o.flags & MF_FLAG_GAP) ? 1 : 0;
    h->push_pull = (o.flags & MF_FLAG_PUSH_PULL) ? 1 : 0;
    h->walk = (o.flags & MF_FLAG_SCAN_FIRST) ? 0 : 1;
    h->local_stage = (o.flags & MF_FLAG_GLOBAL_ONLY) ? 0 : 1;
    h->stall_rounds = o.stall_rounds == 0 ? 3 : (o.stall_rounds < 0 ? 0 : o.stall_rounds);
    h->solo_items = o.solo_items == 0 ? kSoloItems : (o.solo_items < 0 ? 0 : o.solo_items);
    h->lazy_items = o.lazy_items == 0 ? kLazyItems : (o.lazy_items < 0 ? INT32_MAX : o.lazy_items);
    // one cycle per visit: rounds re-queue a vertex that keeps excess, so
    // further cycles in one visit mostly repeat what the next round does
    h->kc = o.kernel_cycles > 0 ? o.kernel_cycles : 1;
    auto bail = [&](int code, const std::string &msg) {
        release(h);
        delete h;
        return fail(nullptr, code, msg);
    };
    hipError_t e = hipSetDevice(o.device);
    if (e != hipSuccess) return bail(MF_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    // device address of this GPU's staging array for mf_apply_updates_noalloc
    if ((e = mf::noalloc_scratch_setup(o.device)) != hipSuccess)
        return bail(MF_EDEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    if ((e = hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(MF_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    h->stream = h->own_stream;
    for (auto &ev : h->ev)
        if ((e = hipEventCreate(&ev)) != hipSuccess)
            return bail(MF_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
    if ((e = hipHostMalloc((void **)&h->h_ctrl, sizeof(mf::Ctrl), hipHostMallocDefault)) != hipSuccess)
        return bail(MF_ENOMEM, "pinned control block");

    // a0: the merged arc-pair layout, built on the device (mf_build.hip); the
    // arc row pointers come back for the host-side lists below
    mf::DevGraph &d = h->g;
    std::vector<int32_t> hrow;
    {
        mf::BuildAlloc mem;
        mem.alloc = [h](void **q, size_t bytes) { return raw_alloc(h, q, bytes); };
        mem.release = [h](void *q) { raw_free(h, q); };
        mem.alloc_keep = [h](void **q, size_t bytes) {
            hipError_t e = raw_alloc(h, q, bytes);
            if (e == hipSuccess) h->allocs.push_back(*q);
            return e;
        };
        mf::DeviceLayout lay;
        std::string berr;
        const bool renumber = o.vertex_order == MF_ORDER_DEGREE || (o.vertex_order == MF_ORDER_AUTO && n > 8192);
        try {
            e = mf::build_layout_device(n, m, g->row_ptr, g->col, cap, renumber, mem, h->stream, &lay, &hrow,
                                        &h->new_of_old, &berr);
            if (e == hipSuccess && !h->new_of_old.empty()) {
                h->old_of_new.assign((size_t)n, 0);
                for (int32_t v = 0; v < n; ++v) h->old_of_new[h->new_of_old[v]] = v;
            }
        } catch (const std::bad_alloc &) {
            return bail(MF_ENOMEM, "host allocation failed while building arc pairs");
        }
        if (e == hipErrorInvalidValue) return bail(MF_EINVAL, berr);
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
            return bail(MF_ENOMEM, "device allocation failed while building arc pairs: " + berr);
        if (e != hipSuccess) return bail(MF_EDEVICE, "arc-pair build: " + berr);
        // per-edge capacity limit: after the deltas of one batch land, an arc's
        // residual is at most twice the pair's capacity sum, which must fit int32
        const int64_t lim = mf::edge_cap_limit(lay.max_pair_mult);
        for (int64_t i = 0; i < m; ++i)
            if (cap[i] > lim) return bail(MF_EINVAL, "capacity above the per-edge limit " + std::to_string(lim));
        h->cap_limit = (int32_t)lim;
        d.A = lay.A;
        d.row_ptr = lay.row_ptr;
        d.arc = lay.arc;
        d.twin = lay.twin;
        d.cap = lay.cap;
        d.edge2arc = lay.edge2arc;
        d.ecap = lay.ecap;
    }
    // s and t in the layout's numbering
    if (!h->new_of_old.empty()) {
        s = h->new_of_old[s];
        t = h->new_of_old[t];
    }
    // heavy vertices (arc lists handled by a wavefront in topology-driven sweeps)
    std::vector<int32_t> heavy;
    int64_t nhuge = 0;  // vertices visited by a whole workgroup
    for (int32_t v = 0; v < n; ++v) {
        const int32_t deg = hrow[v + 1] - hrow[v];
        if (v != s && v != t && deg > mf::kLightMaxDeg) heavy.push_back(v);
        if (v != s && v != t && deg > mf::kHugeDeg) nhuge++;
    }
    // vertices of huge degree draw pushes from many others at once: add them
    // up per workgroup first
    h->combine = nhuge > 0 ? 1 : 0;
    h->nhuge = nhuge;

    d.n = n;
    d.s = s;
    d.t = t;
    d.m = m;
    d.qcap = (int64_t)n + d.A / mf::kChunk + 64;
    d.n_heavy_all = (int32_t)heavy.size();
    const int64_t A = d.A;
#define ALLOC(ptr, count)                                                             \
    do {                                                                              \
        if ((e = dev_alloc(h, &(ptr), (count))) != hipSuccess)                        \
            return bail(MF_ENOMEM, std::string("hipMalloc " #ptr ": ") + hipGetErrorString(e)); \
    } while (0)
    ALLOC(d.stamp, m);
    ALLOC(d.e, n);
    ALLOC(d.h, n);
    ALLOC(d.q[0], d.qcap);
    ALLOC(d.q[1], d.qcap);
    ALLOC(d.list[0], n);
    ALLOC(d.list[1], n);
    ALLOC(d.list[2], n);
    ALLOC(d.huge[0], nhuge);
    ALLOC(d.huge[1], nhuge);
    ALLOC(d.huge[2], nhuge);
    ALLOC(d.mark, n);
    ALLOC(d.rmark, n);
    ALLOC(d.relab, n);
    ALLOC(d.hcount, (int64_t)n + 1);
    ALLOC(d.heavy_all, (int64_t)heavy.size());
    ALLOC(d.ctrl, 1);
    ALLOC(h->d_side, n);
    ALLOC(h->d_pmark, n);
#undef ALLOC
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream) : hipSuccess;
    };
    if ((e = up(d.heavy_all, heavy.data(), sizeof(int32_t) * heavy.size())) != hipSuccess)
        return bail(MF_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    if ((e = mf::launch_fill_i32(d.stamp, m, 0, h->stream)) != hipSuccess ||
        (e = mf::launch_fill_i32(d.mark, n, 0, h->stream)) != hipSuccess ||
        (e = mf::launch_fill_i32(d.rmark, n, 0, h->stream)) != hipSuccess ||
        (e = mf::launch_fill_i32(h->d_pmark, n, 0, h->stream)) != hipSuccess ||

        (e = mf::launch_reset_ctrl(d, h->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(h->stream)) != hipSuccess)
        return bail(MF_EDEVICE, std::string("init: ") + hipGetErrorString(e));

    int clock_khz = 0;
    if ((e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, o.device)) != hipSuccess ||
        clock_khz <= 0)
        clock_khz = 100000;
    h->deadline_ticks = budget_ms * (int64_t)clock_khz;
    h->tick_ms = 1.0 / clock_khz;
    h->barrier_ticks = 10000 * (int64_t)clock_khz;  // 10 s
    // workgroups of the persistent kernel
    int maxb = 0;
    if ((e = mf::loop_max_coresident(o.device, &maxb)) != hipSuccess)
        return bail(MF_EDEVICE, std::string("occupancy query: ") + hipGetErrorString(e));
    // one workgroup for small graphs (no grid barrier at all); otherwise about
    // one 1024-thread workgroup per 64K arcs, at most one per compute unit:
    // a grid barrier costs roughly 60 ns per participating workgroup
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, o.device);
    int grid = o.grid_blocks;
    if (grid == 0) {
        if ((int64_t)n <= 8192 && A <= (1 << 17)) grid = 1;
        else grid = (int)std::min<int64_t>(std::min(maxb, std::max(cus, 1)),
                                           std::max<int64_t>(8, (A + 65535) / 65536));
    }
    if (grid > 1 && grid > maxb)
        return bail(MF_EINVAL, "grid_blocks above the co-resident limit " + std::to_string(maxb));
    h->grid = grid;
    // items of the bottom-up BFS levels (several workgroups only): the first
    // item of every vertex in vertex order, then the further items of long
    // lists, all second items first, so that one wavefront's 64 items come
    // from many vertices
    if (grid > 1 && o.bottom_up >= 0) {
        std::vector<int4> items;
        try {
            items.reserve((size_t)n + (size_t)(A / mf::kChunk) + 1);
            std::vector<int32_t> longv;  // vertices with items left after the k-th
            for (int32_t v = 0; v < n; ++v) {
                const int32_t b = hrow[v], en = hrow[v + 1];
                if (en > b) items.push_back(make_int4(v, b, std::min(en, b + mf::kChunk), 0));
                if (en - b > mf::kChunk) longv.push_back(v);
            }
            for (int32_t k = 1; !longv.empty(); ++k) {
                size_t keep = 0;
                for (const int32_t v : longv) {
                    const int32_t b = hrow[v] + k * mf::kChunk, en = hrow[v + 1];
                    items.push_back(make_int4(v, b, std::min(en, b + mf::kChunk), 0));
                    if (en - b > mf::kChunk) longv[keep++] = v;
                }
                longv.resize(keep);
            }
        } catch (const std::bad_alloc &) {
            return bail(MF_ENOMEM, "host allocation failed while building the bottom-up items");
        }
        int4 *bi = nullptr;
        if ((e = dev_alloc(h, &bi, (int64_t)items.size())) != hipSuccess)
            return bail(MF_ENOMEM, std::string("hipMalloc bu_items: ") + hipGetErrorString(e));
        if ((e = up(bi, items.data(), sizeof(int4) * items.size())) != hipSuccess ||
            (e = hipStreamSynchronize(h->stream)) != hipSuccess)
            return bail(MF_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
        d.bu_items = bi;
        d.n_bu_items = (int32_t)items.size();
        h->bu_alpha = o.bottom_up == 0 ? kBuAlpha : o.bottom_up;
    }
    if (h->push_pull) {
        // the second view up front: push-pull updates then allocate nothing
        const int rc = ensure_views(h);
        if (rc) {
            const std::string why = h->err;
            return bail(rc, why);
        }
    }
    *out = h;
    return MF_OK;
}

MF_API void mf_destroy(mf_handle_t *h) {
    if (!h) return;
    release(h);
    delete h;
}

MF_API int mf_solve(mf_handle_t *h) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, hipEventRecord(h->ev[0], h->stream));
    HIP_TRY(h, mf::launch_reset_ctrl(h->g, h->stream));
    HIP_TRY(h, mf::launch_init_state(h->g, h->stream));
    HIP_TRY(h, mf::launch_saturate_source(h->g, h->stream));
    h->state = State::Partial;
    h->batch_fraction = 1.f;
    return debug_check(h, run_loop_and_finish(h));
}

MF_API int mf_resume(mf_handle_t *h) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    if (h->state == State::NoFlow || h->state == State::NeedsSolve)
        return fail(h, MF_ESTATE, "no flow to resume: call mf_solve");
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, hipEventRecord(h->ev[0], h->stream));
    HIP_TRY(h, mf::launch_reset_ctrl(h->g, h->stream));
    return debug_check(h, run_loop_and_finish(h));
}

MF_API int mf_apply_updates(mf_handle_t *h, const int64_t *edge_ids, const int32_t *new_caps, int64_t k) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    if (h->state != State::Solved && h->state != State::Partial)
        return fail(h, MF_ESTATE, "mf_apply_updates needs a flow: call mf_solve first");
    if (k < 0 || k > h->g.m) return fail(h, MF_EINVAL, "batch size k must be in [0, m]");
    if (k > 0 && (!edge_ids || !new_caps)) return fail(h, MF_EINVAL, "null batch arrays");
    HIP_TRY(h, hipSetDevice(h->device));
    int rc = stage_host_batch(h, edge_ids, new_caps, k);
    if (rc) return rc;
    return apply_device(h, h->d_ids, h->d_caps, k);
}

MF_API int mf_apply_updates_device(mf_handle_t *h, const int64_t *d_edge_ids, const int32_t *d_new_caps,
                                   int64_t k) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    HIP_TRY(h, hipSetDevice(h->device));
    return apply_device(h, d_edge_ids, d_new_caps, k);
}

MF_API int mf_apply_updates_noalloc(mf_handle_t *h, const int64_t *edge_ids, const int32_t *new_caps, int64_t k) {
    static_assert(MF_NOALLOC_MAX_UPDATES == mf::kNoAllocMaxUpdates, "staging size");
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    if (k < 0 || k > h->g.m) return fail(h, MF_EINVAL, "batch size k must be in [0, m]");
    if (k > mf::kNoAllocMaxUpdates)
        return fail(h, MF_EINVAL, "mf_apply_updates_noalloc takes at most " +
                                      std::to_string(mf::kNoAllocMaxUpdates) + " updates per call");
    if (k > 0 && (!edge_ids || !new_caps)) return fail(h, MF_EINVAL, "null batch arrays");
    HIP_TRY(h, hipSetDevice(h->device));
    uint8_t *base = static_cast<uint8_t *>(mf::noalloc_scratch(h->device));
    if (!base) return fail(h, MF_ESTATE, "the device's staging array was not set up");
    int64_t *d_ids = reinterpret_cast<int64_t *>(base);
    int32_t *d_caps = reinterpret_cast<int32_t *>(base + mf::kNoAllocIdsBytes);
    if (k > 0) {
        HIP_TRY(h, hipMemcpyAsync(d_ids, edge_ids, sizeof(int64_t) * k, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, hipMemcpyAsync(d_caps, new_caps, sizeof(int32_t) * k, hipMemcpyHostToDevice, h->stream));
    }
    const int rc = apply_device(h, d_ids, d_caps, k);
    // the caller's arrays and the staging are free again once this returns
    if (rc) (void)hipStreamSynchronize(h->stream);
    return rc;
}

MF_API int mf_set_capacities(mf_handle_t *h, const int64_t *edge_ids, const int32_t *new_caps, int64_t k) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    if (k < 0 || k > h->g.m) return fail(h, MF_EINVAL, "batch size k must be in [0, m]");
    if (k > 0 && (!edge_ids || !new_caps)) return fail(h, MF_EINVAL, "null batch arrays");
    HIP_TRY(h, hipSetDevice(h->device));
    int rc = stage_host_batch(h, edge_ids, new_caps, k);
    if (rc) return rc;
    rc = next_epoch(h);
    if (rc) return rc;
    HIP_TRY(h, hipEventRecord(h->ev[0], h->stream));
    HIP_TRY(h, mf::launch_reset_ctrl(h->g, h->stream));
    HIP_TRY(h, mf::launch_validate_updates(h->g, h->d_ids, h->d_caps, k, h->epoch, h->cap_limit, h->stream));
    HIP_TRY(h, mf::launch_apply_delta(h->g, h->d_ids, h->d_caps, k, h->stream));
    rc = finish_call(h);
    if (rc) return rc;
    if (h->h_ctrl->err) return update_error_text(h, h->h_ctrl->err);
    h->state = State::NeedsSolve;
    return MF_OK;
}

MF_API int mf_edge_flow(mf_handle_t *h, int32_t *flow_out) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    if (!flow_out && h->g.m > 0) return fail(h, MF_EINVAL, "null flow array");
    if (h->state != State::Solved) return fail(h, MF_ESTATE, "not solved");
    HIP_TRY(h, hipSetDevice(h->device));
    int rc = ensure_views(h);
    if (rc) return rc;
    // S / T: the canonical cut of the final global relabel
    rc = tag_parts(h);
    if (rc) return rc;
    HIP_TRY(h, mf::launch_view_make(h->g, h->fv.arc, h->fv.e, 0, h->stream));
    HIP_TRY(h, mf::launch_view_make(h->g, h->rv.arc, h->rv.e, 1, h->stream));
    // S side on a copy, s and t exchanged: its overflowing vertices push their
    // excess back to s (the copy's sink).  T side reversed: its deficient
    // vertices, overflowing in the view, push toward t, i.e. t sends them
    // flow.  Both sides run without RemoveInvalidEdges, so no deficit arises.
    mf::DevGraph gs = h->fv;
    gs.s = h->g.t;
    gs.t = h->g.s;
    gs.part = h->d_part;
    gs.part_want = mf::kPartS;
    gs.part_restrict = 0;
    mf::DevGraph gt = h->rv;
    gt.part = h->d_part;
    gt.part_want = mf::kPartT;
    gt.part_restrict = 0;
    mf::LoopParams p = loop_params(h);
    p.no_rie = 1;
    p.use_gap = 0;
    p.max_iter = -1;
    p.relabel_budget = INT64_MAX / 4;
    p.policy_mode = mf::kPolicyFixed;
    p.policy_w = nullptr;
    p.policy_per_call = 0;
    p.batch_fraction = 0.f;
    rc = run_two_views(h, gs, p, h->seq, gt, p, h->vseq);
    if (rc) return rc;
    // the T side's arcs and excesses into the copy, then the per-edge split
    HIP_TRY(h, mf::launch_view_merge(h->fv, h->rv.arc, h->rv.e, h->d_part, mf::kPartT, 1, h->stream));
    HIP_TRY(h, mf::launch_edge_flow(h->g, h->fv.arc, h->d_rem, h->d_eflow, h->stream));
    if (h->g.m > 0)
        HIP_TRY(h, hipMemcpyAsync(flow_out, h->d_eflow, sizeof(int32_t) * h->g.m, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return MF_OK;
}

MF_API int mf_flow_value(const mf_handle_t *h, int64_t *out) {
    if (!h || !out) return fail(const_cast<mf_handle_t *>(h), MF_EINVAL, "null argument");
    if (h->state != State::Solved)
        return fail(const_cast<mf_handle_t *>(h), MF_ESTATE, "not solved");
    *out = h->value;
    return MF_OK;
}

MF_API int mf_min_cut(mf_handle_t *h, uint8_t *side_out, int64_t *cut_cap_out) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    if (h->state != State::Solved) return fail(h, MF_ESTATE, "not solved");
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, mf::launch_fill_i32(reinterpret_cast<int32_t *>(&h->g.ctrl->cut), 2, 0, h->stream));
    HIP_TRY(h, mf::launch_min_cut(h->g, h->d_side, h->stream));
    const bool renum = !h->new_of_old.empty();
    std::vector<uint8_t> side;
    if (side_out) {
        if (renum) side.resize((size_t)h->g.n);
        HIP_TRY(h, hipMemcpyAsync(renum ? side.data() : side_out, h->d_side, (size_t)h->g.n, hipMemcpyDeviceToHost,
                                  h->stream));
    }
    int64_t cut = 0;
    HIP_TRY(h, hipMemcpyAsync(&cut, &h->g.ctrl->cut, sizeof(int64_t), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (side_out && renum)
        for (int32_t v = 0; v < h->g.n; ++v) side_out[v] = side[h->new_of_old[v]];
    if (cut_cap_out) *cut_cap_out = cut;
    return MF_OK;
}

MF_API int mf_set_max_iterations(mf_handle_t *h, int64_t limit) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    h->max_iter = limit < 0 ? -1 : limit;
    return MF_OK;
}

MF_API int mf_get_stats(const mf_handle_t *h, mf_stats_t *out) {
    if (!h || !out) return fail(const_cast<mf_handle_t *>(h), MF_EINVAL, "null argument");
    *out = h->stats;
    return MF_OK;
}

MF_API int64_t mf_estimate_device_bytes(int32_t n, int64_t m) {
    if (n < 0 || m < 0) return -1;
    const int64_t A = 2 * m;  // upper bound before merging
    const int64_t qcap = (int64_t)n + A / mf::kChunk + 64;
    int64_t b = 0;
    b += 4 * ((int64_t)n + 1);            // row_ptr
    b += (8 + 4 + 4) * A;                 // arc, twin, cap
    b += (4 + 4 + 4) * m;                 // edge2arc, ecap, stamp
    b += (8 + 4) * (int64_t)n;            // e, h
    b += 2 * 8 * qcap;                    // frontier items
    b += (3 + 3) * 4 * (int64_t)n;        // lists, mark, rmark, relab
    b += 3 * 4 * (A / mf::kHugeDeg + 1);  // huge-vertex lists
    b += 4 * ((int64_t)n + 1);            // hcount
    b += 4 * (int64_t)n;                  // heavy vertices (at most n)
    b += (int64_t)n;                      // cut side
    b += (int64_t)sizeof(mf::Ctrl);
    b += 256 * 24;                        // allocation rounding of the ~24 arrays
    return b;
}

MF_API int mf_num_arcs(const mf_handle_t *h, int32_t *A_out) {
    if (!h || !A_out) return fail(const_cast<mf_handle_t *>(h), MF_EINVAL, "null argument");
    *A_out = h->g.A;
    return MF_OK;
}

MF_API int mf_cap_limit(const mf_handle_t *h, int32_t *limit_out) {
    if (!h || !limit_out) return fail(const_cast<mf_handle_t *>(h), MF_EINVAL, "null argument");
    *limit_out = h->cap_limit;
    return MF_OK;
}

MF_API int mf_export_graph(mf_handle_t *h, int32_t *row_ptr, int32_t *col, int32_t *twin, int32_t *edge2arc) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    HIP_TRY(h, hipSetDevice(h->device));
    const mf::DevGraph &d = h->g;
    if (!h->new_of_old.empty()) {
        // the layout of the caller's numbering: arc a of the handle is arc
        // pos[a] there, the caller's vertex v is the handle's nw[v]
        const int rc = ensure_caller_order(h);
        if (rc) return rc;
        const std::vector<int32_t> &pos = h->caller_of_arc, &nw = h->new_of_old, &old = h->old_of_new;
        std::vector<int32_t> rp((size_t)d.n + 1), tw((size_t)d.A), e2a((size_t)d.m);
        std::vector<int2> arc((size_t)d.A);
        HIP_TRY(h, hipMemcpyAsync(rp.data(), d.row_ptr, sizeof(int32_t) * (d.n + 1), hipMemcpyDeviceToHost, h->stream));
        if (d.A) {
            HIP_TRY(h, hipMemcpyAsync(arc.data(), d.arc, sizeof(int2) * d.A, hipMemcpyDeviceToHost, h->stream));
            HIP_TRY(h, hipMemcpyAsync(tw.data(), d.twin, sizeof(int32_t) * d.A, hipMemcpyDeviceToHost, h->stream));
        }
        if (d.m)
            HIP_TRY(h, hipMemcpyAsync(e2a.data(), d.edge2arc, sizeof(int32_t) * d.m, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        if (row_ptr) {
            row_ptr[0] = 0;
            for (int32_t v = 0; v < d.n; ++v) row_ptr[v + 1] = row_ptr[v] + (rp[nw[v] + 1] - rp[nw[v]]);
        }
        for (int64_t a = 0; a < d.A; ++a) {
            if (col) col[pos[a]] = old[arc[a].x];
            if (twin) twin[pos[a]] = pos[tw[a]];
        }
        if (edge2arc)
            for (int64_t i = 0; i < d.m; ++i) edge2arc[i] = e2a[i] < 0 ? -1 : pos[e2a[i]];
        return MF_OK;
    }
    if (row_ptr)
        HIP_TRY(h, hipMemcpyAsync(row_ptr, d.row_ptr, sizeof(int32_t) * (d.n + 1), hipMemcpyDeviceToHost, h->stream));
    if (col && d.A) {
        std::vector<int2> arc((size_t)d.A);
        HIP_TRY(h, hipMemcpyAsync(arc.data(), d.arc, sizeof(int2) * d.A, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        for (int64_t a = 0; a < d.A; ++a) col[a] = arc[a].x;
    }
    if (twin && d.A)
        HIP_TRY(h, hipMemcpyAsync(twin, d.twin, sizeof(int32_t) * d.A, hipMemcpyDeviceToHost, h->stream));
    if (edge2arc && d.m)
        HIP_TRY(h, hipMemcpyAsync(edge2arc, d.edge2arc, sizeof(int32_t) * d.m, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return MF_OK;
}

MF_API int mf_export_state(mf_handle_t *h, int32_t *cap, int32_t *cf, int64_t *e, int32_t *height, int32_t *ecap) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    HIP_TRY(h, hipSetDevice(h->device));
    const mf::DevGraph &d = h->g;
    if (!h->new_of_old.empty()) {
        // per-arc and per-vertex arrays in the caller's numbering
        const int rc = ensure_caller_order(h);
        if (rc) return rc;
        const std::vector<int32_t> &pos = h->caller_of_arc, &nw = h->new_of_old;
        std::vector<int2> arc(cf ? (size_t)d.A : 0);
        std::vector<int32_t> capi(cap ? (size_t)d.A : 0), hi(height ? (size_t)d.n : 0);
        std::vector<int64_t> ei(e ? (size_t)d.n : 0);
        if (cap && d.A)
            HIP_TRY(h, hipMemcpyAsync(capi.data(), d.cap, sizeof(int32_t) * d.A, hipMemcpyDeviceToHost, h->stream));
        if (cf && d.A)
            HIP_TRY(h, hipMemcpyAsync(arc.data(), d.arc, sizeof(int2) * d.A, hipMemcpyDeviceToHost, h->stream));
        if (e) HIP_TRY(h, hipMemcpyAsync(ei.data(), d.e, sizeof(int64_t) * d.n, hipMemcpyDeviceToHost, h->stream));
        if (height)
            HIP_TRY(h, hipMemcpyAsync(hi.data(), d.h, sizeof(int32_t) * d.n, hipMemcpyDeviceToHost, h->stream));
        if (ecap && d.m)
            HIP_TRY(h, hipMemcpyAsync(ecap, d.ecap, sizeof(int32_t) * d.m, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        for (int64_t a = 0; a < d.A; ++a) {
            if (cap) cap[pos[a]] = capi[a];
            if (cf) cf[pos[a]] = arc[a].y;
        }
        for (int32_t v = 0; v < d.n; ++v) {
            if (e) e[v] = ei[nw[v]];
            if (height) height[v] = hi[nw[v]];
        }
        return MF_OK;
    }
    if (cap && d.A)
        HIP_TRY(h, hipMemcpyAsync(cap, d.cap, sizeof(int32_t) * d.A, hipMemcpyDeviceToHost, h->stream));
    if (cf && d.A) {
        std::vector<int2> arc((size_t)d.A);
        HIP_TRY(h, hipMemcpyAsync(arc.data(), d.arc, sizeof(int2) * d.A, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        for (int64_t a = 0; a < d.A; ++a) cf[a] = arc[a].y;
    }
    if (e) HIP_TRY(h, hipMemcpyAsync(e, d.e, sizeof(int64_t) * d.n, hipMemcpyDeviceToHost, h->stream));
    if (height) HIP_TRY(h, hipMemcpyAsync(height, d.h, sizeof(int32_t) * d.n, hipMemcpyDeviceToHost, h->stream));
    if (ecap && d.m)
        HIP_TRY(h, hipMemcpyAsync(ecap, d.ecap, sizeof(int32_t) * d.m, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return MF_OK;
}

MF_API int mf_import_state(mf_handle_t *h, const int32_t *cap, const int32_t *cf, const int64_t *e,
                           const int32_t *ecap) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    if (!e || (h->g.A && (!cap || !cf)) || (h->g.m && !ecap)) return fail(h, MF_EINVAL, "null state arrays");
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const mf::DevGraph &d = h->g;
    // a renumbered handle takes the caller's arrays into its own numbering
    std::vector<int32_t> cap_in, cf_in;
    std::vector<int64_t> e_in;
    if (!h->new_of_old.empty()) {
        const int rc = ensure_caller_order(h);
        if (rc) return rc;
        const std::vector<int32_t> &pos = h->caller_of_arc, &nw = h->new_of_old;
        cap_in.resize((size_t)d.A);
        cf_in.resize((size_t)d.A);
        e_in.resize((size_t)d.n);
        for (int64_t a = 0; a < d.A; ++a) {
            cap_in[a] = cap[pos[a]];
            cf_in[a] = cf[pos[a]];
        }
        for (int32_t v = 0; v < d.n; ++v) e_in[nw[v]] = e[v];
        cap = cap_in.data();
        cf = cf_in.data();
        e = e_in.data();
    }
    std::vector<int2> arc((size_t)d.A);
    std::vector<int32_t> twin((size_t)d.A), e2a((size_t)d.m), rp((size_t)d.n + 1);
    if (d.A) {
        HIP_TRY(h, hipMemcpy(arc.data(), d.arc, sizeof(int2) * d.A, hipMemcpyDeviceToHost));
        HIP_TRY(h, hipMemcpy(twin.data(), d.twin, sizeof(int32_t) * d.A, hipMemcpyDeviceToHost));
    }
    if (d.m) HIP_TRY(h, hipMemcpy(e2a.data(), d.edge2arc, sizeof(int32_t) * d.m, hipMemcpyDeviceToHost));
    HIP_TRY(h, hipMemcpy(rp.data(), d.row_ptr, sizeof(int32_t) * (d.n + 1), hipMemcpyDeviceToHost));
    for (int64_t a = 0; a < d.A; ++a) {
        if (cap[a] < 0 || cf[a] < 0) return fail(h, MF_EINVAL, "negative capacity or residual");
        const int64_t b = twin[a];
        if ((int64_t)cf[a] + cf[b] != (int64_t)cap[a] + cap[b])
            return fail(h, MF_EINVAL, "residuals of an arc pair do not sum to its capacities");
    }
    // arc capacities are the sums of their edges' capacities
    std::vector<int64_t> capsum((size_t)d.A, 0);
    for (int64_t i = 0; i < d.m; ++i) {
        if (ecap[i] < 0 || ecap[i] > h->cap_limit) return fail(h, MF_EINVAL, "edge capacity out of range");
        if (e2a[i] >= 0) capsum[e2a[i]] += ecap[i];
    }
    for (int64_t a = 0; a < d.A; ++a)
        if (capsum[a] != cap[a]) return fail(h, MF_EINVAL, "arc capacities disagree with the edge capacities");
    // every excess is the vertex's residual change: sum over its arcs of c_f - c
    for (int32_t u = 0; u < d.n; ++u) {
        int64_t x = 0;
        for (int32_t a = rp[u]; a < rp[u + 1]; ++a) x += (int64_t)cf[a] - cap[a];
        if (x != e[u]) return fail(h, MF_EINVAL, "excesses disagree with the residuals");
    }
    for (int64_t a = 0; a < d.A; ++a) arc[a].y = cf[a];
    if (d.A) {
        HIP_TRY(h, hipMemcpy(d.arc, arc.data(), sizeof(int2) * d.A, hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(d.cap, cap, sizeof(int32_t) * d.A, hipMemcpyHostToDevice));
    }
    HIP_TRY(h, hipMemcpy(d.e, e, sizeof(int64_t) * d.n, hipMemcpyHostToDevice));
    if (d.m) HIP_TRY(h, hipMemcpy(d.ecap, ecap, sizeof(int32_t) * d.m, hipMemcpyHostToDevice));
    h->state = State::Partial;
    return MF_OK;
}

MF_API int mf_get_trace(const mf_handle_t *h, int32_t *out, int32_t max_phases, int32_t *n_out) {
    if (!h || (max_phases > 0 && !out) || max_phases < 0)
        return fail(const_cast<mf_handle_t *>(h), MF_EINVAL, "bad trace arguments");
    const mf::Ctrl &c = *h->h_ctrl;
    const int32_t nrec = std::min<int32_t>(c.ntrace, mf::kTraceCap);
    const int32_t k = std::min(nrec, max_phases);
    if (k > 0) std::memcpy(out, c.trace, sizeof(int32_t) * mf::kTraceFields * k);
    if (n_out) *n_out = nrec;
    return MF_OK;
}

MF_API int mf_set_policy(mf_handle_t *h, const mf_policy_t *policy, int32_t mode, float margin, float explore,
                         uint64_t seed, int32_t action) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    const int32_t per_call = (mode & MF_POLICY_PER_CALL) ? 1 : 0;
    mode &= ~MF_POLICY_PER_CALL;
    if (mode < MF_POLICY_FIXED || mode > MF_POLICY_FORCED) return fail(h, MF_EINVAL, "unknown policy mode");
    if (mode == MF_POLICY_LEARNED && !policy) return fail(h, MF_EINVAL, "the learned mode needs a policy");
    if (policy && mf::policy_device(policy) != h->device)
        return fail(h, MF_EINVAL, "the policy lives on another device");
    if (!(margin >= 0.f) || !(explore >= 0.f && explore <= 1.f))
        return fail(h, MF_EINVAL, "margin must be >= 0 and explore in [0, 1]");
    if (mode == MF_POLICY_FORCED && (action < 0 || action >= MF_POLICY_ACTIONS))
        return fail(h, MF_EINVAL, "action out of range");
    if (mode != MF_POLICY_FIXED && !h->d_ptrace) {
        HIP_TRY(h, hipSetDevice(h->device));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        void *q = nullptr;
        if (raw_alloc(h, &q, sizeof(float) * mf::kTraceCap * mf::kPolRec) != hipSuccess)
            return fail(h, MF_ENOMEM, "cannot allocate the policy trace");
        h->d_ptrace = static_cast<float *>(q);
        h->g.ptrace = h->d_ptrace;
    }
    h->policy = policy;
    h->policy_mode = mode;
    h->policy_margin = margin;
    h->policy_explore = explore;
    h->policy_seed = seed;
    h->policy_action = action;
    h->policy_per_call = mode == MF_POLICY_FIXED ? 0 : per_call;
    return MF_OK;
}

MF_API int mf_get_policy_trace(mf_handle_t *h, float *out, int32_t max_phases, int32_t *n_out) {
    if (!h || (max_phases > 0 && !out) || max_phases < 0) return fail(h, MF_EINVAL, "bad trace arguments");
    const int32_t nrec = h->d_ptrace && h->policy_mode != MF_POLICY_FIXED
                             ? std::min<int32_t>(h->h_ctrl->ntrace, mf::kTraceCap)
                             : 0;
    const int32_t k = std::min(nrec, max_phases);
    if (k > 0) {
        HIP_TRY(h, hipSetDevice(h->device));
        HIP_TRY(h, hipMemcpyAsync(out, h->d_ptrace, sizeof(float) * mf::kPolRec * k, hipMemcpyDeviceToHost,
                                  h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        for (int32_t i = 0; i < k; ++i) out[(int64_t)i * mf::kPolRec + mf::kPolF + 1] *= (float)h->tick_ms;
    }
    if (n_out) *n_out = nrec;
    return MF_OK;
}

MF_API int mf_set_stream(mf_handle_t *h, void *stream) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->stream = stream ? static_cast<hipStream_t>(stream) : h->own_stream;
    return MF_OK;
}

}  // extern "C"
