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
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    mf::DevGraph g{};
    std::vector<void *> allocs;
    mf::Ctrl *h_ctrl = nullptr;  // pinned read-back of the control block
    int64_t *d_ids = nullptr;    // staging for host update batches
    int32_t *d_caps = nullptr;
    int64_t *p_ids = nullptr;    // pinned host copies they are uploaded from
    int32_t *p_caps = nullptr;
    int64_t staging_cap = 0;
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
    State state = State::NoFlow;
    int64_t value = 0;
    mf_stats_t stats{};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    std::string err;
};

namespace {

// Default frontier size (items) up to which one workgroup runs BFS levels alone.
constexpr int32_t kSoloItems = 128;

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

template <typename T>
hipError_t dev_alloc(mf_handle_t *h, T **p, int64_t count) {
    size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return e;
    h->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return hipSuccess;
}

void release(mf_handle_t *h) {
    if (!h || mf::process_exiting()) return;
    if (h->device >= 0) (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (void *p : h->allocs) (void)hipFree(p);
    h->allocs.clear();
    if (h->d_ids) (void)hipFree(h->d_ids);
    if (h->d_caps) (void)hipFree(h->d_caps);
    if (h->p_ids) (void)hipHostFree(h->p_ids);
    if (h->p_caps) (void)hipHostFree(h->p_caps);
    if (h->d_ptrace) (void)hipFree(h->d_ptrace);
    if (h->h_ctrl) (void)hipHostFree(h->h_ctrl);
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

// Launch the persistent loop, read back, interpret the status.
int run_loop_and_finish(mf_handle_t *h) {
    if (h->seq > (1 << 30)) {  // keep round ids unique: restart them with clean stamps
        HIP_TRY(h, mf::launch_fill_i32(h->g.mark, h->g.n, 0, h->stream));
        HIP_TRY(h, mf::launch_fill_i32(h->g.rmark, h->g.n, 0, h->stream));
        h->seq = 1;
    }
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
    p.combine = h->combine;
    p.policy_mode = h->policy_mode;
    p.policy_w = mf::policy_device_params(h->policy);
    p.policy_margin = h->policy_margin;
    p.policy_explore = h->policy_explore;
    p.policy_seed = h->policy_seed;
    p.policy_action = h->policy_action;
    p.batch_fraction = h->batch_fraction;
    p.policy_per_call = h->policy_per_call;
    // height counts of the gap heuristic start at zero (the loop clears them
    // again before every later global relabel); only the heuristic reads them
    if (h->use_gap) HIP_TRY(h, mf::launch_fill_i32(h->g.hcount, (int64_t)h->g.n + 1, 0, h->stream));
    HIP_TRY(h, hipEventRecord(h->ev[1], h->stream));
    HIP_TRY(h, mf::launch_loop(h->g, p, h->grid, h->stream));
    HIP_TRY(h, hipEventRecord(h->ev[2], h->stream));
    int rc = finish_call(h);
    if (rc) return rc;
    const mf::Ctrl &c = *h->h_ctrl;
    if (c.err) return MF_EINVAL;  // caller reports the message
    h->seq += c.rounds + 1;
    fill_stats(h, true);
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
// is staged by the runtime, synchronously).  Every call ends with a stream
// synchronisation, so the pinned copies are free again by the next call.
int stage_host_batch(mf_handle_t *h, const int64_t *ids, const int32_t *caps, int64_t k) {
    if (k > h->staging_cap) {
        if (h->d_ids) (void)hipFree(h->d_ids);
        if (h->d_caps) (void)hipFree(h->d_caps);
        if (h->p_ids) (void)hipHostFree(h->p_ids);
        if (h->p_caps) (void)hipHostFree(h->p_caps);
        h->d_ids = nullptr;
        h->d_caps = nullptr;
        h->p_ids = nullptr;
        h->p_caps = nullptr;
        h->staging_cap = 0;
        int64_t want = std::max<int64_t>(k, 1024);
        if (hipMalloc(&h->d_ids, sizeof(int64_t) * want) != hipSuccess ||
            hipMalloc(&h->d_caps, sizeof(int32_t) * want) != hipSuccess ||
            hipHostMalloc((void **)&h->p_ids, sizeof(int64_t) * want, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&h->p_caps, sizeof(int32_t) * want, hipHostMallocDefault) != hipSuccess)
            return fail(h, MF_ENOMEM, "cannot allocate the update staging buffers");
        h->staging_cap = want;
    }
    if (k > 0) {
        std::memcpy(h->p_ids, ids, sizeof(int64_t) * k);
        std::memcpy(h->p_caps, caps, sizeof(int32_t) * k);
        HIP_TRY(h, hipMemcpyAsync(h->d_ids, h->p_ids, sizeof(int64_t) * k, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, hipMemcpyAsync(h->d_caps, h->p_caps, sizeof(int32_t) * k, hipMemcpyHostToDevice, h->stream));
    }
    return MF_OK;
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
    HIP_TRY(h, mf::launch_saturate_source(h->g, h->stream));
    h->batch_fraction = h->g.m > 0 ? (float)((double)k / (double)h->g.m) : 0.f;
    rc = run_loop_and_finish(h);
    if (rc == MF_EINVAL) return update_error_text(h, h->h_ctrl->err);
    return rc;
}

bool opts_valid(const mf_opts_t &o, std::string *why) {
    if (o.kernel_cycles < 0) { *why = "kernel_cycles must be >= 0"; return false; }
    if (o.mode != MF_MODE_DATA && o.mode != MF_MODE_TOPOLOGY) { *why = "unknown mode"; return false; }
    if (o.grid_blocks < 0) { *why = "grid_blocks must be >= 0"; return false; }
    if (o.device < 0) { *why = "device must be >= 0"; return false; }
    if (o.time_budget_ms < 0) { *why = "time_budget_ms must be >= 0"; return false; }
    if (o.max_rounds < 0) { *why = "max_rounds must be >= 0"; return false; }
    if (o.relabel_budget < 0) { *why = "relabel_budget must be >= 0"; return false; }
    if (o.flags & ~MF_FLAG_GAP) { *why = "unknown flags"; return false; }
    if (o.reserved[0]) { *why = "reserved fields must be zero"; return false; }
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
    mf::HostPairs hp;
    try {
        if (mf::build_pairs(n, m, g->row_ptr, g->col, cap, &hp, &why))
            return fail(nullptr, MF_EINVAL, why);
    } catch (const std::bad_alloc &) {
        return fail(nullptr, MF_ENOMEM, "host allocation failed while building arc pairs");
    }
    // per-edge capacity limit: after the deltas of one batch land, an arc's
    // residual is at most twice the pair's capacity sum, which must fit int32
    const int64_t lim = mf::edge_cap_limit(hp.max_pair_mult);
    for (int64_t i = 0; i < m; ++i)
        if (cap[i] > lim)
            return fail(nullptr, MF_EINVAL,
                        "capacity above the per-edge limit " + std::to_string(lim));

    mf_handle_t *h = new (std::nothrow) mf_handle_t();
    if (!h) return fail(nullptr, MF_ENOMEM, "host allocation failed");
    h->device = o.device;
    h->cap_limit = (int32_t)lim;
    h->mode = o.mode;
    h->max_iter = o.max_iterations;
    const int64_t budget_ms = o.time_budget_ms > 0 ? o.time_budget_ms : 60000;
    h->max_rounds = o.max_rounds > 0 ? o.max_rounds : 65536;
    h->relabel_budget = o.relabel_budget > 0 ? o.relabel_budget : std::max<int64_t>(1024, n / 16);
    h->rounds_per_level = o.rounds_per_level == 0 ? 1 : (o.rounds_per_level < 0 ? 0 : o.rounds_per_level);
    h->use_gap = (o.flags & MF_FLAG_GAP) ? 1 : 0;
    h->stall_rounds = o.stall_rounds == 0 ? 3 : (o.stall_rounds < 0 ? 0 : o.stall_rounds);
    h->solo_items = o.solo_items == 0 ? kSoloItems : (o.solo_items < 0 ? 0 : o.solo_items);
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
    if ((e = hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(MF_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    h->stream = h->own_stream;
    for (auto &ev : h->ev)
        if ((e = hipEventCreate(&ev)) != hipSuccess)
            return bail(MF_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
    if ((e = hipHostMalloc((void **)&h->h_ctrl, sizeof(mf::Ctrl), hipHostMallocDefault)) != hipSuccess)
        return bail(MF_ENOMEM, "pinned control block");

    // heavy vertices (arc lists handled by a wavefront in topology-driven sweeps)
    std::vector<int32_t> heavy;
    int64_t nhuge = 0;  // vertices visited by a whole workgroup
    for (int32_t v = 0; v < n; ++v) {
        const int32_t deg = hp.row_ptr[v + 1] - hp.row_ptr[v];
        if (v != s && v != t && deg > mf::kLightMaxDeg) heavy.push_back(v);
        if (v != s && v != t && deg > mf::kHugeDeg) nhuge++;
    }
    // vertices of huge degree draw pushes from many others at once: add them
    // up per workgroup first
    h->combine = nhuge > 0 ? 1 : 0;

    mf::DevGraph &d = h->g;
    d.n = n;
    d.s = s;
    d.t = t;
    d.A = hp.A;
    d.m = m;
    d.qcap = (int64_t)n + hp.A / mf::kChunk + 64;
    d.n_heavy_all = (int32_t)heavy.size();
    const int64_t A = hp.A;
#define ALLOC(ptr, count)                                                             \
    do {                                                                              \
        if ((e = dev_alloc(h, &(ptr), (count))) != hipSuccess)                        \
            return bail(MF_ENOMEM, std::string("hipMalloc " #ptr ": ") + hipGetErrorString(e)); \
    } while (0)
    ALLOC(d.row_ptr, (int64_t)n + 1);
    ALLOC(d.arc, A);
    ALLOC(d.twin, A);
    ALLOC(d.cap, A);
    ALLOC(d.edge2arc, m);
    ALLOC(d.ecap, m);
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
#undef ALLOC
    // upload: arc records {head, residual}; the residual is set by the solve
    std::vector<int2> arc((size_t)A);
    for (int64_t a = 0; a < A; ++a) arc[a] = make_int2(hp.col[a], hp.cap[a]);
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream) : hipSuccess;
    };
    if ((e = up(d.row_ptr, hp.row_ptr.data(), sizeof(int32_t) * (n + 1))) != hipSuccess ||
        (e = up(d.arc, arc.data(), sizeof(int2) * A)) != hipSuccess ||
        (e = up(d.twin, hp.twin.data(), sizeof(int32_t) * A)) != hipSuccess ||
        (e = up(d.cap, hp.cap.data(), sizeof(int32_t) * A)) != hipSuccess ||
        (e = up(d.edge2arc, hp.edge2arc.data(), sizeof(int32_t) * m)) != hipSuccess ||
        (e = up(d.ecap, cap, sizeof(int32_t) * m)) != hipSuccess ||
        (e = up(d.heavy_all, heavy.data(), sizeof(int32_t) * heavy.size())) != hipSuccess)
        return bail(MF_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    if ((e = mf::launch_fill_i32(d.stamp, m, 0, h->stream)) != hipSuccess ||
        (e = mf::launch_fill_i32(d.mark, n, 0, h->stream)) != hipSuccess ||
        (e = mf::launch_fill_i32(d.rmark, n, 0, h->stream)) != hipSuccess ||

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
    return run_loop_and_finish(h);
}

MF_API int mf_resume(mf_handle_t *h) {
    if (!h) return fail(nullptr, MF_EINVAL, "null handle");
    if (h->state == State::NoFlow || h->state == State::NeedsSolve)
        return fail(h, MF_ESTATE, "no flow to resume: call mf_solve");
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, hipEventRecord(h->ev[0], h->stream));
    HIP_TRY(h, mf::launch_reset_ctrl(h->g, h->stream));
    return run_loop_and_finish(h);
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
    if (side_out)
        HIP_TRY(h, hipMemcpyAsync(side_out, h->d_side, (size_t)h->g.n, hipMemcpyDeviceToHost, h->stream));
    int64_t cut = 0;
    HIP_TRY(h, hipMemcpyAsync(&cut, &h->g.ctrl->cut, sizeof(int64_t), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
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
    std::vector<int2> arc((size_t)d.A);
    std::vector<int32_t> twin((size_t)d.A);
    if (d.A) {
        HIP_TRY(h, hipMemcpy(arc.data(), d.arc, sizeof(int2) * d.A, hipMemcpyDeviceToHost));
        HIP_TRY(h, hipMemcpy(twin.data(), d.twin, sizeof(int32_t) * d.A, hipMemcpyDeviceToHost));
    }
    for (int64_t a = 0; a < d.A; ++a) {
        if (cap[a] < 0 || cf[a] < 0) return fail(h, MF_EINVAL, "negative capacity or residual");
        const int64_t b = twin[a];
        if ((int64_t)cf[a] + cf[b] != (int64_t)cap[a] + cap[b])
            return fail(h, MF_EINVAL, "residuals of an arc pair do not sum to its capacities");
    }
    for (int64_t i = 0; i < d.m; ++i)
        if (ecap[i] < 0 || ecap[i] > h->cap_limit) return fail(h, MF_EINVAL, "edge capacity out of range");
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
        if (hipMalloc(&q, sizeof(float) * mf::kTraceCap * mf::kPolRec) != hipSuccess)
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
