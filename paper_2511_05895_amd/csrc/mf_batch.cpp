// Batched solve of many independent max-flow instances (mf_batch_* in
// include/mf.h).  The instances are packed block-diagonally into one set of
// device arrays; every instance is solved from scratch by one workgroup of a
// persistent launch (no grid barrier: a workgroup barrier separates the steps
// of its instance).  Instances are grouped into size classes by arc count;
// each class is one launch with its own workgroup size and KERNELCYCLES, the
// classes run side by side on forked streams, and the whole fork/join is
// captured once into a hipGraph that later solves replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/mf.h"
#include "build_pairs.h"
#include "ctrl_stats.h"
#include "mf_internal.h"

namespace {

thread_local std::string g_batch_create_error;

constexpr int kBlocks[3] = {256, 512, 1024};

bool block_ok(int b) { return b == 256 || b == 512 || b == 1024; }

}  // namespace

struct mf_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t side[MF_BATCH_MAX_CLASSES] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[MF_BATCH_MAX_CLASSES] = {};
    hipEvent_t ev[2] = {nullptr, nullptr};
    int32_t count = 0;
    std::vector<mf::DevGraph> g;    // per-instance views into the packed arrays
    std::vector<int32_t> cap_limit;  // per instance
    std::vector<int32_t> kc_auto;    // max(1, round(m/n)) per instance
    std::vector<int64_t> arcs;       // A per instance
    std::vector<int32_t> order;      // instance ids, class by class, largest first
    std::vector<int32_t> class_begin;  // n_classes + 1 offsets into order
    mf::DevGraph *d_graphs = nullptr;
    int32_t *d_order = nullptr;
    int32_t *d_kc = nullptr;
    mf::BatchResult *d_res = nullptr;
    mf::BatchResult *h_res = nullptr;  // pinned
    mf::Ctrl *h_ctrl = nullptr;        // pinned, one instance at a time
    uint8_t *d_side = nullptr;
    int64_t *d_ids = nullptr;
    int32_t *d_caps = nullptr;
    int64_t staging_cap = 0;
    int32_t max_n = 0;
    int32_t epoch = 0;
    mf_batch_opts_t opts{};
    mf::LoopParams params{};
    double tick_ms = 1e-5;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool solved = false;
    std::vector<int64_t> values;
    std::vector<int32_t> status;
    double last_kernel_ms = 0.0;
    int64_t replays = 0;
    std::vector<void *> allocs;
    std::string err;
};

namespace {

int bfail(mf_batch_t *b, int code, const std::string &msg) {
    if (b) b->err = msg;
    else g_batch_create_error = msg;
    return code;
}

#define BHIP(b, expr)                                                                    \
    do {                                                                                 \
        hipError_t _e = (expr);                                                          \
        if (_e != hipSuccess) return bfail((b), MF_EDEVICE, std::string(#expr ": ") + hipGetErrorString(_e)); \
    } while (0)

template <typename T>
hipError_t balloc(mf_batch_t *b, T **p, int64_t count) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * (size_t)std::max<int64_t>(count, 1));
    if (e != hipSuccess) return e;
    b->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return hipSuccess;
}

void drop_graph(mf_batch_t *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

void release(mf_batch_t *b) {
    if (!b || mf::process_exiting()) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    for (void *p : b->allocs) (void)hipFree(p);
    b->allocs.clear();
    if (b->d_ids) (void)hipFree(b->d_ids);
    if (b->d_caps) (void)hipFree(b->d_caps);
    if (b->h_res) (void)hipHostFree(b->h_res);
    if (b->h_ctrl) (void)hipHostFree(b->h_ctrl);
    for (auto &e : b->join_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    for (auto &s : b->side)
        if (s) (void)hipStreamDestroy(s);
    if (b->stream) (void)hipStreamDestroy(b->stream);
}

bool opts_valid(const mf_batch_opts_t &o, std::string *why) {
    if (o.device < 0) { *why = "device must be >= 0"; return false; }
    if (o.time_budget_ms < 0) { *why = "time_budget_ms must be >= 0"; return false; }
    if (o.n_classes < 1 || o.n_classes > MF_BATCH_MAX_CLASSES) {
        *why = "n_classes must be in [1, " + std::to_string(MF_BATCH_MAX_CLASSES) + "]";
        return false;
    }
    for (int c = 0; c < o.n_classes; ++c) {
        if (!block_ok(o.block[c])) { *why = "block must be 256, 512 or 1024"; return false; }
        if (o.kernel_cycles[c] < 0) { *why = "kernel_cycles must be >= 0"; return false; }
        if (c + 1 < o.n_classes && (o.class_max_arcs[c] <= 0 ||
                                    (c > 0 && o.class_max_arcs[c] <= o.class_max_arcs[c - 1]))) {
            *why = "class_max_arcs must be positive and ascending";
            return false;
        }
    }
    if (o.flags & ~MF_FLAG_GAP) { *why = "unknown flags"; return false; }
    if (o.use_graph != 0 && o.use_graph != 1) { *why = "use_graph must be 0 or 1"; return false; }
    for (int32_t r : o.reserved)
        if (r) { *why = "reserved fields must be zero"; return false; }
    return true;
}

// Class of an instance with `a` arcs: the first class whose bound holds; the
// last class takes the rest.
int class_of(const mf_batch_opts_t &o, int64_t a) {
    for (int c = 0; c + 1 < o.n_classes; ++c)
        if (a <= o.class_max_arcs[c]) return c;
    return o.n_classes - 1;
}

// Order the instances class by class, largest first inside a class, and
// upload the order and the per-instance KERNELCYCLES.  Drops the captured
// graph (its launches encode the class split).
int apply_config(mf_batch_t *b) {
    const mf_batch_opts_t &o = b->opts;
    std::vector<int32_t> cls(b->count);
    for (int32_t i = 0; i < b->count; ++i) cls[i] = class_of(o, b->arcs[i]);
    b->order.resize(b->count);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(), [&](int32_t x, int32_t y) {
        if (cls[x] != cls[y]) return cls[x] < cls[y];
        return b->arcs[x] > b->arcs[y];
    });
    b->class_begin.assign(o.n_classes + 1, 0);
    for (int32_t i = 0; i < b->count; ++i) b->class_begin[cls[i] + 1]++;
    for (int c = 0; c < o.n_classes; ++c) b->class_begin[c + 1] += b->class_begin[c];
    std::vector<int32_t> kc(b->count);
    for (int32_t i = 0; i < b->count; ++i)
        kc[i] = o.kernel_cycles[cls[i]] > 0 ? o.kernel_cycles[cls[i]] : b->kc_auto[i];
    BHIP(b, hipMemcpyAsync(b->d_order, b->order.data(), sizeof(int32_t) * b->count, hipMemcpyHostToDevice,
                           b->stream));
    BHIP(b, hipMemcpyAsync(b->d_kc, kc.data(), sizeof(int32_t) * b->count, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    b->params.use_gap = (o.flags & MF_FLAG_GAP) ? 1 : 0;
    b->params.stall_rounds = o.stall_rounds == 0 ? 3 : (o.stall_rounds < 0 ? 0 : o.stall_rounds);
    drop_graph(b);
    return MF_OK;
}

// Launch class c alone on stream st.
hipError_t launch_class(mf_batch_t *b, int c, hipStream_t st) {
    const int32_t beg = b->class_begin[c], cnt = b->class_begin[c + 1] - beg;
    if (cnt == 0) return hipSuccess;
    return mf::launch_batch(b->d_graphs, b->d_order + beg, cnt, b->params, b->d_kc, b->d_res,
                            b->opts.block[c], st);
}

// All classes side by side: fork from the main stream, one class per side
// stream, join back.  Recorded into a graph when the main stream captures.
hipError_t enqueue_all(mf_batch_t *b) {
    hipError_t e = hipEventRecord(b->fork_ev, b->stream);
    if (e != hipSuccess) return e;
    for (int c = 0; c < b->opts.n_classes; ++c) {
        if (b->class_begin[c + 1] == b->class_begin[c]) continue;
        if ((e = hipStreamWaitEvent(b->side[c], b->fork_ev, 0)) != hipSuccess) return e;
        if ((e = launch_class(b, c, b->side[c])) != hipSuccess) return e;
        if ((e = hipEventRecord(b->join_ev[c], b->side[c])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(b->stream, b->join_ev[c], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

int capture(mf_batch_t *b) {
    drop_graph(b);
    BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_all(b);
    hipGraph_t gr = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &gr);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return bfail(b, MF_EDEVICE, std::string("graph capture: ") +
                                        hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = gr;
    BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return MF_OK;
}

// Read back the per-instance results and turn them into a status.
int collect(mf_batch_t *b) {
    BHIP(b, hipMemcpyAsync(b->h_res, b->d_res, sizeof(mf::BatchResult) * b->count, hipMemcpyDeviceToHost,
                           b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, b->ev[0], b->ev[1]) == hipSuccess) b->last_kernel_ms = ms;
    int rc = MF_OK;
    for (int32_t i = 0; i < b->count; ++i) {
        b->values[i] = b->h_res[i].value;
        b->status[i] = b->h_res[i].status;
        if (b->h_res[i].status == mf::kSolved) continue;
        if (b->h_res[i].status == mf::kDeadline && rc == MF_OK) {
            rc = bfail(b, MF_ETIMEOUT, "instance " + std::to_string(i) + " ran out of its time budget");
        } else if (b->h_res[i].status != mf::kDeadline) {
            rc = bfail(b, MF_EDEVICE, "instance " + std::to_string(i) + " ended with loop status " +
                                          std::to_string(b->h_res[i].status));
        }
    }
    b->solved = rc == MF_OK;
    return rc;
}

int stage(mf_batch_t *b, const int64_t *ids, const int32_t *caps, int64_t k) {
    if (k > b->staging_cap) {
        if (b->d_ids) (void)hipFree(b->d_ids);
        if (b->d_caps) (void)hipFree(b->d_caps);
        b->d_ids = nullptr;
        b->d_caps = nullptr;
        b->staging_cap = 0;
        BHIP(b, hipMalloc(&b->d_ids, sizeof(int64_t) * k));
        BHIP(b, hipMalloc(&b->d_caps, sizeof(int32_t) * k));
        b->staging_cap = k;
    }
    if (k > 0) {
        BHIP(b, hipMemcpyAsync(b->d_ids, ids, sizeof(int64_t) * k, hipMemcpyHostToDevice, b->stream));
        BHIP(b, hipMemcpyAsync(b->d_caps, caps, sizeof(int32_t) * k, hipMemcpyHostToDevice, b->stream));
    }
    return MF_OK;
}

}  // namespace

extern "C" {

MF_API void mf_batch_default_opts(mf_batch_opts_t *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->n_classes = 3;
    o->class_max_arcs[0] = 32768;
    o->class_max_arcs[1] = 262144;
    for (int c = 0; c < MF_BATCH_MAX_CLASSES; ++c) o->block[c] = 1024;
    o->block[0] = 256;
    o->use_graph = 1;
}

MF_API const char *mf_batch_last_error(const mf_batch_t *b) {
    return b ? b->err.c_str() : g_batch_create_error.c_str();
}

MF_API int mf_batch_create(int32_t count, const int32_t *n, const int64_t *m, const int64_t *row_ptr,
                           const int32_t *col, const int32_t *cap, const int32_t *s, const int32_t *t,
                           const mf_batch_opts_t *opts, mf_batch_t **out) {
    if (!out) return bfail(nullptr, MF_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1) return bfail(nullptr, MF_EINVAL, "count must be >= 1");
    if (!n || !m || !row_ptr || !s || !t) return bfail(nullptr, MF_EINVAL, "null argument");
    mf_batch_opts_t o;
    mf_batch_default_opts(&o);
    if (opts) o = *opts;
    std::string why;
    if (!opts_valid(o, &why)) return bfail(nullptr, MF_EINVAL, why);
    // per-instance checks and arc-pair layouts
    std::vector<mf::HostPairs> hp(count);
    std::vector<int32_t> lim(count);
    int64_t roff = 0, eoff = 0;
    int64_t sum_n = 0, sum_a = 0, sum_m = 0, sum_q = 0, sum_huge = 0;
    std::vector<int64_t> nhuge(count, 0);
    for (int32_t i = 0; i < count; ++i) {
        const int64_t *rp = row_ptr + roff;
        const int32_t *ci = (m[i] > 0 && col) ? col + eoff : nullptr;
        const int32_t *ca = (m[i] > 0 && cap) ? cap + eoff : nullptr;
        if (m[i] > 0 && (!ci || !ca)) return bfail(nullptr, MF_EINVAL, "null col or cap array");
        std::string w;
        if (mf::check_graph(n[i], m[i], rp, ci, ca, s[i], t[i], &w))
            return bfail(nullptr, MF_EINVAL, "instance " + std::to_string(i) + ": " + w);
        try {
            if (mf::build_pairs(n[i], m[i], rp, ci, ca, &hp[i], &w))
                return bfail(nullptr, MF_EINVAL, "instance " + std::to_string(i) + ": " + w);
        } catch (const std::bad_alloc &) {
            return bfail(nullptr, MF_ENOMEM, "host allocation failed while building arc pairs");
        }
        lim[i] = (int32_t)mf::edge_cap_limit(hp[i].max_pair_mult);
        for (int64_t j = 0; j < m[i]; ++j)
            if (ca[j] > lim[i])
                return bfail(nullptr, MF_EINVAL, "instance " + std::to_string(i) +
                                                     ": capacity above the per-edge limit " +
                                                     std::to_string(lim[i]));
        roff += (int64_t)n[i] + 1;
        eoff += m[i];
        sum_n += n[i];
        sum_a += hp[i].A;
        sum_m += m[i];
        sum_q += (int64_t)n[i] + hp[i].A / mf::kChunk + 64;
        for (int32_t v = 0; v < n[i]; ++v)
            if (v != s[i] && v != t[i] && hp[i].row_ptr[v + 1] - hp[i].row_ptr[v] > mf::kHugeDeg) nhuge[i]++;
        sum_huge += nhuge[i];
    }
    if (sum_a >= (int64_t)INT32_MAX * 8) return bfail(nullptr, MF_EINVAL, "batch too large");

    mf_batch_t *b = new (std::nothrow) mf_batch_t();
    if (!b) return bfail(nullptr, MF_ENOMEM, "host allocation failed");
    auto bail = [&](int code, const std::string &msg) {
        release(b);
        delete b;
        return bfail(nullptr, code, msg);
    };
    b->device = o.device;
    b->count = count;
    b->opts = o;
    hipError_t e = hipSetDevice(o.device);
    if (e != hipSuccess) return bail(MF_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    if ((e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(MF_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    for (int c = 0; c < MF_BATCH_MAX_CLASSES; ++c) {
        if ((e = hipStreamCreateWithFlags(&b->side[c], hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&b->join_ev[c], hipEventDisableTiming)) != hipSuccess)
            return bail(MF_EDEVICE, std::string("stream/event: ") + hipGetErrorString(e));
    }
    if ((e = hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreate(&b->ev[0])) != hipSuccess || (e = hipEventCreate(&b->ev[1])) != hipSuccess)
        return bail(MF_EDEVICE, std::string("event: ") + hipGetErrorString(e));
    if ((e = hipHostMalloc((void **)&b->h_res, sizeof(mf::BatchResult) * count, hipHostMallocDefault)) !=
            hipSuccess ||
        (e = hipHostMalloc((void **)&b->h_ctrl, sizeof(mf::Ctrl), hipHostMallocDefault)) != hipSuccess)
        return bail(MF_ENOMEM, "pinned result buffers");

    // packed arrays
    int32_t *row_ptr_d, *twin_d, *cap_d, *edge2arc_d, *ecap_d, *stamp_d, *h_d, *l0, *l1, *l2, *mark_d,
        *rmark_d, *relab_d, *hcount_d, *u0, *u1, *u2;
    int2 *arc_d, *q0, *q1;
    int64_t *e_d;
    mf::Ctrl *ctrl_d;
#define BALLOC(ptr, cnt)                                                                   \
    do {                                                                                   \
        if ((e = balloc(b, &(ptr), (cnt))) != hipSuccess)                                  \
            return bail(MF_ENOMEM, std::string("hipMalloc " #ptr ": ") + hipGetErrorString(e)); \
    } while (0)
    BALLOC(row_ptr_d, sum_n + count);
    BALLOC(arc_d, sum_a);
    BALLOC(twin_d, sum_a);
    BALLOC(cap_d, sum_a);
    BALLOC(edge2arc_d, sum_m);
    BALLOC(ecap_d, sum_m);
    BALLOC(stamp_d, sum_m);
    BALLOC(e_d, sum_n);
    BALLOC(h_d, sum_n);
    BALLOC(q0, sum_q);
    BALLOC(q1, sum_q);
    BALLOC(l0, sum_n);
    BALLOC(l1, sum_n);
    BALLOC(l2, sum_n);
    BALLOC(u0, sum_huge);
    BALLOC(u1, sum_huge);
    BALLOC(u2, sum_huge);
    BALLOC(mark_d, sum_n);
    BALLOC(rmark_d, sum_n);
    BALLOC(relab_d, sum_n);
    BALLOC(hcount_d, sum_n + count);
    BALLOC(ctrl_d, count);
    BALLOC(b->d_graphs, count);
    BALLOC(b->d_order, count);
    BALLOC(b->d_kc, count);
    BALLOC(b->d_res, count);
#undef BALLOC
    b->g.resize(count);
    b->cap_limit = lim;
    b->kc_auto.resize(count);
    b->arcs.resize(count);
    b->values.assign(count, 0);
    b->status.assign(count, 0);
    std::vector<int2> arc_h;
    int64_t vo = 0, ao = 0, mo = 0, qo = 0, ro = 0, uo = 0;
    eoff = 0;
    for (int32_t i = 0; i < count; ++i) {
        const mf::HostPairs &p = hp[i];
        mf::DevGraph &d = b->g[i];
        d.n = n[i];
        d.s = s[i];
        d.t = t[i];
        d.A = p.A;
        d.m = m[i];
        d.row_ptr = row_ptr_d + ro;
        d.arc = arc_d + ao;
        d.twin = twin_d + ao;
        d.cap = cap_d + ao;
        d.edge2arc = edge2arc_d + mo;
        d.ecap = ecap_d + mo;
        d.stamp = stamp_d + mo;
        d.e = e_d + vo;
        d.h = h_d + vo;
        d.qcap = (int64_t)n[i] + p.A / mf::kChunk + 64;
        d.q[0] = q0 + qo;
        d.q[1] = q1 + qo;
        d.list[0] = l0 + vo;
        d.list[1] = l1 + vo;
        d.list[2] = l2 + vo;
        d.huge[0] = u0 + uo;
        d.huge[1] = u1 + uo;
        d.huge[2] = u2 + uo;
        d.mark = mark_d + vo;
        d.rmark = rmark_d + vo;
        d.relab = relab_d + vo;
        d.hcount = hcount_d + ro;
        d.heavy_all = nullptr;
        d.n_heavy_all = 0;
        d.ctrl = ctrl_d + i;
        arc_h.resize((size_t)p.A);
        for (int64_t a = 0; a < p.A; ++a) arc_h[a] = make_int2(p.col[a], p.cap[a]);
        auto up = [&](void *dst, const void *src, size_t bytes) {
            return bytes ? hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
        };
        if ((e = up(d.row_ptr, p.row_ptr.data(), sizeof(int32_t) * (n[i] + 1))) != hipSuccess ||
            (e = up(d.arc, arc_h.data(), sizeof(int2) * p.A)) != hipSuccess ||
            (e = up(d.twin, p.twin.data(), sizeof(int32_t) * p.A)) != hipSuccess ||
            (e = up(d.cap, p.cap.data(), sizeof(int32_t) * p.A)) != hipSuccess ||
            (e = up(d.edge2arc, p.edge2arc.data(), sizeof(int32_t) * m[i])) != hipSuccess ||
            (e = up(d.ecap, cap + eoff, sizeof(int32_t) * m[i])) != hipSuccess)
            return bail(MF_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
        b->kc_auto[i] = (int32_t)std::max<int64_t>(1, (int64_t)((double)m[i] / n[i] + 0.5));
        b->arcs[i] = p.A;
        b->max_n = std::max(b->max_n, n[i]);
        vo += n[i];
        ro += (int64_t)n[i] + 1;
        ao += p.A;
        mo += m[i];
        eoff += m[i];
        qo += d.qcap;
        uo += nhuge[i];
    }
    hp.clear();
    if ((e = hipMemcpy(b->d_graphs, b->g.data(), sizeof(mf::DevGraph) * count, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = mf::launch_fill_i32(stamp_d, sum_m, 0, b->stream)) != hipSuccess)
        return bail(MF_EDEVICE, std::string("init: ") + hipGetErrorString(e));
    if ((e = balloc(b, &b->d_side, b->max_n)) != hipSuccess)
        return bail(MF_ENOMEM, std::string("hipMalloc side: ") + hipGetErrorString(e));

    int clock_khz = 0;
    if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, o.device) != hipSuccess ||
        clock_khz <= 0)
        clock_khz = 100000;
    b->tick_ms = 1.0 / clock_khz;
    const int64_t budget_ms = o.time_budget_ms > 0 ? o.time_budget_ms : 60000;
    mf::LoopParams &pr = b->params;
    pr.kc = 0;  // per instance, from d_kc
    pr.mode = MF_MODE_DATA;
    pr.max_iter = -1;
    pr.deadline_ticks = budget_ms * (int64_t)clock_khz;
    pr.barrier_ticks = 10000 * (int64_t)clock_khz;
    pr.relabel_budget = 0;  // per instance: max(1024, n/16)
    pr.max_rounds = 65536;
    pr.seq_base = 1;
    pr.rounds_per_level = 1;
    pr.lazy_items = 1024;
    int rc = apply_config(b);
    if (rc) {
        std::string msg = b->err;
        return bail(rc, msg);
    }
    *out = b;
    return MF_OK;
}

MF_API void mf_batch_destroy(mf_batch_t *b) {
    if (!b) return;
    release(b);
    delete b;
}

MF_API int mf_batch_count(const mf_batch_t *b, int32_t *count) {
    if (!b || !count) return bfail(const_cast<mf_batch_t *>(b), MF_EINVAL, "null argument");
    *count = b->count;
    return MF_OK;
}

MF_API int mf_batch_get_opts(const mf_batch_t *b, mf_batch_opts_t *o) {
    if (!b || !o) return bfail(const_cast<mf_batch_t *>(b), MF_EINVAL, "null argument");
    *o = b->opts;
    return MF_OK;
}

MF_API int mf_batch_set_opts(mf_batch_t *b, const mf_batch_opts_t *o) {
    if (!b || !o) return bfail(b, MF_EINVAL, "null argument");
    std::string why;
    if (!opts_valid(*o, &why)) return bfail(b, MF_EINVAL, why);
    if (o->device != b->device) return bfail(b, MF_EINVAL, "device cannot change");
    const int64_t budget_ms = o->time_budget_ms > 0 ? o->time_budget_ms : 60000;
    b->params.deadline_ticks = (int64_t)(budget_ms / b->tick_ms);
    b->opts = *o;
    BHIP(b, hipSetDevice(b->device));
    return apply_config(b);
}

MF_API int mf_batch_solve(mf_batch_t *b) {
    if (!b) return bfail(nullptr, MF_EINVAL, "null batch");
    BHIP(b, hipSetDevice(b->device));
    b->solved = false;
    if (b->opts.use_graph) {
        if (!b->exec) {
            int rc = capture(b);
            if (rc) return rc;
        }
        BHIP(b, hipEventRecord(b->ev[0], b->stream));
        BHIP(b, hipGraphLaunch(b->exec, b->stream));
        BHIP(b, hipEventRecord(b->ev[1], b->stream));
        b->replays++;
    } else {
        BHIP(b, hipEventRecord(b->ev[0], b->stream));
        BHIP(b, enqueue_all(b));
        BHIP(b, hipEventRecord(b->ev[1], b->stream));
    }
    return collect(b);
}

MF_API int mf_batch_solve_class(mf_batch_t *b, int32_t c, double *kernel_ms) {
    if (!b) return bfail(nullptr, MF_EINVAL, "null batch");
    if (c < 0 || c >= b->opts.n_classes) return bfail(b, MF_EINVAL, "class out of range");
    BHIP(b, hipSetDevice(b->device));
    BHIP(b, hipEventRecord(b->ev[0], b->stream));
    BHIP(b, launch_class(b, c, b->stream));
    BHIP(b, hipEventRecord(b->ev[1], b->stream));
    BHIP(b, hipMemcpyAsync(b->h_res, b->d_res, sizeof(mf::BatchResult) * b->count, hipMemcpyDeviceToHost,
                           b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    float ms = 0.f;
    BHIP(b, hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
    if (kernel_ms) *kernel_ms = ms;
    for (int32_t j = b->class_begin[c]; j < b->class_begin[c + 1]; ++j) {
        const int32_t i = b->order[j];
        if (b->h_res[i].status != mf::kSolved)
            return bfail(b, b->h_res[i].status == mf::kDeadline ? MF_ETIMEOUT : MF_EDEVICE,
                         "instance " + std::to_string(i) + " did not finish");
        b->values[i] = b->h_res[i].value;
        b->status[i] = b->h_res[i].status;
    }
    return MF_OK;
}

MF_API int mf_batch_autotune(mf_batch_t *b, int32_t repeats, mf_batch_opts_t *chosen) {
    if (!b) return bfail(nullptr, MF_EINVAL, "null batch");
    if (repeats < 1) return bfail(b, MF_EINVAL, "repeats must be >= 1");
    BHIP(b, hipSetDevice(b->device));
    const int kcs[4] = {0, 1, 2, 4};
    mf_batch_opts_t best = b->opts;
    for (int c = 0; c < b->opts.n_classes; ++c) {
        if (b->class_begin[c + 1] == b->class_begin[c]) continue;
        double best_ms = 1e300;
        std::vector<int64_t> ref;
        for (int bl : kBlocks)
            for (int kc : kcs) {
                mf_batch_opts_t o = best;
                o.block[c] = bl;
                o.kernel_cycles[c] = kc;
                b->opts = o;
                int rc = apply_config(b);
                if (rc) return rc;
                std::vector<double> t;
                for (int r = 0; r < repeats; ++r) {
                    double ms = 0;
                    rc = mf_batch_solve_class(b, c, &ms);
                    if (rc) return rc;
                    t.push_back(ms);
                }
                // every candidate must reach the same values
                std::vector<int64_t> v;
                for (int32_t j = b->class_begin[c]; j < b->class_begin[c + 1]; ++j)
                    v.push_back(b->values[b->order[j]]);
                if (ref.empty()) ref = v;
                else if (v != ref)
                    return bfail(b, MF_EDEVICE, "autotune: candidate values differ in class " + std::to_string(c));
                std::sort(t.begin(), t.end());
                const double med = t[t.size() / 2];
                if (med < best_ms) {
                    best_ms = med;
                    best.block[c] = bl;
                    best.kernel_cycles[c] = kc;
                }
            }
    }
    b->opts = best;
    int rc = apply_config(b);
    if (rc) return rc;
    b->solved = false;
    if (chosen) *chosen = best;
    return MF_OK;
}

MF_API int mf_batch_num_arcs(const mf_batch_t *b, int64_t *arcs) {
    if (!b || !arcs) return bfail(const_cast<mf_batch_t *>(b), MF_EINVAL, "null argument");
    std::copy(b->arcs.begin(), b->arcs.end(), arcs);
    return MF_OK;
}

MF_API int mf_batch_values(const mf_batch_t *b, int64_t *values) {
    if (!b || !values) return bfail(const_cast<mf_batch_t *>(b), MF_EINVAL, "null argument");
    if (!b->solved) return bfail(const_cast<mf_batch_t *>(b), MF_ESTATE, "not solved");
    std::copy(b->values.begin(), b->values.end(), values);
    return MF_OK;
}

MF_API int mf_batch_last_ms(const mf_batch_t *b, double *kernel_ms) {
    if (!b || !kernel_ms) return bfail(const_cast<mf_batch_t *>(b), MF_EINVAL, "null argument");
    *kernel_ms = b->last_kernel_ms;
    return MF_OK;
}

MF_API int mf_batch_min_cut(mf_batch_t *b, int32_t i, uint8_t *side, int64_t *cut_cap) {
    if (!b) return bfail(nullptr, MF_EINVAL, "null batch");
    if (i < 0 || i >= b->count) return bfail(b, MF_EINVAL, "instance out of range");
    if (!b->solved) return bfail(b, MF_ESTATE, "not solved");
    const mf::DevGraph &g = b->g[i];
    BHIP(b, hipSetDevice(b->device));
    BHIP(b, mf::launch_fill_i32(reinterpret_cast<int32_t *>(&g.ctrl->cut), 2, 0, b->stream));
    BHIP(b, mf::launch_min_cut(g, side ? b->d_side : nullptr, b->stream));
    if (side) BHIP(b, hipMemcpyAsync(side, b->d_side, g.n, hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipMemcpyAsync(b->h_ctrl, g.ctrl, sizeof(mf::Ctrl), hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    if (cut_cap) *cut_cap = b->h_ctrl->cut;
    return MF_OK;
}

MF_API int mf_batch_get_stats(mf_batch_t *b, int32_t i, mf_stats_t *st) {
    if (!b || !st) return bfail(b, MF_EINVAL, "null argument");
    if (i < 0 || i >= b->count) return bfail(b, MF_EINVAL, "instance out of range");
    BHIP(b, hipSetDevice(b->device));
    BHIP(b, hipMemcpyAsync(b->h_ctrl, b->g[i].ctrl, sizeof(mf::Ctrl), hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    mf::stats_from_ctrl(*b->h_ctrl, b->tick_ms, st);
    st->grid_blocks = 1;
    st->loop_launches = 1;
    st->loop_kernel_ms = b->last_kernel_ms;
    return MF_OK;
}

MF_API int mf_batch_set_capacities(mf_batch_t *b, int32_t i, const int64_t *edge_ids, const int32_t *new_caps,
                                   int64_t k) {
    if (!b) return bfail(nullptr, MF_EINVAL, "null batch");
    if (i < 0 || i >= b->count) return bfail(b, MF_EINVAL, "instance out of range");
    const mf::DevGraph &g = b->g[i];
    if (k < 0 || k > g.m) return bfail(b, MF_EINVAL, "batch size k must be in [0, m]");
    if (k > 0 && (!edge_ids || !new_caps)) return bfail(b, MF_EINVAL, "null batch arrays");
    BHIP(b, hipSetDevice(b->device));
    int rc = stage(b, edge_ids, new_caps, k);
    if (rc) return rc;
    if (++b->epoch == INT32_MAX) {
        BHIP(b, mf::launch_fill_i32(g.stamp, g.m, 0, b->stream));
        b->epoch = 1;
    }
    BHIP(b, mf::launch_reset_ctrl(g, b->stream));
    BHIP(b, mf::launch_validate_updates(g, b->d_ids, b->d_caps, k, b->epoch, b->cap_limit[i], b->stream));
    BHIP(b, mf::launch_apply_delta(g, b->d_ids, b->d_caps, k, b->stream));
    BHIP(b, hipMemcpyAsync(b->h_ctrl, g.ctrl, sizeof(mf::Ctrl), hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    b->solved = false;
    if (b->h_ctrl->err) {
        std::string w;
        if (b->h_ctrl->err & 1) w += " edge id out of range;";
        if (b->h_ctrl->err & 2) w += " capacity outside [0, " + std::to_string(b->cap_limit[i]) + "];";
        if (b->h_ctrl->err & 4) w += " duplicate edge id;";
        return bfail(b, MF_EINVAL, "update batch rejected (capacities unchanged):" + w);
    }
    return MF_OK;
}

}  // extern "C"
