// Serving runtime (mf_server_* in include/mf.h): resident graphs that take
// asynchronous update requests.
//
// * Admission: a graph is admitted only while the device bytes reserved for
//   all resident graphs (mf_estimate_device_bytes plus batch staging) stay
//   within the server's budget.
// * Requests: validated and copied on submit, then queued FIFO per graph.
// * Group commit: a worker takes every pending request of one graph (up to a
//   request and an edge limit), merges them into one set in which the latest
//   request wins for an edge (the capacities are absolute, so applying the
//   merged set equals applying the requests one after the other), and runs one
//   dynamic repair (mf_apply_updates) for all of them.  Each request then
//   receives the flow value and the graph's version (requests applied so far)
//   after that commit.
// * Several workers drive different graphs at the same time; each graph's
//   handle has its own stream, so their kernels overlap on the device.  A
//   graph's persistent solve kernel is a cooperative grid whose workgroups
//   must all be resident at once; a commit starts only while the grids in
//   flight leave room for its grid (workgroup slots of the device), so
//   concurrent tenants never starve one another's grid barriers.
// * Requests are admitted by memory: the queued requests' bytes stay within
//   max_pending_bytes (else MF_EBUSY, nothing queued), and a request may not
//   exceed the edges one commit stages (max_group_edges), so the staging
//   reserved with the graph always suffices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/mf.h"
#include "mf_internal.h"

namespace {

thread_local std::string g_server_error;

int sfail(int code, const std::string &msg) {
    g_server_error = msg;
    return code;
}

struct Request {
    int64_t id = 0;
    int64_t seq = 0;
    std::vector<int64_t> ids;
    std::vector<int32_t> caps;
    double submit_ms = 0;
};

struct GraphSlot {
    mf_handle_t *h = nullptr;
    int32_t grid = 1;  // workgroups of its solve kernel
    int32_t n = 0;
    int64_t m = 0;
    int32_t cap_limit = 0;
    int64_t reserved = 0;
    int64_t next_seq = 1;
    int64_t version = 0;
    int64_t value = 0;
    std::deque<Request> pending;
    bool busy = false;
    bool removing = false;
    bool alive = true;
    int failed = MF_OK;  // status of a failed commit; later requests fail with MF_ESTATE
    std::string failure;
};

}  // namespace

struct mf_server {
    mf_server_opts_t opts{};
    std::mutex mu;
    std::condition_variable cv_work;  // workers wait for a graph with pending requests
    std::condition_variable cv_done;  // callers wait for results
    std::vector<std::unique_ptr<GraphSlot>> graphs;
    std::unordered_map<int64_t, mf_result_t> done;
    std::unordered_map<int64_t, int32_t> open;  // request -> graph, until committed
    int64_t next_request = 1;
    int64_t reserved = 0;
    int64_t budget = 0;
    int64_t commits = 0;
    int64_t pending_bytes = 0;  // host bytes held by queued requests
    int32_t slots = 0;          // workgroups the device holds at once for a solve kernel
    int32_t slots_used = 0;     // workgroups of the commits in flight
    int64_t resumed = 0;        // commits finished by mf_resume after an aborted launch
    bool stop = false;
    std::vector<std::thread> workers;
    std::chrono::steady_clock::time_point t0;
};

namespace {

double now_ms(const mf_server_t *s) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - s->t0).count();
}

// Bytes a queued request holds (ids and capacities).
int64_t request_bytes(int64_t k) { return 12 * k; }

// The idle graph whose oldest pending request is the oldest overall, among
// those whose solve grid fits the workgroup slots left.
GraphSlot *choose(mf_server_t *s, int32_t *gid) {
    GraphSlot *best = nullptr;
    for (size_t i = 0; i < s->graphs.size(); ++i) {
        GraphSlot *g = s->graphs[i].get();
        if (!g->alive || g->busy || g->pending.empty()) continue;
        if (s->slots_used + g->grid > s->slots) continue;
        if (!best || g->pending.front().id < best->pending.front().id) {
            best = g;
            *gid = (int32_t)i;
        }
    }
    return best;
}

void worker_main(mf_server_t *s) {
    (void)hipSetDevice(s->opts.device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        GraphSlot *g = nullptr;
        int32_t gid = -1;
        s->cv_work.wait(lk, [&] {
            g = choose(s, &gid);
            return g != nullptr || s->stop;
        });
        if (!g) return;  // stop, and nothing left to commit
        std::vector<Request> group;
        int64_t edges = 0;
        while (!g->pending.empty() && (int32_t)group.size() < s->opts.max_group_requests) {
            Request &r = g->pending.front();
            if (!group.empty() && edges + (int64_t)r.ids.size() > s->opts.max_group_edges) break;
            edges += (int64_t)r.ids.size();
            group.push_back(std::move(r));
            g->pending.pop_front();
        }
        g->busy = true;
        s->slots_used += g->grid;
        const int failed_before = g->failed;
        lk.unlock();

        const double start = now_ms(s);
        int rc = MF_OK;
        int64_t value = 0;
        std::string why;
        if (failed_before != MF_OK) {
            rc = MF_ESTATE;
        } else {
            // merge: position of the latest request that names each edge wins
            std::vector<std::pair<int64_t, int64_t>> key;  // (edge id, -order)
            key.reserve((size_t)edges);
            std::vector<int32_t> flat;
            flat.reserve((size_t)edges);
            int64_t pos = 0;
            for (const Request &r : group)
                for (size_t j = 0; j < r.ids.size(); ++j, ++pos) {
                    key.emplace_back(r.ids[j], -pos);
                    flat.push_back(r.caps[j]);
                }
            std::sort(key.begin(), key.end());
            std::vector<int64_t> ids;
            std::vector<int32_t> caps;
            ids.reserve(key.size());
            caps.reserve(key.size());
            for (size_t j = 0; j < key.size(); ++j) {
                if (j > 0 && key[j].first == key[j - 1].first) continue;  // an older write of the same edge
                ids.push_back(key[j].first);
                caps.push_back(flat[(size_t)(-key[j].second)]);
            }
            rc = mf_apply_updates(g->h, ids.data(), caps.data(), (int64_t)ids.size());
            // a launch that ran out of its time budget or whose barrier wait
            // ran out leaves a valid partial state: finish it from there
            for (int tries = 0; tries < 2 && (rc == MF_ETIMEOUT || rc == MF_EDEVICE); ++tries) {
                const int r2 = mf_resume(g->h);
                if (r2 == MF_OK) {
                    std::lock_guard<std::mutex> lk2(s->mu);
                    s->resumed++;
                }
                rc = r2;
            }
            if (rc == MF_OK) rc = mf_flow_value(g->h, &value);
            if (rc != MF_OK) why = mf_last_error(g->h);
        }
        const double end = now_ms(s);

        lk.lock();
        if (rc == MF_OK) {
            g->version += (int64_t)group.size();
            g->value = value;
        } else if (g->failed == MF_OK) {
            g->failed = rc;
            g->failure = why;
        }
        s->commits++;
        s->slots_used -= g->grid;
        for (const Request &r : group) {
            s->pending_bytes -= request_bytes((int64_t)r.ids.size());
            mf_result_t res;
            std::memset(&res, 0, sizeof(res));
            res.status = rc;
            res.graph = gid;
            res.request = r.id;
            res.value = rc == MF_OK ? value : 0;
            res.version = g->version;
            res.seq = r.seq;
            res.group_size = (int64_t)group.size();
            res.submit_ms = r.submit_ms;
            res.start_ms = start;
            res.done_ms = end;
            s->done[r.id] = res;
            s->open.erase(r.id);
        }
        g->busy = false;
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

bool quiet(const mf_server_t *s, const GraphSlot *only) {
    for (const auto &g : s->graphs) {
        if (only && g.get() != only) continue;
        if (g->busy || !g->pending.empty()) return false;
    }
    return true;
}

}  // namespace

extern "C" {

MF_API void mf_server_default_opts(mf_server_opts_t *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->workers = 4;
    o->max_group_edges = 1 << 20;
    o->max_group_requests = 64;
    o->max_pending_bytes = (int64_t)1 << 30;
}

MF_API const char *mf_server_last_error(void) { return g_server_error.c_str(); }

MF_API int mf_server_create(const mf_server_opts_t *opts, mf_server_t **out) {
    if (!out) return sfail(MF_EINVAL, "out is NULL");
    *out = nullptr;
    mf_server_opts_t o;
    mf_server_default_opts(&o);
    if (opts) o = *opts;
    if (o.device < 0) return sfail(MF_EINVAL, "device must be >= 0");
    if (o.workers < 1 || o.workers > 64) return sfail(MF_EINVAL, "workers must be in [1, 64]");
    if (o.memory_budget < 0) return sfail(MF_EINVAL, "memory_budget must be >= 0");
    if (o.max_group_edges < 1) return sfail(MF_EINVAL, "max_group_edges must be >= 1");
    if (o.max_group_requests < 1) return sfail(MF_EINVAL, "max_group_requests must be >= 1");
    if (o.max_pending_bytes < 0) return sfail(MF_EINVAL, "max_pending_bytes must be >= 0");
    if (o.max_pending_bytes == 0) o.max_pending_bytes = (int64_t)1 << 30;
    if (o.reserved0) return sfail(MF_EINVAL, "reserved fields must be zero");
    for (int32_t r : o.reserved)
        if (r) return sfail(MF_EINVAL, "reserved fields must be zero");
    hipError_t e = hipSetDevice(o.device);
    if (e != hipSuccess) return sfail(MF_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    int64_t budget = o.memory_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if ((e = hipMemGetInfo(&fr, &tot)) != hipSuccess)
            return sfail(MF_EDEVICE, std::string("hipMemGetInfo: ") + hipGetErrorString(e));
        budget = (int64_t)(0.9 * (double)fr);
    }
    int slots = 0;
    if ((e = mf::loop_max_coresident(o.device, &slots)) != hipSuccess)
        return sfail(MF_EDEVICE, std::string("occupancy query: ") + hipGetErrorString(e));
    mf_server_t *s = new (std::nothrow) mf_server_t();
    if (!s) return sfail(MF_ENOMEM, "host allocation failed");
    s->opts = o;
    s->budget = budget;
    s->slots = std::max(1, slots);
    s->t0 = std::chrono::steady_clock::now();
    try {
        for (int i = 0; i < o.workers; ++i) s->workers.emplace_back(worker_main, s);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        for (auto &t : s->workers) t.join();
        delete s;
        return sfail(MF_ENOMEM, "could not start worker threads");
    }
    *out = s;
    return MF_OK;
}

MF_API void mf_server_destroy(mf_server_t *s) {
    if (!s) return;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return quiet(s, nullptr); });
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    for (auto &g : s->graphs)
        if (g->h) mf_destroy(g->h);
    delete s;
}

MF_API int mf_server_add_graph(mf_server_t *s, const mf_csr_t *g, const int32_t *cap, int32_t src, int32_t sink,
                               const mf_opts_t *opts, int32_t *graph_id, int64_t *value) {
    if (!s || !g || !graph_id) return sfail(MF_EINVAL, "null argument");
    const int64_t est = mf_estimate_device_bytes(g->n, g->m);
    if (est < 0) return sfail(MF_EINVAL, "negative graph size");
    // the handle's batch staging: at least min(m, 2^17) updates (its floor), up
    // to a commit's worth of edges, 12 bytes each plus the 64-byte header
    const int64_t staged = std::max<int64_t>(std::min<int64_t>(g->m, s->opts.max_group_edges),
                                             std::min<int64_t>(std::max<int64_t>(g->m, 1), 1 << 17));
    const int64_t need = est + 12 * staged + 64;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->reserved + need > s->budget)
            return sfail(MF_ENOMEM, "admission: the graph needs about " + std::to_string(need) +
                                        " device bytes; " + std::to_string(s->reserved) + " of " +
                                        std::to_string(s->budget) + " are reserved");
        s->reserved += need;
    }
    auto unreserve = [&] {
        std::lock_guard<std::mutex> lk(s->mu);
        s->reserved -= need;
    };
    mf_opts_t o;
    mf_default_opts(&o);
    if (opts) o = *opts;
    o.device = s->opts.device;
    mf_handle_t *h = nullptr;
    int rc = mf_create(g, cap, src, sink, &o, &h);
    if (rc != MF_OK) {
        std::string why = mf_last_error(nullptr);
        unreserve();
        return sfail(rc, why);
    }
    int64_t v = 0;
    int32_t lim = 0;
    mf_stats_t st{};
    rc = mf_solve(h);
    if (rc == MF_OK) rc = mf_flow_value(h, &v);
    if (rc == MF_OK) rc = mf_cap_limit(h, &lim);
    if (rc == MF_OK) rc = mf_get_stats(h, &st);
    if (rc != MF_OK) {
        std::string why = mf_last_error(h);
        mf_destroy(h);
        unreserve();
        return sfail(rc, why);
    }
    std::unique_ptr<GraphSlot> slot(new (std::nothrow) GraphSlot());
    if (!slot) {
        mf_destroy(h);
        unreserve();
        return sfail(MF_ENOMEM, "host allocation failed");
    }
    slot->h = h;
    slot->grid = (int32_t)std::max<int64_t>(1, st.grid_blocks);
    slot->n = g->n;
    slot->m = g->m;
    slot->cap_limit = lim;
    slot->reserved = need;
    slot->value = v;
    std::lock_guard<std::mutex> lk(s->mu);
    s->graphs.push_back(std::move(slot));
    *graph_id = (int32_t)(s->graphs.size() - 1);
    if (value) *value = v;
    return MF_OK;
}

MF_API int mf_server_remove_graph(mf_server_t *s, int32_t graph_id) {
    if (!s) return sfail(MF_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size() || !s->graphs[graph_id]->alive)
        return sfail(MF_EINVAL, "unknown graph");
    GraphSlot *g = s->graphs[graph_id].get();
    if (g->removing) return sfail(MF_ESTATE, "graph is being removed");
    g->removing = true;  // no new submissions
    s->cv_done.wait(lk, [&] { return quiet(s, g); });
    g->alive = false;
    mf_handle_t *h = g->h;
    g->h = nullptr;
    s->reserved -= g->reserved;
    lk.unlock();
    mf_destroy(h);
    return MF_OK;
}

MF_API int mf_server_submit(mf_server_t *s, int32_t graph_id, const int64_t *edge_ids, const int32_t *new_caps,
                            int64_t k, int64_t *request_id) {
    if (!s || !request_id) return sfail(MF_EINVAL, "null argument");
    if (k < 0) return sfail(MF_EINVAL, "k must be >= 0");
    if (k > 0 && (!edge_ids || !new_caps)) return sfail(MF_EINVAL, "null batch arrays");
    int64_t m = 0;
    int32_t lim = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size() || !s->graphs[graph_id]->alive ||
            s->graphs[graph_id]->removing)
            return sfail(MF_EINVAL, "unknown graph");
        m = s->graphs[graph_id]->m;
        lim = s->graphs[graph_id]->cap_limit;
    }
    if (k > m) return sfail(MF_EINVAL, "batch size k must be in [0, m]");
    if (k > s->opts.max_group_edges)
        return sfail(MF_EINVAL, "request of " + std::to_string(k) + " edges above the server's max_group_edges (" +
                                    std::to_string(s->opts.max_group_edges) + ")");
    Request r;
    try {
        r.ids.assign(edge_ids, edge_ids + k);
        r.caps.assign(new_caps, new_caps + k);
    } catch (const std::bad_alloc &) {
        return sfail(MF_ENOMEM, "host allocation failed");
    }
    for (int64_t j = 0; j < k; ++j) {
        if (r.ids[j] < 0 || r.ids[j] >= m) return sfail(MF_EINVAL, "edge id out of range");
        if (r.caps[j] < 0 || r.caps[j] > lim)
            return sfail(MF_EINVAL, "capacity outside [0, " + std::to_string(lim) + "]");
    }
    {
        std::vector<int64_t> sorted(r.ids);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return sfail(MF_EINVAL, "duplicate edge id in one request (a batch is a set)");
    }
    std::lock_guard<std::mutex> lk(s->mu);
    GraphSlot *g = s->graphs[graph_id].get();
    if (!g->alive || g->removing) return sfail(MF_EINVAL, "unknown graph");
    if (s->pending_bytes + request_bytes(k) > s->opts.max_pending_bytes)
        return sfail(MF_EBUSY, "admission: queued requests hold " + std::to_string(s->pending_bytes) + " of " +
                                   std::to_string(s->opts.max_pending_bytes) +
                                   " bytes; retry once results are taken");
    s->pending_bytes += request_bytes(k);
    r.id = s->next_request++;
    r.seq = g->next_seq++;
    r.submit_ms = now_ms(s);
    *request_id = r.id;
    s->open[r.id] = graph_id;
    g->pending.push_back(std::move(r));
    s->cv_work.notify_one();
    return MF_OK;
}

MF_API int mf_server_poll(mf_server_t *s, int64_t request_id, mf_result_t *out) {
    if (!s || !out) return sfail(MF_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->done.find(request_id);
    if (it != s->done.end()) {
        *out = it->second;
        return MF_OK;
    }
    if (s->open.count(request_id)) return MF_EPENDING;
    return sfail(MF_EINVAL, "unknown request");
}

MF_API int mf_server_wait(mf_server_t *s, int64_t request_id, mf_result_t *out) {
    if (!s || !out) return sfail(MF_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (!s->done.count(request_id) && !s->open.count(request_id)) return sfail(MF_EINVAL, "unknown request");
    s->cv_done.wait(lk, [&] { return s->done.count(request_id) != 0; });
    *out = s->done[request_id];
    return MF_OK;
}

MF_API int mf_server_release(mf_server_t *s, int64_t request_id) {
    if (!s) return sfail(MF_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->done.erase(request_id)) return MF_OK;
    if (s->open.count(request_id)) return MF_EPENDING;
    return sfail(MF_EINVAL, "unknown request");
}

MF_API int mf_server_drain(mf_server_t *s) {
    if (!s) return sfail(MF_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return quiet(s, nullptr); });
    return MF_OK;
}

MF_API int mf_server_graph_info(mf_server_t *s, int32_t graph_id, int64_t *version, int64_t *value) {
    if (!s) return sfail(MF_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size() || !s->graphs[graph_id]->alive)
        return sfail(MF_EINVAL, "unknown graph");
    const GraphSlot *g = s->graphs[graph_id].get();
    if (g->failed != MF_OK) return sfail(MF_ESTATE, "graph failed: " + g->failure);
    if (version) *version = g->version;
    if (value) *value = g->value;
    return MF_OK;
}

MF_API int mf_server_memory(mf_server_t *s, int64_t *reserved, int64_t *budget, int64_t *commits) {
    if (!s) return sfail(MF_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (reserved) *reserved = s->reserved;
    if (budget) *budget = s->budget;
    if (commits) *commits = s->commits;
    return MF_OK;
}

MF_API int mf_server_load(mf_server_t *s, int64_t *pending_bytes, int32_t *slots_used, int32_t *slots,
                          int64_t *resumed) {
    if (!s) return sfail(MF_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (pending_bytes) *pending_bytes = s->pending_bytes;
    if (slots_used) *slots_used = s->slots_used;
    if (slots) *slots = s->slots;
    if (resumed) *resumed = s->resumed;
    return MF_OK;
}

}  // extern "C"
