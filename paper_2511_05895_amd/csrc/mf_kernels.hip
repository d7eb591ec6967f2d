// gfx950 kernels for push-relabel max-flow with dynamic capacity updates.
//
// Method: Kannappan, Kumar and Nasre, "Efficient Dynamic MaxFlow Computation
// on GPUs" (arXiv 2511.05895).  Static solve: Sec. 3, Alg. 1-3.  Dynamic
// repair: Sec. 4.1, Alg. 4-5.  Execution: data-driven worklists (Sec. 5.3) or
// topology-driven sweeps (Sec. 5.2) over a bi-directional CSR (Sec. 5.1).
//
// Design for CDNA4 (not the paper's CUDA design):
//  * One persistent kernel runs the whole solve loop (global relabel -> active
//    test -> push/relabel -> invalid-edge removal) with grid-wide barriers
//    between phases, so no host round trip happens inside a solve.  With one
//    workgroup the barrier is a plain workgroup barrier.
//  * The backward BFS expands frontier items of at most kChunk arcs with a
//    wavefront-wide load-balanced scan (prefix sum over item lengths, each lane
//    takes one arc), so a hub's arcs spread over many wavefronts and low-degree
//    frontiers still fill all 64 lanes.  The active worklist is built during the
//    same BFS (a discovered vertex with positive excess is active), with
//    ballot/mbcnt compaction and one atomic per wavefront, or per workgroup
//    (LDS staging) on large levels; small frontiers are expanded by one
//    workgroup alone, level after level, without grid barriers.
//  * Push/relabel gives a group of lanes to a vertex with at most kLightMaxDeg
//    arcs, a wavefront to a longer list and a workgroup to a huge one.  Every
//    counter or list that all workgroups share is updated once per workgroup
//    and round (LDS sums and staging): atomics on one address serialise, and a
//    round has thousands of wavefronts.
//  * Memory ordering: only the owner lowers c_f of its arcs and its own excess
//    during a sweep; others only raise them.  The first cycle of a visit takes
//    an arc's residual from the {head, residual} record it loads anyway (read
//    after the round's barrier, so at most stale-low); later cycles of the
//    same visit, and every excess, use device-scope atomic loads, so a push
//    never exceeds the latest residual or excess.  Heights may be stale, which
//    the method tolerates (Sec. 3: invalid edges are repaired by
//    RemoveInvalidEdges).
#include "mf_internal.h"

#include <mutex>

namespace mf {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Scoped atomics.  The one-workgroup solve kernel works at workgroup scope
// (atomics resolve in the compute unit's own caches); the multi-workgroup
// kernel and the update kernels need device scope, because gfx950 spreads a
// grid over eight XCDs with separate L2 caches.
constexpr int kAgent = __HIP_MEMORY_SCOPE_AGENT;
constexpr int kGroup = __HIP_MEMORY_SCOPE_WORKGROUP;

template <int SC>
__device__ __forceinline__ int32_t ld(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, SC);
}
template <int SC>
__device__ __forceinline__ int64_t ld(const int64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, SC);
}
template <int SC>
__device__ __forceinline__ void add(int32_t *p, int32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, SC);
}
template <int SC>
__device__ __forceinline__ void add(int64_t *p, int64_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, SC);
}
template <int SC>
__device__ __forceinline__ int32_t fetch_add(int32_t *p, int32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, SC);
}
template <int SC>
__device__ __forceinline__ int64_t fetch_add(int64_t *p, int64_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, SC);
}
template <int SC>
__device__ __forceinline__ int32_t xchg(int32_t *p, int32_t v) {
    return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, SC);
}
template <int SC>
__device__ __forceinline__ bool cas(int32_t *p, int32_t expected, int32_t desired) {
    return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                                __ATOMIC_RELAXED, SC);
}

// residual capacity field of arc a
__device__ __forceinline__ int32_t *cf_ptr(int2 *arc, int32_t a) {
    return reinterpret_cast<int32_t *>(arc) + 2 * (int64_t)a + 1;
}

__device__ __forceinline__ int wave_incl_scan(int x) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ int64_t wave_incl_scan64(int64_t x) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(x, d, 64);
        if (lane_id() >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ int64_t wave_sum(int64_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ int mask_rank(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Reserve one slot per lane with pred; one atomic per wavefront.  Every lane
// of the wavefront must call it.  Returns the slot, or -1 without pred.
template <int SC>
__device__ __forceinline__ int wave_append1(int32_t *counter, bool pred) {
    uint64_t mask = __ballot(pred);
    if (mask == 0) return -1;
    int leader = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane_id() == leader) base = fetch_add<SC>(counter, __popcll(mask));
    base = __shfl(base, leader, 64);
    return pred ? base + mask_rank(mask) : -1;
}

// Reserve c slots per lane (c >= 0); one atomic per wavefront.  Every lane must
// call it.  Returns the first slot of this lane's range.
template <int SC>
__device__ __forceinline__ int wave_appendn(int32_t *counter, int c) {
    int incl = wave_incl_scan(c);
    int total = __shfl(incl, 63, 64);
    if (total == 0) return 0;
    int base = 0;
    if (lane_id() == 63) base = fetch_add<SC>(counter, total);
    base = __shfl(base, 63, 64);
    return base + incl - c;
}

__device__ __forceinline__ int n_items(int deg) { return (deg + kChunk - 1) / kChunk; }

// Appends of a round to the next round's list are staged per workgroup in
// LDS (up to kStageCap light and kStageCap long-list vertices) and reserved
// with one atomic per workgroup and list at the end of the round; beyond
// that, or without a stage, a lane appends on its own.  A vertex enters a
// list at most once (mark[]), so no list outgrows its |V| slots.
constexpr int kStageCap = 1024;

// A value every lane of the wavefront holds alike (read after a barrier),
// moved to a scalar register so it does not occupy a vector register.
__device__ __forceinline__ int32_t uniform(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uniform(int64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The workgroups that run one solve loop together: ranks 0..size-1.  Either
// the whole grid of a cooperative launch, or a single workgroup of a batched
// launch (then every barrier is a workgroup barrier).
struct Team {
    int rank, size;
    __device__ int64_t tid() const { return (int64_t)rank * blockDim.x + threadIdx.x; }
    __device__ int64_t nthreads() const { return (int64_t)size * blockDim.x; }
    __device__ int64_t wave() const { return (int64_t)rank * (blockDim.x >> 6) + (threadIdx.x >> 6); }
    __device__ int64_t nwaves() const { return (int64_t)size * (blockDim.x >> 6); }
};

// Barrier of a team with a bounded wait.  Arrivals count up monotonic
// counters (cleared before every launch): barrier number `epoch` (0, 1, ...)
// is complete once the top counter reaches (epoch + 1) * size, or, for a team
// of 2 * kBarGroups workgroups or more, (epoch + 1) * kBarGroups, one count per
// group whose own counter reached (epoch + 1) * its size.  One release fence before
// the arrival and one acquire fence after the wait; the polls themselves are
// relaxed loads, so waiting does not keep invalidating the caches that the
// team's other workgroups are still working from.  Returns false when the
// wait ran out (wall clock, `limit` ticks) or another workgroup aborted; the
// caller must then leave the kernel, so every workgroup ends even if
// co-residency ever failed.  Every thread of every workgroup of the team calls
// it with the same epoch, which it advances.
__device__ bool grid_barrier(Ctrl *c, const Team &tm, uint32_t &epoch, int64_t limit) {
    if (tm.size == 1) {
        __syncthreads();
        return true;
    }
    __shared__ int s_ok;
    __syncthreads();
    const uint32_t e1 = epoch + 1u;
    ++epoch;
    if (threadIdx.x == 0) {
        int ok = 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        // Arrivals: a team of 2 * kBarGroups workgroups or more arrives in
        // kBarGroups groups (rank mod kBarGroups), each on a counter of its own
        // line, and the last arrival of a group (the one that completes its
        // count) acquires the group's writes and releases them on to the top
        // counter, which every workgroup polls.  Arrivals on one word
        // serialise; this way each word takes a group's share of them.
        const int G = tm.size < 2 * kBarGroups ? 1 : kBarGroups;
        uint32_t target, before;
        if (G == 1) {
            target = e1 * (uint32_t)tm.size;
            before = __hip_atomic_fetch_add(&c->bar_count.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const int gid = tm.rank % G;
            const uint32_t ng = (uint32_t)((tm.size - gid + G - 1) / G);
            target = e1 * (uint32_t)G;
            before = target - 2u;  // not the last of its group: wait
            if (__hip_atomic_fetch_add(&c->bar_group[gid].v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u ==
                e1 * ng) {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                before = __hip_atomic_fetch_add(&c->bar_count.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if ((int32_t)(before + 1u - target) < 0) {
            const uint64_t tw = wall_clock64();
            uint32_t spins = 0;
            while ((int32_t)(__hip_atomic_load(&c->bar_count.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                             target) < 0) {
                __builtin_amdgcn_s_sleep(1);
                if ((++spins & 255u) == 0) {
                    if (__hip_atomic_load(&c->abort.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        ok = 0;
                        break;
                    }
                    if ((int64_t)(wall_clock64() - tw) > limit) {
                        __hip_atomic_store(&c->abort.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Per-thread event counters (32-bit), summed into the 64-bit Ctrl::stat at the
// end of every loop round and of the kernel, then cleared.
struct Tally {
    uint32_t bfs_v = 0, bfs_a = 0, pr_cyc = 0, pr_a = 0, push = 0, relabel = 0, rie_a = 0, rie_sat = 0;
    int64_t deliv = 0;  // excess this lane delivered into deficient vertices (per round)
};

// Every thread of the workgroup must call it.
template <int SC>
__device__ void flush_tally(Ctrl *c, Tally &t) {
    __shared__ int64_t s_acc[8];
    if (threadIdx.x < 8) s_acc[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t v[8] = {t.bfs_v, t.bfs_a, t.pr_cyc, t.pr_a, t.push, t.relabel, t.rie_a, t.rie_sat};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t w = wave_sum((int64_t)v[i]);
        if (lane_id() == 0 && w) atomicAdd((unsigned long long *)&s_acc[i], (unsigned long long)w);
    }
    __syncthreads();
    const int slot[8] = {kStBfsVertices, kStBfsArcs, kStPrCycles, kStPrArcs,
                         kStPushes,      kStRelabels, kStRieArcs, kStRieSat};
    if (threadIdx.x < 8 && s_acc[threadIdx.x]) add<SC>(&c->stat[slot[threadIdx.x]], s_acc[threadIdx.x]);
    t = Tally{};
}

// ---------------------------------------------------------------------------
// Global relabel (Alg. 4 height reset + BFS_Backward)
// ---------------------------------------------------------------------------

// Height reset: t and every deficient vertex other than s are roots (height
// 0); all others get |V|.  Roots become the level-0 frontier.  With part
// tags, only vertices of the wanted part can be roots, and with part_restrict
// the heights of the other vertices are left alone.
template <int SC>
__device__ void bfs_roots(const DevGraph &g, const Team &tm, bool counts, bool feats, bool track, Tally &tl) {
    const int64_t gtid = tm.tid();
    const int64_t stride = tm.nthreads();
    const int64_t nr = ((int64_t)g.n + 63) & ~63ll;
    for (int64_t i = gtid; i < nr; i += stride) {
        const int v = (int)i;
        bool root = false;
        int beg = 0, end = 0;
        if (i < g.n) {
            const bool mine = !g.part || g.part[v] == g.part_want;
            if (mine || !g.part_restrict) {
                root = mine && ((v == g.t) || (v != g.s && g.e[v] < 0));
                g.h[v] = root ? 0 : g.n;
            }
            if (root) {
                beg = g.row_ptr[v];
                end = g.row_ptr[v + 1];
            }
        }
        const int c = root ? n_items(end - beg) : 0;
        const int nroot = (int)wave_sum((int64_t)root);
        if (counts && lane_id() == 0 && nroot) add<SC>(&g.hcount[0], nroot);
        if (feats && lane_id() == 0 && nroot) add<SC>(&g.ctrl->feat_reached, nroot);
        if (track && nroot) {
            const int64_t ra = wave_sum((int64_t)(end - beg));
            if (lane_id() == 0) {
                add<SC>(&g.ctrl->qverts[0], nroot);
                add<SC>(&g.ctrl->qarcs[0], ra);
            }
        }
        const int base = wave_appendn<SC>(&g.ctrl->qcount[0], c);
        for (int j = 0; j < c; ++j)
            g.q[0][base + j] = make_int2(beg + j * kChunk, min(beg + (j + 1) * kChunk, end));
        tl.bfs_v += root;
    }
}

// Features of the learned schedule: excess sum of the active vertices a BFS
// finds and their count per bin of floor(log2 e) / 4.  Wave-uniform calls.
template <int SC>
__device__ __forceinline__ void feature_tally(Ctrl *c, bool active, int64_t ev) {
    if (__ballot(active) == 0) return;
    const int64_t es = wave_sum(active ? ev : (int64_t)0);
    const int bin = active ? min(7, (63 - __clzll((unsigned long long)ev)) >> 2) : -1;
    if (lane_id() == 0) add<SC>(&c->feat_esum, es);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int cb = __popcll(__ballot(bin == b));
        if (lane_id() == 0 && cb) add<SC>(&c->feat_hist[b], cb);
    }
}

// Per-workgroup staging of a large BFS level's output in LDS: frontier items
// and active-list entries are reserved in LDS first and the workgroup then
// reserves its whole share of each global list with one atomic, instead of
// every wavefront step hitting the same few global counters.  A reservation
// that does not fit goes to the global list directly, so nothing is lost and
// no slot stays unwritten.
constexpr int kBfsStageItems = 2048;
// frontier size (items) from which a level stages its output
constexpr int kBfsStageMin = 1024;
struct BfsStage {
    int2 items[kBfsStageItems];
    int32_t light[kStageCap], heavy[kStageCap];
    int32_t cnt[4];  // items, light, heavy, discovered vertices of this level
    int32_t res[6];  // the level's flush: global bases, then counts, of items, light, heavy
    int64_t arcs;    // arcs of the vertices this level discovered (direction rule)
    // the direction rule's tallies of a level that is not staged (vertices
    // and arcs discovered), added to the global counters once per workgroup:
    // per wavefront step they would queue behind the frontier reservations
    // on the same cache line
    int32_t tverts;
    int64_t tarcs;
};

// Reserve k slots of an LDS counter if they fit under cap (no partial
// reservation); returns the first slot or -1.
__device__ __forceinline__ int stage_reserve(int32_t *ctr, int k, int cap) {
    int old = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (;;) {
        if (old + k > cap) return -1;
        if (__hip_atomic_compare_exchange_strong(ctr, &old, old + k, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP))
            return old;
    }
}

// Output of one 64-lane BFS step (every lane of the wavefront calls it): a
// lane that discovered v (disc; its arc range [vbeg, vend) and excess ev)
// appends v's frontier items for the next level and, when v is active (A of
// Alg. 1: e > 0 and h < |V|, t excluded), v to the active worklist.  The
// frontier items, both halves of the active list through one packed 64-bit
// counter {light, heavy}, and the level's vertex and arc tallies are reserved
// by one lane, back to back so their round trips overlap, or in the
// workgroup's stage (st).  counts: per-height vertex counts (gap heuristic);
// feats: the schedule's features; track: vertices and arcs discovered per
// level (the direction rule of the BFS), tallied in tst when the level is not
// staged (null: straight to the global counters).
template <int SC>
__device__ __forceinline__ void bfs_emit(const DevGraph &g, int L, bool disc, int v, int vbeg, int vend, int64_t ev,
                                         bool feats, bool counts, bool track, BfsStage *st, BfsStage *tst,
                                         int2 *qout, int32_t *qout_count, Tally &tl) {
    const int lane = lane_id();
    const int n = g.n;
    bool active = false;
    if (disc) {
        active = (v != g.t) && ev > 0;
        tl.bfs_v++;
    } else {
        vbeg = vend = 0;
    }
    if (feats) feature_tally<SC>(g.ctrl, active, ev);
    const int vdeg = vend - vbeg;
    const int c = disc ? n_items(vdeg) : 0;
    const int cincl = wave_incl_scan(c);
    const int ctotal = __shfl(cincl, 63, 64);
    const bool light = active && vdeg <= kLightMaxDeg;
    const bool heavy = active && vdeg > kLightMaxDeg && vdeg <= kHugeDeg;
    const bool huge = active && vdeg > kHugeDeg;
    const uint64_t lm = __ballot(light), hm = __ballot(heavy);
    const int ndisc = counts || feats || track ? __popcll(__ballot(disc)) : 0;
    const int64_t darcs = track ? wave_sum((int64_t)vdeg) : 0;
    int qbase = 0, lsb = -1, hsb = -1, qsb = -1;
    int64_t lbase = 0;
    if (lane == 63) {
        const int nl = __popcll(lm), nh = __popcll(hm);
        if (st) {
            if (ctotal) qsb = stage_reserve(&st->cnt[0], ctotal, kBfsStageItems);
            if (nl) lsb = stage_reserve(&st->cnt[1], nl, kStageCap);
            if (nh) hsb = stage_reserve(&st->cnt[2], nh, kStageCap);
            if (ndisc) atomicAdd(&st->cnt[3], ndisc);
            if (darcs) atomicAdd(reinterpret_cast<unsigned long long *>(&st->arcs), (unsigned long long)darcs);
        } else if (ndisc) {
            if (counts) add<SC>(&g.hcount[L + 1], ndisc);
            if (feats) add<SC>(&g.ctrl->feat_reached, ndisc);
            if (track && tst) {
                atomicAdd(&tst->tverts, ndisc);
                atomicAdd(reinterpret_cast<unsigned long long *>(&tst->tarcs), (unsigned long long)darcs);
            } else if (track) {
                add<SC>(&g.ctrl->qverts[(L + 1) % 3], ndisc);
                add<SC>(&g.ctrl->qarcs[(L + 1) % 3], darcs);
            }
        }
        if (ctotal && qsb < 0) qbase = fetch_add<SC>(qout_count, ctotal);
        const int gl = lsb < 0 ? nl : 0, gh = hsb < 0 ? nh : 0;
        if (gl | gh)
            lbase = fetch_add<SC>(reinterpret_cast<int64_t *>(&g.ctrl->lst[0]), ((int64_t)gh << 32) | (int64_t)gl);
    }
    qbase = __shfl(qbase, 63, 64);
    lbase = __shfl(lbase, 63, 64);
    qsb = __shfl(qsb, 63, 64);
    lsb = __shfl(lsb, 63, 64);
    hsb = __shfl(hsb, 63, 64);
    int2 *qdst = qsb < 0 ? qout + qbase : st->items + qsb;
    const int qb = cincl - c;
    for (int k = 0; k < c; ++k) qdst[qb + k] = make_int2(vbeg + k * kChunk, min(vbeg + (k + 1) * kChunk, vend));
    if (light) {
        if (lsb < 0) g.list[0][(int)(uint32_t)lbase + mask_rank(lm)] = v;
        else st->light[lsb + mask_rank(lm)] = v;
    }
    if (heavy) {
        if (hsb < 0) g.list[0][n - 1 - ((int)(lbase >> 32) + mask_rank(hm))] = v;
        else st->heavy[hsb + mask_rank(hm)] = v;
    }
    const int su = wave_append1<SC>(&g.ctrl->lst[0].huge, huge);  // rare: hubs only
    if (huge) g.huge[0][su] = v;
}

// End of a staged BFS level: one reservation per list for the workgroup's
// staged output, then a coalesced copy (the stage counters start from zero
// again).  Every thread of the workgroup calls it.
template <int SC>
__device__ void bfs_flush(const DevGraph &g, int L, BfsStage *st, bool counts, bool feats, bool track, int2 *qout,
                          int32_t *qout_count) {
    const int n = g.n;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nq = st->cnt[0], nl = st->cnt[1], nh = st->cnt[2], nd = st->cnt[3];
        int64_t lb = 0;
        st->res[0] = nq ? fetch_add<SC>(qout_count, nq) : 0;
        if (nl | nh)
            lb = fetch_add<SC>(reinterpret_cast<int64_t *>(&g.ctrl->lst[0]), ((int64_t)nh << 32) | (int64_t)nl);
        if (nd && counts) add<SC>(&g.hcount[L + 1], nd);
        if (nd && feats) add<SC>(&g.ctrl->feat_reached, nd);
        if (nd && track) {
            add<SC>(&g.ctrl->qverts[(L + 1) % 3], nd);
            add<SC>(&g.ctrl->qarcs[(L + 1) % 3], st->arcs);
        }
        st->res[1] = (int)(uint32_t)lb;
        st->res[2] = (int)(lb >> 32);
        st->res[3] = nq;
        st->res[4] = nl;
        st->res[5] = nh;
        st->cnt[0] = st->cnt[1] = st->cnt[2] = st->cnt[3] = 0;
        st->arcs = 0;
    }
    __syncthreads();
    const int nq = st->res[3], nl = st->res[4], nh = st->res[5];
    for (int i = threadIdx.x; i < nq; i += blockDim.x) qout[st->res[0] + i] = st->items[i];
    for (int i = threadIdx.x; i < nl; i += blockDim.x) g.list[0][st->res[1] + i] = st->light[i];
    for (int i = threadIdx.x; i < nh; i += blockDim.x) g.list[0][n - 1 - (st->res[2] + i)] = st->heavy[i];
}

// End of a level that was not staged: the workgroup's direction tallies go to
// the global counters, one atomic each (every thread of the workgroup calls
// it; the next use of the tallies comes after a barrier).
template <int SC>
__device__ void bfs_tally_flush(const DevGraph &g, int L, BfsStage *tst) {
    __syncthreads();
    if (threadIdx.x == 0 && tst->tverts) {
        add<SC>(&g.ctrl->qverts[(L + 1) % 3], tst->tverts);
        add<SC>(&g.ctrl->qarcs[(L + 1) % 3], tst->tarcs);
        tst->tverts = 0;
        tst->tarcs = 0;
    }
}

// One BFS level, top-down: for every arc (w -> v) of a frontier item, v joins
// level L+1 when it is unvisited (height |V|), is not s, and has residual
// capacity toward w (the twin arc v -> w).  Newly reached vertices become
// frontier items of the next level; those with positive excess go to the
// active worklist (A of Alg. 1: e > 0 and h < |V|, s and t excluded).
// With a stage (st), the level's output is staged per workgroup and flushed
// at its end; counts: keep the per-height vertex counts (gap heuristic);
// feats: tally the schedule's features.  Every thread of the workgroup calls
// it.
template <int SC>
__device__ void bfs_level(const DevGraph &g, const Team &tm, int L, int cnt, bool feats, bool counts,
                          bool track, bool lazy, BfsStage *st, BfsStage *tst, Tally &tl) {
    const int2 *__restrict__ qin = g.q[L & 1];
    int2 *qout = g.q[(L + 1) & 1];
    int32_t *qout_count = &g.ctrl->qcount[(L + 1) % 3];
    const int lane = lane_id();
    const int64_t gwave = tm.wave();
    const int64_t nwaves = tm.nwaves();
    const int n = g.n;
    // items per wavefront: up to 64, fewer when the frontier is small, so
    // that every wavefront of the team takes part and each one expands as
    // few 64-arc steps one after another as possible
    const int64_t ipw = min((int64_t)64, max((int64_t)1, ((int64_t)cnt + nwaves - 1) / nwaves));
    for (int64_t base = gwave * ipw; base < cnt; base += nwaves * ipw) {
        const int64_t idx = base + lane;
        int beg = 0, len = 0;
        if (lane < ipw && idx < cnt) {
            const int2 it = qin[idx];  // arc range {first, end} of one item
            beg = it.x;
            len = it.y - it.x;
        }
        const int incl = wave_incl_scan(len);
        const int excl = incl - len;
        const int total = __shfl(incl, 63, 64);
        for (int off = 0; off < total; off += 64) {
            const int j = off + lane;
            // largest lane o with excl[o] <= j (that lane has len > 0)
            int o = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const int cand = o + step;
                const int ex = __shfl(excl, cand, 64);
                if (ex <= j) o = cand;
            }
            const int obeg = __shfl(beg, o, 64);
            const int oexcl = __shfl(excl, o, 64);
            bool disc = false;
            int v = -1, vbeg = 0, vend = 0;
            int64_t ev = 0;
            if (j < total) {
                const int a = obeg + (j - oexcl);
                // the head and the twin index come in one step, the head's height
                // and the twin's residual in the next; on a large level the
                // twin's residual (a gather from anywhere in the arc array) is
                // read only for heads not reached yet
                const int2 rec = g.arc[a];
                const int tw = g.twin[a];
                v = rec.x;
                const int hv = g.h[v];
                const bool cand = v != g.s && hv == n;
                int cft = 1;
                if (!lazy || cand) cft = g.arc[tw].y;
                tl.bfs_a++;
                if (cand && cft > 0 && (!g.part_restrict || g.part[v] == g.part_want)) {
                    // the candidate's row bounds and excess load alongside the
                    // compare-and-swap that decides the discovery
                    vbeg = g.row_ptr[v];
                    vend = g.row_ptr[v + 1];
                    ev = g.e[v];
                    disc = cas<SC>(&g.h[v], n, L + 1);
                }
            }
            bfs_emit<SC>(g, L, disc, v, vbeg, vend, ev, feats, counts, track, st, st ? nullptr : tst, qout,
                         qout_count, tl);
        }
    }
    if (st)
        bfs_flush<SC>(g, L, st, counts, feats, track, qout, qout_count);
    else if (track && tst)
        bfs_tally_flush<SC>(g, L, tst);
}

// One BFS level, bottom-up (the direction-optimising BFS): every vertex v
// not reached yet (height |V|, not s) looks through its own arcs (v -> w)
// for one with residual capacity whose head w is on level L, and joins level
// L+1 at the first it finds.  The same vertices join the level as in the
// top-down step, but only v's own arc records and the heads' heights are
// read (no gather of twin residuals), and a vertex stops at its first
// parent.  The team walks the static item list g.bu_items: a wavefront takes
// 64 items and runs through their remaining arcs 64 at a time (load-balanced
// scan), dropping an item as soon as its vertex has a parent.  Several items
// of one long list can find parents at once; the compare-and-swap on the
// height makes one of them the discovery.  Output as in the top-down step.
// Every thread of the workgroup calls it.
template <int SC>
__device__ void bfs_bottom_up(const DevGraph &g, const Team &tm, int L, bool feats, bool counts, BfsStage *st,
                              Tally &tl) {
    int2 *qout = g.q[(L + 1) & 1];
    int32_t *qout_count = &g.ctrl->qcount[(L + 1) % 3];
    const int lane = lane_id();
    const int n = g.n;
    const int64_t nb = g.n_bu_items;
    const int64_t nwaves = tm.nwaves();
    for (int64_t base = tm.wave() * 64; base < nb; base += nwaves * 64) {
        const int64_t idx = base + lane;
        int v = -1, beg = 0, len = 0;
        if (idx < nb) {
            const int4 it = g.bu_items[idx];
            if (it.x != g.s && g.h[it.x] == n) {
                v = it.x;
                beg = it.y;
                len = it.z - it.y;
            }
        }
        bool disc = false;
        for (;;) {
            const int incl = wave_incl_scan(len);
            const int total = __shfl(incl, 63, 64);
            if (total == 0) break;
            const int excl = incl - len;
            // largest lane o with excl[o] <= lane (that lane still has arcs)
            int o = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const int cand = o + step;
                const int ex = __shfl(excl, cand, 64);
                if (ex <= lane) o = cand;
            }
            const int obeg = __shfl(beg, o, 64);
            const int oexcl = __shfl(excl, o, 64);
            bool hit = false;
            if (lane < total) {
                const int2 r = g.arc[obeg + (lane - oexcl)];
                if (r.y > 0) hit = g.h[r.x] == L;
                tl.bfs_a++;
            }
            const uint64_t hm = __ballot(hit);
            // this lane's item owns the step's arcs [lo, hi)
            const int lo = min(excl, 64), hi = min(incl, 64);
            const int used = hi - lo;
            const bool found = used > 0 && ((hm >> lo) & (used == 64 ? ~0ull : ((1ull << used) - 1))) != 0;
            if (found) {
                len = 0;
                disc = cas<SC>(&g.h[v], n, L + 1);
            } else {
                beg += used;
                len -= used;
            }
        }
        int vbeg = 0, vend = 0;
        int64_t ev = 0;
        if (disc) {
            vbeg = g.row_ptr[v];
            vend = g.row_ptr[v + 1];
            ev = g.e[v];
        }
        bfs_emit<SC>(g, L, disc, v, vbeg, vend, ev, feats, counts, true, st, nullptr, qout, qout_count, tl);
    }
    if (st) bfs_flush<SC>(g, L, st, counts, feats, true, qout, qout_count);
}

// ---------------------------------------------------------------------------
// PushRelabel (Alg. 2), run in rounds
//
// A phase between two global relabels runs rounds.  Round r processes the
// vertices of list r; a vertex whose excess turns positive through a push, or
// that keeps excess after its visit, is added once (round-id stamp) to list
// r+1.  So excess can travel many arcs between global relabels instead of one
// arc per relabel.  A phase ends when a list is empty, or when the relabel
// budget or the round cap is spent; the next global relabel then restarts from
// exact heights.
//
// One cycle (KERNELCYCLES counts cycles) scans the arcs for the lowest residual
// neighbour height h^; if h(u) > h^ it pushes along the arcs at height h^ in
// arc order until the excess is gone (the paper's cycles pick the lowest arc,
// first in arc order, one push each; with the same h^ the next cycles would
// take exactly these arcs), otherwise it relabels h(u) = h^ + 1.
// ---------------------------------------------------------------------------

// Per-workgroup sums of a round's pushes by target vertex (LDS, direct
// mapped): a push into a vertex that holds a slot adds to the slot; the
// workgroup adds every slot to the target's excess with one atomic at the end
// of the round.  Pushes whose slot belongs to another vertex go straight to
// the excess.  Vertices of huge degree take pushes from thousands of others
// in one round, and this turns them into one atomic per workgroup.
constexpr int kCombineBits = 9;
constexpr int kCombine = 1 << kCombineBits;
struct Combine {
    int32_t key[kCombine];  // target vertex, or -1
    int64_t sum[kCombine];
};

struct RoundCtx {
    int32_t *next;     // list of the next round
    int32_t *next_huge;  // its huge-vertex list
    // the workgroup's staging of next-round appends and of first relabels
    // (LDS; null: append directly)
    int32_t *lbuf, *hbuf, *rbuf;
    int32_t *lcnt, *hcnt, *rcnt;
    Combine *comb;     // push sums of the workgroup (LDS), or null
    ListCtr *next_ctr;
    int32_t next_id;   // round id stamped into mark[] for that list
    int32_t phase_id;  // stamped into rmark[] on a vertex's first relabel
    bool use_gap;      // gap heuristic on
};

// Add v to the next round's list unless it is already there.
template <int SC>
__device__ __forceinline__ void list_add(const DevGraph &g, const RoundCtx &rc, int v) {
    const int deg = g.row_ptr[v + 1] - g.row_ptr[v];  // read alongside the exchange
    if (xchg<SC>(&g.mark[v], rc.next_id) == rc.next_id) return;
    if (deg <= kLightMaxDeg) {
        const int k = rc.lbuf ? atomicAdd(rc.lcnt, 1) : kStageCap;
        if (k < kStageCap) {
            rc.lbuf[k] = v;
        } else {
            const int slot = fetch_add<SC>(&rc.next_ctr->light, 1);
            rc.next[slot] = v;
        }
    } else if (deg <= kHugeDeg) {
        const int k = rc.hbuf ? atomicAdd(rc.hcnt, 1) : kStageCap;
        if (k < kStageCap) {
            rc.hbuf[k] = v;
        } else {
            const int slot = fetch_add<SC>(&rc.next_ctr->heavy, 1);
            rc.next[g.n - 1 - slot] = v;
        }
    } else {
        const int slot = fetch_add<SC>(&rc.next_ctr->huge, 1);
        rc.next_huge[slot] = v;
    }
}

// First relabel of u in this phase: remember u for RemoveInvalidEdges.  Only
// the one lane (or group) visiting u in a round touches rmark[u]; `stamp` is
// its value as read at the start of the visit.
template <int SC>
__device__ __forceinline__ void note_relabel(const DevGraph &g, const RoundCtx &rc, int u, int32_t &stamp) {
    if (stamp != rc.phase_id) {
        stamp = rc.phase_id;
        g.rmark[u] = rc.phase_id;
        const int k = rc.rbuf ? atomicAdd(rc.rcnt, 1) : kStageCap;
        if (k < kStageCap) {
            rc.rbuf[k] = u;
        } else {
            const int slot = fetch_add<SC>(&g.ctrl->nrelab, 1);
            g.relab[slot] = u;
        }
    }
}

// Relabel u from height ho to hmin + 1 (Alg. 2), keeping the per-height
// counts of the gap heuristic: a height left empty by this move means every
// vertex above it has no residual path to a root under a valid labelling
// (heights drop by at most one per residual arc), so heights above the lowest
// such gap count as |V|.  A count that hits zero only transiently (racing
// relabels) just deactivates vertices that the next global relabel restores.
// Returns the new height.
template <int SC>
__device__ __forceinline__ int relabel_to(const DevGraph &g, int u, int ho, int hmin, bool use_gap) {
    int hn = hmin + 1;
    if (use_gap) {
        const int gap = ld<SC>(&g.ctrl->gap);
        if (hn > gap) hn = g.n;
        if (hn < g.n) add<SC>(&g.hcount[hn], 1);
        if (fetch_add<SC>(&g.hcount[ho], -1) == 1 && ho > 0)
            __hip_atomic_fetch_min(&g.ctrl->gap, ho, __ATOMIC_RELAXED, SC);
    }
    if (hn > g.n) hn = g.n;
    g.h[u] = hn;
    return hn;
}

// Push d from u along arc a to v = head(a).  Residual capacity moves to the
// twin; excess moves from u to v except that the excess taken from u is
// subtracted by the caller (one atomic per visit chunk).
template <int SC>
__device__ __forceinline__ void push_arc(const DevGraph &g, const RoundCtx &rc, int a, int tw, int v,
                                         int32_t d, int64_t &to_t, Tally &tl) {
    add<SC>(cf_ptr(g.arc, a), -d);
    add<SC>(cf_ptr(g.arc, tw), d);
    if (v == g.t) {
        to_t += d;
    } else {
        if (rc.comb) {
            const int slot = (int)(((uint32_t)v * 2654435761u) >> (32 - kCombineBits));
            int k = rc.comb->key[slot];
            if (k < 0) {
                k = atomicCAS(&rc.comb->key[slot], -1, v);
                if (k < 0) k = v;
            }
            if (k == v) {
                atomicAdd(reinterpret_cast<unsigned long long *>(&rc.comb->sum[slot]), (unsigned long long)d);
                return;
            }
        }
        const int64_t old = fetch_add<SC>(&g.e[v], (int64_t)d);
        if (old < 0) tl.deliv += min((int64_t)d, -old);  // part of a deficit filled
        if (old <= 0 && old + d > 0 && v != g.s) list_add<SC>(g, rc, v);
    }
}

// Lowest residual neighbour height over the arcs first, first + stride, ...
// below last, and the residual capacity of the arcs at that height; four
// arcs per lane in flight.
__device__ __forceinline__ void scan_lowest(const DevGraph &g, int first, int last, int stride, int &hmin,
                                            int64_t &cmin) {
    int a = first;
    for (; a + 3 * stride < last; a += 4 * stride) {
        int2 r[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] = g.arc[a + k * stride];
        int hv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) hv[k] = r[k].y > 0 ? g.h[r[k].x] : INT32_MAX;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (hv[k] < hmin) {
                hmin = hv[k];
                cmin = r[k].y;
            } else if (hv[k] == hmin) {
                cmin += r[k].y;
            }
        }
    }
    for (; a < last; a += stride) {
        const int2 r = g.arc[a];
        const int hv = r.y > 0 ? g.h[r.x] : INT32_MAX;
        if (hv < hmin) {
            hmin = hv;
            cmin = r.y;
        } else if (hv == hmin) {
            cmin += r.y;
        }
    }
}

// A group of G lanes (G = 64: a wavefront) visits vertex u: the lanes scan
// its arcs G at a time for the lowest residual neighbour height, and the push
// pass hands the excess to the lowest arcs in arc order with a prefix sum of
// their residual capacities over the group.  u < 0: the group idles.  Every
// loop bound is uniform inside the group, so its lanes stay converged and the
// shuffles of width G stay inside it.  Returns relabels (on the group's lane
// 0).
template <int SC, int G>
__device__ int discharge_group(const DevGraph &g, int u, int kc, const RoundCtx &rc, Tally &tl,
                               int64_t &to_t) {
    const int gl = lane_id() & (G - 1);
    if (u < 0) return 0;
    const int n = g.n;
    const int beg = g.row_ptr[u], end = g.row_ptr[u + 1];
    int hu = g.h[u];
    int32_t stamp = g.rmark[u];  // phase of u's last first-relabel (read with the rest)
    int relabels = 0;
    if (rc.use_gap && hu < n && hu > ld<SC>(&g.ctrl->gap)) {  // above a gap: cut off
        if (gl == 0) {
            add<SC>(&g.hcount[hu], -1);
            g.h[u] = n;
        }
        hu = n;
    }
    // excess of u as last seen: loaded once, then taken from the returning
    // subtraction of what u pushed (incoming pushes only ever add to it)
    int64_t eu = 0;
    if (gl == 0) eu = ld<SC>(&g.e[u]);
    eu = __shfl(eu, 0, G);
    for (int cyc = 0; cyc < kc && hu < n; ++cyc) {
        if (eu <= 0) break;
        if (gl == 0) tl.pr_cyc++;
        int hmin = INT32_MAX;
        int64_t cmin = 0;  // not needed here
        scan_lowest(g, beg + gl, end, G, hmin, cmin);
        if (gl == 0) tl.pr_a += end - beg;
#pragma unroll
        for (int d = G / 2; d >= 1; d >>= 1) hmin = min(hmin, __shfl_xor(hmin, d, G));
        if (hmin == INT32_MAX) break;
        if (hu > hmin) {
            int64_t sent = 0, now = eu;
            for (int base = beg; base < end && sent < eu; base += G) {
                const int a = base + gl;
                int64_t c = 0;
                int v = -1, tw = 0;
                if (a < end) {
                    const int2 r = g.arc[a];
                    tw = g.twin[a];
                    if (r.y > 0 && g.h[r.x] == hmin) {
                        c = cyc == 0 ? r.y : max(0, ld<SC>(cf_ptr(g.arc, a)));
                        v = r.x;
                    }
                }
                // inclusive prefix sum of c over the group, in arc order
                int64_t incl = c;
#pragma unroll
                for (int d = 1; d < G; d <<= 1) {
                    const int64_t y = __shfl_up(incl, d, G);
                    if (gl >= d) incl += y;
                }
                const int64_t room = eu - sent;
                const int64_t excl = incl - c;
                const int64_t d = (c > 0 && excl < room) ? min(c, room - excl) : 0;
                const int64_t tot = min(__shfl(incl, G - 1, G), room);
                // the group's total leaves u before its lanes push it on, so
                // the returning subtraction overlaps the pushes
                if (gl == 0 && tot > 0) now = fetch_add<SC>(&g.e[u], -tot) - tot;
                if (d > 0) {
                    push_arc<SC>(g, rc, a, tw, v, (int32_t)d, to_t, tl);
                    tl.push++;
                }
                sent += tot;
            }
            eu = __shfl(now, 0, G);
        } else {
            int hn = 0;
            if (gl == 0) {
                hn = relabel_to<SC>(g, u, hu, hmin, rc.use_gap);
                tl.relabel++;
                note_relabel<SC>(g, rc, u, stamp);
            }
            hu = __shfl(hn, 0, G);
            relabels++;
        }
    }
    if (gl == 0 && hu < n && eu > 0) list_add<SC>(g, rc, u);
    return gl == 0 ? relabels : 0;
}

// A wavefront visits vertex u by walking its arcs in arc order, 64 at a
// time: the residual arcs that go downhill (head below u) take the excess in
// arc order (prefix sum of their residual capacities over the wavefront) and
// the walk stops as soon as the excess is gone; only when it reaches the end
// of the list with excess left does u relabel, to one above the lowest head
// among the arcs still residual.  Under exact labels the downhill arcs are
// those at h(u) - 1, the lowest residual heights, so this is the push of
// Alg. 2 without the full scan for the minimum before it; a head that a racy
// relabel left steep is pushed to like any downhill head.  Every lane of the
// wavefront calls it with the same u (u < 0: idle).  Returns relabels (lane 0).
template <int SC>
__device__ int discharge_walk(const DevGraph &g, int u, int kc, const RoundCtx &rc, Tally &tl, int64_t &to_t) {
    const int lane = lane_id();
    if (u < 0) return 0;
    const int n = g.n;
    const int beg = g.row_ptr[u], end = g.row_ptr[u + 1];
    int hu = g.h[u];
    int32_t stamp = g.rmark[u];
    int relabels = 0;
    if (rc.use_gap && hu < n && hu > ld<SC>(&g.ctrl->gap)) {  // above a gap: cut off
        if (lane == 0) {
            add<SC>(&g.hcount[hu], -1);
            g.h[u] = n;
        }
        hu = n;
    }
    int64_t eu = 0;
    if (lane == 0) eu = ld<SC>(&g.e[u]);
    eu = __shfl(eu, 0, 64);
    for (int cyc = 0; cyc < kc && hu < n; ++cyc) {
        if (eu <= 0) break;
        if (lane == 0) tl.pr_cyc++;
        const int64_t e0 = eu;  // what this walk hands out
        int64_t sent = 0, now = eu;
        int hrest = INT32_MAX;  // lowest head among the arcs left residual
        int walked = 0;
        for (int base = beg; base < end && sent < e0; base += 64) {
            const int a = base + lane;
            int64_t c = 0;
            int v = -1, hv = INT32_MAX;
            if (a < end) {
                const int2 r = g.arc[a];
                if (r.y > 0) {
                    hv = g.h[r.x];
                    if (hv < hu) {
                        c = cyc == 0 ? r.y : max(0, ld<SC>(cf_ptr(g.arc, a)));
                        v = r.x;
                    }
                }
            }
            walked += min(64, end - base);
            if (__ballot(c > 0) == 0) {  // nothing downhill in this step (the common case
                                         // of a walk that ends in a relabel)
                if (v < 0 && hv != INT32_MAX) hrest = min(hrest, hv);
                continue;
            }
            const int64_t incl = wave_incl_scan64(c);
            const int64_t room = e0 - sent;
            const int64_t excl = incl - c;
            const int64_t d = (c > 0 && excl < room) ? min(c, room - excl) : 0;
            const int64_t tot = min(__shfl(incl, 63, 64), room);
            if (lane == 0 && tot > 0) now = fetch_add<SC>(&g.e[u], -tot) - tot;
            if (d > 0) {
                push_arc<SC>(g, rc, a, g.twin[a], v, (int32_t)d, to_t, tl);
                tl.push++;
            }
            if (d < c || (v < 0 && hv != INT32_MAX)) hrest = min(hrest, hv);
            sent += tot;
        }
        if (lane == 0) tl.pr_a += walked;
        eu = __shfl(now, 0, 64);
        if (sent >= e0) continue;  // the excess went downhill
        // the walk reached the end of the list with excess left: relabel
        if (eu <= 0) break;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) hrest = min(hrest, __shfl_xor(hrest, d, 64));
        if (hrest == INT32_MAX) break;  // no residual arc left
        int hn = 0;
        if (lane == 0) {
            hn = relabel_to<SC>(g, u, hu, hrest, rc.use_gap);
            tl.relabel++;
            note_relabel<SC>(g, rc, u, stamp);
        }
        hu = __shfl(hn, 0, 64);
        relabels++;
    }
    if (lane == 0 && hu < n && eu > 0) list_add<SC>(g, rc, u);
    return lane == 0 ? relabels : 0;
}

// Lanes per vertex with a short arc list (at most kLightMaxDeg arcs): the
// arcs of a typical vertex load in one step instead of one after another.
constexpr int kLightGroup = 8;

// A whole workgroup visits vertex u (more than kHugeDeg arcs).  Each
// wavefront owns a contiguous chunk of u's arcs and finds, in one pass, its
// lowest residual neighbour height and the residual capacity toward it; the
// chunks' capacities at the overall lowest height h^ split the excess in arc
// order, so every wavefront then pushes its share along its own chunk without
// workgroup barriers.  Without races this makes exactly the pushes of one
// pass over all arcs in arc order (the same as discharge_group); a capacity
// or height that changed since the scan only leaves excess behind.  Every
// thread of the workgroup calls it with the same u; all decisions are
// uniform.
template <int SC>
__device__ int discharge_block(const DevGraph &g, int u, int kc, const RoundCtx &rc, Tally &tl,
                               int64_t &to_t) {
    __shared__ int s_min[32];
    __shared__ int64_t s_sum[32];
    __shared__ int64_t s_now;
    __shared__ int s_h;
    const int t = threadIdx.x, lane = lane_id(), w = t >> 6, nw = blockDim.x >> 6;
    const int n = g.n;
    const int beg = g.row_ptr[u], end = g.row_ptr[u + 1];
    const int chunk = ((end - beg + nw - 1) / nw + 63) & ~63;
    const int cb = min(end, beg + w * chunk), ce = min(end, cb + chunk);
    int hu = g.h[u];
    int32_t stamp = g.rmark[u];
    int relabels = 0;
    if (rc.use_gap && hu < n && hu > ld<SC>(&g.ctrl->gap)) {  // above a gap: cut off
        if (t == 0) {
            add<SC>(&g.hcount[hu], -1);
            g.h[u] = n;
        }
        hu = n;
    }
    if (t == 0) s_now = ld<SC>(&g.e[u]);
    __syncthreads();
    int64_t eu = s_now;
    for (int cyc = 0; cyc < kc && hu < n; ++cyc) {
        if (eu <= 0) break;
        if (t == 0) {
            tl.pr_cyc++;
            tl.pr_a += end - beg;
        }
        int hm = INT32_MAX;
        int64_t cm = 0;
        scan_lowest(g, cb + lane, ce, 64, hm, cm);
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const int oh = __shfl_xor(hm, d, 64);
            const int64_t oc = __shfl_xor(cm, d, 64);
            if (oh < hm) {
                hm = oh;
                cm = oc;
            } else if (oh == hm) {
                cm += oc;
            }
        }
        if (lane == 0) {
            s_min[w] = hm;
            s_sum[w] = cm;
        }
        __syncthreads();
        int hmin = INT32_MAX;
        for (int k = 0; k < nw; ++k) hmin = min(hmin, s_min[k]);
        int64_t off = 0;  // capacity at h^ in the chunks before this one
        for (int k = 0; k < w; ++k)
            if (s_min[k] == hmin) off += s_sum[k];
        const int64_t mine = hm == hmin ? cm : 0;
        __syncthreads();
        if (hmin == INT32_MAX) break;
        if (hu > hmin) {
            // this chunk's part of [0, eu) in arc order
            const int64_t room = max((int64_t)0, min(mine, eu - off));
            int64_t sent = 0;
            for (int base = cb; base < ce && sent < room; base += 64) {
                const int a = base + lane;
                int64_t c = 0;
                int v = -1, tw = 0;
                if (a < ce) {
                    const int2 r = g.arc[a];
                    tw = g.twin[a];
                    if (r.y > 0 && g.h[r.x] == hmin) {
                        c = cyc == 0 ? r.y : max(0, ld<SC>(cf_ptr(g.arc, a)));
                        v = r.x;
                    }
                }
                const int64_t incl = wave_incl_scan64(c);
                const int64_t rem = room - sent;
                const int64_t excl = incl - c;
                const int64_t d = (c > 0 && excl < rem) ? min(c, rem - excl) : 0;
                if (d > 0) {
                    push_arc<SC>(g, rc, a, tw, v, (int32_t)d, to_t, tl);
                    tl.push++;
                }
                sent += min(__shfl(incl, 63, 64), rem);
            }
            if (lane == 0 && sent > 0) add<SC>(&g.e[u], -sent);
            __syncthreads();
            if (t == 0) s_now = ld<SC>(&g.e[u]);
            __syncthreads();
            eu = s_now;
        } else {
            if (t == 0) {
                s_h = relabel_to<SC>(g, u, hu, hmin, rc.use_gap);
                tl.relabel++;
                note_relabel<SC>(g, rc, u, stamp);
            }
            __syncthreads();
            hu = s_h;
            __syncthreads();
            relabels++;
        }
    }
    if (t == 0 && hu < n && eu > 0) list_add<SC>(g, rc, u);
    return t == 0 ? relabels : 0;
}

// The walk of discharge_walk done by a whole workgroup (vertices of more than
// kHugeDeg arcs): one step covers blockDim.x arcs, the downhill residual
// capacities are prefix-summed over the workgroup (wavefront scans, then the
// wavefront totals through LDS), and the walk stops at the step where the
// excess runs out.  Only a walk that reaches the end of the list relabels.
// Every thread of the workgroup calls it with the same u; all decisions are
// uniform.
template <int SC>
__device__ int discharge_block_walk(const DevGraph &g, int u, int kc, const RoundCtx &rc, Tally &tl,
                                    int64_t &to_t) {
    __shared__ int64_t s_wsum[32];
    __shared__ int s_wmin[32];
    __shared__ int64_t s_now;
    __shared__ int s_h;
    const int t = threadIdx.x, lane = lane_id(), w = t >> 6, nw = blockDim.x >> 6;
    const int n = g.n;
    const int beg = g.row_ptr[u], end = g.row_ptr[u + 1];
    int hu = g.h[u];
    int32_t stamp = g.rmark[u];
    int relabels = 0;
    if (rc.use_gap && hu < n && hu > ld<SC>(&g.ctrl->gap)) {  // above a gap: cut off
        if (t == 0) {
            add<SC>(&g.hcount[hu], -1);
            g.h[u] = n;
        }
        hu = n;
    }
    if (t == 0) s_now = ld<SC>(&g.e[u]);
    __syncthreads();
    int64_t eu = s_now;
    for (int cyc = 0; cyc < kc && hu < n; ++cyc) {
        if (eu <= 0) break;
        if (t == 0) tl.pr_cyc++;
        const int64_t e0 = eu;
        int64_t sent = 0;
        int hrest = INT32_MAX;
        int walked = 0;
        for (int base = beg; base < end && sent < e0; base += blockDim.x) {
            const int a = base + t;
            int64_t c = 0;
            int v = -1, hv = INT32_MAX;
            if (a < end) {
                const int2 r = g.arc[a];
                if (r.y > 0) {
                    hv = g.h[r.x];
                    if (hv < hu) {
                        c = cyc == 0 ? r.y : max(0, ld<SC>(cf_ptr(g.arc, a)));
                        v = r.x;
                    }
                }
            }
            walked += min((int)blockDim.x, end - base);
            if (!__syncthreads_or(c > 0)) {  // nothing downhill in this step of the workgroup
                if (v < 0 && hv != INT32_MAX) hrest = min(hrest, hv);
                continue;
            }
            const int64_t incl = wave_incl_scan64(c);
            if (lane == 63) s_wsum[w] = incl;
            __syncthreads();
            int64_t woff = 0, btot = 0;
            for (int k = 0; k < nw; ++k) {
                const int64_t x = s_wsum[k];
                if (k < w) woff += x;
                btot += x;
            }
            __syncthreads();
            const int64_t room = e0 - sent;
            const int64_t excl = woff + incl - c;
            const int64_t d = (c > 0 && excl < room) ? min(c, room - excl) : 0;
            if (d > 0) {
                push_arc<SC>(g, rc, a, g.twin[a], v, (int32_t)d, to_t, tl);
                tl.push++;
            }
            if (d < c || (v < 0 && hv != INT32_MAX)) hrest = min(hrest, hv);
            sent += min(btot, room);
        }
        if (t == 0) {
            tl.pr_a += walked;
            if (sent > 0) add<SC>(&g.e[u], -sent);
        }
        __syncthreads();
        if (t == 0) s_now = ld<SC>(&g.e[u]);
        __syncthreads();
        eu = s_now;
        if (sent >= e0) continue;  // the excess went downhill
        if (eu <= 0) break;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) hrest = min(hrest, __shfl_xor(hrest, d, 64));
        if (lane == 0) s_wmin[w] = hrest;
        __syncthreads();
        int hmin = INT32_MAX;
        for (int k = 0; k < nw; ++k) hmin = min(hmin, s_wmin[k]);
        __syncthreads();
        if (hmin == INT32_MAX) break;  // no residual arc left
        if (t == 0) {
            s_h = relabel_to<SC>(g, u, hu, hmin, rc.use_gap);
            tl.relabel++;
            note_relabel<SC>(g, rc, u, stamp);
        }
        __syncthreads();
        hu = s_h;
        __syncthreads();
        relabels++;
    }
    if (t == 0 && hu < n && eu > 0) list_add<SC>(g, rc, u);
    return t == 0 ? relabels : 0;
}

// Excess pushed into t by the lanes of a wavefront, added with one atomic
// (topology-driven rounds; data-driven rounds sum per workgroup).
template <int SC>
__device__ __forceinline__ void flush_to_t(const DevGraph &g, int64_t &to_t) {
    const int64_t s = wave_sum(to_t);
    if (lane_id() == 0 && s) {
        add<SC>(&g.e[g.t], s);
        add<SC>(&g.ctrl->phase_deliv, s);
    }
    to_t = 0;
}

template <int SC>
__device__ __forceinline__ void flush_relabels(Ctrl *c, int64_t &rl, int64_t pushes, int64_t deliv) {
    const int64_t s = wave_sum(rl);
    const int64_t p = wave_sum(pushes);
    const int64_t dv = wave_sum(deliv);
    if (lane_id() == 0 && s) add<SC>(&c->phase_relabels, s);
    if (lane_id() == 0 && p) add<SC>(&c->phase_pushes, p);
    if (lane_id() == 0 && dv) add<SC>(&c->phase_deliv, dv);
    rl = 0;
}

// Copy the workgroup's staged appends into the next round's list and the
// phase's relabelled list: one reservation per list and workgroup; add the workgroup's round counters
// (acc: excess into t, relabels, pushes, deliveries into deficits).  Every
// thread of the workgroup calls it.
template <int SC>
__device__ void flush_stage(const DevGraph &g, const RoundCtx &rc, const int64_t *acc) {
    __shared__ int s_lb, s_hb, s_rb;
    __syncthreads();
    const int nl = min(*rc.lcnt, kStageCap), nh = min(*rc.hcnt, kStageCap), nr = min(*rc.rcnt, kStageCap);
    if (threadIdx.x == 0) {
        s_lb = nl ? fetch_add<SC>(&rc.next_ctr->light, nl) : 0;
        s_hb = nh ? fetch_add<SC>(&rc.next_ctr->heavy, nh) : 0;
        s_rb = nr ? fetch_add<SC>(&g.ctrl->nrelab, nr) : 0;
        Ctrl *c = g.ctrl;
        if (acc[0]) add<SC>(&g.e[g.t], acc[0]);
        if (acc[0] + acc[3]) add<SC>(&c->phase_deliv, acc[0] + acc[3]);
        if (acc[1]) add<SC>(&c->phase_relabels, acc[1]);
        if (acc[2]) add<SC>(&c->phase_pushes, acc[2]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nl; i += blockDim.x) rc.next[s_lb + i] = rc.lbuf[i];
    for (int i = threadIdx.x; i < nh; i += blockDim.x) rc.next[g.n - 1 - (s_hb + i)] = rc.hbuf[i];
    for (int i = threadIdx.x; i < nr; i += blockDim.x) g.relab[s_rb + i] = rc.rbuf[i];
}

// Add the workgroup's push sums to the targets' excess (every thread of the
// workgroup calls it); a target whose excess turns positive joins the next
// round's list, as after a single push.
template <int SC>
__device__ void flush_combine(const DevGraph &g, const RoundCtx &rc, Tally &tl) {
    __syncthreads();
    for (int i = threadIdx.x; i < kCombine; i += blockDim.x) {
        const int v = rc.comb->key[i];
        if (v < 0) continue;
        const int64_t d = rc.comb->sum[i];
        rc.comb->key[i] = -1;
        rc.comb->sum[i] = 0;
        const int64_t old = fetch_add<SC>(&g.e[v], d);
        if (old < 0) tl.deliv += min(d, -old);
        if (old <= 0 && old + d > 0 && v != g.s) list_add<SC>(g, rc, v);
    }
}

// One data-driven round over list rd: short lists by lane, long ones by
// wavefronts that take the next vertex from a shared counter.
template <int SC, bool WALK>
__device__ void pr_round(const DevGraph &g, const Team &tm, int rd, int nl, int nh, int nu, int kc,
                         const RoundCtx &rc0, Combine *comb, Tally &tl) {
    const int64_t gtid = tm.tid();
    const int64_t stride = tm.nthreads();
    __shared__ int32_t s_lbuf[kStageCap], s_hbuf[kStageCap], s_rbuf[kStageCap];
    __shared__ int32_t s_lcnt, s_hcnt, s_rcnt;
    __shared__ int64_t s_acc[4];  // the workgroup's excess into t, relabels, pushes, deliveries
    if (threadIdx.x == 0) s_lcnt = s_hcnt = s_rcnt = 0;
    if (threadIdx.x < 4) s_acc[threadIdx.x] = 0;
    __syncthreads();
    RoundCtx rc = rc0;
    rc.lbuf = s_lbuf;
    rc.hbuf = s_hbuf;
    rc.rbuf = s_rbuf;
    rc.lcnt = &s_lcnt;
    rc.hcnt = &s_hcnt;
    rc.rcnt = &s_rcnt;
    rc.comb = comb;
    const int32_t *lst = g.list[rd];
    int64_t to_t = 0, rl = 0;
    const uint32_t push0 = tl.push;
    {
        const int64_t grp = gtid / kLightGroup, ngrp = stride / kLightGroup;
        const int64_t trips = (nl + ngrp - 1) / ngrp;  // the same for every group
        for (int64_t k = 0, i = grp; k < trips; ++k, i += ngrp)
            rl += discharge_group<SC, kLightGroup>(g, i < nl ? lst[i] : -1, kc, rc, tl, to_t);
    }
    // huge arc lists: one workgroup per vertex, handed out by a counter
    if (nu > 0) {
        __shared__ int s_idx;
        const int32_t *hl = g.huge[rd];
        for (;;) {
            if (threadIdx.x == 0) s_idx = fetch_add<SC>(&g.ctrl->lst[rd].hgrab, 1);
            __syncthreads();
            const int idx = s_idx;
            __syncthreads();
            if (idx >= nu) break;
            if constexpr (WALK) rl += discharge_block_walk<SC>(g, hl[idx], kc, rc, tl, to_t);
            else rl += discharge_block<SC>(g, hl[idx], kc, rc, tl, to_t);
        }
    }
    // long arc lists: one wavefront per vertex, dealt out round-robin (no
    // shared counter for thousands of wavefronts to contend on)
    for (int64_t i = tm.wave(); i < nh; i += tm.nwaves()) {
        const int u = lst[g.n - 1 - i];
        if constexpr (WALK) rl += discharge_walk<SC>(g, u, kc, rc, tl, to_t);
        else rl += discharge_group<SC, 64>(g, u, kc, rc, tl, to_t);
    }
    if (comb) flush_combine<SC>(g, rc, tl);
    // the round's counters: summed over the workgroup, one atomic each
    {
        const int64_t v[4] = {wave_sum(to_t), wave_sum(rl), wave_sum((int64_t)(tl.push - push0)),
                              wave_sum(tl.deliv)};
        if (lane_id() == 0)
            for (int k = 0; k < 4; ++k)
                if (v[k]) atomicAdd(reinterpret_cast<unsigned long long *>(&s_acc[k]), (unsigned long long)v[k]);
        tl.deliv = 0;
    }
    flush_stage<SC>(g, rc, s_acc);
}

// One topology-driven round: every vertex is visited (idle when inactive).
template <int SC>
__device__ void pr_round_topology(const DevGraph &g, const Team &tm, int kc, const RoundCtx &rc,
                                  Tally &tl) {
    const int64_t gtid = tm.tid();
    const int64_t stride = tm.nthreads();
    int64_t to_t = 0, rl = 0;
    const uint32_t push0 = tl.push;
    {
        const int64_t grp = gtid / kLightGroup, ngrp = stride / kLightGroup;
        const int64_t trips = ((int64_t)g.n + ngrp - 1) / ngrp;
        for (int64_t k = 0, i = grp; k < trips; ++k, i += ngrp) {
            int u = (int)i;
            if (i >= g.n || u == g.s || u == g.t || g.row_ptr[u + 1] - g.row_ptr[u] > kLightMaxDeg) u = -1;
            rl += discharge_group<SC, kLightGroup>(g, u, kc, rc, tl, to_t);
        }
    }
    flush_to_t<SC>(g, to_t);
    for (int64_t i = tm.wave(); i < g.n_heavy_all; i += tm.nwaves())
        rl += discharge_group<SC, 64>(g, g.heavy_all[i], kc, rc, tl, to_t);
    flush_to_t<SC>(g, to_t);
    flush_relabels<SC>(g.ctrl, rl, (int64_t)(tl.push - push0), tl.deliv);
    tl.deliv = 0;
}

// ---------------------------------------------------------------------------
// RemoveInvalidEdges (Alg. 3): saturate every residual arc (u, v) with
// h(u) > h(v) + 1.  Heights never drop inside a phase and start exact, so only
// vertices that relabelled in the phase can own such an arc; the phase keeps
// them in a list.  Only u lowers c_f of its own arcs, so an exchange with 0
// reads and clears the residual in one step.
// ---------------------------------------------------------------------------

template <int SC>
__device__ __forceinline__ void rie_arc(const DevGraph &g, int u, int hu, int a, Tally &tl) {
    const int2 r = g.arc[a];
    if (r.y > 0 && hu > g.h[r.x] + 1) {
        const int32_t c = xchg<SC>(cf_ptr(g.arc, a), 0);
        if (c > 0) {
            add<SC>(cf_ptr(g.arc, g.twin[a]), c);
            add<SC>(&g.e[u], -(int64_t)c);
            add<SC>(&g.e[r.x], (int64_t)c);
            tl.rie_sat++;
        }
    }
}

// With the gap heuristic on, a vertex cut off at height |V| is skipped: its arcs
// look steep only because it was lifted deliberately, and saturating them
// would push flow out of the source side and create deficits (new roots)
// there, undoing the cut.
template <int SC>
__device__ void remove_invalid(const DevGraph &g, const Team &tm, const int32_t *list, int64_t count,
                               bool skip_cut, Tally &tl) {
    // a group of kLightGroup lanes per listed vertex: a short list is scanned by
    // its group (arcs gl, gl + kLightGroup, ..., loads independent of each
    // other); a long one by a whole wavefront after the group step
    constexpr int G = 8;
    const int64_t grp = tm.tid() / G, ngrp = tm.nthreads() / G;
    const int gl = lane_id() & (G - 1);
    const int lane = lane_id();
    const int64_t trips = (count + ngrp - 1) / ngrp;  // the same for every lane
    for (int64_t k = 0, i = grp; k < trips; ++k, i += ngrp) {
        int u = -1, beg = 0, end = 0, hu = 0;
        bool heavy = false;
        if (i < count) {
            u = list[i];
            hu = g.h[u];
            if (skip_cut && hu >= g.n) {
                u = -1;
            } else {
                beg = g.row_ptr[u];
                end = g.row_ptr[u + 1];
                heavy = end - beg > kLightMaxDeg;
            }
        }
        if (u >= 0 && !heavy) {
            for (int a = beg + gl; a < end; a += G) rie_arc<SC>(g, u, hu, a, tl);
            if (gl == 0) tl.rie_a += end - beg;
        }
        uint64_t hm = __ballot(heavy && gl == 0);
        while (hm) {
            const int l = __ffsll((unsigned long long)hm) - 1;
            hm &= hm - 1;
            const int w = __shfl(u, l, 64);
            const int wb = __shfl(beg, l, 64), we = __shfl(end, l, 64);
            const int hw = __shfl(hu, l, 64);
            for (int a = wb + lane; a < we; a += 64) rie_arc<SC>(g, w, hw, a, tl);
            if (lane == 0) tl.rie_a += we - wb;
        }
    }
}

// ---------------------------------------------------------------------------
// Learned phase schedule
//
// Right after a global relabel found active vertices, the schedule picks the
// limits of the coming phase among kPolK actions: relabel budget x b/4,
// rounds per BFS level x r/2, stall limit x l/2 (0: none).  Action 0 is the
// fixed rule.  Every action keeps the result exact: only the moment of the
// next global relabel changes.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int act_budget(int a) { return a == 1 ? 1 : a == 2 ? 2 : a == 3 ? 8 : a == 4 ? 16 : 4; }
__device__ __forceinline__ int act_rpl(int a) { return a == 4 || a == 6 ? 4 : a == 5 ? 1 : 2; }
__device__ __forceinline__ int act_stall(int a) { return a == 6 ? 1 : a == 7 ? 0 : 2; }

// splitmix64 finaliser (Steele, Lea and Flood, 2014): counter-based draws of
// the exploration mode.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Run by the 64 lanes of the leader's wavefront after the barrier that ends
// the BFS.  Features (every lane computes them), then the action: the
// network's lowest predicted cost
// when it beats action 0 by the margin (learned), a seeded draw (explore) or
// a fixed action (forced).  Lane 0 publishes the action in Ctrl; the features
// and the action go to the policy trace.
template <int SC>
__device__ int policy_decide(const DevGraph &g, const LoopParams &p, Ctrl *c, int L, int64_t iter) {
    constexpr int F = kPolF, H = kPolH, K = kPolK;
    constexpr int oW1 = 0, ob1 = oW1 + H * F, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H, ob3 = oW3 + K * H;
    const int lane = lane_id();
    const int64_t reached = ld<SC>(&c->feat_reached);
    const int cnt = ld<SC>(&c->lst[0].light) + ld<SC>(&c->lst[0].heavy) + ld<SC>(&c->lst[0].huge);
    const int64_t es = ld<SC>(&c->feat_esum);
    float x[F];
    x[0] = log2f((float)(1 + cnt)) / 24.f;
    x[1] = log2f((float)(1 + es)) / 40.f;
#pragma unroll
    for (int b = 0; b < 8; ++b) x[2 + b] = cnt ? (float)ld<SC>(&c->feat_hist[b]) / (float)cnt : 0.f;
    x[10] = log2f((float)(1 + L)) / 12.f;
    x[11] = (float)reached / (float)g.n;
    x[12] = log2f((float)(1 + ld<SC>(&c->prev_pushes))) / 32.f;
    x[13] = log2f((float)(1 + ld<SC>(&c->prev_relabels))) / 32.f;
    x[14] = log2f((float)(1 + iter)) / 8.f;
    x[15] = p.batch_fraction;
    int act = 0;
    if (p.policy_per_call && iter > 0) {
        act = ld<SC>(&c->action);  // the call's first decision holds
    } else if (p.policy_mode == kPolicyLearned) {
        const float *W = p.policy_w;
        const int j = lane & (H - 1);
        float z = W[ob1 + j];
#pragma unroll
        for (int i = 0; i < F; ++i) z = fmaf(W[oW1 + j * F + i], x[i], z);
        const float h1 = z > 0.f ? z : 0.f;
        float z2 = W[ob2 + j];
#pragma unroll
        for (int l = 0; l < H; ++l) z2 = fmaf(W[oW2 + j * H + l], __shfl(h1, l, 64), z2);
        const float h2 = z2 > 0.f ? z2 : 0.f;
        const int k = lane & (K - 1);
        float q = W[ob3 + k];
#pragma unroll
        for (int l = 0; l < H; ++l) q = fmaf(W[oW3 + k * H + l], __shfl(h2, l, 64), q);
        const float q0 = __shfl(q, 0, 64);
        float best = q0;
        int ba = 0;
#pragma unroll
        for (int kk = 1; kk < K; ++kk) {
            const float qk = __shfl(q, kk, 64);
            if (qk < best) {
                best = qk;
                ba = kk;
            }
        }
        act = (q0 - best > p.policy_margin) ? ba : 0;
    } else if (p.policy_mode == kPolicyExplore) {
        const uint64_t r = mix64(p.policy_seed ^ mix64(((uint64_t)(uint32_t)p.seq_base << 32) ^ (uint64_t)iter));
        const float u = (float)(r >> 40) * (1.0f / 16777216.0f);
        act = u < p.policy_explore ? (int)((r & 0xffffffffull) % (uint64_t)K) : 0;
    } else if (p.policy_mode == kPolicyForced) {
        act = p.policy_action;
    }
    const int rec = ld<SC>(&c->ntrace);
    if (g.ptrace && rec < kTraceCap) {
        float *pr = g.ptrace + (int64_t)rec * kPolRec;
#pragma unroll
        for (int f = 0; f < F; ++f)
            if (lane == f) pr[f] = x[f];
        if (lane == 0) pr[F] = (float)act;
    }
    if (lane == 0) c->action = act;
    return act;
}

// ---------------------------------------------------------------------------
// The persistent solve loop (Alg. 1 / Alg. 4 while-loop)
// ---------------------------------------------------------------------------

template <int SC, bool WALK>
__device__ void solve_loop(const DevGraph &g, const Team &tm, const LoopParams &p, BfsStage *stage,
                           Combine *comb) {
    Ctrl *c = g.ctrl;
    if (ld<SC>(&c->err)) return;  // update batch rejected: leave the state alone
    Tally tl;
    const bool leader = tm.rank == 0 && threadIdx.x == 0;
    const bool topology = p.mode == 1;
    int64_t iter = 0;
    uint32_t bar_epoch = 0;  // barriers this launch has passed
    const bool policy = p.policy_mode != kPolicyFixed;
    // vertices per height are counted only for the gap heuristic
    const bool counts = p.use_gap != 0;
    const uint64_t t0 = wall_clock64();
    // arcs of the vertices that the previous global relabel of this launch
    // reached (-1: none yet); the BFS direction rule takes the other arcs as
    // those a bottom-up level scans in full without finding a parent
    int64_t reach_prev = -1;
    for (;;) {
        // time budget: the leader raised `stop` before the last barrier, so
        // every workgroup sees the same value here
        if (ld<SC>(&c->stop)) {
            if (leader) c->status = kDeadline;
            break;
        }
        // --- global relabel ---
        if (leader) {
            for (int k = 0; k < 3; ++k) c->lst[k] = ListCtr{};
            c->prev_pushes = c->phase_pushes;
            c->prev_relabels = c->phase_relabels;
            c->feat_esum = 0;
            for (int b = 0; b < 8; ++b) c->feat_hist[b] = 0;
            c->nrelab = 0;
            c->phase_relabels = 0;
            c->phase_pushes = 0;
            c->phase_deliv = 0;
            c->gap = g.n;
            add<SC>(&c->stat[kStGlobalRelabels], 1);
        }
        const uint64_t tb = wall_clock64();
        // the BFS tallies the schedule's features only where a decision uses
        // them: every phase, or the first phase of a call decided per call
        const bool feats = policy && !(p.policy_per_call && iter > 0);
        // direction rule of the BFS (direction-optimising BFS): a level runs
        // bottom-up when its frontier's arcs are a large share of the arcs
        // that a bottom-up pass would scan, and stays so while the frontier is
        // large; small and restricted BFS passes stay top-down.  A bottom-up
        // pass stops early only at vertices it discovers: the vertices that
        // no level will reach (estimated by those the previous global relabel
        // did not reach) have their whole arc lists scanned at every level
        const bool dir = p.bu_alpha > 0 && g.bu_items != nullptr && !g.part_restrict;
        bfs_roots<SC>(g, tm, counts, feats, dir, tl);
        if (!grid_barrier(c, tm, bar_epoch, p.barrier_ticks)) return;
        int L = 0;
        bool bu = false;
        int64_t seen_arcs = 0;  // arcs of the vertices reached so far
        for (;;) {
            // the level's counters are loaded together: one round trip after
            // the barrier, not one per counter
            const int cnt = uniform(ld<SC>(&c->qcount[L % 3]));
            const int64_t fa = dir ? uniform(ld<SC>(&c->qarcs[L % 3])) : 0;
            const int fv = dir ? uniform(ld<SC>(&c->qverts[L % 3])) : 0;
            if (cnt == 0) break;
            if (dir) {
                seen_arcs += fa;
                const int64_t rest = (int64_t)g.A - seen_arcs;
                const int64_t dead = reach_prev < 0 ? 0 : min(rest, max((int64_t)0, (int64_t)g.A - reach_prev));
                bu = bu ? (int64_t)fv * p.bu_beta >= g.n : fa * p.bu_alpha > rest + (p.bu_alpha - 1) * dead;
            }
            // A small frontier is expanded by the first workgroup alone, level
            // after level with workgroup barriers in between (no grid barrier,
            // no L2 invalidation), while the others wait at the next grid
            // barrier.  The stretch ends at a level with no item or more than
            // solo_items items, or after a quarter of the barrier's wait limit.
            const bool alone = !bu && tm.size > 1 && cnt <= p.solo_items;
            if (!alone || tm.rank == 0) {
                const Team bt = alone ? Team{0, 1} : tm;
                const uint64_t ts = wall_clock64();
                for (int k = cnt;;) {
                    if (threadIdx.x == 0 && tm.rank == 0) {
                        c->qcount[(L + 2) % 3] = 0;
                        c->qverts[(L + 2) % 3] = 0;
                        c->qarcs[(L + 2) % 3] = 0;
                    }
                    if (bu)
                        bfs_bottom_up<SC>(g, bt, L, feats, counts, stage, tl);
                    else
                        bfs_level<SC>(g, bt, L, k, feats, counts, dir, k >= p.lazy_items,
                                      !alone && k >= kBfsStageMin ? stage : nullptr, stage, tl);
                    if (!alone) break;
                    __syncthreads();
                    ++L;
                    k = uniform(ld<SC>(&c->qcount[L % 3]));
                    if (k == 0 || k > p.solo_items) break;
                    if (uniform((int64_t)(wall_clock64() - ts)) > p.barrier_ticks / 4) break;
                }
                if (alone && threadIdx.x == 0) c->solo_level = L;
            }
            if (!grid_barrier(c, tm, bar_epoch, p.barrier_ticks)) return;
            L = alone ? uniform(ld<SC>(&c->solo_level)) : L + 1;
        }
        if (dir) reach_prev = seen_arcs;
        const uint64_t tp = wall_clock64();
        if (leader) {
            add<SC>(&c->stat[kStLevels], (int64_t)L);
            add<SC>(&c->stat[kStBfsTicks], (int64_t)(tp - tb));
        }
        // --- termination test right after a fresh global relabel ---
        {
            const int nl = uniform(ld<SC>(&c->lst[0].light));
            const int nh = uniform(ld<SC>(&c->lst[0].heavy));
            const int nu = uniform(ld<SC>(&c->lst[0].huge));
            if (nl + nh + nu == 0) {
                if (leader) c->status = kSolved;
                break;
            }
        }
        if (p.max_iter >= 0 && iter >= p.max_iter) {
            if (leader) c->status = kIterLimit;
            break;
        }
        // --- limits of the coming phase (fixed rule, or the schedule's action) ---
        int act = 0;
        if (policy) {
            if (tm.rank == 0 && threadIdx.x < 64) policy_decide<SC>(g, p, c, L, iter);
            if (!grid_barrier(c, tm, bar_epoch, p.barrier_ticks)) return;
            act = uniform(ld<SC>(&c->action));
        }
        const int64_t budget = act == 0 ? p.relabel_budget : max((int64_t)64, p.relabel_budget * act_budget(act) / 4);
        const int rpl = act == 0 ? p.rounds_per_level : max(1, p.rounds_per_level * act_rpl(act) / 2);
        const int round_cap = p.rounds_per_level > 0 ? min(p.max_rounds, rpl * L + 16) : p.max_rounds;
        const int stall_lim = p.stall_rounds <= 0 ? 0
                              : act == 0      ? max(p.stall_rounds, L)
                                              : (act_stall(act) == 0 ? 0 : max(1, max(p.stall_rounds, L) * act_stall(act) / 2));
        // --- push/relabel rounds ---
        const int32_t rbase = p.seq_base + uniform(ld<SC>(&c->rounds));
        const int active0 =
            uniform(ld<SC>(&c->lst[0].light) + ld<SC>(&c->lst[0].heavy) + ld<SC>(&c->lst[0].huge));
        int r = 0, reason = 0;
        int64_t last_deliv = -1;
        int last_change = 0;
        for (;;) {
            // A small round list (at most solo_items vertices, none huge) is
            // worked by the first workgroup alone, round after round with
            // workgroup barriers, while the others wait at the next grid
            // barrier; the stretch hands its round count and stall state over
            // in Ctrl.  It stops where a list grows, or after a quarter of the
            // barrier's wait limit.
            bool alone = false;
            if (tm.size > 1 && !topology && p.solo_items > 0) {  // a one-workgroup team is always alone
                const int rd0 = r % 3;
                const int64_t lh0 = uniform(ld<SC>(reinterpret_cast<const int64_t *>(&c->lst[rd0])));
                const int nu0 = uniform(ld<SC>(&c->lst[rd0].huge));
                const int size0 = (int)(uint32_t)lh0 + (int)((uint64_t)lh0 >> 32) + nu0;
                alone = nu0 == 0 && size0 > 0 && size0 <= p.solo_items;
            }
            bool done = false;
            if (!alone || tm.rank == 0) {
                const Team rt = alone ? Team{0, 1} : tm;
                const uint64_t ts = wall_clock64();
                for (;;) {
                    const int rd = r % 3, wr = (r + 1) % 3, rs = (r + 2) % 3;
                    // the round's control words, read together before any decision
                    const int64_t lh = uniform(ld<SC>(reinterpret_cast<const int64_t *>(&c->lst[rd])));
                    const int nu = uniform(ld<SC>(&c->lst[rd].huge));
                    const int64_t prl = uniform(ld<SC>(&c->phase_relabels));
                    const int64_t dl = uniform(ld<SC>(&c->phase_deliv));
                    const int nl = (int)(uint32_t)lh;
                    const int nh = (int)((uint64_t)lh >> 32);
                    if (nl + nh + nu == 0) {
                        done = true;
                        break;
                    }
                    if (r >= round_cap) {
                        reason = 1;
                        done = true;
                        break;
                    }
                    if (prl > budget) {
                        reason = 2;
                        done = true;
                        break;
                    }
                    // all values read here were written before the last barrier, so
                    // every workgroup of the team takes the same decision
                    if (dl != last_deliv) {
                        last_deliv = dl;
                        last_change = r;
                    }
                    if (stall_lim > 0 && r - last_change >= stall_lim) {
                        reason = 3;
                        done = true;
                        break;
                    }
                    if (leader) c->lst[rs] = ListCtr{};
                    const RoundCtx rc{g.list[wr], g.huge[wr], nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                      nullptr, &c->lst[wr], rbase + r + 1, rbase, p.use_gap != 0};
                    if (topology) pr_round_topology<SC>(g, rt, p.kc, rc, tl);
                    else pr_round<SC, WALK>(g, rt, rd, nl, nh, nu, p.kc, rc, p.combine ? comb : nullptr, tl);
                    ++r;
                    if (!alone) break;
                    __syncthreads();
                    const int rdn = r % 3;
                    const int64_t lhn = uniform(ld<SC>(reinterpret_cast<const int64_t *>(&c->lst[rdn])));
                    const int nun = uniform(ld<SC>(&c->lst[rdn].huge));
                    if (nun > 0 || (int)(uint32_t)lhn + (int)((uint64_t)lhn >> 32) > p.solo_items) break;
                    if (uniform((int64_t)(wall_clock64() - ts)) > p.barrier_ticks / 4) break;
                }
                if (alone && threadIdx.x == 0) {
                    c->solo_r = r;
                    c->solo_done = done ? 1 : 0;
                    c->solo_reason = reason;
                    c->solo_last_change = last_change;
                    c->solo_last_deliv = last_deliv;
                }
            }
            if (!alone && done) break;  // the phase ends for every workgroup alike
            if (!grid_barrier(c, tm, bar_epoch, p.barrier_ticks)) return;
            if (alone) {
                r = uniform(ld<SC>(&c->solo_r));
                reason = uniform(ld<SC>(&c->solo_reason));
                last_change = uniform(ld<SC>(&c->solo_last_change));
                last_deliv = uniform(ld<SC>(&c->solo_last_deliv));
                if (uniform(ld<SC>(&c->solo_done))) break;
            }
        }
        // --- RemoveInvalidEdges over the vertices that relabelled ---
        const uint64_t tr = wall_clock64();
        const int nrel = uniform(ld<SC>(&c->nrelab));
        if (!p.no_rie) remove_invalid<SC>(g, tm, g.relab, nrel, p.use_gap != 0, tl);
        if (counts)
            for (int64_t i = tm.tid(); i <= g.n; i += tm.nthreads()) g.hcount[i] = 0;
        {
            if (leader && c->ntrace < kTraceCap) {
                int32_t *tr_rec = c->trace[c->ntrace];
                tr_rec[kTrLevels] = L;
                tr_rec[kTrActive] = active0;
                tr_rec[kTrRounds] = r;
                tr_rec[kTrReason] = reason;
                tr_rec[kTrRelabels] = (int32_t)min<int64_t>(ld<SC>(&c->phase_relabels), INT32_MAX);
                tr_rec[kTrRelabelled] = nrel;
                tr_rec[kTrPushes] = (int32_t)min<int64_t>(ld<SC>(&c->phase_pushes), INT32_MAX);
                tr_rec[kTrLastDeliv] = last_change;
                if (policy && g.ptrace)
                    g.ptrace[(int64_t)c->ntrace * kPolRec + kPolF + 1] = (float)(wall_clock64() - tb);
                c->ntrace++;
            }
        }
        if (leader) {
            add<SC>(&c->stat[kStPrTicks], (int64_t)(tr - tp));
            add<SC>(&c->stat[kStRieTicks], (int64_t)(wall_clock64() - tr));
            for (int k = 0; k < 3; ++k) {
                c->qcount[k] = 0;
                c->qverts[k] = 0;
                c->qarcs[k] = 0;
            }
            c->feat_reached = 0;  // counted from the next phase's roots on
            c->rounds += r + 1;
            add<SC>(&c->stat[kStIterations], 1);
            add<SC>(&c->stat[kStRounds], (int64_t)r);
            if ((int64_t)(wall_clock64() - t0) > p.deadline_ticks) c->stop = 1;
        }
        flush_tally<SC>(c, tl);
        if (!grid_barrier(c, tm, bar_epoch, p.barrier_ticks)) return;
        ++iter;
    }
    // --- value: e(t) plus the deficits of vertices other than s and t ---
    // (every workgroup reaches this point after the same, uniform decision)
    {
        __shared__ int64_t s_def;
        if (threadIdx.x == 0) s_def = 0;
        __syncthreads();
        int64_t part = 0;
        for (int64_t v = tm.tid(); v < g.n; v += tm.nthreads()) {
            const int64_t ev = g.e[v];
            if (ev < 0 && v != g.s && v != g.t) part += ev;
        }
        part = wave_sum(part);
        if (lane_id() == 0 && part) atomicAdd((unsigned long long *)&s_def, (unsigned long long)part);
        __syncthreads();
        if (threadIdx.x == 0 && s_def) add<SC>(&c->deficit, s_def);
        if (leader) c->e_t = g.e[g.t];
    }
    flush_tally<SC>(c, tl);
}

// The whole grid is one team (cooperative launch), or a single workgroup.
// WALK: long arc lists are visited by the downhill walk (else scan first);
// the two are separate instances, since both inlined side by side would spill.
template <int BLOCK, int SC, bool WALK>
__global__ void __launch_bounds__(BLOCK) k_loop(DevGraph g, LoopParams p) {
    BfsStage *stage = nullptr;
    Combine *comb = nullptr;
    if constexpr (SC == kAgent) {
        __shared__ BfsStage s_stage;
        __shared__ Combine s_comb;
        if (threadIdx.x < 4) s_stage.cnt[threadIdx.x] = 0;
        if (threadIdx.x == 0) {
            s_stage.arcs = 0;
            s_stage.tverts = 0;
            s_stage.tarcs = 0;
        }
        for (int i = threadIdx.x; i < kCombine; i += blockDim.x) {
            s_comb.key[i] = -1;
            s_comb.sum[i] = 0;
        }
        __syncthreads();
        stage = &s_stage;
        comb = &s_comb;
    }
    solve_loop<SC, WALK>(g, Team{(int)blockIdx.x, (int)gridDim.x}, p, stage, comb);
}

// Two teams in one cooperative launch: workgroups [0, split) run the solve
// loop on view a, the others on view b, each view with its own state and
// control block (its own barrier).  The views must touch disjoint arc pairs
// and vertices (the S and T sides of a cut with no residual arc from S to
// T).  split follows the arc counts work[0] (view a) and work[1] (view b),
// at least one workgroup each.
template <int BLOCK, bool WALK>
__global__ void __launch_bounds__(BLOCK)
    k_teams(const DevGraph *__restrict__ views, const LoopParams *__restrict__ params, const int64_t *work) {
    __shared__ BfsStage s_stage;
    __shared__ Combine s_comb;
    if (threadIdx.x < 4) s_stage.cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        s_stage.arcs = 0;
        s_stage.tverts = 0;
        s_stage.tarcs = 0;
    }
    for (int i = threadIdx.x; i < kCombine; i += blockDim.x) {
        s_comb.key[i] = -1;
        s_comb.sum[i] = 0;
    }
    __syncthreads();
    const int G = (int)gridDim.x;
    const int64_t wa = work[0], wb = work[1];
    int64_t sp = (wa + wb) > 0 ? ((int64_t)G * wa + (wa + wb) / 2) / (wa + wb) : G / 2;
    const int split = (int)min((int64_t)G - 1, max((int64_t)1, sp));
    // one inlined loop; the view and its parameters are read by reference from
    // the device table (a private copy of either would be indexed dynamically
    // and spill)
    const int side = (int)blockIdx.x < split ? 0 : 1;
    const Team tm = side == 0 ? Team{(int)blockIdx.x, split} : Team{(int)blockIdx.x - split, G - split};
    const LoopParams &p = params[side];
    solve_loop<kAgent, WALK>(views[side], tm, p, &s_stage, p.combine ? &s_comb : nullptr);
}

// ---------------------------------------------------------------------------
// Part tags and views of the residual state (Dynamic Push-Pull, Sec. 4.2 /
// Alg. 8; returning excess to s and filling deficits from t, Sec. 3.1 and the
// proof of Sec. 4.1.1)
// ---------------------------------------------------------------------------

// part[v] = T when the last global relabel reached v (h < |V|: v reaches t or
// a deficient vertex in the residual graph), S otherwise (Alg. 8 first loop).
// work[0] / work[1] receive the arcs of the S / T vertices (cleared before).
__global__ void k_part_from_heights(DevGraph g, uint8_t *part, int64_t *work) {
    int64_t ws = 0, wt = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const bool tside = g.h[v] < g.n;
        part[v] = tside ? kPartT : kPartS;
        const int64_t d = g.row_ptr[v + 1] - g.row_ptr[v];
        if (tside) wt += d;
        else ws += d;
    }
    ws = wave_sum(ws);
    wt = wave_sum(wt);
    if (lane_id() == 0) {
        if (ws) add<kAgent>(&work[0], ws);
        if (wt) add<kAgent>(&work[1], wt);
    }
}

// After the two teams of a push-pull update: vertices that neither the
// backward BFS (heights h, from t and the deficient vertices of T) nor the
// forward BFS (heights hv, from s and the overflowing vertices of S) reached
// form P (Alg. 8, the localized stage); the others keep their side.
__global__ void k_part_localized(DevGraph g, const int32_t *hv, uint8_t *part) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
         v += (int64_t)gridDim.x * blockDim.x)
        if (g.h[v] >= g.n && hv[v] >= g.n) part[v] = kPartP;
}

// Saturate every residual arc from S to T (Alg. 8, "remove S to T edges"),
// booking the moved flow as excess at the head and deficit at the tail (the
// paper recomputes every excess afterwards; the change is the same).
__global__ void k_saturate_cut(DevGraph g, const uint8_t *part) {
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < g.A;
         a += (int64_t)gridDim.x * blockDim.x) {
        const int2 r = g.arc[a];
        if (r.y <= 0 || part[r.x] != kPartT) continue;
        const int32_t tw = g.twin[a];
        const int u = g.arc[tw].x;  // tail of a
        if (part[u] != kPartS) continue;
        g.arc[a].y = 0;  // only this thread touches the pair: its twin runs T -> S
        add<kAgent>(cf_ptr(g.arc, tw), r.y);
        add<kAgent>(&g.e[u], -(int64_t)r.y);
        add<kAgent>(&g.e[r.x], (int64_t)r.y);
    }
}

// Build a view of the state: rev = 0 copies arcs and excesses; rev = 1 gives
// arc a = (u, v) the residual of its twin (v, u) and every excess the
// opposite sign.  In the reversed view, pulling d into u along (v, u)
// (Alg. 6: c_f(v, u) -= d, c_f(u, v) += d, e(u) += d, e(v) -= d) is pushing d
// from u to v; the forward BFS of h_- is the backward BFS of the view, and
// the invalid-edge rule of Alg. 7 is that of Alg. 3 in the view.
__global__ void k_view_make(DevGraph g, int2 *varc, int64_t *ve, int rev) {
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t a = gtid; a < g.A; a += stride) {
        const int2 r = g.arc[a];
        varc[a] = rev ? make_int2(r.x, g.arc[g.twin[a]].y) : r;
    }
    for (int64_t v = gtid; v < g.n; v += stride) ve[v] = rev ? -g.e[v] : g.e[v];
}

// Write back a view's arcs between two vertices tagged `want`, and their
// excesses (rev: the view is reversed).
__global__ void k_view_merge(DevGraph g, const int2 *varc, const int64_t *ve, const uint8_t *part,
                             uint8_t want, int rev) {
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t a = gtid; a < g.A; a += stride) {
        const int32_t tw = g.twin[a];
        const int head = g.arc[a].x, tail = g.arc[tw].x;
        if (part[head] == want && part[tail] == want) g.arc[a].y = rev ? varc[tw].y : varc[a].y;
    }
    for (int64_t v = gtid; v < g.n; v += stride)
        if (part[v] == want) g.e[v] = rev ? -ve[v] : ve[v];
}

// Per-edge flow from the pair flows of a valid flow.  The flow on arc a is
// f(a) = cap(a) - c_f(a) where positive; it is shared out among the input
// edges merged into a, each taking min(its capacity, what is left), so that
// 0 <= flow <= capacity for every edge and the edges of a carry f(a).  rem
// (int32[A]) holds what is left per arc; edges of one arc draw from it with a
// compare-and-swap (in no fixed order among duplicates).
__global__ void k_arc_flow(DevGraph g, const int2 *carc, int32_t *rem) {
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < g.A;
         a += (int64_t)gridDim.x * blockDim.x)
        rem[a] = max(0, g.cap[a] - carc[a].y);
}

__global__ void k_edge_flow(DevGraph g, int32_t *rem, int32_t *flow) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = g.edge2arc[i];
        const int32_t c = g.ecap[i];
        int32_t give = 0;
        if (a >= 0 && c > 0) {
            int32_t old = ld<kAgent>(&rem[a]);
            for (;;) {
                give = min(c, old);
                if (give == 0) break;
                if (__hip_atomic_compare_exchange_strong(&rem[a], &old, old - give, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, kAgent))
                    break;
            }
        }
        flow[i] = give;
    }
}

// ---------------------------------------------------------------------------
// Initialisation, source saturation and update repair
// ---------------------------------------------------------------------------

__global__ void k_reset_ctrl(Ctrl *c) {
    int *w = reinterpret_cast<int *>(c);
    const int words = (int)(sizeof(Ctrl) / sizeof(int));
    for (int i = threadIdx.x; i < words; i += blockDim.x) w[i] = 0;
}

// Alg. 1 first loops: e = 0, h = 0, c_f = c.
__global__ void k_init_state(DevGraph g) {
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t a = gtid; a < g.A; a += stride) g.arc[a].y = g.cap[a];
    for (int64_t v = gtid; v < g.n; v += stride) {
        g.e[v] = 0;
        g.h[v] = 0;
    }
}

// Saturate every residual arc out of s: c_f(s,u) -> 0, the twin gains it,
// e(u) += d, e(s) -= d (Alg. 1 third loop; Alg. 4 lines 3-8, where the
// remaining residual is pushed rather than e(u) overwritten).
template <int SC>
__device__ void saturate_source(const DevGraph &g, const Team &tm) {
    if (ld<SC>(&g.ctrl->err)) return;
    __shared__ int64_t s_sum, s_cnt;
    if (threadIdx.x == 0) {
        s_sum = 0;
        s_cnt = 0;
    }
    __syncthreads();
    const int beg = g.row_ptr[g.s], end = g.row_ptr[g.s + 1];
    int64_t sum = 0, cnt = 0;
    for (int64_t a = beg + tm.tid(); a < end; a += tm.nthreads()) {
        const int2 r = g.arc[a];
        if (r.y > 0) {
            g.arc[a].y = 0;
            add<SC>(cf_ptr(g.arc, g.twin[a]), r.y);
            add<SC>(&g.e[r.x], (int64_t)r.y);
            sum += r.y;
            cnt++;
        }
    }
    sum = wave_sum(sum);
    cnt = wave_sum(cnt);
    if (lane_id() == 0 && sum) {
        atomicAdd((unsigned long long *)&s_sum, (unsigned long long)sum);
        atomicAdd((unsigned long long *)&s_cnt, (unsigned long long)cnt);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_sum) {
        add<SC>(&g.e[g.s], -s_sum);
        add<SC>(&g.ctrl->stat[kStSourcePushes], s_cnt);
    }
}

__global__ void k_saturate_source(DevGraph g) {
    saturate_source<kAgent>(g, Team{(int)blockIdx.x, (int)gridDim.x});
}

// Batch validation: ids in [0, m), capacities in [0, cap_limit], ids distinct
// (a batch is a set).  Sets Ctrl::err; later kernels of the call then skip.
__global__ void k_validate_updates(DevGraph g, const int64_t *ids, const int32_t *caps, int64_t k,
                                   int32_t epoch, int32_t cap_limit) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t id = ids[i];
        const int32_t cv = caps[i];
        if (id < 0 || id >= g.m) {
            atomicOr(&g.ctrl->err, 1);
            continue;
        }
        if (cv < 0 || cv > cap_limit) atomicOr(&g.ctrl->err, 2);
        if (atomicExch(&g.stamp[id], epoch) == epoch) atomicOr(&g.ctrl->err, 4);
    }
}

// Alg. 5 first loop: c_f(u,v) += c' - c; the stored capacities follow.
__global__ void k_apply_delta(DevGraph g, const int64_t *ids, const int32_t *caps, int64_t k) {
    if (ld<kAgent>(&g.ctrl->err)) return;
    int64_t cnt = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t id = ids[i];
        const int32_t cv = caps[i];
        const int32_t d = cv - g.ecap[id];
        g.ecap[id] = cv;
        const int32_t a = g.edge2arc[id];
        if (a >= 0 && d != 0) {
            add<kAgent>(&g.cap[a], d);
            add<kAgent>(cf_ptr(g.arc, a), d);
        }
        cnt++;
    }
    cnt = wave_sum(cnt);
    if (lane_id() == 0 && cnt) add<kAgent>(&g.ctrl->stat[kStUpdates], cnt);
}

// Alg. 5 second loop restricted to the updated arc pairs (only they can have
// gone negative), with the excess change booked at once: the flow clamped by
// o = -c_f(a) returns o units to the tail (e += o) and takes them from the
// head (e -= o).  At most one arc of a pair can be negative (their residuals
// sum to the pair's capacity); a compare-and-swap makes each clamp happen
// once even when several updates share a pair.
__global__ void k_clamp(DevGraph g, const int64_t *ids, int64_t k) {
    if (ld<kAgent>(&g.ctrl->err)) return;
    int64_t cnt = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a0 = g.edge2arc[ids[i]];
        if (a0 < 0) continue;
        const int32_t a1 = g.twin[a0];
        for (int side = 0; side < 2; ++side) {
            const int32_t x = side ? a1 : a0;
            const int32_t y = side ? a0 : a1;
            int32_t *cfx = cf_ptr(g.arc, x);
            const int32_t cv = ld<kAgent>(cfx);
            if (cv < 0 && cas<kAgent>(cfx, cv, 0)) {
                const int32_t o = -cv;
                add<kAgent>(cf_ptr(g.arc, y), -o);
                add<kAgent>(&g.e[g.arc[y].x], (int64_t)o);  // tail of x
                add<kAgent>(&g.e[g.arc[x].x], -(int64_t)o); // head of x
                cnt++;
            }
        }
    }
    cnt = wave_sum(cnt);
    if (lane_id() == 0 && cnt) add<kAgent>(&g.ctrl->stat[kStClamps], cnt);
}

// ---------------------------------------------------------------------------
// Local stage of a dynamic update, between the batch repair (Alg. 5) and the
// global loop: the updated arcs that now cross the last cut are saturated,
// and the deficits the batch left are filled from excess nearby (the ideas of
// Dynamic Push-Pull, Sec. 4.2 / Alg. 6 and 8, applied to the batch's own
// arcs).  Every step is a push along a residual arc, so the global loop that
// follows, with its unchanged termination test, still ends at a maximum flow;
// the stage only saves it the work of letting every vertex that holds excess
// on the source side chase a small deficit.
// ---------------------------------------------------------------------------

// Saturate every updated arc that is residual from the source side of the
// last cut (height |V|) to its sink side (height < |V|).  A solved state has
// no such arc, and only arcs whose capacity grew can have gained one: the
// clamp and the source re-saturation only lower residuals across it.  The
// flow moved becomes excess at the head and a deficit at the tail (Alg. 8,
// "remove S to T edges", on the batch).  Heights are those of the last
// global relabel.
__global__ void k_cut_saturate(DevGraph g, const int64_t *ids, int64_t k) {
    if (ld<kAgent>(&g.ctrl->err)) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a0 = g.edge2arc[ids[i]];
        if (a0 < 0) continue;
        const int32_t a1 = g.twin[a0];
        for (int side = 0; side < 2; ++side) {
            const int32_t x = side ? a1 : a0, y = side ? a0 : a1;
            const int head = g.arc[x].x, tail = g.arc[y].x;
            if (g.h[tail] < g.n || g.h[head] >= g.n) continue;
            if (ld<kAgent>(cf_ptr(g.arc, x)) <= 0) continue;
            const int32_t c = xchg<kAgent>(cf_ptr(g.arc, x), 0);  // updates sharing the pair: one takes it
            if (c > 0) {
                add<kAgent>(cf_ptr(g.arc, y), c);
                add<kAgent>(&g.e[tail], -(int64_t)c);
                add<kAgent>(&g.e[head], (int64_t)c);
            }
        }
    }
}

// One round of local pulls.  Every deficient vertex v of list `in` takes what
// it lacks from its in-neighbours w (residual arc w -> v) that hold excess,
// in arc order: d moves as a push from w to v (c_f(w,v) -= d, c_f(v,w) += d,
// e(w) -= d, e(v) += d), as Alg. 6 pulls, here without heights.  With `out`,
// what is still lacking is then taken from in-neighbours along their residual
// arcs whatever their excess, which hands the deficit on to them; a giver
// left with a deficit joins `out` (once, pmark tag).  s and t never give.  A
// wavefront per vertex; v's own excess is touched by its wavefront only.
// Each pass looks at no more than kPullScan arcs of v, the excess pass at the
// front of v's list and the hand-on pass at its back (from the last chunk
// backwards), so that a hub costs a bounded number of steps and the deficit
// is handed on to the neighbours at the end of the list (the low-degree ones
// when vertices are numbered by falling degree); what stays lacking is left
// to the global loop.
constexpr int kPullScan = 4096;
// The first round takes its vertices from the batch itself (ids, k: both
// ends of every updated arc pair, s and t left out, each deficient vertex
// claimed once with tag - 1); the later ones from the list `in` of the round
// before.  Marks only grow (pmark holds the largest tag given to a vertex,
// tags rise from call to call), so a claim or an append takes a vertex only
// if its mark is still below the tag: a vertex that round 0 already put on
// the next round's list (tag) is not claimed again as a batch end (tag - 1)
// while its first visit may still be running.  The list counters rotate over three words, cnt[r % 3] read and
// cnt[(r + 1) % 3] appended to by round r, which clears cnt[(r + 2) % 3] for
// round r + 1; they all start at zero with the call's control block.
__global__ void k_pull_round(DevGraph g, const int64_t *ids, int64_t k, const int32_t *in, int32_t *cnt, int r,
                             int32_t *out, int32_t *pmark, int32_t tag) {
    if (ld<kAgent>(&g.ctrl->err)) return;
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    if (blockIdx.x == 0 && threadIdx.x == 0) cnt[(r + 2) % 3] = 0;
    int32_t *out_cnt = &cnt[(r + 1) % 3];
    const int64_t items = ids ? 2 * k : (int64_t)ld<kAgent>(&cnt[r % 3]);
    for (int64_t i = wave; i < items; i += nwaves) {
        int v = -1;
        int64_t need = 0;
        if (lane == 0) {
            if (ids) {
                const int32_t a0 = g.edge2arc[ids[i >> 1]];
                const int w = a0 < 0 ? -1 : ((i & 1) ? g.arc[g.twin[a0]].x : g.arc[a0].x);
                if (w >= 0 && w != g.s && w != g.t && ld<kAgent>(&g.e[w]) < 0 &&
                    __hip_atomic_fetch_max(&pmark[w], tag - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < tag - 1)
                    v = w;
            } else {
                v = in[i];
            }
            if (v >= 0) need = -ld<kAgent>(&g.e[v]);
        }
        v = __shfl(v, 0, 64);
        need = __shfl(need, 0, 64);
        if (need <= 0) continue;
        const int beg = g.row_ptr[v], end = g.row_ptr[v + 1];
        int64_t got = 0;
        // chunks of 64 arcs aligned to the start of v's list in both passes,
        // so that an arc the first pass pushed along is read again by the
        // same lane (its own earlier atomic orders the read; another lane's
        // would not)
        const int nchunks = (end - beg + 63) / 64;
        for (int hand_on = 0; hand_on < (out ? 2 : 1) && got < need; ++hand_on) {
            const int lo = hand_on ? max(beg, end - kPullScan) : beg;
            const int hi = hand_on ? end : min(end, beg + kPullScan);
            const int c_first = hand_on ? nchunks - 1 : 0;
            const int c_last = hand_on ? (lo - beg) / 64 : (hi - beg + 63) / 64 - 1;
            for (int c = c_first; (hand_on ? c >= c_last : c <= c_last) && got < need; c += hand_on ? -1 : 1) {
                const int a = beg + 64 * c + lane;
                int64_t avail = 0;
                int w = -1, tw = 0;
                if (a >= lo && a < hi) {
                    w = g.arc[a].x;
                    tw = g.twin[a];
                    if (w != g.s && w != g.t) {
                        const int32_t r = ld<kAgent>(cf_ptr(g.arc, tw));
                        if (r > 0) {
                            if (hand_on) {
                                avail = r;
                            } else {
                                const int64_t ew = ld<kAgent>(&g.e[w]);
                                if (ew > 0) avail = min((int64_t)r, ew);
                            }
                        }
                    }
                }
                const int64_t incl = wave_incl_scan64(avail);
                const int64_t excl = incl - avail;
                const int64_t room = need - got;
                const int64_t d = (avail > 0 && excl < room) ? min(avail, room - excl) : 0;
                int64_t moved = 0;
                if (d > 0) {
                    // The excess pass claims its share of w's excess first and
                    // gives back what w no longer holds (other deficits may pull
                    // from the same giver at once), so that it never overdraws a
                    // giver: an overdrawn giver left after the last round is a
                    // deficit that the global loop would reach from the whole
                    // source side.  The hand-on pass takes along the residual
                    // whatever w holds, and lists a giver it leaves in deficit.
                    const int64_t old = fetch_add<kAgent>(&g.e[w], -d);
                    moved = d;
                    if (!hand_on) {
                        moved = old >= d ? d : (old > 0 ? old : 0);
                        if (moved < d) add<kAgent>(&g.e[w], d - moved);
                    }
                    if (moved > 0) {
                        add<kAgent>(cf_ptr(g.arc, tw), -(int32_t)moved);
                        add<kAgent>(cf_ptr(g.arc, a), (int32_t)moved);
                    }
                    if (out && hand_on && old - d < 0 &&
                        __hip_atomic_fetch_max(&pmark[w], tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < tag)
                        out[fetch_add<kAgent>(out_cnt, 1)] = w;
                }
                got += wave_sum(moved);
            }
        }
        if (lane == 0 && got > 0) add<kAgent>(&g.e[v], got);
    }
}

// Certificate: side[v] = 1 when h(v) >= |V|; cut = sum of cap over arcs from
// the source side to the sink side (the tail of arc a is the head of twin(a)).
__global__ void k_min_cut(DevGraph g, uint8_t *side) {
    __shared__ int64_t s_cut;
    if (threadIdx.x == 0) s_cut = 0;
    __syncthreads();
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (side)
        for (int64_t v = gtid; v < g.n; v += stride) side[v] = g.h[v] >= g.n ? 1 : 0;
    int64_t part = 0;
    for (int64_t a = gtid; a < g.A; a += stride) {
        const int head = g.arc[a].x;
        const int tail = g.arc[g.twin[a]].x;
        if (g.h[tail] >= g.n && g.h[head] < g.n) part += g.cap[a];
    }
    part = wave_sum(part);
    if (lane_id() == 0 && part) atomicAdd((unsigned long long *)&s_cut, (unsigned long long)part);
    __syncthreads();
    if (threadIdx.x == 0 && s_cut) add<kAgent>(&g.ctrl->cut, s_cut);
}

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

static int grid_for(int64_t work, int block, int cap = 8192);

// Invariants of a residual state (the debug check after a solving call).
__global__ void k_check_state(DevGraph g, int solved) {
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int32_t f = 0;
    for (int64_t a = gtid; a < g.A; a += stride) {
        const int2 r = g.arc[a];
        const int32_t tw = g.twin[a];
        const int2 q = g.arc[tw];
        if (r.y < 0) f |= 1;
        if ((int64_t)r.y + q.y != (int64_t)g.cap[a] + g.cap[tw]) f |= 2;
        if (solved && r.y > 0 && g.h[q.x] >= g.n && g.h[r.x] < g.n) f |= 16;  // q.x: tail of a
    }
    for (int64_t v = gtid; v < g.n; v += stride) {
        int64_t x = 0;
        for (int a = g.row_ptr[v]; a < g.row_ptr[v + 1]; ++a) x += (int64_t)g.arc[a].y - g.cap[a];
        if (x != g.e[v]) f |= 4;
        if (solved && v != g.s && v != g.t && g.e[v] > 0 && g.h[v] < g.n) f |= 8;
    }
    if (f) atomicOr(&g.ctrl->check, f);
}

hipError_t launch_check_state(const DevGraph &g, int solved, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, &g.ctrl->check, (int64_t)1, 0);
    const int64_t work = g.A > g.n ? g.A : g.n;
    hipLaunchKernelGGL(k_check_state, dim3(grid_for(work, 256, 4096)), dim3(256), 0, st, g, solved);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Batched solve: one workgroup per instance
// ---------------------------------------------------------------------------

// order[blockIdx.x] names the instance.  Its workgroup clears the control
// block, stamps and per-height counts, initialises the state (c_f = c,
// e = h = 0), saturates the source and runs the solve loop to the end, all
// separated by workgroup barriers only; res[i] receives the value and the
// loop status.  Workgroups never wait for each other.
template <int BLOCK>
__global__ void __launch_bounds__(BLOCK)
    k_batch(const DevGraph *__restrict__ graphs, const int32_t *__restrict__ order, LoopParams p,
            const int32_t *__restrict__ kc, BatchResult *__restrict__ res) {
    const int i = order[blockIdx.x];
    // a reference into the read-only table (uniform loads), not a private copy:
    // the solve loop indexes the list and frontier pointer arrays dynamically
    const DevGraph &g = graphs[i];
    const Team tm{0, 1};
    {
        int *w = reinterpret_cast<int *>(g.ctrl);
        const int words = (int)(sizeof(Ctrl) / sizeof(int));
        for (int j = threadIdx.x; j < words; j += BLOCK) w[j] = 0;
    }
    for (int v = threadIdx.x; v < g.n; v += BLOCK) {
        g.mark[v] = 0;
        g.rmark[v] = 0;
        g.e[v] = 0;
        g.h[v] = 0;
    }
    for (int v = threadIdx.x; v <= g.n; v += BLOCK) g.hcount[v] = 0;
    for (int a = threadIdx.x; a < g.A; a += BLOCK) g.arc[a].y = g.cap[a];
    __syncthreads();
    saturate_source<kGroup>(g, tm);
    __syncthreads();
    LoopParams q = p;
    q.kc = kc[i];
    if (q.relabel_budget <= 0) q.relabel_budget = max((int64_t)1024, (int64_t)g.n / 16);
    solve_loop<kGroup, false>(g, tm, q, nullptr, nullptr);
    __syncthreads();
    if (threadIdx.x == 0) {
        BatchResult r;
        r.value = g.ctrl->e_t + g.ctrl->deficit;
        r.status = g.ctrl->status;
        r.pad = 0;
        res[i] = r;
    }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------

static int grid_for(int64_t work, int block, int cap) {
    int64_t b = (work + block - 1) / block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

hipError_t launch_reset_ctrl(const DevGraph &g, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_ctrl, dim3(1), dim3(256), 0, st, g.ctrl);
    return hipGetLastError();
}

hipError_t launch_init_state(const DevGraph &g, hipStream_t st) {
    const int64_t work = g.A > g.n ? g.A : g.n;
    hipLaunchKernelGGL(k_init_state, dim3(grid_for(work, 256)), dim3(256), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_saturate_source(const DevGraph &g, hipStream_t st) {
    // the degree of s is only known on the host side of the handle; a fixed
    // grid with grid-stride loops covers any degree
    hipLaunchKernelGGL(k_saturate_source, dim3(256), dim3(256), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_validate_updates(const DevGraph &g, const int64_t *ids, const int32_t *caps,
                                   int64_t k, int32_t epoch, int32_t cap_limit, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate_updates, dim3(grid_for(k, 256)), dim3(256), 0, st, g, ids, caps, k,
                       epoch, cap_limit);
    return hipGetLastError();
}

hipError_t launch_apply_delta(const DevGraph &g, const int64_t *ids, const int32_t *caps, int64_t k,
                              hipStream_t st) {
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_apply_delta, dim3(grid_for(k, 256)), dim3(256), 0, st, g, ids, caps, k);
    return hipGetLastError();
}

hipError_t launch_clamp(const DevGraph &g, const int64_t *ids, int64_t k, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clamp, dim3(grid_for(k, 256)), dim3(256), 0, st, g, ids, k);
    return hipGetLastError();
}

hipError_t loop_max_coresident(int device, int *blocks) {
    int per_cu = 0, per_cu2 = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(k_loop<kBlock, kAgent, true>), kBlock, 0);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu2, reinterpret_cast<const void *>(k_loop<kBlock, kAgent, false>), kBlock, 0);
    if (e != hipSuccess) return e;
    per_cu = min(per_cu, per_cu2);
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    *blocks = per_cu * cus;
    return hipSuccess;
}

hipError_t launch_loop(const DevGraph &g, const LoopParams &p, int grid, hipStream_t st) {
    if (grid <= 1) {
        if (p.walk) hipLaunchKernelGGL((k_loop<kBlock, kGroup, true>), dim3(1), dim3(kBlock), 0, st, g, p);
        else hipLaunchKernelGGL((k_loop<kBlock, kGroup, false>), dim3(1), dim3(kBlock), 0, st, g, p);
        return hipGetLastError();
    }
    DevGraph ga = g;
    LoopParams pa = p;
    void *args[] = {&ga, &pa};
    const void *fn = p.walk ? reinterpret_cast<const void *>(k_loop<kBlock, kAgent, true>)
                            : reinterpret_cast<const void *>(k_loop<kBlock, kAgent, false>);
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBlock), args, 0, st);
}

hipError_t launch_batch(const DevGraph *graphs, const int32_t *order, int count, const LoopParams &p,
                        const int32_t *kc, BatchResult *res, int block, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    switch (block) {
    case 256:
        hipLaunchKernelGGL((k_batch<256>), dim3(count), dim3(256), 0, st, graphs, order, p, kc, res);
        break;
    case 512:
        hipLaunchKernelGGL((k_batch<512>), dim3(count), dim3(512), 0, st, graphs, order, p, kc, res);
        break;
    case 1024:
        hipLaunchKernelGGL((k_batch<1024>), dim3(count), dim3(1024), 0, st, graphs, order, p, kc, res);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_teams(const DevGraph *d_views, const LoopParams *d_params, bool walk, const int64_t *work,
                        int grid, hipStream_t st) {
    if (grid < 2) return hipErrorInvalidValue;
    const DevGraph *v = d_views;
    const LoopParams *q = d_params;
    const int64_t *w = work;
    void *args[] = {&v, &q, &w};
    const void *fn = walk ? reinterpret_cast<const void *>(k_teams<kBlock, true>)
                          : reinterpret_cast<const void *>(k_teams<kBlock, false>);
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBlock), args, 0, st);
}

hipError_t teams_max_coresident(int device, int *blocks) {
    int per_cu = 0, per_cu2 = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(k_teams<kBlock, true>), kBlock, 0);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu2, reinterpret_cast<const void *>(k_teams<kBlock, false>), kBlock, 0);
    if (e != hipSuccess) return e;
    per_cu = min(per_cu, per_cu2);
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    *blocks = per_cu * cus;
    return hipSuccess;
}

hipError_t launch_part_from_heights(const DevGraph &g, uint8_t *part, int64_t *work, hipStream_t st) {
    hipLaunchKernelGGL(k_part_from_heights, dim3(grid_for(g.n, 256, 2048)), dim3(256), 0, st, g, part, work);
    return hipGetLastError();
}

hipError_t launch_part_localized(const DevGraph &g, const int32_t *hv, uint8_t *part, hipStream_t st) {
    hipLaunchKernelGGL(k_part_localized, dim3(grid_for(g.n, 256, 2048)), dim3(256), 0, st, g, hv, part);
    return hipGetLastError();
}

hipError_t launch_saturate_cut(const DevGraph &g, const uint8_t *part, hipStream_t st) {
    hipLaunchKernelGGL(k_saturate_cut, dim3(grid_for(g.A, 256)), dim3(256), 0, st, g, part);
    return hipGetLastError();
}

hipError_t launch_view_make(const DevGraph &g, int2 *varc, int64_t *ve, int rev, hipStream_t st) {
    const int64_t work = g.A > g.n ? g.A : g.n;
    hipLaunchKernelGGL(k_view_make, dim3(grid_for(work, 256)), dim3(256), 0, st, g, varc, ve, rev);
    return hipGetLastError();
}

hipError_t launch_view_merge(const DevGraph &g, const int2 *varc, const int64_t *ve, const uint8_t *part,
                             uint8_t want, int rev, hipStream_t st) {
    const int64_t work = g.A > g.n ? g.A : g.n;
    hipLaunchKernelGGL(k_view_merge, dim3(grid_for(work, 256)), dim3(256), 0, st, g, varc, ve, part, want, rev);
    return hipGetLastError();
}

hipError_t launch_edge_flow(const DevGraph &g, const int2 *carc, int32_t *rem, int32_t *flow, hipStream_t st) {
    if (g.A > 0) hipLaunchKernelGGL(k_arc_flow, dim3(grid_for(g.A, 256)), dim3(256), 0, st, g, carc, rem);
    if (g.m > 0) hipLaunchKernelGGL(k_edge_flow, dim3(grid_for(g.m, 256)), dim3(256), 0, st, g, rem, flow);
    return hipGetLastError();
}

hipError_t launch_local_stage(const DevGraph &g, const int64_t *ids, int64_t k, int32_t *pmark, int32_t tag0,
                              int rounds, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cut_saturate, dim3(grid_for(k, 256)), dim3(256), 0, st, g, ids, k);
    // the list counters (ctrl->pull_cnt) start at zero with the call's
    // control block; at most 2k deficits in any list, a wavefront each
    int32_t *cnt = g.ctrl->pull_cnt;
    int32_t *lists[2] = {g.list[1], g.list[2]};
    const int blocks = grid_for(2 * k * 64, 256, 4096);
    for (int r = 0; r < rounds; ++r) {
        const bool last = r == rounds - 1;
        int32_t *out = last ? nullptr : lists[(r + 1) & 1];
        hipLaunchKernelGGL(k_pull_round, dim3(blocks), dim3(256), 0, st, g, r == 0 ? ids : nullptr, k, lists[r & 1],
                           cnt, r, out, pmark, tag0 + r + 1);
    }
    return hipGetLastError();
}

hipError_t launch_min_cut(const DevGraph &g, uint8_t *d_side, hipStream_t st) {
    const int64_t work = g.A > g.n ? g.A : g.n;
    hipLaunchKernelGGL(k_min_cut, dim3(grid_for(work, 256, 2048)), dim3(256), 0, st, g, d_side);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(count, 256)), dim3(256), 0, st, p, count, value);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batch staging of the allocation-free update call: one array per GPU, held
// until the process ends.  Host code never hands the array's name to a
// kernel (in host code it is only a stand-in for the symbol); its device
// address comes from hipGetSymbolAddress, once per device with that device
// current, and the kernels take that address like any other batch pointer.
// ---------------------------------------------------------------------------

static __device__ __align__(256) uint8_t scratch[kNoAllocIdsBytes + kNoAllocCapsBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

void *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace mf
