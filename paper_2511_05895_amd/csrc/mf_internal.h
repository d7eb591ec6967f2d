// Internal declarations shared by the host driver (mf_api.cpp) and the gfx950
// kernels (mf_kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

namespace mf {

// A vertex whose arc list is at most this long is handled by one lane in the
// push/relabel and invalid-edge sweeps; longer lists get a whole wavefront.
constexpr int kLightMaxDeg = 32;
// A vertex with more arcs than this is visited by a whole workgroup.
constexpr int kHugeDeg = 4096;
// Arcs per BFS frontier item: a frontier vertex with a longer list is split
// into several items so that hubs are expanded by many wavefronts at once.
constexpr int kChunk = 256;
// Threads per workgroup of the persistent solve kernel.
constexpr int kBlock = 1024;

// Per-phase trace records kept by the persistent kernel (one per global
// relabel that found active vertices): the first kTraceCap of a call.
constexpr int kTraceCap = 256;
constexpr int kTraceFields = 8;
enum : int {
    kTrLevels = 0,   // BFS levels of the global relabel that opened the phase
    kTrActive,       // active vertices it found
    kTrRounds,       // push/relabel rounds run
    kTrReason,       // why the phase ended: 0 no active vertex left, 1 round cap, 2 relabel budget,
                     // 3 no excess delivered for max(stall_rounds, levels) rounds
    kTrRelabels,     // relabels in the phase
    kTrRelabelled,   // distinct vertices relabelled
    kTrPushes,       // pushes in the phase
    kTrLastDeliv     // last round in which excess reached t or a deficient vertex
};

// Learned phase schedule: sizes of the value network (features, hidden
// units, actions), its flat parameter count, and one policy-trace record per
// phase (features, action, phase duration in wall-clock ticks).
constexpr int kPolF = 16;
constexpr int kPolH = 32;
constexpr int kPolK = 8;
constexpr int kPolParams = kPolH * kPolF + kPolH + kPolH * kPolH + kPolH + kPolK * kPolH + kPolK;
constexpr int kPolRec = kPolF + 2;
enum : int32_t { kPolicyFixed = 0, kPolicyLearned = 1, kPolicyExplore = 2, kPolicyForced = 3 };

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
    kStRounds,
    kStBfsTicks,
    kStPrTicks,
    kStRieTicks,
    kStCount
};

// Groups of the two-level grid barrier.
constexpr int kBarGroups = 8;
struct alignas(128) PaddedU32 {
    uint32_t v;
    uint32_t pad[31];
};

// One active-vertex list of the push/relabel rounds: vertices with short arc
// lists fill items[0, light) from the front, long ones items[n-heavy, n) from
// the back, and huge ones (more than kHugeDeg arcs) a list of their own;
// `hgrab` hands out the huge ones to workgroups.  The BFS reserves
// {light, heavy} together as one 64-bit counter (light in the low half).
struct alignas(32) ListCtr {
    int32_t light;
    int32_t heavy;
    int32_t huge;
    int32_t hgrab;
    int32_t pad[4];
};

// Device control block: barrier words on their own cache lines, then loop
// counters.  Reset by k_reset_ctrl before every solving call.
struct Ctrl {
    PaddedU32 bar_count;  // monotonic barrier arrivals of the launch (groups, for large teams)
    PaddedU32 abort;
    PaddedU32 bar_group[kBarGroups];  // arrivals per group of workgroups (two-level barrier)
    int32_t qcount[4];  // frontier items per BFS level, triple-buffered
    int32_t qverts[4];  // vertices discovered per BFS level (direction rule), same buffering
    int64_t qarcs[4];   // their arcs
    ListCtr lst[3];     // active lists of the rounds, triple-buffered
    int32_t nrelab;     // vertices relabelled in the current phase
    int32_t status;
    int32_t err;        // update validation: 1 id range, 2 capacity range, 4 duplicate
    int32_t stop;       // set by the leader when the time budget ran out
    int32_t rounds;     // push/relabel rounds run by this call (round ids)
    int32_t solo_level; // BFS level reached by a stretch one workgroup ran alone
    int64_t phase_relabels;  // relabels of the current phase
    int64_t phase_pushes;    // pushes of the current phase
    int64_t phase_deliv;     // excess delivered into t or deficient vertices this phase
    int32_t ntrace;          // phases recorded in trace[]
    int32_t gap;             // lowest height found empty in this phase (|V| = none)
    int64_t feat_esum;       // excess of the active vertices found by this phase's BFS
    int32_t feat_hist[8];    // their count per bin of floor(log2 e) / 4 (last bin open)
    int32_t action;          // phase action chosen by the schedule
    int32_t feat_reached;    // vertices this phase's BFS reached (roots included)
    int64_t prev_pushes;     // pushes and relabels of the previous phase of the call
    int64_t prev_relabels;
    int32_t trace[kTraceCap][kTraceFields];
    int64_t deficit;    // sum of e(v) < 0 over v not in {s, t} at termination
    int64_t e_t;        // e(t) at termination
    int64_t cut;        // cut capacity (k_min_cut)
    // state of the rounds a workgroup ran alone, handed to the others
    int64_t solo_last_deliv;
    int32_t solo_r, solo_done, solo_reason, solo_last_change;
    int32_t check;      // failed invariants of the debug check (bits, see k_check_state)
    int32_t pad_;
    int32_t pull_cnt[4];  // list sizes of the local pulls (ping-pong)
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
    int32_t *list[3];   // n each: active lists of the push/relabel rounds
    int32_t *huge[3];   // active vertices with more than kHugeDeg arcs, per list
    int32_t *mark;      // n: id of the round list a vertex was last added to
    int32_t *rmark;     // n: id of the phase a vertex last relabelled in
    int32_t *relab;     // n: vertices relabelled in the current phase
    int32_t *hcount;    // n+1: vertices at each height below |V| (gap heuristic)
    int32_t *heavy_all; // vertices with long arc lists (topology-driven sweeps)
    int32_t n_heavy_all;
    // Every vertex's arc list in items of at most kChunk arcs, {vertex, first
    // arc, end arc, 0}: the first item of every vertex in vertex order, then
    // the further items of long lists, second items first (bottom-up BFS
    // levels); null: no bottom-up levels.
    const int4 *bu_items;
    int32_t n_bu_items;
    float *ptrace;      // kTraceCap x kPolRec policy-trace records, or null
    Ctrl *ctrl;
    // Optional part tags (null: none).  Only vertices tagged part_want can be
    // BFS roots; with part_restrict the BFS also enters only such vertices and
    // the height reset leaves every other vertex's height as it is.
    const uint8_t *part;
    int32_t part_want;
    int32_t part_restrict;
};

// Part tags of the push-pull update and of the flow extraction.
enum : uint8_t { kPartS = 0, kPartT = 1, kPartP = 2 };

struct LoopParams {
    int32_t kc;              // KERNELCYCLES: push/relabel operations per vertex visit
    int32_t mode;            // 0 data-driven, 1 topology-driven
    int64_t max_iter;        // < 0 unlimited
    int64_t deadline_ticks;  // wall-clock ticks allowed for one launch (> 0)
    int64_t barrier_ticks;   // wall-clock ticks one grid-barrier wait may take
    int64_t relabel_budget;  // relabels allowed per phase before a global relabel
    int32_t max_rounds;      // push/relabel rounds allowed per phase
    int32_t seq_base;        // first round id of this call (marks stay unique)
    int32_t rounds_per_level;  // > 0: a phase also stops after this many rounds per
                               // level of the BFS that started it (+16)
    int32_t use_gap;           // gap heuristic on (1) or off (0)
    int32_t stall_rounds;      // > 0: a phase ends after max(this, BFS levels) rounds without delivery
    int32_t policy_mode;       // kPolicyFixed / Learned / Explore / Forced
    const float *policy_w;     // value-network parameters (kPolParams), or null
    float policy_margin;       // learned: leave action 0 only when it predicts this much less
    float policy_explore;      // explore: probability of a uniformly drawn action
    uint64_t policy_seed;      // explore: counter-based draws keyed by (seed, seq_base, phase)
    int32_t policy_action;     // forced: the action of every phase
    float batch_fraction;      // edges of the update batch / m (1 for a static solve)
    int32_t policy_per_call;   // 1: the action of a call's first phase holds for all its phases
    int32_t solo_items;        // a BFS level with at most this many frontier items, and a round
                               // whose list holds at most this many vertices (none huge), runs on
                               // one workgroup alone (workgroup barriers); 0 = never
    int32_t combine;           // 1: a workgroup adds up a round's pushes per target vertex before
                               // touching its excess (graphs with vertices of huge degree)
    int32_t no_rie;            // 1: no RemoveInvalidEdges (pushes never exceed the excess, so no
                               // deficit is created; the flow extraction needs that)
    int32_t lazy_items;        // a BFS level of at least this many frontier items reads an arc's
                               // twin residual only for heads not reached yet
    int32_t bu_alpha;          // > 0: a BFS level runs bottom-up when its frontier's arcs times this
                               // exceed the arcs of the vertices not reached yet, and stays
                               // bottom-up while the frontier holds at least n / bu_beta vertices
    int32_t bu_beta;
    int32_t walk;              // 1: long arc lists are visited by a walk that pushes downhill in arc
                               // order and stops when the excess is gone (full scan only to relabel)
};

// Result of one instance of a batched solve.
struct BatchResult {
    int64_t value;   // e(t) plus the deficits
    int32_t status;  // loop status (kSolved, kDeadline, ...)
    int32_t pad;
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
// Local stage of a dynamic update (after the clamp and the source
// re-saturation): saturate the updated arcs that cross the last cut from its
// source side to its sink side, then `rounds` rounds of pulls into the
// deficits at the batch's arc ends (the last round without handing deficits
// on).  Uses list[1], list[2] and ctrl->pull_cnt; pmark tags tag0 .. tag0 + rounds.
hipError_t launch_local_stage(const DevGraph &g, const int64_t *ids, int64_t k, int32_t *pmark, int32_t tag0,
                              int rounds, hipStream_t st);
hipError_t launch_loop(const DevGraph &g, const LoopParams &p, int grid, hipStream_t st);
hipError_t launch_min_cut(const DevGraph &g, uint8_t *d_side, hipStream_t st);
// Invariant check of the state into ctrl->check (cleared first): 1 c_f < 0,
// 2 pair sum broken, 4 excess != residual change, and when solved 8 active
// vertex left, 16 residual arc from the source side to the sink side.
hipError_t launch_check_state(const DevGraph &g, int solved, hipStream_t st);
// Batched solve: `count` workgroups of `block` threads (256, 512 or 1024);
// workgroup j solves instance order[j] of graphs[] from scratch with
// KERNELCYCLES kc[order[j]] and writes res[order[j]].
hipError_t launch_batch(const DevGraph *graphs, const int32_t *order, int count, const LoopParams &p,
                        const int32_t *kc, BatchResult *res, int block, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t st);
hipError_t launch_fill_f32(float *p, int64_t count, float value, hipStream_t st);
// Value network (mf_policy.hip): loss gradient over N samples (grad and loss
// are cleared first), forward outputs, one Adam step.
hipError_t launch_mlp_grad(const float *theta, const float *X, const int32_t *act, const float *y, int N,
                           float *grad, float *loss, hipStream_t st);
hipError_t launch_mlp_forward(const float *theta, const float *X, int N, float *Q, hipStream_t st);
hipError_t launch_adam(float *theta, const float *grad, float *m, float *v, int step, float lr, hipStream_t st);
// Largest co-resident workgroup count of the loop kernel.
hipError_t loop_max_coresident(int device, int *blocks);
// Two solve loops side by side in one cooperative launch of `grid` (>= 2)
// workgroups, split by the arc counts work[0] (view 0) and work[1] (view 1);
// d_views / d_params: device tables of the two views and their loop
// parameters (both with the same walk setting).  The views must touch
// disjoint vertices and arc pairs.
hipError_t launch_teams(const DevGraph *d_views, const LoopParams *d_params, bool walk, const int64_t *work,
                        int grid, hipStream_t st);
hipError_t teams_max_coresident(int device, int *blocks);
// part[v] = T if h(v) < |V| else S; work[0] += arcs of S, work[1] += arcs of T.
hipError_t launch_part_from_heights(const DevGraph &g, uint8_t *part, int64_t *work, hipStream_t st);
// part[v] = P where neither g.h nor hv reached v.
hipError_t launch_part_localized(const DevGraph &g, const int32_t *hv, uint8_t *part, hipStream_t st);
// Saturate every residual arc from an S vertex to a T vertex.
hipError_t launch_saturate_cut(const DevGraph &g, const uint8_t *part, hipStream_t st);
// View of the state (rev: reversed arcs, negated excesses) and its write-back
// for the arcs and vertices tagged `want`.
hipError_t launch_view_make(const DevGraph &g, int2 *varc, int64_t *ve, int rev, hipStream_t st);
hipError_t launch_view_merge(const DevGraph &g, const int2 *varc, const int64_t *ve, const uint8_t *part,
                             uint8_t want, int rev, hipStream_t st);
// Per-edge flow (int32[m]) of the valid flow whose residuals are carc[].y.
hipError_t launch_edge_flow(const DevGraph &g, const int2 *carc, int32_t *rem, int32_t *flow, hipStream_t st);

// Batch staging of mf_apply_updates_noalloc: a static device array per GPU
// (int64 ids, then int32 capacities) for at most kNoAllocMaxUpdates updates.
constexpr int64_t kNoAllocMaxUpdates = 1 << 20;
constexpr int64_t kNoAllocIdsBytes = kNoAllocMaxUpdates * (int64_t)sizeof(int64_t);
constexpr int64_t kNoAllocCapsBytes = kNoAllocMaxUpdates * (int64_t)sizeof(int32_t);
// Resolve the array's device address on `device` (once per device; call with
// the handle's set-up).  noalloc_scratch returns it, or null before set-up.
hipError_t noalloc_scratch_setup(int device);
void *noalloc_scratch(int device);

// Device build of the merged arc-pair layout (mf_build.hip).  alloc /
// release: temporary device memory of the build; alloc_keep: memory the
// handle keeps (and frees with itself).
struct BuildAlloc {
    std::function<hipError_t(void **, size_t)> alloc;
    std::function<void(void *)> release;
    std::function<hipError_t(void **, size_t)> alloc_keep;
};
struct DeviceLayout {
    int32_t A = 0;
    int32_t max_pair_mult = 1;  // most half-edges (input edges, either direction) in one arc pair
    int32_t *row_ptr = nullptr;   // n+1
    int2 *arc = nullptr;          // A: {head, capacity}
    int32_t *twin = nullptr;      // A
    int32_t *cap = nullptr;       // A
    int32_t *edge2arc = nullptr;  // m, -1 for self-loops
    int32_t *ecap = nullptr;      // m: the input capacities
};
// Inputs are host arrays already checked (row pointers monotone from 0 to m,
// heads in range, capacities >= 0).  With renumber, the layout numbers the
// vertices by falling degree (edges at either end, ties by the caller's id):
// vertex v of the caller is vertex (*h_new_of_old)[v] of the layout, and
// edge ids (edge2arc) keep the caller's numbering; without it
// *h_new_of_old comes back empty.  The arc row pointers come back to the host
// in h_arc_row_ptr.  Errors: a HIP error, or hipErrorInvalidValue with *err
// (too many arcs, a capacity sum above int32).
hipError_t build_layout_device(int32_t n, int64_t m, const int64_t *h_row_ptr, const int32_t *h_col,
                               const int32_t *h_cap, bool renumber, const BuildAlloc &mem, hipStream_t st,
                               DeviceLayout *out, std::vector<int32_t> *h_arc_row_ptr,
                               std::vector<int32_t> *h_new_of_old, std::string *err);

// Index of every arc of a renumbered layout in the layout the caller's
// numbering gives (arcs sorted by the caller's (tail, head)), from the
// device arrays arc and twin and the host array old_of_new (the inverse of
// new_of_old); the result comes back to the host.  Temporary device memory
// from mem: about 28 bytes per arc.
hipError_t caller_arc_order(int32_t n, int64_t A, const int2 *arc, const int32_t *twin,
                            const std::vector<int32_t> &old_of_new, const BuildAlloc &mem, hipStream_t st,
                            std::vector<int32_t> *h_caller_of_arc);

// True once the process has begun to exit (the C atexit handlers run).  The
// HIP runtime tears itself down in those handlers, so objects released after
// that point free only their host memory; the device memory goes with the
// process.
bool process_exiting();

}  // namespace mf

struct mf_policy;
namespace mf {
// Device parameters and device of a policy object (mf_policy_api.cpp).
const float *policy_device_params(const mf_policy *p);
int policy_device(const mf_policy *p);
}  // namespace mf
