/*
 * mf.h - exact maximum flow / minimum cut on one AMD Instinct MI355X (gfx950),
 * static and after batches of edge-capacity changes.
 *
 * The method is the GPU push-relabel of Kannappan, Kumar and Nasre,
 * "Efficient Dynamic MaxFlow Computation on GPUs" (arXiv 2511.05895):
 * the static solve of Sec. 3 (Alg. 1-3) and the Dynamic Push Relabel of
 * Sec. 4.1 (Alg. 4-5), run data-driven (Sec. 5.3) or topology-driven
 * (Sec. 5.2) on a bi-directional CSR (Sec. 5.1).
 *
 * Conventions for every call
 *  - Every call returns an int status: MF_OK (0) or one of the MF_E* codes.
 *    mf_last_error() gives the text of the last failure on that handle.
 *  - Host pointers are read (or written) only during the call; the library
 *    never keeps them.  Pointers documented as "device" must be addresses in
 *    the handle's device memory space (e.g. from hipMalloc or a torch CUDA
 *    tensor) and are read on the handle's stream during the call.
 *  - Calls are synchronous: when one returns, its GPU work has finished.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - No C++ exception crosses this interface.
 *  - Integer sizes: capacities int32 (each edge in [0, limit], limit <= 2^30,
 *    see mf_cap_limit), excesses and flow values int64, vertex ids int32,
 *    edge ids int64 in [0, m) (m < 2^31), merged arcs < 2^31.
 */
#ifndef MF_H
#define MF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MF_API __attribute__((visibility("default")))

/* status codes */
#define MF_OK 0
#define MF_EINVAL 1   /* bad argument; the handle is unchanged               */
#define MF_ENOMEM 2   /* device or host allocation failed                    */
#define MF_EDEVICE 3  /* HIP runtime error or device-side abort              */
#define MF_ESTATE 4   /* call not allowed in the handle's current state      */
#define MF_ETIMEOUT 5 /* iteration limit reached before the loop converged   */
#define MF_EPENDING 6 /* (server) the request has not been committed yet     */
#define MF_EBUSY 7    /* (server) the request queue is full; nothing queued  */

/* work distribution of the push/relabel and invalid-edge sweeps */
#define MF_MODE_DATA 0     /* worklist of active vertices (Sec. 5.3)          */
#define MF_MODE_TOPOLOGY 1 /* every vertex, idle when inactive (Sec. 5.2)     */

typedef struct mf_handle mf_handle_t;

/* Directed input graph in CSR form.  Edge id i is CSR position i; its tail is
 * the row v with row_ptr[v] <= i < row_ptr[v+1], its head col[i].  Duplicate
 * edges, antiparallel edges and self-loops are allowed (Sec. 2.1 places no
 * restriction on E).  row_ptr: int64[n+1], col: int32[m]. */
typedef struct {
    int32_t n;
    int64_t m;
    const int64_t *row_ptr;
    const int32_t *col;
} mf_csr_t;

typedef struct {
    int32_t kernel_cycles;  /* KERNELCYCLES of Alg. 2: push/relabel attempts per
                               active vertex per visit; 0 = 1 (Sec. 6.1 uses
                               the average degree, round(m/n); with rounds a
                               vertex that keeps excess is visited again in
                               the next round)                               */
    int32_t mode;           /* MF_MODE_DATA (default) or MF_MODE_TOPOLOGY     */
    int32_t grid_blocks;    /* workgroups of the persistent solve kernel;
                               0 = chosen from the graph size; 1 = one
                               workgroup (no grid-wide barrier)              */
    int32_t device;         /* HIP device ordinal (default 0)                 */
    int64_t max_iterations; /* loop rounds (global relabel + sweeps) allowed
                               per call; < 0 unlimited (default)            */
    int32_t time_budget_ms; /* wall time one solve launch may take before it
                               stops with MF_ETIMEOUT (resumable); 0 = 60 s */
    int32_t max_rounds;     /* push/relabel rounds between two global relabels;
                               0 = 65536                                     */
    int32_t relabel_budget; /* relabels allowed between two global relabels
                               before the next one is forced; 0 = max(1024, n/16) */
    int32_t rounds_per_level; /* a phase also ends after this many rounds per
                               level of the BFS that began it (+16); 0 = 1,
                               < 0 = no such cap                             */
    int32_t flags;          /* MF_FLAG_* bits                                 */
    int32_t stall_rounds;   /* a phase also ends once no excess has reached t
                               or a deficient vertex for max(stall_rounds, L)
                               rounds, L = levels of the BFS that began it
                               (exact labels bring excess that only moves
                               downhill to a root within L rounds);
                               0 = 3, < 0 = no such rule                     */
    int32_t solo_items;     /* a BFS level whose frontier holds at most this
                               many items (arc ranges of up to 256 arcs), and
                               a push/relabel round whose list holds at most
                               this many vertices (none of more than 4096
                               arcs), is run by one workgroup alone, with
                               workgroup barriers between its levels or
                               rounds, while the others wait; 0 = 128,
                               < 0 = never                                   */
    int32_t lazy_items;     /* a BFS level whose frontier holds at least this
                               many items reads the residual of an arc's
                               twin (a gather from anywhere in the arc array)
                               only for heads the BFS has not reached yet,
                               one dependent load later; smaller levels read
                               it alongside the head's height; 0 = 1024,
                               < 0 = never                                   */
    int32_t bottom_up;      /* direction-optimising global relabel: a BFS
                               level runs bottom-up (every vertex not reached
                               yet looks for a parent on the frontier among
                               its own arcs and stops at the first) when the
                               frontier's arcs times this number exceed the
                               arcs of the vertices not reached yet, plus
                               (this number - 1) times the arcs of those that
                               the previous global relabel of the same call
                               did not reach (a bottom-up level scans their
                               lists in full), and stays bottom-up while the
                               frontier holds at least 1/24 of the vertices;
                               the levels and heights are those of the
                               top-down BFS; 0 = 14, < 0 = top-down only
                               (always so with one workgroup)                */
    int32_t vertex_order;   /* MF_ORDER_*: how the handle numbers the vertices
                               internally.  Falling degree puts the hubs'
                               heights and excesses on a few cache lines and
                               starts every arc list with its hub neighbours.
                               Every call takes and returns the caller's
                               vertex and edge ids whatever the order.        */
    /* Device memory of the handle (optional, both or neither): dev_alloc
     * returns `bytes` of device memory on opts.device (aligned to 256 bytes)
     * or NULL, dev_free releases it; both get alloc_ctx.  A caching allocator
     * (torch's, say) can supply the handle this way.  NULL: hipMalloc and
     * hipFree.  dev_free is called from mf_destroy, after the handle's
     * stream has drained. */
    void *(*dev_alloc)(size_t bytes, void *ctx);
    void (*dev_free)(void *ptr, void *ctx);
    void *alloc_ctx;
} mf_opts_t;

/* opts.flags: turn the gap heuristic on (Sec. 2.2 names gap relabelling as a
 * standard push-relabel heuristic; off by default).  With it, a relabel that
 * empties a height makes every vertex above it count as cut off from the sink
 * until the next global relabel. */
#define MF_FLAG_GAP 1
/* opts.flags: dynamic updates by Dynamic Push-Pull (Sec. 4.2, Alg. 8) instead
 * of Dynamic Push Relabel (Alg. 4).  After the capacity changes land (Alg. 5),
 * the vertices the last global relabel reached form T and the rest S; every
 * residual arc from S to T is saturated; deficient vertices of S pull flow
 * (Alg. 6, forward BFS from s and the overflowing vertices of S) while
 * overflowing vertices of T push (backward BFS from t and the deficient
 * vertices of T), the two sides side by side in one launch; the remaining
 * excess and deficits meet in P, the vertices neither BFS reached, where the
 * dynamic push-relabel loop runs on P alone.  Values, cuts and every other
 * output are the same as without the flag. */
#define MF_FLAG_PUSH_PULL 2
/* opts.flags: after every solving call, check the state on the device: c_f >=
 * 0, every arc pair's residuals sum to its capacities, every excess equals
 * its vertex's residual change (sum over its arcs of c_f - c), and, once
 * solved, no active vertex and no residual arc from the source side to the
 * sink side.  A failed check returns MF_EDEVICE naming it. */
#define MF_FLAG_DEBUG_CHECKS 4
/* opts.vertex_order: MF_ORDER_AUTO (0) numbers the vertices by falling
 * degree (edges at either end, ties by id) for graphs of more than 8192
 * vertices and keeps the caller's order for smaller ones; MF_ORDER_INPUT
 * keeps the caller's order; MF_ORDER_DEGREE always numbers by degree. */
#define MF_ORDER_AUTO 0
#define MF_ORDER_INPUT 1
#define MF_ORDER_DEGREE 2
/* opts.flags: visit vertices of more than 32 arcs with the cycle of Alg. 2
 * as written (a scan of the whole arc list for the lowest residual neighbour
 * height, then pushes to the arcs at that height or a relabel) instead of the
 * default walk, which pushes downhill in arc order, stops once the excess is
 * gone and scans the whole list only to relabel.  Results are the same. */
#define MF_FLAG_SCAN_FIRST 8
/* opts.flags: dynamic updates go straight from the batch repair (Alg. 5) to
 * the global loop of Alg. 4, without the default local stage.  The local
 * stage, run from a solved state only, saturates the batch's arcs that now
 * cross the last cut from its source side to its sink side (Alg. 8 on the
 * batch) and then fills the deficits at the ends of the batch's arcs from
 * in-neighbours that hold excess (pulls as in Alg. 6, without heights; a few
 * rounds, handing what is still lacking on to the givers).  Every step is a
 * push along a residual arc and the global loop's termination test is
 * unchanged, so results are the same with or without it. */
#define MF_FLAG_GLOBAL_ONLY 16

/* Counters of the last mf_solve / mf_apply_updates* / mf_resume call. */
typedef struct {
    int64_t iterations;       /* loop rounds that ran push/relabel            */
    int64_t global_relabels;  /* backward BFS passes                          */
    int64_t bfs_levels;       /* BFS levels expanded, summed over passes      */
    int64_t bfs_vertices;     /* vertices given a height by the BFS (roots too) */
    int64_t bfs_arcs;         /* arcs examined by the BFS                     */
    int64_t pr_vertex_cycles; /* push/relabel cycles run on active vertices   */
    int64_t pr_arcs;          /* arcs scanned by push/relabel                 */
    int64_t pushes;
    int64_t relabels;
    int64_t rie_arcs;         /* arcs scanned by RemoveInvalidEdges           */
    int64_t rie_saturations;
    int64_t updates;          /* edge updates applied                         */
    int64_t clamps;           /* arcs whose flow was clamped to a new capacity */
    int64_t source_pushes;    /* arcs out of s saturated                      */
    int64_t rounds;           /* push/relabel rounds                          */
    int64_t loop_launches;    /* launches of the persistent solve kernel      */
    int64_t grid_blocks;      /* workgroups of that kernel                    */
    double bfs_ms;            /* device wall time in global relabels          */
    double pr_ms;             /* ... in push/relabel rounds                   */
    double rie_ms;            /* ... in RemoveInvalidEdges                    */
    double loop_kernel_ms;    /* HIP-event time of the solve kernel launches  */
    double call_ms;           /* HIP-event time of the whole call's GPU work  */
} mf_stats_t;

/* Fill *opts with the defaults described above. */
MF_API void mf_default_opts(mf_opts_t *opts);

/* Create a handle for graph g with per-edge capacities cap (int32[m], host),
 * source s and sink t (Sec. 2.1).  Builds the bi-directional CSR of Sec. 5.1:
 * all input edges between one unordered vertex pair become ONE arc pair (the
 * residual c_f(u,v) = c(u,v) - f(u,v) + f(v,u) of Sec. 2.3 is per vertex pair),
 * arcs of a vertex sorted by neighbour id; self-loops get no arc.  Uploads it
 * to device memory owned by the handle.  Does not solve.
 * opts may be NULL (defaults).  *out receives the handle.
 * Errors: MF_EINVAL (n < 2, m < 0 or m >= 2^31, s == t, s/t/col out of range,
 * row_ptr not non-decreasing from 0 to m, a capacity < 0 or above the limit
 * of mf_cap_limit, opts out of range), MF_ENOMEM, MF_EDEVICE. */
MF_API int mf_create(const mf_csr_t *g, const int32_t *cap, int32_t s, int32_t t,
                     const mf_opts_t *opts, mf_handle_t **out);

/* Free the handle and its device memory.  NULL is ignored. */
MF_API void mf_destroy(mf_handle_t *h);

/* Text of the last error on h (or of the last failed mf_create when h is
 * NULL).  Owned by the library; valid until the next call on h. */
MF_API const char *mf_last_error(const mf_handle_t *h);

/* Static solve from scratch on the current capacities (Alg. 1): reset the
 * flow, saturate the arcs out of s, then loop {global relabel; stop if no
 * active vertex; PushRelabel (Alg. 2); RemoveInvalidEdges (Alg. 3)}.
 * Every deficient vertex is a BFS root too (as in Alg. 4), so the value is
 * exact even when RemoveInvalidEdges leaves deficits.
 * Errors: MF_ETIMEOUT (max_iterations or the time budget reached; the state
 * is a valid intermediate state that mf_resume continues), MF_EDEVICE. */
MF_API int mf_solve(mf_handle_t *h);

/* Dynamic update (Alg. 4 with Alg. 5): set edge_ids[i] to the absolute
 * capacity new_caps[i] (host arrays, k entries, a SET of distinct edge ids:
 * Sec. 4 defines a batch as a set).  Capacity 0 removes an edge, 0 -> c > 0
 * adds one (Sec. 4.1).  Applies the capacity deltas to c and c_f, clamps the
 * flow of every arc whose residual became negative (booking the returned
 * flow as excess at its tail and deficit at its head), pushes any residual
 * capacity left on arcs out of s, and resumes the loop from the previous
 * state with deficient vertices as extra sinks.
 * Requires a solved handle (MF_ESTATE otherwise).  k == 0 is allowed.  The
 * batch is uploaded with one copy through the handle's own device and pinned
 * staging buffers; they start at min(m, 2^17) updates and double when a batch
 * does not fit, so only such a batch allocates (mf_apply_updates_noalloc
 * never does).
 * Errors: MF_EINVAL (id out of range, duplicate id, capacity out of range;
 * the handle is then unchanged), MF_ESTATE, MF_ETIMEOUT, MF_EDEVICE, MF_ENOMEM
 * (staging buffers). */
MF_API int mf_apply_updates(mf_handle_t *h, const int64_t *edge_ids, const int32_t *new_caps,
                            int64_t k);

/* As mf_apply_updates, with edge_ids and new_caps in DEVICE memory (k
 * entries each); validation runs on the device before anything changes. */
MF_API int mf_apply_updates_device(mf_handle_t *h, const int64_t *d_edge_ids,
                                   const int32_t *d_new_caps, int64_t k);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * mf_apply_updates (host arrays, same rules and errors), but the batch is
 * staged in a static device array of this GPU instead of buffers the handle
 * allocates, and the call allocates nothing (no hipMalloc, hipFree or pinned
 * host memory).  At most MF_NOALLOC_MAX_UPDATES updates per call (12 MiB of
 * staging per GPU, held until the process ends); a larger k returns
 * MF_EINVAL and leaves the handle unchanged.  Every handle on one GPU shares
 * that GPU's array: calls that overlap on one GPU (from several threads) race
 * and must be serialised by the caller.  With MF_FLAG_PUSH_PULL the second
 * view of the state is allocated by mf_create, so that path allocates
 * nothing either. */
#define MF_NOALLOC_MAX_UPDATES 1048576
MF_API int mf_apply_updates_noalloc(mf_handle_t *h, const int64_t *edge_ids, const int32_t *new_caps,
                                    int64_t k);

/* Change capacities without repairing or solving (host arrays, same rules
 * as mf_apply_updates).  Leaves the handle unsolved: mf_solve must run before
 * queries.  This is how the static comparator sees an updated graph. */
MF_API int mf_set_capacities(mf_handle_t *h, const int64_t *edge_ids, const int32_t *new_caps,
                             int64_t k);

/* Continue the loop from the current state after MF_ETIMEOUT (or after a
 * call made with max_iterations == 0).  MF_ESTATE if the flow was never
 * initialised. */
MF_API int mf_resume(mf_handle_t *h);

/* Maximum-flow value of the current capacities: e(t) plus the (negative)
 * excesses of deficient vertices, the sum of e over height-0 vertices of
 * Alg. 4 (Sec. 4.1.1, final theorem).  MF_ESTATE unless solved. */
MF_API int mf_flow_value(const mf_handle_t *h, int64_t *out);

/* Minimum cut certificate (Sec. 3.1, Theorem 3 and Note 1): side_out[v] = 1
 * for the source side S = {v : h(v) >= |V|} left by the final global relabel,
 * i.e. the vertices that reach neither t nor a deficient vertex in the
 * residual graph.  This S is the largest minimum source side, the same for
 * every maximum flow.  cut_cap_out: sum of capacities of edges from S to
 * V \ S; equal to the flow value.  Either output may be NULL.
 * side_out: host uint8[n].  MF_ESTATE unless solved. */
MF_API int mf_min_cut(mf_handle_t *h, uint8_t *side_out, int64_t *cut_cap_out);

/* A maximum flow of the current capacities, per input edge (Sec. 3.1: the
 * preflow left by the loop becomes a valid flow once every excess of the
 * source side returns to s and every deficit of the sink side is filled from
 * t, along residual paths that stay inside their side; the proof of Sec.
 * 4.1.1 gives both paths).  Runs both returns on the device, on a copy of the
 * state (the handle's state, value and cut are unchanged), then splits each
 * arc pair's flow among the input edges merged into it.
 * flow_out: host int32[m], 0 <= flow_out[i] <= capacity of edge i; flow is
 * conserved at every vertex other than s and t, and the net flow out of s is
 * the flow value.  Among parallel edges the split is in no fixed order.
 * MF_ESTATE unless solved; MF_ENOMEM when the copy cannot be allocated (about
 * 20 bytes per arc and 40 per vertex, kept until mf_destroy). */
MF_API int mf_edge_flow(mf_handle_t *h, int32_t *flow_out);

/* Change the iteration limit of later calls (< 0 unlimited; 0 runs no
 * loop round, leaving the state right after initialisation or repair). */
MF_API int mf_set_max_iterations(mf_handle_t *h, int64_t limit);

/* Counters and timings of the last solving call. */
MF_API int mf_get_stats(const mf_handle_t *h, mf_stats_t *out);

/* Upper bound of the device bytes one handle of a graph with n vertices and
 * m edges allocates (merged arcs bounded by 2m), staging of update batches
 * excluded; -1 for negative sizes.  Used for admission by the server. */
MF_API int64_t mf_estimate_device_bytes(int32_t n, int64_t m);

/* Number of merged arcs A and the per-edge capacity limit: the largest
 * capacity an edge may take, min(2^30, (2^31-1) / (2k)) for k the largest
 * number of input edges between one vertex pair, so that an arc's residual
 * stays inside int32 even after one batch of deltas lands before the clamp. */
MF_API int mf_num_arcs(const mf_handle_t *h, int32_t *A_out);
MF_API int mf_cap_limit(const mf_handle_t *h, int32_t *limit_out);

/* Copy the merged layout to host arrays: row_ptr int32[n+1], col int32[A],
 * twin int32[A] (index of the reverse arc), edge2arc int32[m] (-1 for
 * self-loops).  Any pointer may be NULL. */
MF_API int mf_export_graph(mf_handle_t *h, int32_t *row_ptr, int32_t *col, int32_t *twin,
                           int32_t *edge2arc);

/* Copy the residual state to host arrays: cap int32[A] (current arc
 * capacities), cf int32[A] (residual capacities), e int64[n] (excesses),
 * height int32[n] (heights of the last global relabel or sweep), ecap
 * int32[m] (current per-edge capacities).  Any pointer may be NULL. */
MF_API int mf_export_state(mf_handle_t *h, int32_t *cap, int32_t *cf, int64_t *e,
                           int32_t *height, int32_t *ecap);

/* Restore a residual state exported by mf_export_state from a handle of the
 * same graph (cap, cf: int32[A]; e: int64[n]; ecap: int32[m]; host arrays,
 * read during the call).  Checks residuals and capacities for signs, every
 * arc pair's residuals against its capacities, every arc capacity against the
 * sum of its edges' capacities, and every excess against its vertex's
 * residual change (sum over its arcs of c_f - c); MF_EINVAL otherwise.  The
 * handle is left partial: mf_apply_updates* continue from the restored
 * state, mf_resume finishes it (the value is available after either).  Used
 * to replay one update from one state under different schedules. */
MF_API int mf_import_state(mf_handle_t *h, const int32_t *cap, const int32_t *cf, const int64_t *e,
                           const int32_t *ecap);

/* Per-phase trace of the last solving call.  A phase is the work between two
 * global relabels (Alg. 1/4 loop): one record of 8 int32 per phase, in order,
 * {BFS levels of the global relabel that opened it, active vertices it found,
 * push/relabel rounds run, end reason (0 = no active vertex left, 1 = round
 * cap, 2 = relabel budget, 3 = rounds without delivery), relabels, distinct
 * vertices relabelled, pushes, last round in which excess reached t or a
 * deficient vertex}.  Copies min(recorded, max_phases) records into out (host,
 * int32[8 * max_phases]); *n_out receives the number recorded (at most 256).
 * These are the features of the learned global-relabel schedule. */
MF_API int mf_get_trace(const mf_handle_t *h, int32_t *out, int32_t max_phases, int32_t *n_out);

/* Run the handle's GPU work on `stream` (a hipStream_t; NULL = the
 * handle's own stream). */
MF_API int mf_set_stream(mf_handle_t *h, void *stream);

/* ------------------------------------------------------------------------
 * Batched solve of many independent instances.
 *
 * Each instance is its own directed graph with its own s and t, solved from
 * scratch (the static method of Alg. 1: saturate the source, then global
 * relabel / push-relabel / RemoveInvalidEdges until no active vertex is
 * left).  The instances are packed block-diagonally into one set of device
 * arrays and each is solved by ONE workgroup of a persistent launch, so no
 * grid barrier is involved and workgroups never wait for each other.
 * Instances are grouped by their number of residual arcs into size classes;
 * each class is one launch with its own workgroup size and KERNELCYCLES,
 * instances ordered largest first inside it; the classes run side by side.
 * With use_graph the launches are captured into a hipGraph on the first solve
 * after a configuration change and that graph is replayed by later solves.
 * Values and cuts follow the same definitions as for a single handle.
 * ------------------------------------------------------------------------ */
#define MF_BATCH_MAX_CLASSES 4

typedef struct mf_batch mf_batch_t;

typedef struct {
    int32_t device;
    int32_t time_budget_ms;  /* per instance; 0 = 60 s                      */
    int32_t n_classes;       /* 1..MF_BATCH_MAX_CLASSES (default 3)         */
    int32_t use_graph;       /* 1 = capture once and replay (default), 0 = plain launches */
    int64_t class_max_arcs[MF_BATCH_MAX_CLASSES]; /* class c takes the instances
                                with at most this many residual arcs that no
                                earlier class took; ascending; the last class
                                takes the rest (default 32768, 262144)       */
    int32_t block[MF_BATCH_MAX_CLASSES];         /* threads per workgroup of a
                                class: 256, 512 or 1024 (default 256, 1024, 1024) */
    int32_t kernel_cycles[MF_BATCH_MAX_CLASSES]; /* 0 = max(1, round(m/n)) per instance */
    int32_t flags;           /* MF_FLAG_GAP                                   */
    int32_t stall_rounds;    /* as in mf_opts_t                               */
    int32_t reserved[2];     /* must be zero                                  */
} mf_batch_opts_t;

MF_API void mf_batch_default_opts(mf_batch_opts_t *opts);

/* count instances.  Instance i has n[i] vertices and m[i] edges; its CSR rows
 * are row_ptr[R_i .. R_i + n[i]] with R_i = sum_{j<i} (n[j] + 1), values local
 * to the instance (0 .. m[i]); its edges are col[E_i .. E_i + m[i]) and
 * cap[E_i ..] with E_i = sum_{j<i} m[j], col holding local vertex ids;
 * source s[i], sink t[i].  Edge ids of instance i are 0 .. m[i]-1.  Every
 * instance is checked as mf_create checks one graph (MF_EINVAL names the
 * instance).  Host arrays are read during the call only.  Does not solve. */
MF_API int mf_batch_create(int32_t count, const int32_t *n, const int64_t *m, const int64_t *row_ptr,
                           const int32_t *col, const int32_t *cap, const int32_t *s, const int32_t *t,
                           const mf_batch_opts_t *opts, mf_batch_t **out);
MF_API void mf_batch_destroy(mf_batch_t *b);
MF_API const char *mf_batch_last_error(const mf_batch_t *b);
MF_API int mf_batch_count(const mf_batch_t *b, int32_t *count);
MF_API int mf_batch_get_opts(const mf_batch_t *b, mf_batch_opts_t *opts);
/* New class split / workgroup sizes / cycles; the captured graph is rebuilt
 * by the next solve.  The device cannot change. */
MF_API int mf_batch_set_opts(mf_batch_t *b, const mf_batch_opts_t *opts);

/* Solve every instance from scratch on its current capacities.  MF_ETIMEOUT
 * when an instance ran out of its time budget, MF_EDEVICE on a device error;
 * the values of the call are then not available. */
MF_API int mf_batch_solve(mf_batch_t *b);
/* Solve only the instances of class `cls`, as one plain launch on the batch's
 * stream; *kernel_ms receives the launch's event-timed duration. */
MF_API int mf_batch_solve_class(mf_batch_t *b, int32_t cls, double *kernel_ms);
/* For every non-empty class, time each workgroup size (256, 512, 1024) x
 * KERNELCYCLES (per instance default, 1, 2, 4) with `repeats` class-alone
 * launches, keep the fastest median, and adopt the result; every candidate
 * must reach the same values (else MF_EDEVICE).  *chosen (may be NULL)
 * receives the adopted options.  Leaves the batch unsolved. */
MF_API int mf_batch_autotune(mf_batch_t *b, int32_t repeats, mf_batch_opts_t *chosen);

/* Residual arcs of every instance (int64[count]), after merging. */
MF_API int mf_batch_num_arcs(const mf_batch_t *b, int64_t *arcs);
/* values int64[count] of the last solve (MF_ESTATE before one). */
MF_API int mf_batch_values(const mf_batch_t *b, int64_t *values);
/* Event-timed duration of the last solve (all classes, fork to join). */
MF_API int mf_batch_last_ms(const mf_batch_t *b, double *kernel_ms);
/* Canonical minimum cut of instance i, as mf_min_cut (side uint8[n[i]], may
 * be NULL). */
MF_API int mf_batch_min_cut(mf_batch_t *b, int32_t i, uint8_t *side, int64_t *cut_cap);
/* Counters of instance i in its last solve. */
MF_API int mf_batch_get_stats(mf_batch_t *b, int32_t i, mf_stats_t *stats);
/* New absolute capacities for edges of instance i (local ids, distinct, in
 * [0, m[i]); capacities within that instance's per-edge limit); the next
 * solve uses them.  A rejected batch (MF_EINVAL) changes nothing. */
MF_API int mf_batch_set_capacities(mf_batch_t *b, int32_t i, const int64_t *edge_ids,
                                   const int32_t *new_caps, int64_t k);

/* ------------------------------------------------------------------------
 * Learned phase schedule.
 *
 * The paper sets how long push/relabel runs between two global relabels
 * with one fixed knob (KERNELCYCLES, Sec. 6: too few cycles cost extra
 * global relabels, too many push in the wrong direction).  Here each phase
 * (the work between two global relabels) may take one of MF_POLICY_ACTIONS
 * limit settings, chosen right after the global relabel that opens it:
 *   action:                 0    1    2    3    4    5    6    7
 *   relabel budget x        1  1/4  1/2    2    4    1    1    1
 *   rounds per BFS level x  1    1    1    1    2  1/2    2    1
 *   stall limit x           1    1    1    1    1    1  1/2  none
 * Action 0 is the fixed rule of mf_opts_t.  Every action keeps the results
 * exact (only the moment of the next global relabel changes).
 *
 * The choice is made by a value network q = W3 relu(W2 relu(W1 x + b1) + b2)
 * + b3 (fp32; MF_POLICY_FEATURES inputs, MF_POLICY_HIDDEN units per hidden
 * layer, one output per action) that predicts, for each action, the log of
 * the remaining solve time in ms.  The features x of a phase, computed on
 * the device right after its global relabel:
 *   x0  log2(1 + active vertices) / 24
 *   x1  log2(1 + sum of their excess) / 40
 *   x2..x9  fraction of them with floor(log2 e) / 4 = 0, 1, ..., 6, >= 7
 *   x10 log2(1 + BFS levels) / 12
 *   x11 fraction of the vertices the BFS reached (h < |V|)
 *   x12 log2(1 + pushes of the previous phase of the call) / 32
 *   x13 log2(1 + relabels of the previous phase) / 32
 *   x14 log2(1 + phase index in the call) / 8
 *   x15 edges of the update batch / m (1 for a static solve)
 * Parameters: one flat fp32 vector, W1 (H x F, row-major), b1, W2 (H x H),
 * b2, W3 (K x H), b3.  Training (mf_policy_train) runs full-batch Adam on the
 * device over samples (x, taken action a, target y), minimising
 * (1/N) sum (q[a] - y)^2.
 * ------------------------------------------------------------------------ */
#define MF_POLICY_FEATURES 16
#define MF_POLICY_HIDDEN 32
#define MF_POLICY_ACTIONS 8
#define MF_POLICY_FIXED 0    /* action 0 always; no network, no features      */
#define MF_POLICY_LEARNED 1  /* argmin of q when it beats q[0] by the margin,
                                else action 0 (the fixed rule is the fallback) */
#define MF_POLICY_EXPLORE 2  /* a uniformly drawn action with probability
                                `explore`, else action 0 (training data)       */
#define MF_POLICY_FORCED 3   /* `action` in every phase                        */
#define MF_POLICY_PER_CALL 16 /* OR-ed into a mode: decide at the first phase of
                                each solving call only and keep that action for
                                the call's later phases (the learned mode's
                                value then predicts the whole call's time).
                                The BFS then tallies x1..x9 and x11 in the
                                first phase only: later phases' trace records
                                hold zeros there                              */

typedef struct mf_policy mf_policy_t;

MF_API const char *mf_policy_last_error(void);
MF_API int32_t mf_policy_num_params(void);
/* Network on `device` with He-initialised weights drawn from `seed`
 * (splitmix64 counters, Box-Muller), zero biases. */
MF_API int mf_policy_create(int32_t device, uint64_t seed, mf_policy_t **out);
MF_API void mf_policy_destroy(mf_policy_t *p);
MF_API int mf_policy_get_params(mf_policy_t *p, float *out);
/* Also resets the Adam moments. */
MF_API int mf_policy_set_params(mf_policy_t *p, const float *in);
/* Q (host, N x MF_POLICY_ACTIONS) for features X (host, N x
 * MF_POLICY_FEATURES), computed on the device. */
MF_API int mf_policy_forward(mf_policy_t *p, const float *X, int32_t N, float *Q);
/* Loss and its gradient (host, mf_policy_num_params() floats) at the current
 * parameters; nothing is updated. */
MF_API int mf_policy_gradient(mf_policy_t *p, const float *X, const int32_t *actions, const float *targets,
                              int32_t N, float *grad, float *loss);
/* `steps` full-batch Adam steps (lr; beta 0.9 / 0.999; eps 1e-8) on the
 * device; *final_loss (may be NULL) is the loss after the last step. */
MF_API int mf_policy_train(mf_policy_t *p, const float *X, const int32_t *actions, const float *targets,
                           int32_t N, int32_t steps, float lr, float *final_loss);
/* Schedule of a handle's later solving calls.  The policy object must
 * outlive its use by the handle.  margin >= 0 (learned), explore in [0, 1]
 * and seed (explore), action (forced). */
MF_API int mf_set_policy(mf_handle_t *h, const mf_policy_t *policy, int32_t mode, float margin, float explore,
                         uint64_t seed, int32_t action);
/* Per-phase records of the last solving call under a non-fixed mode:
 * MF_POLICY_FEATURES + 2 floats each (features, action taken, phase
 * duration in ms); copies min(recorded, max_phases); *n_out = recorded. */
MF_API int mf_get_policy_trace(mf_handle_t *h, float *out, int32_t max_phases, int32_t *n_out);

/* ------------------------------------------------------------------------
 * Serving runtime: resident graphs taking asynchronous update requests.
 *
 * Each graph admitted to a server keeps its handle (and its solved state)
 * on the device.  A request is one update batch of one graph (absolute new
 * capacities of distinct edges, Sec. 4.1); it is validated and copied on
 * submit and queued FIFO behind the graph's earlier requests.  Worker threads
 * take ALL pending requests of a graph (up to max_group_requests and
 * max_group_edges) and commit them together: the requests are merged into one
 * set in which the latest request wins for an edge -- since capacities are
 * absolute this equals applying them one after the other -- and one dynamic
 * repair (Alg. 4/5) runs for the group.  Every request of the group then
 * receives the flow value after that commit and the graph's version, the
 * number of its requests applied so far (at least the request's own sequence
 * number): the value equals the maximum flow of the graph after its first
 * `version` requests.  Different graphs are committed by different workers at
 * the same time on their own streams, as long as their solve kernels'
 * workgroups fit on the device together (a commit waits otherwise); a launch
 * that stops early (time budget, barrier wait) is finished by mf_resume.
 * Admission: a graph is accepted only while the device bytes reserved for all
 * resident graphs (mf_estimate_device_bytes + staging for max_group_edges
 * updates) stay within memory_budget, otherwise MF_ENOMEM and nothing changes;
 * a request only while the queued requests' bytes stay within
 * max_pending_bytes, otherwise MF_EBUSY and nothing is queued.
 * All mf_server_* calls are thread-safe; errors are reported per thread by
 * mf_server_last_error().
 * ------------------------------------------------------------------------ */
typedef struct mf_server mf_server_t;

typedef struct {
    int32_t device;
    int32_t workers;            /* threads committing groups (default 4)      */
    int64_t memory_budget;      /* device bytes for resident graphs; 0 = 90 %
                                   of the free device memory at creation     */
    int64_t max_group_edges;    /* edges one commit may merge (default 2^20);
                                   also the largest request submit accepts    */
    int32_t max_group_requests; /* requests one commit may merge (default 64; 1
                                   = no group commit)                         */
    int32_t reserved0;          /* must be zero                               */
    int64_t max_pending_bytes;  /* host bytes the queued requests may hold (12
                                   per edge); beyond it mf_server_submit returns
                                   MF_EBUSY; 0 = 1 GiB                        */
    int32_t reserved[2];        /* must be zero                               */
} mf_server_opts_t;

typedef struct {
    int32_t status;      /* MF_OK, or the error of the commit (MF_ESTATE after
                            an earlier commit of the graph failed)          */
    int32_t graph;
    int64_t request;
    int64_t value;       /* flow value after the commit                     */
    int64_t version;     /* requests of the graph applied by then           */
    int64_t seq;         /* this request's 1-based sequence number in its graph */
    int64_t group_size;  /* requests merged into the commit                 */
    double submit_ms;    /* server clock (ms since creation): submitted,    */
    double start_ms;     /* commit started,                                  */
    double done_ms;      /* result available                                 */
} mf_result_t;

MF_API void mf_server_default_opts(mf_server_opts_t *opts);
MF_API const char *mf_server_last_error(void);
MF_API int mf_server_create(const mf_server_opts_t *opts, mf_server_t **out);
/* Waits until every submitted request is committed, then frees everything. */
MF_API void mf_server_destroy(mf_server_t *s);
/* Admit a graph (arguments as mf_create; opts->device is the server's),
 * solve it statically; *graph_id and *value (may be NULL) receive its id and
 * initial flow value. */
MF_API int mf_server_add_graph(mf_server_t *s, const mf_csr_t *g, const int32_t *cap, int32_t src, int32_t sink,
                               const mf_opts_t *opts, int32_t *graph_id, int64_t *value);
/* Stop taking requests for the graph, wait for its queue, free its handle
 * and its reservation. */
MF_API int mf_server_remove_graph(mf_server_t *s, int32_t graph_id);
/* Queue one request; returns at once with *request_id.  MF_EINVAL (nothing
 * queued) for an unknown graph, an id outside [0, m), a capacity outside the
 * graph's per-edge limit, a repeated id, or more than max_group_edges edges;
 * MF_EBUSY (nothing queued) when the queue's byte limit is reached. */
MF_API int mf_server_submit(mf_server_t *s, int32_t graph_id, const int64_t *edge_ids, const int32_t *new_caps,
                            int64_t k, int64_t *request_id);
/* MF_OK with *out filled once the request is committed; MF_EPENDING before.
 * A committed result stays readable (poll, wait) until mf_server_release. */
MF_API int mf_server_poll(mf_server_t *s, int64_t request_id, mf_result_t *out);
/* Block until the request is committed. */
MF_API int mf_server_wait(mf_server_t *s, int64_t request_id, mf_result_t *out);
/* Forget a committed request's result, after which its id is unknown; a
 * long-running caller releases what it has read, or the results it keeps
 * grow with every request.  MF_EPENDING if not committed yet. */
MF_API int mf_server_release(mf_server_t *s, int64_t request_id);
/* Block until every submitted request is committed. */
MF_API int mf_server_drain(mf_server_t *s);
/* Version and flow value of the graph's last commit. */
MF_API int mf_server_graph_info(mf_server_t *s, int32_t graph_id, int64_t *version, int64_t *value);
/* Reserved device bytes, the budget and the number of commits so far (any
 * pointer may be NULL). */
MF_API int mf_server_memory(mf_server_t *s, int64_t *reserved, int64_t *budget, int64_t *commits);
/* Queue bytes held, workgroup slots in use by commits in flight and the
 * device's total, and how many commits were finished by mf_resume (any
 * pointer may be NULL). */
MF_API int mf_server_load(mf_server_t *s, int64_t *pending_bytes, int32_t *slots_used, int32_t *slots,
                          int64_t *resumed);

#ifdef __cplusplus
}
#endif

#endif /* MF_H */
