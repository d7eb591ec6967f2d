/*
 * CPU oracle for exact maximum flow / minimum cut, static and after capacity
 * updates.  TEST INFRASTRUCTURE ONLY: nothing in the product library links or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code with the GPU path.
 *
 * Plain, sequential and slow on purpose.  Contents:
 *
 *  O1  Dinic's blocking-flow algorithm (the textbook method the paper cites in
 *      Sec. 2.2) on an UNMERGED residual network: one forward arc and one
 *      zero-capacity reverse arc per input edge.  Returns the maximum flow value
 *      (definition of Sec. 2.1), a valid per-edge flow, and the canonical minimum
 *      cut S* = V \ {v : v reaches t in the final residual graph}.
 *  O2  Sequential FIFO push-relabel (Goldberg-Tarjan, cited in Sec. 2.2) with
 *      global relabelling, phase one only; a second independent algorithm.
 *  O4  The paper's own method run sequentially on MERGED arc pairs (the
 *      bi-directional CSR of Sec. 5.1): initialisation and source saturation
 *      (Alg. 1), backward-BFS global relabel, PushRelabel (Alg. 2),
 *      RemoveInvalidEdges (Alg. 3), the dynamic driver (Alg. 4) and Updates
 *      Processing (Alg. 5), with the full excess recomputation the paper asks
 *      for after the updates.  Used as the bit-exact reference for the
 *      deterministic steps (initial state, update repair, BFS heights).
 *  V   Validator: checks a merged-pair residual state (capacity, pair sums,
 *      excess bookkeeping, no active vertex on the sink side, cut = value) and
 *      completes it to a valid flow by the two repair flows of the correctness
 *      proofs (excess back to s inside S, Lemma 4; deficits from t inside T,
 *      Lemma 6), each computed with O1.
 *
 * Readings of the paper that this file fixes (every one is also a comment at
 * the place it applies): merged antiparallel/duplicate edges (Sec. 2.3 residual
 * definition), deficient vertices as extra BFS roots in every solve (Alg. 4),
 * termination tested right after a fresh global relabel, re-saturation that
 * pushes the source's residual capacity instead of overwriting the excess.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EXPORT __attribute__((visibility("default")))

/* ======================================================================== */
/* Unmerged residual network                                                */
/* ======================================================================== */

typedef struct {
    int32_t n;
    int64_t narcs;   /* 2 * number of edges                                  */
    int64_t *first;  /* n+1: arcs of tail v are adj[first[v] .. first[v+1])   */
    int64_t *adj;    /* narcs: arc ids grouped by tail                       */
    int32_t *to;     /* narcs: head of arc                                   */
    int64_t *res;    /* narcs: residual capacity                             */
} unet_t;

static void unet_free(unet_t *g) {
    free(g->first); free(g->adj); free(g->to); free(g->res);
    memset(g, 0, sizeof(*g));
}

/* Edge i (tail[i] -> head[i], capacity cap[i]) becomes arc 2i with residual
 * cap[i] and its partner arc 2i+1 (head -> tail) with residual 0.  The partner
 * of arc a is a ^ 1. */
static int unet_build(unet_t *g, int32_t n, int64_t m, const int32_t *tail,
                      const int32_t *head, const int64_t *cap) {
    memset(g, 0, sizeof(*g));
    g->n = n;
    g->narcs = 2 * m;
    g->first = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->adj = (int64_t *)malloc(sizeof(int64_t) * (size_t)(g->narcs ? g->narcs : 1));
    g->to = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->narcs ? g->narcs : 1));
    g->res = (int64_t *)malloc(sizeof(int64_t) * (size_t)(g->narcs ? g->narcs : 1));
    if (!g->first || !g->adj || !g->to || !g->res) { unet_free(g); return -1; }
    for (int64_t i = 0; i < m; i++) {
        g->first[tail[i] + 1]++;
        g->first[head[i] + 1]++;
    }
    for (int32_t v = 0; v < n; v++) g->first[v + 1] += g->first[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!fill) { unet_free(g); return -1; }
    memcpy(fill, g->first, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < m; i++) {
        int64_t a = 2 * i, b = 2 * i + 1;
        g->to[a] = head[i]; g->res[a] = cap[i];
        g->to[b] = tail[i]; g->res[b] = 0;
        g->adj[fill[tail[i]]++] = a;
        g->adj[fill[head[i]]++] = b;
    }
    free(fill);
    return 0;
}

/* Tails of the CSR input (edge i belongs to row v when row_ptr[v] <= i < row_ptr[v+1]). */
static int32_t *csr_tails(int32_t n, int64_t m, const int64_t *row_ptr) {
    int32_t *tail = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    if (!tail) return NULL;
    for (int32_t v = 0; v < n; v++)
        for (int64_t i = row_ptr[v]; i < row_ptr[v + 1]; i++) tail[i] = v;
    return tail;
}

/* side[v] = 1 iff v cannot reach t in the residual network (canonical cut S*). */
static void unet_sink_side(const unet_t *g, int32_t t, uint8_t *side) {
    int32_t n = g->n;
    uint8_t *reach = (uint8_t *)calloc((size_t)n, 1);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t qh = 0, qt = 0;
    reach[t] = 1; queue[qt++] = t;
    while (qh < qt) {
        int32_t w = queue[qh++];
        for (int64_t k = g->first[w]; k < g->first[w + 1]; k++) {
            int64_t a = g->adj[k];       /* w -> v */
            int32_t v = g->to[a];
            if (!reach[v] && g->res[a ^ 1] > 0) { /* residual v -> w */
                reach[v] = 1; queue[qt++] = v;
            }
        }
    }
    for (int32_t v = 0; v < n; v++) side[v] = reach[v] ? 0 : 1;
    free(reach); free(queue);
}

/* ======================================================================== */
/* O1: Dinic                                                                */
/* ======================================================================== */

static int64_t dinic_run(unet_t *g, int32_t s, int32_t t) {
    int32_t n = g->n;
    if (s == t) return 0;
    int32_t *level = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *it = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *path = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t flow = 0;
    for (;;) {
        /* BFS levels from s over residual arcs */
        for (int32_t v = 0; v < n; v++) level[v] = -1;
        int64_t qh = 0, qt = 0;
        level[s] = 0; queue[qt++] = s;
        while (qh < qt) {
            int32_t u = queue[qh++];
            for (int64_t k = g->first[u]; k < g->first[u + 1]; k++) {
                int64_t a = g->adj[k];
                int32_t v = g->to[a];
                if (g->res[a] > 0 && level[v] < 0) { level[v] = level[u] + 1; queue[qt++] = v; }
            }
        }
        if (level[t] < 0) break;
        for (int32_t v = 0; v < n; v++) it[v] = g->first[v];
        /* blocking flow by repeated depth-first augmentation with current-arc pointers */
        int32_t top = 0, u = s;
        for (;;) {
            if (u == t) {
                int64_t b = INT64_MAX; int32_t bi = 0;
                for (int32_t i = 0; i < top; i++)
                    if (g->res[path[i]] < b) { b = g->res[path[i]]; bi = i; }
                for (int32_t i = 0; i < top; i++) { g->res[path[i]] -= b; g->res[path[i] ^ 1] += b; }
                flow += b;
                top = bi;                              /* retreat to the first saturated arc */
                u = top == 0 ? s : g->to[path[top - 1]];
                continue;
            }
            int found = 0;
            for (; it[u] < g->first[u + 1]; it[u]++) {
                int64_t a = g->adj[it[u]];
                if (g->res[a] > 0 && level[g->to[a]] == level[u] + 1) { found = 1; break; }
            }
            if (found) {
                path[top++] = g->adj[it[u]];
                u = g->to[path[top - 1]];
            } else {
                level[u] = -2;                          /* dead end for this phase */
                if (top == 0) break;
                top--;
                u = top == 0 ? s : g->to[path[top - 1]];
                it[u]++;
            }
        }
    }
    free(level); free(it); free(queue); free(path);
    return flow;
}

/* O1.  Returns the max-flow value, or -1 on allocation failure.
 * side_out (n, may be NULL): canonical source side S*.
 * flow_out (m, may be NULL): a valid flow on every input edge. */
ORC_EXPORT int64_t orc_dinic(int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *col,
                             const int32_t *cap, int32_t s, int32_t t, uint8_t *side_out,
                             int64_t *flow_out) {
    int32_t *tail = csr_tails(n, m, row_ptr);
    int64_t *c64 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    if (!tail || !c64) { free(tail); free(c64); return -1; }
    for (int64_t i = 0; i < m; i++) c64[i] = cap[i];
    unet_t g;
    if (unet_build(&g, n, m, tail, col, c64)) { free(tail); free(c64); return -1; }
    int64_t value = dinic_run(&g, s, t);
    if (side_out) unet_sink_side(&g, t, side_out);
    if (flow_out)
        for (int64_t i = 0; i < m; i++) flow_out[i] = c64[i] - g.res[2 * i];
    unet_free(&g); free(tail); free(c64);
    return value;
}

/* ======================================================================== */
/* O2: FIFO push-relabel with global relabelling (phase one)                */
/* ======================================================================== */

static void fifo_global_relabel(const unet_t *g, int32_t s, int32_t t, int32_t *h, int32_t *queue) {
    int32_t n = g->n;
    for (int32_t v = 0; v < n; v++) h[v] = n;
    int64_t qh = 0, qt = 0;
    h[t] = 0; queue[qt++] = t;
    while (qh < qt) {
        int32_t w = queue[qh++];
        for (int64_t k = g->first[w]; k < g->first[w + 1]; k++) {
            int64_t a = g->adj[k];
            int32_t v = g->to[a];
            if (v != s && h[v] == n && g->res[a ^ 1] > 0) { h[v] = h[w] + 1; queue[qt++] = v; }
        }
    }
    h[s] = n;
}

ORC_EXPORT int64_t orc_fifo_push_relabel(int32_t n, int64_t m, const int64_t *row_ptr,
                                         const int32_t *col, const int32_t *cap, int32_t s,
                                         int32_t t, uint8_t *side_out) {
    if (s == t) return 0;
    int32_t *tail = csr_tails(n, m, row_ptr);
    int64_t *c64 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    if (!tail || !c64) { free(tail); free(c64); return -1; }
    for (int64_t i = 0; i < m; i++) c64[i] = cap[i];
    unet_t g;
    if (unet_build(&g, n, m, tail, col, c64)) { free(tail); free(c64); return -1; }
    int32_t *h = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *e = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *fifo = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *scratch = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t *inq = (uint8_t *)calloc((size_t)n, 1);
    /* saturate every arc out of s */
    for (int64_t k = g.first[s]; k < g.first[s + 1]; k++) {
        int64_t a = g.adj[k];
        int64_t d = g.res[a];
        if (d > 0) { g.res[a] = 0; g.res[a ^ 1] += d; e[g.to[a]] += d; e[s] -= d; }
    }
    int64_t relabels_since = 0;
    int need_global = 1;
    int64_t qh = 0, qt = 0; /* circular FIFO of capacity n */
    int64_t qcount = 0;
    for (;;) {
        if (need_global) {
            fifo_global_relabel(&g, s, t, h, scratch);
            for (int32_t v = 0; v < n; v++) { cur[v] = g.first[v]; inq[v] = 0; }
            qh = qt = qcount = 0;
            for (int32_t v = 0; v < n; v++)
                if (v != s && v != t && e[v] > 0 && h[v] < n) {
                    fifo[qt] = v; qt = (qt + 1) % n; qcount++; inq[v] = 1;
                }
            need_global = 0;
            relabels_since = 0;
        }
        if (qcount == 0) break;
        int32_t u = fifo[qh]; qh = (qh + 1) % n; qcount--; inq[u] = 0;
        while (e[u] > 0 && h[u] < n) {
            if (cur[u] == g.first[u + 1]) {
                int32_t minh = INT32_MAX;
                for (int64_t k = g.first[u]; k < g.first[u + 1]; k++) {
                    int64_t a = g.adj[k];
                    if (g.res[a] > 0 && h[g.to[a]] < minh) minh = h[g.to[a]];
                }
                h[u] = (minh >= n) ? n : minh + 1;
                cur[u] = g.first[u];
                relabels_since++;
                continue;
            }
            int64_t a = g.adj[cur[u]];
            int32_t v = g.to[a];
            if (g.res[a] > 0 && h[u] == h[v] + 1) {
                int64_t d = e[u] < g.res[a] ? e[u] : g.res[a];
                g.res[a] -= d; g.res[a ^ 1] += d; e[u] -= d; e[v] += d;
                if (v != s && v != t && !inq[v] && h[v] < n) {
                    fifo[qt] = v; qt = (qt + 1) % n; qcount++; inq[v] = 1;
                }
            } else {
                cur[u]++;
            }
        }
        if (relabels_since >= n) need_global = 1;
    }
    int64_t value = e[t];
    if (side_out) unet_sink_side(&g, t, side_out);
    free(h); free(e); free(cur); free(fifo); free(scratch); free(inq);
    unet_free(&g); free(tail); free(c64);
    return value;
}

/* ======================================================================== */
/* Merged arc pairs (bi-directional CSR, Sec. 5.1)                          */
/* ======================================================================== */
/* Every unordered vertex pair {u, v} (u != v) joined by at least one input
 * edge gets ONE arc u->v in u's list and ONE arc v->u in v's list, twins of
 * each other.  The residual definition of Sec. 2.3, c_f(u,v) = c(u,v) -
 * f(u,v) + f(v,u), is per vertex pair, so parallel and antiparallel input
 * edges are summed: cap[u->v] = sum of capacities of input edges u->v.
 * Self-loops get no arc.  Layout: arcs of each vertex sorted by neighbour id. */

typedef struct { int32_t owner, nbr; int64_t edge; int32_t fwd; } pentry_t;

static int pentry_cmp(const void *x, const void *y) {
    const pentry_t *a = (const pentry_t *)x, *b = (const pentry_t *)y;
    if (a->owner != b->owner) return a->owner < b->owner ? -1 : 1;
    if (a->nbr != b->nbr) return a->nbr < b->nbr ? -1 : 1;
    if (a->edge != b->edge) return a->edge < b->edge ? -1 : 1;
    return a->fwd - b->fwd;
}

static pentry_t *pairs_entries(int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *col,
                               int64_t *cnt_out) {
    int64_t cnt = 0;
    pentry_t *ent = (pentry_t *)malloc(sizeof(pentry_t) * (size_t)(2 * m + 1));
    if (!ent) return NULL;
    for (int32_t u = 0; u < n; u++)
        for (int64_t i = row_ptr[u]; i < row_ptr[u + 1]; i++) {
            int32_t v = col[i];
            if (u == v) continue;
            ent[cnt].owner = u; ent[cnt].nbr = v; ent[cnt].edge = i; ent[cnt].fwd = 1; cnt++;
            ent[cnt].owner = v; ent[cnt].nbr = u; ent[cnt].edge = i; ent[cnt].fwd = 0; cnt++;
        }
    qsort(ent, (size_t)cnt, sizeof(pentry_t), pentry_cmp);
    *cnt_out = cnt;
    return ent;
}

/* Number of merged arcs, or -1 on allocation failure. */
ORC_EXPORT int64_t orc_pairs_count(int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *col) {
    int64_t cnt;
    pentry_t *ent = pairs_entries(n, m, row_ptr, col, &cnt);
    if (!ent) return -1;
    int64_t A = 0;
    for (int64_t k = 0; k < cnt; k++)
        if (k == 0 || ent[k].owner != ent[k - 1].owner || ent[k].nbr != ent[k - 1].nbr) A++;
    free(ent);
    return A;
}

/* Fill the merged layout.  arc_row_ptr: n+1; arc_col, arc_twin, arc_cap: A;
 * edge2arc: m (-1 for self-loops).  Capacities are summed in int64 and
 * stored as int32; returns -2 if a summed capacity overflows int32. */
ORC_EXPORT int32_t orc_pairs_build(int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *col,
                                   const int32_t *cap, int32_t *arc_row_ptr, int32_t *arc_col,
                                   int32_t *arc_twin, int32_t *arc_cap, int32_t *edge2arc) {
    int64_t cnt;
    pentry_t *ent = pairs_entries(n, m, row_ptr, col, &cnt);
    if (!ent) return -1;
    int64_t *capsum = (int64_t *)calloc((size_t)(cnt + 1), sizeof(int64_t));
    int32_t *rev_arc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    if (!capsum || !rev_arc) { free(ent); free(capsum); free(rev_arc); return -1; }
    for (int64_t i = 0; i < m; i++) { edge2arc[i] = -1; rev_arc[i] = -1; }
    for (int32_t v = 0; v <= n; v++) arc_row_ptr[v] = 0;
    int32_t A = -1;
    for (int64_t k = 0; k < cnt; k++) {
        if (k == 0 || ent[k].owner != ent[k - 1].owner || ent[k].nbr != ent[k - 1].nbr) {
            A++;
            arc_col[A] = ent[k].nbr;
            arc_row_ptr[ent[k].owner + 1]++;
        }
        if (ent[k].fwd) { capsum[A] += cap[ent[k].edge]; edge2arc[ent[k].edge] = A; }
        else rev_arc[ent[k].edge] = A;
    }
    A++;
    for (int32_t v = 0; v < n; v++) arc_row_ptr[v + 1] += arc_row_ptr[v];
    int32_t rc = 0;
    for (int32_t a = 0; a < A; a++) {
        if (capsum[a] > INT32_MAX) rc = -2;
        arc_cap[a] = (int32_t)capsum[a];
    }
    for (int64_t i = 0; i < m; i++)
        if (edge2arc[i] >= 0) { arc_twin[edge2arc[i]] = rev_arc[i]; arc_twin[rev_arc[i]] = edge2arc[i]; }
    free(ent); free(capsum); free(rev_arc);
    return rc;
}

/* ======================================================================== */
/* O4: the paper's method, sequential, on merged arc pairs                  */
/* ======================================================================== */

/* Alg. 1 initialisation: e = 0, h = 0, c_f = c on every arc; then saturate
 * every residual arc out of s.  With merged pairs, c_f(u,s) <- c(u,s) + c(s,u)
 * is the same as adding the pushed amount to the twin. */
ORC_EXPORT void orc_paper_init(int32_t n, int32_t A, const int32_t *row_ptr, const int32_t *col,
                               const int32_t *twin, const int32_t *cap, int32_t s,
                               int32_t *cf, int64_t *e, int32_t *h) {
    for (int32_t v = 0; v < n; v++) { e[v] = 0; h[v] = 0; }
    for (int32_t a = 0; a < A; a++) cf[a] = cap[a];
    for (int32_t a = row_ptr[s]; a < row_ptr[s + 1]; a++) {
        int32_t d = cf[a];
        if (d > 0) { cf[a] = 0; cf[twin[a]] += d; e[col[a]] += d; e[s] -= d; }
    }
}

/* Global relabel (Alg. 4 height reset + BFS_Backward): roots are t and every
 * deficient vertex other than s (height 0); every other vertex starts at |V|.
 * A vertex v joins level L+1 when it has a residual arc v->w to a vertex w of
 * level L.  s is never entered, so it stays at |V|. */
ORC_EXPORT void orc_paper_global_relabel(int32_t n, const int32_t *row_ptr, const int32_t *col,
                                         const int32_t *twin, const int32_t *cf, const int64_t *e,
                                         int32_t s, int32_t t, int32_t *h) {
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t qh = 0, qt = 0;
    for (int32_t v = 0; v < n; v++) {
        if (v == t || (v != s && e[v] < 0)) { h[v] = 0; queue[qt++] = v; }
        else h[v] = n;
    }
    while (qh < qt) {
        int32_t w = queue[qh++];
        for (int32_t a = row_ptr[w]; a < row_ptr[w + 1]; a++) {
            int32_t v = col[a];
            if (v != s && h[v] == n && cf[twin[a]] > 0) { h[v] = h[w] + 1; queue[qt++] = v; }
        }
    }
    free(queue);
}

/* Alg. 2 on one vertex, sequentially: up to kc push-or-relabel cycles, each
 * picking the lowest residual neighbour (strict <, first in arc order). */
static void paper_push_relabel_vertex(int32_t n, const int32_t *row_ptr, const int32_t *col,
                                      const int32_t *twin, int32_t *cf, int64_t *e, int32_t *h,
                                      int32_t u, int32_t kc, int64_t *pushes, int64_t *relabels) {
    for (int32_t cnt = 0; cnt < kc; cnt++) {
        if (!(h[u] < n && e[u] > 0)) continue;
        int64_t ep = e[u];
        int32_t vhat = -1, ahat = -1;
        int64_t hhat = INT64_MAX;
        for (int32_t a = row_ptr[u]; a < row_ptr[u + 1]; a++) {
            if (cf[a] <= 0) continue;
            int32_t hp = h[col[a]];
            if (hp < hhat) { vhat = col[a]; ahat = a; hhat = hp; }
        }
        if (vhat < 0) continue;                 /* no residual arc: nothing to do */
        if (h[u] > hhat) {
            int64_t d = ep < cf[ahat] ? ep : cf[ahat];
            cf[ahat] -= (int32_t)d; cf[twin[ahat]] += (int32_t)d;
            e[u] -= d; e[vhat] += d;
            (*pushes)++;
        } else {
            h[u] = (int32_t)hhat + 1;
            (*relabels)++;
        }
    }
}

/* Alg. 3 on one vertex: saturate every residual arc that is steep under h+. */
static void paper_remove_invalid_vertex(const int32_t *row_ptr, const int32_t *col,
                                        const int32_t *twin, int32_t *cf, int64_t *e,
                                        const int32_t *h, int32_t u) {
    for (int32_t a = row_ptr[u]; a < row_ptr[u + 1]; a++) {
        if (cf[a] <= 0) continue;
        int32_t v = col[a];
        if (h[u] > h[v] + 1) {
            int32_t c = cf[a];
            e[u] -= c; e[v] += c; cf[twin[a]] += c; cf[a] = 0;
        }
    }
}

/* value = e(t) + sum of the (negative) excesses of deficient vertices, i.e. the
 * sum of e over the height-0 vertices at termination (Alg. 4 last loop). */
ORC_EXPORT int64_t orc_paper_value(int32_t n, const int64_t *e, int32_t s, int32_t t) {
    int64_t v = e[t];
    for (int32_t u = 0; u < n; u++)
        if (u != s && u != t && e[u] < 0) v += e[u];
    return v;
}

/* The while-loop of Alg. 1 / Alg. 4: global relabel, then the active set
 * A = {u not in {s,t} : e(u) > 0, h(u) < |V|} is tested right after the fresh
 * BFS; if empty the loop ends, else PushRelabel then RemoveInvalidEdges run
 * over A (increasing vertex id).  max_iter < 0 means unbounded.
 * stats (may be NULL): [0] iterations, [1] pushes, [2] relabels.
 * Returns 0 when solved, 1 when max_iter ran out first. */
ORC_EXPORT int32_t orc_paper_loop(int32_t n, const int32_t *row_ptr, const int32_t *col,
                                  const int32_t *twin, int32_t *cf, int64_t *e, int32_t *h,
                                  int32_t s, int32_t t, int32_t kc, int64_t max_iter,
                                  int64_t *stats) {
    int32_t *act = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t iters = 0, pushes = 0, relabels = 0;
    int32_t rc = 0;
    for (;;) {
        orc_paper_global_relabel(n, row_ptr, col, twin, cf, e, s, t, h);
        int32_t na = 0;
        for (int32_t u = 0; u < n; u++)
            if (u != s && u != t && e[u] > 0 && h[u] < n) act[na++] = u;
        if (na == 0) break;
        if (max_iter >= 0 && iters >= max_iter) { rc = 1; break; }
        for (int32_t i = 0; i < na; i++)
            paper_push_relabel_vertex(n, row_ptr, col, twin, cf, e, h, act[i], kc, &pushes, &relabels);
        for (int32_t i = 0; i < na; i++)
            paper_remove_invalid_vertex(row_ptr, col, twin, cf, e, h, act[i]);
        iters++;
    }
    if (stats) { stats[0] = iters; stats[1] = pushes; stats[2] = relabels; }
    free(act);
    return rc;
}

/* Alg. 5 (Updates Processing) followed by the excess recomputation and source
 * re-saturation of Alg. 4.
 *  - each update (edge id, new capacity c'): c_f(u,v) += c' - c and the stored
 *    capacities follow (the paper leaves the store implicit);
 *  - every arc whose residual went negative folds the overflow into its twin
 *    (flow clamped to the new capacity), scanning all arcs as the paper does;
 *  - e(u) recomputed from scratch: e(u) = sum over u's arcs of (c_f - c);
 *  - the residual capacity of every arc out of s is pushed (c_f(s,u) -> 0,
 *    twin += d, e(u) += d, e(s) -= d).  The paper writes e(u) <- c(s,u) here;
 *    read literally that would erase the recomputed excess, so the push of
 *    the remaining residual is used (it produces the pair state the paper
 *    states for c_f).
 * Edge ids must be distinct.  Returns 0. */
ORC_EXPORT int32_t orc_paper_apply_updates(int32_t n, int32_t A, const int32_t *row_ptr,
                                           const int32_t *col, const int32_t *twin, int32_t *cap,
                                           const int32_t *edge2arc, int32_t *ecap, int32_t *cf,
                                           int64_t *e, int32_t s, const int64_t *ids,
                                           const int32_t *new_caps, int64_t k) {
    for (int64_t i = 0; i < k; i++) {
        int64_t id = ids[i];
        int32_t delta = new_caps[i] - ecap[id];
        ecap[id] = new_caps[i];
        int32_t a = edge2arc[id];
        if (a < 0) continue;
        cf[a] += delta;
        cap[a] += delta;
    }
    for (int32_t a = 0; a < A; a++)
        if (cf[a] < 0) { cf[twin[a]] += cf[a]; cf[a] = 0; }
    for (int32_t u = 0; u < n; u++) {
        int64_t x = 0;
        for (int32_t a = row_ptr[u]; a < row_ptr[u + 1]; a++) x += (int64_t)cf[a] - cap[a];
        e[u] = x;
    }
    for (int32_t a = row_ptr[s]; a < row_ptr[s + 1]; a++) {
        int32_t d = cf[a];
        if (d > 0) { cf[a] = 0; cf[twin[a]] += d; e[col[a]] += d; e[s] -= d; }
    }
    return 0;
}

/* ======================================================================== */
/* V: validator and phase-two completion to a valid flow                    */
/* ======================================================================== */

/* Route `need` units from the super source through residual arcs restricted
 * to the vertex set `in_set` (side[v] == want) and apply the result to cf.
 * Sources: vertices with positive `supply`; sinks: vertices with positive
 * `demand`.  Returns the amount routed. */
static int64_t route_inside(int32_t n, const int32_t *row_ptr, const int32_t *col,
                            const int32_t *twin, int32_t *cf, const uint8_t *side, uint8_t want,
                            const int64_t *supply, const int64_t *demand) {
    /* count arcs */
    int64_t m = 0;
    for (int32_t u = 0; u < n; u++) {
        if (side[u] != want) continue;
        if (supply[u] > 0) m++;
        if (demand[u] > 0) m++;
        for (int32_t a = row_ptr[u]; a < row_ptr[u + 1]; a++)
            if (side[col[a]] == want && cf[a] > 0) m++;
    }
    int32_t *tl = (int32_t *)calloc((size_t)(m + 1), sizeof(int32_t));
    int32_t *hd = (int32_t *)calloc((size_t)(m + 1), sizeof(int32_t));
    int64_t *cp = (int64_t *)calloc((size_t)(m + 1), sizeof(int64_t));
    int32_t *arc_of = (int32_t *)calloc((size_t)(m + 1), sizeof(int32_t));
    int64_t k = 0;
    int32_t SRC = n, SNK = n + 1;
    for (int32_t u = 0; u < n; u++) {
        if (side[u] != want) continue;
        if (supply[u] > 0) { tl[k] = SRC; hd[k] = u; cp[k] = supply[u]; arc_of[k] = -1; k++; }
        if (demand[u] > 0) { tl[k] = u; hd[k] = SNK; cp[k] = demand[u]; arc_of[k] = -1; k++; }
        for (int32_t a = row_ptr[u]; a < row_ptr[u + 1]; a++)
            if (side[col[a]] == want && cf[a] > 0) { tl[k] = u; hd[k] = col[a]; cp[k] = cf[a]; arc_of[k] = a; k++; }
    }
    unet_t g;
    int64_t routed = -1;
    if (unet_build(&g, n + 2, m, tl, hd, cp) == 0) {
        routed = dinic_run(&g, SRC, SNK);
        for (int64_t i = 0; i < m; i++) {
            int32_t a = arc_of[i];
            if (a < 0) continue;
            int64_t phi = cp[i] - g.res[2 * i];
            if (phi) { cf[a] -= (int32_t)phi; cf[twin[a]] += (int32_t)phi; }
        }
        unet_free(&g);
    }
    free(tl); free(hd); free(cp); free(arc_of);
    return routed;
}

/* Validate a merged-pair residual state and complete it to a valid flow.
 * Returns 0 if valid, else the number of the first failed check:
 *   1 c_f < 0            2 twin or pair-sum broken     3 excess bookkeeping
 *   4 s reaches a root   5 active vertex left on the sink side
 *   6 cut capacity != value                 7 excess not returnable to s
 *   8 deficit not fillable from t            9 repaired flow not conserved
 * side_out (n): source side (vertices that reach no root). value_out: value.
 * flow_out (A, may be NULL): net pair flow cap - c_f' after the repair. */
ORC_EXPORT int32_t orc_validate(int32_t n, int32_t A, const int32_t *row_ptr, const int32_t *col,
                                const int32_t *twin, const int32_t *cap, const int32_t *cf_in,
                                const int64_t *e, int32_t s, int32_t t, uint8_t *side_out,
                                int64_t *value_out, int64_t *flow_out) {
    int32_t rc = 0;
    int32_t *cf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(A ? A : 1));
    int32_t *h = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *sup = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int64_t *dem = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    memcpy(cf, cf_in, sizeof(int32_t) * (size_t)A);
    for (int32_t a = 0; a < A && !rc; a++) if (cf[a] < 0) rc = 1;
    for (int32_t a = 0; a < A && !rc; a++) {
        int32_t b = twin[a];
        if (b < 0 || b >= A || twin[b] != a) rc = 2;
        else if ((int64_t)cf[a] + cf[b] != (int64_t)cap[a] + cap[b]) rc = 2;
    }
    for (int32_t u = 0; u < n && !rc; u++) {
        int64_t x = 0;
        for (int32_t a = row_ptr[u]; a < row_ptr[u + 1]; a++) x += (int64_t)cf[a] - cap[a];
        if (x != e[u]) rc = 3;
    }
    int64_t value = 0;
    if (!rc) {
        orc_paper_global_relabel(n, row_ptr, col, twin, cf, e, s, t, h);
        for (int32_t v = 0; v < n; v++) side_out[v] = h[v] >= n ? 1 : 0;
        /* s is never entered by the BFS; check separately that s reaches no root */
        for (int32_t a = row_ptr[s]; a < row_ptr[s + 1] && !rc; a++)
            if (cf[a] > 0 && h[col[a]] < n) rc = 4;
        for (int32_t v = 0; v < n && !rc; v++)
            if (v != s && v != t && e[v] > 0 && h[v] < n) rc = 5;
    }
    if (!rc) {
        value = orc_paper_value(n, e, s, t);
        int64_t cut = 0;
        for (int32_t u = 0; u < n; u++)
            if (side_out[u])
                for (int32_t a = row_ptr[u]; a < row_ptr[u + 1]; a++)
                    if (!side_out[col[a]]) cut += cap[a];
        if (cut != value) rc = 6;
    }
    if (!rc) {
        int64_t need = 0;
        for (int32_t v = 0; v < n; v++)
            if (v != s && v != t && e[v] > 0) { sup[v] = e[v]; need += e[v]; }
        dem[s] = need;
        if (need && route_inside(n, row_ptr, col, twin, cf, side_out, 1, sup, dem) != need) rc = 7;
    }
    if (!rc) {
        memset(sup, 0, sizeof(int64_t) * (size_t)n);
        memset(dem, 0, sizeof(int64_t) * (size_t)n);
        int64_t need = 0;
        for (int32_t v = 0; v < n; v++)
            if (v != s && v != t && e[v] < 0) { dem[v] = -e[v]; need += -e[v]; }
        sup[t] = need;
        if (need && route_inside(n, row_ptr, col, twin, cf, side_out, 0, sup, dem) != need) rc = 8;
    }
    if (!rc) {
        for (int32_t u = 0; u < n && !rc; u++) {
            int64_t x = 0;
            for (int32_t a = row_ptr[u]; a < row_ptr[u + 1]; a++) {
                if (cf[a] < 0) rc = 9;
                x += (int64_t)cf[a] - cap[a];
            }
            if (u == t) { if (x != value) rc = 9; }
            else if (u == s) { if (x != -value) rc = 9; }
            else if (x != 0) rc = 9;
        }
        if (!rc && flow_out)
            for (int32_t a = 0; a < A; a++) flow_out[a] = (int64_t)cap[a] - cf[a];
    }
    if (value_out) *value_out = value;
    free(cf); free(h); free(sup); free(dem);
    return rc;
}
