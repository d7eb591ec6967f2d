// Host-side conversion of a read-back control block into the public counters.
#pragma once

#include "../../include/mf.h"
#include "mf_internal.h"

namespace mf {

// Counters of Ctrl::stat into *s; tick_ms is one wall-clock tick in ms.
// Launch counts, grid size and event timings are left to the caller.
inline void stats_from_ctrl(const Ctrl &c, double tick_ms, mf_stats_t *s) {
    *s = mf_stats_t{};
    s->iterations = c.stat[kStIterations];
    s->global_relabels = c.stat[kStGlobalRelabels];
    s->bfs_levels = c.stat[kStLevels];
    s->bfs_vertices = c.stat[kStBfsVertices];
    s->bfs_arcs = c.stat[kStBfsArcs];
    s->pr_vertex_cycles = c.stat[kStPrCycles];
    s->pr_arcs = c.stat[kStPrArcs];
    s->pushes = c.stat[kStPushes];
    s->relabels = c.stat[kStRelabels];
    s->rie_arcs = c.stat[kStRieArcs];
    s->rie_saturations = c.stat[kStRieSat];
    s->updates = c.stat[kStUpdates];
    s->clamps = c.stat[kStClamps];
    s->source_pushes = c.stat[kStSourcePushes];
    s->rounds = c.stat[kStRounds];
    s->bfs_ms = c.stat[kStBfsTicks] * tick_ms;
    s->pr_ms = c.stat[kStPrTicks] * tick_ms;
    s->rie_ms = c.stat[kStRieTicks] * tick_ms;
}

}  // namespace mf
