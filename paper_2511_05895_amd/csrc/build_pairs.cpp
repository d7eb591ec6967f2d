// Bi-directional CSR builder (Sec. 5.1 of the paper), host side, run once per
// mf_create.  Every unordered vertex pair {u, v} (u != v) joined by at least
// one input edge gets one arc u->v in u's list and one arc v->u in v's list,
// twins of each other.  Parallel and antiparallel input edges share the pair
// (the residual of Sec. 2.3 is per vertex pair): cap[u->v] is the sum of the
// capacities of the input edges u->v.  Arcs of a vertex are sorted by
// neighbour id; self-loops get no arc.
//
// Two stable counting sorts (by neighbour, then by owner) give the sorted
// half-edge list in O(n + m) time, without comparisons.
#include "build_pairs.h"

#include <algorithm>
#include <cstring>

namespace mf {

int check_graph(int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const int32_t *cap,
                int32_t s, int32_t t, std::string *err) {
    auto bad = [&](const char *why) {
        *err = why;
        return -1;
    };
    if (n < 2) return bad("n must be >= 2");
    if (m < 0 || m >= (int64_t)INT32_MAX) return bad("m must be in [0, 2^31-1)");
    if (s < 0 || s >= n || t < 0 || t >= n) return bad("s or t out of range");
    if (s == t) return bad("s == t");
    if (!row_ptr || (m > 0 && (!col || !cap))) return bad("null graph or capacity array");
    if (row_ptr[0] != 0 || row_ptr[n] != m) return bad("row_ptr must run from 0 to m");
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return bad("row_ptr not non-decreasing");
    for (int64_t i = 0; i < m; ++i) {
        if (col[i] < 0 || col[i] >= n) return bad("col out of range");
        if (cap[i] < 0) return bad("negative capacity");
    }
    return 0;
}

int64_t edge_cap_limit(int32_t mult) {
    const int64_t lim = (int64_t)INT32_MAX / (2 * (int64_t)(mult > 0 ? mult : 1));
    return lim < (1ll << 30) ? lim : (1ll << 30);
}

int build_pairs(int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const int32_t *cap,
                HostPairs *out, std::string *err) {
    // half-edges: for edge i (u -> v, u != v) one entry owned by u (forward) and
    // one owned by v (reverse).  Encoded as (edge << 1) | reverse.
    int64_t nh = 0;
    for (int32_t u = 0; u < n; ++u)
        for (int64_t i = row_ptr[u]; i < row_ptr[u + 1]; ++i)
            if (col[i] != u) nh += 2;
    if (nh / 2 > INT32_MAX / 2) {
        *err = "too many arcs for int32 arc indices";
        return -1;
    }
    std::vector<int32_t> tail(m);
    for (int32_t u = 0; u < n; ++u)
        for (int64_t i = row_ptr[u]; i < row_ptr[u + 1]; ++i) tail[i] = u;
    auto owner_of = [&](int64_t code) -> int32_t {
        int64_t i = code >> 1;
        return (code & 1) ? col[i] : tail[i];
    };
    auto nbr_of = [&](int64_t code) -> int32_t {
        int64_t i = code >> 1;
        return (code & 1) ? tail[i] : col[i];
    };
    // pass 1: counting sort by neighbour
    std::vector<int64_t> cnt((size_t)n + 1, 0);
    for (int64_t i = 0; i < m; ++i)
        if (col[i] != tail[i]) {
            cnt[col[i] + 1]++;   // forward entry, neighbour = head
            cnt[tail[i] + 1]++;  // reverse entry, neighbour = tail
        }
    for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    std::vector<int64_t> by_nbr(nh);
    for (int64_t i = 0; i < m; ++i)
        if (col[i] != tail[i]) {
            by_nbr[cnt[col[i]]++] = (i << 1);
            by_nbr[cnt[tail[i]]++] = (i << 1) | 1;
        }
    // pass 2: stable counting sort by owner
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t k = 0; k < nh; ++k) cnt[owner_of(by_nbr[k]) + 1]++;
    for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    std::vector<int64_t> sorted(nh);
    for (int64_t k = 0; k < nh; ++k) sorted[cnt[owner_of(by_nbr[k])]++] = by_nbr[k];
    by_nbr.clear();
    by_nbr.shrink_to_fit();

    out->n = n;
    out->m = m;
    out->row_ptr.assign((size_t)n + 1, 0);
    out->edge2arc.assign((size_t)m, -1);
    std::vector<int32_t> rev_arc((size_t)m, -1);
    std::vector<int64_t> capsum;
    capsum.reserve((size_t)(nh / 2 + 1));
    out->col.clear();
    out->col.reserve((size_t)(nh / 2 + 1));
    // multiplicity of each arc pair (input edges in either direction)
    std::vector<int32_t> mult;
    mult.reserve((size_t)(nh / 2 + 1));
    int64_t A = -1;
    int32_t prev_owner = -1, prev_nbr = -1;
    for (int64_t k = 0; k < nh; ++k) {
        const int64_t code = sorted[k];
        const int32_t o = owner_of(code), v = nbr_of(code);
        if (o != prev_owner || v != prev_nbr) {
            ++A;
            out->col.push_back(v);
            capsum.push_back(0);
            mult.push_back(0);
            out->row_ptr[o + 1]++;
            prev_owner = o;
            prev_nbr = v;
        }
        const int64_t i = code >> 1;
        mult[A]++;
        if (code & 1) {
            rev_arc[i] = (int32_t)A;
        } else {
            capsum[A] += cap[i];
            out->edge2arc[i] = (int32_t)A;
        }
    }
    ++A;
    for (int32_t v = 0; v < n; ++v) out->row_ptr[v + 1] += out->row_ptr[v];
    out->A = (int32_t)A;
    out->twin.assign((size_t)A, -1);
    for (int64_t i = 0; i < m; ++i) {
        const int32_t a = out->edge2arc[i];
        if (a >= 0) {
            out->twin[a] = rev_arc[i];
            out->twin[rev_arc[i]] = a;
        }
    }
    out->cap.resize((size_t)A);
    int32_t kmax = 1;
    for (int64_t a = 0; a < A; ++a) {
        if (capsum[a] > INT32_MAX) {
            *err = "summed capacity of one arc exceeds int32";
            return -1;
        }
        out->cap[a] = (int32_t)capsum[a];
        kmax = std::max(kmax, mult[a]);
    }
    out->max_pair_mult = kmax;
    return 0;
}

}  // namespace mf
