// Device build of the merged arc-pair layout (the bi-directional CSR of
// Sec. 5.1), run once per mf_create.  Every unordered vertex pair {u, v}
// (u != v) joined by at least one input edge gets one arc u->v in u's list
// and one arc v->u in v's list, twins of each other; parallel and antiparallel
// input edges share the pair (the residual of Sec. 2.3 is per vertex pair),
// cap[u->v] is the sum of the capacities of the input edges u->v, arcs of a
// vertex are sorted by neighbour id and self-loops get no arc.
//
// Steps (all on the device):
//  1. tail of every input edge (binary search in the input row pointers);
//  2. two half-edges per edge that is not a self-loop, one owned by each end,
//     keyed (owner, neighbour), compacted;
//  3. a stable least-significant-digit radix sort of the keys (4-bit digits:
//     per-tile digit counts, one exclusive scan over all tiles, a stable
//     scatter that ranks each item within its tile);
//  4. runs of equal keys are arcs: arc index by a scan of the run starts,
//     capacity sums, edge -> arc map, twins, multiplicity, row pointers.
#include "mf_internal.h"

namespace mf {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;  // 2048 values per workgroup
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;  // 4096 items per tile
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kDigits = 16;  // 4-bit digits

__device__ __forceinline__ int lane_of() { return (int)__lane_id(); }

// Exclusive scan of one value per thread over the workgroup; returns this
// thread's prefix and sets *total.  Every thread calls it.
template <int T>
__device__ __forceinline__ int64_t block_excl_scan(int64_t x, int64_t *total) {
    __shared__ int64_t s_w[T / 64];
    const int lane = lane_of(), w = threadIdx.x >> 6;
    int64_t incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < T / 64; ++k) {
        const int64_t v = s_w[k];
        if (k < w) off += v;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return off + incl - x;
}

// --- exclusive scan of int64 data in place (recursive over block sums) ---

__global__ void __launch_bounds__(kScanThreads) k_scan_local(int64_t *data, int64_t n, int64_t *sums) {
    const int64_t base = ((int64_t)blockIdx.x * kScanThreads + threadIdx.x) * kScanItems;
    int64_t v[kScanItems];
    int64_t t = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = base + j < n ? data[base + j] : 0;
        t += v[j];
    }
    int64_t tot = 0;
    int64_t run = block_excl_scan<kScanThreads>(t, &tot);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) data[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_add(int64_t *data, int64_t n, const int64_t *offs) {
    const int64_t base = ((int64_t)blockIdx.x * kScanThreads + threadIdx.x) * kScanItems;
    const int64_t o = offs[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j < n) data[base + j] += o;
}

constexpr int64_t kScanBlockSpan = (int64_t)kScanThreads * kScanItems;

int64_t scan_tmp_count(int64_t n) {
    int64_t t = 0;
    while (n > 1) {
        n = (n + kScanBlockSpan - 1) / kScanBlockSpan;
        t += n + 1;
    }
    return t + 1;
}

hipError_t scan_exclusive(int64_t *data, int64_t n, int64_t *tmp, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kScanBlockSpan - 1) / kScanBlockSpan;
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanThreads), 0, st, data, n, tmp);
    if (nb > 1) {
        hipError_t e = scan_exclusive(tmp, nb, tmp + nb + 1, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, st, data, n, tmp);
    }
    return hipGetLastError();
}

// --- stable LSD radix sort of (uint64 key, uint32 value) pairs ---

// Digit counts of every tile: hist[d * tiles + tile].
__global__ void __launch_bounds__(kSortThreads) k_rs_hist(const uint64_t *keys, int64_t n, int shift,
                                                          int64_t *hist, int64_t tiles) {
    __shared__ int s_cnt[kDigits];
    if (threadIdx.x < kDigits) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int j = threadIdx.x; j < kSortTile; j += kSortThreads) {
        const int64_t i = base + j;
        if (i < n) atomicAdd(&s_cnt[(int)((keys[i] >> shift) & (kDigits - 1))], 1);
    }
    __syncthreads();
    if (threadIdx.x < kDigits) hist[(int64_t)threadIdx.x * tiles + blockIdx.x] = s_cnt[threadIdx.x];
}

// Stable scatter of one tile: thread t holds items [16t, 16t+16) of the tile
// in order.  Its digit counts go to cnt[d][t]; an exclusive scan of cnt in
// digit-major order gives, for (d, t), the items of the tile with a smaller
// digit plus those with digit d in earlier threads.  Subtracting the first
// (the tile's start of digit d) and adding the scanned tile offset of digit d
// gives the global position of t's first item with digit d.
__global__ void __launch_bounds__(kSortThreads)
    k_rs_scatter(const uint64_t *keys, const uint32_t *vals, int64_t n, int shift, const int64_t *offs,
                 int64_t tiles, uint64_t *keys_out, uint32_t *vals_out) {
    __shared__ int s_cnt[kDigits * kSortThreads];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)t * kSortItems;
    uint64_t k[kSortItems];
    uint32_t v[kSortItems];
    int dg[kSortItems];
    int c[kDigits];
#pragma unroll
    for (int d = 0; d < kDigits; ++d) c[d] = 0;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const bool ok = base + j < n;
        k[j] = ok ? keys[base + j] : 0;
        v[j] = ok ? vals[base + j] : 0;
        dg[j] = ok ? (int)((k[j] >> shift) & (kDigits - 1)) : -1;
#pragma unroll
        for (int d = 0; d < kDigits; ++d) c[d] += dg[j] == d;
    }
#pragma unroll
    for (int d = 0; d < kDigits; ++d) s_cnt[d * kSortThreads + t] = c[d];
    __syncthreads();
    // exclusive scan of the 4096 counts, 16 consecutive entries per thread
    int loc[kDigits];
    int sum = 0;
#pragma unroll
    for (int j = 0; j < kDigits; ++j) {
        loc[j] = s_cnt[t * kDigits + j];
        sum += loc[j];
    }
    int64_t tot = 0;
    int run = (int)block_excl_scan<kSortThreads>((int64_t)sum, &tot);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kDigits; ++j) {
        s_cnt[t * kDigits + j] = run;
        run += loc[j];
    }
    __syncthreads();
    int64_t pos[kDigits];
#pragma unroll
    for (int d = 0; d < kDigits; ++d)
        pos[d] = offs[(int64_t)d * tiles + blockIdx.x] + (s_cnt[d * kSortThreads + t] - s_cnt[d * kSortThreads]);
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        if (dg[j] < 0) continue;
        int64_t p = -1;
#pragma unroll
        for (int d = 0; d < kDigits; ++d)
            if (dg[j] == d) p = pos[d]++;
        if (p < 0 || p >= n) continue;  // only on a broken scan: never write out of bounds
        keys_out[p] = k[j];
        vals_out[p] = v[j];
    }
}

// --- the layout ---

// Tail of every input edge: the row v with row_ptr[v] <= i < row_ptr[v+1].
__global__ void k_tails(const int64_t *rp, int32_t n, int64_t m, int32_t *tail) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0, hi = n - 1;  // largest v with rp[v] <= i
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo + 1) / 2;
            if (rp[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        tail[i] = lo;
    }
}

// 1 for an edge that is not a self-loop.
__global__ void k_nonloop(const int32_t *tail, const int32_t *col, int64_t m, int64_t *flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = tail[i] != col[i] ? 1 : 0;
}

// The two half-edges of every edge that is not a self-loop, at 2 * pos[i]:
// key (owner << b) | neighbour, value (edge << 1) | reverse.  With perm, the
// ends are the vertices' numbers in the handle's order (perm[caller's id]).
__global__ void k_half_edges(const int32_t *tail, const int32_t *col, int64_t m, const int64_t *pos, int b,
                             const int32_t *perm, uint64_t *keys, uint32_t *vals) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t u = tail[i], v = col[i];
        if (u == v) continue;
        if (perm) {
            u = perm[u];
            v = perm[v];
        }
        const int64_t p = 2 * pos[i];
        keys[p] = ((uint64_t)u << b) | (uint64_t)v;
        vals[p] = (uint32_t)((uint64_t)i << 1);
        keys[p + 1] = ((uint64_t)v << b) | (uint64_t)u;
        vals[p + 1] = (uint32_t)(((uint64_t)i << 1) | 1u);
    }
}

// 1 where a run of equal keys (one arc) starts.
__global__ void k_run_starts(const uint64_t *keys, int64_t nh, int64_t *flag) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nh; k += (int64_t)gridDim.x * blockDim.x)
        flag[k] = (k == 0 || keys[k] != keys[k - 1]) ? 1 : 0;
}

// Per half-edge k (sorted): its arc a = idx[k] + start(k) - 1 (idx: the
// exclusive scan of the run starts).  A run start records the arc's neighbour, owner and first
// position; a forward half-edge adds its capacity and fixes edge2arc, a
// reverse one the arc of the reverse direction.
__global__ void k_arcs(const uint64_t *keys, const uint32_t *vals, const int64_t *idx, int64_t nh, int64_t A, int b,
                       const int32_t *cap, int32_t *col_out, int32_t *owner, int64_t *start, int64_t *capsum,
                       int32_t *edge2arc, int32_t *rev_arc) {
    const uint64_t mask = (1ull << b) - 1;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nh; k += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[k];
        const bool first = k == 0 || keys[k - 1] != key;
        const int64_t a = idx[k] + (first ? 0 : -1);
        if (a < 0 || a >= A) continue;  // only on a broken scan
        if (first) {
            col_out[a] = (int32_t)(key & mask);
            owner[a] = (int32_t)(key >> b);
            start[a] = k;
        }
        const uint32_t code = vals[k];
        const int64_t i = (int64_t)(code >> 1);
        if (code & 1u) {
            rev_arc[i] = (int32_t)a;
        } else {
            edge2arc[i] = (int32_t)a;
            atomicAdd((unsigned long long *)&capsum[a], (unsigned long long)cap[i]);
        }
    }
}

// Arc records, capacities, the largest multiplicity (half-edges per arc) and
// a flag for a capacity sum above int32.
__global__ void k_arc_records(const int32_t *col, const int64_t *capsum, const int64_t *start, int64_t A, int64_t nh,
                              int2 *arc, int32_t *cap, int32_t *maxmult, int32_t *overflow) {
    int32_t mm = 0;
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < A; a += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = capsum[a];
        if (c > INT32_MAX) atomicOr(overflow, 1);
        const int32_t cc = (int32_t)min(c, (int64_t)INT32_MAX);
        cap[a] = cc;
        arc[a] = make_int2(col[a], cc);
        const int64_t len = (a + 1 < A ? start[a + 1] : nh) - start[a];
        mm = max(mm, (int32_t)min(len, (int64_t)INT32_MAX));
    }
    atomicMax(maxmult, mm);
}

// row_ptr[v] = first arc owned by a vertex >= v (arcs are sorted by owner).
__global__ void k_row_ptr(const int32_t *owner, int64_t A, int32_t n, int32_t *row_ptr) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = A;
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (owner[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        row_ptr[v] = (int32_t)lo;
    }
}

__global__ void k_twins(const int32_t *edge2arc, const int32_t *rev_arc, int64_t m, int64_t A, int32_t *twin) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = edge2arc[i];
        const int32_t r = rev_arc[i];
        if (a < 0 || r < 0 || a >= A || r >= A) continue;
        twin[a] = r;
        twin[r] = a;
    }
}

// Edges at every vertex (either end; self-loops left out).
__global__ void k_degree(const int32_t *tail, const int32_t *col, int64_t m, int32_t *deg) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = tail[i], v = col[i];
        if (u == v) continue;
        atomicAdd(&deg[u], 1);
        atomicAdd(&deg[v], 1);
    }
}

// Sort keys of the vertices for falling degree, ties by id:
// ((kDegMax - min(deg, kDegMax)) << b) | v.
constexpr int kDegBits = 24;
constexpr int32_t kDegMax = (1 << kDegBits) - 1;
__global__ void k_vertex_keys(const int32_t *deg, int32_t n, int b, uint64_t *keys, uint32_t *vals) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t d = deg[v] < kDegMax ? deg[v] : kDegMax;
        keys[v] = ((uint64_t)(kDegMax - d) << b) | (uint64_t)v;
        vals[v] = (uint32_t)v;
    }
}

// perm[v] = position of v in the sorted order.
__global__ void k_rank_of(const uint32_t *sorted_vals, int64_t n, int32_t *perm) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        perm[sorted_vals[i]] = (int32_t)i;
}

// Key of every arc in the caller's numbering: (owner << b) | head, through
// old_of_new (the tail of arc a is the head of its twin).
__global__ void k_caller_arc_keys(const int2 *arc, const int32_t *twin, int64_t A, const int32_t *old_of_new, int b,
                                  uint64_t *keys, uint32_t *vals) {
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < A; a += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t u = (uint64_t)old_of_new[arc[twin[a]].x], v = (uint64_t)old_of_new[arc[a].x];
        keys[a] = (u << b) | v;
        vals[a] = (uint32_t)a;
    }
}

__global__ void k_fill32(int32_t *p, int64_t count, int32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

int grid_of(int64_t work) {
    int64_t b = (work + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

// Stable LSD sort of n (key, value) pairs on their low `bits` key bits, 4 bits
// a pass, between the buffer pairs (k0, v0) and (k1, v1); the sorted pairs end
// in (*k0, *v0) (the pointers are swapped as the passes go).  hist and scan:
// kDigits * tiles and scan_tmp_count(kDigits * tiles) entries.
hipError_t radix_sort(uint64_t **k0, uint32_t **v0, uint64_t **k1, uint32_t **v1, int64_t n, int bits,
                      int64_t *hist, int64_t *scan, hipStream_t st) {
    const int64_t tiles = (n + kSortTile - 1) / kSortTile;
    if (n <= 1) return hipSuccess;
    hipError_t e = hipMemsetAsync(hist, 0, sizeof(int64_t) * kDigits * tiles, st);
    if (e != hipSuccess) return e;
    for (int shift = 0; shift < bits; shift += 4) {
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)tiles), dim3(kSortThreads), 0, st, *k0, n, shift, hist, tiles);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = scan_exclusive(hist, kDigits * tiles, scan, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)tiles), dim3(kSortThreads), 0, st, *k0, *v0, n, shift, hist,
                           tiles, *k1, *v1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        std::swap(*k0, *k1);
        std::swap(*v0, *v1);
    }
    return hipSuccess;
}

int id_bits(int64_t n) {
    int b = 1;
    while ((1ll << b) < n) ++b;
    return b;
}

}  // namespace

hipError_t build_layout_device(int32_t n, int64_t m, const int64_t *h_row_ptr, const int32_t *h_col,
                               const int32_t *h_cap, bool renumber, const BuildAlloc &mem, hipStream_t st,
                               DeviceLayout *out, std::vector<int32_t> *h_row_ptr_out,
                               std::vector<int32_t> *h_new_of_old, std::string *err) {
    std::vector<void *> tmp;
    auto talloc = [&](void **p, size_t bytes) -> hipError_t {
        hipError_t e = mem.alloc(p, bytes < 256 ? 256 : bytes);
        if (e == hipSuccess) tmp.push_back(*p);
        return e;
    };
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        for (void *p : tmp) mem.release(p);
        tmp.clear();
    };
#define BTRY(expr)                                                    \
    do {                                                              \
        hipError_t e_ = (expr);                                       \
        if (e_ != hipSuccess) {                                       \
            *err = std::string(#expr) + ": " + hipGetErrorString(e_); \
            cleanup();                                                \
            return e_;                                                \
        }                                                             \
    } while (0)
    int64_t *d_rp = nullptr, *d_flag = nullptr, *d_scan = nullptr, *d_hist = nullptr;
    int32_t *d_tail = nullptr, *d_col = nullptr, *d_ecap = nullptr, *d_info = nullptr;
    BTRY(talloc((void **)&d_rp, sizeof(int64_t) * (n + 1)));
    BTRY(talloc((void **)&d_col, sizeof(int32_t) * (m > 0 ? m : 1)));
    BTRY(talloc((void **)&d_tail, sizeof(int32_t) * (m > 0 ? m : 1)));
    BTRY(talloc((void **)&d_info, sizeof(int32_t) * 4));
    // the edge capacities stay with the handle (ecap)
    BTRY(mem.alloc_keep((void **)&d_ecap, sizeof(int32_t) * (m > 0 ? m : 1)));
    BTRY(hipMemcpyAsync(d_rp, h_row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, st));
    if (m > 0) {
        BTRY(hipMemcpyAsync(d_col, h_col, sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
        BTRY(hipMemcpyAsync(d_ecap, h_cap, sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
    }
    // 1-2: tails, non-loop positions, half-edges
    const int64_t mm = m > 0 ? m : 1;
    BTRY(talloc((void **)&d_flag, sizeof(int64_t) * (mm + 1)));
    BTRY(talloc((void **)&d_scan, sizeof(int64_t) * scan_tmp_count(2 * mm + 1)));
    int64_t nonloop = 0;
    if (m > 0) {
        hipLaunchKernelGGL(k_tails, dim3(grid_of(m)), dim3(256), 0, st, d_rp, n, m, d_tail);
        hipLaunchKernelGGL(k_nonloop, dim3(grid_of(m)), dim3(256), 0, st, d_tail, d_col, m, d_flag);
        BTRY(hipGetLastError());
        int64_t last_flag = 0;
        BTRY(hipMemcpyAsync(&last_flag, d_flag + m - 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        BTRY(hipStreamSynchronize(st));
        BTRY(scan_exclusive(d_flag, m, d_scan, st));
        int64_t last_pos = 0;
        BTRY(hipMemcpyAsync(&last_pos, d_flag + m - 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        BTRY(hipStreamSynchronize(st));
        nonloop = last_pos + last_flag;
    }
    const int64_t nh = 2 * nonloop;
    if (nh / 2 > INT32_MAX / 2) {
        *err = "too many arcs for int32 arc indices";
        cleanup();
        return hipErrorInvalidValue;
    }
    const int b = id_bits(n);  // bits of a vertex id
    uint64_t *d_k0 = nullptr, *d_k1 = nullptr;
    uint32_t *d_v0 = nullptr, *d_v1 = nullptr;
    const int64_t nhh = std::max<int64_t>(nh > 0 ? nh : 1, renumber ? n : 1);
    BTRY(talloc((void **)&d_k0, sizeof(uint64_t) * nhh));
    BTRY(talloc((void **)&d_k1, sizeof(uint64_t) * nhh));
    BTRY(talloc((void **)&d_v0, sizeof(uint32_t) * nhh));
    BTRY(talloc((void **)&d_v1, sizeof(uint32_t) * nhh));
    const int64_t tiles = (nhh + kSortTile - 1) / kSortTile;
    int64_t *d_scan2 = nullptr;
    BTRY(talloc((void **)&d_hist, sizeof(int64_t) * kDigits * tiles));
    BTRY(talloc((void **)&d_scan2, sizeof(int64_t) * scan_tmp_count(kDigits * tiles)));
    // 2b: the handle's vertex order: falling degree (ties by id), so that the
    // hubs' heights, excesses and row bounds share a few cache lines and
    // every arc list starts with its hub neighbours
    int32_t *d_perm = nullptr;
    if (renumber && n > 0) {
        BTRY(talloc((void **)&d_perm, sizeof(int32_t) * n));
        BTRY(hipMemsetAsync(d_perm, 0, sizeof(int32_t) * n, st));
        if (m > 0) hipLaunchKernelGGL(k_degree, dim3(grid_of(m)), dim3(256), 0, st, d_tail, d_col, m, d_perm);
        hipLaunchKernelGGL(k_vertex_keys, dim3(grid_of(n)), dim3(256), 0, st, d_perm, n, b, d_k0, d_v0);
        BTRY(hipGetLastError());
        BTRY(radix_sort(&d_k0, &d_v0, &d_k1, &d_v1, n, b + kDegBits, d_hist, d_scan2, st));
        hipLaunchKernelGGL(k_rank_of, dim3(grid_of(n)), dim3(256), 0, st, d_v0, (int64_t)n, d_perm);
        BTRY(hipGetLastError());
        h_new_of_old->assign((size_t)n, 0);
        BTRY(hipMemcpyAsync(h_new_of_old->data(), d_perm, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    } else {
        h_new_of_old->clear();
    }
    if (m > 0) {
        hipLaunchKernelGGL(k_half_edges, dim3(grid_of(m)), dim3(256), 0, st, d_tail, d_col, m, d_flag, b, d_perm,
                           d_k0, d_v0);
        BTRY(hipGetLastError());
    }
    // 3: sort by (owner, neighbour)
    BTRY(radix_sort(&d_k0, &d_v0, &d_k1, &d_v1, nh, 2 * b, d_hist, d_scan2, st));
    // 4: arcs
    int64_t A = 0;
    int64_t *d_idx = nullptr;
    BTRY(talloc((void **)&d_idx, sizeof(int64_t) * (nhh + 1)));
    if (nh > 0) {
        hipLaunchKernelGGL(k_run_starts, dim3(grid_of(nh)), dim3(256), 0, st, d_k0, nh, d_idx);
        BTRY(hipGetLastError());
        int64_t last_flag = 0, last_idx = 0;
        BTRY(hipMemcpyAsync(&last_flag, d_idx + nh - 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        BTRY(hipStreamSynchronize(st));
        BTRY(scan_exclusive(d_idx, nh, d_scan, st));
        BTRY(hipMemcpyAsync(&last_idx, d_idx + nh - 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        BTRY(hipStreamSynchronize(st));
        A = last_idx + last_flag;
    }
    if (A > INT32_MAX) {
        *err = "too many arcs for int32 arc indices";
        cleanup();
        return hipErrorInvalidValue;
    }
    const int64_t AA = A > 0 ? A : 1;
    int32_t *d_colA = nullptr, *d_owner = nullptr, *d_rev = nullptr;
    int64_t *d_start = nullptr, *d_capsum = nullptr;
    BTRY(talloc((void **)&d_colA, sizeof(int32_t) * AA));
    BTRY(talloc((void **)&d_owner, sizeof(int32_t) * AA));
    BTRY(talloc((void **)&d_start, sizeof(int64_t) * AA));
    BTRY(talloc((void **)&d_capsum, sizeof(int64_t) * AA));
    BTRY(talloc((void **)&d_rev, sizeof(int32_t) * mm));
    // the handle's arrays
    BTRY(mem.alloc_keep((void **)&out->row_ptr, sizeof(int32_t) * (n + 1)));
    BTRY(mem.alloc_keep((void **)&out->arc, sizeof(int2) * AA));
    BTRY(mem.alloc_keep((void **)&out->twin, sizeof(int32_t) * AA));
    BTRY(mem.alloc_keep((void **)&out->cap, sizeof(int32_t) * AA));
    BTRY(mem.alloc_keep((void **)&out->edge2arc, sizeof(int32_t) * mm));
    out->ecap = d_ecap;
    BTRY(hipMemsetAsync(d_capsum, 0, sizeof(int64_t) * AA, st));
    BTRY(hipMemsetAsync(d_info, 0, sizeof(int32_t) * 4, st));
    hipLaunchKernelGGL(k_fill32, dim3(grid_of(mm)), dim3(256), 0, st, out->edge2arc, mm, -1);
    hipLaunchKernelGGL(k_fill32, dim3(grid_of(mm)), dim3(256), 0, st, d_rev, mm, -1);
    if (nh > 0)
        hipLaunchKernelGGL(k_arcs, dim3(grid_of(nh)), dim3(256), 0, st, d_k0, d_v0, d_idx, nh, A, b, d_ecap, d_colA,
                           d_owner, d_start, d_capsum, out->edge2arc, d_rev);
    if (A > 0)
        hipLaunchKernelGGL(k_arc_records, dim3(grid_of(A)), dim3(256), 0, st, d_colA, d_capsum, d_start, A, nh,
                           out->arc, out->cap, d_info, d_info + 1);
    hipLaunchKernelGGL(k_row_ptr, dim3(grid_of((int64_t)n + 1)), dim3(256), 0, st, d_owner, A, n, out->row_ptr);
    if (m > 0) hipLaunchKernelGGL(k_twins, dim3(grid_of(m)), dim3(256), 0, st, out->edge2arc, d_rev, m, A, out->twin);
    BTRY(hipGetLastError());
    int32_t info[4] = {0, 0, 0, 0};
    BTRY(hipMemcpyAsync(info, d_info, sizeof(info), hipMemcpyDeviceToHost, st));
    h_row_ptr_out->assign((size_t)n + 1, 0);
    BTRY(hipMemcpyAsync(h_row_ptr_out->data(), out->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, st));
    BTRY(hipStreamSynchronize(st));
    cleanup();
#undef BTRY
    if (info[1]) {
        *err = "summed capacity of one arc exceeds int32";
        return hipErrorInvalidValue;
    }
    out->A = (int32_t)A;
    out->max_pair_mult = info[0] > 0 ? info[0] : 1;
    return hipSuccess;
}

hipError_t caller_arc_order(int32_t n, int64_t A, const int2 *arc, const int32_t *twin,
                            const std::vector<int32_t> &old_of_new, const BuildAlloc &mem, hipStream_t st,
                            std::vector<int32_t> *h_caller_of_arc) {
    std::vector<void *> tmp;
    auto talloc = [&](void **p, size_t bytes) -> hipError_t {
        hipError_t e = mem.alloc(p, bytes < 256 ? 256 : bytes);
        if (e == hipSuccess) tmp.push_back(*p);
        return e;
    };
    hipError_t e = hipSuccess;
    auto done = [&](hipError_t r) {
        (void)hipStreamSynchronize(st);
        for (void *p : tmp) mem.release(p);
        return r;
    };
    const int64_t AA = A > 0 ? A : 1;
    const int64_t tiles = (AA + kSortTile - 1) / kSortTile;
    uint64_t *k0 = nullptr, *k1 = nullptr;
    uint32_t *v0 = nullptr, *v1 = nullptr;
    int32_t *d_old = nullptr, *d_rank = nullptr;
    int64_t *hist = nullptr, *scan = nullptr;
    if ((e = talloc((void **)&k0, sizeof(uint64_t) * AA)) != hipSuccess ||
        (e = talloc((void **)&k1, sizeof(uint64_t) * AA)) != hipSuccess ||
        (e = talloc((void **)&v0, sizeof(uint32_t) * AA)) != hipSuccess ||
        (e = talloc((void **)&v1, sizeof(uint32_t) * AA)) != hipSuccess ||
        (e = talloc((void **)&d_old, sizeof(int32_t) * (n > 0 ? n : 1))) != hipSuccess ||
        (e = talloc((void **)&d_rank, sizeof(int32_t) * AA)) != hipSuccess ||
        (e = talloc((void **)&hist, sizeof(int64_t) * kDigits * tiles)) != hipSuccess ||
        (e = talloc((void **)&scan, sizeof(int64_t) * scan_tmp_count(kDigits * tiles))) != hipSuccess)
        return done(e);
    if (n > 0 && (e = hipMemcpyAsync(d_old, old_of_new.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st)) !=
                     hipSuccess)
        return done(e);
    const int b = id_bits(n);
    if (A > 0) {
        hipLaunchKernelGGL(k_caller_arc_keys, dim3(grid_of(A)), dim3(256), 0, st, arc, twin, A, d_old, b, k0, v0);
        if ((e = hipGetLastError()) != hipSuccess) return done(e);
        if ((e = radix_sort(&k0, &v0, &k1, &v1, A, 2 * b, hist, scan, st)) != hipSuccess) return done(e);
        hipLaunchKernelGGL(k_rank_of, dim3(grid_of(A)), dim3(256), 0, st, v0, A, d_rank);
        if ((e = hipGetLastError()) != hipSuccess) return done(e);
    }
    h_caller_of_arc->assign((size_t)A, 0);
    if (A > 0 && (e = hipMemcpyAsync(h_caller_of_arc->data(), d_rank, sizeof(int32_t) * A, hipMemcpyDeviceToHost,
                                     st)) != hipSuccess)
        return done(e);
    return done(hipSuccess);
}

}  // namespace mf
