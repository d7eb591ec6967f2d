"""Seeded synthetic inputs for the dynamic max-flow workloads.

This module is shared test/benchmark infrastructure. Both the CPU oracle side and
the GPU side draw their inputs from it, so it deliberately holds none of the
max-flow arithmetic: it only draws directed graphs (as CSR arrays), integer
capacities and update batches from seeded numpy generators.

Conventions
-----------
* A graph is returned as ``Graph(n, row_ptr, col, cap, s, t)``: ``row_ptr`` is
  int64[n+1], ``col`` int32[m] and ``cap`` int32[m]. Edge ``i`` is the CSR
  position ``i``; its tail is the row that holds it. Within a row, edges are
  sorted by head (stable, so duplicates keep their draw order; R-MAT rows are
  sorted by head, then capacity).
* A batch is ``(edge_ids int64[k], new_caps int32[k])`` of *distinct* edge ids
  with absolute new capacities (a batch is a set of edges with new capacities,
  Sec. 4 of the paper). The first ceil(k/2) entries raise the capacity, the
  rest lower it (new value uniform in [0, c]), as in the mixed experiments
  (Sec. 6.4).
* Seeds: workload ``i`` uses ``SEED_BASE + i``; batch ``j`` of a chain uses the
  seed sequence ``[seed, j]``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 251105895


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[m]
    cap: np.ndarray      # int32[m]
    s: int
    t: int

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def tails(self) -> np.ndarray:
        """int32[m]: tail vertex of every edge (expanded from row_ptr)."""
        deg = np.diff(self.row_ptr)
        return np.repeat(np.arange(self.n, dtype=np.int32), deg)


def rng_for(seed, *stream) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), *[int(x) for x in stream]]))


def edges_to_csr(n: int, src: np.ndarray, dst: np.ndarray, cap: np.ndarray,
                 s: int, t: int) -> Graph:
    """Sort an edge list by (tail, head), stable, into CSR arrays."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    key = src * np.int64(n) + dst
    order = np.argsort(key, kind="stable")
    src_s = src[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src_s, minlength=n), out=row_ptr[1:])
    return Graph(n, row_ptr, dst[order].astype(np.int32),
                 np.asarray(cap)[order].astype(np.int32), int(s), int(t))


# --------------------------------------------------------------------------
# Uniform random directed graph (small parity workload)
# --------------------------------------------------------------------------

def random_graph(n: int, m: int, cap_lo: int, cap_hi: int, seed, s: int = 0,
                 t: int | None = None, allow_self_loops: bool = False) -> Graph:
    """Uniform endpoints; self-loops redrawn unless allowed; duplicates and
    antiparallel pairs kept. Capacities uniform in [cap_lo, cap_hi]."""
    rng = rng_for(seed, 0)
    src = rng.integers(0, n, m, dtype=np.int64)
    dst = rng.integers(0, n, m, dtype=np.int64)
    if not allow_self_loops and n > 1:
        bad = src == dst
        while bad.any():
            dst[bad] = rng.integers(0, n, int(bad.sum()), dtype=np.int64)
            bad = src == dst
    cap = rng.integers(cap_lo, cap_hi + 1, m, dtype=np.int64)
    return edges_to_csr(n, src, dst, cap, s, n - 1 if t is None else t)


def c1_random_1k(seed=SEED_BASE + 0) -> Graph:
    """1,000 vertices, 8,000 edges, capacities U[1,100], s=0, t=999."""
    return random_graph(1000, 8000, 1, 100, seed, s=0, t=999)


# --------------------------------------------------------------------------
# Image-segmentation grid
# --------------------------------------------------------------------------

def _blurred_intensity(side: int, blur_sigma: float, rng: np.random.Generator) -> np.ndarray:
    from scipy.ndimage import gaussian_filter
    noise = rng.standard_normal((side, side))
    img = gaussian_filter(noise, sigma=blur_sigma, mode="reflect", truncate=3.0)
    lo, hi = float(img.min()), float(img.max())
    return (img - lo) / (hi - lo) if hi > lo else np.zeros_like(img)


def seg_grid(side: int, seed, sigma: float = 0.1, blur_sigma: float = 2.0,
             tlink_hi: int = 200, nlink_scale: int = 100, tlink_lo: int = 0) -> Graph:
    """4-connected side x side grid, pixels row-major 0..side^2-1, s = side^2,
    t = side^2+1. Both directions of each neighbour pair carry
    1 + round(scale * exp(-(I_p - I_q)^2 / (2 sigma^2))); every pixel has
    s->p and p->t with independent U[tlink_lo, tlink_hi] capacities."""
    rng = rng_for(seed, 0)
    img = _blurred_intensity(side, blur_sigma, rng)
    npx = side * side
    s, t = npx, npx + 1
    idx = np.arange(npx, dtype=np.int64).reshape(side, side)
    # horizontal and vertical neighbour pairs
    pa = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    pb = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    ia = img.ravel()[pa]
    ib = img.ravel()[pb]
    w = 1 + np.floor(nlink_scale * np.exp(-((ia - ib) ** 2) / (2.0 * sigma * sigma)) + 0.5)
    w = w.astype(np.int64)
    src = np.concatenate([pa, pb, np.full(npx, s, np.int64), np.arange(npx, dtype=np.int64)])
    dst = np.concatenate([pb, pa, np.arange(npx, dtype=np.int64), np.full(npx, t, np.int64)])
    tl = rng.integers(tlink_lo, tlink_hi + 1, 2 * npx, dtype=np.int64)
    cap = np.concatenate([w, w, tl])
    return edges_to_csr(npx + 2, src, dst, cap, s, t)


def c2_grid_512(seed=SEED_BASE + 1) -> Graph:
    return seg_grid(512, seed)


# --------------------------------------------------------------------------
# R-MAT power-law graph
# --------------------------------------------------------------------------

def _rmat_chunk(scale: int, cnt: int, rng: np.random.Generator, t1: int, t2: int, t3: int):
    """cnt R-MAT edges: at every level one 16-bit draw picks the quadrant
    (below t1: top-left, t1..t2: top-right, t2..t3: bottom-left, else
    bottom-right); four levels come from one 64-bit draw.  Self-loops are
    redrawn from the same generator."""
    def draw(k):
        u = np.zeros(k, dtype=np.uint32)
        v = np.zeros(k, dtype=np.uint32)
        for base in range(0, scale, 4):
            raw = rng.bit_generator.random_raw(k)
            for j in range(min(4, scale - base)):
                r = ((raw >> np.uint64(16 * j)) & np.uint64(0xFFFF)).astype(np.uint16)
                ge1, ge2, ge3 = r >= t1, r >= t2, r >= t3
                u |= ge2.astype(np.uint32) << np.uint32(base + j)
                v |= (ge1 ^ ge2 ^ ge3).astype(np.uint32) << np.uint32(base + j)
        return u, v

    u, v = draw(cnt)
    bad = np.flatnonzero(u == v)
    while bad.size:
        uu, vv = draw(bad.size)
        u[bad] = uu
        v[bad] = vv
        bad = bad[uu == vv]
    return u, v


def rmat(scale: int, edge_factor: int, seed, a=0.57, b=0.19, c=0.19,
         cap_lo: int = 1, cap_hi: int = 1000, permute: bool = True,
         chunk: int = 1 << 21, workers: int = 8) -> Graph:
    """R-MAT(a,b,c,d) with 2^scale vertices and edge_factor*2^scale edges.
    The quadrant probabilities are taken in units of 2^-16.  Self-loops are
    redrawn, duplicates kept as separate edges, vertex ids randomly permuted.
    s / t = highest / second-highest total degree (ties to the lower id).
    Capacities U[cap_lo, cap_hi].  Edges are drawn in chunks, each from its
    own seeded stream (so the graph does not depend on `workers`); rows are
    sorted by head, then capacity."""
    import concurrent.futures as cf
    n = 1 << scale
    m = edge_factor * n
    t1 = int(round(a * 65536))
    t2 = int(round((a + b) * 65536))
    t3 = int(round((a + b + c) * 65536))
    bounds = [(lo, min(m, lo + chunk)) for lo in range(0, m, chunk)]
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)

    def fill(i):
        lo, hi = bounds[i]
        u, v = _rmat_chunk(scale, hi - lo, rng_for(seed, 0, i), t1, t2, t3)
        src[lo:hi] = u
        dst[lo:hi] = v

    with cf.ThreadPoolExecutor(max(1, workers)) as ex:
        list(ex.map(fill, range(len(bounds))))
    if permute:
        perm = rng_for(seed, 1).permutation(n).astype(np.uint32)
        src = perm[src]
        dst = perm[dst]
    cap = rng_for(seed, 2).integers(cap_lo, cap_hi + 1, m, dtype=np.int64)
    deg = np.bincount(src, minlength=n) + np.bincount(dst, minlength=n)
    order = np.lexsort((np.arange(n), -deg))  # highest degree first, ties -> lower id
    s, t = int(order[0]), int(order[1])
    return _csr_by_packed_key(n, src, dst, cap, s, t, workers)


def _csr_by_packed_key(n: int, src, dst, cap, s: int, t: int, workers: int = 8) -> Graph:
    """CSR with rows sorted by head, then capacity, through one sort of
    packed (tail, head, capacity - min) keys; falls back to edges_to_csr when
    they do not fit 64 bits."""
    import concurrent.futures as cf
    cap = np.asarray(cap, dtype=np.int64)
    m = int(src.shape[0])
    c0 = int(cap.min()) if m else 0
    vb = max(1, (n - 1).bit_length())
    cb = max(1, (int(cap.max()) - c0).bit_length()) if m else 1
    if 2 * vb + cb > 63:
        return edges_to_csr(n, src, dst, cap, s, t)
    key = (src.astype(np.uint64) << np.uint64(vb + cb)) | (dst.astype(np.uint64) << np.uint64(cb)) | \
        (cap - c0).astype(np.uint64)
    # sort in slices of tail ranges, side by side
    nb = 16
    shift = max(0, vb - 4)
    bucket = (np.asarray(src) >> shift).astype(np.uint8)
    key = key[np.argsort(bucket, kind="stable")]
    edges = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(np.bincount(bucket, minlength=nb), out=edges[1:])

    def sort_slice(i):
        key[edges[i]:edges[i + 1]].sort()

    with cf.ThreadPoolExecutor(max(1, workers)) as ex:
        list(ex.map(sort_slice, range(nb)))
    tails = (key >> np.uint64(vb + cb)).astype(np.int64)
    heads = ((key >> np.uint64(cb)) & np.uint64((1 << vb) - 1)).astype(np.int32)
    caps = ((key & np.uint64((1 << cb) - 1)).astype(np.int64) + c0).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(tails, minlength=n), out=row_ptr[1:])
    return Graph(n, row_ptr, heads, caps, int(s), int(t))


def c3_rmat20(seed=SEED_BASE + 2) -> Graph:
    return rmat(20, 16, seed)


# --------------------------------------------------------------------------
# Update batches
# --------------------------------------------------------------------------

def batch_size(m: int, fraction: float) -> int:
    return max(1, int(round(m * fraction)))


def st_edges(g: Graph) -> np.ndarray:
    """Ids of the edges out of the source or into the sink."""
    tails = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    return np.flatnonzero((tails == g.s) | (g.col == g.t)).astype(np.int64)


def pick_edges(m: int, k: int, rng: np.random.Generator, st_ids: np.ndarray | None = None,
               p_st: float = 0.0) -> np.ndarray:
    """k distinct edge ids.  With p_st > 0 each of the k picks comes from the
    source/sink edges st_ids with probability p_st (a binomial count, capped by
    how many there are) and from the other edges otherwise: the paper's
    experiments draw edges out of s and into t more often than the rest."""
    k = min(int(k), m)
    if st_ids is None or p_st <= 0.0 or st_ids.shape[0] == 0:
        return rng.choice(m, size=k, replace=False).astype(np.int64)
    other = np.setdiff1d(np.arange(m, dtype=np.int64), st_ids, assume_unique=True)
    k_st = min(int(rng.binomial(k, p_st)), int(st_ids.shape[0]))
    k_st = max(k_st, k - int(other.shape[0]))
    a = rng.choice(st_ids, size=k_st, replace=False)
    b = rng.choice(other, size=k - k_st, replace=False)
    return rng.permutation(np.concatenate([a, b])).astype(np.int64)


def mixed_batch(cur_cap: np.ndarray, k: int, inc_hi: int, rng: np.random.Generator,
                inc_fraction: float = 0.5, ids: np.ndarray | None = None,
                st_ids: np.ndarray | None = None, p_st: float = 0.0):
    """k distinct edges (pick_edges); the first ceil(k*inc_fraction) get
    cap + U[1, inc_hi], the rest a new capacity U[0, cap]."""
    m = int(cur_cap.shape[0])
    k = min(int(k), m)
    if ids is None:
        ids = pick_edges(m, k, rng, st_ids, p_st)
    else:
        ids = np.asarray(ids, dtype=np.int64)
    n_inc = int(math.ceil(k * inc_fraction))
    cur = cur_cap[ids].astype(np.int64)
    new = np.empty(k, dtype=np.int64)
    new[:n_inc] = cur[:n_inc] + rng.integers(1, inc_hi + 1, n_inc, dtype=np.int64)
    new[n_inc:] = rng.integers(0, cur[n_inc:] + 1, dtype=np.int64)
    return ids, new.astype(np.int32)


def batch_chain(g: Graph, fraction: float, count: int, inc_hi: int, seed,
                inc_fraction: float = 0.5, k: int | None = None, p_st: float = 0.0):
    """Yield `count` successive batches (ids, new_caps); capacities evolve as
    each batch is applied, so batch j is drawn against the capacities that
    batches 0..j-1 left behind.  inc_fraction 1 / 0 / 0.5 gives the paper's
    incremental, decremental and mixed update families; p_st biases the picks
    toward edges out of s and into t."""
    cur = g.cap.copy()
    kk = batch_size(g.m, fraction) if k is None else int(k)
    st = st_edges(g) if p_st > 0.0 else None
    for j in range(count):
        ids, new = mixed_batch(cur, kk, inc_hi, rng_for(seed, 1, j), inc_fraction, st_ids=st, p_st=p_st)
        cur[ids] = new
        yield ids, new


def apply_batch(cap: np.ndarray, ids: np.ndarray, new: np.ndarray) -> np.ndarray:
    out = cap.copy()
    out[ids] = new
    return out


# --------------------------------------------------------------------------
# Many independent instances (batched solve)
# --------------------------------------------------------------------------

def grid_instance(side: int, seed, cap_lo: int = 1, cap_hi: int = 1000) -> Graph:
    """side x side 4-connected grid, both directions of every neighbour pair,
    plus s->p and p->t for every pixel; all capacities U[cap_lo, cap_hi].
    Pixels row-major, s = side^2, t = side^2 + 1."""
    rng = rng_for(seed, 0)
    npx = side * side
    s, t = npx, npx + 1
    idx = np.arange(npx, dtype=np.int64).reshape(side, side)
    pa = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    pb = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    src = np.concatenate([pa, pb, np.full(npx, s, np.int64), np.arange(npx, dtype=np.int64)])
    dst = np.concatenate([pb, pa, np.arange(npx, dtype=np.int64), np.full(npx, t, np.int64)])
    cap = rng.integers(cap_lo, cap_hi + 1, src.shape[0], dtype=np.int64)
    return edges_to_csr(npx + 2, src, dst, cap, s, t)


def c4_instances(count: int = 256, seed=SEED_BASE + 3):
    """Uneven batch: even i -> grid of side round(32 * 8^u), u ~ U[0,1]
    (32..256); odd i -> random graph with round(1000 * 50^u) vertices
    (1k..50k), 8 edges per vertex, s = 0, t = n-1; capacities U[1,1000]."""
    rng = rng_for(seed, 0)
    out = []
    for i in range(count):
        u = float(rng.random())
        if i % 2 == 0:
            out.append(grid_instance(int(round(32 * 8 ** u)), int(seed) * 1000 + i))
        else:
            n = int(round(1000 * 50 ** u))
            out.append(random_graph(n, 8 * n, 1, 1000, int(seed) * 1000 + i, s=0, t=n - 1))
    return out


def c5_rmat22(seed=SEED_BASE + 4) -> Graph:
    """R-MAT scale 22 (4,194,304 vertices, 67,108,864 edges), generator as C3."""
    return rmat(22, 16, seed)


def request_stream(g: Graph, count: int, seed, k_lo: int = 10, k_hi: int = 100_000, inc_hi: int = 1000):
    """Yield `count` update requests (ids, new_caps) for a served graph: request
    j has k = round(k_lo * (k_hi/k_lo)^u) distinct edges, u ~ U[0,1] (log-uniform),
    half raised by U[1, inc_hi] and half lowered to U[0, c]; capacities evolve
    as the requests are applied in order."""
    cur = g.cap.copy()
    for j in range(count):
        rng = rng_for(seed, 2, j)
        u = float(rng.random())
        k = min(g.m, max(1, int(round(k_lo * (k_hi / k_lo) ** u))))
        ids, new = mixed_batch(cur, k, inc_hi, rng)
        cur[ids] = new
        yield ids, new

