"""Small graph builders and fixture readers shared by the tests."""
from __future__ import annotations

import os

import numpy as np

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def from_edges(n, edges, s, t):
    """edges: iterable of (u, v, c)."""
    edges = list(edges)
    if edges:
        u, v, c = (np.array(x, dtype=np.int64) for x in zip(*edges))
    else:
        u = v = c = np.zeros(0, dtype=np.int64)
    return W.edges_to_csr(n, u, v, c, s, t)


def from_edges_keep_order(n, edges, s, t):
    """CSR whose edge ids follow the given order (edges must be grouped by tail
    in increasing tail order)."""
    edges = list(edges)
    tails = np.array([e[0] for e in edges], dtype=np.int64)
    assert np.all(np.diff(tails) >= 0), "edges must be sorted by tail"
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(tails, minlength=n), out=row_ptr[1:])
    col = np.array([e[1] for e in edges], dtype=np.int32)
    cap = np.array([e[2] for e in edges], dtype=np.int32)
    return W.Graph(n, row_ptr, col, cap, s, t)


def read_golden(name):
    """Returns (graph, [(batch or None, value), ...])."""
    lines = []
    with open(os.path.join(GOLDEN, name)) as f:
        for ln in f:
            ln = ln.split("#", 1)[0].strip()
            if ln:
                lines.append(ln)
    n, s, t = (int(x) for x in lines[0].split())
    edges, steps, pending = [], [], None
    for ln in lines[1:]:
        tok = ln.split()
        if tok[0] == "value":
            steps.append((pending, int(tok[1])))
            pending = None
        elif tok[0] == "batch":
            pairs = [p.split(":") for p in tok[1:]]
            pending = (np.array([int(a) for a, _ in pairs], dtype=np.int64),
                       np.array([int(b) for _, b in pairs], dtype=np.int32))
        else:
            edges.append(tuple(int(x) for x in tok))
    return from_edges_keep_order(n, edges, s, t), steps


def tiny_random(seed, n_lo=2, n_hi=10, m_hi=30, cap_hi=9):
    """Random tiny graph with zero capacities, self-loops, duplicates and
    antiparallel edges, random s != t."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(n_lo, n_hi + 1))
    m = int(rng.integers(0, m_hi + 1))
    s, t = (int(x) for x in rng.choice(n, 2, replace=False))
    g = W.random_graph(n, m, 0, cap_hi, seed=int(rng.integers(1 << 30)), s=s, t=t,
                       allow_self_loops=True)
    return g
