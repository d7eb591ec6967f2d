"""Benchmark: dynamic max-flow update latency vs static recompute on one MI355X.

Workload (default): an R-MAT graph of scale 22 (4,194,304 vertices,
67,108,864 edges, capacities U[1,1000]) resident on the device, taking update
requests of 10..100,000 edges (log-uniform; half raised by U[1,1000], half
lowered to U[0,c]).

One step = one request: the dynamic repair on a resident handle, end to end
from host arrays (mf_apply_updates: upload of the batch, repair, solve, value
back on the host), and the static recompute of the same updated graph on a
second handle (mf_set_capacities + mf_solve).  Both values must be equal after
every step; one step is also checked against the CPU oracle, whose
from-scratch recompute is the CPU baseline.  The R-MAT scale-20 graph with 1%
mixed batches is measured the same way and reported beside it ("secondary").

Prints one JSON line.  `value` is residual arcs per second of dynamic update
latency: K * A / (sum of the K dynamic latencies)."""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

# Algorithmic bytes per counted event ("Roofline model").
BYTES = {
    "height_reset_vertex": 12,   # per vertex per global relabel: read e (8), write h (4)
    "bfs_vertices": 16,          # per vertex reached: row_ptr pair (8), frontier item (8)
    "bfs_arcs": 16,              # per arc examined: head (4), twin (4), twin residual (4), head height (4)
    "pr_vertex_cycles": 16,      # per push/relabel cycle: e (8), h (4), row_ptr (4)
    "pr_arcs": 12,               # per arc scanned: {head, residual} (8), head height (4)
    "pushes": 48,                # twin (4) + residual RMW x2 (16) + excess RMW x2 (32) - rounded
    "relabels": 4,
    "rie_arcs": 12,
    "rie_saturations": 48,
    "updates": 40,
    "clamps": 40,
    "source_pushes": 48,
}

CONFIGS = {
    "rmat22": dict(desc="R-MAT scale 22 (4,194,304 V / 67,108,864 E), requests of 10..100k edges "
                        "(log-uniform), mixed", base="R-MAT scale 22 (avg degree 16)", frac=0.0, inc_hi=1000,
                   requests=True),
    "grid512": dict(desc="segmentation grid 512x512, 1% mixed batches", base="segmentation grid 512x512",
                    frac=0.01, inc_hi=100),
    "rmat20": dict(desc="R-MAT scale 20 (avg degree 16), 1% mixed batches", base="R-MAT scale 20 (avg degree 16)",
                   frac=0.01, inc_hi=1000),
    "random1k": dict(desc="random graph 1,000 V / 8,000 E, 100-edge mixed batches",
                     base="random graph 1,000 V / 8,000 E", frac=0.0125, inc_hi=100),
    "c4": dict(desc="256 uneven instances (grids 32^2..256^2, random graphs 1k..50k V at degree 8), "
                    "batched static solve"),
    "learned20": dict(desc="learned vs fixed phase schedule on R-MAT scale 20"),
    "c5": dict(desc="R-MAT scale 22 (4,194,304 V / 67,108,864 E) served: requests of 10..100k edges "
                    "(log-uniform), Poisson arrivals"),
}


def make_graph(name):
    import workloads as W
    if name == "rmat22":
        return W.c5_rmat22(), W.SEED_BASE + 4
    if name == "grid512":
        return W.c2_grid_512(), W.SEED_BASE + 1
    if name == "rmat20":
        return W.c3_rmat20(), W.SEED_BASE + 2
    if name == "random1k":
        return W.c1_random_1k(), W.SEED_BASE + 0
    raise SystemExit(f"unknown config {name}")


def algorithmic_bytes(stats, n):
    b = stats["global_relabels"] * n * BYTES["height_reset_vertex"]
    for k, per in BYTES.items():
        if k in stats:
            b += stats[k] * per
    return b


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("mf_kernels.hip", "mf_internal.h"):
        with open(os.path.join(ROOT, "paper_2511_05895_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(config, launches_key):
    """HBM traffic of the dominant kernel from the committed rocprofv3 PMC
    summary, or None when it is missing or the kernel changed since."""
    path = os.path.join(ROOT, "profiles", f"k_loop_{config}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_digest") != kernel_source_digest():
        return None
    return rec.get(launches_key)


def cpu_baseline(g, cap0, batches, A, max_seconds):
    """The oracle (O1, Dinic) recomputing from scratch on the host, on the first
    timed batches of the same chain (capacities cap0 = after the warmup
    batches) until about max_seconds of CPU work."""
    import oracle as O
    cap = cap0.copy()
    times, values = [], []
    t_start = time.perf_counter()
    for ids, new in batches:
        cap[ids] = new
        t0 = time.perf_counter()
        v, _, _ = O.dinic(g, cap)
        times.append(time.perf_counter() - t0)
        values.append(v)
        if time.perf_counter() - t_start > max_seconds:
            break
    per = float(np.mean(times))
    return {"value": A / per, "unit": "residual edges/s", "cores": 1, "kind": "oracle",
            "sample": f"Dinic (O1) from-scratch recompute after each of the first {len(times)} "
                      f"batches of the chain, mean {per:.2f} s per recompute, single thread",
            "values": values}


def run_batch(args):
    """C4: one batched solve of 256 independent instances (one workgroup per
    instance, size classes autotuned, hipGraph replay) per step, against 256
    sequential solves on single handles and against the same handles driven
    from 16 host threads (one stream per handle)."""
    import concurrent.futures as cf
    import torch
    import workloads as W
    from paper_2511_05895_amd import mf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.perf_counter()
    gs = W.c4_instances()
    print(f"[bench] c4: {len(gs)} instances generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    B = mf.Batch(gs)
    arcs = B.num_arcs()
    A = int(arcs.sum())
    chosen = B.autotune(repeats=3)
    print(f"[bench] autotuned: block {chosen['block'][:3]}, cycles {chosen['kernel_cycles'][:3]}",
          file=sys.stderr, flush=True)
    ref = B.solve()
    K, Wm = args.steps, args.warmup
    for _ in range(Wm):
        B.solve()
    torch.cuda.synchronize()
    wall, kern = [], []
    t_begin = time.perf_counter()
    for j in range(K):
        a = time.perf_counter()
        v = B.solve()
        wall.append((time.perf_counter() - a) * 1e3)
        kern.append(B.last_ms())
        if not np.array_equal(v, ref):
            raise SystemExit(f"FAIL: batched values changed at step {j}")
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    print(f"[bench] batched: p50 {np.percentile(wall, 50):.2f} ms", file=sys.stderr, flush=True)
    # per-instance counters of the last solve -> algorithmic bytes of one launch
    alg = 0
    for i, g in enumerate(gs):
        st = B.stats(i)
        alg += algorithmic_bytes(st, g.n) + int(arcs[i]) * 12  # + state initialisation (cap read, c_f write)
    # comparators on single handles
    hs = [mf.MaxFlow(g) for g in gs]
    for F in hs:
        F.solve()
    torch.cuda.synchronize()
    seq = []
    for _ in range(max(1, K // 4)):
        a = time.perf_counter()
        vs = [F.solve() for F in hs]
        seq.append((time.perf_counter() - a) * 1e3)
        if vs != list(ref):
            raise SystemExit("FAIL: sequential single-handle values differ from the batch")
    print(f"[bench] sequential: {np.median(seq):.1f} ms", file=sys.stderr, flush=True)
    par = []
    with cf.ThreadPoolExecutor(16) as ex:
        for _ in range(max(1, K // 4)):
            a = time.perf_counter()
            vs = list(ex.map(lambda F: F.solve(), hs))
            par.append((time.perf_counter() - a) * 1e3)
            if vs != list(ref):
                raise SystemExit("FAIL: stream-per-instance values differ from the batch")
    print(f"[bench] stream per instance: {np.median(par):.1f} ms", file=sys.stderr, flush=True)
    for F in hs:
        F.close()
    B.close()
    wall = np.array(wall)
    kern = np.array(kern)
    achieved = alg / (kern.mean() * 1e-3) / 1e9
    out = {
        "metric": "batched static solve: aggregate residual edges/s over 256 uneven instances, exact flow",
        "value": A / (wall.mean() * 1e-3),
        "unit": "residual edges/s (batched solve)",
        "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": (t_end - t_begin) * 1e3 / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 capacities / int64 excess", "data": "synthetic (seeded generator)",
        "config": {"workload": CONFIGS["c4"]["desc"], "instances": len(gs),
                   "sum_n": int(sum(g.n for g in gs)), "sum_m": int(sum(g.m for g in gs)), "sum_arcs": A,
                   "autotuned": {k: chosen[k] for k in ("n_classes", "class_max_arcs", "block", "kernel_cycles")}},
        "batched_ms": {"p50": float(np.percentile(wall, 50)), "p99": float(np.percentile(wall, 99)),
                       "kernel_mean": float(kern.mean())},
        "sequential_ms": float(np.median(seq)),
        "stream_per_instance_ms": float(np.median(par)),
        "speedup_vs_sequential": float(np.median(seq) / np.percentile(wall, 50)),
        "speedup_vs_stream_per_instance": float(np.median(par) / np.percentile(wall, 50)),
        "exact": "batched values == single-handle values (sequential and concurrent) on every step",
        "roofline": {"kernel": "k_batch (one workgroup per instance)", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "alg_bytes_per_launch": alg,
                     "avg_launch_ms": float(kern.mean())},
    }
    if not args.no_cpu_baseline:
        import oracle as O
        times, a_s = [], 0
        t_start = time.perf_counter()
        for i in range(0, len(gs), 8):
            a = time.perf_counter()
            v, _, _ = O.dinic(gs[i], gs[i].cap)
            times.append(time.perf_counter() - a)
            a_s += int(arcs[i])
            if v != ref[i]:
                raise SystemExit(f"FAIL: oracle value {v} != batched value {ref[i]} for instance {i}")
            if time.perf_counter() - t_start > args.cpu_seconds:
                break
        out["cpu_baseline"] = {"value": a_s / sum(times), "unit": "residual edges/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"Dinic (O1) static solve of every 8th instance ({len(times)} "
                                         f"instances, {sum(times):.1f} s), single thread",
                               "checked_against_gpu": len(times)}
    print(json.dumps(out), flush=True)


def run_serving(args):
    """C5: one resident R-MAT scale-22 graph behind the serving runtime.
    A closed loop (submit, wait) over the first requests calibrates the mean
    service time S; then two open-loop phases submit Poisson arrivals at rate
    rho/S for rho = 0.5 and 0.8, and report arrival-to-result latency and
    update throughput.  The final value is checked against a static solve of
    the final capacities on a second handle."""
    import threading
    import torch
    import workloads as W
    from paper_2511_05895_amd import mf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.perf_counter()
    g = W.c5_rmat22()
    print(f"[bench] c5 graph generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    nc, no = args.closed_requests, args.open_requests
    reqs = list(W.request_stream(g, nc + 2 * no, W.SEED_BASE + 4))
    S = mf.Server(workers=args.workers, max_group_requests=args.group_requests, max_group_edges=args.group_edges)
    t0 = time.perf_counter()
    gid, v0 = S.add_graph(g)
    print(f"[bench] admitted and solved in {time.perf_counter() - t0:.1f} s (value {v0})",
          file=sys.stderr, flush=True)
    closed = []
    for j in range(nc):
        rid = S.submit(gid, *reqs[j])
        closed.append(S.wait(rid))
        S.release(rid)
    service = float(np.mean([r["done_ms"] - r["start_ms"] for r in closed]))
    print(f"[bench] closed loop: mean service {service:.1f} ms", file=sys.stderr, flush=True)
    phases = {}
    nxt = nc
    for rho in (0.5, 0.8):
        rate = rho / (service * 1e-3)  # arrivals per second
        rng = np.random.default_rng(int(rho * 10))
        gaps = rng.exponential(1.0 / rate, no)
        rids = []
        start = time.perf_counter()
        t_arr = start
        for j in range(no):
            t_arr += gaps[j]
            delay = t_arr - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            rids.append((S.submit(gid, *reqs[nxt + j]), int(reqs[nxt + j][0].shape[0])))
        res = [S.wait(r) for r, _ in rids]
        span = time.perf_counter() - start
        for r, _ in rids:
            S.release(r)
        nxt += no
        lat = np.array([r["done_ms"] - r["submit_ms"] for r in res])
        edges = sum(k for _, k in rids)
        phases[rho] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                       "update_edges_per_s": edges / span, "requests": no,
                       "commits": len({(r["start_ms"], r["done_ms"]) for r in res}),
                       "mean_group": float(np.mean([r["group_size"] for r in res]))}
        print(f"[bench] rho {rho}: p50 {phases[rho]['p50_ms']:.1f} ms, p99 {phases[rho]['p99_ms']:.1f} ms",
              file=sys.stderr, flush=True)
    version, value = S.graph_info(gid)
    S.close()
    # final value against a static solve of the final capacities
    cap = g.cap.copy()
    for ids, new in reqs:
        cap[ids] = new
    with mf.MaxFlow(g, cap=cap) as F:
        A = F.num_arcs
        t0 = time.perf_counter()
        static_value = F.solve()
        static_ms = (time.perf_counter() - t0) * 1e3
    if version != len(reqs) or static_value != value:
        raise SystemExit(f"FAIL: served value {value} at version {version} != static {static_value}")
    svc = np.array([r["done_ms"] - r["start_ms"] for r in closed])
    hi = phases[0.8]
    out = {
        "metric": "serving: arrival-to-result latency p50/p99 and update edges/s at load 0.8, exact flow",
        "value": hi["update_edges_per_s"],
        "unit": "update edges/s (served, load 0.8)",
        "n_gpus": 1, "steps": 2 * no, "warmup": nc,
        "ms_per_step": float(np.mean(svc)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 capacities / int64 excess", "data": "synthetic (seeded generator)",
        "config": {"workload": CONFIGS["c5"]["desc"], "n": g.n, "m": g.m, "arcs": A,
                   "workers": args.workers, "closed_requests": nc, "open_requests_per_load": no,
                   "max_group_requests": args.group_requests, "max_group_edges": args.group_edges},
        "closed_loop_service_ms": {"mean": float(svc.mean()), "p50": float(np.percentile(svc, 50)),
                                   "p99": float(np.percentile(svc, 99))},
        "load_0.5": phases[0.5], "load_0.8": hi,
        "residual_edges_per_s_closed": A / (svc.mean() * 1e-3),
        "static_solve_ms": static_ms,
        "exact": f"final served value == static solve of the final capacities ({value})",
    }
    print(json.dumps(out), flush=True)


_SCHED_FRACTIONS = (0.001, 0.01, 0.1)


def _sched_chain(g, count, seed):
    """Update chain of the schedule comparison: mixed batches of 0.1 %, 1 %
    and 10 % of the edges in turn, each drawn against the capacities the
    earlier ones left."""
    import workloads as W
    cur = g.cap.copy()
    for j in range(count):
        k = W.batch_size(g.m, _SCHED_FRACTIONS[j % 3])
        ids, new = W.mixed_batch(cur, k, 1000, W.rng_for(seed, 1, j))
        cur[ids] = new
        yield ids, new


def run_learned(args):
    """Learned phase schedule against the fixed rule on the R-MAT scale-20
    graph.  Training: every update call of chains on smaller R-MAT graphs
    (scales 17 and 18, seeds disjoint from the evaluation graph's) is replayed
    from one exported state under each of the 8 actions; sample = (features
    of the call's first phase, action, log of its loop time over the time
    under action 0).  The value network is trained on the device.
    Evaluation: every call of a chain on the R-MAT scale-20 graph is replayed
    from one state under the fixed rule and under the learned per-call
    schedule (the order alternates), values must match, and the loop times
    are paired per call: median ratio, two-sided sign test, bootstrap 95 %
    interval of the mean log ratio."""
    import torch
    import workloads as W
    from paper_2511_05895_amd import mf
    from scipy.stats import binomtest

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    train = [W.rmat(17, 16, 903 + i) for i in range(2)] + [W.rmat(18, 16, 905 + i) for i in range(2)]
    X, A, Y = [], [], []
    for gi, g in enumerate(train):
        with mf.MaxFlow(g) as F:
            F.solve()
            for ids, new in _sched_chain(g, args.train_calls, 50 + gi):
                cap, cf, e, _, ecap = F.export_state()
                times, feats, values = [], None, set()
                for a in range(8):
                    F.import_state(cap, cf, e, ecap)
                    F.set_policy(None, mf.MF_POLICY_FORCED, action=a)
                    values.add(F.update(ids, new))
                    tr = F.policy_trace()
                    if tr.shape[0] == 0:
                        break
                    if feats is None:
                        feats = tr[0, :16].copy()
                    times.append(F.stats()["loop_kernel_ms"])
                if len(values) != 1:
                    raise SystemExit("FAIL: actions gave different values")
                if len(times) == 8:
                    for a in range(8):
                        X.append(feats)
                        A.append(a)
                        Y.append(np.log(times[a] / times[0]))
                F.import_state(cap, cf, e, ecap)
                F.set_policy(None, mf.MF_POLICY_FIXED)
                F.update(ids, new)
        print(f"[bench] learned: training graph {gi} (n={g.n}) collected, {len(X)} samples",
              file=sys.stderr, flush=True)
    X = np.array(X, np.float32)
    A = np.array(A, np.int32)
    Y = np.array(Y, np.float32)
    g = W.c3_rmat20()
    fixed, learned, acts = [], [], []
    with mf.Policy(seed=1) as P, mf.MaxFlow(g) as F:
        loss = P.train(X, A, Y, steps=2000, lr=3e-3)
        F.solve()
        for j, (ids, new) in enumerate(_sched_chain(g, args.steps, W.SEED_BASE + 2 + 100)):
            cap, cf, e, _, ecap = F.export_state()
            vals, ms = {}, {}
            for which in ((0, 1) if j % 2 == 0 else (1, 0)):
                F.import_state(cap, cf, e, ecap)
                if which == 0:
                    F.set_policy(None, mf.MF_POLICY_FIXED)
                else:
                    F.set_policy(P, mf.MF_POLICY_LEARNED | mf.MF_POLICY_PER_CALL, margin=0.05)
                vals[which] = F.update(ids, new)
                ms[which] = F.stats()["loop_kernel_ms"]
                if which == 1:
                    tr = F.policy_trace()
                    acts.append(int(tr[0, 16]) if tr.shape[0] else 0)
            if vals[0] != vals[1]:
                raise SystemExit(f"FAIL: learned value {vals[1]} != fixed value {vals[0]} at call {j}")
            fixed.append(ms[0])
            learned.append(ms[1])
            print(f"[bench] learned: call {j} ({ids.shape[0]} edges): fixed {ms[0]:.2f} ms, "
                  f"learned {ms[1]:.2f} ms, action {acts[-1]}", file=sys.stderr, flush=True)
    fixed = np.array(fixed)
    learned = np.array(learned)
    lr_ = np.log(learned / fixed)
    rng = np.random.default_rng(0)
    boot = [float(np.mean(rng.choice(lr_, lr_.size))) for _ in range(2000)]
    wins = int((learned < fixed).sum())
    decided = int((learned != fixed).sum())
    out = {
        "metric": "learned vs fixed phase schedule: loop time per update call (paired), exact flow",
        "value": float(fixed.sum() / learned.sum()),
        "unit": "x less loop time than the fixed rule (total over the chain)",
        "n_gpus": 1, "steps": int(fixed.size), "warmup": 0,
        "ms_per_step": float(learned.mean()),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 capacities / int64 excess; fp32 value network", "data": "synthetic (seeded generator)",
        "config": {"workload": "R-MAT scale 20 (avg degree 16), mixed 0.1/1/10 % batches; trained on R-MAT "
                               "scales 17/18 (other seeds)", "n": g.n, "m": g.m,
                   "train_samples": int(X.shape[0]), "train_loss": loss},
        "fixed_ms": {"mean": float(fixed.mean()), "p50": float(np.median(fixed))},
        "learned_ms": {"mean": float(learned.mean()), "p50": float(np.median(learned))},
        "per_call_ratio": {"median": float(np.exp(np.median(lr_))),
                           "mean_log_ci95": [float(np.percentile(boot, 2.5)), float(np.percentile(boot, 97.5))]},
        "sign_test": {"learned_faster": wins, "calls": decided,
                      "p_two_sided": float(binomtest(wins, decided, 0.5).pvalue) if decided else 1.0},
        "actions": np.bincount(acts, minlength=8).tolist(),
        "exact": "learned value == fixed value on every call",
    }
    print(json.dumps(out), flush=True)


def summarize_profile(path):
    """Per-kernel duration table from a rocprofv3 kernel-trace output: the
    rocpd SQLite database or the kernel_trace CSV."""
    rows = {}
    if path.endswith(".db"):
        import sqlite3
        cur = sqlite3.connect(path).cursor()
        for name, dur in cur.execute("select name, duration from kernels"):
            rows.setdefault(name, []).append(dur)
    else:
        import csv
        with open(path) as f:
            for r in csv.DictReader(f):
                rows.setdefault(r["Kernel_Name"], []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    total = sum(sum(v) for v in rows.values())
    print("| kernel | calls | total ms | avg ms | min ms | max ms | % |")
    print("|---|---|---|---|---|---|---|")
    for name, v in sorted(rows.items(), key=lambda kv: -sum(kv[1])):
        print(f"| `{name[:70]}` | {len(v)} | {sum(v) / 1e6:.3f} | {np.mean(v) / 1e6:.4f} | "
              f"{min(v) / 1e6:.4f} | {max(v) / 1e6:.4f} | {100.0 * sum(v) / total:.2f} |")


def _pmc_rows(db, counter):
    """(kernel name, dispatch id, value) of one counter from a rocprofv3 rocpd database."""
    import sqlite3
    cur = sqlite3.connect(db).cursor()
    q = ("select kernel_name, dispatch_id, value from counters_collection "
         "where counter_name = ? order by dispatch_id")
    return list(cur.execute(q, (counter,)))


def summarize_pmc(fetch_db, write_db, config, calib_mib, skip_first, command):
    """HBM traffic of the persistent solve loop from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE; both in KiB per dispatch).  Each counter is
    scaled by what it reads for the calibration kernel of the same process, an
    elementwise float32 negate over calib_mib MiB (reads and writes exactly
    that many bytes).  The first `skip_first` loop launches (the initial
    from-scratch solves, outside the timed steps) are left out.  Writes
    profiles/k_loop_<config>_pmc.json and prints a Markdown summary."""
    known = calib_mib * 1024.0  # KiB moved by one calibration dispatch
    out = {"kernel_digest": kernel_source_digest(), "command": command,
           "calibration": f"float32 negate over {calib_mib} MiB (torch.neg), {known:.0f} KiB read and written"}
    lines = [f"# HBM traffic of k_loop, {CONFIGS[config]['desc']}", "", "Command:", "", "```", command, "```", "",
             "| counter | calibration KiB/dispatch (known) | factor | k_loop launches | k_loop KiB/launch (raw) | "
             "k_loop bytes/launch (scaled) |", "|---|---|---|---|---|---|"]
    total = 0.0
    for key, db, counter in (("fetch", fetch_db, "FETCH_SIZE"), ("write", write_db, "WRITE_SIZE")):
        rows = _pmc_rows(db, counter)
        cal = [v for name, _, v in rows if "neg" in name and "elementwise" in name]
        loop = [v for name, _, v in rows if "k_loop" in name][skip_first:]
        if not cal or not loop:
            raise SystemExit(f"{db}: no calibration ({len(cal)}) or k_loop ({len(loop)}) dispatches for {counter}")
        cal_kib = float(np.median(cal))
        factor = known / cal_kib
        per = float(np.mean(loop)) * 1024.0 * factor
        total += per
        out[f"{key}_bytes_per_launch"] = per
        out[f"{key}_factor"] = factor
        out[f"{key}_launches"] = len(loop)
        lines.append(f"| {counter} | {cal_kib:.0f} ({known:.0f}) | {factor:.4f} | {len(loop)} | "
                     f"{np.mean(loop):.0f} | {per:.4g} |")
    out["bytes_per_launch"] = total
    lines += ["", f"HBM bytes per k_loop launch (fetch + write, scaled): {total:.4g}"]
    path = os.path.join(ROOT, "profiles", f"k_loop_{config}_pmc.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("\n".join(lines))


def main():
    if len(sys.argv) == 3 and sys.argv[1] == "--summarize-profile":
        summarize_profile(sys.argv[2])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-pmc":
        sp = argparse.ArgumentParser()
        sp.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DB", "WRITE_DB"))
        sp.add_argument("--config", default="grid512", choices=sorted(CONFIGS))
        sp.add_argument("--calibration-copy-mib", type=int, default=256)
        sp.add_argument("--skip-first", type=int, default=2)
        sp.add_argument("--command", default="")
        a = sp.parse_args()
        summarize_pmc(a.summarize_pmc[0], a.summarize_pmc[1], a.config, a.calibration_copy_mib,
                      a.skip_first, a.command)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="rmat22", choices=sorted(CONFIGS))
    ap.add_argument("--no-secondary", dest="secondary", action="store_false",
                    help="skip the R-MAT scale-20 leg of the default run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--grid-blocks", type=int, default=0)  # 0: the library sizes the grid
    ap.add_argument("--kernel-cycles", type=int, default=1)
    ap.add_argument("--mode", type=int, default=0)
    ap.add_argument("--updates", choices=["mixed", "inc", "dec"], default="mixed",
                    help="update family: half increments (default), all increments, all decrements")
    ap.add_argument("--batch-fraction", type=float, default=0.0,
                    help="edges per batch / m (0: the workload's own, 1%% or 100 edges)")
    ap.add_argument("--p-st", type=float, default=0.0,
                    help="probability that a batch edge is drawn from the edges out of s / into t")
    ap.add_argument("--workers", type=int, default=2, help="serving workers (c5)")
    ap.add_argument("--group-requests", type=int, default=64, help="requests one commit may merge (c5)")
    ap.add_argument("--group-edges", type=int, default=1 << 20, help="edges one commit may merge (c5)")
    ap.add_argument("--closed-requests", type=int, default=30, help="closed-loop requests (c5)")
    ap.add_argument("--open-requests", type=int, default=100, help="open-loop requests per load (c5)")
    ap.add_argument("--train-calls", type=int, default=18, help="update calls per training graph (learned20)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="run a float32 negate over this many MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the solver here is a single-GPU solver; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.config == "c4":
        run_batch(args)
        return
    if args.config == "c5":
        run_serving(args)
        return
    if args.config == "learned20":
        run_learned(args)
        return

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibration_copy_mib > 0:
        dev = torch.device("cuda:0")
        src = torch.ones(args.calibration_copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    out = run_dynamic(args.config, args, args.steps, args.warmup, cpu=not args.no_cpu_baseline)
    if args.config == "rmat22" and args.secondary:
        sec = run_dynamic("rmat20", args, min(args.steps, 10), min(args.warmup, 2), cpu=False)
        out["secondary"] = {k: sec[k] for k in ("config", "value", "unit", "dynamic_ms", "static_ms",
                                                 "speedup_dynamic_vs_static_p50", "roofline", "exact")}
    print(json.dumps(out), flush=True)


def run_dynamic(config, args, K, Wm, cpu):
    """Dynamic repair against static recompute on one workload: K timed steps
    after Wm untimed ones.  Every handle is closed before returning."""
    import torch
    import workloads as W
    from paper_2511_05895_amd import mf

    cfg = dict(CONFIGS[config])
    t0 = time.perf_counter()
    g, seed = make_graph(config)
    print(f"[bench] {config}: graph generated in {time.perf_counter() - t0:.1f} s (n={g.n}, m={g.m})",
          file=sys.stderr, flush=True)
    inc_fraction = {"mixed": 0.5, "inc": 1.0, "dec": 0.0}[args.updates]
    if cfg.get("requests"):
        chain = list(W.request_stream(g, Wm + K, seed))
    else:
        if args.batch_fraction > 0 or args.updates != "mixed" or args.p_st > 0:
            frac = args.batch_fraction if args.batch_fraction > 0 else cfg["frac"]
            kind = {"mixed": "mixed", "inc": "incremental", "dec": "decremental"}[args.updates]
            cfg["desc"] = cfg["base"] + f", {frac * 100:g}% {kind} batches" + \
                (f", s/t bias {args.p_st:g}" if args.p_st > 0 else "")
            cfg["frac"] = frac
        chain = list(W.batch_chain(g, cfg["frac"], Wm + K, cfg["inc_hi"], seed=seed,
                                   inc_fraction=inc_fraction, p_st=args.p_st))
    ks = [int(c[0].shape[0]) for c in chain[Wm:]]

    opts = dict(grid_blocks=args.grid_blocks, kernel_cycles=args.kernel_cycles, mode=args.mode)
    t0 = time.perf_counter()
    D = mf.MaxFlow(g, **opts)
    create_ms = (time.perf_counter() - t0) * 1e3
    S = mf.MaxFlow(g, **opts)
    print(f"[bench] {config}: handle created in {create_ms:.0f} ms", file=sys.stderr, flush=True)
    try:
        A = D.num_arcs
        t0 = time.perf_counter()
        v0 = D.solve()
        initial_static_ms = (time.perf_counter() - t0) * 1e3
        assert S.solve() == v0

        def step(j):
            ids, caps = chain[j]
            a = time.perf_counter()
            vd = D.update(ids, caps)  # host arrays: upload, repair, solve, value back
            b = time.perf_counter()
            sd = D.stats()
            S.set_capacities(ids, caps)
            c = time.perf_counter()
            vs = S.solve()
            d = time.perf_counter()
            ss = S.stats()
            if vd != vs:
                raise SystemExit(f"FAIL: dynamic value {vd} != static value {vs} at batch {j}")
            return (b - a) * 1e3, (d - c) * 1e3, sd, ss, vd

        for j in range(Wm):
            step(j)
        torch.cuda.synchronize()
        t_begin = time.perf_counter()
        rec = []
        for j in range(K):
            rec.append(step(Wm + j))
            print(f"[bench] {config} step {j}: k={ks[j]}, dynamic {rec[-1][0]:.2f} ms, static {rec[-1][1]:.2f} ms",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t_end = time.perf_counter()
        grid_blocks = D.stats()["grid_blocks"]
    finally:
        D.close()
        S.close()

    dyn = np.array([r[0] for r in rec])
    sta = np.array([r[1] for r in rec])
    values = [r[4] for r in rec]
    # dominant kernel: the persistent solve loop (dynamic and static launches)
    loop_ms = sum(r[2]["loop_kernel_ms"] + r[3]["loop_kernel_ms"] for r in rec)
    loop_launches = sum(r[2]["loop_launches"] + r[3]["loop_launches"] for r in rec)
    alg_bytes = sum(algorithmic_bytes(r[2], g.n) + algorithmic_bytes(r[3], g.n) for r in rec)
    achieved = alg_bytes / (loop_ms * 1e-3) / 1e9
    traffic = load_traffic(config, "bytes_per_launch")
    dyn_loop_ms = sum(r[2]["loop_kernel_ms"] for r in rec)
    dyn_bytes = sum(algorithmic_bytes(r[2], g.n) for r in rec)
    bfs_arcs = [r[2]["bfs_arcs"] for r in rec]

    out = {
        "metric": "update-batch latency ms (p50/p99) + residual edges/s, dynamic vs static, exact flow",
        "value": K * A / (dyn.sum() * 1e-3),
        "unit": "residual edges/s (dynamic update)",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": (t_end - t_begin) * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32 capacities / int64 excess",
        "data": "synthetic (seeded generator)",
        "config": {"workload": cfg["desc"], "n": g.n, "m": g.m, "arcs": A,
                   "batch_edges": {"min": min(ks), "median": int(np.median(ks)), "max": max(ks)},
                   "kernel_cycles": args.kernel_cycles or max(1, int(round(g.m / g.n))),
                   "grid_blocks": grid_blocks, "mode": ["data", "topology"][args.mode],
                   "batch_upload": "host arrays (mf_apply_updates; upload inside the timed latency)"},
        "dynamic_ms": {"p50": float(np.percentile(dyn, 50)), "p99": float(np.percentile(dyn, 99)),
                       "mean": float(dyn.mean())},
        "static_ms": {"p50": float(np.percentile(sta, 50)), "p99": float(np.percentile(sta, 99)),
                      "mean": float(sta.mean())},
        "static_edges_per_s": K * A / (sta.sum() * 1e-3),
        "update_edges_per_s": sum(ks) / (dyn.sum() * 1e-3),
        "speedup_dynamic_vs_static_p50": float(np.percentile(sta, 50) / np.percentile(dyn, 50)),
        "initial_static_ms": initial_static_ms,
        "create_ms": create_ms,
        "dynamic_iterations_mean": float(np.mean([r[2]["iterations"] for r in rec])),
        "static_iterations_mean": float(np.mean([r[3]["iterations"] for r in rec])),
        "dynamic_bfs_arcs_mean": float(np.mean(bfs_arcs)),
        "time_split_ms": {leg: {k: float(np.mean([r[i][k] for r in rec])) for k in ("bfs_ms", "pr_ms", "rie_ms")}
                          for leg, i in (("dynamic", 2), ("static", 3))},
        "exact": "dynamic value == static value on every step",
        "roofline": {
            "kernel": "k_loop<1024, agent scope, walk> (persistent solve loop; dynamic and static launches)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "launches": loop_launches,
            "avg_launch_ms": loop_ms / max(1, loop_launches),
            "alg_bytes_per_launch": alg_bytes / max(1, loop_launches),
            "dynamic_only_achieved": dyn_bytes / max(1e-9, dyn_loop_ms * 1e-3) / 1e9,
        },
    }
    if config == "grid512":
        out["roofline"]["note"] = "state (about 45 MB) is resident in the 256 MB Infinity Cache: not HBM-bound"
    if cpu:
        cap0 = g.cap.copy()
        for ids, new in chain[:Wm]:
            cap0[ids] = new
        cb = cpu_baseline(g, cap0, chain[Wm:], A, args.cpu_seconds)
        ref = cb.pop("values")
        if ref != values[: len(ref)]:
            raise SystemExit(f"FAIL: GPU values {values[:len(ref)]} != oracle values {ref}")
        cb["checked_against_gpu"] = len(ref)
        out["cpu_baseline"] = cb
    return out


if __name__ == "__main__":
    main()
