"""FastWalk throughput on one MI355X.

Default workload: the largest single-GPU configuration -- R-MAT scale 23 ((a, b, c) = (.57,
.19, .19), 5 edge draws per node, largest connected component: 3.34 M nodes, 41.3 M edges),
weights U[1, 4], 5000 rooted spanning trees sampled by Wilson's algorithm in one persistent
launch, RWC assembled in FP64, plus the adjoint of the RWC sum over 1000 targets (JL sketch,
k = 64).  One timed step is the whole hot path on device-resident inputs: CSR build
(rwc_build_csr), sampling (rwc_sample_forests), the pivot solve plus assembly (rwc_estimate)
and the adjoint (rwc_backward).

Prints one JSON line.  `value` is rooted trees per second for the whole step; walk steps/s,
grad edges/s, the dominant kernel's roofline, the CPU oracle's rate on the host cores (all of
them and one), and the BA(10^6) and BA(10^5) adjoint configurations ride along.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rooted trees/s + walk steps/s at fixed RWC rel. error; plain vs batched; grad edges/s"
# The paper's own measurements, for context only: it publishes accuracy and wall-clock plots but
# no trees/s or walk steps/s, on other graphs and hardware.
PAPER_CONTEXT = {"hardware": "Intel Xeon Gold 6240 @ 2.60 GHz, one thread, Julia, 256 GB",
                 "throughput": None,
                 "note": "no trees/s or walk steps/s published; on a graph of over 10 M nodes FastWalk reaches "
                         "0.5 % MRE in somewhat more than the ~4000 s its incomplete-Cholesky method needs for "
                         "3 % (Introduction)"}
HBM_PEAK_GBS = 8000.0
# HBM byte counters of the walk kernel, per workload, taken with rocprofv3 (FETCH_SIZE and
# WRITE_SIZE runs, scaled by the same counters on a plain copy kernel); valid only for the walk
# kernel sources they were taken on, which each file records by SHA-256.
TRAFFIC_FILES = {"rmat23": os.path.join(ROOT, "profiles", "wilson_team_rmat23_traffic.json"),
                 "ba1m": os.path.join(ROOT, "profiles", "wilson_team_ba1m_traffic.json")}
SAMPLER_SOURCES = ("paper_2510_20604_amd/csrc/walk.hpp", "paper_2510_20604_amd/csrc/select.hpp",
                   "paper_2510_20604_amd/csrc/device.hpp", "paper_2510_20604_amd/csrc/csr_build.hip")


def sampler_code_sha256() -> str:
    """SHA-256 of the walk kernel's sources and of the CSR build (which decides the node order in
    memory), comments removed and whitespace collapsed: the committed counters stay valid
    exactly while the code they were taken on is unchanged."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in SAMPLER_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_counters(config: str, kernel: str, trees: int, trees_in_flight: int):
    """The committed counter summary of the walk launch (HBM bytes, L2 misses), or None when it
    is missing or was taken on other code, another kernel or another plan."""
    if config not in TRAFFIC_FILES:
        return None
    try:
        with open(TRAFFIC_FILES[config]) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("code_sha256") != sampler_code_sha256() or t.get("kernel") != kernel or t.get("trees") != trees
            or t.get("trees_in_flight") != trees_in_flight):
        return None
    return t


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="rmat23",
                    choices=["rmat23", "ba1m", "er1000", "batch256", "grad100k", "trap", "group", "strata",
                             "fastchol"])
    ap.add_argument("--no-extras", action="store_true",
                    help="rmat23: skip the BA(1e6) and BA(1e5)-adjoint side measurements")
    ap.add_argument("--trees", type=int, default=0, help="override the number of trees")
    ap.add_argument("--walkers", type=int, default=0, help="walkers per tree (0 = automatic)")
    ap.add_argument("--tif", type=int, default=0, help="trees in flight (0 = automatic)")
    ap.add_argument("--no-lds", action="store_true", help="keep every tree's state in HBM (no LDS-resident trees)")
    ap.add_argument("--no-tune", action="store_true", help="batch256: automatic plan instead of rwc_autotune_batch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 1 GiB streaming copy (reference for HBM byte counters)")
    return ap.parse_args()


def workload(name):
    import rwcgen
    if name == "ba1m":
        g = rwcgen.barabasi_albert(1_000_000, 5, 1002)
        return g, 10_000, 2002, "BA(n=1e6, m=5) unit weights, 1e4 trees"
    g = rwcgen.erdos_renyi_lcc(1000, 8, 1001)
    return g, 2000, 2001, "ER(n=1000, d=8) LCC unit weights, 2000 trees"


def walk_bytes(total_steps: int, trees: int, n: int, weighted: bool, mean_probe: float = 0.0) -> float:
    """Algorithmic bytes of one walk launch: per walk step row_ptr[x], row_ptr[x+1] (8 B),
    col[k] (4 B), the state word of the next node (8 B) and the store of x's state word (8 B)
    (+ the CDF probes when weighted); per attached node the retrace reads and writes its state
    word (16 B); per tree the start scan reads each node's state word once (8 B)."""
    per_step = 28.0 + (8.0 * (1.0 + mean_probe) if weighted else 0.0)
    return per_step * total_steps + trees * (16.0 * (n - 1) + 8.0 * n)


def walk_accesses(total_steps: int, trees: int, n: int) -> float:
    """Random memory accesses of one walk launch (row_ptr pair, col, state load, state store
    per step; state load and store per attached node; one state load per scanned node)."""
    return 4.0 * total_steps + trees * (2.0 * (n - 1) + n)


def host_info() -> dict:
    """Host cores visible to this process and the CPU model (from /proc/cpuinfo)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline(g, l, seed, seconds, single_seconds=None):
    """The oracle's serial Wilson sampler (C) on this host: on all cores available to the
    process (the sample range split across threads), and on one core (the paper's
    single-thread setting), each over a bounded prefix of the workload's trees."""
    from oracle import wilson
    o = wilson.OracleCSR(g.n, g.src, g.dst, g.w)
    host = host_info()
    # the host cores this process may use: all it sees, capped by the thread budget the
    # environment sets for it (the GPU host shares its cores between GPUs)
    threads = max(1, min(host["nproc"], int(os.environ.get("OMP_NUM_THREADS", host["nproc"]))))
    t0 = time.perf_counter()
    one = wilson.fastwalk_sample(o, o.pivot, seed, 0, 0, 1)
    t1 = time.perf_counter() - t0
    print(f"cpu baseline: one tree in {t1:.2f} s", file=sys.stderr, flush=True)
    per_thread = max(1, int(seconds / max(t1, 1e-6)))
    nsamp = min(l, per_thread * threads)
    t0 = time.perf_counter()
    r = wilson.fastwalk_sample(o, o.pivot, seed, 0, 0, nsamp, threads=threads)
    dt = time.perf_counter() - t0
    print(f"cpu baseline: {nsamp} trees on {threads} threads in {dt:.1f} s", file=sys.stderr, flush=True)
    out = {"value": nsamp / dt, "unit": "trees/s", "cores": threads, "kind": "oracle",
           "sample": f"first {nsamp} of the {l} trees (samples 0..{nsamp - 1}), serial Wilson per thread, "
                     f"{threads} threads",
           "walk_steps_per_s": float(r["steps"].sum()) / dt, "host": host}
    if single_seconds:
        n1 = max(1, min(l, int(single_seconds / max(t1, 1e-6))))
        t0 = time.perf_counter()
        r1 = wilson.fastwalk_sample(o, o.pivot, seed, 0, 0, n1, threads=1)
        d1 = time.perf_counter() - t0
        print(f"cpu baseline: {n1} trees on 1 thread in {d1:.1f} s", file=sys.stderr, flush=True)
        out["single_thread"] = {"value": n1 / d1, "unit": "trees/s", "cores": 1,
                                "sample": f"first {n1} trees (samples 0..{n1 - 1}), one thread",
                                "walk_steps_per_s": float(r1["steps"].sum()) / d1}
    return out, r


def batch_main(args):
    """256 uneven graphs, 1000 trees each: one persistent hipGraph-captured launch against one
    plain launch per graph (same outputs, bit for bit)."""
    import torch
    import paper_2510_20604_amd as P
    import rwcgen
    t0 = time.perf_counter()
    gl = rwcgen.batch_mix(256, 1e3, 1e5, seed=1003)
    print(f"generated {len(gl)} graphs, sum n = {sum(g.n for g in gl)} in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    l, seed = args.trees or 1000, 2003
    dev = [P.Graph(g.n, g.src, g.dst, g.w, "cuda:0") for g in gl]
    torch.cuda.synchronize()

    keep = {}
    tune, tune_s, kw = None, None, {"lds_state": False if args.no_lds else None}
    if not args.no_tune:
        t0 = time.perf_counter()
        tune = P.autotune_batch(dev, l, seed)
        tune_s = time.perf_counter() - t0
        kw = {"walkers_per_graph": tune["walkers_per_graph"], "path_ring": tune["path_ring"],
              "bfs_starts": tune["bfs_starts"], "lds_state": tune["lds_state"]}
        print(f"autotuned in {tune_s:.1f}s: {tune}", file=sys.stderr, flush=True)

    def batched():
        # the same workspace and outputs each step: after the first call captures the launches
        # into a hipGraph, the later calls replay it
        r = P.sample_forests(dev, l, seed, persistent=True, capture=True, want_sq=False,
                             workspace=keep.get("workspace"), out=keep.get("out"), **kw)
        keep["workspace"], keep["out"] = r["workspace"], r
        return r

    def plain():
        out = []
        for i, G in enumerate(dev):
            out.append(P.sample_forests(G, l, seed, graph_index_base=i, want_sq=False,
                                        lds_state=False if args.no_lds else None))
            if i % 32 == 31:
                print(f"plain: {i + 1} graphs done", file=sys.stderr, flush=True)
        return out

    for _ in range(args.warmup):
        batched()
    times_b, times_p = [], []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        sb = batched()
        torch.cuda.synchronize()
        times_b.append(time.perf_counter() - t)
        print(f"batched step {time.perf_counter() - t:.3f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    sp = plain()
    torch.cuda.synchronize()
    times_p.append(time.perf_counter() - t)
    print(f"plain pass {times_p[-1]:.3f}s", file=sys.stderr, flush=True)
    same = all(torch.equal(sb["tree_hash"][i], r["tree_hash"][0]) for i, r in enumerate(sp))
    steps = int(P.as_uint64(sb["total_steps"]).sum())
    tb, tp = float(np.mean(times_b)), float(np.mean(times_p))
    line = {
        "metric": METRIC, "value": round(len(gl) * l / tb, 3), "unit": "trees/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * tb, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "256 graphs: 128 BA(m=3) + 128 grids with 10% edges deleted, n log-uniform "
                               "[1e3, 1e5], w ~ U[0.5, 2], 1000 trees each", "sum_n": int(sum(g.n for g in gl)),
                   "trees": len(gl) * l, "launch": "batched persistent + hipGraph"},
        "walk_steps_per_s": round(steps / tb, 1),
        "plain_trees_per_s": round(len(gl) * l / tp, 3), "plain_ms": round(1e3 * tp, 3),
        "batched_over_plain": round(tp / tb, 3), "bit_identical": bool(same),
        "graph_replayed": sb["graph_replayed"], "lds_graphs": sb["lds_graphs"],
        "tuned_plan": None if tune is None else {k: tune[k] for k in ("walkers_mesh", "walkers_other", "path_ring",
                                                                       "bfs_starts", "lds_state", "candidates",
                                                                       "probe_samples")},
        "tuning_s": None if tune_s is None else round(tune_s, 3),
    }
    print(json.dumps(line), flush=True)


def grad_main(args):
    """Adjoint throughput: BA(1e5, 4), w ~ U[0.5, 2], loss = sum of RWC over 100 random
    targets, JL sketch with k = 64 (rwc_backward)."""
    import torch
    import paper_2510_20604_amd as P
    import rwcgen
    g = rwcgen.barabasi_albert(100_000, 4, 1004)
    g = g.with_weights(rwcgen.uniform_weights(g.m, 0.5, 2.0, 1005))
    t = np.random.default_rng(6).choice(g.n, size=100, replace=False).astype(np.int32)
    gv = np.ones(100)
    G = P.Graph(g.n, g.src, g.dst, g.w, "cuda:0")
    gd = P.dense_g(g.n, t, gv, "cuda:0")
    for _ in range(args.warmup):
        P.backward(G, gd, k=64, seed=2004, tol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = P.backward(G, gd, k=64, seed=2004, tol=1e-8)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    line = {"metric": METRIC, "value": round(g.m / el, 1), "unit": "grad edges/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(1e3 * el, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
            "config": {"workload": "BA(n=1e5, m=4), w ~ U[0.5, 2], 100 targets, JL sketch k = 64", "n": g.n,
                       "m": g.m, "solve_columns": 66, "pcg_iters": r["iters"], "tol": 1e-8}}
    print(json.dumps(line), flush=True)


def probe_gather(ws, dev):
    """Measured random-access roofline: 524 288 dependent random 8-byte gather chains of 64
    loads each over the sampler's own workspace (its footprint), timed with HIP events."""
    import ctypes
    import torch
    from paper_2510_20604_amd import _lib
    words = ws.numel() // 8
    lanes, chain = 256 * 2048, 64
    sink = torch.empty(lanes, dtype=torch.int64, device=dev)
    ms = ctypes.c_float()
    lib = _lib.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for seed_probe in (1, 2):   # the first call warms up
        _lib.check(lib.rwc_probe_random_gather(ctypes.c_void_p(ws.data_ptr()), words, lanes, chain, seed_probe,
                                               ctypes.c_void_p(sink.data_ptr()), ctypes.byref(ms), stream),
                   "rwc_probe_random_gather")
    return lanes * chain / (ms.value * 1e-3), f"dependent random 8-byte gathers, {lanes} chains x {chain}, " \
                                              f"footprint {ws.numel() / 2**30:.1f} GiB"


def copy_probe(dev):
    """One 1 GiB streaming copy (rwc_probe_copy): the reference whose HBM byte counters scale
    the walk kernel's."""
    import ctypes
    import torch
    from paper_2510_20604_amd import _lib
    words = (1 << 30) // 8
    a = torch.zeros(words, dtype=torch.int64, device=dev)
    b = torch.empty(words, dtype=torch.int64, device=dev)
    ms = ctypes.c_float()
    _lib.check(_lib.lib().rwc_probe_copy(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), words,
                                         ctypes.byref(ms), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
               "rwc_probe_copy")
    return {"bytes_read": words * 8, "bytes_written": words * 8, "ms": ms.value,
            "GB_per_s": 2 * words * 8 / (ms.value * 1e-3) / 1e9}


def roofline_line(config, kernel, total_steps, l, n, weighted, walk_ms_launch, trees_in_flight, launches):
    bytes_launch = walk_bytes(total_steps, l, n, weighted) / launches
    achieved = bytes_launch / (walk_ms_launch * 1e-3) / 1e9
    counters = measured_counters(config, kernel, l, trees_in_flight)
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": counters["traffic_bytes_per_launch"] if counters else None,
            "kernel": kernel, "avg_launch_ms": round(walk_ms_launch, 3),
            "algorithmic_bytes_per_launch": bytes_launch, "traffic_unit": "HBM bytes per launch"}
    return roof, counters


def ba1m_side(args):
    """BA(1e6, 5), unit weights, 1e4 trees: CSR build + sampling + estimate per step."""
    import torch
    import paper_2510_20604_amd as P
    g, l, seed, desc = workload("ba1m")
    dev = torch.device("cuda:0")
    src, dst = torch.as_tensor(g.src).to(dev), torch.as_tensor(g.dst).to(dev)
    ws = {"sample": None}

    def step():
        G = P.Graph(g.n, src, dst, None, dev)
        s = P.sample_forests(G, l, seed, want_sq=False, want_hash=False, workspace=ws["sample"], sync=False)
        ws["sample"] = s["workspace"]
        P.estimate(G, s["counts"], l, want_hit=False)
        P.workspace_status(s["workspace"])
        return s

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 3
    for _ in range(k):
        s = step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / k
    steps = int(P.as_uint64(s["total_steps"])[0])
    del ws["sample"], s
    return {"workload": desc, "trees_per_s": round(l / el, 3), "ms_per_step": round(1e3 * el, 3),
            "walk_steps_per_s": round(steps / el, 1), "steps": k}


def grad_side(args):
    """BA(1e5, 4), w ~ U[0.5, 2], 100 targets, k = 64: grad edges per second."""
    import torch
    import paper_2510_20604_amd as P
    import rwcgen
    g = rwcgen.barabasi_albert(100_000, 4, 1004)
    g = g.with_weights(rwcgen.uniform_weights(g.m, 0.5, 2.0, 1005))
    t = np.random.default_rng(6).choice(g.n, size=100, replace=False).astype(np.int32)
    G = P.Graph(g.n, g.src, g.dst, g.w, "cuda:0")
    gd = P.dense_g(g.n, t, np.ones(100), "cuda:0")
    P.backward(G, gd, k=64, seed=2004, tol=1e-8)
    torch.cuda.synchronize()
    k = 5
    t0 = time.perf_counter()
    for _ in range(k):
        r = P.backward(G, gd, k=64, seed=2004, tol=1e-8)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / k
    return {"workload": "BA(n=1e5, m=4), w ~ U[0.5, 2], 100 targets, JL sketch k = 64", "m": g.m,
            "grad_edges_per_s": round(g.m / el, 1), "ms": round(1e3 * el, 3), "pcg_iters": r["iters"]}


def rmat_main(args):
    """The default: R-MAT scale 23 (a, b, c) = (.57, .19, .19), 5 edge draws per node, largest
    component, w ~ U[1, 4]; one step = CSR build + 5000 trees in a persistent launch + pivot
    solve and assembly + the adjoint of the RWC sum over 1000 targets (k = 64)."""
    import torch
    import paper_2510_20604_amd as P
    import rwcgen
    t0 = time.perf_counter()
    g = rwcgen.rmat_lcc(23, 5, 0.57, 0.19, 0.19, 1005)
    g = g.with_weights(rwcgen.uniform_weights(g.m, 1.0, 4.0, 1006))
    print(f"generated R-MAT LCC n={g.n} m={g.m} in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    l, seed = args.trees or 5000, 2005
    targets = np.random.default_rng(7).choice(g.n, size=1000, replace=False).astype(np.int32)
    dev = torch.device("cuda:0")
    src, dst = torch.as_tensor(g.src).to(dev), torch.as_tensor(g.dst).to(dev)
    w = torch.as_tensor(g.w).to(dev)
    gvec = P.dense_g(g.n, targets, np.ones(1000), dev)
    ws = {"sample": None}

    def step():
        G = P.Graph(g.n, src, dst, w, dev)
        s = P.sample_forests(G, l, seed, persistent=True, want_sq=True, want_hash=False, workspace=ws["sample"],
                             timing=True, walkers_per_tree=args.walkers, trees_in_flight=args.tif)
        ws["sample"] = s["workspace"]
        e = P.estimate(G, s["counts"], l, counts_sq=s["counts_sq"], want_stderr=True)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        r = P.backward(G, gvec, k=64, seed=2006, tol=1e-8)
        torch.cuda.synchronize()
        return G, s, e, r, time.perf_counter() - tb

    for _ in range(args.warmup):
        step()
        print("warmup step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    walk_ms, back_s = [], []
    for i in range(args.steps):
        G, s, e, r, tb = step()
        walk_ms.append(s["walk_ms"])
        back_s.append(tb)
        if i % 5 == 4 or i == args.steps - 1:
            print(f"timed step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = (time.perf_counter() - t0) / args.steps
    total_steps = int(P.as_uint64(s["total_steps"])[0])
    wms = float(np.mean(walk_ms)) / s["batches"]
    roof, counters = roofline_line("rmat23", s["walk_kernel"], total_steps, l, g.n, True, wms, s["trees_in_flight"],
                                   s["batches"])
    rel_se = (e["stderr"] / e["rwc"]).double()
    mask = torch.ones(g.n, dtype=torch.bool, device=dev)
    mask[G.pivot] = False
    line = {
        "metric": METRIC, "value": round(l / elapsed, 3), "unit": "trees/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64/f64", "data": "synthetic",
        "config": {"workload": "R-MAT scale 23 (.57, .19, .19), 5n draws, LCC, w ~ U[1, 4]; 5000 trees persistent "
                               "+ adjoint for 1000 targets, k = 64", "n": g.n, "m": g.m, "trees": l,
                   "walkers_per_tree": s["walkers_per_tree"], "trees_in_flight": s["trees_in_flight"],
                   "walk_launches": s["batches"], "starts": s["starts"], "launch": "persistent"},
        "walk_steps_per_s": round(total_steps / elapsed, 1),
        "walk_steps_per_tree": total_steps / l,
        "sampler_trees_per_s": round(l / (np.mean(walk_ms) * 1e-3), 3),
        "grad_edges_per_s": round(g.m / float(np.mean(back_s)), 1),
        "backward_ms": round(1e3 * float(np.mean(back_s)), 3),
        "pcg_iters": e["iters"], "adjoint_iters": r["iters"],
        "rwc_rel_stderr_mean": float(rel_se[mask].mean()),
        "roofline": roof,
    }
    if not args.no_probe:
        peak_acc, desc = probe_gather(ws["sample"], dev)
        gr = {"probe": desc, "peak_accesses_per_s": peak_acc,
              "walk_algorithmic_accesses_per_s": walk_accesses(total_steps, l, g.n) / s["batches"] / (wms * 1e-3)}
        if counters:
            miss = counters["tcc_miss_per_dispatch"] / (wms * 1e-3)
            gr.update({"walk_l2_misses_per_s": miss, "frac": round(miss / peak_acc, 4)})
        else:
            gr["frac"] = None
        line["gather_roofline"] = gr
    del ws["sample"], s, e, r, G
    torch.cuda.empty_cache()
    if args.copy_probe:
        line["copy_probe"] = copy_probe(dev)
    if not args.no_extras:
        line["ba1m"] = ba1m_side(args)
        print("BA(1e6) side measurement done", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        line["grad100k"] = grad_side(args)
        print("BA(1e5) adjoint side measurement done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        cb, _ = cpu_baseline(g, l, seed, args.cpu_seconds, single_seconds=args.cpu_seconds * 0.67)
        line["cpu_baseline"] = cb
    line["paper_context"] = PAPER_CONTEXT
    print(json.dumps(line), flush=True)


def _golden_rwc(name):
    """Stored exact RWC values (node -> value) written by the committed oracle scripts under
    tests/golden (plain text; nothing is computed here)."""
    path = os.path.join(ROOT, "tests", "golden", name)
    rows = [line.split("|") for line in open(path) if not line.startswith("#")]
    return np.array([int(a) for a, _ in rows]), np.array([float(b) for _, b in rows])


def trap_main(args):
    """Same-GPU ablation of Wilson's reuse of every walk step (FastWalk, Algorithm 3) against the
    trap walks of Lemma 5.1 (independent walks from every node, counting returns), at equal
    accuracy: both estimate diag(calL_v^{-1}) and go through the same rwc_estimate.  The trap
    walks' count per node is chosen from a pilot run so that their mean relative error matches
    Wilson's (the error falls as 1/sqrt(l)); reported are the device times to that accuracy."""
    import torch
    import paper_2510_20604_amd as P
    import rwcgen
    cases = [("ER(n=1000, d=8) LCC, unit weights", rwcgen.erdos_renyi_lcc(1000, 8, 1001), "er1000_exact_rwc.txt",
              2000, 2001),
             ("BA(n=20000, m=5), unit weights", rwcgen.barabasi_albert(20_000, 5, 1002), "ba20k_exact_rwc.txt",
              2000, 2002)]
    out = []
    for desc, g, golden, l_w, seed in cases:
        nodes, exact = _golden_rwc(golden)
        G = P.Graph(g.n, g.src, g.dst, g.w, "cuda:0")

        def mre(rwc):
            got = rwc.cpu().numpy()[nodes]
            return float(np.mean(np.abs(got - exact) / exact))

        def timed(fn, reps=3):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                r = fn()
            torch.cuda.synchronize()
            return r, (time.perf_counter() - t0) / reps

        def wilson():
            s = P.sample_forests(G, l_w, seed, want_sq=False, want_hash=False)
            return s, P.estimate(G, s["counts"], l_w, want_hit=False)["rwc"]

        def trap(l_t):
            def run():
                t = P.sample_trap_walks(G, l_t, seed, want_sq=False)
                return t, P.estimate(G, t["counts"], l_t, want_hit=False)["rwc"]
            return run

        (sw, rw), tw = timed(wilson)
        e_w = mre(rw)
        l0 = 200
        (_, r0), _ = timed(trap(l0), reps=1)
        e0 = mre(r0)
        l_t = max(1, int(np.ceil(l0 * (e0 / e_w) ** 2)))
        (st_, rt), tt = timed(trap(l_t))
        e_t = mre(rt)
        steps_w = int(P.as_uint64(sw["total_steps"])[0])
        steps_t = int(P.as_uint64(st_["total_steps"])[0])
        out.append({"workload": desc, "wilson": {"trees": l_w, "mre": e_w, "ms": round(1e3 * tw, 3),
                                                 "walk_steps": steps_w},
                    "trap_walks": {"walks_per_node": l_t, "mre": e_t, "ms": round(1e3 * tt, 3), "walk_steps": steps_t,
                                   "pilot": {"walks_per_node": l0, "mre": e0}},
                    "time_ratio_trap_over_wilson": round(tt / tw, 3),
                    "step_ratio_trap_over_wilson": round(steps_t / steps_w, 3)})
        print(f"{desc}: Wilson {1e3 * tw:.2f} ms (MRE {e_w:.4%}), trap walks {1e3 * tt:.2f} ms "
              f"(MRE {e_t:.4%}, {l_t} walks per node)", file=sys.stderr, flush=True)
    line = {"metric": METRIC, "value": out[0]["time_ratio_trap_over_wilson"], "unit": "x (trap / Wilson time)",
            "n_gpus": 1, "higher_is_better": True, "dtype": "u64/f64", "data": "synthetic",
            "config": {"workload": "trap walks (Lemma 5.1) vs Wilson forests at equal MRE"}, "cases": out}
    print(json.dumps(line), flush=True)


def group_main(args):
    """Group RWC (root sets): BA(1e6, 5), unit weights, S = the 16 nodes of largest degree; one
    step = CSR build + 10^4 spanning forests rooted at S + the group estimate (H_S and H_{S+u}
    for every u)."""
    import torch
    import paper_2510_20604_amd as P
    g, _, seed, _ = workload("ba1m")
    l = args.trees or 10_000
    dev = torch.device("cuda:0")
    src, dst = torch.as_tensor(g.src).to(dev), torch.as_tensor(g.dst).to(dev)
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)
    roots = np.sort(np.argsort(-deg, kind="stable")[:16]).astype(np.int32)
    ws = {}

    def step():
        G = P.Graph(g.n, src, dst, None, dev)
        s = P.sample_forests(G, l, seed, roots=roots, want_sq=False, want_hash=False, workspace=ws.get("s"),
                             timing=True)
        ws["s"] = s["workspace"]
        e = P.estimate_group(G, roots, s["counts"], l)
        return s, e

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    walk_ms = []
    for _ in range(args.steps):
        s, e = step()
        walk_ms.append(s["walk_ms"])
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    steps = int(P.as_uint64(s["total_steps"])[0])
    line = {"metric": METRIC, "value": round(l / el, 3), "unit": "forests/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(1e3 * el, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u64/f64", "data": "synthetic",
            "config": {"workload": "BA(n=1e6, m=5) unit weights, 1e4 forests rooted at the 16 nodes of largest "
                                   "degree, group estimate", "n": g.n, "m": g.m, "roots": len(roots),
                       "walkers_per_tree": s["walkers_per_tree"], "walk_kernel": s["walk_kernel"]},
            "walk_steps_per_s": round(steps / el, 1), "walk_steps_per_forest": steps / l,
            "sampler_forests_per_s": round(l / (np.mean(walk_ms) * 1e-3), 3),
            "group_rwc": float(e["group_rwc"][0]), "best_addition": int(torch.argmin(e["marginal"]))}
    print(json.dumps(line), flush=True)


def strata_main(args):
    """Variance reduction at equal trees (the Conclusion's "more efficient sampling"): every
    stack entry stratified over the l samples (Latin hypercube, rwc_sample_params.strata = l)
    against independent draws, same graphs, same l, same estimator.  On graphs with stored exact
    RWC: mean relative error over 16 seeds.  On BA(1e6, 5) with 10^4 trees: the relative mean
    squared error of RWC estimated from the spread over 6 seeds (both estimators are unbiased).
    Reported: the error ratio, the trees independent draws need for the same error
    ((MRE ratio)^2 or the MSE ratio) and the walk kernel's time in both modes."""
    import torch
    import paper_2510_20604_amd as P
    import rwcgen

    def run(G, l, seed, strata):
        s = P.sample_forests(G, l, seed, want_sq=False, want_hash=False, timing=True, strata=strata)
        return P.estimate(G, s["counts"], l, want_hit=False)["rwc"].cpu().numpy(), s["walk_ms"], s["walk_kernel"]

    cases = []
    for desc, g, golden, l in (("ER(n=1000, d=8) LCC, unit weights", rwcgen.erdos_renyi_lcc(1000, 8, 1001),
                                "er1000_exact_rwc.txt", 2000),
                               ("BA(n=20000, m=5), unit weights", rwcgen.barabasi_albert(20_000, 5, 1002),
                                "ba20k_exact_rwc.txt", 2000)):
        nodes, exact = _golden_rwc(golden)
        G = P.Graph(g.n, g.src, g.dst, g.w, "cuda:0")
        res = {}
        for mode, strata in (("independent", 0), ("stratified", l)):
            run(G, l, 1, strata)
            mre, ms = [], []
            for seed in range(16):
                rwc, wm, kern = run(G, l, 5000 + seed, strata)
                mre.append(float(np.mean(np.abs(rwc[nodes] - exact) / exact)))
                ms.append(wm)
            res[mode] = {"mre": float(np.mean(mre)), "mre_sd": float(np.std(mre, ddof=1)),
                         "walk_ms": round(float(np.median(ms)), 3), "walk_kernel": kern}
        ratio = res["stratified"]["mre"] / res["independent"]["mre"]
        cases.append({"workload": desc, "trees": l, "seeds": 16, **res, "mre_ratio": round(ratio, 4),
                      "independent_trees_for_equal_mre": round(l / ratio ** 2, 1)})
        print(f"{desc}: MRE {res['independent']['mre']:.4%} -> {res['stratified']['mre']:.4%} at {l} trees",
              file=sys.stderr, flush=True)

    g, l, _, desc = workload("ba1m")
    l = args.trees or l
    G = P.Graph(g.n, g.src, g.dst, g.w, "cuda:0")
    big = {}
    for mode, strata in (("independent", 0), ("stratified", l)):
        run(G, l, 1, strata)
        est, ms = [], []
        for seed in range(6):
            rwc, wm, kern = run(G, l, 7000 + seed, strata)
            est.append(rwc)
            ms.append(wm)
        est = np.asarray(est)
        rel_mse = float(np.mean(est.var(0, ddof=1) / est.mean(0) ** 2))
        big[mode] = {"rel_mse": rel_mse, "walk_ms": round(float(np.median(ms)), 3), "walk_kernel": kern,
                     "trees_per_s_walk": round(l / (np.median(ms) * 1e-3), 1)}
        print(f"{desc} {mode}: relative MSE {rel_mse:.3e}, walk {np.median(ms):.1f} ms", file=sys.stderr, flush=True)
    mse_ratio = big["stratified"]["rel_mse"] / big["independent"]["rel_mse"]
    cases.append({"workload": desc, "trees": l, "seeds": 6, **big, "rel_mse_ratio": round(mse_ratio, 4),
                  "independent_trees_for_equal_error": round(l / mse_ratio, 1),
                  "walk_time_ratio": round(big["stratified"]["walk_ms"] / big["independent"]["walk_ms"], 4)})
    line = {"metric": METRIC, "value": round(1.0 / mse_ratio, 4),
            "unit": "x (independent trees per stratified tree at equal error)", "n_gpus": 1,
            "higher_is_better": True, "dtype": "u64/f64", "data": "synthetic",
            "config": {"workload": "stratified vs independent stack entries at equal trees (BA(1e6, 5), 1e4 trees; "
                                   "ER(1000) and BA(20000) against exact RWC)"}, "cases": cases}
    print(json.dumps(line), flush=True)


def fastchol_main(args):
    """FastChol (Section 4, Algorithm 2) on the GPU: the threshold incomplete Cholesky factor
    (delta = 1e-4, columns in input order) and its windowed, sparsified inverse (w_s = zeta =
    ceil(log2 n), eps_p = 1e-3), then the same AppRWC assembly.  Per graph with stored exact RWC:
    the device time of the estimate (dense right-looking IChol, the default at these sizes) and of
    the assembly, the left-looking one-wave chain timed beside it (same bits), the MRE, the
    factor's size, and the serial oracle's time on the host."""
    import torch
    import paper_2510_20604_amd as P
    import rwcgen
    cases = [("ER(n=1000, d=8) LCC, unit weights", lambda: rwcgen.erdos_renyi_lcc(1000, 8, 1001), "er1000_exact_rwc.txt"),
             ("BA(n=20000, m=5), unit weights", lambda: rwcgen.barabasi_albert(20_000, 5, 1002), "ba20k_exact_rwc.txt"),
             ("BA(n=60000, m=5), unit weights (no stored exact RWC)", lambda: rwcgen.barabasi_albert(60_000, 5, 1003),
              None)]
    out = []
    for desc, make, golden in cases:
        g = make()
        nodes, exact = _golden_rwc(golden) if golden else (None, None)
        G = P.Graph(g.n, g.src, g.dst, g.w, "cuda:0")
        lg = int(np.ceil(np.log2(g.n)))
        kw = dict(droptol=1e-4, window=float(lg), zeta=lg, eps_p=1e-3)
        P.estimate_diag(G, P.fastchol(G, **kw)["tau"], want_hit=False)   # warm-up of the whole timed path
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = P.fastchol(G, **kw)
        e = P.estimate_diag(G, r["tau"], want_hit=False)
        torch.cuda.synchronize()
        gpu_s = time.perf_counter() - t0
        rwc = e["rwc"].cpu().numpy()
        mre = float(np.mean(np.abs(rwc[nodes] - exact) / exact)) if golden else None
        t0 = time.perf_counter()
        rc = P.fastchol(G, method="chain", **kw)
        torch.cuda.synchronize()
        chain_s = time.perf_counter() - t0
        item = {"workload": desc, "n": g.n, "m": g.m, "params": kw, "gpu_ms": round(1e3 * gpu_s, 2), "mre": mre,
                "factor_entries": r["factor_entries"], "inverse_entries": r["inverse_entries"],
                "ichol_method": "dense", "chain_ms": round(1e3 * chain_s, 2),
                "chain_tau_bit_identical": bool(torch.equal(rc["tau"], r["tau"]))}
        if not args.no_cpu_baseline:
            from oracle import fastchol as OF
            t1 = time.perf_counter()
            o = OF.fastchol(g.n, g.src, g.dst, g.w, G.pivot, **{"droptol": 1e-4, "ws": float(lg), "zeta": lg,
                                                                 "eps_p": 1e-3})
            cpu_s = time.perf_counter() - t1
            same = bool(np.array_equal(o["tau"], r["tau"].cpu().numpy()))
            item["cpu_baseline"] = {"seconds": round(cpu_s, 3), "cores": 1, "kind": "oracle",
                                    "sample": "the whole FastChol estimate (both chains), one thread",
                                    "tau_bit_identical": same}
        out.append(item)
        print(f"{desc}: FastChol {1e3 * gpu_s:.1f} ms on the GPU, MRE {mre}, factor {r['factor_entries']} "
              f"entries", file=sys.stderr, flush=True)
        del r, rc, e
        torch.cuda.empty_cache()   # the next graph's dense array takes the room of this one's
    line = {"metric": METRIC, "value": out[1]["gpu_ms"], "unit": "ms per FastChol estimate", "n_gpus": 1,
            "higher_is_better": False, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "FastChol (Algorithm 2) on BA(20000, 5) (the value), ER(1000, 8) against exact "
                                   "RWC, and BA(60000, 5)"},
            "cases": out}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sampler shards by "
              "sample range with one all-reduce of the visit totals, which is not implemented here.",
              file=sys.stderr)
        sys.exit(2)
    if args.config == "grad100k":
        return grad_main(args)
    if args.config == "rmat23":
        return rmat_main(args)
    if args.config == "batch256":
        return batch_main(args)
    if args.config == "trap":
        return trap_main(args)
    if args.config == "group":
        return group_main(args)
    if args.config == "strata":
        return strata_main(args)
    if args.config == "fastchol":
        return fastchol_main(args)
    import torch
    import paper_2510_20604_amd as P
    from paper_2510_20604_amd import _lib

    g, l, seed, desc = workload(args.config)
    if args.trees:
        l = args.trees
    dev = torch.device("cuda:0")
    src = torch.as_tensor(g.src).to(dev)
    dst = torch.as_tensor(g.dst).to(dev)
    ws = {"sample": None}

    def step():
        G = P.Graph(g.n, src, dst, None, dev)
        s = P.sample_forests(G, l, seed, want_sq=True, want_hash=False, workspace=ws["sample"], timing=True,
                             walkers_per_tree=args.walkers, trees_in_flight=args.tif,
                             lds_state=False if args.no_lds else None)
        ws["sample"] = s["workspace"]
        e = P.estimate(G, s["counts"], l, counts_sq=s["counts_sq"], want_stderr=True)
        return G, s, e

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    walk_ms, reduce_ms, steps_total = [], [], 0
    for _ in range(args.steps):
        G, s, e = step()
        walk_ms.append(s["walk_ms"])
        reduce_ms.append(s["reduce_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    total_steps = int(P.as_uint64(s["total_steps"])[0])
    trees_in_flight = s["trees_in_flight"]
    launches = s["batches"]
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps * l / elapsed

    # roofline of the dominant kernel (the walk)
    wms = float(np.mean(walk_ms)) / launches
    roof, counters = roofline_line(args.config, s["walk_kernel"], total_steps, l, g.n, False, wms, trees_in_flight,
                                   launches)
    extra = {}
    if not args.no_probe:
        peak_acc, desc_probe = probe_gather(ws["sample"], dev)
        gr = {"probe": desc_probe, "peak_accesses_per_s": peak_acc,
              "walk_algorithmic_accesses_per_s": walk_accesses(total_steps, l, g.n) / launches / (wms * 1e-3)}
        if counters:
            # every L2 miss of the walk is one random line access to the fabric, the quantity the
            # probe saturates (its own accesses all miss)
            miss = counters["tcc_miss_per_dispatch"] / (wms * 1e-3)
            gr.update({"walk_l2_misses_per_s": miss, "frac": round(miss / peak_acc, 4)})
        else:
            gr["frac"] = None
        extra["gather_roofline"] = gr

    if args.copy_probe:
        extra["copy_probe"] = copy_probe(dev)

    rel_se = (e["stderr"] / e["rwc"]).double()
    mask = torch.ones(g.n, dtype=torch.bool, device=dev)
    mask[G.pivot] = False
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "trees/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": desc, "n": g.n, "m": g.m, "trees": l, "trees_in_flight": trees_in_flight,
                   "walkers_per_tree": s["walkers_per_tree"], "starts": s["starts"], "walk_launches": launches,
                   "launch": "plain", "walk_kernel": s["walk_kernel"]},
        "walk_steps_per_s": round(args.steps * total_steps / elapsed, 1),
        "walk_steps_per_tree": total_steps / l,
        "sampler_trees_per_s": round(l / (np.mean(walk_ms) + np.mean(reduce_ms)) * 1e3, 3),
        "rwc_rel_stderr_mean": float(rel_se[mask].mean()),
        "pcg_iters": e["iters"],
        "roofline": roof,
    }
    line.update(extra)
    if not args.no_cpu_baseline:
        cb, _ = cpu_baseline(g, l, seed, args.cpu_seconds, single_seconds=args.cpu_seconds * 0.67)
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
