#!/usr/bin/env python3
"""Benchmark: level-synchronous BFS on seeded R-MAT graphs on one MI355X.

Headline workload: R-MAT scale 26 (edge factor 16, a/b/c/d = 0.57/0.19/0.19/
0.05, symmetrised, relabelled) with its 64 seeded roots of positive degree.
A step is one pass over all 64 roots, each one BFS (init, every level's
expand and fold, output) on a graph already resident in HBM. The value is
the harmonic mean of per-root TEPS over every timed pass, with TEPS =
(undirected edges of the searched component) / (BFS time), in GTEPS; roots
outside the large component are searched but left out of the mean (the
paper's section 6 counts sources in the large component only).
ms_per_step is the wall time of one pass. The timed passes run with
profiling off.

The JSON line also carries:
  roofline      the level kernel with the most device time: algorithmic
                bytes per launch (from each search's per-level record) /
                average launch duration, from HIP events recorded around every
                launch in one profiled pass over the same roots right after
                the timed passes (one launch per enqueued level, all counted);
                traffic = HBM bytes per launch from the committed rocprofv3
                counter summary of that kernel and workload, while its
                sources are unchanged
  level_kernels the same figures for each level kernel
  bfs_roofline_frac   whole-BFS algorithmic bytes of a push search
                (4 A + A/8 + 24 |R| + 8 n + n/4 per root) / BFS time
  bfs_examined_frac   the bytes the search's levels actually examined (per
                level record: pushed adjacencies, pull searches, bitmap
                passes, init and output) / BFS time
  cpu_baseline  the CPU oracle (serial C) timed on a bounded sample of roots
  workloads     the other BFS configurations (Erdos-Renyi 26, R-MAT 22 with
                its 64 roots, R-MAT 12's microseconds per BFS)
  spmspv        the 2D share (2^26 x 2^26 DCSC, 2^24 uniform nonzeros): 200
                local products, 50 at each frontier density, p50 per density,
                beside the floor of an empty call
  mix           1024 queries over R-MAT scales 14-22 and 512^2 / 2048^2
                grids: one-at-a-time plain path, one batched launch, and the
                continuous-batching server under Poisson arrivals at 0.5x, 4x
                and 16x the plain path's capacity (GTEPS, p50/p99 latency)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GTEPS (harmonic mean over roots) + % HBM roofline; batched p50/p99 latency"
KERNELS = ("k_expand", "k_expand_mark", "k_finish", "k_small_levels")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------------- byte counts
# Algorithmic bytes per level, from a search's per-level record (one dict per
# launched level: mark = 0 claim, 1 push mark, 2 pull, 3 claim-touch claim
# level (collected by the level in the parent words), 4 claim level run by the device level loop; frontier/edges = the level's input frontier and its
# adjacencies; pull_candidates/pull_edges = a pull level's searchers and the
# adjacencies they examined, or a push mark level's resolved vertices and the
# adjacencies their searches examined). "new" is the next level's input
# frontier, i.e. the vertices this level reached. A read-modify-write of a
# word counts its bytes twice (read and write).

def _new(levels, i):
    return levels[i + 1]["frontier"] if i + 1 < len(levels) else 0


def _beyond_head(L):
    """Adjacencies a search examined past the first three of each searcher,
    which the head entry already holds (a lower bound)."""
    return max(L["pull_edges"] - 3 * L["pull_candidates"], 0)


def claim_bytes(levels, nwords: int) -> float:
    """k_expand. Claim level: per scanned adjacency 4 B (the adjacency) + 1/8 B
    (the target's visited bit); per input frontier vertex 20 B (its queue
    entry: id, adjacency start, edge prefix); per vertex claimed 53 B (its
    packed word read and atomic min, 16 B; its two row offsets, 16 B; its queue
    entry, 20 B; its tag, 1 B). Claim-touch level: per new vertex 16 B (the
    atomic min of its word). Mark and pull
    levels: the level-(k-1) bitmap built from the tags over the whole
    graph, 32 B of tags read and 4 B written per bitmap word."""
    total = 0.0
    for i, L in enumerate(levels):
        if L["frontier"] == 0 or L["mark"] == 4:
            continue
        if L["mark"] in (1, 2):
            total += 36.0 * nwords
            continue
        per_new = 16.0 if L["mark"] == 3 else 53.0
        total += 4.125 * L["edges"] + 20.0 * L["frontier"] + per_new * _new(levels, i)
    return total


def mark_expand_bytes(levels) -> float:
    """k_expand_mark on push mark levels: per scanned adjacency 4 B + 1/8 B;
    per input frontier vertex 16 B (adjacency start, edge prefix); per vertex
    reached 1 B (its touch byte). The level's resolve (run by the next launch
    of the same kernel): per resolved vertex 44 B (queue entry 20 B, head
    entry 16 B, packed word 8 B) and 4 B + 1/8 B per adjacency examined past
    the head entry."""
    total = 0.0
    for i, L in enumerate(levels):
        if L["mark"] != 1 or L["frontier"] == 0:
            continue
        total += 4.125 * L["edges"] + 16.0 * L["frontier"] + 1.0 * _new(levels, i)
        total += 44.0 * L["pull_candidates"] + 4.125 * _beyond_head(L)
    return total


def pull_bytes(levels, n_active: int) -> float:
    """k_expand_mark on pull levels: the visited bits of the n_active
    vertices of positive degree; per searching vertex 16 B (its head entry);
    4 B + 1/8 B per adjacency examined past the head entry; per vertex found
    13 B (its packed word, its touch byte, the parent's caller id)."""
    total = 0.0
    for i, L in enumerate(levels):
        if L["mark"] != 2 or L["frontier"] == 0:
            continue
        total += (n_active / 8.0 + 16.0 * L["pull_candidates"] + 4.125 * _beyond_head(L)
                  + 13.0 * _new(levels, i))
    return total


def finish_bytes(levels, nwords: int, n_active: int | None = None) -> float:
    """k_finish. Claim level: per new vertex its queue id read and the atomic
    OR of its visited word (12 B); a large claim level (new frontier at
    least n/64) instead rebuilds the bitmap from the tags, 32 B read and 4 B
    written per word. Mark and pull levels: the tags of the whole graph (32 B
    per word) read. Claim-touch levels: the visited bitmap (4 B per word),
    the parent word of every vertex of positive degree not visited before the
    level (8 B), and the tags of the words that hold a new vertex (32 B per
    word, at most one word per new vertex). Then on all three: per new vertex
    its tag and visited bit rewritten with its word (1 B + 1/8 B), and its
    two row offsets and queue entry (36 B) unless the level pulls and so does
    the next one (no queue is built then)."""
    total = 0.0
    n = nwords * 32
    n_act = n if n_active is None else n_active
    seen = 0   # vertices visited before the level (the input frontiers so far)
    for i, L in enumerate(levels):
        seen += L["frontier"]
        if L["frontier"] == 0 or L["mark"] == 4:
            continue
        new = _new(levels, i)
        if L["mark"] == 0:
            total += 36.0 * nwords if new * 64 >= n else 12.0 * new
            continue
        next_pulls = i + 1 < len(levels) and levels[i + 1]["mark"] == 2
        queue = 0.0 if (L["mark"] == 2 and next_pulls) else 36.0
        if L["mark"] == 3:
            scan = 4.0 * nwords + 8.0 * max(n_act - seen, 0) + 32.0 * min(nwords, new)
        else:
            scan = 32.0 * nwords
        total += scan + (1.125 + queue) * new
    return total


def small_levels_bytes(levels) -> float:
    """k_small_levels (the device level loop): per level it runs, 4 B + 1/8 B
    per scanned adjacency (the adjacency, the target's word read as the
    visited test counts its 1/8 B bit), 20 B per frontier vertex staged (its
    queue entry), and per vertex claimed 53 B as on a claim level."""
    total = 0.0
    for i, L in enumerate(levels):
        if L["mark"] != 4 or L["frontier"] == 0:
            continue
        total += 4.125 * L["edges"] + 20.0 * L["frontier"] + 53.0 * _new(levels, i)
    return total


def init_out_bytes(n: int, n_active: int, nwords: int, symmetric: bool = True) -> float:
    """k_init (packed words of the n_active searchable vertices, visited
    bitmap, tag bytes) and k_out (rank 4 B, packed word 8 B, parent and level
    8 B per caller id)."""
    return 8.0 * n_active + 4.0 * nwords + (32.0 * nwords if symmetric else 0.0) + 20.0 * n


def examined_bytes(levels, n: int, n_active: int) -> float:
    """Whole-BFS bytes the levels examined (the sum of the kernels above)."""
    nwords = (n + 31) // 32
    return (claim_bytes(levels, nwords) + mark_expand_bytes(levels)
            + pull_bytes(levels, n_active) + finish_bytes(levels, nwords, n_active)
            + small_levels_bytes(levels) + init_out_bytes(n, n_active, nwords))


def bfs_bytes(n: int, edges: int, reached: int) -> float:
    """Whole-BFS algorithmic bytes of a push search: 4 A + A/8 + 24 |R| + 8 n +
    n/4, with A the adjacencies of the searched component."""
    return 4.125 * edges + 24.0 * reached + 8.0 * n + n / 4.0


KERNEL_SOURCES = {"k_expand_mark": ("bfs_mark.hip", "bfs_search.h", "bfs_level.h"),
                  "k_expand": ("bfs_csr.hip", "bfs_level.h"),
                  "k_finish": ("bfs_csr.hip", "bfs_level.h"),
                  "k_small_levels": ("bfs_small.hip", "bfs_level.h"),
                  "k_spmspv_bin": ("bfs_dcsc.hip",),
                  "k_spmspv_reduce": ("bfs_dcsc.hip",)}


def kernel_source_hash(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1104_4518_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel: str, workload: str):
    """HBM bytes per launch of the kernel from the committed rocprofv3
    counter summary, or None when its sources changed since it was taken."""
    import re
    prof = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    try:
        with open(prof) as fh:
            text = fh.read()
        want = re.search(r"source_sha256_16:\s*([0-9a-f]+)", text).group(1)
        val = float(re.search(r"traffic_bytes_per_launch:\s*([0-9.]+)", text).group(1))
        have = kernel_source_hash(kernel)
    except (OSError, AttributeError, ValueError, KeyError):
        return None
    return val if have == want else None


def harmonic(xs):
    xs = [x for x in xs if x > 0]
    return len(xs) / sum(1.0 / x for x in xs) if xs else 0.0


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else 0.0


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 0
    return model, nproc


def cpu_baseline(g, roots, budget_s: float):
    """The oracle (serial FIFO BFS in C, one thread) on the first roots of the
    timed list until the budget is spent, each timed alone."""
    import oracle

    rates, used = [], []
    t_all = time.perf_counter()
    for r in roots:
        t0 = time.perf_counter()
        _, lv = oracle.bfs_graph(g, int(r))
        dt = time.perf_counter() - t0
        m = oracle.reached_edges(g, lv)
        rates.append(m / dt / 1e9)
        used.append(int(r))
        if time.perf_counter() - t_all > budget_s:
            break
    model, nproc = host_cpu()
    return {
        "value": round(harmonic(rates), 6),
        "unit": "GTEPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"serial FIFO BFS (gcc -O2, one thread) from the first {len(used)} of the "
                  f"timed roots in the large component, on the same graph, each timed alone; "
                  f"harmonic mean",
        "cpu_model": model,
        "nproc": nproc,
    }


# ------------------------------------------------------------------ BFS leg
def kernel_split(stats, levels, n: int, n_active: int):
    """Per-kernel launches, device time and algorithmic bytes over a profiled
    pass (one stats record and one per-level record per search)."""
    nwords = (n + 31) // 32
    kb = {k: 0.0 for k in KERNELS}
    kms = {k: 0.0 for k in KERNELS}
    launches = 0
    for st, lv in zip(stats, levels):
        kb["k_expand_mark"] += mark_expand_bytes(lv) + pull_bytes(lv, n_active)
        kms["k_expand_mark"] += st.mark_ms + st.pull_ms
        kb["k_expand"] += claim_bytes(lv, nwords)
        kms["k_expand"] += st.expand_ms - st.mark_ms - st.pull_ms
        kb["k_finish"] += finish_bytes(lv, nwords, n_active)
        kms["k_finish"] += st.finish_ms
        kb["k_small_levels"] += small_levels_bytes(lv)
        kms["k_small_levels"] += st.small_ms
        launches += st.expand_launches   # one launch of each kernel per launch group
    out = {}
    for k in KERNELS:
        out[k] = {"launches": launches,
                  "device_ms": round(kms[k], 4),
                  "avg_launch_us": round(kms[k] / max(launches, 1) * 1e3, 3),
                  "bytes_per_launch": round(kb[k] / max(launches, 1), 1),
                  "achieved_gbs": round(kb[k] / (kms[k] * 1e-3) / 1e9, 2) if kms[k] > 0 else 0.0}
    return out


def bfs_workload(name, args, torch, graphgen, B, np, cpu: bool, steps: int, warmup: int):
    t0 = time.time()
    log(f"{name}: generating")
    g = graphgen.config_graph(name)
    roots = [int(r) for r in graphgen.config_roots(name, g)]
    log(f"{name}: n={g.n} nnz={g.nnz} in {time.time() - t0:.1f}s; {len(roots)} roots")
    t1 = time.time()
    G = B.Graph.from_csr(g.n, g.off, g.col, trusted=True, symmetric=True)
    log(f"{name}: resident on device in {time.time() - t1:.1f}s")
    t_tune = time.time()
    if args.options:
        # fixed options (e.g. those a tuned run reported), no timing sweep
        G.set_options(**{k: int(v) for k, v in
                         (kv.split("=") for kv in args.options.split(",") if kv)})
    else:
        G.tune(args.tune_cache)   # launch shapes and level floors, measured here (untimed)
    opt = G.get_options()
    tuned = {"grid_blocks": opt.grid_blocks, "batch_levels": opt.batch_levels,
             "claim_min_frontier": opt.claim_min_frontier, "pull_alpha": opt.pull_alpha,
             "claim_threshold": opt.claim_threshold, "small_frontier": opt.small_frontier}
    log(f"{name}: tuned in {time.time() - t_tune:.1f}s: {tuned}")
    G.set_options(profile=-1)
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    level = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for _ in range(warmup):
        for r in roots:
            G.run(r, parent, level)
    torch.cuda.synchronize()

    # timed passes: profiling off, one event pair around every search
    nr = len(roots)
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(nr)] for _ in range(steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(steps):
        for i, r in enumerate(roots):
            ev[s][i][0].record()
            G.run(r, parent, level)
            ev[s][i][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms = [[ev[s][i][0].elapsed_time(ev[s][i][1]) for i in range(nr)] for s in range(steps)]

    # one profiled pass over the same roots: per-root statistics, per-level
    # records and per-launch event times (the searches are deterministic, so
    # their records are those of the timed passes)
    G.set_options(profile=1)
    stats, levels = [], []
    for r in roots:
        G.run(r, parent, level)
        stats.append(G.last_stats())
        levels.append(G.level_info())
    G.set_options(profile=-1)
    torch.cuda.synchronize()
    kinds = {0: "claim", 1: "push", 2: "pull", 3: "claim-touch", 4: "loop"}
    for L in levels[0]:
        log(f"{name} root {roots[0]} level {L['level']:3d} {kinds.get(L['mark'], '?'):11s} "
            f"F={L['frontier']:>9d} T={L['edges']:>11d} searched={L['pull_candidates']:>9d} "
            f"examined={L['pull_edges']:>10d} expand={L['expand_ms'] * 1e3:8.1f}us "
            f"(mark kernel {(L['mark_ms'] + L['pull_ms']) * 1e3:8.1f}us) "
            f"finish={L['finish_ms'] * 1e3:7.1f}us loop={L['small_ms'] * 1e3:7.1f}us")

    deg = np.diff(np.asarray(g.off))
    # the pull scans the vertices of positive degree of the degree-ordered copy
    # (graphs of 2^20 vertices and more), else all vertices
    n_active = int((deg > 0).sum()) if g.n >= (1 << 20) else g.n
    giant_size = max(st.reached for st in stats)
    giant = [i for i, st in enumerate(stats) if st.reached == giant_size]
    per_root, frac_push, frac_exam, pass_vals = [], [], [], []
    for s in range(steps):
        vals = []
        for i in giant:
            st = stats[i]
            t = ms[s][i] * 1e-3
            vals.append(st.edges_traversed // 2 / t / 1e9)
            frac_push.append(bfs_bytes(g.n, st.edges_traversed, st.reached) / t / 1e9
                             / HBM_PEAK_GBS)
            frac_exam.append(examined_bytes(levels[i], g.n, n_active) / t / 1e9 / HBM_PEAK_GBS)
        per_root += vals
        pass_vals.append(round(harmonic(vals), 3))
    value = harmonic(per_root)
    split = kernel_split(stats, levels, g.n, n_active)
    kern = max(split, key=lambda k: split[k]["device_ms"])
    kd = split[kern]
    for k in KERNELS:
        split[k]["traffic"] = profiled_traffic(k, name)
    all_ms = [x for row in ms for x in row]
    log(f"{name}: {steps} passes x {nr} roots in {wall:.3f}s wall; {value:.2f} GTEPS; "
        f"p50 {pct(all_ms, 50):.3f} ms; dominant {kern} avg {kd['avg_launch_us']:.1f} us; "
        + ", ".join(f"{k} {split[k]['device_ms']:.2f} ms" for k in KERNELS))
    res = {
        "gteps": value,
        "ms_per_pass": wall * 1e3 / max(steps, 1),
        "pass_gteps": pass_vals,
        "config": {
            "workload": name,
            "n": g.n,
            "adjacencies": g.nnz,
            "edgefactor": 16,
            "roots": nr,
            "roots_in_large_component": len(giant),
            "roots_outside": nr - len(giant),
            "graph_hash": hex(g.hash()),
            "tuned_options": tuned,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kern,
            "achieved": kd["achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(kd["achieved_gbs"] / HBM_PEAK_GBS, 4),
            "traffic": split[kern]["traffic"],
            "launches": kd["launches"],
            "avg_launch_us": kd["avg_launch_us"],
            "bytes_per_launch": kd["bytes_per_launch"],
            "timing": "HIP events around every launch, one profiled pass over the same roots",
        },
        "level_kernels": split,
        "bfs_roofline_frac": round(harmonic(frac_push), 4),
        "bfs_examined_frac": round(harmonic(frac_exam), 4),
        "ms_per_bfs_p50": round(pct(all_ms, 50), 4),
        "us_per_bfs_p50": round(pct(all_ms, 50) * 1e3, 1),
        "levels_p50": int(pct([st.levels for st in stats], 50)),
        "pull_levels_p50": int(pct([st.pull_levels for st in stats], 50)),
    }
    cb = None
    if cpu:
        log(f"{name}: cpu baseline")
        cb = cpu_baseline(g, [roots[i] for i in giant], args.cpu_budget)
    if args.upper_storage and name == args.workload:
        res["upper_storage"] = upper_storage(g, G, roots, giant, value, all_ms, torch, graphgen,
                                             B, np, min(steps, 3))
    G.destroy()
    del g
    return res, cb


def upper_storage(g, G, roots, giant, gteps_full, ms_full, torch, graphgen, B, np, steps):
    """The same searches on symmetric storage (each undirected edge once, in
    the row of its smaller endpoint): device bytes and time against the full
    CSR, and the outputs of a few roots compared with the full CSR's."""
    t0 = time.time()
    u = graphgen.upper_csr(g)
    log(f"{g.name}: upper-triangle copy ({u.nnz} adjacencies) in {time.time() - t0:.1f}s")
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    level = torch.empty(g.n, dtype=torch.int32, device="cuda")
    ref = []
    for r in roots[:2]:
        G.run(r, parent, level)
        ref.append((parent.clone(), level.clone()))
    full_bytes = G.info()[2]
    G.destroy()   # freed first: the two copies never share the device
    Gu = B.Graph.from_csr(u.n, u.off, u.col, trusted=True, upper=True)
    Gu.tune()
    Gu.set_options(profile=-1)
    same = True
    for (rp, rl), r in zip(ref, roots[:2]):
        Gu.run(r, parent, level)
        same &= bool(torch.equal(parent, rp)) and bool(torch.equal(level, rl))
    del ref
    for r in roots:   # warm-up pass
        Gu.run(r, parent, level)
    nr = len(roots)
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(nr)] for _ in range(steps)]
    torch.cuda.synchronize()
    for s in range(steps):
        for i, r in enumerate(roots):
            ev[s][i][0].record()
            Gu.run(r, parent, level)
            ev[s][i][1].record()
    torch.cuda.synchronize()
    ms = [[ev[s][i][0].elapsed_time(ev[s][i][1]) for i in range(nr)] for s in range(steps)]
    Gu.run(roots[giant[0]], parent, level)
    edges = Gu.last_stats().edges_traversed
    vals = [edges // 2 / (ms[s][i] * 1e-3) / 1e9 for s in range(steps) for i in giant]
    up_bytes = Gu.info()[2]
    Gu.destroy()
    gteps = harmonic(vals)
    all_ms = [x for row in ms for x in row]
    log(f"{g.name}: upper-triangle storage {up_bytes / 1e9:.2f} GB on device "
        f"(full CSR {full_bytes / 1e9:.2f} GB), {gteps:.2f} GTEPS (full {gteps_full:.2f}), "
        f"p50 {pct(all_ms, 50):.3f} ms, outputs equal to the full CSR's: {same}")
    return {"adjacencies_stored": int(u.nnz), "adjacencies_full": int(g.nnz),
            "device_bytes_upper": int(up_bytes), "device_bytes_full": int(full_bytes),
            "gteps_upper": round(gteps, 3), "gteps_full": round(gteps_full, 3),
            "ms_per_bfs_p50_upper": round(pct(all_ms, 50), 4),
            "ms_per_bfs_p50_full": round(pct(ms_full, 50), 4),
            "passes": steps, "outputs_equal_full_csr": same}


def bfs_floor(torch, graphgen, B, np):
    """The fixed cost of one search: BFS on a single edge (2 vertices), with
    the default options, timed like the workloads (an event pair around each
    call)."""
    g = graphgen.from_edges(2, [(0, 1)])
    G = B.Graph.from_csr(g.n, g.off, g.col, trusted=True, symmetric=True)
    G.set_options(profile=-1)
    parent = torch.empty(2, dtype=torch.int32, device="cuda")
    level = torch.empty(2, dtype=torch.int32, device="cuda")
    ms = []
    for rep in range(41):
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        G.run(rep & 1, parent, level)
        e.record()
        torch.cuda.synchronize()
        if rep:
            ms.append(s.elapsed_time(e))
    opt = G.get_options()
    G.destroy()
    us = pct(ms, 50) * 1e3
    log(f"bfs floor (one edge): p50 {us:.1f} us per search")
    return {"graph": "one edge, 2 vertices", "us_per_bfs_p50": round(us, 1),
            "batch_levels": opt.batch_levels}


# ------------------------------------------------------------------ SpMSpV leg
def spmspv_leg(args, torch, graphgen, B, np):
    t0 = time.time()
    blk = graphgen.dcsc_block(26, 1 << 24, 4)
    log(f"share 2^26 x 2^26: nnz={blk.nnz} nzc={blk.nzc} in {time.time() - t0:.1f}s")
    Gb = B.Graph.from_dcsc(blk.nrows, blk.ncols, blk.jc, blk.cp, blk.ir, trusted=True)
    Gb.tune(args.tune_cache)   # the polyalgorithm's switch (sort path vs binned), measured here
    sort_max = Gb.get_options().spmspv_sort_max
    log(f"spmspv sort path for frontiers up to {sort_max} entries")
    cap = blk.nnz
    oi = torch.empty(cap, dtype=torch.int32, device="cuda")
    ov = torch.empty(cap, dtype=torch.int32, device="cuda")
    colnnz = np.diff(blk.cp).astype(np.int64)

    def timed(fd, k):
        torch.cuda.synchronize()
        s, t = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        cnt = Gb.spmspv(fd, k, oi, ov, cap)
        t.record()
        torch.cuda.synchronize()
        return cnt, s.elapsed_time(t) * 1e3

    # the floor: a call with an empty frontier (the call's launches and its
    # read-back of the output count)
    floor = []
    for rep in range(21):
        _, us = timed(None, 0)
        if rep:
            floor.append(us)
    out = {"empty_call_p50_us": round(pct(floor, 50), 2)}
    call = 0
    samples = {}
    for density in [float(x) for x in args.spmspv_densities.split(",")]:
        k = int(density * (1 << 26))
        # the density's 51 frontiers and their algorithmic bytes, prepared and
        # uploaded first, so the calls run back to back like a 2D search's
        # levels (the first one is a warm-up)
        fds, algo, edges = [], [], []
        for rep in range(51):
            f = graphgen.frontier_sample(26, k, 1003 + call)
            call += 1
            pos = np.searchsorted(blk.jc, f)
            pos_c = np.minimum(pos, blk.nzc - 1)
            hit = (pos < blk.nzc) & (blk.jc[pos_c] == f)
            e = int(colnnz[pos_c[hit]].sum())
            fds.append(torch.from_numpy(f).cuda())
            algo.append((8.0 * k + 8.0 * int(hit.sum()) + 4.0 * e, e))
            if rep == 0:
                samples[density] = f
        torch.cuda.synchronize()
        times, bytes_, edges_s = [], [], []
        for rep in range(51):
            cnt, us = timed(fds[rep], k)
            if rep == 0:
                continue
            times.append(us)
            bytes_.append(algo[rep][0] + 8.0 * cnt)
            edges_s.append(algo[rep][1] / (us * 1e-6))
        del fds
        p50 = pct(times, 50)
        frac = (float(np.median(bytes_)) / (p50 * 1e-6) / 1e9) / HBM_PEAK_GBS
        out[f"{density * 100:g}%"] = {
            "frontier": k,
            "p50_us": round(p50, 2),
            "p99_us": round(pct(times, 99), 2),
            "edges_per_s": round(float(np.median(edges_s)), 1),
            "bytes_per_call": round(float(np.median(bytes_)), 1),
            "roofline_frac": round(frac, 4) if density >= 0.01 else None,
        }
        log(f"spmspv {density * 100:g}%: p50 {p50:.1f} us")
    out["sort_path_max_frontier"] = sort_max
    if not args.no_cpu:
        # the oracle's product on the first (warm-up) frontier of each density,
        # timed alone on one host thread
        import oracle
        cpu = {}
        for density, f in samples.items():
            t1 = time.perf_counter()
            oracle.spmspv_block(blk, f)
            cpu[f"{density * 100:g}%"] = round((time.perf_counter() - t1) * 1e6, 1)
        model, nproc = host_cpu()
        out["cpu_baseline"] = {"us_per_call": cpu, "unit": "us", "cores": 1, "kind": "oracle",
                               "sample": "one call per density (serial C), timed alone",
                               "cpu_model": model, "nproc": nproc}
    Gb.destroy()
    return out


# ------------------------------------------------------------------ mix leg
def mix_leg(torch, graphgen, B, np, nq: int):
    t0 = time.time()
    specs = [("rmat14", lambda: graphgen.rmat_csr(14, 16, 5)),
             ("rmat16", lambda: graphgen.rmat_csr(16, 16, 5)),
             ("rmat18", lambda: graphgen.rmat_csr(18, 16, 5)),
             ("rmat20", lambda: graphgen.rmat_csr(20, 16, 5)),
             ("rmat22", lambda: graphgen.rmat_csr(22, 16, 5)),
             ("grid512", lambda: graphgen.grid_csr(512)),
             ("grid2048", lambda: graphgen.grid_csr(2048))]
    graphs, devs, cand = [], [], []
    for name, mk in specs:
        g = mk()
        g.name = name
        graphs.append(g)
        devs.append(B.Graph.from_csr(g.n, g.off, g.col, trusted=True, symmetric=True))
        cand.append(np.nonzero(np.diff(g.off) > 0)[0].astype(np.int32))
    log(f"mix graphs ready in {time.time() - t0:.1f}s")
    rng = np.random.default_rng(1004)
    qg = rng.integers(0, len(graphs), nq)
    qr = np.array([cand[i][rng.integers(0, cand[i].size)] for i in qg], np.int32)
    # a seeded sample of every graph's queries, compared with the plain path
    # after every leg
    check = []
    for gi in range(len(graphs)):
        idx = np.nonzero(qg == gi)[0]
        check += [int(i) for i in idx[:3]]

    # plain path, one query at a time (closed loop)
    bufs = [(torch.empty(g.n, dtype=torch.int32, device="cuda"),
             torch.empty(g.n, dtype=torch.int32, device="cuda")) for g in graphs]
    for i in range(min(14, nq)):
        devs[qg[i]].run(int(qr[i]), *bufs[qg[i]])
    torch.cuda.synchronize()
    edges = np.zeros(nq, np.int64)
    per_class = np.zeros(len(graphs))
    t1 = time.perf_counter()
    for i in range(nq):
        G = devs[qg[i]]
        tq = time.perf_counter()
        G.run(int(qr[i]), *bufs[qg[i]])
        edges[i] = G.last_stats().edges_traversed // 2
        per_class[qg[i]] += time.perf_counter() - tq
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t1
    m_total = float(edges.sum())
    plain = {"gteps": round(m_total / plain_s / 1e9, 4), "seconds": round(plain_s, 4),
             "qps": round(nq / plain_s, 2),
             "seconds_by_graph": {specs[i][0]: round(float(per_class[i]), 4)
                                  for i in range(len(graphs))}}
    log(f"plain: {plain}")
    del bufs
    ref = {}
    for i in check:
        p = torch.empty(graphs[qg[i]].n, dtype=torch.int32, device="cuda")
        lv = torch.empty_like(p)
        devs[qg[i]].run(int(qr[i]), p, lv)
        ref[i] = (p, lv)
    torch.cuda.synchronize()

    def agree(outs):
        return all(bool(torch.equal(ref[i][0], outs[i][0]) and torch.equal(ref[i][1], outs[i][1]))
                   for i in check)

    outs = [(torch.empty(graphs[i].n, dtype=torch.int32, device="cuda"),
             torch.empty(graphs[i].n, dtype=torch.int32, device="cuda")) for i in qg]
    B.run_batch([devs[i] for i in qg[:32]], qr[:32], [o[0] for o in outs[:32]],
                [o[1] for o in outs[:32]])
    torch.cuda.synchronize()
    for o in outs:
        o[0].fill_(-7)
    t1 = time.perf_counter()
    B.run_batch([devs[i] for i in qg], qr, [o[0] for o in outs], [o[1] for o in outs])
    torch.cuda.synchronize()
    batch_s = time.perf_counter() - t1
    batched = {"gteps": round(m_total / batch_s / 1e9, 4), "seconds": round(batch_s, 4),
               "speedup_vs_plain": round(plain_s / batch_s, 2), "sample_equal": agree(outs)}
    # each graph class alone: its queries in one batch against the same
    # queries one at a time on the plain path
    by_graph = {}
    for gi, (name, _) in enumerate(specs):
        idx = [int(i) for i in np.nonzero(qg == gi)[0]]
        if not idx:
            continue
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        B.run_batch([devs[gi]] * len(idx), qr[idx], [outs[i][0] for i in idx],
                    [outs[i][1] for i in idx])
        torch.cuda.synchronize()
        bs = time.perf_counter() - t1
        ps = float(per_class[gi])
        by_graph[name] = {"queries": len(idx), "plain_s": round(ps, 4), "batched_s": round(bs, 4),
                          "batched_vs_plain": round(ps / bs, 2) if bs > 0 else None}
    batched["by_graph"] = by_graph
    batched["sample_equal_by_graph"] = agree(outs)
    log(f"batched: {batched}")

    served = {}
    cap_qps = nq / plain_s
    for factor in (0.5, 4.0, 16.0):
        for o in outs:
            o[0].fill_(-7)
        qps = factor * cap_qps
        arrivals = graphgen.poisson_arrivals(nq, qps, 2000 + int(factor * 10))
        S = B.Server(slots=512)
        tickets = []
        t_base = time.perf_counter()
        for i in range(nq):
            while time.perf_counter() - t_base < arrivals[i]:
                pass
            tickets.append(S.submit(devs[qg[i]], int(qr[i]), outs[i][0], outs[i][1]))
        S.drain()
        res = [S.poll(t) for t in tickets]
        S.destroy()
        torch.cuda.synchronize()
        lat = [(r.t_done - r.t_arrive) * 1e3 for r in res]
        span = max(r.t_done for r in res) - min(r.t_arrive for r in res)
        m_served = float(sum(r.edges_traversed for r in res)) / 2
        served[f"{factor:g}x"] = {
            "qps": round(qps, 2),
            "gteps": round(m_served / span / 1e9, 4),
            "vs_plain": round(m_served / span / 1e9 / max(plain["gteps"], 1e-9), 2),
            "p50_ms": round(pct(lat, 50), 3),
            "p99_ms": round(pct(lat, 99), 3),
            "span_s": round(span, 3),
            "sample_equal": agree(outs),
        }
        log(f"served {factor}x: {served[f'{factor:g}x']}")
    del outs, devs, ref
    return {"queries": nq, "graphs": [s[0] for s in specs], "plain": plain,
            "batched": batched, "served": served, "checked_queries": len(check)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3,
                    help="timed passes over the workload's roots")
    ap.add_argument("--warmup", type=int, default=1, help="untimed passes before them")
    ap.add_argument("--workload", default="rmat26",
                    choices=["rmat12", "rmat22", "rmat26", "er26"])
    ap.add_argument("--extra", default="er26,rmat22,rmat12",
                    help="comma list of further BFS workloads reported under 'workloads'")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune-cache", default=None,
                    help="text file the tuning is read from / appended to, so profiled "
                         "runs reuse an earlier run's choice without timing sweeps")
    ap.add_argument("--legs", default="bfs,spmspv,mix",
                    help="comma list of legs to run: bfs, spmspv, mix")
    ap.add_argument("--mix-queries", type=int, default=1024)
    ap.add_argument("--options", default="",
                    help="comma list name=value of graph options to set instead of tuning "
                         "(e.g. the tuned_options of an earlier line), for profiled runs")
    ap.add_argument("--spmspv-densities", default="0.0001,0.001,0.01,0.1",
                    help="frontier densities of the SpMSpV leg")
    ap.add_argument("--no-floor", dest="floor", action="store_false",
                    help="skip the one-edge search that measures a search's fixed cost")
    ap.add_argument("--no-upper-storage", dest="upper_storage", action="store_false",
                    help="skip the headline graph's run on symmetric (upper-triangle) storage")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (3 times), to scale HBM counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              f"1D/2D designs are not built. Exiting.", file=sys.stderr, flush=True)
        return 2

    if args.copy_calibration:
        import torch
        x = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 1 << 30, "bytes_written": 1 << 30,
                          "repeats": 3}), flush=True)
        return 0

    import numpy as np
    import torch

    import graphgen
    from paper_1104_4518_amd import bfs as B

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    legs = set(args.legs.split(","))
    steps, warmup = max(args.steps, 1), max(args.warmup, 0)

    out = {"metric": METRIC, "value": None, "unit": "GTEPS", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic (seeded R-MAT / Erdos-Renyi / grids / uniform DCSC share)"}
    if "bfs" in legs:
        res, cpu = bfs_workload(args.workload, args, torch, graphgen, B, np,
                                cpu=not args.no_cpu, steps=steps, warmup=warmup)
        out["value"] = round(res["gteps"], 4)
        out["ms_per_step"] = round(res["ms_per_pass"], 4)
        out["config"] = res.pop("config")
        out["config"]["step"] = "one pass over all roots, one BFS each"
        for k in ("roofline", "level_kernels", "bfs_roofline_frac", "bfs_examined_frac",
                  "ms_per_bfs_p50", "pass_gteps", "levels_p50", "pull_levels_p50"):
            out[k] = res[k]
        if "upper_storage" in res:
            out["upper_storage"] = res["upper_storage"]
        if cpu is not None:
            out["cpu_baseline"] = cpu
        extra = {}
        for name in [w for w in args.extra.split(",") if w and w != args.workload]:
            r2, _ = bfs_workload(name, args, torch, graphgen, B, np, cpu=False, steps=steps,
                                 warmup=warmup)
            cfg = r2.pop("config")
            extra[name] = {"gteps": round(r2["gteps"], 4), "ms_per_pass": round(r2["ms_per_pass"], 4),
                           "ms_per_bfs_p50": r2["ms_per_bfs_p50"],
                           "us_per_bfs_p50": r2["us_per_bfs_p50"],
                           "bfs_roofline_frac": r2["bfs_roofline_frac"],
                           "bfs_examined_frac": r2["bfs_examined_frac"],
                           "roofline": r2["roofline"], "level_kernels": r2["level_kernels"],
                           "pass_gteps": r2["pass_gteps"], "config": cfg}
        out["workloads"] = extra
        if args.floor:
            out["bfs_floor"] = bfs_floor(torch, graphgen, B, np)
    if "spmspv" in legs:
        out["spmspv"] = spmspv_leg(args, torch, graphgen, B, np)
    if "mix" in legs:
        out["mix"] = mix_leg(torch, graphgen, B, np, args.mix_queries)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
