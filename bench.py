#!/usr/bin/env python
"""One-GPU throughput of the geometric-search hot path on MI355X.

A step is one pass of the whole path over one synthetic batch: BVH build over
N points, radius search with CSR output, the fused COUNT and COUNT_SUMDIST
reductions, and kNN (k = 16) for M queries.  Default workload: N = M = 10^7
float32 points uniform in the unit cube, radius for ~10 neighbours.

Prints ONE JSON line on stdout (progress goes to stderr):
  value      = queries answered per second over the timed steps, build included
               (4 query passes of M queries per step);
  components = per-phase rates from events recorded on the launch stream, and,
               timed after the steps and outside them, the early-terminating
               count, the radius search with per-match distances (callback
               with output), DBSCAN and the pair search on the step's tree,
               standalone reduce and kNN calls that order their queries, and
               rays against a tree of 2*10^6 boxes (hit counts, first hit, all
               hits, all hits in the order met);
  roofline   = the dominant kernel's algorithmic bytes / its average duration
               against MI355X HBM peak (8 TB/s), with the measured HBM traffic
               while profiles/traffic.json matches the kernel sources, and the
               measured device-copy rate;
  cpu_baseline = the CPU oracle on a bounded sample of the same queries;
  batched_vs_plain / chamfer = the forest and Chamfer workloads.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profile_collect(L):
    names = ctypes.create_string_buffer(32 * 64)
    ms = (ctypes.c_double * 64)()
    launches = (ctypes.c_int64 * 64)()
    cnt = ctypes.c_int32()
    st = L.arborx_profile_collect(names, ms, launches, 64, ctypes.byref(cnt))
    if st != 0:
        raise RuntimeError(L.arborx_last_error().decode())
    out = {}
    for i in range(cnt.value):
        nm = names.raw[32 * i:32 * (i + 1)].split(b"\0", 1)[0].decode()
        out[nm] = (ms[i], launches[i])
    return out


def algorithmic_bytes(kernel, n, m, dim, k, total):
    """Compulsory HBM bytes of one launch: inputs read once, outputs written once,
    the tree read once.  Tree bytes use the fixed accounting of a 16-byte point
    leaf plus a 32-byte internal node per value (48 N in 3D)."""
    tree = 48 * n if dim == 3 else (32 + 64) * n
    q = 4 * dim * m + 4 * m  # query coordinates + the Morton permutation
    return {
        "knn": q + tree + 8 * k * m,
        "spatial_count": q + tree + 4 * m,
        "spatial_fill": q + tree + 16 * m + 4 * total,
        "reduce_count": q + tree + 4 * m,
        "reduce_sumdist": q + tree + 12 * m,
        "build_hierarchy": (8 + 4 + 4 * dim) * n + 64 * max(n - 1, 1) + 8 * n,
    }.get(kernel)


def source_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2507_23700_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_2507_23700_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled(kernel, workload, field):
    """A per-launch figure from committed rocprofv3 counter runs, if they match this source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(workload, {}).get(kernel)
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get(field)


def traffic_for(kernel, workload):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)."""
    return profiled(kernel, workload, "bytes_per_launch")


KERNEL_PHASE = [  # rocprofv3 kernel name pattern -> phase name used by the in-library profiler
    (r"k_spatial_count(_packet)?<\d+, ax::RayPred", "ray_all_hits"), (r"k_spatial_count(_packet)?<", "spatial_count"),
    (r"k_spatial_reduce(_packet)?<\d+, false", "reduce_count"), (r"k_spatial_reduce(_packet)?<\d+, true", "reduce_sumdist"),
    (r"k_valu_probe", "valu_probe"), (r"k_knn<", "knn"), (r"k_spatial_fill_rows<", "spatial_fill"),
    (r"hierarchy_(chunk|top)_kernel<", "build_hierarchy"), (r"k_copy_stash", "copy_stash"),
    (r"k_copy_overflow", "copy_overflow"), (r"k_sort_rows", "sort_rows"), (r"k_count_up_to", "count_up_to"),
    (r"k_match_distances", "match_distances"), (r"k_pair_degree", "pair_degree"), (r"k_dbscan_", "dbscan"),
    (r"k_ray_count", "ray_count"), (r"k_ray_nearest", "ray_nearest"), (r"radix_scatter<", "radix_scatter"),
    (r"radix_hist<", "radix_hist"), (r"k_query_codes<", "order"), (r"morton_kernel<", "build_morton"),
    (r"k_forest_reduce", "forest_reduce"), (r"k_forest_knn", "forest_knn"), (r"k_chamfer|k_pair_loss", "chamfer"),
]


def summarize_counters(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, stats_csv, workload, copy_bytes,
                       sq_csv=None, sq_probe_csv=None):
    """Per-phase HBM bytes per launch from rocprofv3 --pmc runs, scaled by what the same
    counters read for a plain device copy of copy_bytes bytes; with sq_csv and sq_probe_csv
    (SQ_INSTS_VALU and SQ_BUSY_CYCLES of the kernels and of the library's VALU issue probe),
    each kernel's VALU instructions per busy cycle as a fraction of the probe's, the issue
    rate independent FMA chains reach.  Writes profiles/traffic.json and returns a markdown
    table."""
    import collections
    import csv

    import re

    def phase(name):
        nm = name.replace("(anonymous namespace)::", "")
        for pat, ph in KERNEL_PHASE:
            if re.search(pat, nm):
                return ph
        return None

    def per_dispatch(path, counter):
        out = collections.defaultdict(float)
        launches = collections.defaultdict(set)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            ph = phase(r["Kernel_Name"]) or r["Kernel_Name"]
            out[ph] += float(r["Counter_Value"]) * 1024.0
            launches[ph].add(r["Dispatch_Id"])
        return out, launches

    cf, _ = per_dispatch(copy_fetch_csv, "FETCH_SIZE")
    cw, _ = per_dispatch(copy_write_csv, "WRITE_SIZE")
    fscale = 3 * copy_bytes / cf["__amd_rocclr_copyBuffer"]
    wscale = 3 * copy_bytes / cw["__amd_rocclr_copyBuffer"]
    fetch, fl = per_dispatch(fetch_csv, "FETCH_SIZE")
    write, wl = per_dispatch(write_csv, "WRITE_SIZE")
    hit, _ = per_dispatch(write_csv, "TCC_HIT_sum")
    miss, _ = per_dispatch(write_csv, "TCC_MISS_sum")
    valu, busy, peak = {}, {}, None
    if sq_csv and sq_probe_csv:
        valu, _ = per_dispatch(sq_csv, "SQ_INSTS_VALU")
        busy, _ = per_dispatch(sq_csv, "SQ_BUSY_CYCLES")
        pv, _ = per_dispatch(sq_probe_csv, "SQ_INSTS_VALU")
        pb, _ = per_dispatch(sq_probe_csv, "SQ_BUSY_CYCLES")
        peak = pv["valu_probe"] / pb["valu_probe"]
    dur = collections.defaultdict(list)
    for r in csv.DictReader(open(stats_csv)):
        ph = phase(r["Name"])
        if ph:
            dur[ph].append((float(r["AverageNs"]), int(r["Calls"])))
    src = source_hash()
    table = {}
    lines = [f"| phase | launches | avg ms (kernel trace) | HBM read MB/launch | HBM write MB/launch | L2 hit |"
             f" VALU busy |", "|---|---|---|---|---|---|---|"]
    for ph in sorted(fetch, key=lambda k: -fetch[k]):
        if ph not in {p for _, p in KERNEL_PHASE}:
            continue
        nl = max(len(fl[ph]), 1)
        rd = fetch[ph] * fscale / nl
        wr = write.get(ph, 0.0) * wscale / max(len(wl.get(ph, ())), 1)
        h = hit.get(ph, 0.0) / max(hit.get(ph, 0.0) + miss.get(ph, 0.0), 1e-9)
        ms = sum(a * c for a, c in dur[ph]) / max(sum(c for _, c in dur[ph]), 1) / 1e6 if dur[ph] else float("nan")
        vb = valu[ph] / busy[ph] / peak if peak and busy.get(ph) else None  # sums over the phase's launches
        table[ph] = {"bytes_per_launch": rd + wr, "read_bytes": rd, "write_bytes": wr, "l2_hit": h,
                     "valu_busy": vb, "source_hash": src}
        lines.append(f"| {ph} | {nl} | {ms:.3f} | {rd / 1e6:.1f} | {wr / 1e6:.1f} | {h:.3f} | "
                     f"{'%.2f' % vb if vb is not None else '-'} |")
    path = os.path.join(ROOT, "profiles", "traffic.json")
    allw = json.load(open(path)) if os.path.exists(path) else {}
    allw[workload] = table
    allw["_calibration"] = {"fetch_scale": fscale, "write_scale": wscale, "copy_bytes": copy_bytes}
    with open(path, "w") as f:
        json.dump(allw, f, indent=1, sort_keys=True)
    lines.append("")
    lines.append(f"Counter scale from a {copy_bytes / 2 ** 30:.0f} GiB device copy: FETCH_SIZE x {fscale:.3f}, "
                 f"WRITE_SIZE x {wscale:.3f}.  Kernel sources hash {src}.")
    if peak:
        lines.append(f"VALU issue probe: {peak:.2f} VALU instructions per SQ busy cycle (the busy column's 1.0).")
    return "\n".join(lines)


def cpu_baseline(data, queries, radius, k, target_s=15.0, max_sample=20000):
    import numpy as np

    import oracle
    oracle.lib()

    dim = data.shape[1]

    def run(sq):
        t0 = time.perf_counter()
        off, idx = oracle.spatial(data, sq, radius, dim=dim)
        c, _ = oracle.reduce(data, sq, radius, dim=dim, op=oracle.COUNT)
        c2, s2 = oracle.reduce(data, sq, radius, dim=dim, op=oracle.COUNT_SUMDIST)
        d2, ix = oracle.knn(data, sq, k, dim=dim)
        return time.perf_counter() - t0, (off, idx, c, c2, s2, d2, ix)

    g = np.random.default_rng(12345)
    run(queries[g.choice(len(queries), 16, replace=False)])  # thread pool and page warm-up, not timed
    probe = 256
    dt, _ = run(queries[g.choice(len(queries), probe, replace=False)])
    s = int(min(max_sample, max(probe, probe * target_s / max(dt, 1e-6))))
    sel = np.sort(g.choice(len(queries), s, replace=False))
    dt, res = run(queries[sel])
    return dict(value=4 * s / dt, unit="queries/s", cores=oracle.threads(), kind="oracle", **host_cpu(),
                sample=f"{s} seeded queries of the same workload (CSR radius, COUNT, COUNT_SUMDIST, kNN k={k}) "
                       f"against all {len(data)} points; {dt:.1f} s"), sel, res


def host_cpu():
    """Model name and vector extensions of the host CPU the oracle ran on."""
    model, flags = "unknown", set()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model == "unknown":
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("flags") and not flags:
                    flags = set(line.split(":", 1)[1].split())
    except OSError:
        pass
    simd = [x for x in ("sse4_2", "avx", "avx2", "fma", "avx512f", "avx512bw", "avx512vl", "avx512_bf16")
            if x in flags]
    return {"cpu_model": model, "simd": " ".join(simd), "host_threads": os.cpu_count()}


def timed(fn, reps=3):
    """Median milliseconds of fn() between two device synchronisations."""
    import torch
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(1000.0 * (time.perf_counter() - t0))
    return sorted(ts)[len(ts) // 2]


def forest_bench(reps=3):
    """Batched forest path vs the per-tree loop on the same inputs, with identical outputs."""
    import torch

    import paper_2507_23700_amd as ax
    from paper_2507_23700_amd import inputs

    log("generating forest workload (64 trees, 4096 batches)")
    cfg = inputs.forest()
    k = cfg["k"]
    toff, boff, bt, br = cfg["tree_offsets"], cfg["batch_offsets"], cfg["batch_tree"], cfg["batch_radius"]
    v = torch.from_numpy(cfg["values"]).cuda()
    q = torch.from_numpy(cfg["queries"]).cuda()
    dbo, dbt, dbr = (torch.from_numpy(x).cuda() for x in (boff, bt, br))
    m = q.shape[0]
    out = {}

    def batched():
        f = ax.arborx_forest_build(v, toff)
        c, s = ax.arborx_forest_query_reduce(f, q, dbo, dbt, dbr, ax.COUNT_SUMDIST)
        d2, ix = ax.arborx_forest_query_knn(f, q, dbo, dbt, k)
        out["batched"] = (c, s, d2, ix)

    tree_views = [v[toff[t]:toff[t + 1]] for t in range(len(toff) - 1)]
    q_views = [q[boff[b]:boff[b + 1]] for b in range(len(bt))]

    def plain():
        trees = [ax.arborx_bvh_build(tv) for tv in tree_views]
        c = torch.empty(m, dtype=torch.int32, device="cuda")
        s = torch.empty(m, dtype=torch.int64, device="cuda")
        d2 = torch.empty((m, k), dtype=torch.float32, device="cuda")
        ix = torch.empty((m, k), dtype=torch.int32, device="cuda")
        for b in range(len(bt)):
            sl = slice(int(boff[b]), int(boff[b + 1]))
            cb, sb = ax.arborx_query_spatial_reduce(trees[bt[b]], q_views[b], float(br[b]), ax.COUNT_SUMDIST)
            db, ib = ax.arborx_query_knn(trees[bt[b]], q_views[b], k)
            c[sl], s[sl], d2[sl], ix[sl] = cb, sb, db, ib
        out["plain"] = (c, s, d2, ix)

    batched()
    plain()
    t_b = timed(batched, reps)
    t_p = timed(plain, reps)
    same = all(torch.equal(a, b) for a, b in zip(out["batched"], out["plain"]))
    log(f"forest: batched {t_b:.1f} ms, per-tree loop {t_p:.1f} ms, identical={same}")
    # the same batched work captured once in a hipGraph: rebuild in place, reduce, kNN; nothing allocates
    fo = ax.arborx_forest_create(int(toff[-1]), len(toff) - 1, 3)
    off_d = torch.from_numpy(toff.astype("int64")).cuda()
    ax.arborx_forest_reserve(fo, m)
    torch.cuda.synchronize()
    gs = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(gs):
        with torch.cuda.graph(graph, stream=gs):
            ax.arborx_forest_rebuild(fo, v, off_d, stream=gs)
            gc_, gsum = ax.arborx_forest_query_reduce(fo, q, dbo, dbt, dbr, ax.COUNT_SUMDIST, stream=gs)
            gd2, gix = ax.arborx_forest_query_knn(fo, q, dbo, dbt, k, stream=gs)
    graph.replay()
    torch.cuda.synchronize()
    t_g = timed(graph.replay, reps)
    same_g = all(torch.equal(a, b) for a, b in zip((gc_, gsum, gd2, gix), out["batched"]))
    log(f"forest: one hipGraph replay {t_g:.1f} ms, identical={same_g}")
    res = {"workload": "forest_t64_b4096", "trees": len(toff) - 1, "points": int(toff[-1]), "batches": len(bt),
           "queries": int(m), "ops": f"build + COUNT_SUMDIST + kNN k={k}", "batched_ms": t_b, "plain_ms": t_p,
           "speedup": t_p / t_b, "identical": bool(same),
           "batched_queries_per_s": 2 * m / (t_b * 1e-3),
           "graph_ms": t_g, "graph_speedup": t_p / t_g, "graph_identical": bool(same_g)}
    del out, graph, gc_, gsum, gd2, gix, fo
    torch.cuda.empty_cache()
    return res


def chamfer_bench(reps=3):
    """Chamfer forward (forest build + kNN k=1 both ways + loss) and backward on 256 pairs."""
    import torch

    import paper_2507_23700_amd as ax
    from paper_2507_23700_amd import inputs

    log("generating Chamfer workload (256 pairs)")
    cfg = inputs.chamfer_pairs()
    a = torch.from_numpy(cfg["a"]).cuda()
    b = torch.from_numpy(cfg["b"]).cuda()
    ao, bo = cfg["a_off"], cfg["b_off"]
    P = len(ao) - 1
    g = torch.ones(P, dtype=torch.float32, device="cuda")
    st = {}

    def fwd():
        st["f"] = ax.arborx_chamfer_forward(a, ao, b, bo)

    def bwd():
        _, nab, nba = st["f"]
        ax.arborx_chamfer_backward(a, ao, b, bo, nab, nba, g)

    fwd()
    t_f = timed(fwd, reps)
    t_b = timed(bwd, reps)
    pts = int(ao[-1] + bo[-1])
    return {"workload": f"chamfer_p{P}", "pairs": P, "points": pts, "forward_ms": t_f, "backward_ms": t_b,
            "pairs_per_s": P / ((t_f + t_b) * 1e-3), "points_per_s": pts / ((t_f + t_b) * 1e-3)}


def copy_bandwidth(torch, gib=1.0, reps=5):
    """Measured device-to-device copy rate (bytes read + written per second, GB/s): the practical
    HBM ceiling the roofline fraction is also reported against."""
    n = int(gib * 2 ** 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="points (= queries); default per workload")
    ap.add_argument("--dist", default="cube", choices=["cube", "shell", "gmm6", "small"],
                    help="cube / shell: 10^7 3D points; gmm6: 2*10^6 6D Gaussian mixture; small: 2*10^4 3D cube")
    ap.add_argument("--k", type=int, default=None, help="kNN k; default per workload (16, 8 for gmm6, 10 for small)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-forest", action="store_true", help="skip the batched-vs-plain forest comparison")
    ap.add_argument("--no-chamfer", action="store_true", help="skip the Chamfer timing")
    ap.add_argument("--calibrate-copy", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device copy of GIB gibibytes (counter calibration) and exit")
    ap.add_argument("--calibrate-valu", action="store_true",
                    help="only run the library's VALU issue probe (counter calibration) and exit")
    ap.add_argument("--summarize-counters", nargs="+", metavar="CSV",
                    help="FETCH WRITE COPYFETCH COPYWRITE STATS [SQ SQPROBE]: turn rocprofv3 counter CSVs into "
                         "profiles/traffic.json and print a markdown table")
    args = ap.parse_args()
    if args.summarize_counters:
        n0 = args.n or {"gmm6": 2_000_000, "small": 20_000}.get(args.dist, 10_000_000)
        wl = f"gmm6d_n{n0}_m{n0}" if args.dist == "gmm6" else f"{'cube' if args.dist == 'small' else args.dist}3d_n{n0}_m{n0}"
        if len(args.summarize_counters) not in (5, 7):
            ap.error("--summarize-counters takes FETCH WRITE COPYFETCH COPYWRITE STATS [SQ SQPROBE]")
        csvs = args.summarize_counters
        print(summarize_counters(*csvs[:5], workload=wl, copy_bytes=2 ** 30,
                                 sq_csv=csvs[5] if len(csvs) == 7 else None,
                                 sq_probe_csv=csvs[6] if len(csvs) == 7 else None))
        return
    if args.calibrate_valu:
        import torch
        from paper_2507_23700_amd import _lib
        blocks, iters = 8192, 4096
        out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
        for _ in range(3):
            st = _lib.lib().arborx_debug_valu_probe(ctypes.c_void_p(out.data_ptr()), blocks, iters, None)
            if st != 0:
                sys.exit(f"valu probe failed: {_lib.lib().arborx_last_error().decode()}")
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_valu_blocks": blocks, "iters": iters, "launches": 3}))
        return
    if args.calibrate_copy > 0:
        import torch
        nbytes = int(args.calibrate_copy * 2 ** 30)
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "launches": 3}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one MI355X: the library has no multi-GPU path (queries would shard over GPUs "
              "with a replicated tree); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2507_23700_amd as ax
    from paper_2507_23700_amd import _lib, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    L = _lib.lib()
    log(f"generating {args.dist} workload")
    if args.dist == "gmm6":
        cfg = inputs.config_gmm6(n=args.n or 2_000_000)
    elif args.dist == "small":
        cfg = inputs.config_small(n=args.n or 20_000, m=args.n or 20_000)
    else:
        cfg = inputs.config_paper(args.dist, n=args.n or 10_000_000)
    data, queries, radius = cfg["data"], cfg["queries"], float(cfg["radius"])
    k = args.k or cfg["k"]
    n, m, dim = len(data), len(queries), data.shape[1]
    d = torch.from_numpy(data).cuda()
    q = torch.from_numpy(queries).cuda()
    torch.cuda.synchronize()

    phases = ["build", "spatial_csr", "reduce_count", "reduce_sumdist", "knn"]
    ev = {p: [] for p in phases}
    state = {}

    def step(record):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(len(phases) + 1)]
        e[0].record()
        tree = ax.arborx_bvh_build(d)
        e[1].record()
        off, idx = ax.arborx_query_spatial(tree, q, radius)
        e[2].record()
        c, _ = ax.arborx_query_spatial_reduce(tree, q, radius, ax.COUNT)
        e[3].record()
        c2, s2 = ax.arborx_query_spatial_reduce(tree, q, radius, ax.COUNT_SUMDIST)
        e[4].record()
        d2, ix = ax.arborx_query_knn(tree, q, k)
        e[5].record()
        state.update(tree=tree, off=off, idx=idx, c=c, c2=c2, s2=s2, d2=d2, ix=ix)
        if record:
            for i, p in enumerate(phases):
                ev[p].append((e[i], e[i + 1]))

    for i in range(args.warmup):
        step(False)
        log(f"warmup {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    L.arborx_profile_enable(1)
    profile_collect(L)
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    L.arborx_profile_enable(0)
    prof = profile_collect(L)
    log(f"timed {args.steps} steps in {elapsed:.3f} s")

    ms_per_step = 1000.0 * elapsed / args.steps
    value = 4 * m * args.steps / elapsed
    phase_ms = {p: float(np.median([a.elapsed_time(b) for a, b in ev[p]])) for p in phases}
    total = int(state["off"][-1].item())
    comps = {
        "build_mpts_s": n / phase_ms["build"] / 1e3,
        "spatial_csr_qps": m / phase_ms["spatial_csr"] * 1e3,
        "reduce_count_qps": m / phase_ms["reduce_count"] * 1e3,
        "reduce_sumdist_qps": m / phase_ms["reduce_sumdist"] * 1e3,
        f"knn{k}_qps": m / phase_ms["knn"] * 1e3,
        "phase_ms_median": phase_ms,
        "mean_neighbours": total / m,
        "kernel_ms_per_step": {kname: v[0] / args.steps for kname, v in sorted(prof.items())},
    }
    # outside the step: the early-terminating count at limits below and above the mean row length
    tree = state["tree"]
    for n_max in (1, 5):
        ms = timed(lambda: ax.arborx_query_spatial_count_up_to(tree, q, radius, n_max), 5)
        comps[f"count_up_to{n_max}_qps"] = m / ms * 1e3
    # the callback-with-output form: one radius search whose walk writes each match's squared distance
    # beside its index (compare spatial_csr_qps, the same search without the output), and the gather
    # of the same distances over the step's finished CSR result
    ms = timed(lambda: ax.arborx_query_spatial_with_distances(tree, q, radius), 5)
    comps["spatial_with_distances_qps"] = m / ms * 1e3
    # the same search with rows left in the order the walk found their matches (no row sorts);
    # compare with the same standalone call in ascending order
    ms = timed(lambda: ax.arborx_query_spatial(tree, q, radius), 5)
    comps["spatial_csr_standalone_qps"] = m / ms * 1e3
    ms = timed(lambda: ax.arborx_query_spatial(tree, q, radius, ordered=False), 5)
    comps["spatial_csr_unsorted_qps"] = m / ms * 1e3
    ms = timed(lambda: ax.arborx_query_match_distances(tree, d, q, state["off"], state["idx"]), 5)
    comps["match_distances_per_s"] = total / ms * 1e3
    # rays against 2*10^6 small random boxes: hit counts and the first hit of 10^6 rays
    g = np.random.default_rng(2507)
    bc = g.random((2_000_000, 3)).astype(np.float32)
    bh = (g.random((2_000_000, 3)) * 0.004 + 0.001).astype(np.float32)
    boxes = torch.from_numpy(np.ascontiguousarray(np.stack([bc - bh, bc + bh], axis=1))).cuda()
    rays = torch.from_numpy(np.ascontiguousarray(np.stack([g.random((1_000_000, 3)), g.standard_normal((1_000_000, 3))],
                                                          axis=1).astype(np.float32))).cuda()
    btree = ax.arborx_bvh_build(boxes, ax.BOXES)
    ms = timed(lambda: ax.arborx_query_ray_count(btree, rays), 3)
    comps["ray_count_rays_s"] = rays.shape[0] / ms * 1e3
    ms = timed(lambda: ax.arborx_query_ray_nearest(btree, rays, 1), 3)
    comps["ray_first_hit_rays_s"] = rays.shape[0] / ms * 1e3
    hits = ax.arborx_query_ray_intersect(btree, rays)[0][-1].item()
    ms = timed(lambda: ax.arborx_query_ray_intersect(btree, rays), 3)
    comps["ray_intersect_rays_s"] = rays.shape[0] / ms * 1e3
    ms = timed(lambda: ax.arborx_query_ray_ordered_intersect(btree, rays), 3)
    comps["ray_ordered_intersect_rays_s"] = rays.shape[0] / ms * 1e3
    comps["ray_mean_hits"] = hits / rays.shape[0]
    del btree, boxes, rays
    # DBSCAN over the tree's points (eps = the step's radius, min_pts = 10), and the pair search it is
    # built on (the self-join of the tree's points at the same radius)
    ms = timed(lambda: ax.arborx_dbscan(tree, d, radius, 10), 3)
    comps["dbscan_mpts_s"] = n / ms / 1e3
    ms = timed(lambda: ax.arborx_self_join_degree(tree, radius), 3)
    comps["self_join_mpts_s"] = n / ms / 1e3
    # standalone calls: inside the step the reductions and kNN reuse the query order that the CSR call
    # computed and cached on the tree; alternating two copies of the queries makes every call order
    # its queries again, as a call on fresh queries does
    q_alt = q.clone()
    qs = [q, q_alt]
    for name, fn in (("reduce_count", lambda qq: ax.arborx_query_spatial_reduce(tree, qq, radius, ax.COUNT)),
                     (f"knn{k}", lambda qq: ax.arborx_query_knn(tree, qq, k))):
        ctr = [0]

        def call(fn=fn, ctr=ctr):
            ctr[0] += 1
            fn(qs[ctr[0] % 2])
        ms = timed(call, 5)
        comps[f"{name}_standalone_qps"] = m / ms * 1e3
    del q_alt, qs
    # walk statistics (the debug entry point, outside the step): node fetches per query of the
    # one-query-per-thread radius walk and of the seeded kNN walk, and the node bytes those fetches
    # touch in float nodes (16*dim + 16 B) and in quantized nodes (8*dim + 8 B, 16-byte aligned)
    vr = ax.arborx_debug_node_visits(tree, q, radius=radius).cpu().numpy().astype(np.float64)
    vk = ax.arborx_debug_node_visits(tree, q, k=k).cpu().numpy().astype(np.float64)
    fb, qb = 16 * dim + 16, (8 * dim + 8 + 15) // 16 * 16
    comps["walk_statistics"] = {
        "radius_visits_mean": vr.mean().item(), "radius_visits_p99": np.percentile(vr, 99).item(),
        f"knn{k}_visits_mean": vk.mean().item(), f"knn{k}_visits_p99": np.percentile(vk, 99).item(),
        "node_bytes_float": fb, "node_bytes_quantized": qb,
        "radius_touched_bytes_float": vr.mean().item() * fb, "radius_touched_bytes_quantized": vr.mean().item() * qb,
        f"knn{k}_touched_bytes_float": vk.mean().item() * fb, f"knn{k}_touched_bytes_quantized": vk.mean().item() * qb,
        "tree_height": ax.arborx_bvh_info(tree)["height"],
    }
    del vr, vk

    # dominant kernel by GPU time in the timed region
    dom = max((kn for kn in prof if algorithmic_bytes(kn, n, m, dim, k, total)), key=lambda kn: prof[kn][0])
    avg_ms = prof[dom][0] / prof[dom][1]
    alg = algorithmic_bytes(dom, n, m, dim, k, total)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    copy_gbs = copy_bandwidth(torch)
    roofline = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(dom, cfg["workload"]),
                "valu_busy": profiled(dom, cfg["workload"], "valu_busy"),
                "algorithmic_bytes_per_launch": alg, "avg_launch_ms": avg_ms,
                "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs}
    # node bytes the dominant walk touches (served mostly by L1/L2): node fetches per query from the
    # walk statistics times the node size of the format the library's defaults walk (kNN on float
    # nodes up to 3D and quantized in 6D; the radius walks on quantized nodes)
    ws = comps["walk_statistics"]
    visits = ws[f"knn{k}_visits_mean"] if dom == "knn" else (ws["radius_visits_mean"] if dom in (
        "spatial_count", "reduce_count", "reduce_sumdist") else None)
    if visits is not None:
        nbytes = ws["node_bytes_float"] if (dom == "knn" and dim <= 3) else ws["node_bytes_quantized"]
        touched = visits * nbytes * m
        roofline["touched_node_bytes_per_launch"] = touched
        roofline["touched_node_gbs"] = touched / (avg_ms * 1e-3) / 1e9

    cpu = None
    parity = None
    if not args.no_cpu:
        log("timing the CPU oracle on a sample")
        cpu, sel, res = cpu_baseline(data, queries, radius, k)
        off_o, idx_o, c_o, c2_o, s2_o, d2_o, ix_o = res
        off_g = state["off"].cpu().numpy()
        idx_g = state["idx"].cpu().numpy()
        ok = all(np.array_equal(idx_g[off_g[j]:off_g[j + 1]], idx_o[off_o[i]:off_o[i + 1]]) for i, j in enumerate(sel))
        ok = ok and np.array_equal(state["c"].cpu().numpy()[sel], c_o)
        ok = ok and np.array_equal(state["s2"].cpu().numpy()[sel], s2_o)
        ok = ok and np.array_equal(state["ix"].cpu().numpy()[sel], ix_o)
        ok = ok and np.array_equal(state["d2"].cpu().numpy()[sel], d2_o)
        parity = f"{'exact' if ok else 'MISMATCH'} on {len(sel)} sampled queries"
        log(f"parity: {parity}")

    state.clear()
    torch.cuda.empty_cache()
    forest = None if args.no_forest else forest_bench()
    chamfer = None if args.no_chamfer else chamfer_bench()

    line = {
        "metric": "radius/kNN queries/s at 10M 3D pts; BVH build Mpts/s; batched vs plain",
        "value": value, "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded numpy generators)",
        "config": {"workload": cfg["workload"], "n": n, "m": m, "dim": dim, "distribution": args.dist,
                   "radius": radius, "k": k,
                   "step": f"build + radius CSR + COUNT + COUNT_SUMDIST + kNN k={k}; value counts 4*M queries per step"},
        "components": comps, "roofline": roofline, "cpu_baseline": cpu, "parity": parity,
        "batched_vs_plain": forest, "chamfer": chamfer,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
