"""Benchmark: single-source BVSS BFS on one MI355X.

Workload (the configuration the headline metric is quoted on): an R-MAT graph
of scale 22 (4,194,304 vertices, edge factor 16, a,b,c = 0.57,0.19,0.19,
symmetrised, self loops and duplicates removed, randomly relabelled, then
relabelled by the build's JaccardWithWindows as its degree distribution is
scale-free-like), 64 seeded sources run one at a time. One step = the 64 traversals. The graph is
built and resident in HBM before timing starts.

value = harmonic-mean GTEPS over the sources, where a traversal's edge count
is half the degree sum of the vertices it reaches (undirected edges of the
source's component). The switch policy is the learned network when a trained
model is installed (paper_2606_05081_amd/switch_model.json) and three trial
traversals on other sources show it faster than Eq. 3 on this graph (the
paper's per-graph enable); otherwise Eq. 3. Both are measured and reported.

Also measured in the same run and printed in the JSON line: the plain
method (BVSS top-down at every level) on the same sources with its roofline,
the 2048x2048 grid with 10% edge deletion (RCM-reordered), batched
multi-source BFS sources/s on scale-20 R-MAT (960 sources in batches of
64/128/256/512, one launch), exact closeness (all 262,144 sources of
scale-18 R-MAT; 16,384 sources of scale-23 R-MAT) with the pairs rule and
with the multi-source switch network (paper_2606_05081_amd/switch_model_ms.json,
kept per graph only if a trial batch of 512 other sources was faster with it)
and the CPU oracle on a bounded sample.
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

METRIC = "GTEPS on 1 MI355X (R-MAT s22) learned vs heuristic switch; msBFS sources/s"
HBM_PEAK_GBS = 8000.0


def harmonic_gteps(edges, times_ms):
    e = np.asarray(edges, dtype=np.float64)
    t = np.asarray(times_ms, dtype=np.float64) * 1e-3
    per = e / t / 1e9
    return float(len(per) / np.sum(1.0 / per))


def traversal_edges(rp, levels):
    deg = np.diff(rp).astype(np.int64)
    return int(deg[levels >= 0].sum() // 2)


def algorithmic_bytes(stats, n, sigma, slice_bytes, deg, levels, relabelled):
    """Bytes a traversal must move, from its per-level log, by these per-unit
    counts: a top-down step (Alg. 3 Stage 1, queue or panel form) moves the
    slice word plus the sigma/8 frontier bytes of its set per slice of a
    queued VSS, and 9 B per queued VSS (its descriptor and frontier word); a
    bottom-up step 8 B per unvisited vertex of nonzero degree and 4 B per
    scanned edge; a push step 8 B per frontier vertex and 4 B per edge; each
    Stage 2 3n/8 B (marks, visited and frontier words) plus 4 B per new vertex
    and 4 B per enqueued VSS; and a traversal 4n B of initialisation, 4n of
    levels, and 4n of input ids when the graph was relabelled. Slots of the
    panel copy outside the queued VSSs are read but not counted."""
    total = 8 * n + (4 * n if relabelled else 0)
    lev = np.where(levels < 0, np.iinfo(np.int32).max, levels)
    for i, r in enumerate(stats[:-1]):
        eng = r["engine"]
        if eng == 0:
            total += (slice_bytes + sigma // 8) * r["queue_slices"] + 9 * r["queue"]
        elif eng == 1:
            total += 4 * r["work"] + 8 * r["frontier"]
        else:
            unv_deg = int(((lev > r["level"]) & (deg > 0)).sum())
            total += 4 * r["work"] + 8 * unv_deg
        nxt = stats[i + 1]
        total += 3 * n // 8 + 4 * nxt["frontier"] + 4 * nxt["queue"]
    return int(total)


def timed_sources(g, srcs, out, torch):
    """Per-source device time (ms) with HIP events on the launch stream."""
    st = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(srcs) + 1)]
    evs[0].record(st)
    for i, s in enumerate(srcs):
        g.bfs(int(s), out)
        evs[i + 1].record(st)
    g.sync()
    torch.cuda.synchronize()
    return [evs[i].elapsed_time(evs[i + 1]) for i in range(len(srcs))]


def load_switch_model(name="switch_model.json"):
    path = os.path.join(ROOT, "paper_2606_05081_amd", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def timed_call(fn, torch):
    """Device time (ms) of one call of fn on the current stream, after a sync."""
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def ms_learned_enable(g, trial_srcs, torch, blest):
    """Per-graph enable of the multi-source network: one trial batch of 512
    sources per policy; the learned policy stays only if it was faster."""
    t = {}
    for name, pol in (("heuristic", blest.Policy.HEURISTIC), ("learned", blest.Policy.LEARNED)):
        g.set_policy(pol)
        g.closeness(trial_srcs)
        t[name] = timed_call(lambda: (g.closeness(trial_srcs), g.sync()), torch)
    return t["learned"] < t["heuristic"], t


def host_description():
    """Host CPU model, logical CPUs and the thread count the oracle legs use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = nproc
    # at most 16 threads (one GPU's share of a shared host), fewer if OMP_NUM_THREADS or the affinity mask says so
    threads = max(1, min(avail, int(os.environ.get("OMP_NUM_THREADS", "16") or 16), 16))
    smt = None
    try:
        with open("/sys/devices/system/cpu/smt/active") as f:
            smt = f.read().strip() == "1"
    except OSError:
        pass
    return {"cpu_model": model, "nproc": nproc, "affinity_cpus": avail, "smt_active": smt, "threads_used": threads}


def cpu_baseline(rp, col, srcs, edges, gpu_levels, ms_graphs, budget_s=8.0):
    """The oracle on the host, on bounded samples of the same workloads.

    value: all-core throughput of the oracle's queue BFS, one traversal per
    source spread over the threads, on the R-MAT scale-22 sources (GTEPS =
    their undirected component edges / wall time). Also: one thread alone,
    the multi-source workload (scale-20 R-MAT) and the closeness workloads
    (scale-18 and scale-23 R-MAT) in sources/s, and the sampled learned-switch
    traversals of the timed run compared with the oracle's levels."""
    import oracle
    host = host_description()
    thr = host["threads_used"]
    t_lev, times, one_edges, parity = time.time(), [], [], []
    for i, s in enumerate(srcs):
        t0 = time.perf_counter()
        lev = oracle.bfs(rp, col, int(s))
        times.append((time.perf_counter() - t0) * 1e3)
        one_edges.append(edges[i])
        if i < len(gpu_levels):
            parity.append(bool(np.array_equal(lev, gpu_levels[i])))
        if time.time() - t_lev > budget_s and i + 1 >= len(gpu_levels):
            break
    single = harmonic_gteps(one_edges, times)
    # all threads: one BFS per source (the oracle's threaded closeness runs exactly that)
    k_all = min(len(srcs), 4 * thr)
    t0 = time.perf_counter()
    oracle.closeness(rp, col, np.asarray(srcs[:k_all], np.int32), threads=thr)
    wall = time.perf_counter() - t0
    allcore = float(np.sum(edges[:k_all])) / wall / 1e9
    legs = {}
    for tag, (grp, gcol, gsrcs, kind) in ms_graphs.items():
        t0 = time.perf_counter()
        if kind == "msbfs":
            oracle.msbfs16(grp, gcol, gsrcs, threads=thr)
        else:
            oracle.closeness(grp, gcol, gsrcs, threads=thr)
        legs[tag] = {"sources": int(len(gsrcs)), "sources_per_s": round(len(gsrcs) / (time.perf_counter() - t0), 2),
                     "threads": thr}
    return {"value": round(allcore, 4), "unit": "GTEPS", "cores": thr, "kind": "oracle",
            "sample": f"{k_all} of the {len(srcs)} R-MAT scale-22 sources, one FIFO-queue BFS per source over "
                      f"{thr} host threads",
            "single_thread": {"value": round(single, 4), "unit": "GTEPS", "sources": len(times)},
            "host": host, "legs_sources_per_s": legs,
            "learned_levels_equal_oracle": f"{sum(parity)} of {len(parity)} sampled learned-switch traversals"}


# The persistent kernel and what fixes its launch (block size, panel layout):
# a counter summary taken on other versions of these files is not reported.
KERNEL_SOURCES = ["paper_2606_05081_amd/csrc/bfs.hip", "paper_2606_05081_amd/csrc/device_common.h",
                  "paper_2606_05081_amd/csrc/mlp_infer.h",
                  "paper_2606_05081_amd/csrc/blest_internal.h", "paper_2606_05081_amd/csrc/api.cpp",
                  "paper_2606_05081_amd/csrc/host_build.cpp"]
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_bfs_persistent_rmat22_bvss_traffic.txt")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile():
    """HBM bytes per launch of the plain-method persistent kernel from the committed
    rocprofv3 summary, or None if it is missing or was taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    vals = {}
    with open(TRAFFIC_SUMMARY) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return int(float(vals["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def profile_leg(leg, n_sources=8):
    """A short run for rocprofv3: a 512 MiB device copy (counter calibration),
    then one workload: `bvss` / `heuristic` -- n_sources traversals of the
    scale-22 R-MAT with that policy; `msbfs` -- the scale-20 multi-source
    workload (960 sources, batches 64/128/256/512, one launch); `msbfs_mfma`
    -- the same with the neighbour check on the matrix cores; `closeness` --
    4,096 sources of scale-18 R-MAT in batches of 512."""
    import torch
    from paper_2606_05081_amd import blest, inputs
    if leg in ("bvss", "heuristic"):
        rp, col = inputs.rmat_graph(22, 1020)
    elif leg in ("msbfs", "msbfs_mfma"):
        rp, col = inputs.rmat_graph(20, 1040)
    else:
        rp, col = inputs.rmat_graph(18, 1050)
    g = blest.Graph(rp, col, device=0, msbfs_width=512, ms_mfma=int(leg == "msbfs_mfma"), **{"async": 1})
    a = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    c.copy_(a)
    torch.cuda.synchronize()
    try:
        if leg in ("bvss", "heuristic"):
            g.set_policy(getattr(blest.Policy, leg.upper()))
            out = torch.empty(g.n, dtype=torch.int32, device="cuda")
            ms = float(np.mean(timed_sources(g, inputs.sources(rp, n_sources, seed=1021), out, torch)))
        elif leg in ("msbfs", "msbfs_mfma"):
            srcs = inputs.sources(rp, 960, seed=1041)
            out = torch.empty((960, g.n), dtype=torch.int16, device="cuda")
            ms = timed_call(lambda: (g.msbfs_batched(srcs, [64, 128, 256, 512], out), g.sync()), torch)
        else:
            srcs = np.arange(0, 4096, dtype=np.int32)
            ms = timed_call(lambda: (g.closeness(srcs), g.sync()), torch)
    finally:
        g.close()  # release device memory before the profiler's own exit handlers run
    copy_bytes = 2 * a.numel() * 4
    del a, c
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps({"profile_leg": leg, "ms": ms, "calibration_copy_bytes": copy_bytes,
                      "kernel_source_sha256_16": kernel_source_hash()}), flush=True)


def load_eta_tuned():
    """eta of Eq. 3 tuned on the switch network's training graphs
    (python -m paper_2606_05081_amd.switch --tune-eta), or None."""
    path = os.path.join(ROOT, "paper_2606_05081_amd", "switch_eta.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return float(json.load(f)["eta"])


def install_model(g, model):
    g.set_switch_model(np.array(model["params"], np.float32), np.array(model["mean"], np.float32),
                       np.array(model["std"], np.float32), model.get("min_confidence", 0.5))


def switching_enable(g, trial_srcs, eta, torch, blest, trials=3):
    """The paper's per-graph enable of direction switching (switching
    analysis of its experiments): three trial traversals with Eq. 3 and
    three without switching (BVSS top-down at every level); switching stays on
    only if its trials were faster. Returns (enabled, {name: ms})."""
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    t = {}
    for name, pol in (("switching", blest.Policy.HEURISTIC), ("no_switching", blest.Policy.BVSS)):
        g.set_policy(pol, eta)
        g.bfs(int(trial_srcs[0]), out)
        t[name] = float(np.mean(timed_sources(g, trial_srcs[:trials], out, torch)))
    return t["switching"] < t["no_switching"], t


def policy_gteps(g, srcs, edges, out, pol, eta, torch, reps=1):
    g.set_policy(pol, eta)
    timed_sources(g, srcs[:2], out, torch)
    per = np.mean(np.array([timed_sources(g, srcs, out, torch) for _ in range(reps)]), axis=0)
    return harmonic_gteps(edges, per), per


def c3_leg(kind, scale, gseed, sseed, model, eta_tuned, torch, blest, inputs, nsrc=16):
    """Learned vs heuristic switch on a held-out graph: R-MAT scale 24 or
    Erdos-Renyi 2^24 (8 * 2^24 uniform pairs). Heuristic = Eq. 3 with the
    paper's per-graph enable of switching, at eta = 10 and at the tuned eta;
    learned = the switch network, kept for the graph only if three trial
    traversals beat Eq. 3 (eta = 10)."""
    t0 = time.time()
    rp, col = inputs.rmat_graph(scale, gseed) if kind == "rmat" else inputs.er_graph(scale, gseed)
    srcs = inputs.sources(rp, nsrc, seed=sseed)
    g = blest.Graph(rp, col, device=0, **{"async": 1})
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    edges = []
    g.set_policy(blest.Policy.HEURISTIC)
    for s in srcs:
        g.bfs(int(s), out)
        g.sync()
        edges.append(traversal_edges(rp, out.cpu().numpy()))
    res = {"graph": f"{kind}{scale}", "n": g.n, "m": g.m, "sources": nsrc, "build_s": round(time.time() - t0, 1)}
    trial = inputs.sources(rp, 3, seed=sseed + 1)
    plain, _ = policy_gteps(g, srcs, edges, out, blest.Policy.BVSS, 10.0, torch)
    res["plain_method_gteps"] = round(plain, 3)
    for tag, eta in (("eta10", 10.0), ("eta_tuned", eta_tuned)):
        if eta is None:
            continue
        gt, _ = policy_gteps(g, srcs, edges, out, blest.Policy.HEURISTIC, eta, torch)
        en, tt = switching_enable(g, trial, eta, torch, blest)
        res[f"heuristic_{tag}"] = {"eta": eta, "gteps_switching": round(gt, 3), "switching_enabled_by_trials": en,
                                   "gteps": round(gt if en else plain, 3)}
    if model is not None:
        install_model(g, model)
        lg, _ = policy_gteps(g, srcs, edges, out, blest.Policy.LEARNED, 10.0, torch)
        from paper_2606_05081_amd import switch
        en, tt = switch.per_graph_enable(g, trial)
        res["learned"] = {"gteps_network": round(lg, 3), "enabled_by_trials": bool(en),
                          "gteps": round(lg if en else res["heuristic_eta10"]["gteps_switching"], 3)}
        for tag in ("eta10", "eta_tuned"):
            if f"heuristic_{tag}" in res:
                res[f"learned_over_heuristic_{tag}"] = round(res["learned"]["gteps"] / res[f"heuristic_{tag}"]["gteps"],
                                                            4)
    g.close()
    print(f"# C3 {res}", file=sys.stderr, flush=True)
    return res


def ms_algorithmic_bytes(recs, n, nsets, sigma, slice_bytes, k):
    """Lower bound of the bytes a multi-source call must move, from its level
    records: per level, (slice word + sigma/8) B per slice of a queued VSS and
    the sigma * kappa / 8 frontier bytes each queued VSS stages; kappa/8 B per
    hit row (the next-word flush) and 3 kappa/8 B per dirty vertex (next,
    visited and frontier words), bounded below by the new (vertex, traversal)
    pairs, since a vertex has at most kappa of them: new_pairs / 8 and
    3 new_pairs / 8; and the int16 levels: 2 B per (source, vertex) filled,
    and 2 B per visited pair written."""
    total = 2 * k * n
    for r in recs:
        kappa = r["width"]
        total += (slice_bytes + sigma // 8) * r["queue_slices"] + sigma * kappa // 8 * r["queue"]
        total += r["new_pairs"] // 2 + 2 * r["new_pairs"]
    return int(total)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sources", type=int, default=64)
    ap.add_argument("--no-extras", action="store_true", help="skip grid, msBFS, C3 and CPU legs")
    ap.add_argument("--no-c3", action="store_true", help="skip the scale-24 R-MAT and 2^24 ER legs")
    ap.add_argument("--profile-leg", choices=["heuristic", "bvss", "msbfs", "msbfs_mfma", "closeness"], default=None,
                    help="only a short run of one workload plus a calibration copy, for rocprofv3")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the path is built for one GPU, "
                                   "multi-GPU sharding (by source batches or by rows) is not", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.profile_leg:
        profile_leg(args.profile_leg)
        return

    import torch
    from paper_2606_05081_amd import blest, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    t0 = time.time()
    rp, col = inputs.rmat_graph(22, 1020)
    srcs = inputs.sources(rp, args.sources, seed=1021)
    g = blest.Graph(rp, col, device=0, **{"async": 1})
    info = g.info()
    print(f"# graph built in {time.time() - t0:.1f}s: n={info['n']} m={info['m']} slices={info['n_slices']} "
          f"vss={info['n_vss']} grid={info['grid_blocks']}x{info['block_size']}", file=sys.stderr, flush=True)
    out = torch.empty(g.n, dtype=torch.int32, device=dev)

    # exact edge counts per source
    edges = []
    for s in srcs:
        g.set_policy(blest.Policy.HEURISTIC)
        g.bfs(int(s), out)
        g.sync()
        edges.append(traversal_edges(rp, out.cpu().numpy()))

    model = load_switch_model()
    eta_tuned = load_eta_tuned()
    policy = "heuristic"
    if model is not None:
        install_model(g, model)

    def run_policy(pol, steps, warmup, eta=10.0):
        g.set_policy(pol, eta)
        for _ in range(warmup):
            timed_sources(g, srcs, out, torch)
        step_ms, all_t = [], []
        for _ in range(steps):
            torch.cuda.synchronize()
            t_s = time.perf_counter()
            ts = timed_sources(g, srcs, out, torch)
            torch.cuda.synchronize()
            step_ms.append((time.perf_counter() - t_s) * 1e3)
            all_t.append(ts)
        per_src = np.mean(np.array(all_t), axis=0)
        return harmonic_gteps(edges, per_src), float(np.mean(step_ms)), per_src

    heur_gteps, heur_step_ms, heur_t = run_policy(blest.Policy.HEURISTIC, args.steps, args.warmup)
    print(f"# heuristic: {heur_gteps:.1f} GTEPS, mean {np.mean(heur_t):.3f} ms/source", file=sys.stderr, flush=True)
    tuned = None
    if eta_tuned is not None:
        tg, _, _ = run_policy(blest.Policy.HEURISTIC, 1, 1, eta_tuned)
        tuned = {"eta": eta_tuned, "gteps": round(tg, 3)}
    sw_enabled, sw_trial = switching_enable(g, inputs.sources(rp, 3, seed=1022), 10.0, torch, blest)
    learned_gteps, enabled, trial_ms = None, None, None
    value, step_ms = heur_gteps, heur_step_ms
    learned_levels = []
    if model is not None:
        learned_gteps, learned_step_ms, _ = run_policy(blest.Policy.LEARNED, args.steps, args.warmup)
        print(f"# learned: {learned_gteps:.1f} GTEPS", file=sys.stderr, flush=True)
        # per-graph enable by three trial traversals on sources outside the timed set
        from paper_2606_05081_amd import switch
        enabled, trial_ms = switch.per_graph_enable(g, inputs.sources(rp, 3, seed=1022))
        if enabled:
            value, step_ms, policy = learned_gteps, learned_step_ms, "learned"
        else:
            policy = "heuristic (learned switch disabled for this graph by its trial traversals)"
        # levels of sampled learned traversals, for the oracle comparison in the CPU leg (not timed)
        g.set_policy(blest.Policy.LEARNED)
        for s in srcs[:8]:
            g.bfs(int(s), out)
            g.sync()
            learned_levels.append(out.cpu().numpy().copy())

    # plain method (BVSS top-down every level): roofline of the persistent kernel
    td_gteps, _, td_t = run_policy(blest.Policy.BVSS, 1, 1)
    g.set_log_work(True)  # per-level adjacency counts for the byte accounting (not timed)
    nb = []
    deg = np.diff(rp).astype(np.int64)
    pan_b, pan_us = [], []  # the panel steps alone: bytes read and Stage 1 time (fused Stage 2 and barrier included)
    for s in srcs[:8]:
        g.bfs(int(s), out)
        g.sync()
        lev = out.cpu().numpy()
        st = g.level_stats()
        nb.append(algorithmic_bytes(st, info["n"], info["sigma"], info["slice_bytes"], deg, lev,
                                    info["reordered"] != 0))
        for r in st[:-1]:
            if r["engine"] == 0 and r.get("bvss_panel"):
                pan_b.append(4 * r["work"] + 4 * (r["work"] // 256) + info["n"] // 8)
                pan_us.append(r["t_stage1_us"])
    bytes_per_launch = float(np.mean(nb))
    launch_ms = float(np.mean(td_t[:8]))
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile(),
                "kernel": "k_bfs_persistent (plain method: BVSS top-down every level)",
                "bytes_per_launch": int(bytes_per_launch), "launch_ms": round(launch_ms, 4)}
    # same for the switched run
    g.set_policy(blest.Policy.HEURISTIC)
    nb2 = []
    for s in srcs[:8]:
        g.bfs(int(s), out)
        g.sync()
        lev = out.cpu().numpy()
        nb2.append(algorithmic_bytes(g.level_stats(), info["n"], info["sigma"], info["slice_bytes"], deg, lev,
                                     info["reordered"] != 0))
    sw_ach = float(np.mean(nb2)) / (float(np.mean(heur_t[:8])) * 1e-3) / 1e9
    g.set_log_work(False)

    extras = {"heuristic_gteps": round(heur_gteps, 3), "heuristic_tuned_eta": tuned,
              "switching_enabled_by_trials": sw_enabled,
              "switching_trial_ms_per_source": {k: round(v, 4) for k, v in sw_trial.items()},
              "learned_gteps": None if learned_gteps is None else round(learned_gteps, 3),
              "learned_over_heuristic": None if learned_gteps is None else round(learned_gteps / heur_gteps, 4),
              "learned_over_heuristic_tuned_eta": None if (learned_gteps is None or tuned is None) else
              round(learned_gteps / tuned["gteps"], 4),
              "learned_enabled_by_trials": enabled,
              "trial_ms_per_source": None if trial_ms is None else {k: round(v, 4) for k, v in trial_ms.items()},
              "plain_method_gteps": round(td_gteps, 3),
              "ms_per_source": round(float(np.mean(heur_t)), 4), "switched_achieved_GBs": round(sw_ach, 1),
              "panel_step": None if not pan_b else {
                  "levels": len(pan_b), "GB_per_level": round(float(np.mean(pan_b)) / 1e9, 4),
                  "us_per_level": round(float(np.mean(pan_us)), 1),
                  "GBs": round(float(np.sum(pan_b)) / (float(np.sum(pan_us)) * 1e-6) / 1e9, 1)}}
    g.close()
    # the same sources on the autotuner's options for this graph size (the
    # switch network and the tuned eta were fitted at the default 128 slices
    # per VSS, which the headline keeps)
    tg = blest.Graph(rp, col, device=0, autotune=True, **{"async": 1})
    if model is not None:
        install_model(tg, model)
    tinfo = tg.info()
    tres = {"cache_entry": tg.autotuned, "tau": tinfo["tau"], "sigma": tinfo["sigma"]}
    tout = torch.empty(tg.n, dtype=torch.int32, device=dev)
    for tag, pol, eta in (("learned", blest.Policy.LEARNED, 10.0), ("heuristic_eta10", blest.Policy.HEURISTIC, 10.0),
                          ("plain", blest.Policy.BVSS, 10.0)):
        if pol == blest.Policy.LEARNED and model is None:
            continue
        tres[f"{tag}_gteps"] = round(policy_gteps(tg, srcs, edges, tout, pol, eta, torch)[0], 3)
    extras["rmat22_autotuned"] = tres
    tg.close()

    cpu = None
    if not args.no_extras:
        # grid 2048 x 2048, 10% deletion, RCM-reordered inside the build
        grp, gcol = inputs.grid_graph(2048, 1022)
        gs = inputs.sources(grp, 16, seed=1023)
        gg = blest.Graph(grp, gcol, device=0, **{"async": 1})
        gout = torch.empty(gg.n, dtype=torch.int32, device=dev)
        gedges = []
        for s in gs:
            gg.bfs(int(s), gout)
            gg.sync()
            gedges.append(traversal_edges(grp, gout.cpu().numpy()))
        gt = timed_sources(gg, gs, gout, torch)
        ginfo = gg.info()
        nlev = len(gg.level_stats())
        extras["grid2048_ms_per_source"] = round(float(np.mean(gt)), 3)
        extras["grid2048_gteps"] = round(harmonic_gteps(gedges, gt), 4)
        extras["grid2048_levels"] = nlev
        extras["grid2048_update_scheme"] = "eager" if ginfo["update_scheme"] == blest.Update.EAGER else "lazy"
        extras["grid2048_u_div"] = round(ginfo["u_div"], 1)
        gg.close()
        # the other vertex-update scheme on the same sources (Alg. 2 vs Alg. 3)
        other = blest.Update.LAZY if ginfo["update_scheme"] == blest.Update.EAGER else blest.Update.EAGER
        go = blest.Graph(grp, gcol, device=0, update_scheme=int(other), **{"async": 1})
        timed_sources(go, gs[:2], gout, torch)
        ot = timed_sources(go, gs, gout, torch)
        tag = "lazy" if other == blest.Update.LAZY else "eager"
        extras[f"grid2048_{tag}_ms_per_source"] = round(float(np.mean(ot)), 3)
        extras["grid2048_us_per_level"] = {extras["grid2048_update_scheme"]: round(float(np.mean(gt)) * 1e3 / nlev, 2),
                                           tag: round(float(np.mean(ot)) * 1e3 / len(go.level_stats()), 2)}
        go.close()
        del grp, gcol
        # batched multi-source BFS: scale-20 R-MAT, 960 sources, batches 64/128/256/512 in one launch
        mrp, mcol = inputs.rmat_graph(20, 1040)
        msrcs = inputs.sources(mrp, 960, seed=1041)
        # slice width and VSS size from the autotuner (the batch widths are the workload's)
        mg = blest.Graph(mrp, mcol, device=0, autotune=True, **{"async": 1})
        minfo = mg.info()
        extras["msbfs_autotuned"] = {"cache_entry": mg.autotuned, "sigma": minfo["sigma"], "tau": minfo["tau"],
                                     "slice_bytes": minfo["slice_bytes"]}
        mout = torch.empty((960, mg.n), dtype=torch.int16, device=dev)
        mg.msbfs_batched(msrcs, [64, 128, 256, 512], mout)
        mg.sync()
        ms_ms = timed_call(lambda: mg.msbfs_batched(msrcs, [64, 128, 256, 512], mout), torch)
        extras["msbfs_sources_per_s"] = round(960 / ms_ms * 1e3, 1)
        extras["msbfs_ms"] = round(ms_ms, 3)
        mb = ms_algorithmic_bytes(mg.ms_level_stats(), minfo["n"], minfo["n_slice_sets"], minfo["sigma"],
                                  minfo["slice_bytes"], 960)
        extras["msbfs_roofline"] = {"bound": "hbm", "kernel": "k_ms_persistent (pairs rule)",
                                    "algorithmic_bytes_lower_bound": mb, "ms": round(ms_ms, 3),
                                    "achieved_GBs": round(mb / (ms_ms * 1e-3) / 1e9, 1),
                                    "frac": round(mb / (ms_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        per_width = {}
        for w in (64, 128, 256, 512):  # each batch width alone over the same 960 sources
            per_width[str(w)] = round(960 / timed_call(lambda: mg.msbfs_batched(msrcs, [w], mout), torch) * 1e3, 1)
        extras["msbfs_sources_per_s_by_width"] = per_width
        ms_model = load_switch_model("switch_model_ms.json")
        if ms_model is not None:  # the same 960 sources with the multi-source switch network
            mg.set_ms_switch_model(np.array(ms_model["params"], np.float32), np.array(ms_model["mean"], np.float32),
                                   np.array(ms_model["std"], np.float32), ms_model.get("min_confidence", 0.5))
            mg.set_policy(blest.Policy.LEARNED)
            mg.msbfs_batched(msrcs, [64, 128, 256, 512], mout)
            lms = timed_call(lambda: (mg.msbfs_batched(msrcs, [64, 128, 256, 512], mout), mg.sync()), torch)
            extras["msbfs_learned_sources_per_s"] = round(960 / lms * 1e3, 1)
            mg.set_policy(blest.Policy.HEURISTIC)
        # the paper's multi-source ablation ladder on the same 960 sources
        # (Section "Ablation Studies"): naive = one single-source traversal per
        # source; (A) no getVI remap and no dynamic slice-set tracking; (AB) no
        # tracking; (Full) = the msbfs leg above
        sout1 = torch.empty(mg.n, dtype=torch.int32, device=dev)
        mg.set_policy(blest.Policy.HEURISTIC)
        naive_ms = timed_call(lambda: [mg.bfs(int(x), sout1) for x in msrcs], torch)
        ladder = {"naive_single_source": round(960 / naive_ms * 1e3, 1)}
        mg.close()
        for tag, flags in (("A_no_getvi_no_tracking", 3), ("AB_no_tracking", 2)):
            ag = blest.Graph(mrp, mcol, device=0, ms_ablation=flags, autotune=True, **{"async": 1})
            ag.msbfs_batched(msrcs, [64, 128, 256, 512], mout)
            ladder[tag] = round(960 / timed_call(lambda: ag.msbfs_batched(msrcs, [64, 128, 256, 512], mout),
                                                 torch) * 1e3, 1)
            ag.close()
        ladder["full"] = extras["msbfs_sources_per_s"]
        extras["msbfs_ablation_sources_per_s"] = ladder
        # the neighbour check on the matrix cores (int8 MFMA) instead of bitwise, same sources
        xg = blest.Graph(mrp, mcol, device=0, ms_mfma=1, autotune=True, **{"async": 1})
        xg.msbfs_batched(msrcs, [64, 128, 256, 512], mout)
        extras["msbfs_mfma_sources_per_s"] = round(
            960 / timed_call(lambda: xg.msbfs_batched(msrcs, [64, 128, 256, 512], mout), torch) * 1e3, 1)
        xg.close()
        del mout
        # the same 960 sources with the levels as a replayed hipGraph of per-phase kernels
        gmg = blest.Graph(mrp, mcol, device=0, msbfs_graph=1, autotune=True, **{"async": 1})
        gmout = torch.empty((960, gmg.n), dtype=torch.int16, device=dev)
        gmg.msbfs_batched(msrcs, [64, 128, 256, 512], gmout)
        gmg.sync()
        extras["msbfs_graph_sources_per_s"] = round(
            960 / timed_call(lambda: (gmg.msbfs_batched(msrcs, [64, 128, 256, 512], gmout), gmg.sync()), torch) * 1e3, 1)
        gmg.close()
        del gmout
        # small single-source case: R-MAT scale 16, plain method and Eq. 3
        srp, scol = inputs.rmat_graph(16, 1010)
        ss = inputs.sources(srp, 64, seed=1011)
        sg = blest.Graph(srp, scol, device=0, **{"async": 1})
        sout = torch.empty(sg.n, dtype=torch.int32, device=dev)
        sedges = []
        for s in ss:
            sg.bfs(int(s), sout)
            sg.sync()
            sedges.append(traversal_edges(srp, sout.cpu().numpy()))
        for name, pol in (("rmat16_plain_gteps", blest.Policy.BVSS), ("rmat16_heuristic_gteps", blest.Policy.HEURISTIC)):
            sg.set_policy(pol)
            timed_sources(sg, ss, sout, torch)
            extras[name] = round(harmonic_gteps(sedges, timed_sources(sg, ss, sout, torch)), 3)
        sinfo = sg.info()
        extras["rmat16_update_scheme"] = "eager" if sinfo["update_scheme"] == blest.Update.EAGER else "lazy"
        extras["rmat16_u_div"] = round(sinfo["u_div"], 1)
        sg.close()
        # the plain method on the lazy scheme too (the dispatch sends graphs this small to Alg. 2)
        sl = blest.Graph(srp, scol, device=0, update_scheme=int(blest.Update.LAZY), **{"async": 1})
        sl.set_policy(blest.Policy.BVSS)
        timed_sources(sl, ss, sout, torch)
        extras["rmat16_plain_lazy_gteps"] = round(harmonic_gteps(sedges, timed_sources(sl, ss, sout, torch)), 3)
        sl.close()
        # exact closeness: all sources of scale-18 R-MAT, 16,384 sources of scale-23 R-MAT (512 per
        # batch), with the pairs rule and with the multi-source switch network (per-graph enabled)
        ms_model = load_switch_model("switch_model_ms.json")
        cgraphs = {}
        for tag, scale, gseed, k in (("closeness_rmat18_all", 18, 1050, None), ("closeness_rmat23_16k", 23, 1052, 16384)):
            crp, ccol = inputs.rmat_graph(scale, gseed)
            cs = np.arange(crp.size - 1, dtype=np.int32) if k is None else inputs.sources(crp, k, seed=gseed + 1)
            cgraphs[tag] = (crp, ccol, cs)
            cg = blest.Graph(crp, ccol, device=0, msbfs_width=512, autotune=True, **{"async": 1})
            res = {"sources": int(cs.size), "autotuned": cg.autotuned, "tau": cg.info()["tau"]}
            pols = [("heuristic", blest.Policy.HEURISTIC)]
            if ms_model is not None:
                cg.set_ms_switch_model(np.array(ms_model["params"], np.float32), np.array(ms_model["mean"], np.float32),
                                       np.array(ms_model["std"], np.float32), ms_model.get("min_confidence", 0.5))
                en, trial = ms_learned_enable(cg, inputs.sources(crp, 512, seed=gseed + 7), torch, blest)
                res["learned_enabled_by_trial"] = bool(en)
                res["trial_ms"] = {k2: round(v, 2) for k2, v in trial.items()}
                pols.append(("learned", blest.Policy.LEARNED))
            for name, pol in pols:
                cg.set_policy(pol)
                cg.closeness(cs[:512])
                cms = timed_call(lambda: (cg.closeness(cs), cg.sync()), torch)
                res[f"ms_{name}"] = round(cms, 1)
                print(f"# {tag} {name}: {cs.size} sources in {cms:.1f} ms", file=sys.stderr, flush=True)
            chosen = "learned" if res.get("learned_enabled_by_trial") else "heuristic"
            res["policy"] = chosen
            res["ms"] = res[f"ms_{chosen}"]
            res["sources_per_s"] = round(cs.size / res["ms"] * 1e3, 1)
            extras[tag] = res
            cg.close()
        # CPU oracle: the scale-22 sources, plus bounded samples of the multi-source and closeness workloads
        c18, c23 = cgraphs["closeness_rmat18_all"], cgraphs["closeness_rmat23_16k"]
        cpu = cpu_baseline(rp, col, srcs, edges, learned_levels,
                           {"msbfs_rmat20": (mrp, mcol, msrcs[:64], "msbfs"),
                            "closeness_rmat18": (c18[0], c18[1], c18[2][::512], "closeness"),
                            "closeness_rmat23": (c23[0], c23[1], c23[2][:32], "closeness")})
        del cgraphs, c18, c23, mrp, mcol
        if not args.no_c3:
            # learned vs heuristic switch at full size on held-out graphs
            extras["c3_rmat24"] = c3_leg("rmat", 24, 1030, 1031, model, eta_tuned, torch, blest, inputs)
            extras["c3_er24"] = c3_leg("er", 24, 1032, 1033, model, eta_tuned, torch, blest, inputs)

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "R-MAT scale 22 edge factor 16 (a,b,c=.57,.19,.19, permuted; "
                                "relabelled by the build's JaccardWithWindows, W=1024), 64 sources one at a time",
                   "policy": policy, "sigma": info["sigma"], "tau": info["tau"], "sources": len(srcs)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
