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


def algorithmic_bytes(stats, n, nsets, sigma, slice_bytes, deg, levels):
    """Bytes a traversal must move, from its per-level log: init 4n + 2n/8;
    per step the engine's reads (BVSS over the queue: slice words + 16 B per
    queued VSS; BVSS over the panel copy: 4 B per slice slot + 4 B per
    256-slot chunk + the n/8 visited bytes read at the flush; push: 4 B per
    edge + 12 B per frontier vertex; bottom-up: 4 B per scanned edge + 8 B per
    unvisited vertex of nonzero degree) and the finalisation (n_hat mark bytes
    + 12 B per new vertex + 16 B per enqueued VSS + n/4 visited/frontier
    words)."""
    total = 4 * n + 2 * n // 8
    nhat = nsets * sigma
    lev = np.where(levels < 0, np.iinfo(np.int32).max, levels)
    for i, r in enumerate(stats[:-1]):
        eng = r["engine"]
        if eng == 0 and r.get("bvss_panel"):
            total += 4 * r["work"] + 4 * (r["work"] // 256) + n // 8
        elif eng == 0:
            total += slice_bytes * r["work"] + 16 * r["queue"]
        elif eng == 1:
            total += 4 * r["work"] + 12 * r["frontier"]
        else:
            unv_deg = int(((lev > r["level"]) & (deg > 0)).sum())
            total += 4 * r["work"] + 8 * unv_deg
        nxt = stats[i + 1]
        total += nhat + 12 * nxt["frontier"] + 16 * nxt["queue"] + n // 4
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


def cpu_baseline(rp, col, srcs, budget_s=20.0):
    """The oracle's queue BFS, one thread, on as many of the sources as fit the budget."""
    import oracle
    edges, times = [], []
    t_all = time.time()
    for s in srcs:
        t0 = time.perf_counter()
        lev = oracle.bfs(rp, col, int(s))
        t = time.perf_counter() - t0
        times.append(t * 1e3)
        edges.append(traversal_edges(rp, lev))
        if time.time() - t_all > budget_s:
            break
    return {"value": round(harmonic_gteps(edges, times), 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{len(times)} of the {len(srcs)} R-MAT scale-22 sources, FIFO-queue BFS on one host thread"}


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


def profile_leg(policy_name, n_sources=8):
    """A short run for rocprofv3: a 512 MiB device copy (counter calibration),
    then n_sources traversals of the scale-22 workload with one policy."""
    import torch
    from paper_2606_05081_amd import blest, inputs
    rp, col = inputs.rmat_graph(22, 1020)
    srcs = inputs.sources(rp, n_sources, seed=1021)
    g = blest.Graph(rp, col, device=0, **{"async": 1})
    a = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    c.copy_(a)
    torch.cuda.synchronize()
    try:
        g.set_policy(getattr(blest.Policy, policy_name.upper()))
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        ts = timed_sources(g, srcs, out, torch)
    finally:
        g.close()  # release device memory before the profiler's own exit handlers run
    print(json.dumps({"profile_leg": policy_name, "sources": n_sources, "ms_per_source": float(np.mean(ts)),
                      "calibration_copy_bytes": 2 * a.numel() * 4, "kernel_source_sha256_16": kernel_source_hash()}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sources", type=int, default=64)
    ap.add_argument("--no-extras", action="store_true", help="skip grid, msBFS and CPU legs")
    ap.add_argument("--profile-leg", choices=["heuristic", "bvss"], default=None,
                    help="only a short run of one policy plus a calibration copy, for rocprofv3")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is not built "
                                   "(see DESIGN.md, 'How the path would shard')", "n_gpus": args.gpus}))
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

    # exact edge counts per source (and a parity spot check against the certificate later)
    edges = []
    for s in srcs:
        g.set_policy(blest.Policy.HEURISTIC)
        g.bfs(int(s), out)
        g.sync()
        edges.append(traversal_edges(rp, out.cpu().numpy()))

    model = load_switch_model()
    policy = "heuristic"
    if model is not None:
        g.set_switch_model(np.array(model["params"], np.float32), np.array(model["mean"], np.float32),
                           np.array(model["std"], np.float32), model.get("min_confidence", 0.5))

    def run_policy(pol, steps, warmup):
        g.set_policy(pol, 10.0)
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
    learned_gteps, enabled, trial_ms = None, None, None
    value, step_ms = heur_gteps, heur_step_ms
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
        nb.append(algorithmic_bytes(st, info["n"], info["n_slice_sets"], info["sigma"],
                                    info["slice_bytes"], deg, lev))
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
        nb2.append(algorithmic_bytes(g.level_stats(), info["n"], info["n_slice_sets"], info["sigma"],
                                     info["slice_bytes"], deg, lev))
    sw_ach = float(np.mean(nb2)) / (float(np.mean(heur_t[:8])) * 1e-3) / 1e9
    g.set_log_work(False)

    extras = {"heuristic_gteps": round(heur_gteps, 3), "learned_gteps": None if learned_gteps is None else
              round(learned_gteps, 3), "learned_over_heuristic": None if learned_gteps is None else
              round(learned_gteps / heur_gteps, 4), "learned_enabled_by_trials": enabled,
              "trial_ms_per_source": None if trial_ms is None else {k: round(v, 4) for k, v in trial_ms.items()},
              "plain_method_gteps": round(td_gteps, 3),
              "ms_per_source": round(float(np.mean(heur_t)), 4), "switched_achieved_GBs": round(sw_ach, 1),
              "panel_step": None if not pan_b else {
                  "levels": len(pan_b), "GB_per_level": round(float(np.mean(pan_b)) / 1e9, 4),
                  "us_per_level": round(float(np.mean(pan_us)), 1),
                  "GBs": round(float(np.sum(pan_b)) / (float(np.sum(pan_us)) * 1e-6) / 1e9, 1)}}
    g.close()

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
        extras["grid2048_ms_per_source"] = round(float(np.mean(gt)), 3)
        extras["grid2048_gteps"] = round(harmonic_gteps(gedges, gt), 4)
        extras["grid2048_levels"] = len(gg.level_stats())
        gg.close()
        # batched multi-source BFS: scale-20 R-MAT, 960 sources, batches 64/128/256/512 in one launch
        mrp, mcol = inputs.rmat_graph(20, 1040)
        msrcs = inputs.sources(mrp, 960, seed=1041)
        mg = blest.Graph(mrp, mcol, device=0, **{"async": 1})
        mout = torch.empty((960, mg.n), dtype=torch.int16, device=dev)
        mg.msbfs_batched(msrcs, [64, 128, 256, 512], mout)
        mg.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        mg.msbfs_batched(msrcs, [64, 128, 256, 512], mout)
        e1.record()
        mg.sync()
        torch.cuda.synchronize()
        ms_ms = e0.elapsed_time(e1)
        extras["msbfs_sources_per_s"] = round(960 / ms_ms * 1e3, 1)
        extras["msbfs_ms"] = round(ms_ms, 3)
        per_width = {}
        for w in (64, 128, 256, 512):  # each batch width alone over the same 960 sources
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            mg.msbfs_batched(msrcs, [w], mout)
            e1.record()
            mg.sync()
            torch.cuda.synchronize()
            per_width[str(w)] = round(960 / e0.elapsed_time(e1) * 1e3, 1)
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
        mg.close()
        # the same 960 sources with the levels as a replayed hipGraph of per-phase kernels
        gmg = blest.Graph(mrp, mcol, device=0, msbfs_graph=1, **{"async": 1})
        gmg.msbfs_batched(msrcs, [64, 128, 256, 512], mout)
        gmg.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        gmg.msbfs_batched(msrcs, [64, 128, 256, 512], mout)
        e1.record()
        gmg.sync()
        torch.cuda.synchronize()
        extras["msbfs_graph_sources_per_s"] = round(960 / e0.elapsed_time(e1) * 1e3, 1)
        gmg.close()
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
        sg.close()
        # exact closeness: all sources of scale-18 R-MAT, 16,384 sources of scale-23 R-MAT (512 per
        # batch), with the pairs rule and with the multi-source switch network (per-graph enabled)
        ms_model = load_switch_model("switch_model_ms.json")
        for tag, scale, gseed, k in (("closeness_rmat18_all", 18, 1050, None), ("closeness_rmat23_16k", 23, 1052, 16384)):
            crp, ccol = inputs.rmat_graph(scale, gseed)
            cs = np.arange(crp.size - 1, dtype=np.int32) if k is None else inputs.sources(crp, k, seed=gseed + 1)
            cg = blest.Graph(crp, ccol, device=0, msbfs_width=512, **{"async": 1})
            res = {"sources": int(cs.size)}
            pols = [("heuristic", blest.Policy.HEURISTIC)]
            if ms_model is not None:
                cg.set_ms_switch_model(np.array(ms_model["params"], np.float32), np.array(ms_model["mean"], np.float32),
                                       np.array(ms_model["std"], np.float32), ms_model.get("min_confidence", 0.5))
                enabled, trial = ms_learned_enable(cg, inputs.sources(crp, 512, seed=gseed + 7), torch, blest)
                res["learned_enabled_by_trial"] = bool(enabled)
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
        cpu = cpu_baseline(rp, col, srcs)

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
