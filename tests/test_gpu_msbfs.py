"""Multi-source BFS and closeness on the GPU against the CPU oracle.

int16 levels and int64 sums/reach are exact integers (array equality); the
FP64 closeness is one IEEE division of exact integers on both sides, so it is
compared bit for bit (relative error 0 <= 1e-12)."""
import numpy as np
import pytest

import oracle
from paper_2606_05081_amd import inputs
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def blest():
    import torch
    from paper_2606_05081_amd import blest as b
    assert torch.cuda.is_available()
    b.lib()
    return b


POLICIES = ["HEURISTIC", "BVSS", "BOTTOM_UP", "RANDOM"]


@pytest.mark.parametrize("width", [64, 128, 256, 512])
def test_msbfs_rmat_all_widths_and_policies(blest, width):
    rp, col = inputs.rmat_graph(12, 51)
    srcs = inputs.sources(rp, 300, seed=52, distinct=False)  # ragged last batch, repeated sources
    ref = oracle.msbfs16(rp, col, srcs)
    g = blest.Graph(rp, col, msbfs_width=width)
    for pol in POLICIES:
        g.set_policy(getattr(blest.Policy, pol), 10.0, 7)
        got = g.msbfs(srcs).cpu().numpy()
        assert np.array_equal(got, ref), (pol, width, np.argwhere(got != ref)[:5])
    g.close()


def test_msbfs_uneven_batches_one_launch(blest):
    rp, col = inputs.rmat_graph(13, 61)
    srcs = inputs.sources(rp, 960, seed=62)
    ref = oracle.msbfs16(rp, col, srcs)
    g = blest.Graph(rp, col)
    got = g.msbfs_batched(srcs, [64, 128, 256, 512]).cpu().numpy()
    assert np.array_equal(got, ref)
    got = g.msbfs_batched(srcs[:100], [64]).cpu().numpy()
    assert np.array_equal(got, ref[:100])
    g.close()


@pytest.mark.parametrize("name", ["grid", "path", "hypercube", "disconnected", "tiny"])
def test_msbfs_structured(blest, name):
    if name == "grid":
        rp, col = inputs.grid_graph(60, 3)
    elif name == "path":
        rp, col = H.path(2000)
    elif name == "hypercube":
        rp, col = H.hypercube(10)
    elif name == "disconnected":
        rp, col = inputs.from_pairs(29, [0, 1, 2, 10, 11, 20], [1, 2, 3, 11, 12, 21])
    else:
        rp, col = inputs.from_pairs(3, [0], [1])
    n = rp.size - 1
    srcs = np.arange(n, dtype=np.int32) if n <= 300 else inputs.sources(rp, 200, seed=4)
    ref = oracle.msbfs16(rp, col, srcs)
    for opts in ({}, {"reorder": 1}, {"sigma": 16}, {"tau": 64}):
        g = blest.Graph(rp, col, **opts)
        for pol in POLICIES:
            g.set_policy(getattr(blest.Policy, pol), 10.0, 3)
            assert np.array_equal(g.msbfs(srcs).cpu().numpy(), ref), (name, opts, pol)
        g.close()


def test_msbfs_staging_grows_with_the_batch_width(blest):
    """The int16 levels go through a staging row per vertex that is sized for
    the widest batch seen so far: calls with growing and shrinking widths on a
    relabelled graph, with engines mixed per level, closeness in between (no
    levels), all equal the oracle."""
    rp, col = inputs.rmat_graph(13, 63)
    srcs = inputs.sources(rp, 700, seed=64)
    ref = oracle.msbfs16(rp, col, srcs)
    osum, oreach, _ = oracle.closeness(rp, col, srcs[:300])
    g = blest.Graph(rp, col)
    assert g.info()["reordered"] != 0
    for widths, pol in [([64], "BVSS"), ([512], "RANDOM"), ([128, 256], "BOTTOM_UP"), ([64, 512], "HEURISTIC")]:
        g.set_policy(getattr(blest.Policy, pol), 10.0, 5)
        got = g.msbfs_batched(srcs, widths).cpu().numpy()
        assert np.array_equal(got, ref), (widths, pol)
        s, r, _ = g.closeness(srcs[:300])
        assert np.array_equal(s.cpu().numpy(), osum) and np.array_equal(r.cpu().numpy(), oreach), (widths, pol)
    g.close()


def test_msbfs_overflow_and_errors(blest):
    rp, col = H.path(33000)
    g = blest.Graph(rp, col)
    with pytest.raises(blest.BlestError) as ei:
        g.msbfs([0, 5])
    assert ei.value.status == blest.Status.OVERFLOW
    ok = g.msbfs([16000]).cpu().numpy()  # still usable after the error
    assert np.array_equal(ok, oracle.msbfs16(rp, col, [16000]))
    with pytest.raises(blest.BlestError) as ei:
        g.msbfs([0, 33000])
    assert ei.value.status == blest.Status.OUT_OF_RANGE
    assert g.msbfs([]).shape == (0, 33000)
    g.close()


def test_closeness_matches_oracle(blest):
    for rp, col, k in [(*inputs.rmat_graph(12, 71), 700), (*inputs.grid_graph(40, 72), 300),
                       (*inputs.from_pairs(9, [0, 1, 4], [1, 2, 5]), 9)]:
        n = rp.size - 1
        srcs = np.arange(n, dtype=np.int32) if k >= n else inputs.sources(rp, k, seed=73, nonzero_degree=False)
        osum, oreach, occ = oracle.closeness(rp, col, srcs)
        g = blest.Graph(rp, col)
        for pol in POLICIES:
            g.set_policy(getattr(blest.Policy, pol), 10.0, 5)
            s, r, c = g.closeness(srcs)
            assert np.array_equal(s.cpu().numpy(), osum), pol
            assert np.array_equal(r.cpu().numpy(), oreach), pol
            assert np.array_equal(c.cpu().numpy(), occ), pol  # bit-identical doubles
        g.close()


def test_closeness_all_sources_equals_per_target_far(blest):
    rp, col = inputs.rmat_graph(11, 81)
    n = rp.size - 1
    allv = np.arange(n, dtype=np.int32)
    g = blest.Graph(rp, col)
    s, _, _ = g.closeness(allv)
    ofar = oracle.far(rp, col, allv)
    assert np.array_equal(s.cpu().numpy(), ofar)
    assert np.array_equal(g.far(allv).cpu().numpy(), ofar)  # Eq. 4 on the device: equal when S = V
    g.close()


@pytest.mark.parametrize("graph_mode", [0, 1])
def test_per_target_far_subsets(blest, graph_mode):
    """Eq. 4's per-target sums for source subsets (repeats count twice),
    relabelled graphs and several batch widths."""
    for rp, col, opts in [(*inputs.rmat_graph(12, 91), {}), (*inputs.grid_graph(40, 92), {"reorder": 1}),
                          (*inputs.rmat_graph(12, 93), {"msbfs_width": 64}),
                          (*inputs.from_pairs(9, [0, 1, 4], [1, 2, 5]), {})]:
        n = rp.size - 1
        srcs = inputs.sources(rp, min(n, 300), seed=94, nonzero_degree=False, distinct=False)
        g = blest.Graph(rp, col, msbfs_graph=graph_mode, **opts)
        assert np.array_equal(g.far(srcs).cpu().numpy(), oracle.far(rp, col, srcs))
        assert np.array_equal(g.far([]).cpu().numpy(), np.zeros(n, np.int64))
        g.close()


def test_msbfs_full_size_rmat20_sampled_rows(blest):
    """Scale-20 R-MAT, 960 sources in batches of 64/128/256/512 (one launch)."""
    rp, col = inputs.rmat_graph(20, 1040)
    srcs = inputs.sources(rp, 960, seed=1041)
    g = blest.Graph(rp, col)
    got = g.msbfs_batched(srcs, [64, 128, 256, 512])
    rows = [0, 63, 64, 191, 192, 447, 448, 959]
    for r in rows:
        lev = got[r].cpu().numpy().astype(np.int32)
        assert np.array_equal(lev, oracle.bfs(rp, col, int(srcs[r]))), r
    got = got.cpu().numpy()
    for r in range(5, 960, 15):  # 64 more rows, spread over all four batches
        lev = got[r].astype(np.int32)
        assert oracle.certificate(rp, col, int(srcs[r]), lev) == (0, -1), r
    g.close()


def test_er18_msbfs_and_closeness_every_policy(blest):
    """Erdos-Renyi, 2^18 vertices, mean degree 16 (no hubs, no dense
    low-degree levels the R-MAT-trained switch has seen): multi-source levels,
    sums, reach and closeness exact under every policy, the multi-source
    switch network included."""
    rp, col = inputs.er_graph(18, 2321)
    srcs = inputs.sources(rp, 700, seed=2322)
    ref = oracle.msbfs16(rp, col, srcs)
    osum, oreach, occ = oracle.closeness(rp, col, srcs)
    g = blest.Graph(rp, col)
    H.install_switch_models(g)
    for pol in POLICIES + ["LEARNED"]:
        g.set_policy(getattr(blest.Policy, pol), 10.0, 3)
        assert np.array_equal(g.msbfs_batched(srcs, [64, 128, 256, 512]).cpu().numpy(), ref), pol
        s_, r_, c_ = g.closeness(srcs)
        assert np.array_equal(s_.cpu().numpy(), osum), pol
        assert np.array_equal(r_.cpu().numpy(), oreach), pol
        assert np.array_equal(c_.cpu().numpy(), occ), pol
    g.close()


def test_closeness_rmat18_subset(blest):
    """Scale-18 R-MAT closeness on a 512-source subset of all vertices."""
    rp, col = inputs.rmat_graph(18, 1050)
    srcs = np.arange(0, rp.size - 1, 512, dtype=np.int32)
    osum, oreach, occ = oracle.closeness(rp, col, srcs)
    g = blest.Graph(rp, col)
    s, r, c = g.closeness(srcs)
    assert np.array_equal(s.cpu().numpy(), osum)
    assert np.array_equal(r.cpu().numpy(), oreach)
    assert np.array_equal(c.cpu().numpy(), occ)
    g.close()


def _component_sizes(rp, col):
    lab = oracle.components(rp, col)
    return np.bincount(lab)[lab]


@pytest.mark.parametrize("which", ["rmat18_all", "rmat23_16k"])
def test_closeness_full_size(blest, which):
    """The closeness workloads at full size: all 262,144 sources of scale-18
    R-MAT, and 16,384 seeded sources of scale-23 R-MAT (512 per batch). Every
    source's reach equals its component size, every cc is
    (reach-1)/sum in IEEE double (0 when sum = 0), and sampled sources' sums
    equal the oracle's. Component sizes come from the oracle's labelling."""
    if which == "rmat18_all":
        rp, col = inputs.rmat_graph(18, 1050)
        srcs = np.arange(rp.size - 1, dtype=np.int32)
        sample = srcs[::4099]
    else:
        rp, col = inputs.rmat_graph(23, 1052)
        srcs = inputs.sources(rp, 16384, seed=1053)
        sample = srcs[::64]  # 256 sources, every batch of 512 contributes eight
    print(f"[{which}] n={rp.size - 1} m={col.size} k={srcs.size}", flush=True)
    g = blest.Graph(rp, col, msbfs_width=512)
    s, r, c = g.closeness(srcs)
    s, r, c = s.cpu().numpy(), r.cpu().numpy(), c.cpu().numpy()
    g.close()
    comp = _component_sizes(rp, col)
    assert np.array_equal(r, comp[srcs])
    assert np.array_equal(s == 0, r == 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        want = np.where(s > 0, (r - 1).astype(np.float64) / s.astype(np.float64), 0.0)
    assert np.array_equal(c, want)
    idx = np.searchsorted(srcs, sample) if which == "rmat18_all" else np.arange(0, srcs.size, 64)
    osum, oreach, occ = oracle.closeness(rp, col, sample)
    assert np.array_equal(s[idx], osum)
    assert np.array_equal(r[idx], oreach)
    assert np.array_equal(c[idx], occ)


@pytest.mark.parametrize("name", ["rmat13", "grid60", "path2000", "disconnected"])
def test_msbfs_graph_mode(blest, name):
    """msbfs_graph=1: per-phase kernels captured in a hipGraph and replayed
    (many replays per call, the graph object reused across calls) give the same
    levels and closeness as the oracle, for uneven batches and every policy."""
    if name == "rmat13":
        rp, col = inputs.rmat_graph(13, 61)
    elif name == "grid60":
        rp, col = inputs.grid_graph(60, 3)
    elif name == "path2000":
        rp, col = H.path(2000)
    else:
        rp, col = inputs.from_pairs(29, [0, 1, 2, 10, 11, 20], [1, 2, 3, 11, 12, 21])
    n = rp.size - 1
    srcs = np.arange(n, dtype=np.int32) if n <= 300 else inputs.sources(rp, 300, seed=4)
    ref = oracle.msbfs16(rp, col, srcs)
    g = blest.Graph(rp, col, msbfs_graph=1)
    for pol in POLICIES:
        g.set_policy(getattr(blest.Policy, pol), 10.0, 3)
        got = g.msbfs_batched(srcs, [64, 128, 256, 512]).cpu().numpy()
        assert np.array_equal(got, ref), (name, pol)
    osum, oreach, occ = oracle.closeness(rp, col, srcs)
    s, r, c = g.closeness(srcs)
    assert np.array_equal(s.cpu().numpy(), osum)
    assert np.array_equal(r.cpu().numpy(), oreach)
    assert np.array_equal(c.cpu().numpy(), occ)
    # one captured graph served every call: each policy's, and closeness with
    # its different outputs (these policies share the kernel and LDS size)
    assert g.info()["ms_graph_captures"] == 1
    g.close()


def test_msbfs_graph_mode_overflow(blest):
    rp, col = H.path(33000)
    g = blest.Graph(rp, col, msbfs_graph=1)
    with pytest.raises(blest.BlestError) as ei:
        g.msbfs([0, 5])
    assert ei.value.status == blest.Status.OVERFLOW
    assert np.array_equal(g.msbfs([16000]).cpu().numpy(), oracle.msbfs16(rp, col, [16000]))
    g.close()


def _random_model(seed):
    """Untrained weights scaled so the network is often confident; std 8 keeps
    every standardised feature of these graphs inside [-6, 6]."""
    from paper_2606_05081_amd import switch
    params = (switch.init_params(seed) * 4.0).astype(np.float32)
    return params, np.zeros(12, np.float32), np.full(12, 8.0, np.float32)


def test_msbfs_probe_levels_and_records(blest):
    rp, col = inputs.rmat_graph(13, 61)
    srcs = inputs.sources(rp, 300, seed=62)
    ref = oracle.msbfs16(rp, col, srcs)
    g = blest.Graph(rp, col)
    got = g.msbfs_probe(srcs, [64, 128, 256]).cpu().numpy()
    assert np.array_equal(got, ref)
    recs = g.ms_level_stats()
    # one record per level of every batch (64, 128, then the last 108 sources)
    nb = [64, 128, 108]
    per_batch = [int(ref[sum(nb[:b]):sum(nb[:b + 1])].max()) + 1 for b in range(3)]
    assert [sum(1 for r in recs if r["batch"] == b) for b in range(3)] == per_batch
    assert all(min(r["t_engine_us"]) > 0 for r in recs)
    assert all(np.isfinite(r["feat"]).all() for r in recs)
    assert [r["width"] for r in recs if r["level"] == 0] == nb
    # new pairs per level equal the oracle's level counts; live traversals are
    # those with a vertex at that level
    for b in range(3):
        rows = ref[sum(nb[:b]):sum(nb[:b + 1])]
        rb = [r for r in recs if r["batch"] == b]
        assert [r["new_pairs"] for r in rb] == [int((rows == l).sum()) for l in range(per_batch[b])]
        assert [r["live"] for r in rb] == [int((rows == l).any(axis=1).sum()) for l in range(per_batch[b])]
    g.close()


@pytest.mark.parametrize("graph_mode", [0, 1])
def test_msbfs_dead_traversals(blest, graph_mode):
    """Sources in small components (isolated vertices, short paths) finish
    after a level or two; the bottom-up engine then ignores their bits. Every
    policy must still match the oracle, and the live counts must drop."""
    rp0, col0 = inputs.rmat_graph(12, 81)
    n0 = rp0.size - 1
    src = np.repeat(np.arange(n0), np.diff(rp0))
    keep = src < col0
    extra_u = [n0, n0 + 1, n0 + 3]
    extra_v = [n0 + 1, n0 + 2, n0 + 4]
    rp, col = inputs.from_pairs(n0 + 6, np.concatenate([src[keep], extra_u]),
                                np.concatenate([col0[keep], extra_v]))
    assert np.array_equal(np.diff(rp)[:n0], np.diff(rp0))
    big = inputs.sources(rp0, 120, seed=82)
    small = np.array([n0, n0 + 2, n0 + 3, n0 + 5], np.int32)  # path ends, an edge, an isolated vertex
    srcs = np.concatenate([small[:2], big[:60], small[2:], big[60:]]).astype(np.int32)
    ref = oracle.msbfs16(rp, col, srcs)
    g = blest.Graph(rp, col, msbfs_graph=graph_mode)
    for pol in POLICIES:
        g.set_policy(getattr(blest.Policy, pol), 10.0, 5)
        got = g.msbfs_batched(srcs, [64]).cpu().numpy()
        assert np.array_equal(got, ref), (pol, np.argwhere(got != ref)[:5])
        recs = [r for r in g.ms_level_stats() if r["batch"] == 0]
        rows = ref[:64]
        assert [r["live"] for r in recs] == [int((rows == l).any(axis=1).sum()) for l in range(len(recs))]
        assert recs[0]["live"] == 64 and recs[2]["live"] <= 62
    g.close()


@pytest.mark.parametrize("graph_mode", [0, 1])
def test_msbfs_learned_policy_exact_and_inference(blest, graph_mode):
    """Policy LEARNED with arbitrary weights changes only the engines, never
    the results; the engine recorded per level is the oracle network's choice
    (pairs rule where the network declines: confidence or non-BVSS/BU output)."""
    from oracle import mlp as omlp
    rp, col = inputs.rmat_graph(13, 71)
    srcs = inputs.sources(rp, 400, seed=72)
    ref = oracle.msbfs16(rp, col, srcs)
    osum, oreach, occ = oracle.closeness(rp, col, srcs)
    blest.blest_set_switch_confidence(None, 0.5)
    used = {0: 0, 1: 0}
    for seed in (1, 2, 3):
        params, mean, std = _random_model(seed)
        g = blest.Graph(rp, col, msbfs_graph=graph_mode)
        g.set_ms_switch_model(params, mean, std)
        g.set_policy(blest.Policy.LEARNED)
        got = g.msbfs_batched(srcs, [64, 256, 512]).cpu().numpy()
        assert np.array_equal(got, ref), seed
        recs = g.ms_level_stats()
        for r in recs:
            z = (np.asarray(r["feat"], np.float64) - mean) / std
            logits, _ = omlp.forward(params.astype(np.float64), z[None, :])
            lg = logits[0]
            p = np.exp(lg - lg.max())
            p /= p.sum()
            c = int(np.argmax(lg))
            rule = 2 if r["unvisited_pairs"] < 10.0 * r["queue"] else 0
            ood = (np.abs(z) > 6).any()
            sure = p.max() >= 0.5 + 1e-4
            if not ood and sure and c in (0, 2) and abs(np.sort(lg)[-1] - np.sort(lg)[-2]) > 1e-4:
                assert r["engine"] == c and r["mlp_fallback"] == 0, r
                used[0] += 1
            elif ood or p.max() < 0.5 - 1e-4 or c == 1:
                assert r["engine"] == rule and r["mlp_fallback"] == 1, r
                used[1] += 1
        s, rr, cc = g.closeness(srcs)
        assert np.array_equal(s.cpu().numpy(), osum)
        assert np.array_equal(rr.cpu().numpy(), oreach)
        assert np.array_equal(cc.cpu().numpy(), occ)
        g.close()
    assert used[0] > 0 and used[1] > 0, used


def test_closeness_resumable_checkpoint(blest, tmp_path):
    """A closeness run cut into pieces by max_sources resumes from its
    checkpoint file and ends with the oracle's results; a file written for
    another source list is refused."""
    rp, col = inputs.rmat_graph(12, 101)
    srcs = inputs.sources(rp, 700, seed=102)
    osum, oreach, occ = oracle.closeness(rp, col, srcs)
    g = blest.Graph(rp, col, msbfs_width=64)  # chunks of 64 batches = 4096 sources
    path = str(tmp_path / "cc.ckpt")
    s, r, c, done = g.closeness_resumable(srcs, path, max_sources=300)
    assert done == 300
    assert np.array_equal(s.cpu().numpy()[:300], osum[:300]) and np.array_equal(r.cpu().numpy()[:300], oreach[:300])
    s, r, c, done = g.closeness_resumable(srcs, path, max_sources=250)
    assert done == 550
    s, r, c, done = g.closeness_resumable(srcs, path)
    assert done == 700
    assert np.array_equal(s.cpu().numpy(), osum) and np.array_equal(r.cpu().numpy(), oreach)
    assert np.array_equal(c.cpu().numpy(), occ)
    # a finished file gives the results without new work
    s, r, c, done = g.closeness_resumable(srcs, path, max_sources=1)
    assert done == 700 and np.array_equal(c.cpu().numpy(), occ)
    with pytest.raises(blest.BlestError) as ei:
        g.closeness_resumable(srcs[::-1].copy(), path)
    assert ei.value.status == blest.Status.INVALID_ARG
    g.close()


@pytest.mark.parametrize("ablation", [1, 2, 3])
def test_ablation_variants_exact(blest, ablation):
    """The multi-source ablation steps (no getVI remap, no dynamic slice-set
    tracking, neither) change the work, never the results."""
    for rp, col in [inputs.rmat_graph(12, 2401), inputs.grid_graph(50, 2402)]:
        srcs = inputs.sources(rp, 200, seed=2403)
        ref = oracle.msbfs16(rp, col, srcs)
        osum, oreach, occ = oracle.closeness(rp, col, srcs)
        g = blest.Graph(rp, col, ms_ablation=ablation)
        for pol in ("HEURISTIC", "BVSS", "BOTTOM_UP"):
            g.set_policy(getattr(blest.Policy, pol), 10.0)
            assert np.array_equal(g.msbfs_batched(srcs, [64, 128]).cpu().numpy(), ref), (ablation, pol)
            s_, r_, c_ = g.closeness(srcs)
            assert np.array_equal(s_.cpu().numpy(), osum) and np.array_equal(r_.cpu().numpy(), oreach)
            assert np.array_equal(c_.cpu().numpy(), occ)
        g.close()


@pytest.mark.parametrize("wide", [0, 1])
def test_mfma_neighbour_check_exact(blest, wide):
    """The multi-source top-down check as an int8 matrix product on the matrix
    cores (opts.ms_mfma): identical levels, sums, reach and closeness."""
    for rp, col in [inputs.rmat_graph(12, 2501), inputs.grid_graph(40, 2502), H.hypercube(9)]:
        srcs = inputs.sources(rp, 300, seed=2503, distinct=False)
        ref = oracle.msbfs16(rp, col, srcs)
        osum, oreach, occ = oracle.closeness(rp, col, srcs)
        g = blest.Graph(rp, col, ms_mfma=1, wide_slices=wide)
        for pol in ("BVSS", "HEURISTIC", "RANDOM"):
            g.set_policy(getattr(blest.Policy, pol), 10.0, 4)
            assert np.array_equal(g.msbfs_batched(srcs, [64, 128, 256, 512]).cpu().numpy(), ref), pol
            s_, r_, c_ = g.closeness(srcs)
            assert np.array_equal(s_.cpu().numpy(), osum) and np.array_equal(r_.cpu().numpy(), oreach)
            assert np.array_equal(c_.cpu().numpy(), occ)
        g.close()
