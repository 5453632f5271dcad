"""Single-source BFS on the GPU, through the C ABI, against the CPU oracle.

Levels are integers with one correct value, so every comparison is exact
(array equality). Sizes span many wavefront tiles and ragged tails; the
full-size workloads (R-MAT scale 22, 2048x2048 grid) are checked exactly on
sampled sources and by the O(m) distance certificate.
"""
import numpy as np
import pytest

import oracle
from paper_2606_05081_amd import inputs
from tests import helpers as H

pytestmark = pytest.mark.gpu

POLICIES = ["HEURISTIC", "BVSS", "PUSH", "BOTTOM_UP", "RANDOM"]


@pytest.fixture(scope="module")
def blest():
    import torch
    from paper_2606_05081_amd import blest as b
    assert torch.cuda.is_available()
    b.lib()
    return b


def _lazy(blest, rp, col, **opt):
    """A graph on the lazy scheme (Alg. 3): every test of its machinery (panel
    copy, Stage 2 variants, single-workgroup levels) must run it even where the
    update-divergence dispatch would pick the eager kernel (small graphs)."""
    return blest.Graph(rp, col, **{"update_scheme": blest.Update.LAZY, **opt})


def run_all_policies(blest, g, src, ref, seeds=(1, 2, 3)):
    for pol in POLICIES:
        for sd in (seeds if pol == "RANDOM" else (1,)):
            g.set_policy(getattr(blest.Policy, pol), 10.0, sd)
            lev = g.bfs(src).cpu().numpy()
            assert np.array_equal(lev, ref), (pol, sd, src, np.nonzero(lev != ref)[0][:10])


@pytest.mark.parametrize("name", ["path", "cycle", "star", "hypercube", "grid40perm", "bipartite", "gnp"])
def test_closed_form_families(blest, name):
    if name == "path":
        rp, col = H.path(1000)
    elif name == "cycle":
        rp, col = H.cycle(777)
    elif name == "star":
        rp, col = H.star(3000)
    elif name == "hypercube":
        rp, col = H.hypercube(12)
    elif name == "grid40perm":
        rp0, col0 = inputs.grid(40, 0.0, seed=1, permute=False)
        rp, col, _ = inputs.permute(rp0, col0, seed=3)
    elif name == "bipartite":
        rp, col = H.complete_bipartite(37, 91)
    else:
        rp, col = H.gnp(300, 0.02, 5)
    g = _lazy(blest, rp, col)
    n = rp.size - 1
    for src in {0, n // 3, n - 1}:
        run_all_policies(blest, g, src, oracle.bfs(rp, col, src))
    g.close()


def test_rmat_s16_all_policies(blest):
    """Scale-16 R-MAT (65,536 vertices, edge factor 16, a,b,c = .57,.19,.19)."""
    rp, col = inputs.rmat_graph(16, 1010)
    g = _lazy(blest, rp, col)
    srcs = inputs.sources(rp, 4, seed=1011)
    for s in srcs:
        run_all_policies(blest, g, int(s), oracle.bfs(rp, col, int(s)))
    g.close()


@pytest.mark.parametrize("opt", [
    dict(sigma=16), dict(sigma=32), dict(tau=64), dict(tau=256), dict(tau=192), dict(wide_slices=1),
    dict(block_size=256), dict(block_size=1024), dict(persistent=0), dict(prefilter=0), dict(reorder=1),
    dict(reorder=0), dict(blocks_per_cu=1), dict(sigma=16, tau=64, block_size=256, persistent=0),
    dict(single_block=0), dict(single_block=0, block_size=1024), dict(block_size=256, sigma=32),
    dict(panel=0), dict(panel=2), dict(panel=2, block_size=256), dict(panel=2, persistent=0),
    dict(panel=2, blocks_per_cu=1, single_block=0),
    dict(stage2_count_first=0), dict(stage2_count_first=2), dict(stage2_count_first=2, single_block=0, panel=0),
    dict(reorder=3), dict(reorder=3, jaccard_window=64, panel=2),
])
def test_option_matrix(blest, opt):
    for rp, col in [inputs.rmat_graph(13, 77), inputs.grid_graph(70, 78)]:
        g = _lazy(blest, rp, col, **opt)
        for s in inputs.sources(rp, 2, seed=79):
            run_all_policies(blest, g, int(s), oracle.bfs(rp, col, int(s)), seeds=(4,))
        g.close()


@pytest.mark.parametrize("name", ["path", "star", "hypercube", "grid40perm", "gnp", "rmat12", "tiny"])
def test_panel_copy_every_bvss_level(blest, name):
    """panel=2: every BVSS level reads the panel-blocked copy (LDS marks,
    stale frontier words filtered at the flush); levels must not change."""
    if name == "path":
        rp, col = H.path(1000)
    elif name == "star":
        rp, col = H.star(3000)
    elif name == "hypercube":
        rp, col = H.hypercube(12)
    elif name == "grid40perm":
        rp0, col0 = inputs.grid(40, 0.0, seed=1, permute=False)
        rp, col, _ = inputs.permute(rp0, col0, seed=3)
    elif name == "gnp":
        rp, col = H.gnp(300, 0.02, 5)
    elif name == "rmat12":
        rp, col = inputs.rmat_graph(12, 88)
    else:
        rp, col = inputs.from_pairs(13, [0, 1, 2, 5, 6], [1, 2, 3, 6, 7])
    g = _lazy(blest, rp, col, panel=2)
    assert g.info()["panel_log2_rows"] >= 5
    n = rp.size - 1
    for src in sorted({0, n // 3, n - 1}):
        ref = oracle.bfs(rp, col, src)
        for pol in ("BVSS", "HEURISTIC", "RANDOM"):
            g.set_policy(getattr(blest.Policy, pol), 10.0, 9)
            lev = g.bfs(src).cpu().numpy()
            assert np.array_equal(lev, ref), (name, pol, src)
        g.set_policy(blest.Policy.BVSS, 10.0)
        g.bfs(src)
        st = g.level_stats()
        assert all(r["bvss_panel"] == 1 for r in st[:-1]), (name, src)
    g.close()


def test_edge_cases(blest):
    # ragged n (not a multiple of sigma), isolated source, unreachable parts
    rp, col = inputs.from_pairs(13, [0, 1, 2, 5, 6], [1, 2, 3, 6, 7])
    g = _lazy(blest, rp, col)
    for s in range(13):
        run_all_policies(blest, g, s, oracle.bfs(rp, col, s))
    g.close()
    # no edges at all
    rp, col = inputs.from_pairs(9, [], [])
    g = _lazy(blest, rp, col)
    run_all_policies(blest, g, 4, oracle.bfs(rp, col, 4))
    g.close()
    # a single vertex
    g = _lazy(blest, np.array([0, 0], np.int32), np.zeros(0, np.int32))
    assert g.bfs(0).cpu().tolist() == [0]
    g.close()


def test_errors(blest):
    rp, col = H.path(10)
    g = _lazy(blest, rp, col)
    for bad in (-1, 10, 1 << 30):
        with pytest.raises(blest.BlestError) as ei:
            g.bfs(bad)
        assert ei.value.status == blest.Status.OUT_OF_RANGE
    assert np.array_equal(g.bfs(3).cpu().numpy(), np.abs(np.arange(10) - 3))  # still usable
    g.close()


def test_bvss_export_matches_oracle_and_fig1(blest, golden):
    from tests.test_oracle_pins import bits_lsb_first, fig1_graph
    fig = golden("fig1_bvss.txt")
    rp, col = fig1_graph()
    g = _lazy(blest, rp, col, tau=64, reorder=0)
    b = g.export_bvss()
    ob = oracle.bvss(rp, col, 8, 64)
    for k in ("real_ptrs", "v2r", "slice_ptr", "slice_row", "slice_mask"):
        assert np.array_equal(b[k].astype(np.int64), ob[k].astype(np.int64)), k
    lo, hi = b["slice_ptr"][2], b["slice_ptr"][3]
    rows = b["slice_row"][lo:hi].tolist()
    assert int(b["slice_mask"][lo + rows.index(3)]) == bits_lsb_first(fig["mask_row3_set2"][0])
    lev = g.bfs(17).cpu().numpy()
    assert lev[3] == 1
    g.close()
    for sigma, tau, wide in [(8, 128, 0), (8, 256, 1), (16, 64, 1), (32, 192, 1)]:
        rp, col = inputs.rmat_graph(11, 5)
        g = _lazy(blest, rp, col, sigma=sigma, tau=tau, wide_slices=wide, reorder=0)
        b = g.export_bvss()
        ob = oracle.bvss(rp, col, sigma, tau)
        for k in ("real_ptrs", "v2r", "slice_ptr", "slice_row", "slice_mask"):
            assert np.array_equal(b[k].astype(np.int64), ob[k].astype(np.int64)), (k, sigma, tau)
        g.close()


def test_rcm_export_is_bvss_of_permuted_graph(blest):
    rp, col = inputs.grid_graph(50, 9)
    g = _lazy(blest, rp, col, reorder=1)
    b = g.export_bvss()
    assert g.info()["reordered"] == 1
    perm = b["perm"]
    assert sorted(perm.tolist()) == list(range(rp.size - 1))
    # relabel the input by perm and rebuild the oracle BVSS
    n = rp.size - 1
    u = np.repeat(np.arange(n), np.diff(rp))
    rp2, col2 = inputs.from_pairs(n, perm[u], perm[col])
    ob = oracle.bvss(rp2, col2, 8, 128)
    for k in ("real_ptrs", "slice_ptr", "slice_row", "slice_mask"):
        assert np.array_equal(b[k].astype(np.int64), ob[k].astype(np.int64)), k
    g.close()


@pytest.mark.parametrize("single", [1, 0])
def test_level_log_matches_oracle_counts_and_eq3_replay(blest, single):
    for rp, col in [inputs.rmat_graph(16, 1010), inputs.grid_graph(96, 4)]:
        g = _lazy(blest, rp, col, reorder=0, single_block=single)
        b = g.export_bvss()
        for s in inputs.sources(rp, 3, seed=12):
            s = int(s)
            g.set_policy(blest.Policy.HEURISTIC, 10.0)
            g.bfs(s)
            ref = oracle.bfs(rp, col, s)
            stats = g.level_stats()
            cnt = oracle.level_counts(ref)
            assert [r["frontier"] for r in stats] == cnt.tolist()
            rep = oracle.switch_replay(ref, rp, b["real_ptrs"], 8, eta=10.0)
            assert [r["queue"] for r in stats] == [r["queue"] for r in rep]
            assert [r["unvisited"] for r in stats] == [r["unvisited"] for r in rep]
            dec = [r["engine"] == blest.Engine.BOTTOM_UP for r in stats[:-1]]
            assert dec == [r["bottom_up"] for r in rep[:-1]]
            deg = np.diff(rp)
            for r in stats:
                fr = ref == r["level"]
                assert r["frontier_edges"] == int(deg[fr].sum())
                assert r["deg_ge_32"] == int((deg[fr] >= 32).sum())
        g.close()


def test_relabelling_equivariance(blest):
    rp, col = inputs.rmat_graph(14, 31)
    rp2, col2, perm = inputs.permute(rp, col, seed=32)
    g1, g2 = _lazy(blest, rp, col), _lazy(blest, rp2, col2)
    for s in inputs.sources(rp, 3, seed=33):
        a = g1.bfs(int(s)).cpu().numpy()
        b = g2.bfs(int(perm[s])).cpu().numpy()
        assert np.array_equal(b[perm], a)
    g1.close()
    g2.close()


def test_probe_mode_same_levels_and_times(blest):
    rp, col = inputs.rmat_graph(15, 41)
    g = _lazy(blest, rp, col)
    s = int(inputs.sources(rp, 1, seed=42)[0])
    lev = g.bfs_probe(s).cpu().numpy()
    assert np.array_equal(lev, oracle.bfs(rp, col, s))
    st = g.level_stats()
    assert all(min(r["t_engine_us"]) > 0 for r in st[:-1])
    g.close()


@pytest.mark.parametrize("which", ["rmat22", "grid2048"])
def test_full_size_sampled_sources(blest, which):
    """The single-GPU workload at full size: 4,194,304-vertex R-MAT (scale 22,
    edge factor 16) and 2048x2048 grid with 10% edge deletion (RCM-reordered),
    under every policy the benchmark times or the learned switch may pick:
    certificate on three sources, oracle equality on the first."""
    if which == "rmat22":
        rp, col = inputs.rmat_graph(22, 1020)
        srcs = inputs.sources(rp, 64, seed=1021)
    else:
        rp, col = inputs.grid_graph(2048, 1022)
        srcs = inputs.sources(rp, 64, seed=1023)
    print(f"[{which}] n={rp.size - 1} m={col.size}", flush=True)
    g = blest.Graph(rp, col)
    H.install_switch_models(g, multi=False)
    pols = ("HEURISTIC", "BVSS", "LEARNED", "PUSH") if which == "rmat22" else ("HEURISTIC", "BVSS", "LEARNED")
    for i, s in enumerate(srcs[:3]):
        s = int(s)
        ref = oracle.bfs(rp, col, s) if i == 0 else None
        for pol in pols:
            g.set_policy(getattr(blest.Policy, pol), 10.0)
            lev = g.bfs(s).cpu().numpy()
            assert oracle.certificate(rp, col, s, lev) == (0, -1), pol
            if ref is not None:
                assert np.array_equal(lev, ref), pol
            if which == "rmat22" and pol == "BVSS":
                # the dense levels of the plain method read the panel-blocked copy
                assert any(r["bvss_panel"] for r in g.level_stats()[:-1])
    g.close()
    if which == "grid2048":
        # the dispatch runs the grid on the eager kernel; the lazy scheme at full size too
        g = _lazy(blest, rp, col)
        s = int(srcs[0])
        for pol in ("HEURISTIC", "BVSS"):
            g.set_policy(getattr(blest.Policy, pol), 10.0)
            lev = g.bfs(s).cpu().numpy()
            assert oracle.certificate(rp, col, s, lev) == (0, -1), pol
        g.close()


# Learned vs heuristic switch workloads at full size: R-MAT scale 24 (16.8M
# vertices, edge factor 16) and Erdos-Renyi with 2^24 vertices and 8 * 2^24
# uniform pairs. At 2^24 vertices the packed 32-bit slice word reaches its
# 24-bit row limit and the panel layout holds more panels than workgroups.
_C3 = {}


@pytest.fixture(scope="module", params=["rmat24", "er24"])
def c3_graph(request, blest):
    which = request.param
    if which == "rmat24":
        rp, col = inputs.rmat_graph(24, 1030)
        srcs = inputs.sources(rp, 3, seed=1031)
    else:
        rp, col = inputs.er_graph(24, 1032)
        srcs = inputs.sources(rp, 3, seed=1033)
    print(f"[{which}] n={rp.size - 1} m={col.size}", flush=True)
    g = blest.Graph(rp, col)
    H.install_switch_models(g, multi=False)
    info = g.info()
    ref = oracle.bfs(rp, col, int(srcs[0]))
    yield which, rp, col, srcs, g, info, ref
    g.close()


@pytest.mark.parametrize("pol", ["HEURISTIC", "LEARNED", "BVSS"])
def test_c3_full_size(blest, c3_graph, pol):
    which, rp, col, srcs, g, info, ref = c3_graph
    assert info["slice_bytes"] == 4  # the 32-bit (row << 8 | mask) form at its 24-bit row limit
    g.set_policy(getattr(blest.Policy, pol), 10.0)
    for i, s in enumerate(srcs):
        s = int(s)
        lev = g.bfs(s).cpu().numpy()
        print(f"[{which} {pol}] source {s}: {int(lev.max()) + 1} levels", flush=True)
        assert oracle.certificate(rp, col, s, lev) == (0, -1), (which, pol, s)
        if i == 0:
            assert np.array_equal(lev, ref), (which, pol)
        if pol == "BVSS" and which == "rmat24":
            assert any(r["bvss_panel"] for r in g.level_stats()[:-1])


def test_er20_every_policy(blest):
    """Erdos-Renyi, 2^20 vertices, mean degree 16: every policy exact."""
    rp, col = inputs.er_graph(20, 2301)
    g = blest.Graph(rp, col)
    H.install_switch_models(g, multi=False)
    for s in inputs.sources(rp, 2, seed=2302):
        ref = oracle.bfs(rp, col, int(s))
        run_all_policies(blest, g, int(s), ref, seeds=(5, 6))
        g.set_policy(blest.Policy.LEARNED, 10.0)
        assert np.array_equal(g.bfs(int(s)).cpu().numpy(), ref)
    g.close()


@pytest.mark.parametrize("panel", [1, 2])
def test_more_panels_than_workgroups(blest, panel):
    """32-row panels on scale-14 R-MAT: 512 panels, so each persistent
    workgroup owns several and runs the fused Stage 2 once per panel."""
    rp, col = inputs.rmat_graph(14, 2311)
    g = _lazy(blest, rp, col, panel=panel, panel_log2_rows=5)
    info = g.info()
    assert info["panel_log2_rows"] == 5 and (info["n"] >> 5) > info["grid_blocks"]
    for s in inputs.sources(rp, 3, seed=2312):
        ref = oracle.bfs(rp, col, int(s))
        run_all_policies(blest, g, int(s), ref, seeds=(8,))
        g.set_policy(blest.Policy.BVSS, 10.0)
        g.bfs(int(s))
        assert any(r["bvss_panel"] for r in g.level_stats()[:-1])
    g.close()


def test_jaccard_reordering_exact_and_compresses(blest):
    """JaccardWithWindows relabelling (Section "Increasing Compression
    Ratio"): fewer slices than the input order on R-MAT, and every output is
    still in input ids and exact (the relabelling only changes the BVSS)."""
    import oracle.jaccard as J
    rp, col = inputs.rmat_graph(13, 91)
    base = _lazy(blest, rp, col, reorder=0)
    g = _lazy(blest, rp, col, reorder=3, jaccard_window=256)
    sb, sj = base.info(), g.info()
    assert sj["reordered"] == 3 and sb["reordered"] == 0
    nof = blest.blest_reorder_jaccard(rp, col, 8, 256)
    assert sj["n_slices"] == J.count_slices(rp, col, nof, 8) < sb["n_slices"]
    for s in inputs.sources(rp, 3, seed=92):
        run_all_policies(blest, g, int(s), oracle.bfs(rp, col, int(s)), seeds=(2,))
    srcs = inputs.sources(rp, 130, seed=93)
    assert np.array_equal(g.msbfs(srcs).cpu().numpy(), oracle.msbfs16(rp, col, srcs))
    osum, oreach, occ = oracle.closeness(rp, col, srcs)
    s_, r_, c_ = g.closeness(srcs)
    assert np.array_equal(s_.cpu().numpy(), osum) and np.array_equal(c_.cpu().numpy(), occ)
    base.close()
    g.close()
    # AUTO (Section "Reordering the Graph"): JaccardWithWindows for the
    # scale-free-like R-MAT, RCM for the grid
    auto = blest.Graph(rp, col)
    nof_auto = blest.blest_reorder_jaccard(rp, col, 8, 1024)
    assert auto.info()["reordered"] == 3 and auto.info()["n_slices"] == J.count_slices(rp, col, nof_auto, 8)
    auto.close()
    grp, gcol = inputs.grid_graph(40, 94)
    auto = blest.Graph(grp, gcol)
    assert auto.info()["reordered"] == 1
    auto.close()


def test_long_single_workgroup_episode_is_not_a_timeout(blest):
    """A 600,000-vertex path: on the lazy scheme every level runs on
    workgroup 0 alone (one episode of ~600K small levels, longer than the 10 s
    bound of a barrier wait); the waiting workgroups restart their bound at
    every finished level, so the traversal completes. Both schemes exact."""
    n = 600_000
    rp, col = H.path(n)
    want = np.arange(n, dtype=np.int32)
    for scheme in (blest.Update.LAZY, blest.Update.EAGER):
        g = blest.Graph(rp, col, update_scheme=int(scheme), reorder=0)
        lev = g.bfs(0).cpu().numpy()
        assert np.array_equal(lev, want), scheme
        g.close()
