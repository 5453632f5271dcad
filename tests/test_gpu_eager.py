"""Eager vertex updates (Alg. 2) and the update-divergence dispatch, on the
GPU through the C ABI, against the oracle: levels are integers with one
correct value, so every comparison is array equality."""
import numpy as np
import pytest

import oracle
from paper_2606_05081_amd import inputs
from tests import helpers as H
from tests.test_gpu_bfs import run_all_policies

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def blest():
    import torch
    from paper_2606_05081_amd import blest as b
    assert torch.cuda.is_available()
    b.lib()
    return b


def _graph(name):
    if name == "path":
        return H.path(1000)
    if name == "star":
        return H.star(3000)
    if name == "hypercube":
        return H.hypercube(12)
    if name == "grid":
        return inputs.grid_graph(70, 78)
    if name == "gnp":
        return H.gnp(300, 0.02, 5)
    if name == "rmat":
        return inputs.rmat_graph(13, 77)
    if name == "er":
        return inputs.er_graph(13, 79)
    return inputs.from_pairs(13, [0, 1, 2, 5, 6], [1, 2, 3, 6, 7])


@pytest.mark.parametrize("name", ["path", "star", "hypercube", "grid", "gnp", "rmat", "er", "tiny"])
def test_eager_every_policy(blest, name):
    rp, col = _graph(name)
    g = blest.Graph(rp, col, update_scheme=blest.Update.EAGER)
    assert g.info()["update_scheme"] == blest.Update.EAGER
    n = rp.size - 1
    H.install_switch_models(g, multi=False)
    for src in sorted({0, n // 3, n - 1}):
        ref = oracle.bfs(rp, col, src)
        run_all_policies(blest, g, src, ref, seeds=(1, 2))
        g.set_policy(blest.Policy.LEARNED, 10.0)
        assert np.array_equal(g.bfs(src).cpu().numpy(), ref)
    g.close()


@pytest.mark.parametrize("opt", [dict(sigma=16), dict(sigma=32), dict(tau=64), dict(tau=256), dict(tau=192),
                                 dict(wide_slices=1), dict(block_size=256), dict(block_size=1024),
                                 dict(blocks_per_cu=2), dict(reorder=0), dict(reorder=3), dict(persistent=0)])
def test_eager_option_matrix(blest, opt):
    for rp, col in [inputs.rmat_graph(12, 81), inputs.grid_graph(50, 82)]:
        g = blest.Graph(rp, col, update_scheme=blest.Update.EAGER, **opt)
        for s in inputs.sources(rp, 2, seed=83):
            run_all_policies(blest, g, int(s), oracle.bfs(rp, col, int(s)), seeds=(3,))
        g.close()


def test_eager_level_log_matches_oracle_counts_and_eq3_replay(blest):
    for rp, col in [inputs.rmat_graph(15, 84), inputs.grid_graph(96, 85)]:
        g = blest.Graph(rp, col, reorder=0, update_scheme=blest.Update.EAGER)
        b = g.export_bvss()
        for s in inputs.sources(rp, 3, seed=86):
            s = int(s)
            g.set_policy(blest.Policy.HEURISTIC, 10.0)
            ref = g.bfs(s).cpu().numpy()
            assert np.array_equal(ref, oracle.bfs(rp, col, s))
            stats = g.level_stats()
            assert [r["frontier"] for r in stats] == oracle.level_counts(ref).tolist()
            rep = oracle.switch_replay(ref, rp, b["real_ptrs"], 8, eta=10.0)
            assert [r["queue"] for r in stats] == [r["queue"] for r in rep]
            assert [r["unvisited"] for r in stats] == [r["unvisited"] for r in rep]
            assert [r["engine"] == blest.Engine.BOTTOM_UP for r in stats[:-1]] == [r["bottom_up"] for r in rep[:-1]]
            deg = np.diff(rp)
            for r in stats:
                fr = ref == r["level"]
                assert r["frontier_edges"] == int(deg[fr].sum())
                assert r["deg_ge_32"] == int((deg[fr] >= 32).sum())
        g.close()


def test_update_divergence_dispatch(blest):
    """AUTO follows the paper's rule: eager iff the built graph's U_div <=
    25,000. The reported U_div is the host value of the relabelled graph."""
    # the 2048 x 2048 grid after RCM: clustered rows, eager
    rp, col = inputs.grid_graph(2048, 1022)
    g = blest.Graph(rp, col, update_scheme=blest.Update.AUTO)
    info = g.info()
    assert info["reordered"] == 1 and info["u_div"] <= 25000 and info["update_scheme"] == blest.Update.EAGER
    srcs = inputs.sources(rp, 3, seed=1023)
    ref = oracle.bfs(rp, col, int(srcs[0]))
    for i, s in enumerate(srcs):
        lev = g.bfs(int(s)).cpu().numpy()
        assert oracle.certificate(rp, col, int(s), lev) == (0, -1)
        if i == 0:
            assert np.array_equal(lev, ref)
    g.close()
    # the same grid in its random labelling (no reordering): scattered rows, lazy
    g = blest.Graph(rp, col, reorder=0, update_scheme=blest.Update.AUTO)
    assert g.info()["u_div"] > 25000 and g.info()["update_scheme"] == blest.Update.LAZY
    assert g.info()["u_div"] == pytest.approx(blest.blest_update_divergence(rp, col), rel=1e-12)
    g.close()
    # scale-20 R-MAT (JaccardWithWindows order): lazy
    rp, col = inputs.rmat_graph(20, 1040)
    g = blest.Graph(rp, col, update_scheme=blest.Update.AUTO)
    assert g.info()["u_div"] > 25000 and g.info()["update_scheme"] == blest.Update.LAZY
    g.close()


def test_eager_equals_lazy_on_many_sources(blest):
    rp, col = inputs.grid_graph(300, 87)
    ge = blest.Graph(rp, col, update_scheme=blest.Update.EAGER)
    gl = blest.Graph(rp, col, update_scheme=blest.Update.LAZY)
    for s in inputs.sources(rp, 12, seed=88):
        assert np.array_equal(ge.bfs(int(s)).cpu().numpy(), gl.bfs(int(s)).cpu().numpy())
    ge.close()
    gl.close()
