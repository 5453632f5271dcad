"""Directed graphs on the GPU through the C ABI (opts.directed = 1): the
transposed adjacency of the Background (A[i][j] = 1 iff arc j -> i) feeds the
BVSS, the bottom-up engines read in-arcs (Alg. 4 on the transpose), and every
output follows arcs from the sources. Checked against the oracle's queue BFS
over out-arcs, which its CPU tests pin to Floyd-Warshall and Eq. 1 on
digraphs, and by the directed distance certificate."""
import numpy as np
import pytest

import oracle
from paper_2606_05081_amd import inputs

pytestmark = pytest.mark.gpu

POLICIES = ["HEURISTIC", "BVSS", "PUSH", "BOTTOM_UP", "RANDOM"]


@pytest.fixture(scope="module")
def blest():
    import torch
    from paper_2606_05081_amd import blest as b
    assert torch.cuda.is_available()
    b.lib()
    return b


def _digraph(name):
    if name == "rmat":
        return inputs.rmat_directed(13, 401)
    if name == "rmat_dense":
        return inputs.rmat_directed(12, 402, edgefactor=48)
    if name == "path":
        n = 3000
        return inputs.directed_from_pairs(n, np.arange(n - 1), np.arange(1, n))
    if name == "cycle":
        n = 1000
        return inputs.directed_from_pairs(n, np.arange(n), (np.arange(n) + 1) % n)
    if name == "random":
        rng = np.random.default_rng(403)
        n, m = 4000, 20000
        return inputs.directed_from_pairs(n, rng.integers(0, n, m), rng.integers(0, n, m))
    # a symmetric graph given as directed: the same answers as undirected
    return inputs.rmat_graph(12, 404)


@pytest.mark.parametrize("name", ["rmat", "rmat_dense", "path", "cycle", "random", "symmetric"])
@pytest.mark.parametrize("scheme", [0, 1])
def test_directed_every_policy(blest, name, scheme):
    rp, col = _digraph(name)
    n = rp.size - 1
    g = blest.Graph(rp, col, directed=1, update_scheme=scheme)
    assert g.info()["directed"] == 1
    for src in sorted({0, n // 3, n - 1, int(np.argmax(np.diff(rp)))}):
        ref = oracle.bfs(rp, col, src)
        for pol in POLICIES:
            g.set_policy(getattr(blest.Policy, pol), 10.0, 5)
            lev = g.bfs(src).cpu().numpy()
            assert np.array_equal(lev, ref), (name, scheme, pol, src)
        assert oracle.certificate_directed(rp, col, src, ref) == (0, -1)
    g.close()


@pytest.mark.parametrize("opt", [dict(reorder=0), dict(reorder=1), dict(reorder=3), dict(sigma=16),
                                 dict(sigma=32, tau=64), dict(panel=2, update_scheme=0),
                                 dict(single_block=0, update_scheme=0), dict(persistent=0, update_scheme=0)])
def test_directed_options(blest, opt):
    rp, col = inputs.rmat_directed(12, 405)
    g = blest.Graph(rp, col, directed=1, **opt)
    for s in inputs.sources(rp, 3, seed=406):
        ref = oracle.bfs(rp, col, int(s))
        for pol in POLICIES:
            g.set_policy(getattr(blest.Policy, pol), 10.0, 6)
            assert np.array_equal(g.bfs(int(s)).cpu().numpy(), ref), (opt, pol)
    g.close()


def test_directed_msbfs_closeness_far(blest):
    rp, col = inputs.rmat_directed(13, 407)
    srcs = inputs.sources(rp, 300, seed=408, nonzero_degree=False)
    g = blest.Graph(rp, col, directed=1)
    ref = oracle.msbfs16(rp, col, srcs)
    osum, oreach, occ = oracle.closeness(rp, col, srcs)
    for pol in ("HEURISTIC", "BVSS", "BOTTOM_UP", "RANDOM"):
        g.set_policy(getattr(blest.Policy, pol), 10.0, 2)
        assert np.array_equal(g.msbfs_batched(srcs, [64, 128]).cpu().numpy(), ref), pol
        s_, r_, c_ = g.closeness(srcs)
        assert np.array_equal(s_.cpu().numpy(), osum), pol
        assert np.array_equal(r_.cpu().numpy(), oreach), pol
        assert np.array_equal(c_.cpu().numpy(), occ), pol
    assert np.array_equal(g.far(srcs).cpu().numpy(), oracle.far(rp, col, srcs))
    g.close()


def test_directed_full_size_rmat20(blest):
    """Directed R-MAT scale 20 (the scale-20 samples kept as arcs): certificate
    on three sources under every switch policy, oracle equality on one."""
    rp, col = inputs.rmat_directed(20, 1040)
    g = blest.Graph(rp, col, directed=1)
    srcs = inputs.sources(rp, 3, seed=1041)
    ref = oracle.bfs(rp, col, int(srcs[0]))
    for i, s in enumerate(srcs):
        for pol in ("HEURISTIC", "BVSS", "BOTTOM_UP"):
            g.set_policy(getattr(blest.Policy, pol), 10.0)
            lev = g.bfs(int(s)).cpu().numpy()
            assert oracle.certificate_directed(rp, col, int(s), lev) == (0, -1), pol
            if i == 0:
                assert np.array_equal(lev, ref), pol
    g.close()


def test_asymmetric_input_needs_the_directed_flag(blest):
    rp, col = inputs.directed_from_pairs(5, [0, 1], [1, 2])
    with pytest.raises(blest.BlestError) as ei:
        blest.Graph(rp, col)
    assert ei.value.status == blest.Status.INVALID_GRAPH
    g = blest.Graph(rp, col, directed=1)
    assert g.bfs(0).cpu().tolist() == [0, 1, 2, -1, -1]
    assert g.bfs(2).cpu().tolist() == [-1, -1, 0, -1, -1]
    g.close()
