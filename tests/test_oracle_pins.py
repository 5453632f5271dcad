"""Pins the CPU oracle to facts that do not come from the oracle itself:
brute force on tiny graphs, closed forms, the paper's worked examples,
identities, and planted mistakes the certificate must reject."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2606_05081_amd import inputs
from tests import helpers as H


# ---------------------------------------------------------------- BFS levels

@pytest.mark.parametrize("seed", range(12))
def test_bfs_matches_floyd_warshall_and_dense_eq1(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 60))
    p = float(rng.choice([0.02, 0.05, 0.1, 0.3]))
    rp, col = H.gnp(n, p, seed)
    fw = H.floyd_warshall(rp, col)
    for src in range(n):
        lev = oracle.bfs(rp, col, src)
        assert np.array_equal(lev, fw[src]), (seed, src)
    for src in rng.integers(0, n, 3):
        assert np.array_equal(oracle.bfs(rp, col, int(src)), H.dense_eq1_levels(rp, col, int(src)))


def test_bfs_rmat_tiny_matches_brute_force():
    for scale, seed in [(6, 3), (7, 4), (8, 5)]:
        rp, col = inputs.rmat_graph(scale, seed)
        fw = H.floyd_warshall(rp, col)
        for src in range(0, rp.size - 1, 7):
            assert np.array_equal(oracle.bfs(rp, col, src), fw[src])


def test_closed_forms_path_cycle_star_complete():
    n = 37
    rp, col = H.path(n)
    for s in (0, 5, 36):
        assert np.array_equal(oracle.bfs(rp, col, s), np.abs(np.arange(n) - s))
    rp, col = H.cycle(n)
    for s in (0, 11):
        d = np.abs(np.arange(n) - s)
        assert np.array_equal(oracle.bfs(rp, col, s), np.minimum(d, n - d))
    rp, col = H.star(n)
    lev = oracle.bfs(rp, col, 0)
    assert lev[0] == 0 and (lev[1:] == 1).all()
    lev = oracle.bfs(rp, col, 4)
    exp = np.full(n, 2)
    exp[4], exp[0] = 0, 1
    assert np.array_equal(lev, exp)
    rp, col = H.complete(12)
    lev = oracle.bfs(rp, col, 3)
    assert lev[3] == 0 and (np.delete(lev, 3) == 1).all()
    a, b = 5, 7
    rp, col = H.complete_bipartite(a, b)
    lev = oracle.bfs(rp, col, 0)
    assert lev[0] == 0 and (lev[1:a] == 2).all() and (lev[a:] == 1).all()


def test_closed_form_hypercube_hamming():
    d = 10
    rp, col = H.hypercube(d)
    v = np.arange(1 << d)
    for s in (0, 5, 1023):
        ham = np.array([bin(x).count("1") for x in (v ^ s)])
        assert np.array_equal(oracle.bfs(rp, col, s), ham)


def test_closed_form_full_grid_manhattan_under_permutation():
    side = 40
    rp, col = inputs.grid(side, 0.0, seed=7, permute=False)
    rp2, col2, perm = inputs.permute(rp, col, seed=11)
    x, y = np.arange(side * side) % side, np.arange(side * side) // side
    for s in (0, 77, side * side - 1):
        manh = np.abs(x - x[s]) + np.abs(y - y[s])
        lev = oracle.bfs(rp2, col2, int(perm[s]))
        assert np.array_equal(lev[perm], manh)


def test_unreachable_is_minus_one_and_isolated_source():
    rp, col = inputs.from_pairs(6, [0, 1, 3], [1, 2, 4])
    assert oracle.bfs(rp, col, 0).tolist() == [0, 1, 2, -1, -1, -1]
    assert oracle.bfs(rp, col, 5).tolist() == [-1, -1, -1, -1, -1, 0]


# -------------------------------------------------------------- certificate

def test_certificate_accepts_truth_and_rejects_planted_mistakes():
    rp, col = inputs.rmat_graph(10, 21)
    deg = np.diff(rp)
    src = int(np.argmax(deg))
    lev = oracle.bfs(rp, col, src)
    assert oracle.certificate(rp, col, src, lev) == (0, -1)
    reached = np.nonzero(lev > 0)[0]
    v = int(reached[len(reached) // 2])
    bad = lev.copy(); bad[v] += 1
    assert oracle.certificate(rp, col, src, bad)[0] in (3, 4)
    bad = lev.copy(); bad[v] -= 1
    assert oracle.certificate(rp, col, src, bad)[0] in (3, 4)
    bad = lev.copy(); bad[v] = -1
    assert oracle.certificate(rp, col, src, bad)[0] == 2
    bad = lev.copy(); bad[src] = 1
    assert oracle.certificate(rp, col, src, bad)[0] == 1
    # a whole level shifted by one breaks the one-level rule on its parent edges
    bad = lev.copy(); bad[lev == lev.max()] += 1
    assert oracle.certificate(rp, col, src, bad)[0] == 3
    # every edge within one level, but vertex 2 has no parent: path 0-1-2 as [0,1,1]
    rp3, col3 = H.path(3)
    assert oracle.certificate(rp3, col3, 0, np.array([0, 1, 1]))[0] == 4
    # an unreachable component given finite levels: caught by the parent rule
    rp2, col2 = inputs.from_pairs(5, [0, 3], [1, 4])
    assert oracle.certificate(rp2, col2, 0, np.array([0, 1, -1, 1, 2]))[0] == 4


# ---------------------------------------------------- multi-source/closeness

def test_msbfs_rows_equal_single_source():
    rp, col = inputs.rmat_graph(9, 31)
    srcs = inputs.sources(rp, 20, seed=5)
    ms = oracle.msbfs16(rp, col, srcs)
    for c, s in enumerate(srcs):
        assert np.array_equal(ms[c].astype(np.int32), oracle.bfs(rp, col, int(s)))


def test_msbfs_overflow_detected():
    n = 33000
    rp, col = H.path(n)
    with pytest.raises(OverflowError):
        oracle.msbfs16(rp, col, [0])
    assert int(oracle.msbfs16(rp, col, [16000]).max()) == 16999


def test_closeness_closed_forms():
    n = 50
    rp, col = H.path(n)
    srcs = np.arange(n)
    sums, reach, cc = oracle.closeness(rp, col, srcs)
    i = np.arange(n)
    assert np.array_equal(sums, i * (i + 1) // 2 + (n - 1 - i) * (n - i) // 2)
    assert (reach == n).all()
    assert np.array_equal(cc, (n - 1) / sums.astype(np.float64))
    d = 9
    rp, col = H.hypercube(d)
    sums, reach, _ = oracle.closeness(rp, col, np.arange(1 << d))
    assert (sums == d * 2 ** (d - 1)).all()
    rp, col = H.star(n)
    sums, _, _ = oracle.closeness(rp, col, np.arange(n))
    assert sums[0] == n - 1 and (sums[1:] == 2 * n - 3).all()
    side = 12
    rp, col = inputs.grid(side, 0.0, seed=1, permute=False)
    sums, _, _ = oracle.closeness(rp, col, np.arange(side * side))
    x, y = np.arange(side * side) % side, np.arange(side * side) // side
    exp = np.array([np.abs(x - x[s]).sum() + np.abs(y - y[s]).sum() for s in range(side * side)])
    assert np.array_equal(sums, exp)


def test_closeness_isolated_source_and_disconnected():
    rp, col = inputs.from_pairs(5, [0, 1], [1, 2])
    sums, reach, cc = oracle.closeness(rp, col, [0, 4, 1])
    assert sums.tolist() == [3, 0, 2]
    assert reach.tolist() == [3, 1, 3]
    assert cc.tolist() == [2 / 3, 0.0, 1.0]


def test_far_equals_sums_when_all_sources_and_total_identity():
    rp, col = inputs.rmat_graph(9, 41)
    n = rp.size - 1
    allv = np.arange(n)
    sums, _, _ = oracle.closeness(rp, col, allv)
    assert np.array_equal(oracle.far(rp, col, allv), sums)
    sub = inputs.sources(rp, 37, seed=3)
    s2, _, _ = oracle.closeness(rp, col, sub)
    assert oracle.far(rp, col, sub).sum() == s2.sum()


def test_far_source_subsets_closed_forms():
    """Eq. 4 over a proper subset S of the vertices: far[u] adds d(s, u) for
    the sources s only, at the target u (not at the source)."""
    n = 11
    rp, col = H.path(n)
    u = np.arange(n)
    assert np.array_equal(oracle.far(rp, col, [0]), u)  # one end of a path: far[u] = u
    assert np.array_equal(oracle.far(rp, col, [0, n - 1]), np.full(n, n - 1))  # both ends: u + (n-1-u)
    assert np.array_equal(oracle.far(rp, col, [3, 3]), 2 * np.abs(u - 3))  # a repeated source counts twice
    k = 9
    rp, col = H.star(k + 1)  # centre 0, leaves 1..k
    f = oracle.far(rp, col, np.arange(1, k + 1))
    assert f[0] == k  # every leaf is one hop from the centre
    assert (f[1:] == 2 * (k - 1)).all()  # two hops from the other k-1 leaves, 0 from itself
    f = oracle.far(rp, col, [0])
    assert f[0] == 0 and (f[1:] == 1).all()
    d = 7
    rp, col = H.hypercube(d)
    v = np.arange(1 << d)
    pc = np.array([bin(x).count("1") for x in v])
    assert np.array_equal(oracle.far(rp, col, [0]), pc)  # Hamming distance to 0
    assert np.array_equal(oracle.far(rp, col, [0, (1 << d) - 1]), np.full(1 << d, d))
    # unreachable pairs add nothing: path 0-1-2 and edge 3-4, sources 0 and 3
    rp, col = inputs.from_pairs(5, [0, 1, 3], [1, 2, 4])
    assert oracle.far(rp, col, [0, 3]).tolist() == [0, 1, 2, 0, 1]


# --------------------------------------------------------------------- BVSS

def fig1_graph():
    """A 24-vertex graph whose BVSS reproduces the BVSS figure (built here)."""
    pairs = [(3, 17), (3, 19), (3, 22), (16, 0), (16, 1), (18, 2), (20, 4), (5, 6), (7, 21), (8, 23)]
    u, v = zip(*pairs)
    return inputs.from_pairs(24, u, v)


def bits_lsb_first(s):
    return sum(1 << i for i, ch in enumerate(s) if ch == "1")


def test_bvss_fig1_worked_example(golden):
    g = golden("fig1_bvss.txt")
    rp, col = fig1_graph()
    b = oracle.bvss(rp, col, sigma=int(g["sigma"][0]), tau=4)
    assert b["real_ptrs"].tolist() == [int(x) for x in g["real_ptrs"]]
    assert b["v2r"].tolist() == [int(x) for x in g["virtual_to_real"]]
    assert [v for v in range(b["n_vss"]) if b["v2r"][v] == 2] == [int(x) for x in g["vss_of_set2"]]
    lo, hi = b["slice_ptr"][2], b["slice_ptr"][3]
    rows = b["slice_row"][lo:hi].tolist()
    mask3 = int(b["slice_mask"][lo + rows.index(3)])
    assert mask3 == bits_lsb_first(g["mask_row3_set2"][0])
    alpha = bits_lsb_first(g["frontier_set2"][0])
    hits = [r for r, m in zip(rows, b["slice_mask"][lo:hi].tolist()) if m & alpha]
    assert int(g["hit_row"][0]) in hits
    hit = int(g["hit_row"][0])
    assert hit // 8 == int(g["next_set"][0]) and hit % 8 == int(g["next_bit"][0])
    s = hit // 8
    assert list(range(b["real_ptrs"][s], b["real_ptrs"][s + 1])) == [int(x) for x in g["next_vss"]]
    # the BFS itself: from frontier {16, 17} vertex 3 is one hop away
    assert oracle.bfs(rp, col, 17)[3] == 1


@pytest.mark.parametrize("sigma,tau", [(8, 128), (8, 4), (16, 64), (32, 32), (1, 3)])
def test_bvss_decodes_back_to_csr(sigma, tau):
    rp, col = inputs.rmat_graph(9, 77)
    n = rp.size - 1
    b = oracle.bvss(rp, col, sigma, tau)
    edges = set()
    for s in range(b["n_slice_sets"]):
        lo, hi = b["slice_ptr"][s], b["slice_ptr"][s + 1]
        rows = b["slice_row"][lo:hi]
        assert (np.diff(rows) > 0).all()  # ascending, one slice per row
        nv = b["real_ptrs"][s + 1] - b["real_ptrs"][s]
        assert nv == -(-(hi - lo) // tau)  # VSSs of at most tau slices
        for r, m in zip(rows.tolist(), b["slice_mask"][lo:hi].tolist()):
            assert m != 0
            for bit in range(sigma):
                if m >> bit & 1:
                    edges.add((s * sigma + bit, r))
    exp = {(u, int(v)) for u in range(n) for v in col[rp[u]:rp[u + 1]]}
    assert edges == exp
    assert b["v2r"].tolist() == [s for s in range(b["n_slice_sets"])
                                 for _ in range(b["real_ptrs"][s + 1] - b["real_ptrs"][s])]


def test_get_vi_worked_example(golden):
    g = golden("getvi_n24.txt")
    n, sigma, rho = int(g["n"][0]), int(g["sigma"][0]), int(g["rho"][0])
    layout = [int(x) for x in g["layout"]]
    vi = oracle.get_vi(np.arange(n), sigma, rho)
    assert sorted(vi.tolist()) == list(range(n))  # bijective
    assert [int(u) for u in np.argsort(vi)] == layout


# ------------------------------------------------------------ Eq. 3 replay

def test_switch_replay_star_by_hand():
    rp, col = H.star(16)
    b = oracle.bvss(rp, col, 8, 128)
    lev = oracle.bfs(rp, col, 0)
    rep = oracle.switch_replay(lev, rp, b["real_ptrs"], 8, eta=10)
    # level 0: frontier {0}, one VSS, 15 unvisited -> 15 < 10 is false: top-down
    assert rep[0] == {"level": 0, "frontier": 1, "queue": 1, "unvisited": 15, "bottom_up": False}
    # level 1: leaves 1..15 cover slice sets 0 and 1 -> 2 VSSs, 0 unvisited -> bottom-up
    assert rep[1] == {"level": 1, "frontier": 15, "queue": 2, "unvisited": 0, "bottom_up": True}


def test_level_counts_sum_to_component():
    rp, col = inputs.rmat_graph(10, 5)
    lev = oracle.bfs(rp, col, int(np.argmax(np.diff(rp))))
    cnt = oracle.level_counts(lev)
    assert cnt[0] == 1 and cnt.sum() == (lev >= 0).sum() and (cnt > 0).all()


@pytest.mark.parametrize("seed", range(4))
def test_components_match_union_find_and_scipy(seed):
    # union-find written here on the edge list, and scipy's BFS labelling
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 400))
    k = int(rng.integers(0, n))
    rp, col = inputs.from_pairs(n, rng.integers(0, n, k), rng.integers(0, n, k))
    lab = oracle.components(rp, col)
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for u in range(n):
        for v in col[rp[u]:rp[u + 1]]:
            parent[find(u)] = find(int(v))
    roots = [find(u) for u in range(n)]
    for u in range(n):
        for v in range(0, n, 7):
            assert (lab[u] == lab[v]) == (roots[u] == roots[v])
    # numbered by smallest vertex
    first = {}
    for u in range(n):
        first.setdefault(lab[u], u)
    assert [first[i] for i in range(len(first))] == sorted(first.values())
    ncomp, slab = connected_components(csr_matrix((np.ones(col.size), col, rp), shape=(n, n)), directed=False)
    assert lab.max() + 1 == ncomp
    # reach of each vertex = its component size (closeness's reach)
    sizes = np.bincount(lab)[lab]
    _, reach, _ = oracle.closeness(rp, col, np.arange(n, dtype=np.int32))
    assert np.array_equal(reach, sizes)


# ---------------------------------------------------------------------- MLP

def _rand_params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, mlp.N_PARAMS)


def test_mlp_zero_weights_loss_is_ln3_and_logit_grad():
    x = np.random.default_rng(0).normal(size=(17, 12))
    y = np.arange(17) % 3
    loss, g = mlp.loss_and_grad(np.zeros(mlp.N_PARAMS), x, y)
    assert loss == pytest.approx(math.log(3), abs=1e-15)
    gb3 = mlp.unpack(g)["b3"]
    exp = np.array([(1 / 3) - np.mean(y == k) for k in range(3)])
    assert np.allclose(gb3, exp, atol=1e-15)


def test_mlp_forward_hand_built_network():
    # W1 copies the 12 inputs into the first 12 hidden units, W2 copies them
    # again, W3 sums inputs 0..3 into logit 0, 4..7 into logit 1, 8..11 into 2.
    p = {name: np.zeros(shp) for name, shp in mlp.SHAPES}
    p["W1"][:12, :12] = np.eye(12)
    p["W2"][:12, :12] = np.eye(12)
    for k in range(3):
        p["W3"][k, 4 * k:4 * k + 4] = 1.0
    p["b3"] = np.array([0.5, -1.0, 2.0])
    x = np.abs(np.random.default_rng(1).normal(size=(5, 12)))
    z, _ = mlp.forward(mlp.pack(p), x)
    exp = np.stack([x[:, 0:4].sum(1) + 0.5, x[:, 4:8].sum(1) - 1.0, x[:, 8:12].sum(1) + 2.0], 1)
    assert np.allclose(z, exp, atol=1e-14)
    z2, _ = mlp.forward(mlp.pack(p), -x)  # negative inputs die in the first ReLU
    assert np.allclose(z2, np.broadcast_to(p["b3"], z2.shape))


def test_mlp_gradient_central_differences():
    rng = np.random.default_rng(2)
    theta = _rand_params(3)
    x = rng.normal(size=(9, 12))
    y = rng.integers(0, 3, 9)
    w = rng.uniform(0.5, 2.0, 9)
    _, g = mlp.loss_and_grad(theta, x, y, w)
    h = 1e-6
    idx = rng.choice(mlp.N_PARAMS, 120, replace=False)
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        num = (mlp.loss_and_grad(tp, x, y, w)[0] - mlp.loss_and_grad(tm, x, y, w)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, i


def test_adam_first_step_closed_form():
    theta = _rand_params(4)
    g = np.random.default_rng(5).normal(size=mlp.N_PARAMS)
    lr, eps = 1e-3, 1e-8
    t1, m1, v1 = mlp.adam_step(theta, g, np.zeros_like(g), np.zeros_like(g), 1, lr=lr, eps=eps)
    assert np.allclose(t1, theta - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


# ---- JaccardWithWindows (Section "Increasing Compression Ratio") ----------

def _planted_blocks(sizes, rows_per_group, seed):
    """Columns 0..sum(sizes)-1 in groups; the columns of a group share the same
    private row set (identical neighbourhoods, so their Jaccard similarity is 1
    and 0 across groups). Column labels are shuffled."""
    rng = np.random.default_rng(seed)
    ncol = sum(sizes)
    perm = rng.permutation(ncol)
    us, vs, groups, nxt = [], [], [], ncol
    start = 0
    for size, nr in zip(sizes, rows_per_group):
        cols = perm[start:start + size]
        start += size
        rows = list(range(nxt, nxt + nr))
        nxt += nr
        groups.append(set(int(c) for c in cols))
        for c in cols:
            for r in rows:
                us.append(int(c))
                vs.append(r)
    rp, col = inputs.from_pairs(nxt, us, vs)
    return rp, col, groups


def test_jaccard_recovers_planted_slice_sets():
    from oracle import jaccard as J
    # window 16 = four slice sets of 4; group sizes 4, row sets of distinct sizes
    rp, col, groups = _planted_blocks([4, 4, 4, 4], [5, 9, 3, 7], seed=3)
    nof = J.jaccard_with_windows(rp, col, sigma=4, window=16)
    sets = [set(np.nonzero(nof[:16] // 4 == k)[0].tolist()) for k in range(4)]
    assert sorted(map(sorted, sets)) == sorted(map(sorted, groups))
    # seeds go by degree: the first slice set is the group with the largest row set
    assert sets[0] == groups[1] and sets[1] == groups[3]
    # the window's four slice sets then hold one slice per (group, row): the
    # minimum, 5 + 9 + 3 + 7; the shuffled order needs more
    def window_slices(order):
        src = np.repeat(np.arange(rp.size - 1), np.diff(rp))
        sel = src < 16
        return len(set(zip((np.asarray(order)[src[sel]] // 4).tolist(), col[sel].tolist())))
    assert window_slices(nof) == 24
    assert window_slices(np.arange(rp.size - 1)) > 24


def test_jaccard_is_a_windowwise_permutation_seeded_by_degree():
    from oracle import jaccard as J
    rp, col = inputs.rmat_graph(8, 17)
    n = rp.size - 1
    deg = np.diff(rp)
    for sigma, window in [(8, 32), (8, 64), (4, 12), (2, 6)]:
        nof = J.jaccard_with_windows(rp, col, sigma, window)
        assert np.array_equal(np.sort(nof), np.arange(n))
        for ws in range(0, n, window):
            we = min(ws + window, n)
            assert nof[ws:we].min() == ws and nof[ws:we].max() == we - 1
            first = int(np.nonzero(nof == ws)[0][0])
            best = ws + int(np.argmax(deg[ws:we]))  # argmax returns the smallest id among ties
            assert first == best


def test_jaccard_without_edges_keeps_the_order_and_handles_a_ragged_window():
    from oracle import jaccard as J
    rp = np.zeros(21, dtype=np.int32)
    col = np.zeros(0, dtype=np.int32)
    assert np.array_equal(J.jaccard_with_windows(rp, col, 8, 16), np.arange(20))
    # a path: degrees 1, 2, ..., 2, 1 -- ties resolved to the smaller id
    rp, col = H.path(10)
    nof = J.jaccard_with_windows(rp, col, 2, 4)
    assert np.array_equal(np.sort(nof), np.arange(10))
    assert nof[1] == 0  # vertex 1 (degree 2, smallest such id) seeds the first window


def _jaccard_case(seed_deg, cand):
    """Window 0 = vertices 0..3 with sigma = 2: vertex 3 is the seed column
    (the highest degree), vertex 0 a filler column with one private row, and
    vertices 1, 2 the candidates, each given as (rows shared with the seed,
    private rows). Every row is a vertex of id >= 4 adjacent to its columns only."""
    us, vs = [], []
    nxt = 4
    seed_rows = list(range(nxt, nxt + seed_deg))
    nxt += seed_deg
    for r in seed_rows:
        us.append(3)
        vs.append(r)
    for c, (shared, private) in zip((1, 2), cand):
        for r in seed_rows[:shared]:
            us.append(c)
            vs.append(r)
        for r in range(nxt, nxt + private):
            us.append(c)
            vs.append(r)
        nxt += private
    us.append(0)
    vs.append(nxt)
    nxt += 1
    return inputs.from_pairs(nxt, us, vs)


def test_jaccard_score_is_the_ratio_not_the_overlap():
    """The second column of a slice set maximises inter / (|R| + deg - inter)
    (the Jaccard similarity of Section "Increasing Compression Ratio"), which
    differs from maximising the overlap inter or inter / deg. Values by hand,
    seed column 3 of degree 13, so |R| = 13:
      case 1: vertex 1 has inter 3, deg 12 -> 3/22; vertex 2 inter 2, deg 2 -> 2/13.
              2/13 > 3/22, so vertex 2 joins the seed (overlap alone picks 1).
      case 2: vertex 1 has inter 4, deg 8 -> 4/17; vertex 2 inter 3, deg 3 -> 3/13.
              4/17 > 3/13, so vertex 1 joins the seed (inter / deg picks 2).
    The second slice set is seeded by the higher-degree remaining column; the
    filler (vertex 0) shares no row with it and comes last."""
    from oracle import jaccard as J
    rp, col = _jaccard_case(13, [(3, 9), (2, 0)])
    nof = J.jaccard_with_windows(rp, col, sigma=2, window=4)
    assert nof[:4].tolist() == [3, 2, 1, 0]
    rp, col = _jaccard_case(13, [(4, 4), (3, 0)])
    nof = J.jaccard_with_windows(rp, col, sigma=2, window=4)
    assert nof[:4].tolist() == [3, 1, 2, 0]


def test_update_divergence_hand_worked():
    """U_div (Section "Boosting Cache Locality") on a graph worked by hand:
    vertex 0 adjacent to rows R = 9, 12, 20, 28, 33, 41, 50, 62, 63; sigma = 8,
    tau = 8, theta = 4. Slice set 0 holds nine slices (rows R): its first VSS
    is the 2 x 4 matrix with columns {9, 33}, {12, 41}, {20, 50}, {28, 62}
    (standard deviations 12, 14.5, 15, 17, mean 14.625); its second VSS is the
    single slice of row 63 (0). Sets 1..7 hold one slice each (row 0): 0.
    U_div = 14.625 / 9 VSSs = 1.625. A column-major reading of the matrix
    (slice j in column j // 2) would give 0.4306, the sample standard
    deviation 2.2981, an average over slice sets 1.828."""
    R = [9, 12, 20, 28, 33, 41, 50, 62, 63]
    rp, col = inputs.from_pairs(64, [0] * len(R), R)
    assert oracle.update_divergence(rp, col, sigma=8, tau=8, theta=4) == pytest.approx(1.625, rel=1e-15)
    # a star on 9 vertices, tau = 128 (the 32 x 4 matrix): set 0 has the
    # slices of rows 0..8 in one VSS, columns {0, 4, 8}, {1, 5}, {2, 6}, {3, 7}
    # (deviations sqrt(32/3), 2, 2, 2); set 1 one slice: 0
    rp, col = H.star(9)
    want = (np.sqrt(32.0 / 3.0) + 6.0) / 4.0 / 2.0
    assert oracle.update_divergence(rp, col) == pytest.approx(want, rel=1e-15)
    # no edges: no VSS at all
    rp, col = inputs.from_pairs(20, [], [])
    assert oracle.update_divergence(rp, col) == 0.0


def _digraph(n, p, seed):
    rng = np.random.default_rng(seed)
    a = rng.random((n, n)) < p
    np.fill_diagonal(a, False)
    u, v = np.nonzero(a)
    return inputs.directed_from_pairs(n, u, v)


def test_directed_bfs_brute_force_and_eq1():
    """Directed graphs (Background: A is the transposed adjacency, A[i][j] = 1
    iff arc j -> i): the oracle's queue BFS over out-arcs equals Floyd-Warshall
    on the arcs and the literal Boolean-semiring iteration of Eq. 1."""
    for n, p, seed in [(40, 0.05, 1), (60, 0.03, 2), (25, 0.15, 3), (50, 0.0, 4)]:
        rp, col = _digraph(n, p, seed)
        fw = H.floyd_warshall(rp, col)
        for s in range(0, n, 7):
            lev = oracle.bfs(rp, col, s)
            assert np.array_equal(lev, fw[s]), (n, p, s)
            assert np.array_equal(lev, H.dense_eq1_levels(rp, col, s)), (n, p, s)
            assert oracle.certificate_directed(rp, col, s, lev) == (0, -1)


def test_directed_closed_forms():
    n = 200
    rp, col = inputs.directed_from_pairs(n, np.arange(n - 1), np.arange(1, n))  # path 0 -> 1 -> ... -> n-1
    for s in (0, 57, n - 1):
        want = np.where(np.arange(n) >= s, np.arange(n) - s, -1)
        assert np.array_equal(oracle.bfs(rp, col, s), want)
    rp, col = inputs.directed_from_pairs(n, np.arange(n), (np.arange(n) + 1) % n)  # directed cycle
    for s in (0, 123):
        assert np.array_equal(oracle.bfs(rp, col, s), (np.arange(n) - s) % n)
    # per-source sums along arcs: the cycle's are n(n-1)/2 for every source
    srcs = np.array([0, 5, 199], np.int32)
    sums, reach, _ = oracle.closeness(rp, col, srcs)
    assert sums.tolist() == [n * (n - 1) // 2] * 3 and reach.tolist() == [n] * 3


def test_directed_certificate_rejects_planted_mistakes():
    rp, col = _digraph(60, 0.04, 9)
    s = max(range(60), key=lambda x: int((oracle.bfs(rp, col, x) >= 0).sum()))
    good = oracle.bfs(rp, col, s)
    assert 3 < (good >= 0).sum() < 60
    assert oracle.certificate_directed(rp, col, s, good)[0] == 0
    reached = np.nonzero(good > 0)[0]
    unreached = np.nonzero(good < 0)[0]
    v = int(reached[-1])
    bad = good.copy()
    bad[v] += 1  # too far: some in-arc from level good[v]-1 now skips a level
    assert oracle.certificate_directed(rp, col, s, bad)[0] in (3, 4)
    bad = good.copy()
    bad[v] -= 1  # too close: no parent one level up
    assert oracle.certificate_directed(rp, col, s, bad)[0] in (3, 4)
    bad = good.copy()
    bad[v] = -1  # a reached vertex claimed unreachable
    assert oracle.certificate_directed(rp, col, s, bad)[0] == 2
    if unreached.size:
        bad = good.copy()
        bad[int(unreached[0])] = int(good.max()) + 1  # an unreachable vertex with a level
        assert oracle.certificate_directed(rp, col, s, bad)[0] == 4
    bad = good.copy()
    bad[s] = 1
    assert oracle.certificate_directed(rp, col, s, bad)[0] == 1
