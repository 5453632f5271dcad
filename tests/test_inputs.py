"""The seeded input generators: canonical form, determinism, sanity ranges."""
import numpy as np
import pytest

from paper_2606_05081_amd import inputs


def check_canonical(rp, col):
    n = rp.size - 1
    assert rp[0] == 0 and (np.diff(rp) >= 0).all() and rp[-1] == col.size
    assert col.min(initial=0) >= 0 and col.max(initial=0) < n
    u = np.repeat(np.arange(n), np.diff(rp))
    assert not (u == col).any(), "self loop"
    key = u.astype(np.int64) * n + col
    assert (np.diff(key) > 0).all(), "rows unsorted or duplicated"
    rkey = col.astype(np.int64) * n + u
    assert np.array_equal(np.sort(rkey), key), "not symmetric"


@pytest.mark.parametrize("maker", [
    lambda t: inputs.rmat(10, 16, 0.57, 0.19, 0.19, seed=9, threads=t),
    lambda t: inputs.grid(37, 0.1, seed=9, threads=t),
    lambda t: inputs.erdos_renyi(5000, 40000, seed=9, threads=t),
])
def test_canonical_and_thread_independent(maker):
    a = maker(1)
    b = maker(7)
    check_canonical(*a)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_seeds_differ_and_shapes_match_workload_recipes():
    rp, col = inputs.rmat_graph(16, 1010)
    n = rp.size - 1
    assert n == 65536
    # symmetrised ef-16 R-MAT at scale 16: ~1.8M directed edges, ~29% isolated
    assert 1.7e6 < col.size < 1.95e6
    iso = (np.diff(rp) == 0).mean()
    assert 0.24 < iso < 0.33
    rp2, _ = inputs.rmat_graph(16, 1011)
    assert not np.array_equal(rp, rp2)
    grp, gcol = inputs.grid_graph(256, 1022)
    assert grp.size - 1 == 65536
    full = 2 * 2 * 256 * 255
    assert 0.88 * full < gcol.size < 0.92 * full
    assert np.diff(grp).max() <= 4
    erp, ecol = inputs.er_graph(14, 3)
    assert 15.5 < ecol.size / (erp.size - 1) < 16.1


def test_sources():
    rp, col = inputs.rmat_graph(12, 4)
    s = inputs.sources(rp, 64, seed=1)
    assert len(set(s.tolist())) == 64 and (np.diff(rp)[s] > 0).all()
    assert np.array_equal(s, inputs.sources(rp, 64, seed=1))
    allv = inputs.sources(rp, rp.size - 1, seed=2, nonzero_degree=False)
    assert sorted(allv.tolist()) == list(range(rp.size - 1))
    with pytest.raises(ValueError):
        inputs.sources(rp, rp.size, seed=2, nonzero_degree=False)


def test_permute_is_a_relabelling():
    rp, col = inputs.rmat(8, 8, 0.57, 0.19, 0.19, seed=3, permute=False)
    rp2, col2, perm = inputs.permute(rp, col, seed=4)
    check_canonical(rp2, col2)
    assert sorted(perm.tolist()) == list(range(rp.size - 1))
    for u in range(rp.size - 1):
        assert sorted(perm[col[rp[u]:rp[u + 1]]].tolist()) == col2[rp2[perm[u]]:rp2[perm[u] + 1]].tolist()
