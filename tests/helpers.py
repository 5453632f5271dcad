"""Small graph builders for tests (closed-form families) and brute force."""
import numpy as np

from paper_2606_05081_amd import inputs


def path(n):
    return inputs.from_pairs(n, np.arange(n - 1), np.arange(1, n))


def cycle(n):
    return inputs.from_pairs(n, np.arange(n), (np.arange(n) + 1) % n)


def star(n):
    return inputs.from_pairs(n, np.zeros(n - 1, np.int32), np.arange(1, n))


def complete(n):
    u, v = np.triu_indices(n, 1)
    return inputs.from_pairs(n, u, v)


def complete_bipartite(a, b):
    u, v = np.meshgrid(np.arange(a), a + np.arange(b), indexing="ij")
    return inputs.from_pairs(a + b, u.ravel(), v.ravel())


def hypercube(d):
    n = 1 << d
    us, vs = [], []
    for i in range(d):
        u = np.arange(n)
        u = u[(u >> i) & 1 == 0]
        us.append(u)
        vs.append(u | (1 << i))
    return inputs.from_pairs(n, np.concatenate(us), np.concatenate(vs))


def gnp(n, p, seed):
    rng = np.random.default_rng(seed)
    u, v = np.triu_indices(n, 1)
    keep = rng.random(u.size) < p
    return inputs.from_pairs(n, u[keep], v[keep])


def dense_adjacency(rp, col):
    n = rp.size - 1
    a = np.zeros((n, n), dtype=bool)
    for u in range(n):
        a[u, col[rp[u]:rp[u + 1]]] = True
    return a


def floyd_warshall(rp, col):
    """All-pairs hop distances, -1 for unreachable (O(n^3) brute force)."""
    n = rp.size - 1
    inf = n + 1
    d = np.full((n, n), inf, dtype=np.int64)
    a = dense_adjacency(rp, col)
    d[a] = 1
    np.fill_diagonal(d, 0)
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    d[d >= inf] = -1
    return d


def dense_eq1_levels(rp, col, src):
    """Literal Boolean-semiring iteration x <- (A x) and not v, level = first k with x_k[i] = 1."""
    a = dense_adjacency(rp, col).T  # A[i][j] = 1 iff (j, i) is an edge
    n = a.shape[0]
    x = np.zeros(n, dtype=bool)
    x[src] = True
    v = x.copy()
    lev = np.full(n, -1, dtype=np.int64)
    lev[src] = 0
    k = 0
    while x.any():
        k += 1
        x = ((a.astype(np.int64) @ x.astype(np.int64)) > 0) & ~v
        lev[x] = k
        v |= x
    return lev


def install_switch_models(g, single=True, multi=True):
    """Installs the committed switch networks (single- and multi-source) on g."""
    import json
    import os
    pkg = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2606_05081_amd")
    for name, on, setter in (("switch_model.json", single, g.set_switch_model),
                             ("switch_model_ms.json", multi, g.set_ms_switch_model)):
        if not on:
            continue
        with open(os.path.join(pkg, name)) as f:
            m = json.load(f)
        setter(np.array(m["params"], np.float32), np.array(m["mean"], np.float32), np.array(m["std"], np.float32),
               m.get("min_confidence", 0.5))
