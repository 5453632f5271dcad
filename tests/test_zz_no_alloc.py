"""blest_msbfs_noalloc (the multi-source entry point that allocates nothing)
against blest_msbfs and the oracle, through the C ABI: two calls in a row,
the second with fewer sources; its size limit and its set-up requirement."""
import numpy as np
import pytest

import oracle
from paper_2606_05081_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def blest():
    import torch
    from paper_2606_05081_amd import blest as b
    assert torch.cuda.is_available()
    b.lib()
    return b


@pytest.mark.parametrize("width", [64, 256])
def test_noalloc_matches_msbfs(blest, width):
    import torch
    rp, col = inputs.rmat_graph(14, 2201)
    g = blest.Graph(rp, col, msbfs_width=width)
    n = g.n
    srcs = inputs.sources(rp, 300, seed=2202)
    out = torch.full((srcs.size, n), 7, dtype=torch.int16, device="cuda")
    # before any multi-source call the graph's buffers do not exist: refused, nothing allocated
    with pytest.raises(blest.BlestError) as ei:
        g.msbfs_noalloc(srcs, out)
    assert ei.value.status == blest.Status.UNSUPPORTED
    ref1 = g.msbfs(srcs).cpu().numpy()
    assert np.array_equal(ref1, oracle.msbfs16(rp, col, srcs))
    g.msbfs_noalloc(srcs, out)
    g.sync()
    assert np.array_equal(out.cpu().numpy(), ref1)
    # second call, fewer sources (a ragged last batch), the array keeps the first call's tail
    s2 = srcs[::7][:37].copy()
    out2 = torch.full((s2.size, n), 7, dtype=torch.int16, device="cuda")
    g.msbfs_noalloc(s2, out2)
    g.sync()
    ref2 = g.msbfs(s2).cpu().numpy()
    assert np.array_equal(out2.cpu().numpy(), ref2)
    assert np.array_equal(ref2, oracle.msbfs16(rp, col, s2))
    # the limit, checked before anything runs
    big = np.zeros(65537, dtype=np.int32)
    with pytest.raises(blest.BlestError) as ei:
        blest.blest_msbfs_noalloc(g._h, big, out2)
    assert ei.value.status == blest.Status.INVALID_ARG
    g.close()


def test_noalloc_relabelled_graph(blest):
    """A graph the build relabels (RCM on a grid): sources are mapped on the host."""
    import torch
    rp, col = inputs.grid_graph(90, 2203)
    g = blest.Graph(rp, col)
    assert g.info()["reordered"] != 0
    srcs = inputs.sources(rp, 130, seed=2204)
    g.msbfs(srcs[:64])
    out = torch.empty((srcs.size, g.n), dtype=torch.int16, device="cuda")
    g.msbfs_noalloc(srcs, out)
    g.sync()
    assert np.array_equal(out.cpu().numpy(), oracle.msbfs16(rp, col, srcs))
    g.close()
