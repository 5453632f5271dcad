"""The C ABI library loads and exports what include/blest.h declares; host-side
argument checking works without a GPU (no compute calls here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "blest.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(blest_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_core_entry_points():
    names = declared_functions()
    for want in ["blest_build", "blest_bfs", "blest_msbfs", "blest_closeness", "blest_free",
                 "blest_set_switch_model", "blest_mlp_loss_grad", "blest_mlp_train"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2606_05081_amd import blest
    L = blest.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # and the Python binding wraps every one of them
    assert set(declared_functions()) == set(blest.SIGNATURES)


def test_status_strings_and_defaults():
    from paper_2606_05081_amd import blest
    L = blest.lib()
    assert L.blest_status_str(0) == b"OK"
    assert L.blest_status_str(-8) == b"TIMEOUT"
    o = blest.default_opts()
    assert (o.sigma, o.tau, o.eta, o.policy, o.persistent, o.msbfs_width) == (8, 128, 10.0, 0, 1, 512)
    # layout of blest_opts in include/blest.h: 12 int32/float fields, a uint64, an int32, int32[11]
    assert ctypes.sizeof(blest.Opts) == 104 and blest.Opts.random_seed.offset == 48
    assert ctypes.sizeof(blest.LevelStat) == 8 + 8 * 8 + 16 + 24 + 8 + 8 + 8
    assert ctypes.sizeof(blest.GraphStats) == 16 + 16 + 48 + 12 + 20 + 8
    assert o.update_scheme == blest.Update.AUTO and o.directed == 0


@pytest.mark.parametrize("case,status", [
    ("asym", -2), ("selfloop", -2), ("unsorted", -2), ("dup", -2), ("range", -2), ("sigma", -7), ("tau", -7),
])
def test_build_rejects_bad_input_on_host(case, status):
    from paper_2606_05081_amd import blest
    rp = np.array([0, 1, 2, 2], np.int32)
    col = np.array([1, 0], np.int32)
    opts = blest.default_opts()
    if case == "asym":
        rp, col = np.array([0, 1, 1, 1], np.int32), np.array([1], np.int32)
    elif case == "selfloop":
        rp, col = np.array([0, 2, 3, 3], np.int32), np.array([0, 1, 0], np.int32)
    elif case == "unsorted":
        rp, col = np.array([0, 2, 3, 4], np.int32), np.array([2, 1, 0, 0], np.int32)
    elif case == "dup":
        rp, col = np.array([0, 2, 4, 4], np.int32), np.array([1, 1, 0, 0], np.int32)
    elif case == "range":
        rp, col = np.array([0, 1, 2, 2], np.int32), np.array([7, 0], np.int32)
    elif case == "sigma":
        opts.sigma = 12
    elif case == "tau":
        opts.tau = 100
    with pytest.raises(blest.BlestError) as ei:
        blest.blest_build(rp, col, opts)
    assert ei.value.status == status


def test_struct_layout_matches_c_compiler(tmp_path):
    """Compiles a probe against include/blest.h with gcc and compares sizes/offsets."""
    import shutil
    import subprocess
    from paper_2606_05081_amd import blest
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "probe.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "blest.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(blest_opts),'
        ' offsetof(blest_opts, random_seed), offsetof(blest_opts, device), sizeof(blest_level_stat),'
        ' offsetof(blest_level_stat, t_step_us), sizeof(blest_graph_stats), sizeof(blest_csr),'
        ' sizeof(blest_ms_level_stat), offsetof(blest_ms_level_stat, t_engine_us),'
        ' offsetof(blest_ms_level_stat, feat)); printf("%zu %zu %zu\\n", offsetof(blest_opts, jaccard_window),'
        ' offsetof(blest_opts, update_scheme), offsetof(blest_graph_stats, u_div)); return 0;}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    exp = [ctypes.sizeof(blest.Opts), blest.Opts.random_seed.offset, blest.Opts.device.offset,
           ctypes.sizeof(blest.LevelStat), blest.LevelStat.t_step_us.offset, ctypes.sizeof(blest.GraphStats),
           ctypes.sizeof(blest.CSR), ctypes.sizeof(blest.MsLevelStat), blest.MsLevelStat.t_engine_us.offset,
           blest.MsLevelStat.feat.offset, blest.Opts.jaccard_window.offset, blest.Opts.update_scheme.offset,
           blest.GraphStats.u_div.offset]
    assert got == exp
