"""Host code under sanitizers (CPU only): the library's preprocessing
(host_build.cpp: CSR validation, threaded RCM, JaccardWithWindows, BVSS and
panel builds), the seeded generators and the oracle's threaded job split are
built with AddressSanitizer + UndefinedBehaviorSanitizer and, separately,
ThreadSanitizer, and driven by the programs in tests/sanitize/. A sanitizer
report makes the program exit non-zero (no recovery) and the test fail."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2606_05081_amd", "csrc")
GEN = os.path.join(ROOT, "paper_2606_05081_amd", "inputs", "graphgen.cpp")
ORACLE = os.path.join(ROOT, "oracle", "oracle.c")

MODES = {
    "asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"],
    "tsan": ["-fsanitize=thread"],
}


def _run(cmd, env=None):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.fixture(scope="module")
def outdir(tmp_path_factory):
    if shutil.which("g++") is None or shutil.which("gcc") is None:
        pytest.skip("g++/gcc not available")
    return tmp_path_factory.mktemp("sanitize")


def _env(mode):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1:second_deadlock_stack=1"
    return env


@pytest.mark.parametrize("mode", sorted(MODES))
def test_host_build_under_sanitizer(mode, outdir):
    exe = str(outdir / f"host_build_{mode}")
    flags = ["-O1", "-g", "-std=c++17", "-pthread", *MODES[mode]]
    _run(["g++", *flags, "-I", CSRC, os.path.join(SAN, "host_build_check.cpp"), os.path.join(CSRC, "host_build.cpp"),
          GEN, "-o", exe])
    r = _run([exe], env=_env(mode))
    assert "0 failures" in r.stdout


@pytest.mark.parametrize("mode", sorted(MODES))
def test_oracle_under_sanitizer(mode, outdir):
    exe = str(outdir / f"oracle_{mode}")
    cflags = ["-O1", "-g", "-pthread", *MODES[mode]]
    obj_o = str(outdir / f"oracle_{mode}.o")
    obj_c = str(outdir / f"oracle_check_{mode}.o")
    _run(["gcc", *cflags, "-std=c11", "-c", ORACLE, "-o", obj_o])
    _run(["gcc", *cflags, "-std=c11", "-c", os.path.join(SAN, "oracle_check.c"), "-o", obj_c])
    _run(["g++", *cflags, "-std=c++17", obj_o, obj_c, GEN, "-o", exe])
    r = _run([exe], env=_env(mode))
    assert "0 failures" in r.stdout
