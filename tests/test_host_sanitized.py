"""Host code under sanitizers (no GPU).

Builds tests/host/host_checks.cpp with the library's host-only sources (the
planner, the tuning-cache and checkpoint file formats, the serving policy)
and the CPU oracle, once with AddressSanitizer + UndefinedBehaviorSanitizer
and once with ThreadSanitizer, and runs: the planner over n = 1..60 (int32,
the int32 exactness edge, float32, non-finite input), the JSON cache and
checkpoint readers on 20000 and 4000 mutated inputs, the serving policy
driven by a mock queue and device (the mock finishes each request with the
oracle; results are checked per ticket against a second oracle evaluation),
and the oracle's threaded entry points.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_04857_amd", "csrc")
HOST_SRC = [os.path.join(ROOT, "tests", "host", "host_checks.cpp"),
            os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "hostio.cpp"),
            os.path.join(CSRC, "serve_policy.cpp")]
ORACLE_SRC = os.path.join(ROOT, "oracle", "qubo_oracle.c")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc and g++")


def _build(out_dir, sanitize):
    flags = ["-O1", "-g", f"-fsanitize={sanitize}", "-fno-sanitize-recover=all", "-pthread"]
    if "thread" in sanitize:
        flags = ["-O1", "-g", "-fsanitize=thread", "-pthread"]
    obj = os.path.join(out_dir, "oracle.o")
    # the oracle's per-ISA clones are resolved by the loader before a
    # sanitizer runtime starts: one code path in sanitizer builds
    subprocess.check_call(["gcc", *flags, "-std=c11", "-DORACLE_NO_TARGET_CLONES", "-c",
                           ORACLE_SRC, "-o", obj])
    exe = os.path.join(out_dir, "host_checks")
    subprocess.check_call(["g++", *flags, "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", CSRC, *HOST_SRC, obj, "-o", exe])
    return exe


@pytest.fixture(scope="module")
def asan_exe(tmp_path_factory):
    return _build(str(tmp_path_factory.mktemp("asan")), "address,undefined")


@pytest.fixture(scope="module")
def tsan_exe(tmp_path_factory):
    return _build(str(tmp_path_factory.mktemp("tsan")), "thread")


def _run(exe, what, tmp_path):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    p = subprocess.run([exe, what, str(tmp_path)], capture_output=True, text=True, timeout=600,
                       env=env)
    print(p.stdout, p.stderr[-4000:])
    assert p.returncode == 0, (what, p.stdout, p.stderr[-4000:])
    return p.stdout


@pytest.mark.parametrize("what", ["plan", "json", "ckpt", "sched", "oracle"])
def test_host_checks_asan_ubsan(asan_exe, what, tmp_path):
    _run(asan_exe, what, tmp_path)


@pytest.mark.parametrize("what", ["oracle", "sched"])
def test_host_checks_tsan(tsan_exe, what, tmp_path):
    _run(tsan_exe, what, tmp_path)
